"""AddressSanitizer and UndefinedBehaviorSanitizer over the host code (CPU only).

Two builds with gcc's sanitizers, each exercised by the existing CPU tests in a child
process that preloads the sanitizer runtimes (the Python interpreter itself is not
instrumented):
* the C oracle, under the oracle pins (single robot, multi-agent, sampling loop);
* the library's host C++ (problem validation, the FP64 precompute, the QP-contraction
  estimate, error reporting, the network entry points' checks), linked with the
  kernels' objects unchanged, under the C-ABI tests.
Undefined behaviour aborts (no recovery) and any ASan report fails the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_10731_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
       "-O1", "-g", "-fPIC"]


def _runtime(name):
    path = subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"gcc has no {name}")
    return path


def _child(tmp_path, env_extra, tests, extra_args=()):
    env = dict(os.environ)
    env.update(env_extra)
    env["LD_PRELOAD"] = _runtime("libasan.so") + ":" + _runtime("libubsan.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           *extra_args, *[os.path.join(ROOT, "tests", t) for t in tests]]
    r = subprocess.run(cmd, env=env, cwd=str(tmp_path), capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return out


def test_oracle_under_sanitizers(tmp_path):
    lib = str(tmp_path / "oracle_san.so")
    subprocess.check_call(["gcc", *SAN, "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-shared",
                           os.path.join(ROOT, "oracle", "trajam_oracle.c"), "-o", lib, "-lm"])
    out = _child(tmp_path, {"TRAJAM_ORACLE_LIB": lib},
                 ["test_oracle_pins.py", "test_oracle_agents.py", "test_cem.py"])
    assert " passed" in out


def test_host_library_under_sanitizers(tmp_path):
    from paper_2408_10731_amd import build as hb
    objs = [os.path.join(hb.HERE, "_build", s + ".o") for s in hb.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in objs):
        hb.build()
    host = []
    for src in [s for s in hb.SOURCES if s.endswith(".cpp")]:
        o = str(tmp_path / (src + ".o"))
        subprocess.check_call(["g++", *SAN, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                               "-c", os.path.join(CSRC, src), "-o", o])
        host.append(o)
    lib = str(tmp_path / "libtrajam_san.so")
    subprocess.check_call(["g++", "-shared", "-fsanitize=address,undefined", *host, *objs,
                           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", lib])
    out = _child(tmp_path, {"TRAJAM_LIBRARY": lib}, ["test_abi.py"])
    assert " passed" in out


def test_instrumented_oracle_reports_an_overflow(tmp_path):
    """The instrumented build is live: a basis request larger than the buffers it is
    given (a mistake planted in the caller, on the CPU) is reported by ASan."""
    lib = str(tmp_path / "oracle_san.so")
    subprocess.check_call(["gcc", *SAN, "-std=c11", "-D_DEFAULT_SOURCE", "-shared",
                           os.path.join(ROOT, "oracle", "trajam_oracle.c"), "-o", lib, "-lm"])
    code = ("import ctypes, numpy as np\n"
            f"L = ctypes.CDLL({lib!r})\n"
            "dp = ctypes.POINTER(ctypes.c_double)\n"
            "L.orc_bernstein.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp, dp]\n"
            "a = [np.zeros(8) for _ in range(3)]\n"
            "L.orc_bernstein(10, 100, 1.0, *[x.ctypes.data_as(dp) for x in a])\n")
    env = dict(os.environ)
    env["LD_PRELOAD"] = _runtime("libasan.so") + ":" + _runtime("libubsan.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0"
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr, r.stderr[-2000:]
