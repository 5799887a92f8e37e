"""Bounds the float32 arctangent of the materialised polar kernel (the angles of
thesis ch. 6 eqs comp_alpha, comp_beta) on the CPU.  (Vectors shorter than FLT_MIN
are outside these grids: the kernel keeps the larger magnitude at least FLT_MIN.)

The coefficients are read from the kernel source itself, so this checks the
committed polynomial, and its float32 evaluation (fma steps, the reciprocal, the
octant and quadrant corrections) is emulated in numpy and compared with FP64
arctan2 of the same float32 inputs on dense grids.  The hardware reciprocal is
within 1 ulp; the emulation takes the correctly rounded reciprocal and both of its
float neighbours and keeps the worst case."""
import os
import re

import numpy as np

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2408_10731_amd", "csrc", "polar_kernels.hip")
f32 = np.float32


def _coefficients():
    src = open(SRC).read()
    head = "__device__ __forceinline__ float polar_atan_poly(float a)"
    body = src[src.index(head):]
    body = body[:body.index("\n}\n")]
    lits = [float(v) for v in re.findall(r"(-?\d+\.\d+(?:e-?\d+)?)f", body)]
    assert len(lits) == 8, lits          # the odd polynomial's 8 coefficients
    return lits


def _fma(a, b, c):
    # float32 products are exact in float64; one rounding of the sum to float32
    return (a.astype(np.float64) * b.astype(np.float64) + np.float64(c)).astype(f32)


def _atan2(y, x, rcp_shift=0):
    """The kernel's float atan2: ratio min/max with max kept >= FLT_MIN, the polynomial,
    pi/2 - r above the diagonal, pi - r for x < 0, the sign of y."""
    poly = _coefficients()
    y = y.astype(f32)
    x = x.astype(f32)
    ax, ay = np.abs(x), np.abs(y)
    mx = np.maximum(np.maximum(ax, ay), f32(1.17549435e-38)).astype(f32)
    mn = np.minimum(ax, ay)
    rc = (f32(1) / mx).astype(f32)
    if rcp_shift:
        rc = np.nextafter(rc, f32(np.inf) if rcp_shift > 0 else f32(0)).astype(f32)
    a = (mn * rc).astype(f32)
    s = (a * a).astype(f32)
    q = np.full_like(a, f32(poly[0]))
    for c in poly[1:]:
        q = _fma(q, s, c)
    r = (a * q).astype(f32)
    r = np.where(ay > ax, (f32(np.pi / 2) - r).astype(f32), r)
    r = np.where(x < 0, (f32(np.pi) - r).astype(f32), r)
    return np.copysign(r, y).astype(f32)


def _err(got, y, x):
    ref = np.arctan2(y.astype(np.float64), x.astype(np.float64))
    d = np.abs(got.astype(np.float64) - ref)
    return np.minimum(d, np.abs(d - 2 * np.pi))


def test_first_octant_polynomial_error():
    a = np.linspace(0.0, 1.0, 2_000_001).astype(f32)
    one = np.ones_like(a)
    worst = max(_err(_atan2(a, one, s), a, one).max() for s in (-1, 0, 1))
    assert worst <= 2.0e-7, worst   # 1.3e-7 with a correctly rounded reciprocal


def test_full_atan2_error_and_special_cases():
    ang = np.linspace(-np.pi, np.pi, 2_000_001)
    worst = 0.0
    for rad in (1e-3, 1.0, 37.0):
        y = (rad * np.sin(ang)).astype(f32)
        x = (rad * np.cos(ang)).astype(f32)
        for s in (-1, 0, 1):
            worst = max(worst, _err(_atan2(y, x, s), y, x).max())
    # the quadrant corrections round pi - r to float (half an ulp of pi is 1.2e-7)
    assert worst <= 3.8e-7, worst
    z = np.zeros(1, dtype=f32)
    assert _atan2(z, z)[0] == 0.0                      # atan2(0, 0) = 0
    assert _atan2(z, -np.ones(1, f32))[0] == f32(np.pi)
    assert _atan2(-z, -np.ones(1, f32))[0] == -f32(np.pi)   # IEEE: atan2(-0, x < 0) = -pi
    assert _atan2(np.ones(1, f32), z)[0] == f32(np.pi / 2)
    assert _atan2(-np.ones(1, f32), z)[0] == -f32(np.pi / 2)
