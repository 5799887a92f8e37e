"""Pins of the oracle's counter-based generator (oracle/rng.py): the Philox4x64-10
blocks against numpy's independent implementation, and the normals against the
Box-Muller closed form and their distribution."""
import numpy as np
import pytest
from scipy import stats

from oracle import rng


@pytest.mark.parametrize("key,counter", [(7, 0), (0, 0), (2 ** 64 - 1, 2 ** 64 - 5), (123456789, 42)])
def test_philox_blocks_match_numpy(key, counter):
    """numpy's Philox advances its 256-bit counter before each block: its block b under
    counter c is ours at c + 1 + b."""
    bg = np.random.Philox(key=np.array([key, 0], dtype=np.uint64),
                          counter=np.array([counter, 0, 0, 0], dtype=np.uint64))
    raw = [int(x) for x in bg.random_raw(4 * 6)]
    for b in range(6):
        c = (counter + 1 + b) % 2 ** 64
        carry = 1 if counter + 1 + b >= 2 ** 64 else 0
        got = rng.philox4x64_10((c, carry, 0, 0), (key, 0))
        assert got == raw[4 * b:4 * b + 4], b


def test_box_muller_closed_form():
    words = rng.philox4x64_10((9, 0, 0, 0), (3, 0))
    u = rng.uniforms(words)
    assert np.all((u > 0) & (u < 1))
    z = rng.normals(4, 3, 9)
    # the two pairs lie on circles of radius sqrt(-2 ln u_0), sqrt(-2 ln u_2) at the
    # angles 2 pi u_1, 2 pi u_3
    np.testing.assert_allclose(z[0] ** 2 + z[1] ** 2, -2 * np.log(u[0]), rtol=1e-13)
    np.testing.assert_allclose(z[2] ** 2 + z[3] ** 2, -2 * np.log(u[2]), rtol=1e-13)
    np.testing.assert_allclose(np.arctan2(z[1], z[0]) % (2 * np.pi), 2 * np.pi * u[1], rtol=1e-12)
    np.testing.assert_allclose(np.arctan2(z[3], z[2]) % (2 * np.pi), 2 * np.pi * u[3], rtol=1e-12)
    # a stream's prefix does not depend on the count asked for; blocks follow the counter
    np.testing.assert_array_equal(rng.normals(7, 3, 9)[:4], z)
    np.testing.assert_array_equal(rng.normals(8, 3, 9)[4:], rng.normals(4, 3, 10))


def test_normals_are_standard_normal():
    z = rng.normals(20000, 2024, 0)
    assert abs(z.mean()) < 0.03 and abs(z.std() - 1) < 0.02
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # the two members of a pair are uncorrelated
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 0.03
