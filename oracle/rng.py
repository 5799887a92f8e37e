"""Counter-based generator of the sampling loop's draws, written from its published
definition: Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC 2011), and standard normals from its output by the
Box-Muller transform.  TEST INFRASTRUCTURE ONLY (see oracle/__init__).

Stream (key, counter): block b is Philox4x64-10 of the 256-bit counter
(counter + b mod 2^64, 0, 0, 0) under the 128-bit key (key, 0); its four 64-bit words
x_0..x_3 become uniforms u_j = (floor(x_j / 2^11) + 1/2) 2^-53 in (0, 1), and the
pairs (u_0, u_1), (u_2, u_3) the normals
    z_{4b}   = sqrt(-2 ln u_0) cos(2 pi u_1),  z_{4b+1} = sqrt(-2 ln u_0) sin(2 pi u_1),
    z_{4b+2} = sqrt(-2 ln u_2) cos(2 pi u_3),  z_{4b+3} = sqrt(-2 ln u_2) sin(2 pi u_3).
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157     # round multipliers
W0, W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B     # key schedule (Weyl) increments
MASK = (1 << 64) - 1


def philox4x64_10(ctr, key):
    """Four 64-bit words of one block (Python integers)."""
    c = [int(x) & MASK for x in ctr]
    k = [int(x) & MASK for x in key]
    for r in range(10):
        if r > 0:
            k = [(k[0] + W0) & MASK, (k[1] + W1) & MASK]
        p0, p1 = M0 * c[0], M1 * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k[0], p1 & MASK, (p0 >> 64) ^ c[3] ^ k[1], p0 & MASK]
    return c


def uniforms(words):
    return np.array([((w >> 11) + 0.5) * 2.0 ** -53 for w in words])


def normals(count: int, key: int, counter: int) -> np.ndarray:
    """The first `count` normals of the stream (float64)."""
    out = np.empty(4 * ((count + 3) // 4))
    for b in range(len(out) // 4):
        u = uniforms(philox4x64_10(((counter + b) & MASK, 0, 0, 0), (key, 0)))
        for j in (0, 2):
            r = np.sqrt(-2.0 * np.log(u[j]))
            out[4 * b + j] = r * np.cos(2.0 * np.pi * u[j + 1])
            out[4 * b + j + 1] = r * np.sin(2.0 * np.pi * u[j + 1])
    return out[:count]
