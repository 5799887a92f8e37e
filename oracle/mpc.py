"""FP64 oracle of the receding-horizon loop around the projection (thesis ch. 5,
Paper II, Implementation Details: an MPC built on the batch optimizer that starts
every control cycle from the preceding cycle's solution, multipliers included).
TEST INFRASTRUCTURE ONLY (see oracle/__init__).

One control cycle c on a problem of horizon T (degree n Bernstein coefficients per
axis, boundary rows (x0, v0, a0, xf)):
  1. project the batch with K AM iterations from (xi_bar0, lam0) (the C oracle);
  2. execute: the sample whose result has the lowest residual, compared at a resolution
     of 1e-6 (ties, such as every feasible sample: the lowest index), is
     followed for delta seconds; its position, velocity and acceleration at delta are
     the next cycle's start rows, the goal row stays;
  3. the obstacles move on: c_j <- c_j + w_j delta;
  4. every sample is re-expressed on the shifted window: the same polynomial with the
     time origin moved to delta, xi_next = S(delta) xi_bar per axis; the next cycle
     projects the samples xi_next from xi_bar0 = xi_next and lam0 = lam (reuse, as
     the thesis does) or lam0 = 0.
Readings (listed in the design notes): the thesis says only that the multipliers start
from the preceding loop's solution; here the next cycle's samples are the shifted
projected samples of the cycle before, the multiplier is carried over unchanged (no
time shift of its own), and the executed sample is the one of lowest residual at a
1e-6 resolution (residuals within rounding of each other would otherwise decide).

S(delta) comes from the power basis: with u = t / T, p(u) = sum_m c_m u^m where
c = M xi (M: Bernstein to power), p(u + d) = sum_j (sum_{m>=j} c_m C(m, j) d^(m-j)) u^j
(d = delta / T), and xi_next = M^-1 (shifted c).
"""
from __future__ import annotations

import dataclasses
from math import comb

import numpy as np

from . import project, residuals


def bernstein_to_power(n: int) -> np.ndarray:
    """M with c = M xi: sum_k xi_k C(n,k) u^k (1-u)^(n-k) = sum_m c_m u^m."""
    M = np.zeros((n + 1, n + 1))
    for k in range(n + 1):
        for m in range(k, n + 1):
            M[m, k] = comb(n, k) * comb(n - k, m - k) * (-1.0) ** (m - k)
    return M


def shift_matrix(n: int, T: float, delta: float) -> np.ndarray:
    """S(delta): Bernstein coefficients on [0, T] -> those of the same polynomial with
    its time origin moved to delta (the window [delta, delta + T])."""
    d = delta / T
    Tm = np.zeros((n + 1, n + 1))   # power coefficients of p(u + d)
    for j in range(n + 1):
        for m in range(j, n + 1):
            Tm[j, m] = comb(m, j) * d ** (m - j)
    M = bernstein_to_power(n)
    return np.linalg.solve(M, Tm @ M)


def state_at(coeffs: np.ndarray, T: float, t: float):
    """(p, v, a) [D] at time t of the trajectories with Bernstein coefficients
    coeffs [D, n_v] on [0, T] (closed-form derivatives of the basis)."""
    coeffs = np.asarray(coeffs, dtype=np.float64)
    n = coeffs.shape[-1] - 1
    u = t / T

    def basis(deg, k):
        return comb(deg, k) * u ** k * (1 - u) ** (deg - k) if 0 <= k <= deg else 0.0
    p = sum(coeffs[:, k] * basis(n, k) for k in range(n + 1))
    d1 = np.diff(coeffs, 1, axis=1) * n / T
    v = sum(d1[:, k] * basis(n - 1, k) for k in range(n))
    d2 = np.diff(coeffs, 2, axis=1) * n * (n - 1) / T ** 2
    a = sum(d2[:, k] * basis(n - 2, k) for k in range(n - 1))
    return p, v, a


@dataclasses.dataclass
class Cycle:
    xi: np.ndarray        # [B, D, n_v] the samples projected in this cycle
    xi_bar: np.ndarray    # [B, D, n_v] after K iterations
    lam: np.ndarray
    trace: np.ndarray     # [K, B] residual per iteration
    boundary: np.ndarray  # [D, 4] the cycle's boundary rows
    executed: int         # the sample followed for delta seconds


QUANTUM = 1e-6   # residuals are compared at this resolution when the executed sample is chosen


def executed_sample(res) -> int:
    """The sample of lowest residual key floor(r / QUANTUM); ties (every feasible
    sample shares key 0): the lowest index."""
    return int(np.argmin(np.floor(np.asarray(res, dtype=np.float64) / QUANTUM)))


def mpc(w, n_cycles: int, delta: float, iters: int, keep_lambda: bool = True, n_threads: int = 0):
    """The receding-horizon loop on workload w (its xi are the first cycle's samples,
    projected from a cold start).  Returns the list of Cycle records."""
    S = shift_matrix(w.degree, w.horizon, delta)
    xi = np.array(w.xi, dtype=np.float64)
    xb0, lam0 = None, None
    bnd = np.array(w.boundary, dtype=np.float64)
    centre = np.array(w.obs_centre, dtype=np.float64)
    out = []
    for _ in range(n_cycles):
        wc = dataclasses.replace(w, xi=xi, boundary=bnd, obs_centre=centre)
        xb, lam, tr, _ = project(wc, xi_bar=xb0, lam=lam0, iters=iters, n_threads=n_threads)
        res = residuals(wc, xb, n_threads=n_threads)[0]
        i = executed_sample(res)
        out.append(Cycle(xi, xb, lam, tr, bnd, i))
        p, v, a = state_at(xb[i], w.horizon, delta)
        bnd = bnd.copy()
        bnd[:, 0], bnd[:, 1], bnd[:, 2] = p, v, a
        centre = centre + np.array(w.obs_vel, dtype=np.float64) * delta
        xi = np.einsum("jk,bdk->bdj", S, xb)
        xb0 = xi.copy()
        lam0 = lam.copy() if keep_lambda else np.zeros_like(lam)
    return out
