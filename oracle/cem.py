"""FP64 oracle of the projection-guided sampling loop (thesis ch. 6, Alg 3, eqs
update_mean / update_covariance).  TEST INFRASTRUCTURE ONLY (see oracle/__init__).

One CEM iteration l:
  1. draw N_b samples xi_i = mu + L z_i, L L^T = Sigma + eps I (z_i ~ N(0, I) are
     inputs: the random numbers the method draws are passed in);
  2. project every sample with K AM iterations from a cold start (the C oracle);
  3. residual r_i of the projected sample (Alg 3 "compute the residuals set");
  4. ConstraintEliteSet: the N_proj samples with the lowest residual;
  5. augmented cost c_aug = c_1 + r with c_1 = sum_t |xdd(t)|^2 (acceleration cost);
  6. EliteSet: the N_elite samples of step 4 with the lowest c_aug;
  7. weights c_m = exp(-(c_aug_m - delta) / (gamma * std)), delta = min c_aug over the
     elite set, std = its standard deviation;  mu and Sigma move towards the weighted
     mean and covariance (about the new mean) with learning rate sigma.
The loop returns the projected sample of the last elite set with the lowest c_aug.

Readings (listed in the design notes):
  * the printed weight exp(gamma^-1 (c_aug - delta)) would up-weight worse samples; the
    sign is flipped, and gamma is relative to the elite set's cost spread;
  * residuals are compared at a resolution of `quantum` (1e-6): residual keys are
    floor(r / quantum), ties are ranked by c_aug and then by sample index, so the
    ConstraintEliteSet is unique even when many samples are feasible (r ~ 0); the
    EliteSet ranks by c_aug, ties by sample index;
  * Sigma gets eps = 1e-10 on its diagonal before the Cholesky factorization (the
    boundary coefficients of every projected sample coincide, so their variance
    only decays).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import bernstein, project, residuals

EPS_CHOL = 1e-10


def sample(mu, Sigma, z):
    """xi = mu + L z for each row of z; L = chol(Sigma + eps I)."""
    L = np.linalg.cholesky(Sigma + EPS_CHOL * np.eye(Sigma.shape[0]))
    return mu[None, :] + z @ L.T, L


def acceleration_cost(w, xb):
    """c_1 = sum over time samples and axes of (Pdd xb)^2, per sample."""
    _, _, Pdd = bernstein(w.degree, w.n_steps, w.horizon)
    acc = np.einsum("tm,bdm->btd", Pdd, xb)
    return np.sum(acc * acc, axis=(1, 2))


def select(keys, n_keep):
    """Indices of the n_keep smallest keys; keys is a tuple of arrays compared
    lexicographically (first array most significant), ties broken by index."""
    idx = np.arange(len(keys[0]))
    order = np.lexsort(tuple([idx] + [np.asarray(k) for k in reversed(keys)]))
    return order[:n_keep]


def weighted_update(mu, Sigma, xb_elite, caug_elite, sigma, gamma):
    delta = caug_elite.min()
    spread = caug_elite.std()
    scale = gamma * spread if spread > 0 else 1.0
    wgt = np.exp(-(caug_elite - delta) / scale)
    mu_new = (1 - sigma) * mu + sigma * (wgt @ xb_elite) / wgt.sum()
    d = xb_elite - mu_new[None, :]
    Sigma_new = (1 - sigma) * Sigma + sigma * (d.T * wgt) @ d / wgt.sum()
    return mu_new, Sigma_new, wgt


@dataclasses.dataclass
class CemTrace:
    mu: list
    Sigma: list
    proj_idx: list
    elite_idx: list
    caug: list
    res: list
    best: np.ndarray
    best_cost: float


def cem(w, mu0, Sigma0, z, am_iters, n_proj, n_elite, sigma=0.5, gamma=1.0, quantum=1e-6,
        n_threads=0):
    """Alg 3 on the problem of workload `w` (its samples are ignored).
    z: [N, N_b, D * n_v] standard normal draws; returns a CemTrace."""
    mu = np.asarray(mu0, dtype=np.float64).copy()
    Sigma = np.asarray(Sigma0, dtype=np.float64).copy()
    D, nv = w.dims, w.degree + 1
    tr = CemTrace([], [], [], [], [], [], None, np.inf)
    for l in range(z.shape[0]):
        xi, _ = sample(mu, Sigma, z[l])
        xi = xi.reshape(-1, D, nv)
        xb, _, _, _ = project(w, iters=am_iters, n_threads=n_threads, xi=xi)
        r, _ = residuals(w, xb, n_threads=n_threads)
        caug = acceleration_cost(w, xb) + r
        rkey = np.floor(r / quantum)
        proj = select((rkey, caug), n_proj)
        elite = proj[select((caug[proj], proj), n_elite)]
        xe = xb.reshape(len(xb), -1)[elite]
        mu, Sigma, _ = weighted_update(mu, Sigma, xe, caug[elite], sigma, gamma)
        tr.mu.append(mu.copy())
        tr.Sigma.append(Sigma.copy())
        tr.proj_idx.append(proj)
        tr.elite_idx.append(elite)
        tr.caug.append(caug)
        tr.res.append(r)
        b = elite[np.argmin(caug[elite])]
        tr.best = xb[b].copy()
        tr.best_cost = float(caug[b])
    return tr
