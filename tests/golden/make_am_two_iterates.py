"""Writes am_two_iterates.json: the first two AM iterates of a tiny problem, worked by
hand in exact rational arithmetic (thesis ch. 6: polar step eqs comp_alpha..comp_d,
multiplier eq lag, QP eqs affine_trans / matrix_vec; step order of the AM list, which
puts the fresh multiplier lambda^{k+1} into the QP of the same iteration).

The problem is chosen so that every quantity is a rational number and the derivation
fits on paper; this script calls nothing but Python's `fractions` and only repeats the
arithmetic of the derivation below.

  2D, degree n = 4, n_p = 5 samples over T = 4 s (tau_k = k/4), rho = 1, no velocity
  or acceleration block (F = P, one copy per obstacle), one circle of radius 1/2 at
  c = (5/4, 0).  Boundary: x from 0 (at rest) to 4, y from 0 to 0.  Sample
  xi_x = (0, 0, 0, 3, 4), xi_y = 0; cold start xb^0 = xi, lambda^0 = 0.

  The boundary rows fix xb_0 = x0, xb_1 = x0 + v0 T/n, xb_2 = x0 + 2 v0 T/n +
  a0 T^2/(n(n-1)), xb_4 = xf, so only xb_3 is free.  With xb_y = 0 every point lies
  on the x axis: the obstacle step moves a point inside the circle to the nearer end
  of the diameter (alpha = pi, d = 1), so e_y = 0 and the y axis stays 0.

  Per iteration (k = 0, 1):
    p_t   = sum_m B_m(tau_t) xb_m            (B_m(tau) = C(4,m) tau^m (1-tau)^(4-m))
    e_t   = c_x - 1/2 if |p_t - c_x| < 1/2 and p_t < c_x, else p_t (here the only
            point inside is t = 2, p_2 < c_x)
    r_t   = p_t - e_t
    lambda^{k+1} = lambda^k - rho P^T r
    QP on the free coefficient (its row of the KKT system; the boundary rows keep the
    fixed coefficients):  (H xb^{k+1})_3 = xi_3 + lambda^{k+1}_3 + rho (P^T e)_3,
    H = I + rho P^T P, P^T e = P^T P xb^k - P^T r, xb^{k+1} = xb^k + delta e_3
    =>  delta = (xi_3 - xb^k_3 + lambda^{k+1}_3 - rho (P^T r)_3) / H_33.
  With lambda^k in the QP instead (the other order), delta would lack lambda's
  update and the iterates differ (also written below, as `wrong_order`).
"""
import json
import os
from fractions import Fraction as Fr
from math import comb

N, NP, T, RHO = 4, 5, Fr(4), Fr(1)
C, R = Fr(5, 4), Fr(1, 2)
XI = [Fr(0), Fr(0), Fr(0), Fr(3), Fr(4)]
TAU = [Fr(k, NP - 1) for k in range(NP)]
B = [[comb(N, m) * t ** m * (1 - t) ** (N - m) for m in range(N + 1)] for t in TAU]
H33 = 1 + RHO * sum(B[t][3] ** 2 for t in range(NP))


def step(xb, lam, fresh=True):
    p = [sum(B[t][m] * xb[m] for m in range(N + 1)) for t in range(NP)]
    r = []
    for pt in p:
        inside = abs(pt - C) < R
        assert not (inside and pt >= C)
        r.append(pt - (C - R) if inside else Fr(0))
    Ptr = [sum(B[t][m] * r[t] for t in range(NP)) for m in range(N + 1)]
    lam_new = [lam[m] - RHO * Ptr[m] for m in range(N + 1)]
    lam_qp = lam_new if fresh else lam
    delta = (XI[3] - xb[3] + lam_qp[3] - RHO * Ptr[3]) / H33
    xb_new = list(xb)
    xb_new[3] = xb[3] + delta
    res = sum(x * x for x in r)  # squared residual norm (x axis; y is 0)
    return xb_new, lam_new, res, p


def run(fresh):
    xb, lam = list(XI), [Fr(0)] * (N + 1)
    out = []
    for _ in range(2):
        xb_new, lam_new, res2, p = step(xb, lam, fresh)
        out.append({"waypoints_x": [str(v) for v in p], "residual_sq": str(res2),
                    "xi_bar_x": [str(v) for v in xb_new], "lambda_x": [str(v) for v in lam_new]})
        xb, lam = xb_new, lam_new
    return out


def main():
    doc = {
        "what": "First two AM iterates of a tiny problem, worked by hand in exact rational "
                "arithmetic; derivation in make_am_two_iterates.py's docstring. Iterate k "
                "lists the waypoints of xb^k, the squared residual |F xb^k - e^{k+1}|^2 and "
                "the state (xb^{k+1}, lambda^{k+1}) after the iteration; y coefficients and "
                "multipliers are 0 throughout.",
        "cites": "thesis ch. 6: eqs comp_alpha..comp_d (polar step), eq lag (multiplier, "
                 "with the freshly projected e), eqs affine_trans / matrix_vec (QP taking "
                 "lambda^{k+1}), the order of the AM step list",
        "problem": {"dims": 2, "degree": N, "n_steps": NP, "horizon": 4.0, "v_max": 0.0,
                    "a_max": 0.0, "rho": 1.0, "obs_centre": [[1.25, 0.0]],
                    "obs_axes": [[0.5, 0.5]], "boundary": [[0, 0, 0, 4], [0, 0, 0, 0]],
                    "xi_x": [0, 0, 0, 3, 4]},
        "iterates": run(True),
        "wrong_order": run(False),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "am_two_iterates.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print(path)


if __name__ == "__main__":
    main()
