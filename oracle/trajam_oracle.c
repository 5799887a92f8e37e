/*
 * trajam_oracle.c -- plain, slow, FP64 CPU oracle of the batched
 * alternating-minimization (AM) projection of Bernstein-polynomial trajectories.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this file's library.  The product path (the HIP
 * library under paper_2408_10731_amd/) shares no code, header, table or helper
 * with it.
 *
 * What it computes (thesis ch. 6, "Projection Optimization"):
 *   project every sample xi_i onto {A xi = b_eq, g(xi) <= 0} by the AM fixed
 *   point of eqs (fixed_point_1)-(fixed_point_2): per iteration k
 *     1. waypoints p = P xb, v = Pd xb, a = Pdd xb          (eq parameter)
 *     2. polar step for every obstacle j and time t          (eqs comp_alpha..comp_d,
 *        closed forms eqs zeta_2, compute_d_mij, d_max; spherical form eq collision_priest)
 *     3. polar step for the velocity / acceleration bounds   (eqs fv_priest, fa_priest,
 *        closed forms eqs alpha_v, alpha_a, compute_dv, compute_da)
 *     4. residual r = F xb - e and its 2-norm               (Alg 3, "compute the residuals")
 *     5. multiplier  lam <- lam - rho F^T (F xb - e)        (eq lag)
 *     6. QP          [I + rho F^T F, A^T; A, 0] [xb; nu] = [xi + lam + rho F^T e; b_eq]
 *                                                            (eqs affine_trans, matrix_vec)
 *   F stacks, per axis, P once per obstacle, then Pd and Pdd (eq f_e); it is never
 *   formed: F^T F = n_o P^T P + Pd^T Pd + Pdd^T Pdd and F^T e sums block by block.
 *
 * Readings of the thesis taken here (each one is listed with its reason in the
 * design notes of the repository):
 *   - the sign of rho F^T e in eta is '+', from the stationarity of the augmented
 *     Lagrangian (eq lagrange); the printed '-' is a typo;
 *   - the multiplier update uses the freshly projected e of the same iteration;
 *   - the multiplier lives in coefficient space (one entry per coefficient);
 *   - time grid t_k = k T / (n_p - 1), endpoints included;
 *   - four boundary rows per axis: position, velocity, acceleration at t = 0 and
 *     position at t = T;
 *   - for an ellipse/ellipsoid the angles are taken in coordinates scaled by the
 *     semi-axes: alpha = atan2(y~/s_y, x~/s_x), beta = atan2(hypot(x~/s_x, y~/s_y), z~/s_z);
 *     d then follows eq d_max;
 *   - the velocity / acceleration scale is the 1-D projection min(1, |v|/v_max),
 *     which makes the kinematic step the exact projection onto the ball;
 *   - a point exactly at an obstacle centre takes atan2(+0, +0) = 0 (and beta = 0 in
 *     3D): it is pushed along +x in 2D and along +z in 3D; a zero velocity gives e_v = 0;
 *   - rho is one fixed scalar for all blocks.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int dims;          /* 2 or 3 */
    int degree;        /* Bernstein degree n; n_v = n + 1 coefficients per axis */
    int n_steps;       /* n_p time samples */
    double horizon;    /* T [s] */
    double v_max;      /* <= 0 removes the velocity block from F */
    double a_max;      /* <= 0 removes the acceleration block from F */
    double rho;        /* penalty weight of the augmented Lagrangian */
    int n_obs;         /* n_o obstacles (each contributes one copy of P to F) */
    int workspace;     /* 1: workspace bounds G xb <= tau, G = [-P; P], tau = [-ws_lo; ws_hi]
                          per axis (Paper III eq bound_con), through a slack variable */
    double ws_lo[3], ws_hi[3];
} orc_problem;

/* Deliberate-mistake switch used only by the mutation tests: each code plants
 * one plausible error in this oracle so the tests can show that a pin catches it.
 * 0 = correct oracle. */
static int g_fault = 0;
void orc_set_fault(int code) { g_fault = code; }

/* ------------------------------------------------------------------ basis -- */

static double binom(int n, int k)
{
    double r = 1.0;
    int i;
    if (k < 0 || k > n) return 0.0;
    for (i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

/* Bernstein polynomial B_{m,n}(tau) = C(n,m) tau^m (1-tau)^(n-m); 0 outside 0..n. */
static double bern(int m, int n, double tau)
{
    if (m < 0 || m > n || n < 0) return 0.0;
    return binom(n, m) * pow(tau, m) * pow(1.0 - tau, n - m);
}

/* Basis matrices of eq (parameter) for a Bernstein basis, row-major [n_p][n_v].
 * Derivatives use d/dt B_{m,n}(t/T) = (n/T)(B_{m-1,n-1} - B_{m,n-1}). */
int orc_bernstein(int n, int n_p, double T, double *P, double *Pd, double *Pdd)
{
    int k, m, nv = n + 1;
    if (n < 2 || n_p < 2 || !(T > 0.0)) return -1;
    for (k = 0; k < n_p; ++k) {
        double tau = (double)k / (double)(n_p - 1);
        for (m = 0; m < nv; ++m) {
            P[k * nv + m] = bern(m, n, tau);
            Pd[k * nv + m] = (double)n / T * (bern(m - 1, n - 1, tau) - bern(m, n - 1, tau));
            Pdd[k * nv + m] = (double)n * (double)(n - 1) / (T * T) *
                              (bern(m - 2, n - 2, tau) - 2.0 * bern(m - 1, n - 2, tau) +
                               bern(m, n - 2, tau));
        }
    }
    return 0;
}

/* ------------------------------------------------------- fixed matrices -- */

/* A = [P_0; Pd_0; Pdd_0; P_{-1}] (4 x n_v) and H = I + rho F^T F (n_v x n_v). */
int orc_constraint_matrices(const orc_problem *pr, double *A, double *H)
{
    int nv = pr->degree + 1, np = pr->n_steps, i, j, k;
    double *P = malloc(sizeof(double) * np * nv), *Pd = malloc(sizeof(double) * np * nv),
           *Pdd = malloc(sizeof(double) * np * nv);
    if (orc_bernstein(pr->degree, np, pr->horizon, P, Pd, Pdd) != 0) {
        free(P); free(Pd); free(Pdd);
        return -1;
    }
    for (j = 0; j < nv; ++j) {
        A[0 * nv + j] = P[0 * nv + j];
        A[1 * nv + j] = Pd[0 * nv + j];
        A[2 * nv + j] = Pdd[0 * nv + j];
        A[3 * nv + j] = P[(np - 1) * nv + j];
    }
    for (i = 0; i < nv; ++i)
        for (j = 0; j < nv; ++j) {
            double ff = 0.0;
            for (k = 0; k < np; ++k) {
                ff += (double)pr->n_obs * P[k * nv + i] * P[k * nv + j];
                /* the rows G = [-P; P] of the workspace bounds: G^T G = 2 P^T P */
                if (pr->workspace) ff += 2.0 * P[k * nv + i] * P[k * nv + j];
                if (pr->v_max > 0.0) ff += Pd[k * nv + i] * Pd[k * nv + j];
                if (pr->a_max > 0.0) ff += Pdd[k * nv + i] * Pdd[k * nv + j];
            }
            H[i * nv + j] = (i == j ? 1.0 : 0.0) + pr->rho * ff;
        }
    free(P); free(Pd); free(Pdd);
    return 0;
}

/* KKT matrix [[H, A^T], [A, 0]] of eq (matrix_vec), row-major (n_v+4)^2. */
int orc_kkt_matrix(const orc_problem *pr, double *K)
{
    int nv = pr->degree + 1, N = nv + 4, i, j;
    double *A = malloc(sizeof(double) * 4 * nv), *H = malloc(sizeof(double) * nv * nv);
    int rc = orc_constraint_matrices(pr, A, H);
    if (rc == 0) {
        memset(K, 0, sizeof(double) * N * N);
        for (i = 0; i < nv; ++i)
            for (j = 0; j < nv; ++j) K[i * N + j] = H[i * nv + j];
        for (i = 0; i < 4; ++i)
            for (j = 0; j < nv; ++j) {
                K[(nv + i) * N + j] = A[i * nv + j];
                K[j * N + nv + i] = A[i * nv + j];
            }
    }
    free(A); free(H);
    return rc;
}

/* In-place LU with partial pivoting (Doolittle); returns -1 on a zero pivot. */
int orc_lu_factor(int n, double *M, int *piv)
{
    int i, j, k;
    for (k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(M[k * n + k]);
        for (i = k + 1; i < n; ++i)
            if (fabs(M[i * n + k]) > best) { best = fabs(M[i * n + k]); p = i; }
        piv[k] = p;
        if (best == 0.0) return -1;
        if (p != k)
            for (j = 0; j < n; ++j) {
                double t = M[k * n + j]; M[k * n + j] = M[p * n + j]; M[p * n + j] = t;
            }
        for (i = k + 1; i < n; ++i) {
            double l = M[i * n + k] / M[k * n + k];
            M[i * n + k] = l;
            for (j = k + 1; j < n; ++j) M[i * n + j] -= l * M[k * n + j];
        }
    }
    return 0;
}

void orc_lu_solve(int n, const double *LU, const int *piv, double *x)
{
    int i, j;
    for (i = 0; i < n; ++i)
        if (piv[i] != i) { double t = x[i]; x[i] = x[piv[i]]; x[piv[i]] = t; }
    for (i = 0; i < n; ++i)
        for (j = 0; j < i; ++j) x[i] -= LU[i * n + j] * x[j];
    for (i = n - 1; i >= 0; --i) {
        for (j = i + 1; j < n; ++j) x[i] -= LU[i * n + j] * x[j];
        x[i] /= LU[i * n + i];
    }
}

/* One equality-constrained QP (eq over_2 / matrix_vec) solved through the KKT LU:
 * out = argmin 1/2 x^T H x - q^T x  s.t. A x = b.   q, out: [n_v]; b: [4]. */
int orc_kkt_solve(const orc_problem *pr, const double *q, const double *b, double *out)
{
    int nv = pr->degree + 1, N = nv + 4, i, rc;
    double *K = malloc(sizeof(double) * N * N), *x = malloc(sizeof(double) * N);
    int *piv = malloc(sizeof(int) * N);
    rc = orc_kkt_matrix(pr, K);
    if (rc == 0) rc = orc_lu_factor(N, K, piv);
    if (rc == 0) {
        for (i = 0; i < nv; ++i) x[i] = q[i];
        for (i = 0; i < 4; ++i) x[nv + i] = b[i];
        orc_lu_solve(N, K, piv, x);
        for (i = 0; i < nv; ++i) out[i] = x[i];
    }
    free(K); free(x); free(piv);
    return rc;
}

/* The same QP by a second, independent route (test cross-check only): the four
 * boundary rows fix xi_0, xi_1, xi_2 and xi_n; the free block then solves
 * H_ff x_f = q_f - H_fb x_b by Cholesky. */
int orc_qp_nullspace(const orc_problem *pr, const double *q, const double *b, double *out)
{
    int n = pr->degree, nv = n + 1, nf = nv - 4, i, j, k;
    double T = pr->horizon;
    double *A = malloc(sizeof(double) * 4 * nv), *H = malloc(sizeof(double) * nv * nv);
    double *L = malloc(sizeof(double) * (nf > 0 ? nf * nf : 1));
    double *y = malloc(sizeof(double) * (nf > 0 ? nf : 1));
    int rc = orc_constraint_matrices(pr, A, H);
    if (rc != 0 || n < 3) { free(A); free(H); free(L); free(y); return -1; }
    out[0] = b[0];
    out[1] = b[0] + b[1] * T / n;
    out[2] = b[0] + 2.0 * b[1] * T / n + b[2] * T * T / ((double)n * (n - 1));
    out[n] = b[3];
    for (i = 0; i < nf; ++i) {
        int fi = 3 + i;
        y[i] = q[fi] - H[fi * nv + 0] * out[0] - H[fi * nv + 1] * out[1] -
               H[fi * nv + 2] * out[2] - H[fi * nv + n] * out[n];
        for (j = 0; j <= i; ++j) {
            double s = H[fi * nv + 3 + j];
            for (k = 0; k < j; ++k) s -= L[i * nf + k] * L[j * nf + k];
            if (i == j) {
                if (s <= 0.0) { free(A); free(H); free(L); free(y); return -1; }
                L[i * nf + i] = sqrt(s);
            } else {
                L[i * nf + j] = s / L[j * nf + j];
            }
        }
    }
    for (i = 0; i < nf; ++i) {
        for (k = 0; k < i; ++k) y[i] -= L[i * nf + k] * y[k];
        y[i] /= L[i * nf + i];
    }
    for (i = nf - 1; i >= 0; --i) {
        for (k = i + 1; k < nf; ++k) y[i] -= L[k * nf + i] * y[k];
        y[i] /= L[i * nf + i];
    }
    for (i = 0; i < nf; ++i) out[3 + i] = y[i];
    free(A); free(H); free(L); free(y);
    return 0;
}

/* ------------------------------------------------------------ polar steps -- */

/* Obstacle polar step for one (obstacle, time) pair: given x~ = p - c and the
 * semi-axes s, return alpha, beta, d (eqs zeta_2, compute_d_mij, d_max) and the
 * offset s .* d .* dir(alpha, beta), so that e = c + offset. */
void orc_polar_obstacle(int D, const double *xt, const double *s, double *alpha,
                        double *beta, double *d, double *off)
{
    double u[3] = {0, 0, 0}, rn = 0.0, al, be, dd, dir[3];
    int i;
    for (i = 0; i < D; ++i) { u[i] = xt[i] / s[i]; rn += u[i] * u[i]; }
    rn = sqrt(rn);
    al = atan2(u[1], u[0]);
    be = (D == 3) ? atan2(hypot(u[0], u[1]), u[2]) : M_PI / 2.0;
    dd = rn > 1.0 ? rn : 1.0;                     /* d >= 1 (eq collision_d) */
    if (g_fault == 5) dd = rn;                    /* planted: lower bound on d dropped */
    if (D == 3) {
        dir[0] = cos(al) * sin(be);
        dir[1] = sin(al) * sin(be);
        dir[2] = cos(be);
    } else {
        dir[0] = cos(al);
        dir[1] = sin(al);
    }
    for (i = 0; i < D; ++i) off[i] = s[i] * dd * dir[i];
    *alpha = al;
    *beta = be;
    *d = dd;
}

/* Velocity / acceleration polar step (eqs alpha_v, compute_dv): target of
 * magnitude bound * d, d = min(1, |v| / bound) in [0, 1], along (alpha, beta). */
void orc_polar_bound(int D, const double *v, double bound, double *e)
{
    double nrm = 0.0, al, be, dd, dir[3];
    int i;
    for (i = 0; i < D; ++i) nrm += v[i] * v[i];
    nrm = sqrt(nrm);
    al = atan2(v[1], v[0]);
    be = (D == 3) ? atan2(hypot(v[0], v[1]), v[2]) : M_PI / 2.0;
    dd = nrm / bound;
    if (dd > 1.0) dd = 1.0;
    if (D == 3) {
        dir[0] = cos(al) * sin(be);
        dir[1] = sin(al) * sin(be);
        dir[2] = cos(be);
    } else {
        dir[0] = cos(al);
        dir[1] = sin(al);
    }
    for (i = 0; i < D; ++i) e[i] = bound * dd * dir[i];
}

/* ------------------------------------------------------ one trajectory -- */

typedef struct {
    const orc_problem *pr;
    int nv, np, D;
    const double *P, *Pd, *Pdd;       /* [n_p][n_v] */
    const double *oc, *ow, *os;       /* obstacles [n_o][D] */
} orc_ctx;

/* Steps 1-4 at coefficients xb ([D][n_v]).  Outputs (any may be NULL):
 *   FtE[D][n_v] = F^T e, FtR[D][n_v] = F^T (F xb - e), r2 = |F xb - e|^2,
 *   rmax = max |component of F xb - e|. */
static void polar_and_residual(const orc_ctx *c, const double *xb, double *FtE,
                               double *FtR, double *r2, double *rmax)
{
    const orc_problem *pr = c->pr;
    int D = c->D, nv = c->nv, np = c->np, t, j, ax, m;
    double acc = 0.0, mx = 0.0;
    if (FtE) memset(FtE, 0, sizeof(double) * D * nv);
    if (FtR) memset(FtR, 0, sizeof(double) * D * nv);
    for (t = 0; t < np; ++t) {
        double tk = (double)t * pr->horizon / (double)(np - 1);
        double p[3] = {0, 0, 0}, v[3] = {0, 0, 0}, a[3] = {0, 0, 0};
        double eo[3] = {0, 0, 0}, ro[3] = {0, 0, 0}, ev[3] = {0, 0, 0}, ea[3] = {0, 0, 0};
        double rv[3] = {0, 0, 0}, ra[3] = {0, 0, 0};
        for (ax = 0; ax < D; ++ax)
            for (m = 0; m < nv; ++m) {
                p[ax] += c->P[t * nv + m] * xb[ax * nv + m];
                v[ax] += c->Pd[t * nv + m] * xb[ax * nv + m];
                a[ax] += c->Pdd[t * nv + m] * xb[ax * nv + m];
            }
        for (j = 0; j < pr->n_obs; ++j) {
            double ctr[3], xt[3], off[3], al, be, dd;
            for (ax = 0; ax < D; ++ax) {
                ctr[ax] = c->oc[j * D + ax] + c->ow[j * D + ax] * tk;
                xt[ax] = p[ax] - ctr[ax];
            }
            orc_polar_obstacle(D, xt, &c->os[j * D], &al, &be, &dd, off);
            for (ax = 0; ax < D; ++ax) {
                double e = ctr[ax] + off[ax], r = p[ax] - e;
                eo[ax] += e;
                ro[ax] += r;
                acc += r * r;
                if (fabs(r) > mx) mx = fabs(r);
            }
        }
        if (pr->v_max > 0.0) {
            orc_polar_bound(D, v, pr->v_max, ev);
            for (ax = 0; ax < D; ++ax) {
                rv[ax] = v[ax] - ev[ax];
                acc += rv[ax] * rv[ax];
                if (fabs(rv[ax]) > mx) mx = fabs(rv[ax]);
            }
        }
        if (pr->a_max > 0.0) {
            orc_polar_bound(D, a, pr->a_max, ea);
            for (ax = 0; ax < D; ++ax) {
                ra[ax] = a[ax] - ea[ax];
                acc += ra[ax] * ra[ax];
                if (fabs(ra[ax]) > mx) mx = fabs(ra[ax]);
            }
        }
        /* workspace bounds (Paper III, eq bound_con and the slack step of its AM list):
         * per axis the row values g = G xb are (-p, p) with bounds tau = (-lo, hi); the
         * slack s = max(0, -g + tau) makes e_G = tau - s and the residual r_G = g - e_G.
         * F^T e gains G^T e_G = P^T (e_hi - e_lo); F^T r gains P^T (r_hi - r_lo). */
        double ew[3] = {0, 0, 0}, rw[3] = {0, 0, 0};
        if (pr->workspace)
            for (ax = 0; ax < D; ++ax) {
                double g_lo = -p[ax], t_lo = -pr->ws_lo[ax];
                double g_hi = p[ax], t_hi = pr->ws_hi[ax];
                double s_lo = fmax(0.0, -g_lo + t_lo), s_hi = fmax(0.0, -g_hi + t_hi);
                if (g_fault == 10) s_lo = fmax(0.0, g_lo - t_lo);   /* planted: slack sign */
                double e_lo = t_lo - s_lo, e_hi = t_hi - s_hi;
                double r_lo = g_lo - e_lo, r_hi = g_hi - e_hi;
                ew[ax] = e_hi - e_lo;
                rw[ax] = r_hi - r_lo;
                acc += r_lo * r_lo + r_hi * r_hi;
                if (fabs(r_lo) > mx) mx = fabs(r_lo);
                if (fabs(r_hi) > mx) mx = fabs(r_hi);
            }
        for (ax = 0; ax < D; ++ax)
            for (m = 0; m < nv; ++m) {
                /* F^T stacks P^T once per obstacle, then Pd^T and Pdd^T */
                double pm = c->P[t * nv + m];
                if (g_fault == 3) pm = c->P[t * nv + (nv - 1 - m)]; /* planted: column order */
                if (FtE) {
                    FtE[ax * nv + m] += pm * eo[ax] + c->P[t * nv + m] * ew[ax];
                    if (g_fault != 2) FtE[ax * nv + m] += c->Pd[t * nv + m] * ev[ax];
                    FtE[ax * nv + m] += c->Pdd[t * nv + m] * ea[ax];
                }
                if (FtR)
                    FtR[ax * nv + m] += pm * ro[ax] + c->P[t * nv + m] * rw[ax] + c->Pd[t * nv + m] * rv[ax] +
                                        c->Pdd[t * nv + m] * ra[ax];
            }
    }
    if (r2) *r2 = acc;
    if (rmax) *rmax = mx;
}

/* ---------------------------------------------------------------- public -- */

/* Projects B samples.  Layouts (row-major, float64):
 *   xi, xi_bar, lam : [B][D][n_v]   (xi_bar, lam: in = initial values, out = final)
 *   oc, ow, os      : [n_o][D] obstacle centre at t = 0, velocity, semi-axes
 *   bnd             : [D][4] = (x0, v0, a0, xf) per axis
 *   res_trace       : [iters][B] 2-norm of F xb^k - e^{k+1} (may be NULL)
 *   resmax_trace    : [iters][B] max-abs of the same vector (may be NULL)
 *   freeze_lambda   : 1 keeps lam fixed (test variant)
 *   n_threads       : OpenMP threads over trajectories (<= 0: runtime default)
 * Returns 0, or -1 for an invalid problem / singular KKT. */
int orc_project(const orc_problem *pr, int B, const double *xi, const double *oc,
                const double *ow, const double *os, const double *bnd, double *xi_bar,
                double *lam, int iters, double *res_trace, double *resmax_trace,
                int freeze_lambda, int n_threads)
{
    int D = pr->dims, nv = pr->degree + 1, np = pr->n_steps, N = nv + 4;
    double *P, *Pd, *Pdd, *K;
    int *piv, rc = 0, i;
    orc_ctx c;
    if ((D != 2 && D != 3) || pr->degree < 3 || np < 2 || B < 0 || iters < 0) return -1;
    P = malloc(sizeof(double) * np * nv);
    Pd = malloc(sizeof(double) * np * nv);
    Pdd = malloc(sizeof(double) * np * nv);
    K = malloc(sizeof(double) * N * N);
    piv = malloc(sizeof(int) * N);
    if (orc_bernstein(pr->degree, np, pr->horizon, P, Pd, Pdd) != 0 ||
        orc_kkt_matrix(pr, K) != 0 || orc_lu_factor(N, K, piv) != 0) {
        rc = -1;
        goto done;
    }
    c.pr = pr; c.nv = nv; c.np = np; c.D = D;
    c.P = P; c.Pd = Pd; c.Pdd = Pdd; c.oc = oc; c.ow = ow; c.os = os;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (i = 0; i < B; ++i) {
        double *xb = xi_bar + (size_t)i * D * nv, *lm = lam + (size_t)i * D * nv;
        const double *x0 = xi + (size_t)i * D * nv;
        double *FtE = malloc(sizeof(double) * D * nv), *FtR = malloc(sizeof(double) * D * nv);
        double *rhs = malloc(sizeof(double) * N);
        double *lm_old = malloc(sizeof(double) * D * nv);
        int k, ax, m;
        for (k = 0; k < iters; ++k) {
            double r2, rmax;
            const double *lq = lm;
            polar_and_residual(&c, xb, FtE, FtR, &r2, &rmax);
            if (res_trace) res_trace[(size_t)k * B + i] = sqrt(r2);
            if (resmax_trace) resmax_trace[(size_t)k * B + i] = rmax;
            if (g_fault == 8) {                                   /* planted: QP takes lambda^k */
                memcpy(lm_old, lm, sizeof(double) * D * nv);
                lq = lm_old;
            }
            if (!freeze_lambda)
                for (m = 0; m < D * nv; ++m) {
                    if (g_fault == 4) lm[m] += pr->rho * FtR[m];   /* planted: sign */
                    else lm[m] -= pr->rho * FtR[m];
                }
            for (ax = 0; ax < D; ++ax) {
                for (m = 0; m < nv; ++m) {
                    double fe = pr->rho * FtE[ax * nv + m];
                    if (g_fault == 1) fe = -fe;                    /* planted: printed sign */
                    rhs[m] = x0[ax * nv + m] + lq[ax * nv + m] + fe;
                }
                for (m = 0; m < 4; ++m) rhs[nv + m] = bnd[ax * 4 + m];
                orc_lu_solve(N, K, piv, rhs);
                for (m = 0; m < nv; ++m) xb[ax * nv + m] = rhs[m];
            }
        }
        free(FtE); free(FtR); free(rhs); free(lm_old);
    }
done:
    free(P); free(Pd); free(Pdd); free(K); free(piv);
    return rc;
}

/* ------------------------------------------------------ rho-continuation -- */

/* Penalty continuation (thesis ch. 4, Alg 1: the penalty weights are raised while the
 * residuals stay above a threshold; ch. 7: the QP inverse is precomputed for ten
 * increasing penalties and used in later iterations).  Readings taken here: a ladder of
 * n_levels penalties rho_l = rho * growth^l; per trajectory a level (starting at the
 * state passed in), an iteration count since the last check and the residual at that
 * check (0 before the first check).  Iteration k runs steps 1-6 with rho_level in the
 * multiplier update and in the QP (its own KKT matrix [I + rho_l F^T F, A^T; A, 0]);
 * then the count is raised, and when it reaches `window` the check compares res^k with
 * the reference: if res^k > tol and res^k > stall * reference, the level goes up by one
 * (at most n_levels - 1); the reference becomes res^k and the count restarts.  (So the
 * first check raises the level whenever the residual is still above tol: the threshold
 * rule of Alg 1, with no earlier residual to show progress.)  With one level (or
 * growth 1) this is orc_project exactly. */
typedef struct {
    int n_levels;      /* >= 1 */
    double growth;     /* rho_l = rho * growth^l */
    int window;        /* iterations between checks, >= 1 */
    double stall;      /* raise the level when res > stall * res at the previous check */
    double tol;        /* ... and res > tol */
} orc_cont;

int orc_project_cont(const orc_problem *pr, const orc_cont *cc, int B, const double *xi,
                     const double *oc, const double *ow, const double *os, const double *bnd,
                     double *xi_bar, double *lam, int *level, int *count, double *ref, int iters,
                     double *res_trace, int *level_trace, int n_threads)
{
    int D = pr->dims, nv = pr->degree + 1, np = pr->n_steps, N = nv + 4, L = cc->n_levels;
    double *P, *Pd, *Pdd, *K, *rhos;
    int *piv, rc = 0, i, l;
    orc_ctx c;
    if ((D != 2 && D != 3) || pr->degree < 3 || np < 2 || B < 0 || iters < 0 || L < 1 ||
        cc->window < 1 || !(cc->growth >= 1.0))
        return -1;
    P = malloc(sizeof(double) * np * nv);
    Pd = malloc(sizeof(double) * np * nv);
    Pdd = malloc(sizeof(double) * np * nv);
    K = malloc(sizeof(double) * N * N * L);
    piv = malloc(sizeof(int) * N * L);
    rhos = malloc(sizeof(double) * L);
    if (orc_bernstein(pr->degree, np, pr->horizon, P, Pd, Pdd) != 0) {
        rc = -1;
        goto done;
    }
    /* one KKT matrix and LU per penalty of the ladder */
    for (l = 0; l < L; ++l) {
        orc_problem pl = *pr;
        rhos[l] = pr->rho * pow(cc->growth, (double)l);
        pl.rho = rhos[l];
        if (orc_kkt_matrix(&pl, K + (size_t)l * N * N) != 0 ||
            orc_lu_factor(N, K + (size_t)l * N * N, piv + (size_t)l * N) != 0) {
            rc = -1;
            goto done;
        }
    }
    c.pr = pr; c.nv = nv; c.np = np; c.D = D;
    c.P = P; c.Pd = Pd; c.Pdd = Pdd; c.oc = oc; c.ow = ow; c.os = os;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (i = 0; i < B; ++i) {
        double *xb = xi_bar + (size_t)i * D * nv, *lm = lam + (size_t)i * D * nv;
        const double *x0 = xi + (size_t)i * D * nv;
        double *FtE = malloc(sizeof(double) * D * nv), *FtR = malloc(sizeof(double) * D * nv);
        double *rhs = malloc(sizeof(double) * N);
        int k, ax, m;
        for (k = 0; k < iters; ++k) {
            double r2, res;
            const int lv = level[i];
            const double rho = rhos[lv];
            const double *Kl = K + (size_t)lv * N * N;
            const int *pl = piv + (size_t)lv * N;
            polar_and_residual(&c, xb, FtE, FtR, &r2, NULL);
            res = sqrt(r2);
            if (res_trace) res_trace[(size_t)k * B + i] = res;
            if (level_trace) level_trace[(size_t)k * B + i] = lv;
            for (m = 0; m < D * nv; ++m) lm[m] -= rho * FtR[m];
            for (ax = 0; ax < D; ++ax) {
                for (m = 0; m < nv; ++m) rhs[m] = x0[ax * nv + m] + lm[ax * nv + m] + rho * FtE[ax * nv + m];
                for (m = 0; m < 4; ++m) rhs[nv + m] = bnd[ax * 4 + m];
                orc_lu_solve(N, Kl, pl, rhs);
                for (m = 0; m < nv; ++m) xb[ax * nv + m] = rhs[m];
            }
            /* the check after the iteration decides the penalty of the next one */
            count[i] += 1;
            if (count[i] >= cc->window) {
                int up = res > cc->tol && res > cc->stall * ref[i];
                if (g_fault == 9) up = res > cc->tol && res < cc->stall * ref[i];
                if (up && level[i] < L - 1) level[i] += 1;
                ref[i] = res;
                count[i] = 0;
            }
        }
        free(FtE); free(FtR); free(rhs);
    }
done:
    free(P); free(Pd); free(Pdd); free(K); free(piv); free(rhos);
    return rc;
}

/* Steps 1-4 only, at the given coefficients: res_l2[B], res_max[B]. */
int orc_residuals(const orc_problem *pr, int B, const double *xi_bar, const double *oc,
                  const double *ow, const double *os, double *res_l2, double *res_max,
                  int n_threads)
{
    int D = pr->dims, nv = pr->degree + 1, np = pr->n_steps, i;
    double *P, *Pd, *Pdd;
    orc_ctx c;
    if ((D != 2 && D != 3) || pr->degree < 2 || np < 2 || B < 0) return -1;
    P = malloc(sizeof(double) * np * nv);
    Pd = malloc(sizeof(double) * np * nv);
    Pdd = malloc(sizeof(double) * np * nv);
    if (orc_bernstein(pr->degree, np, pr->horizon, P, Pd, Pdd) != 0) {
        free(P); free(Pd); free(Pdd);
        return -1;
    }
    c.pr = pr; c.nv = nv; c.np = np; c.D = D;
    c.P = P; c.Pd = Pd; c.Pdd = Pdd; c.oc = oc; c.ow = ow; c.os = os;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (i = 0; i < B; ++i) {
        double r2, mx;
        polar_and_residual(&c, xi_bar + (size_t)i * D * nv, NULL, NULL, &r2, &mx);
        res_l2[i] = sqrt(r2);
        if (res_max) res_max[i] = mx;
    }
    free(P); free(Pd); free(Pdd);
    return 0;
}

/* F^T e and F^T r at one coefficient vector (test access to steps 1-4). */
int orc_polar_products(const orc_problem *pr, const double *xb, const double *oc,
                       const double *ow, const double *os, double *FtE, double *FtR,
                       double *r2)
{
    int D = pr->dims, nv = pr->degree + 1, np = pr->n_steps;
    double *P = malloc(sizeof(double) * np * nv), *Pd = malloc(sizeof(double) * np * nv),
           *Pdd = malloc(sizeof(double) * np * nv);
    orc_ctx c;
    if (orc_bernstein(pr->degree, np, pr->horizon, P, Pd, Pdd) != 0) {
        free(P); free(Pd); free(Pdd);
        return -1;
    }
    c.pr = pr; c.nv = nv; c.np = np; c.D = D;
    c.P = P; c.Pd = Pd; c.Pdd = Pdd; c.oc = oc; c.ow = ow; c.os = os;
    polar_and_residual(&c, xb, FtE, FtR, r2, NULL);
    free(P); free(Pd); free(Pdd);
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------ multi-agent -- */
/*
 * Joint projection of N agents (thesis ch. 7, Paper IV, in the projection form of
 * ch. 6).  Each agent a has its own trajectory xi_a ([D][n_v]), its own boundary
 * rows, and the single-robot rows of the problem (every obstacle, velocity and
 * acceleration bounds).  In addition every unordered pair a < b and time t has the
 * row  p_a(t) - p_b(t) = e_ab(t)  with the polar target of a sphere of combined
 * radius R around the other agent: e_ab = R d dir(alpha, beta), d >= 1, where
 * alpha, beta, d follow the same closed forms as an obstacle (eqs sphere_proposed,
 * com_alpha_i, com_beta_i, com_d_i; a pair is counted once).  The AM steps are those
 * of the single robot with F now the joint matrix:
 *   (F^T e)_a = (single-robot part)_a + sum_{b > a} P^T e_ab - sum_{b < a} P^T e_ba
 * and likewise for F^T r; the multiplier lam_a <- lam_a - rho (F^T r)_a; the QP is
 * the joint KKT system per axis,
 *   [H_J  A_J^T; A_J  0] [xb; nu] = [xi + lam + rho F^T e; b]
 * with H_J = blockdiag(H) + rho sum_{a<b} (E_a - E_b)^T P^T P (E_a - E_b) assembled
 * pair by pair here (E_a selects agent a's block) and A_J = blockdiag(A).
 */

/* Pair polar rows at joint coefficients xb ([N][D][n_v]); adds to FtE, FtR
 * ([N][D][n_v]), r2 and rmax.  R = combined radius. */
static void pair_rows(const orc_ctx *c, int N, double R, const double *xb, double *FtE,
                      double *FtR, double *r2, double *rmax)
{
    int D = c->D, nv = c->nv, np = c->np, t, a, b, ax, m;
    double *p = malloc(sizeof(double) * N * D);
    double s[3] = {R, R, R};
    for (t = 0; t < np; ++t) {
        for (a = 0; a < N; ++a)
            for (ax = 0; ax < D; ++ax) {
                double acc = 0.0;
                for (m = 0; m < nv; ++m) acc += c->P[t * nv + m] * xb[(a * D + ax) * nv + m];
                p[a * D + ax] = acc;
            }
        for (a = 0; a < N; ++a)
            for (b = a + 1; b < N; ++b) {
                double xt[3], off[3], al, be, dd;
                for (ax = 0; ax < D; ++ax) xt[ax] = p[a * D + ax] - p[b * D + ax];
                orc_polar_obstacle(D, xt, s, &al, &be, &dd, off);
                for (ax = 0; ax < D; ++ax) {
                    double r = xt[ax] - off[ax];
                    double sb = (g_fault == 6) ? 1.0 : -1.0;   /* planted: sign for agent b */
                    *r2 += r * r;
                    if (fabs(r) > *rmax) *rmax = fabs(r);
                    for (m = 0; m < nv; ++m) {
                        double pm = c->P[t * nv + m];
                        if (FtE) {
                            FtE[(a * D + ax) * nv + m] += pm * off[ax];
                            FtE[(b * D + ax) * nv + m] += sb * pm * off[ax];
                        }
                        if (FtR) {
                            FtR[(a * D + ax) * nv + m] += pm * r;
                            FtR[(b * D + ax) * nv + m] += sb * pm * r;
                        }
                    }
                }
            }
    }
    free(p);
}

/* Joint KKT matrix of N agents (one axis), row-major, size N (n_v + 4):
 * variables agent-major, then the 4 N boundary multipliers. */
int orc_agents_kkt_matrix(const orc_problem *pr, int N, double *K)
{
    int nv = pr->degree + 1, np = pr->n_steps, S = N * (nv + 4), a, b, i, j, k;
    double *A = malloc(sizeof(double) * 4 * nv), *H = malloc(sizeof(double) * nv * nv);
    double *P = malloc(sizeof(double) * np * nv), *Pd = malloc(sizeof(double) * np * nv),
           *Pdd = malloc(sizeof(double) * np * nv), *G = malloc(sizeof(double) * nv * nv);
    int rc = orc_constraint_matrices(pr, A, H);
    if (rc == 0) rc = orc_bernstein(pr->degree, np, pr->horizon, P, Pd, Pdd);
    if (rc == 0) {
        for (i = 0; i < nv; ++i)
            for (j = 0; j < nv; ++j) {
                double g = 0.0;
                for (k = 0; k < np; ++k) g += P[k * nv + i] * P[k * nv + j];
                G[i * nv + j] = pr->rho * g;
            }
        memset(K, 0, sizeof(double) * S * S);
        for (a = 0; a < N; ++a)
            for (i = 0; i < nv; ++i)
                for (j = 0; j < nv; ++j) K[(a * nv + i) * S + a * nv + j] = H[i * nv + j];
        /* rho (P_a - P_b)^T (P_a - P_b) for every pair */
        for (a = 0; a < N; ++a)
            for (b = a + 1; b < N; ++b)
                for (i = 0; i < nv; ++i)
                    for (j = 0; j < nv; ++j) {
                        double g = G[i * nv + j];
                        K[(a * nv + i) * S + a * nv + j] += g;
                        K[(b * nv + i) * S + b * nv + j] += (g_fault == 7) ? 2.0 * g : g;
                        K[(a * nv + i) * S + b * nv + j] -= g;
                        K[(b * nv + i) * S + a * nv + j] -= g;
                    }
        for (a = 0; a < N; ++a)
            for (i = 0; i < 4; ++i)
                for (j = 0; j < nv; ++j) {
                    K[(N * nv + a * 4 + i) * S + a * nv + j] = A[i * nv + j];
                    K[(a * nv + j) * S + N * nv + a * 4 + i] = A[i * nv + j];
                }
    }
    free(A); free(H); free(P); free(Pd); free(Pdd); free(G);
    return rc;
}

/* One joint QP (one axis): out = argmin sum_a 1/2 x_a^T H x_a
 *   + rho/2 sum_{a<b} |P (x_a - x_b)|^2 - sum_a q_a^T x_a   s.t. A x_a = b_a.
 * q, out: [N][n_v]; b: [N][4]. */
int orc_agents_qp(const orc_problem *pr, int N, const double *q, const double *b, double *out)
{
    int nv = pr->degree + 1, S = N * (nv + 4), i, rc;
    double *K = malloc(sizeof(double) * S * S), *x = malloc(sizeof(double) * S);
    int *piv = malloc(sizeof(int) * S);
    rc = orc_agents_kkt_matrix(pr, N, K);
    if (rc == 0) rc = orc_lu_factor(S, K, piv);
    if (rc == 0) {
        for (i = 0; i < N * nv; ++i) x[i] = q[i];
        for (i = 0; i < 4 * N; ++i) x[N * nv + i] = b[i];
        orc_lu_solve(S, K, piv, x);
        for (i = 0; i < N * nv; ++i) out[i] = x[i];
    }
    free(K); free(x); free(piv);
    return rc;
}

/* Steps 1-4 of the joint problem at xb ([N][D][n_v]): FtE, FtR ([N][D][n_v], may be
 * NULL), r2 = |F xb - e|^2 over all rows of all agents and pairs, rmax. */
static void agents_polar(const orc_ctx *c, int N, double R, const double *xb, double *FtE,
                         double *FtR, double *r2, double *rmax)
{
    int D = c->D, nv = c->nv, a;
    double acc = 0.0, mx = 0.0;
    for (a = 0; a < N; ++a) {
        double ra, ma;
        polar_and_residual(c, xb + (size_t)a * D * nv, FtE ? FtE + (size_t)a * D * nv : NULL,
                           FtR ? FtR + (size_t)a * D * nv : NULL, &ra, &ma);
        acc += ra;
        if (ma > mx) mx = ma;
    }
    pair_rows(c, N, R, xb, FtE, FtR, &acc, &mx);
    *r2 = acc;
    *rmax = mx;
}

static int agents_ctx(const orc_problem *pr, const double *oc, const double *ow,
                      const double *os, orc_ctx *c, double **bufs)
{
    int nv = pr->degree + 1, np = pr->n_steps;
    bufs[0] = malloc(sizeof(double) * np * nv);
    bufs[1] = malloc(sizeof(double) * np * nv);
    bufs[2] = malloc(sizeof(double) * np * nv);
    if (orc_bernstein(pr->degree, np, pr->horizon, bufs[0], bufs[1], bufs[2]) != 0) return -1;
    c->pr = pr; c->nv = nv; c->np = np; c->D = pr->dims;
    c->P = bufs[0]; c->Pd = bufs[1]; c->Pdd = bufs[2]; c->oc = oc; c->ow = ow; c->os = os;
    return 0;
}

/* F^T e, F^T r and |r|^2 of the joint problem at one joint coefficient vector. */
int orc_agents_polar_products(const orc_problem *pr, int N, double R, const double *xb,
                              const double *oc, const double *ow, const double *os,
                              double *FtE, double *FtR, double *r2)
{
    int D = pr->dims, nv = pr->degree + 1, rc;
    double *bufs[3] = {NULL, NULL, NULL}, mx;
    orc_ctx c;
    rc = agents_ctx(pr, oc, ow, os, &c, bufs);
    if (rc == 0) {
        if (FtE) memset(FtE, 0, sizeof(double) * N * D * nv);
        if (FtR) memset(FtR, 0, sizeof(double) * N * D * nv);
        agents_polar(&c, N, R, xb, FtE, FtR, r2, &mx);
    }
    free(bufs[0]); free(bufs[1]); free(bufs[2]);
    return rc;
}

/* Projects B joint samples of N agents.  Layouts (row-major, float64):
 *   xi, xi_bar, lam : [B][N][D][n_v];  bnd : [N][D][4];  obstacles as orc_project;
 *   res_trace, resmax_trace : [iters][B] (may be NULL).  R = combined radius. */
int orc_project_agents(const orc_problem *pr, int N, double R, int B, const double *xi,
                       const double *oc, const double *ow, const double *os,
                       const double *bnd, double *xi_bar, double *lam, int iters,
                       double *res_trace, double *resmax_trace, int n_threads)
{
    int D = pr->dims, nv = pr->degree + 1, S = N * (nv + 4), rc = 0, i;
    double *bufs[3] = {NULL, NULL, NULL}, *K = NULL;
    int *piv = NULL;
    orc_ctx c;
    if ((D != 2 && D != 3) || pr->degree < 3 || pr->n_steps < 2 || N < 1 || B < 0 ||
        iters < 0 || !(R >= 0.0))
        return -1;
    K = malloc(sizeof(double) * S * S);
    piv = malloc(sizeof(int) * S);
    if (agents_ctx(pr, oc, ow, os, &c, bufs) != 0 || orc_agents_kkt_matrix(pr, N, K) != 0 ||
        orc_lu_factor(S, K, piv) != 0) {
        rc = -1;
        goto done;
    }
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (i = 0; i < B; ++i) {
        size_t J = (size_t)N * D * nv;
        double *xb = xi_bar + i * J, *lm = lam + i * J;
        const double *x0 = xi + i * J;
        double *FtE = malloc(sizeof(double) * J), *FtR = malloc(sizeof(double) * J);
        double *rhs = malloc(sizeof(double) * S);
        int k, a, ax, m;
        for (k = 0; k < iters; ++k) {
            double r2, rmax;
            memset(FtE, 0, sizeof(double) * J);
            memset(FtR, 0, sizeof(double) * J);
            agents_polar(&c, N, R, xb, FtE, FtR, &r2, &rmax);
            if (res_trace) res_trace[(size_t)k * B + i] = sqrt(r2);
            if (resmax_trace) resmax_trace[(size_t)k * B + i] = rmax;
            for (m = 0; m < (int)J; ++m) lm[m] -= pr->rho * FtR[m];
            for (ax = 0; ax < D; ++ax) {
                for (a = 0; a < N; ++a) {
                    for (m = 0; m < nv; ++m) {
                        size_t g = ((size_t)a * D + ax) * nv + m;
                        rhs[a * nv + m] = x0[g] + lm[g] + pr->rho * FtE[g];
                    }
                    for (m = 0; m < 4; ++m) rhs[N * nv + a * 4 + m] = bnd[(a * D + ax) * 4 + m];
                }
                orc_lu_solve(S, K, piv, rhs);
                for (a = 0; a < N; ++a)
                    for (m = 0; m < nv; ++m) xb[((size_t)a * D + ax) * nv + m] = rhs[a * nv + m];
            }
        }
        free(FtE); free(FtR); free(rhs);
    }
done:
    free(bufs[0]); free(bufs[1]); free(bufs[2]); free(K); free(piv);
    return rc;
}

/* Joint residuals at xb ([B][N][D][n_v]): res_l2[B], res_max[B]. */
int orc_residuals_agents(const orc_problem *pr, int N, double R, int B, const double *xi_bar,
                         const double *oc, const double *ow, const double *os, double *res_l2,
                         double *res_max, int n_threads)
{
    int D = pr->dims, nv = pr->degree + 1, rc, i;
    double *bufs[3] = {NULL, NULL, NULL};
    orc_ctx c;
    rc = agents_ctx(pr, oc, ow, os, &c, bufs);
    if (rc == 0) {
#ifdef _OPENMP
        if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
        for (i = 0; i < B; ++i) {
            double r2, mx;
            agents_polar(&c, N, R, xi_bar + (size_t)i * N * D * nv, NULL, NULL, &r2, &mx);
            res_l2[i] = sqrt(r2);
            if (res_max) res_max[i] = mx;
        }
    }
    free(bufs[0]); free(bufs[1]); free(bufs[2]);
    return rc;
}
