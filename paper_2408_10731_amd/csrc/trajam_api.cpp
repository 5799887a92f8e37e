// C-ABI layer of the MI355X AM projection: argument validation, the one-time FP64
// precompute of the fixed matrices, device constants, and kernel launches.
//
// Fixed matrices (thesis ch. 6, "Scalability": M needs a one-time computation):
//  * Bernstein basis P, Pd, Pdd at t_k = k T / (n_p - 1) (eq parameter), evaluated
//    here with the triangular recurrence B_{m,r} = (1 - tau) B_{m,r-1} + tau B_{m-1,r-1},
//    which yields the degree n, n-1 and n-2 rows the derivatives need.
//  * H = I + rho F^T F with F^T F = n_o P^T P + Pd^T Pd + Pdd^T Pdd (eq f_e stacks P
//    once per obstacle), identical for every axis.
//  * The four boundary rows [P_0; Pd_0; Pdd_0; P_{-1}] touch only coefficients
//    0, 1, 2 and n of a Bernstein basis, so the KKT system of eq matrix_vec splits:
//    those four coefficients are fixed by the boundary values in closed form and the
//    n - 3 free ones solve H_ff x_f = q_f - H_fb x_b.  The library stores
//    W_ff = H_ff^{-1} (Cholesky, FP64) and the operator
//        W = [ W_ff | -W_ff H_fb ]   (n - 3) x (n + 1), columns in coefficient order,
//    and applies it in delta form: with g = q - H xb^k (the KKT defect of the
//    current iterate) and Delta_b = xb*_b - xb^k_b,
//        xb^{k+1}_f = xb^k_f + W_ff (g_f - H_fb Delta_b),   xb^{k+1}_b = xb*_b.
//    This equals the KKT solve exactly; in reduced precision the product only
//    touches the defect, which tends to zero.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/trajam.h"
#include "am_internal.h"

using trajam::AmArgs;

namespace {
thread_local std::string g_init_err;
}

namespace trajam {
void set_thread_error(const std::string &msg) { g_init_err = msg; }
}

struct trajam_solver {
    trajam_problem prob;
    int nv, nf, nvp, tpad, tb;
    int variant;  // trajam::kVariant*
    bool packed = false;   // obstacles set with trajam_set_obstacles
    bool dynamic = false;  // ... with velocities
    int device;
    // host FP64 copies
    std::vector<double> P, Pd, Pdd, H, W, Wff;
    // device constants (precision scalar)
    void *d_phi = nullptr;   // [3][n_p][nvp]
    void *d_W = nullptr;     // [nvp][nvp] (rows >= nf zero)
    void *d_obs = nullptr;   // [n_o][REC]
    void *d_soa = nullptr;   // [groups][fields][group]
    void *d_bf16 = nullptr;  // BF16_REFINE: Whi, Wlo [16][16] uint16 each
    void *d_Hff = nullptr;   // BF16_REFINE: [16][16] float
    // multi-agent problems
    void *d_W2 = nullptr;    // [nvp][nvp] QP operator of H + n_agents rho P^T P
    double qp_rho = 0.0;     // contraction of the QP step in the solver's precision
    void *d_xiBag = nullptr; // [n_agents][D][4] boundary coefficients per agent
    std::vector<double> bnd_cache;  // boundary rows the device copy was built from
    // penalty continuation (trajam_set_continuation)
    trajam_continuation cont{};
    bool cont_on = false;
    void *d_cont_W = nullptr;    // [levels][nvp][nvp]
    void *d_cont_rho = nullptr;  // [levels]
    std::string err;
};

namespace {

int pad_coeffs(int nv) { return nv <= 8 ? 8 : (nv <= 12 ? 12 : 16); }

trajam_status fail(trajam_solver *s, trajam_status st, const std::string &msg)
{
    if (s) s->err = msg;
    else g_init_err = msg;
    return st;
}

trajam_status validate(const trajam_problem *p, std::string &why)
{
    if (!p) { why = "problem is NULL"; return TRAJAM_ERR_INVALID; }
    if (p->dims != 2 && p->dims != 3) { why = "dims must be 2 or 3"; return TRAJAM_ERR_INVALID; }
    if (p->degree < 3 || p->degree + 1 > trajam::kMaxCoeffs) {
        why = "degree must be in [3, 15]";
        return TRAJAM_ERR_INVALID;
    }
    if (p->n_steps < p->degree + 1 || p->n_steps > trajam::kMaxThreads) {
        why = "n_steps must be in [degree + 1, 256]";
        return TRAJAM_ERR_INVALID;
    }
    if (!(p->horizon > 0.0) || !std::isfinite(p->horizon)) {
        why = "horizon must be finite and > 0";
        return TRAJAM_ERR_INVALID;
    }
    if (!(p->rho > 0.0) || !std::isfinite(p->rho)) { why = "rho must be finite and > 0"; return TRAJAM_ERR_INVALID; }
    if (!std::isfinite(p->v_max) || !std::isfinite(p->a_max)) {
        why = "v_max and a_max must be finite";
        return TRAJAM_ERR_INVALID;
    }
    if (p->n_obstacles < 0) { why = "n_obstacles must be >= 0"; return TRAJAM_ERR_INVALID; }
    if (p->max_batch < 1) { why = "max_batch must be >= 1"; return TRAJAM_ERR_INVALID; }
    if (p->precision != TRAJAM_FP64 && p->precision != TRAJAM_FP32 &&
        p->precision != TRAJAM_BF16_REFINE) {
        why = "unknown precision";
        return TRAJAM_ERR_INVALID;
    }
    if (p->obstacle_model != TRAJAM_ELLIPSOID && p->obstacle_model != TRAJAM_SPHERE) {
        why = "unknown obstacle model";
        return TRAJAM_ERR_INVALID;
    }
    if (p->workspace != 0 && p->workspace != 1) { why = "workspace must be 0 or 1"; return TRAJAM_ERR_INVALID; }
    if (p->workspace)
        for (int ax = 0; ax < p->dims; ++ax)
            if (!std::isfinite(p->ws_lo[ax]) || !std::isfinite(p->ws_hi[ax]) || !(p->ws_lo[ax] <= p->ws_hi[ax])) {
                why = "workspace bounds must be finite with lo <= hi";
                return TRAJAM_ERR_INVALID;
            }
    if (p->n_agents < 1 || p->n_agents > 64) { why = "n_agents must be in [1, 64]"; return TRAJAM_ERR_INVALID; }
    if (p->n_agents > 1) {
        if (!(p->agent_radius > 0.0) || !std::isfinite(p->agent_radius)) {
            why = "agent_radius must be finite and > 0";
            return TRAJAM_ERR_INVALID;
        }
        if (p->precision == TRAJAM_BF16_REFINE) {
            why = "multi-agent problems run in FP64 or FP32";
            return TRAJAM_ERR_UNSUPPORTED;
        }
        if (p->degree + 1 > 12) { why = "multi-agent problems need degree <= 11"; return TRAJAM_ERR_UNSUPPORTED; }
    }
    return TRAJAM_OK;
}

// Bernstein rows of degree n, n-1, n-2 at tau by the triangular recurrence.
void bernstein_rows(int n, double tau, std::vector<double> &bn, std::vector<double> &bn1,
                    std::vector<double> &bn2)
{
    std::vector<double> row(n + 1, 0.0), next(n + 1, 0.0);
    row[0] = 1.0;  // degree 0
    bn1.assign(n + 1, 0.0);
    bn2.assign(n + 1, 0.0);
    for (int r = 1; r <= n; ++r) {
        for (int m = 0; m <= r; ++m) {
            const double left = (m >= 1) ? row[m - 1] : 0.0;
            const double same = (m <= r - 1) ? row[m] : 0.0;
            next[m] = (1.0 - tau) * same + tau * left;
        }
        row.swap(next);
        if (r == n - 2) bn2.assign(row.begin(), row.begin() + n + 1);
        if (r == n - 1) bn1.assign(row.begin(), row.begin() + n + 1);
    }
    if (n == 1) bn2.assign(n + 1, 0.0);
    bn = row;
    bn.resize(n + 1);
}

// Basis and derivative matrices, row-major [n_p][n+1].
void basis(int n, int np, double T, std::vector<double> &P, std::vector<double> &Pd,
           std::vector<double> &Pdd)
{
    const int nv = n + 1;
    P.assign((size_t)np * nv, 0.0);
    Pd.assign((size_t)np * nv, 0.0);
    Pdd.assign((size_t)np * nv, 0.0);
    std::vector<double> bn, bn1, bn2;
    for (int k = 0; k < np; ++k) {
        const double tau = (double)k / (double)(np - 1);
        bernstein_rows(n, tau, bn, bn1, bn2);
        for (int m = 0; m < nv; ++m) {
            auto b1 = [&](int i) { return (i >= 0 && i <= n - 1) ? bn1[i] : 0.0; };
            auto b2 = [&](int i) { return (i >= 0 && i <= n - 2) ? bn2[i] : 0.0; };
            P[(size_t)k * nv + m] = bn[m];
            Pd[(size_t)k * nv + m] = n / T * (b1(m - 1) - b1(m));
            Pdd[(size_t)k * nv + m] = (double)n * (n - 1) / (T * T) * (b2(m - 2) - 2.0 * b2(m - 1) + b2(m));
        }
    }
}

// Inverse of a symmetric positive-definite matrix via Cholesky (false if not SPD).
bool spd_inverse(int n, const std::vector<double> &A, std::vector<double> &Ainv)
{
    std::vector<double> L((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double d = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        L[(size_t)j * n + j] = std::sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double s = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = s / L[(size_t)j * n + j];
        }
    }
    Ainv.assign((size_t)n * n, 0.0);
    std::vector<double> col(n);
    for (int c = 0; c < n; ++c) {
        for (int i = 0; i < n; ++i) {  // L y = e_c
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * col[k];
            col[i] = s / L[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {  // L^T x = y
            double s = col[i];
            for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * col[k];
            col[i] = s / L[(size_t)i * n + i];
        }
        for (int i = 0; i < n; ++i) Ainv[(size_t)i * n + c] = col[i];
    }
    return true;
}

bool is_boundary(int m, int n) { return m == 0 || m == 1 || m == 2 || m == n; }

void boundary_coeffs(int n, double T, const double *b4, double *c4)
{
    const double x0 = b4[0], v0 = b4[1], a0 = b4[2], xf = b4[3];
    c4[0] = x0;
    c4[1] = x0 + v0 * T / n;
    c4[2] = x0 + 2.0 * v0 * T / n + a0 * T * T / ((double)n * (n - 1));
    c4[3] = xf;
}

// QP update operator of a Hessian H (n_v x n_v): W_ff = H_ff^-1 and, in coefficient
// order with rows = free coefficients, W = [W_ff | -W_ff H_fb].
trajam_status qp_operator(const std::vector<double> &H, int n, std::vector<double> &Wff,
                          std::vector<double> &W, std::string &msg)
{
    const int nv = n + 1, nf = nv - 4;
    std::vector<double> Hff((size_t)std::max(nf, 1) * std::max(nf, 1), 0.0);
    for (int a = 0; a < nf; ++a)
        for (int b = 0; b < nf; ++b) Hff[(size_t)a * nf + b] = H[(size_t)(3 + a) * nv + (3 + b)];
    Wff.clear();
    if (nf > 0 && !spd_inverse(nf, Hff, Wff)) {
        msg = "free block of the QP Hessian is not positive definite";
        return TRAJAM_ERR_NUMERIC;
    }
    W.assign((size_t)std::max(nf, 0) * nv, 0.0);
    for (int a = 0; a < nf; ++a)
        for (int m = 0; m < nv; ++m) {
            double v = 0.0;
            if (!is_boundary(m, n)) {
                v = Wff[(size_t)a * nf + (m - 3)];
            } else {
                for (int b = 0; b < nf; ++b) v -= Wff[(size_t)a * nf + b] * H[(size_t)(3 + b) * nv + m];
            }
            W[(size_t)a * nv + m] = v;
        }
    for (double v : W)
        if (!std::isfinite(v)) {
            msg = "non-finite QP operator";
            return TRAJAM_ERR_NUMERIC;
        }
    return TRAJAM_OK;
}

// Host FP64 precompute of every fixed matrix of one problem class.
trajam_status precompute(const trajam_problem &pr, std::vector<double> &P, std::vector<double> &Pd,
                         std::vector<double> &Pdd, std::vector<double> &H,
                         std::vector<double> &Wff, std::vector<double> &W, std::string &msg)
{
    const trajam_problem *p = &pr;
    const int n = p->degree, nv = n + 1, np = p->n_steps, nf = nv - 4;
    basis(n, np, p->horizon, P, Pd, Pdd);
    H.assign((size_t)nv * nv, 0.0);
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
            double ff = 0.0;
            for (int k = 0; k < np; ++k) {
                const size_t ri = (size_t)k * nv;
                // every obstacle adds a copy of P to F; the workspace rows G = [-P; P] two
                ff += (p->n_obstacles + (p->workspace ? 2 : 0)) * P[ri + i] * P[ri + j];
                if (p->v_max > 0.0) ff += Pd[ri + i] * Pd[ri + j];
                if (p->a_max > 0.0) ff += Pdd[ri + i] * Pdd[ri + j];
            }
            H[(size_t)i * nv + j] = (i == j ? 1.0 : 0.0) + p->rho * ff;
        }
    return qp_operator(H, n, Wff, W, msg);
}

template <typename T>
hipError_t upload(void **dst, const std::vector<double> &src)
{
    std::vector<T> tmp(src.size());
    for (size_t i = 0; i < src.size(); ++i) tmp[i] = (T)src[i];
    hipError_t e = hipMalloc(dst, sizeof(T) * (tmp.size() ? tmp.size() : 1));
    if (e != hipSuccess) return e;
    if (tmp.empty()) return hipSuccess;
    return hipMemcpy(*dst, tmp.data(), sizeof(T) * tmp.size(), hipMemcpyHostToDevice);
}

uint16_t bf16_bits(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;  // round to nearest even
    return (uint16_t)(u >> 16);
}

float bf16_value(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}

// trajam_init rejects a problem class whose QP step contracts its error by less than
// this factor per iteration in the chosen precision.
constexpr double kMaxQpContraction = 0.5;

// Hessian seen by the agents' deviations from their mean in a joint problem:
// H + N rho P^T P (the complete-graph Laplacian of the pair rows, eq A_f).
std::vector<double> agents_hessian(const trajam_problem &p, const std::vector<double> &P,
                                   const std::vector<double> &H)
{
    const int nv = p.degree + 1, np = p.n_steps;
    std::vector<double> H2 = H;
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
            double g = 0.0;
            for (int k = 0; k < np; ++k) g += P[(size_t)k * nv + i] * P[(size_t)k * nv + j];
            H2[(size_t)i * nv + j] += p.n_agents * p.rho * g;
        }
    return H2;
}

// Spectral radius of E = I - W~ H_ff, W~ the free-coefficient operator as the device
// applies it in `precision` (FP64: W_ff; FP32: W_ff rounded to float; BF16_REFINE: the
// bf16 hi + lo split of the float W_ff).  The delta-form QP step xb_f += W~ (q - H_ff
// xb_f) contracts its error by E, so this must stay well below 1.  Estimated by the
// Gelfand formula ||E^k||_F^(1/k) at k = 256 (repeated squaring, renormalised each
// step): an upper estimate within a factor n_f^(1/512) of the radius.
double qp_contraction(const std::vector<double> &H, int n, const std::vector<double> &Wff, int precision)
{
    const int nv = n + 1, nf = nv - 4;
    if (nf <= 0) return 0.0;
    std::vector<double> Wt((size_t)nf * nf), E((size_t)nf * nf), T2((size_t)nf * nf);
    for (size_t i = 0; i < Wt.size(); ++i) {
        const double w = Wff[i];
        if (precision == TRAJAM_FP32) {
            Wt[i] = (double)(float)w;
        } else if (precision == TRAJAM_BF16_REFINE) {
            const float wf = (float)w;
            const uint16_t hi = bf16_bits(wf), lo = bf16_bits(wf - bf16_value(hi));
            Wt[i] = (double)bf16_value(hi) + (double)bf16_value(lo);
        } else {
            Wt[i] = w;
        }
    }
    for (int a = 0; a < nf; ++a)
        for (int b = 0; b < nf; ++b) {
            double acc = a == b ? 1.0 : 0.0;
            for (int c = 0; c < nf; ++c) acc -= Wt[(size_t)a * nf + c] * H[(size_t)(3 + c) * nv + (3 + b)];
            E[(size_t)a * nf + b] = acc;
        }
    auto fro = [&](const std::vector<double> &M) {
        double q = 0.0;
        for (double v : M) q += v * v;
        return std::sqrt(q);
    };
    double nrm = fro(E);
    if (!(nrm > 0.0)) return 0.0;
    if (!std::isfinite(nrm)) return INFINITY;
    double log_scale = std::log(nrm);   // log ||E^k||_F = log_scale + log ||M||_F, M normalised
    for (double &v : E) v /= nrm;
    int k = 1;
    for (int sq = 0; sq < 8; ++sq) {
        for (int a = 0; a < nf; ++a)
            for (int b = 0; b < nf; ++b) {
                double acc = 0.0;
                for (int c = 0; c < nf; ++c) acc += E[(size_t)a * nf + c] * E[(size_t)c * nf + b];
                T2[(size_t)a * nf + b] = acc;
            }
        k *= 2;
        log_scale *= 2.0;
        const double m = fro(T2);
        if (!(m > 0.0)) return 0.0;   // nilpotent
        log_scale += std::log(m);
        for (size_t i = 0; i < E.size(); ++i) E[i] = T2[i] / m;
    }
    return std::exp(log_scale / k);
}

// Largest QP-step contraction of a problem class in its precision (the agents'
// deviation operator included for joint problems).
trajam_status problem_contraction(const trajam_problem &p, const std::vector<double> &P,
                                  const std::vector<double> &H, const std::vector<double> &Wff, double &rho,
                                  std::string &msg)
{
    rho = qp_contraction(H, p.degree, Wff, p.precision);
    if (p.n_agents > 1) {
        std::vector<double> H2 = agents_hessian(p, P, H), Wff2, W2;
        trajam_status st = qp_operator(H2, p.degree, Wff2, W2, msg);
        if (st != TRAJAM_OK) return st;
        rho = std::max(rho, qp_contraction(H2, p.degree, Wff2, p.precision));
    }
    return TRAJAM_OK;
}


}  // namespace

namespace trajam {
// Host helpers shared with the heading variant's entry points (heading_api.cpp).
void host_basis(int n, int np, double T, std::vector<double> &P, std::vector<double> &Pd,
                std::vector<double> &Pdd)
{
    basis(n, np, T, P, Pd, Pdd);
}
bool host_spd_inverse(int n, const std::vector<double> &A, std::vector<double> &Ainv)
{
    return spd_inverse(n, A, Ainv);
}
void host_boundary_coeffs(int n, double T, const double *b4, double *c4) { boundary_coeffs(n, T, b4, c4); }
}  // namespace trajam

extern "C" {

const char *trajam_status_string(trajam_status st)
{
    switch (st) {
    case TRAJAM_OK: return "ok";
    case TRAJAM_ERR_INVALID: return "invalid argument";
    case TRAJAM_ERR_UNSUPPORTED: return "unsupported";
    case TRAJAM_ERR_NUMERIC: return "numerically singular fixed matrix";
    case TRAJAM_ERR_DEVICE: return "HIP device error";
    case TRAJAM_ERR_CAPACITY: return "batch exceeds max_batch";
    }
    return "unknown status";
}

const char *trajam_last_error(const trajam_solver *s) { return s ? s->err.c_str() : g_init_err.c_str(); }

trajam_status trajam_boundary_coefficients(const trajam_problem *p, const double *b4, double *c4)
{
    std::string why;
    trajam_status st = validate(p, why);
    if (st != TRAJAM_OK && st != TRAJAM_ERR_UNSUPPORTED) return fail(nullptr, st, why);
    if (!b4 || !c4) return fail(nullptr, TRAJAM_ERR_INVALID, "NULL pointer");
    boundary_coeffs(p->degree, p->horizon, b4, c4);
    return TRAJAM_OK;
}

void trajam_destroy(trajam_solver *s)
{
    if (!s) return;
    if (s->d_phi) (void)hipFree(s->d_phi);
    if (s->d_W) (void)hipFree(s->d_W);
    if (s->d_obs) (void)hipFree(s->d_obs);
    if (s->d_soa) (void)hipFree(s->d_soa);
    if (s->d_bf16) (void)hipFree(s->d_bf16);
    if (s->d_Hff) (void)hipFree(s->d_Hff);
    if (s->d_W2) (void)hipFree(s->d_W2);
    if (s->d_xiBag) (void)hipFree(s->d_xiBag);
    if (s->d_cont_W) (void)hipFree(s->d_cont_W);
    if (s->d_cont_rho) (void)hipFree(s->d_cont_rho);
    delete s;
}

trajam_status trajam_init(const trajam_problem *p, trajam_solver **out)
{
    if (!out) return fail(nullptr, TRAJAM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    std::string why;
    trajam_status st = validate(p, why);
    if (st != TRAJAM_OK) return fail(nullptr, st, why);

    trajam_solver *s = new (std::nothrow) trajam_solver();
    if (!s) return fail(nullptr, TRAJAM_ERR_DEVICE, "host allocation failed");
    s->prob = *p;
    const int n = p->degree, nv = n + 1, np = p->n_steps;
    s->nv = nv;
    s->nf = nv - 4;
    s->nvp = pad_coeffs(nv);
    s->tpad = ((np + 63) / 64) * 64;
    s->variant = TRAJAM_KERNEL_MULTIWAVE;
    s->tb = 1;

    std::string msg;
    st = precompute(*p, s->P, s->Pd, s->Pdd, s->H, s->Wff, s->W, msg);
    if (st == TRAJAM_OK) st = problem_contraction(*p, s->P, s->H, s->Wff, s->qp_rho, msg);
    if (st == TRAJAM_OK && !(s->qp_rho < kMaxQpContraction)) {
        st = TRAJAM_ERR_NUMERIC;
        msg = "the QP step does not contract in this precision (spectral radius " + std::to_string(s->qp_rho) +
              " of I - W H_ff); use a higher precision";
    }
    if (st != TRAJAM_OK) {
        trajam_destroy(s);
        return fail(nullptr, st, msg);
    }
    const int nf = s->nf;
    std::vector<double> Hff((size_t)std::max(nf, 1) * std::max(nf, 1), 0.0);
    for (int a = 0; a < nf; ++a)
        for (int b = 0; b < nf; ++b) Hff[(size_t)a * nf + b] = s->H[(size_t)(3 + a) * nv + (3 + b)];
    // padded device layouts
    const int nvp = s->nvp;
    std::vector<double> phi((size_t)3 * np * nvp, 0.0), Wp((size_t)nvp * nvp, 0.0);
    for (int k = 0; k < np; ++k)
        for (int m = 0; m < nv; ++m) {
            phi[((size_t)0 * np + k) * nvp + m] = s->P[(size_t)k * nv + m];
            phi[((size_t)1 * np + k) * nvp + m] = s->Pd[(size_t)k * nv + m];
            phi[((size_t)2 * np + k) * nvp + m] = s->Pdd[(size_t)k * nv + m];
        }
    for (int a = 0; a < nf; ++a)
        for (int m = 0; m < nv; ++m) Wp[(size_t)a * nvp + m] = s->W[(size_t)a * nv + m];
    if (hipGetDevice(&s->device) != hipSuccess) {
        trajam_destroy(s);
        return fail(nullptr, TRAJAM_ERR_DEVICE, "hipGetDevice failed (no GPU?)");
    }
    const bool f64 = p->precision == TRAJAM_FP64;
    const size_t rec = trajam::kObstacleRecord;
    std::vector<double> zeros_obs((size_t)std::max(p->n_obstacles, 1) * rec, 0.0);
    hipError_t e = f64 ? upload<double>(&s->d_phi, phi) : upload<float>(&s->d_phi, phi);
    if (e == hipSuccess) e = f64 ? upload<double>(&s->d_W, Wp) : upload<float>(&s->d_W, Wp);
    if (e == hipSuccess) e = f64 ? upload<double>(&s->d_obs, zeros_obs) : upload<float>(&s->d_obs, zeros_obs);
    const size_t scal = f64 ? sizeof(double) : sizeof(float);
    std::vector<double> zeros_soa((size_t)std::max(trajam::obstacle_groups(p->n_obstacles, scal), 1) *
                                      trajam::kObstacleFields * trajam::group_store(scal), 0.0);
    if (e == hipSuccess) e = f64 ? upload<double>(&s->d_soa, zeros_soa) : upload<float>(&s->d_soa, zeros_soa);
    if (e == hipSuccess && p->precision == TRAJAM_BF16_REFINE) {
        // bf16 hi/lo split of W_ff = H_ff^-1 (16 x 16, zero padded), and H_ff, H_fb in fp32
        std::vector<uint16_t> hl(2 * 256, 0);
        for (int a = 0; a < nf; ++a)
            for (int b = 0; b < nf; ++b) {
                const float w = (float)s->Wff[(size_t)a * nf + b];
                const uint16_t hi = bf16_bits(w);
                const uint16_t lo = bf16_bits(w - bf16_value(hi));
                hl[a * 16 + b] = hi;
                hl[256 + a * 16 + b] = lo;
            }
        e = hipMalloc(&s->d_bf16, hl.size() * sizeof(uint16_t));
        if (e == hipSuccess)
            e = hipMemcpy(s->d_bf16, hl.data(), hl.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
        std::vector<double> Hm(256 + 64, 0.0);
        const int bidx[4] = {0, 1, 2, n};
        for (int a = 0; a < nf; ++a) {
            for (int b = 0; b < nf; ++b) Hm[a * 16 + b] = Hff[(size_t)a * nf + b];
            for (int j = 0; j < 4; ++j) Hm[256 + a * 4 + j] = s->H[(size_t)(3 + a) * nv + bidx[j]];
        }
        if (e == hipSuccess) e = upload<float>(&s->d_Hff, Hm);
    }
    if (e == hipSuccess && p->n_agents > 1) {
        // deviations of the agents from their mean see H + N rho P^T P
        std::vector<double> H2 = agents_hessian(*p, s->P, s->H), Wff2, W2;
        st = qp_operator(H2, n, Wff2, W2, msg);
        if (st != TRAJAM_OK) {
            trajam_destroy(s);
            return fail(nullptr, st, msg);
        }
        std::vector<double> W2p((size_t)nvp * nvp, 0.0);
        for (int a = 0; a < nf; ++a)
            for (int m = 0; m < nv; ++m) W2p[(size_t)a * nvp + m] = W2[(size_t)a * nv + m];
        std::vector<double> zb((size_t)p->n_agents * p->dims * 4, 0.0);
        e = f64 ? upload<double>(&s->d_W2, W2p) : upload<float>(&s->d_W2, W2p);
        if (e == hipSuccess) e = f64 ? upload<double>(&s->d_xiBag, zb) : upload<float>(&s->d_xiBag, zb);
    }
    if (e != hipSuccess) {
        std::string m = std::string("device allocation/copy failed: ") + hipGetErrorString(e);
        trajam_destroy(s);
        return fail(nullptr, TRAJAM_ERR_DEVICE, m);
    }
    *out = s;
    return TRAJAM_OK;
}

trajam_status trajam_fixed_matrices(const trajam_problem *p, double *P, double *Pd, double *Pdd,
                                    double *H, double *W)
{
    std::string why;
    trajam_status st = validate(p, why);
    if (st != TRAJAM_OK) return fail(nullptr, st, why);
    std::vector<double> vP, vPd, vPdd, vH, vWff, vW;
    st = precompute(*p, vP, vPd, vPdd, vH, vWff, vW, why);
    if (st != TRAJAM_OK) return fail(nullptr, st, why);
    if (P) std::memcpy(P, vP.data(), sizeof(double) * vP.size());
    if (Pd) std::memcpy(Pd, vPd.data(), sizeof(double) * vPd.size());
    if (Pdd) std::memcpy(Pdd, vPdd.data(), sizeof(double) * vPdd.size());
    if (H) std::memcpy(H, vH.data(), sizeof(double) * vH.size());
    if (W && !vW.empty()) std::memcpy(W, vW.data(), sizeof(double) * vW.size());
    return TRAJAM_OK;
}

trajam_status trajam_qp_contraction(const trajam_problem *p, double *rho)
{
    if (!rho) return fail(nullptr, TRAJAM_ERR_INVALID, "rho must not be NULL");
    std::string why;
    trajam_status st = validate(p, why);
    if (st != TRAJAM_OK) return fail(nullptr, st, why);
    std::vector<double> vP, vPd, vPdd, vH, vWff, vW;
    st = precompute(*p, vP, vPd, vPdd, vH, vWff, vW, why);
    if (st == TRAJAM_OK) st = problem_contraction(*p, vP, vH, vWff, *rho, why);
    if (st != TRAJAM_OK) return fail(nullptr, st, why);
    return TRAJAM_OK;
}

trajam_status trajam_set_launch(trajam_solver *s, int32_t kernel, int32_t spw)
{
    if (!s) return TRAJAM_ERR_INVALID;
    if (kernel == TRAJAM_KERNEL_MULTIWAVE) {
        if (spw < 1 || spw * s->tpad > trajam::kMaxThreads)
            return fail(s, TRAJAM_ERR_INVALID, "multi-wave kernel: spw * roundup64(n_steps) must be in [64, 256]");
    } else if (kernel == TRAJAM_KERNEL_WAVE) {
        if (spw < 1 || spw * 64 > trajam::kMaxThreads)
            return fail(s, TRAJAM_ERR_INVALID, "wave kernel: spw must be in [1, 4]");
    } else {
        return fail(s, TRAJAM_ERR_INVALID, "unknown kernel variant");
    }
    s->variant = kernel;
    s->tb = spw;
    return TRAJAM_OK;
}

trajam_status trajam_get_launch(const trajam_solver *s, int32_t *kernel, int32_t *spw)
{
    if (!s) return TRAJAM_ERR_INVALID;
    if (kernel) *kernel = s->variant;
    if (spw) *spw = s->tb;
    return TRAJAM_OK;
}

}  // extern "C"

namespace {

template <typename T>
void fill_args(const trajam_solver *s, AmArgs<T> &a, int batch, int iters)
{
    const trajam_problem &p = s->prob;
    std::memset(&a, 0, sizeof(a));
    a.batch = batch;
    a.dims = p.dims;
    a.n_p = p.n_steps;
    a.nv = s->nv;
    a.n_o = p.n_obstacles;
    a.iters = iters;
    a.tpad = s->tpad;
    a.tb = s->tb;
    a.use_v = p.v_max > 0.0;
    a.use_a = p.a_max > 0.0;
    a.sphere = p.obstacle_model == TRAJAM_SPHERE;
    a.rho = (T)p.rho;
    a.vmax = (T)p.v_max;
    a.amax = (T)p.a_max;
    a.dt = (T)(p.horizon / (p.n_steps - 1));
    a.phi = (const T *)s->d_phi;
    a.W = (const T *)s->d_W;
    a.obs = (const T *)s->d_obs;
    a.obs_soa = (const T *)s->d_soa;
    if (s->d_bf16) {
        a.Whi = (const uint16_t *)s->d_bf16;
        a.Wlo = (const uint16_t *)s->d_bf16 + 256;
    }
    a.Hmq = (const float *)s->d_Hff;
    a.n_agents = p.n_agents;
    a.pair_r = (T)(2.0 * p.agent_radius);
    a.W2 = (const T *)s->d_W2;
    a.xiB_ag = (const T *)s->d_xiBag;
    a.use_ws = p.workspace;
    for (int ax = 0; ax < 3; ++ax) {
        a.ws_lo[ax] = (T)(ax < p.dims ? p.ws_lo[ax] : 0.0);
        a.ws_hi[ax] = (T)(ax < p.dims ? p.ws_hi[ax] : 0.0);
    }
}

// Samples per workgroup of the single-robot residual kernel (roundup64(n_steps)
// threads per sample): its own shape, independent of the projection's launch
// variant, whose samples-per-workgroup count means 64-lane waves for the wave kernel.
int residual_spw(const trajam_solver *s) { return std::max(1, trajam::kMaxThreads / s->tpad); }

// Boundary coefficients of every agent ([n_agents][D][4]) from boundary rows
// [n_agents][D][4] (x0, v0, a0, xf).
std::vector<double> agent_boundary_coeffs(const trajam_problem &p, const double *rows)
{
    std::vector<double> c((size_t)p.n_agents * p.dims * 4);
    for (int i = 0; i < p.n_agents * p.dims; ++i) boundary_coeffs(p.degree, p.horizon, rows + 4 * i, &c[4 * (size_t)i]);
    return c;
}

// Floats of the per-wave LDS obstacle stage of the multi-agent kernels (0: the
// obstacles are tested without the stage, when there are none or they do not fit).
int agent_stage(const trajam_solver *s, size_t scalar, int waves)
{
    const trajam_problem &p = s->prob;
    if (p.n_obstacles == 0) return 0;
    const int st = trajam::stage_fields(p.dims, p.obstacle_model == TRAJAM_SPHERE) * p.n_obstacles;
    return (size_t)st * scalar * waves <= (size_t)trajam::kStageMaxFloats * sizeof(float) * 4 ? st : 0;
}

// Multi-agent boundary: the device copy is rebuilt only when the rows change; a
// change waits for the stream (no graph capture then) and copies synchronously.
trajam_status agents_boundary(trajam_solver *s, const double *rows, hipStream_t st)
{
    const trajam_problem &p = s->prob;
    const size_t cnt = (size_t)p.n_agents * p.dims * 4;
    for (size_t i = 0; i < cnt; ++i)
        if (!std::isfinite(rows[i])) return fail(s, TRAJAM_ERR_INVALID, "non-finite boundary value");
    if (s->bnd_cache.size() == cnt && std::equal(s->bnd_cache.begin(), s->bnd_cache.end(), rows))
        return TRAJAM_OK;
    std::vector<double> c = agent_boundary_coeffs(p, rows);
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) {
        if (p.precision == TRAJAM_FP64) {
            e = hipMemcpy(s->d_xiBag, c.data(), sizeof(double) * cnt, hipMemcpyHostToDevice);
        } else {
            std::vector<float> cf(c.begin(), c.end());
            e = hipMemcpy(s->d_xiBag, cf.data(), sizeof(float) * cnt, hipMemcpyHostToDevice);
        }
    }
    if (e != hipSuccess) return fail(s, TRAJAM_ERR_DEVICE, std::string("agent boundary upload: ") + hipGetErrorString(e));
    s->bnd_cache.assign(rows, rows + cnt);
    return TRAJAM_OK;
}

// Packs the obstacles of a call into the solver.  With obs_centre and obs_axes both
// NULL, the obstacles packed last (by a call or by trajam_set_obstacles) are reused.
trajam_status pack(trajam_solver *s, const void *c, const void *w, const void *ax, hipStream_t st)
{
    const trajam_problem &p = s->prob;
    if (p.n_obstacles == 0) return TRAJAM_OK;
    if (!c && !ax && !w && s->packed) return TRAJAM_OK;
    if (!c || !ax) return fail(s, TRAJAM_ERR_INVALID, "obstacle centre/axes pointer is NULL (and none packed)");
    hipError_t e = (p.precision == TRAJAM_FP64)
                       ? trajam::launch_pack_obstacles_f64(p.dims, p.n_obstacles, (const double *)c,
                                                           (const double *)w, (const double *)ax,
                                                           (double *)s->d_obs, (double *)s->d_soa, st)
                       : trajam::launch_pack_obstacles_f32(p.dims, p.n_obstacles, (const float *)c,
                                                           (const float *)w, (const float *)ax,
                                                           (float *)s->d_obs, (float *)s->d_soa, st);
    if (e != hipSuccess) return fail(s, TRAJAM_ERR_DEVICE, std::string("obstacle pack launch: ") + hipGetErrorString(e));
    s->packed = true;
    s->dynamic = w != nullptr;
    return TRAJAM_OK;
}

}  // namespace

extern "C" trajam_status trajam_project(trajam_solver *s, int32_t batch, const void *xi,
                                        const double *boundary_host, const void *obs_centre,
                                        const void *obs_vel, const void *obs_axes, void *xi_bar,
                                        void *lambda, int32_t iters, void *res_trace,
                                        uint32_t *flags, void *stream)
{
    if (!s) return TRAJAM_ERR_INVALID;
    s->err.clear();
    if (batch < 0 || iters < 0) return fail(s, TRAJAM_ERR_INVALID, "batch and iters must be >= 0");
    if (batch > s->prob.max_batch) return fail(s, TRAJAM_ERR_CAPACITY, "batch > max_batch");
    if (batch == 0 || iters == 0) return TRAJAM_OK;
    if (!xi || !xi_bar || !lambda || !boundary_host)
        return fail(s, TRAJAM_ERR_INVALID, "xi, xi_bar, lambda and boundary must not be NULL");
    for (int i = 0; i < s->prob.dims * 4; ++i)
        if (!std::isfinite(boundary_host[i])) return fail(s, TRAJAM_ERR_INVALID, "non-finite boundary value");
    hipStream_t st = (hipStream_t)stream;
    trajam_status ps = pack(s, obs_centre, obs_vel, obs_axes, st);
    if (ps != TRAJAM_OK) return ps;
    const trajam_problem &p = s->prob;
    const int dynamic = s->dynamic;
    hipError_t e;
    if (p.n_agents > 1) {
        ps = agents_boundary(s, boundary_host, st);
        if (ps != TRAJAM_OK) return ps;
        if (p.precision == TRAJAM_FP64) {
            AmArgs<double> a;
            fill_args(s, a, batch, iters);
            a.dynamic = dynamic;
            a.cull_lds = agent_stage(s, sizeof(double), a.tb);
            a.xi = (const double *)xi;
            a.xb = (double *)xi_bar;
            a.lam = (double *)lambda;
            a.res = (double *)res_trace;
            a.flags = flags;
            e = trajam::launch_agents_f64(p.dims, s->nvp, a, st);
        } else {
            AmArgs<float> a;
            fill_args(s, a, batch, iters);
            a.dynamic = dynamic;
            a.cull_lds = agent_stage(s, sizeof(float), a.tb);
            a.xi = (const float *)xi;
            a.xb = (float *)xi_bar;
            a.lam = (float *)lambda;
            a.res = (float *)res_trace;
            a.flags = flags;
            e = trajam::launch_agents_f32(p.dims, s->nvp, a, st);
        }
        if (e != hipSuccess) return fail(s, TRAJAM_ERR_DEVICE, std::string("multi-agent launch: ") + hipGetErrorString(e));
        return TRAJAM_OK;
    }
    if (p.precision == TRAJAM_FP64) {
        AmArgs<double> a;
        fill_args(s, a, batch, iters);
        a.dynamic = dynamic;
        for (int ax = 0; ax < p.dims; ++ax) {
            double c4[4];
            boundary_coeffs(p.degree, p.horizon, boundary_host + 4 * ax, c4);
            for (int i = 0; i < 4; ++i) a.xiB[ax][i] = c4[i];
        }
        a.xi = (const double *)xi;
        a.xb = (double *)xi_bar;
        a.lam = (double *)lambda;
        a.res = (double *)res_trace;
        a.flags = flags;
        e = trajam::launch_project_f64(p.dims, s->nvp, s->variant, a, st);
    } else {
        AmArgs<float> a;
        fill_args(s, a, batch, iters);
        a.dynamic = dynamic;
        for (int ax = 0; ax < p.dims; ++ax) {
            double c4[4];
            boundary_coeffs(p.degree, p.horizon, boundary_host + 4 * ax, c4);
            for (int i = 0; i < 4; ++i) a.xiB[ax][i] = (float)c4[i];
        }
        a.xi = (const float *)xi;
        a.xb = (float *)xi_bar;
        a.lam = (float *)lambda;
        a.res = (float *)res_trace;
        a.flags = flags;
        e = trajam::launch_project_f32(p.dims, s->nvp, s->variant, p.precision == TRAJAM_BF16_REFINE, a, st);
    }
    if (e != hipSuccess) return fail(s, TRAJAM_ERR_DEVICE, std::string("AM launch: ") + hipGetErrorString(e));
    return TRAJAM_OK;
}

extern "C" trajam_status trajam_set_continuation(trajam_solver *s, const trajam_continuation *c)
{
    if (!s) return TRAJAM_ERR_INVALID;
    s->err.clear();
    if (!c) {   // off
        s->cont_on = false;
        return TRAJAM_OK;
    }
    const trajam_problem &p = s->prob;
    if (p.n_agents != 1) return fail(s, TRAJAM_ERR_UNSUPPORTED, "penalty continuation is single-robot");
    if (p.precision == TRAJAM_BF16_REFINE)
        return fail(s, TRAJAM_ERR_UNSUPPORTED, "penalty continuation needs precision FP64 or FP32");
    if (c->levels < 1 || c->levels > TRAJAM_CONT_MAX_LEVELS || !(c->growth >= 1.0) || !std::isfinite(c->growth) ||
        c->window < 1 || !(c->stall_ratio >= 0.0) || !std::isfinite(c->stall_ratio) || !(c->tol >= 0.0) ||
        !std::isfinite(c->tol))
        return fail(s, TRAJAM_ERR_INVALID,
                    "continuation: levels in [1, 16], growth >= 1, window >= 1, stall_ratio >= 0, tol >= 0");
    const int n = p.degree, nv = n + 1, nf = nv - 4, nvp = s->nvp, L = c->levels;
    std::vector<double> Wt((size_t)L * nvp * nvp, 0.0), rt(L);
    for (int l = 0; l < L; ++l) {
        trajam_problem pl = p;
        pl.rho = p.rho * std::pow(c->growth, (double)l);   // the ladder rho * growth^l
        rt[l] = pl.rho;
        std::vector<double> P, Pd, Pdd, H, Wff, W;
        std::string msg;
        trajam_status st = precompute(pl, P, Pd, Pdd, H, Wff, W, msg);
        double qr = 0.0;
        if (st == TRAJAM_OK) st = problem_contraction(pl, P, H, Wff, qr, msg);
        if (st == TRAJAM_OK && !(qr < kMaxQpContraction)) {
            st = TRAJAM_ERR_NUMERIC;
            msg = "the QP step of penalty level " + std::to_string(l) + " does not contract in this precision";
        }
        if (st != TRAJAM_OK) return fail(s, st, msg);
        for (int a = 0; a < nf; ++a)
            for (int m = 0; m < nv; ++m) Wt[((size_t)l * nvp + a) * nvp + m] = W[(size_t)a * nv + m];
    }
    if (s->d_cont_W) (void)hipFree(s->d_cont_W);
    if (s->d_cont_rho) (void)hipFree(s->d_cont_rho);
    s->d_cont_W = s->d_cont_rho = nullptr;
    const bool f64 = p.precision == TRAJAM_FP64;
    hipError_t e = f64 ? upload<double>(&s->d_cont_W, Wt) : upload<float>(&s->d_cont_W, Wt);
    if (e == hipSuccess) e = f64 ? upload<double>(&s->d_cont_rho, rt) : upload<float>(&s->d_cont_rho, rt);
    if (e != hipSuccess) {
        s->cont_on = false;
        return fail(s, TRAJAM_ERR_DEVICE, std::string("continuation tables: ") + hipGetErrorString(e));
    }
    s->cont = *c;
    s->cont_on = true;
    return TRAJAM_OK;
}

extern "C" trajam_status trajam_project_continuation(trajam_solver *s, int32_t batch, const void *xi,
                                                     const double *boundary_host, const void *obs_centre,
                                                     const void *obs_vel, const void *obs_axes, void *xi_bar,
                                                     void *lambda, trajam_cont_state *state, int32_t iters,
                                                     void *res_trace, uint32_t *flags, void *stream)
{
    if (!s) return TRAJAM_ERR_INVALID;
    s->err.clear();
    if (!s->cont_on) return fail(s, TRAJAM_ERR_INVALID, "no penalty continuation set (trajam_set_continuation)");
    if (batch < 0 || iters < 0) return fail(s, TRAJAM_ERR_INVALID, "batch and iters must be >= 0");
    if (batch > s->prob.max_batch) return fail(s, TRAJAM_ERR_CAPACITY, "batch > max_batch");
    if (batch == 0 || iters == 0) return TRAJAM_OK;
    if (!xi || !xi_bar || !lambda || !boundary_host || !state)
        return fail(s, TRAJAM_ERR_INVALID, "xi, xi_bar, lambda, state and boundary must not be NULL");
    for (int i = 0; i < s->prob.dims * 4; ++i)
        if (!std::isfinite(boundary_host[i])) return fail(s, TRAJAM_ERR_INVALID, "non-finite boundary value");
    hipStream_t st = (hipStream_t)stream;
    trajam_status ps = pack(s, obs_centre, obs_vel, obs_axes, st);
    if (ps != TRAJAM_OK) return ps;
    const trajam_problem &p = s->prob;
    // the wave-per-sample kernel carries the continuation; its tuned shape when it is
    // the tuned variant, one sample a workgroup otherwise
    const int spw = s->variant == TRAJAM_KERNEL_WAVE ? s->tb : 1;
    hipError_t e;
    if (p.precision == TRAJAM_FP64) {
        AmArgs<double> a;
        fill_args(s, a, batch, iters);
        a.tb = spw;
        a.dynamic = s->dynamic;
        for (int ax = 0; ax < p.dims; ++ax) {
            double c4[4];
            boundary_coeffs(p.degree, p.horizon, boundary_host + 4 * ax, c4);
            for (int i = 0; i < 4; ++i) a.xiB[ax][i] = c4[i];
        }
        a.xi = (const double *)xi;
        a.xb = (double *)xi_bar;
        a.lam = (double *)lambda;
        a.res = (double *)res_trace;
        a.flags = flags;
        a.cont_levels = s->cont.levels;
        a.cont_window = s->cont.window;
        a.cont_stall = s->cont.stall_ratio;
        a.cont_tol = s->cont.tol;
        a.cont_rho = (const double *)s->d_cont_rho;
        a.cont_W = (const double *)s->d_cont_W;
        a.cont_state = state;
        e = trajam::launch_project_f64(p.dims, s->nvp, TRAJAM_KERNEL_WAVE, a, st);
    } else {
        AmArgs<float> a;
        fill_args(s, a, batch, iters);
        a.tb = spw;
        a.dynamic = s->dynamic;
        for (int ax = 0; ax < p.dims; ++ax) {
            double c4[4];
            boundary_coeffs(p.degree, p.horizon, boundary_host + 4 * ax, c4);
            for (int i = 0; i < 4; ++i) a.xiB[ax][i] = (float)c4[i];
        }
        a.xi = (const float *)xi;
        a.xb = (float *)xi_bar;
        a.lam = (float *)lambda;
        a.res = (float *)res_trace;
        a.flags = flags;
        a.cont_levels = s->cont.levels;
        a.cont_window = s->cont.window;
        a.cont_stall = (float)s->cont.stall_ratio;
        a.cont_tol = (float)s->cont.tol;
        a.cont_rho = (const float *)s->d_cont_rho;
        a.cont_W = (const float *)s->d_cont_W;
        a.cont_state = state;
        e = trajam::launch_project_f32(p.dims, s->nvp, TRAJAM_KERNEL_WAVE, false, a, st);
    }
    if (e != hipSuccess) return fail(s, TRAJAM_ERR_DEVICE, std::string("AM launch: ") + hipGetErrorString(e));
    return TRAJAM_OK;
}

extern "C" trajam_status trajam_residuals(trajam_solver *s, int32_t batch, const void *xi_bar,
                                          const void *obs_centre, const void *obs_vel,
                                          const void *obs_axes, void *res_l2, void *res_max,
                                          void *stream)
{
    if (!s) return TRAJAM_ERR_INVALID;
    s->err.clear();
    if (batch < 0) return fail(s, TRAJAM_ERR_INVALID, "batch must be >= 0");
    if (batch > s->prob.max_batch) return fail(s, TRAJAM_ERR_CAPACITY, "batch > max_batch");
    if (batch == 0) return TRAJAM_OK;
    if (!xi_bar || !res_l2) return fail(s, TRAJAM_ERR_INVALID, "xi_bar and res_l2 must not be NULL");
    hipStream_t st = (hipStream_t)stream;
    trajam_status ps = pack(s, obs_centre, obs_vel, obs_axes, st);
    if (ps != TRAJAM_OK) return ps;
    const trajam_problem &p = s->prob;
    hipError_t e;
    if (p.precision == TRAJAM_FP64) {
        AmArgs<double> a;
        fill_args(s, a, batch, 0);
        if (p.n_agents == 1) a.tb = residual_spw(s);
        a.dynamic = s->dynamic;
        a.xb = (double *)xi_bar;
        a.res = (double *)res_l2;
        a.res_max = (double *)res_max;
        if (p.n_agents > 1) a.cull_lds = agent_stage(s, sizeof(double), a.tb);
        e = p.n_agents > 1 ? trajam::launch_agents_residual_f64(p.dims, s->nvp, a, st)
                           : trajam::launch_residual_f64(p.dims, s->nvp, a, st);
    } else {
        AmArgs<float> a;
        fill_args(s, a, batch, 0);
        if (p.n_agents == 1) a.tb = residual_spw(s);
        a.dynamic = s->dynamic;
        a.xb = (float *)xi_bar;
        a.res = (float *)res_l2;
        a.res_max = (float *)res_max;
        if (p.n_agents > 1) a.cull_lds = agent_stage(s, sizeof(float), a.tb);
        e = p.n_agents > 1 ? trajam::launch_agents_residual_f32(p.dims, s->nvp, a, st)
                           : trajam::launch_residual_f32(p.dims, s->nvp, a, st);
    }
    if (e != hipSuccess) return fail(s, TRAJAM_ERR_DEVICE, std::string("residual launch: ") + hipGetErrorString(e));
    return TRAJAM_OK;
}

extern "C" trajam_status trajam_polar(trajam_solver *s, int32_t batch, const void *xi_bar, const void *obs_centre,
                                      const void *obs_vel, const void *obs_axes, void *obs_alpha, void *obs_beta,
                                      void *obs_d, void *kin, void *stream)
{
    if (!s) return TRAJAM_ERR_INVALID;
    s->err.clear();
    if (s->prob.n_agents != 1) return fail(s, TRAJAM_ERR_UNSUPPORTED, "trajam_polar is single-robot");
    if (batch < 0) return fail(s, TRAJAM_ERR_INVALID, "batch must be >= 0");
    if (batch > s->prob.max_batch) return fail(s, TRAJAM_ERR_CAPACITY, "batch > max_batch");
    if (batch == 0) return TRAJAM_OK;
    if (!xi_bar) return fail(s, TRAJAM_ERR_INVALID, "xi_bar must not be NULL");
    hipStream_t st = (hipStream_t)stream;
    trajam_status ps = pack(s, obs_centre, obs_vel, obs_axes, st);
    if (ps != TRAJAM_OK) return ps;
    const trajam_problem &p = s->prob;
    if (p.n_obstacles == 0) obs_alpha = obs_beta = obs_d = nullptr;
    hipError_t e;
    if (p.precision == TRAJAM_FP64) {
        AmArgs<double> a;
        fill_args(s, a, batch, 0);
        a.dynamic = s->dynamic;
        a.xb = (double *)xi_bar;
        e = trajam::launch_polar_f64(p.dims, s->nvp, a, obs_alpha, obs_beta, obs_d, kin, st);
    } else {
        AmArgs<float> a;
        fill_args(s, a, batch, 0);
        a.dynamic = s->dynamic;
        a.xb = (float *)xi_bar;
        e = trajam::launch_polar_f32(p.dims, s->nvp, a, obs_alpha, obs_beta, obs_d, kin, st);
    }
    if (e != hipSuccess) return fail(s, TRAJAM_ERR_DEVICE, std::string("polar launch: ") + hipGetErrorString(e));
    return TRAJAM_OK;
}

// ---- sampling loop ------------------------------------------------------------

namespace {

// Bernstein coefficients of the window [d, 1 + d] (in units of the horizon) from those
// of [0, 1]: the blossom of the polynomial at n - j arguments d and j arguments 1 + d,
// evaluated by de Casteljau steps; row j of S, column k, from the unit control
// polygon e_k.
void shift_blossom(int n, double d, double *S /* [kShiftMaxCoeffs][kShiftMaxCoeffs] */)
{
    double pts[trajam::kShiftMaxCoeffs];
    for (int i = 0; i < trajam::kShiftMaxCoeffs * trajam::kShiftMaxCoeffs; ++i) S[i] = 0.0;
    for (int k = 0; k <= n; ++k)
        for (int j = 0; j <= n; ++j) {
            for (int i = 0; i <= n; ++i) pts[i] = i == k ? 1.0 : 0.0;
            for (int r = 1; r <= n; ++r) {
                const double t = r <= n - j ? d : 1.0 + d;
                for (int i = 0; i <= n - r; ++i) pts[i] = (1.0 - t) * pts[i] + t * pts[i + 1];
            }
            S[j * trajam::kShiftMaxCoeffs + k] = pts[0];
        }
}

}  // namespace

namespace trajam {
// The shift matrix S(d) for the heading variant's entry points (heading_api.cpp).
void host_shift_matrix(int n, double d, double *S) { shift_blossom(n, d, S); }
}  // namespace trajam

extern "C" trajam_status trajam_mpc_shift(trajam_solver *s, int32_t batch, double delta, int32_t keep_lambda,
                                          const void *xi_bar, const void *lambda, void *xi_next,
                                          void *xi_bar_next, void *lambda_next, void *stream)
{
    if (!s) return TRAJAM_ERR_INVALID;
    s->err.clear();
    if (batch < 0 || !std::isfinite(delta) || (keep_lambda != 0 && keep_lambda != 1))
        return fail(s, TRAJAM_ERR_INVALID, "batch >= 0, finite delta, keep_lambda 0 or 1 required");
    if (batch > s->prob.max_batch) return fail(s, TRAJAM_ERR_CAPACITY, "batch > max_batch");
    if (batch == 0) return TRAJAM_OK;
    if (!xi_bar || !xi_next || !xi_bar_next || !lambda_next || (keep_lambda && !lambda))
        return fail(s, TRAJAM_ERR_INVALID, "NULL pointer");
    if (s->nv > trajam::kShiftMaxCoeffs) return fail(s, TRAJAM_ERR_UNSUPPORTED, "degree above 15");
    trajam::ShiftMatrix S;
    S.nv = s->nv;
    shift_blossom(s->prob.degree, delta / s->prob.horizon, S.s);
    const int rows = batch * s->prob.n_agents * s->prob.dims;
    hipError_t e = trajam::launch_mpc_shift(s->prob.precision == TRAJAM_FP64, rows, S, xi_bar, lambda, xi_next,
                                            xi_bar_next, lambda_next, keep_lambda, (hipStream_t)stream);
    if (e != hipSuccess) return fail(s, TRAJAM_ERR_DEVICE, std::string("mpc shift: ") + hipGetErrorString(e));
    return TRAJAM_OK;
}

extern "C" trajam_status trajam_normals(int64_t count, uint64_t key, uint64_t counter, int32_t fp64, void *z,
                                        void *stream)
{
    if (count < 0 || (fp64 != 0 && fp64 != 1)) {
        trajam::set_thread_error("count >= 0 and fp64 0 or 1 required");
        return TRAJAM_ERR_INVALID;
    }
    if (count == 0) return TRAJAM_OK;
    if (!z) {
        trajam::set_thread_error("NULL output");
        return TRAJAM_ERR_INVALID;
    }
    hipError_t e = trajam::launch_normals(fp64 == 1, count, key, counter, z, (hipStream_t)stream);
    if (e != hipSuccess) {
        trajam::set_thread_error(std::string("normals: ") + hipGetErrorString(e));
        return TRAJAM_ERR_DEVICE;
    }
    return TRAJAM_OK;
}

extern "C" trajam_status trajam_cem_sample(trajam_solver *s, int32_t n, const void *mu, const void *chol,
                                           const void *z, void *xi, void *xi_bar, void *lambda, void *stream)
{
    if (!s) return TRAJAM_ERR_INVALID;
    s->err.clear();
    if (s->prob.n_agents != 1) return fail(s, TRAJAM_ERR_UNSUPPORTED, "the sampling loop is single-robot");
    if (n < 0) return fail(s, TRAJAM_ERR_INVALID, "n must be >= 0");
    if (n > s->prob.max_batch) return fail(s, TRAJAM_ERR_CAPACITY, "n > max_batch");
    if (n == 0) return TRAJAM_OK;
    if (!mu || !chol || !z || !xi) return fail(s, TRAJAM_ERR_INVALID, "NULL pointer");
    const int dim = s->prob.dims * s->nv;
    hipError_t e = trajam::launch_cem_sample(s->prob.precision == TRAJAM_FP64, n, dim, mu, chol, z, xi, xi_bar,
                                             lambda, (hipStream_t)stream);
    if (e != hipSuccess) return fail(s, TRAJAM_ERR_DEVICE, std::string("cem sample: ") + hipGetErrorString(e));
    return TRAJAM_OK;
}

extern "C" trajam_status trajam_cem_cost(trajam_solver *s, int32_t n, const void *xi_bar, const void *res,
                                         double quantum, void *c_aug, int32_t *res_key, void *stream)
{
    if (!s) return TRAJAM_ERR_INVALID;
    s->err.clear();
    if (s->prob.n_agents != 1) return fail(s, TRAJAM_ERR_UNSUPPORTED, "the sampling loop is single-robot");
    if (n < 0 || !(quantum > 0.0)) return fail(s, TRAJAM_ERR_INVALID, "n >= 0 and quantum > 0 required");
    if (n > s->prob.max_batch) return fail(s, TRAJAM_ERR_CAPACITY, "n > max_batch");
    if (n == 0) return TRAJAM_OK;
    if (!xi_bar || !res || !c_aug || !res_key) return fail(s, TRAJAM_ERR_INVALID, "NULL pointer");
    hipError_t e = trajam::launch_cem_cost(s->prob.precision == TRAJAM_FP64, n, s->prob.dims, s->nv,
                                           s->prob.n_steps, s->nvp, s->d_phi, xi_bar, res, quantum, c_aug,
                                           res_key, (hipStream_t)stream);
    if (e != hipSuccess) return fail(s, TRAJAM_ERR_DEVICE, std::string("cem cost: ") + hipGetErrorString(e));
    return TRAJAM_OK;
}

extern "C" trajam_status trajam_cem_select(trajam_solver *s, int32_t n, const int32_t *res_key,
                                           const void *c_aug, int32_t n_proj, int32_t n_elite,
                                           int32_t *proj_idx, int32_t *elite_idx, void *stream)
{
    if (!s) return TRAJAM_ERR_INVALID;
    s->err.clear();
    if (s->prob.n_agents != 1) return fail(s, TRAJAM_ERR_UNSUPPORTED, "the sampling loop is single-robot");
    if (n < 1 || n > 4096 || n_elite < 1 || n_elite > n_proj || n_proj > n)
        return fail(s, TRAJAM_ERR_INVALID, "need 1 <= n_elite <= n_proj <= n <= 4096");
    if (!res_key || !c_aug || !proj_idx || !elite_idx) return fail(s, TRAJAM_ERR_INVALID, "NULL pointer");
    hipError_t e = trajam::launch_cem_select(s->prob.precision == TRAJAM_FP64, n, res_key, c_aug, n_proj,
                                             n_elite, proj_idx, elite_idx, (hipStream_t)stream);
    if (e != hipSuccess) return fail(s, TRAJAM_ERR_DEVICE, std::string("cem select: ") + hipGetErrorString(e));
    return TRAJAM_OK;
}

extern "C" trajam_status trajam_cem_update(trajam_solver *s, int32_t n_elite, const int32_t *elite_idx,
                                           const void *xi_bar, const void *c_aug, double sigma, double gamma,
                                           void *mu, void *Sigma, void *chol, void *stream)
{
    if (!s) return TRAJAM_ERR_INVALID;
    s->err.clear();
    if (s->prob.n_agents != 1) return fail(s, TRAJAM_ERR_UNSUPPORTED, "the sampling loop is single-robot");
    if (n_elite < 1 || n_elite > 4096 || !(sigma > 0.0 && sigma <= 1.0) || !(gamma > 0.0))
        return fail(s, TRAJAM_ERR_INVALID, "need 1 <= n_elite <= 4096, 0 < sigma <= 1, gamma > 0");
    if (!elite_idx || !xi_bar || !c_aug || !mu || !Sigma || !chol) return fail(s, TRAJAM_ERR_INVALID, "NULL pointer");
    const int dim = s->prob.dims * s->nv;
    hipError_t e = trajam::launch_cem_update(s->prob.precision == TRAJAM_FP64, n_elite, dim, elite_idx, xi_bar,
                                             c_aug, sigma, gamma, 1e-10, mu, Sigma, chol, (hipStream_t)stream);
    if (e != hipSuccess) return fail(s, TRAJAM_ERR_DEVICE, std::string("cem update: ") + hipGetErrorString(e));
    return TRAJAM_OK;
}

// ---- obstacles as solver state, autotuner, ragged plans -------------------------

extern "C" trajam_status trajam_set_obstacles(trajam_solver *s, const void *c, const void *v, const void *ax,
                                              void *stream)
{
    if (!s) return TRAJAM_ERR_INVALID;
    s->err.clear();
    if (s->prob.n_obstacles > 0 && (!c || !ax)) return fail(s, TRAJAM_ERR_INVALID, "obstacle centre/axes pointer is NULL");
    return pack(s, c, v, ax, (hipStream_t)stream);
}

namespace {

std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tune;
bool g_tune_loaded = false;

int pow2_at_least(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

std::string tune_key(const trajam_solver *s, int batch)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, s->device) == hipSuccess) arch = prop.gcnArchName;
    for (char &ch : arch)
        if (ch == ' ') ch = '_';
    std::ostringstream k;
    k << arch << "|d" << s->prob.dims << "|np" << s->prob.n_steps << "|no" << pow2_at_least(std::max(1, s->prob.n_obstacles))
      << "|b" << pow2_at_least(std::max(1, batch)) << "|p" << s->prob.precision << "|m" << s->prob.obstacle_model;
    return k.str();
}

void tune_load_file()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("TRAJAM_AUTOTUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string key;
    int kern, spw;
    while (f >> key >> kern >> spw) g_tune[key] = {kern, spw};
}

void tune_store(const std::string &key, int kern, int spw)
{
    g_tune[key] = {kern, spw};
    const char *path = std::getenv("TRAJAM_AUTOTUNE_CACHE");
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << kern << " " << spw << "\n";
}

}  // namespace

extern "C" trajam_status trajam_autotune(trajam_solver *s, int32_t batch, const void *xi, const double *boundary,
                                         const void *c, const void *v, const void *ax, void *xb, void *lam,
                                         int32_t probe_iters, int32_t *kernel_out, int32_t *spw_out, void *stream)
{
    if (!s) return TRAJAM_ERR_INVALID;
    if (batch < 1 || probe_iters < 1 || !xi || !xb || !lam || !boundary)
        return fail(s, TRAJAM_ERR_INVALID, "autotune needs batch >= 1, probe_iters >= 1 and buffers");
    if (batch > s->prob.max_batch) return fail(s, TRAJAM_ERR_CAPACITY, "batch > max_batch");
    hipStream_t st = (hipStream_t)stream;
    const std::string key = tune_key(s, batch);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_file();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            trajam_status r = trajam_set_launch(s, it->second.first, it->second.second);
            if (r == TRAJAM_OK) {
                if (kernel_out) *kernel_out = it->second.first;
                if (spw_out) *spw_out = it->second.second;
                return TRAJAM_OK;
            }
        }
    }
    const size_t bytes = (size_t)batch * s->prob.n_agents * s->prob.dims * s->nv *
                         (s->prob.precision == TRAJAM_FP64 ? sizeof(double) : sizeof(float));
    // The current launch shape is timed first and stays unless another one is more
    // than 3 % faster (timing noise must not flip the choice between runs).
    std::vector<std::pair<int, int>> cands{{s->variant, s->tb}};
    // multi-agent launches have one shape parameter: joint samples (waves) per workgroup
    if (s->prob.n_agents == 1)
        for (int spw = 1; spw * s->tpad <= trajam::kMaxThreads; spw *= 2) cands.push_back({TRAJAM_KERNEL_MULTIWAVE, spw});
    for (int spw = 1; spw * 64 <= trajam::kMaxThreads; spw *= 2) cands.push_back({TRAJAM_KERNEL_WAVE, spw});
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(s, TRAJAM_ERR_DEVICE, "hipEventCreate failed");
    float best = 1e30f;
    std::pair<int, int> pick = {s->variant, s->tb};
    trajam_status status = TRAJAM_OK;
    for (const auto &cd : cands) {
        if (trajam_set_launch(s, cd.first, cd.second) != TRAJAM_OK) continue;
        float t_best = 1e30f;
        for (int rep = 0; rep < 3 && status == TRAJAM_OK; ++rep) {
            if (hipMemcpyAsync(xb, xi, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemsetAsync(lam, 0, bytes, st) != hipSuccess) {
                status = fail(s, TRAJAM_ERR_DEVICE, "autotune reset failed");
                break;
            }
            if (hipEventRecord(e0, st) != hipSuccess) {
                status = fail(s, TRAJAM_ERR_DEVICE, "autotune timing failed");
                break;
            }
            status = trajam_project(s, batch, xi, boundary, c, v, ax, xb, lam, probe_iters, nullptr, nullptr, stream);
            if (status != TRAJAM_OK) break;
            if (hipEventRecord(e1, st) != hipSuccess) {
                status = fail(s, TRAJAM_ERR_DEVICE, "autotune timing failed");
                break;
            }
            if (hipEventSynchronize(e1) != hipSuccess) {
                status = fail(s, TRAJAM_ERR_DEVICE, "autotune timing failed");
                break;
            }
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                status = fail(s, TRAJAM_ERR_DEVICE, "autotune timing failed");
                break;
            }
            if (rep > 0) t_best = std::min(t_best, ms);  // first run warms caches
        }
        if (status != TRAJAM_OK) break;
        if (best >= 1e29f || t_best < 0.97f * best) {
            best = t_best;
            pick = cd;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != TRAJAM_OK) return status;
    trajam_set_launch(s, pick.first, pick.second);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_store(key, pick.first, pick.second);
    }
    if (kernel_out) *kernel_out = pick.first;
    if (spw_out) *spw_out = pick.second;
    return TRAJAM_OK;
}

// Two work queues: single-robot problems (group 0) and multi-agent problems (group 1),
// each a table sorted longest-first, its unit offsets and its counter.
struct trajam_ragged_plan {
    void *d_bnd = nullptr;  // boundary coefficients of the multi-agent items
    void *d_probs[2] = {nullptr, nullptr};
    int *d_offsets[2] = {nullptr, nullptr};
    int *d_counter = nullptr;  // [2]
    int n[2] = {0, 0}, total[2] = {0, 0}, blocks[2] = {0, 0};
    int agent_stage = 0;  // floats per wave of the multi-agent kernel's obstacle stage
};

extern "C" void trajam_ragged_plan_destroy(trajam_ragged_plan *p)
{
    if (!p) return;
    for (int g = 0; g < 2; ++g) {
        if (p->d_probs[g]) (void)hipFree(p->d_probs[g]);
        if (p->d_offsets[g]) (void)hipFree(p->d_offsets[g]);
    }
    if (p->d_counter) (void)hipFree(p->d_counter);
    if (p->d_bnd) (void)hipFree(p->d_bnd);
    delete p;
}

extern "C" trajam_status trajam_ragged_plan_create(const trajam_ragged_item *items, int32_t n, int32_t iters,
                                                   trajam_ragged_plan **out)
{
    if (!out) return fail(nullptr, TRAJAM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!items || n < 1 || iters < 0) return fail(nullptr, TRAJAM_ERR_INVALID, "need items, n >= 1, iters >= 0");
    std::vector<AmArgs<float>> args(n);
    std::vector<double> cost(n);
    std::vector<float> agent_bnd;        // all multi-agent items' boundary coefficients
    std::vector<size_t> agent_off(n, 0);
    for (int i = 0; i < n; ++i) {
        const trajam_ragged_item &it = items[i];
        trajam_solver *s = it.solver;
        if (!s) return fail(nullptr, TRAJAM_ERR_INVALID, "item without solver");
        const trajam_problem &p = s->prob;
        if (p.precision != TRAJAM_FP32) return fail(nullptr, TRAJAM_ERR_UNSUPPORTED, "ragged launches need FP32 solvers");
        if (s->nv > 12 || p.n_steps > 128) return fail(nullptr, TRAJAM_ERR_UNSUPPORTED, "ragged: degree <= 11, n_steps <= 128");
        if (p.n_obstacles > 0 && !s->packed) return fail(nullptr, TRAJAM_ERR_INVALID, "ragged: call trajam_set_obstacles first");
        if (it.batch < 0 || it.batch > p.max_batch) return fail(nullptr, TRAJAM_ERR_INVALID, "ragged: bad batch");
        if (it.batch > 0 && (!it.xi || !it.xi_bar || !it.lambda || !it.boundary_host))
            return fail(nullptr, TRAJAM_ERR_INVALID, "ragged: NULL buffer");
        if (it.batch > 0)
            for (int q = 0; q < p.dims * 4; ++q)
                if (!std::isfinite(it.boundary_host[q])) return fail(nullptr, TRAJAM_ERR_INVALID, "ragged: non-finite boundary");
        AmArgs<float> &a = args[i];
        fill_args(s, a, it.batch, iters);
        a.dynamic = s->dynamic;
        if (p.n_agents > 1) {
            if (p.n_obstacles > 0) {
                const int stg = trajam::stage_fields(p.dims, p.obstacle_model == TRAJAM_SPHERE) * p.n_obstacles;
                a.cull_lds = stg <= trajam::kStageMaxFloats ? stg : 0;
            }
            const size_t cnt = (size_t)p.n_agents * p.dims * 4;
            if (it.batch > 0)
                for (size_t q = 0; q < cnt; ++q)
                    if (!std::isfinite(it.boundary_host[q])) return fail(nullptr, TRAJAM_ERR_INVALID, "ragged: non-finite boundary");
            std::vector<double> c(cnt, 0.0);
            if (it.batch > 0) c = agent_boundary_coeffs(p, it.boundary_host);
            agent_off[i] = agent_bnd.size();
            agent_bnd.insert(agent_bnd.end(), c.begin(), c.end());
        } else if (it.batch > 0)
            for (int ax = 0; ax < p.dims; ++ax) {
                double c4[4];
                boundary_coeffs(p.degree, p.horizon, it.boundary_host + 4 * ax, c4);
                for (int k = 0; k < 4; ++k) a.xiB[ax][k] = (float)c4[k];
            }
        a.xi = (const float *)it.xi;
        a.xb = (float *)it.xi_bar;
        a.lam = (float *)it.lambda;
        a.res = (float *)it.res_trace;
        a.flags = it.flags;
        cost[i] = (double)p.n_agents * (p.n_obstacles + p.n_agents + 2) * p.n_steps * p.dims;
    }
    trajam_ragged_plan *plan = new (std::nothrow) trajam_ragged_plan();
    if (!plan) return fail(nullptr, TRAJAM_ERR_DEVICE, "host allocation failed");
    for (int i = 0; i < n; ++i) plan->agent_stage = std::max(plan->agent_stage, args[i].cull_lds);
    hipError_t e = hipSuccess;
    if (!agent_bnd.empty()) {
        e = hipMalloc(&plan->d_bnd, sizeof(float) * agent_bnd.size());
        if (e == hipSuccess)
            e = hipMemcpy(plan->d_bnd, agent_bnd.data(), sizeof(float) * agent_bnd.size(), hipMemcpyHostToDevice);
        for (int i = 0; i < n; ++i)
            if (args[i].n_agents > 1) args[i].xiB_ag = (const float *)plan->d_bnd + agent_off[i];
    }
    if (e == hipSuccess) e = hipMalloc(&plan->d_counter, 2 * sizeof(int));
    for (int g = 0; g < 2 && e == hipSuccess; ++g) {
        std::vector<int> order;
        for (int i = 0; i < n; ++i)
            if ((args[i].n_agents > 1) == (g == 1)) order.push_back(i);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
        const int m = (int)order.size();
        std::vector<AmArgs<float>> sorted(m);
        std::vector<int> offsets(m + 1, 0);
        for (int k = 0; k < m; ++k) {
            sorted[k] = args[order[k]];
            offsets[k + 1] = offsets[k] + sorted[k].batch;
        }
        plan->n[g] = m;
        plan->total[g] = offsets[m];
        plan->blocks[g] = std::max(1, std::min((plan->total[g] + 3) / 4, 2048));
        if (m == 0) continue;
        e = hipMalloc(&plan->d_probs[g], sizeof(AmArgs<float>) * m);
        if (e == hipSuccess) e = hipMalloc(&plan->d_offsets[g], sizeof(int) * (m + 1));
        if (e == hipSuccess) e = hipMemcpy(plan->d_probs[g], sorted.data(), sizeof(AmArgs<float>) * m, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(plan->d_offsets[g], offsets.data(), sizeof(int) * (m + 1), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        trajam_ragged_plan_destroy(plan);
        return fail(nullptr, TRAJAM_ERR_DEVICE, std::string("ragged plan upload: ") + hipGetErrorString(e));
    }
    *out = plan;
    return TRAJAM_OK;
}

extern "C" trajam_status trajam_ragged_launch(trajam_ragged_plan *p, void *stream)
{
    if (!p) return fail(nullptr, TRAJAM_ERR_INVALID, "plan is NULL");
    for (int g = 0; g < 2; ++g) {
        if (p->total[g] == 0) continue;
        hipError_t e = trajam::launch_ragged((const AmArgs<float> *)p->d_probs[g], p->d_offsets[g], p->n[g],
                                             p->total[g], p->d_counter + g, p->blocks[g], g == 1, p->agent_stage,
                                             (hipStream_t)stream);
        if (e != hipSuccess)
            return fail(nullptr, TRAJAM_ERR_DEVICE, std::string("ragged launch: ") + hipGetErrorString(e));
    }
    return TRAJAM_OK;
}
