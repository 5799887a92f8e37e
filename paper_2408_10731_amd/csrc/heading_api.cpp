// C ABI of the heading / multi-circle variant (thesis ch. 5, Paper II, eqs
// reform_cost..d_bound and Alg 2): handle, host FP64 precompute of the two fixed QP
// operators, scene upload and the launch of heading_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "../../include/trajam.h"
#include "am_internal.h"

namespace trajam {
void host_basis(int n, int np, double T, std::vector<double> &P, std::vector<double> &Pd,
                std::vector<double> &Pdd);
bool host_spd_inverse(int n, const std::vector<double> &A, std::vector<double> &Ainv);
void host_boundary_coeffs(int n, double T, const double *b4, double *c4);
void set_thread_error(const std::string &msg);
void host_shift_matrix(int n, double d, double *S);
}  // namespace trajam

struct trajam_heading {
    trajam_heading_problem prob;
    int nv = 0;
    bool scene = false;
    trajam::HeadingArgs args{};
    void *d_phi = nullptr, *d_xdes = nullptr, *d_obs = nullptr, *d_W = nullptr, *d_Wpsi = nullptr;
    std::string err;
};

namespace {

constexpr int kHV = trajam::kHeadingMaxCoeffs;
constexpr int kHF = 2 * kHV - 4;

trajam_status hfail(trajam_heading *h, trajam_status st, const std::string &msg)
{
    if (h) h->err = msg;
    else trajam::set_thread_error(msg);
    return st;
}

template <typename T>
hipError_t put(void **dst, const std::vector<double> &src)
{
    std::vector<T> tmp(src.size());
    for (size_t i = 0; i < src.size(); ++i) tmp[i] = (T)src[i];
    if (!*dst) {
        hipError_t e = hipMalloc(dst, sizeof(T) * (tmp.empty() ? 1 : tmp.size()));
        if (e != hipSuccess) return e;
    }
    if (tmp.empty()) return hipSuccess;
    return hipMemcpy(*dst, tmp.data(), sizeof(T) * tmp.size(), hipMemcpyHostToDevice);
}

hipError_t put_prec(bool f64, void **dst, const std::vector<double> &src)
{
    return f64 ? put<double>(dst, src) : put<float>(dst, src);
}

trajam_status validate(const trajam_heading_problem *p, std::string &why)
{
    if (!p) { why = "problem is NULL"; return TRAJAM_ERR_INVALID; }
    if (p->degree < 4 || p->degree + 1 > kHV) { why = "degree must be in [4, 11]"; return TRAJAM_ERR_INVALID; }
    if (p->n_steps < p->degree + 1 || p->n_steps > 128) {
        why = "n_steps must be in [degree + 1, 128]";
        return TRAJAM_ERR_INVALID;
    }
    for (double v : {p->horizon, p->v_max, p->a_max, p->rho})
        if (!(v > 0.0) || !std::isfinite(v)) {
            why = "horizon, v_max, a_max and rho must be finite and > 0";
            return TRAJAM_ERR_INVALID;
        }
    if (p->n_circles < 1 || p->n_circles > TRAJAM_HEADING_MAX_CIRCLES) {
        why = "n_circles must be in [1, 8]";
        return TRAJAM_ERR_INVALID;
    }
    for (int m = 0; m < p->n_circles; ++m)
        if (!std::isfinite(p->radii[m])) { why = "radii must be finite"; return TRAJAM_ERR_INVALID; }
    if (p->n_obstacles < 0) { why = "n_obstacles must be >= 0"; return TRAJAM_ERR_INVALID; }
    if (p->max_batch < 1) { why = "max_batch must be >= 1"; return TRAJAM_ERR_INVALID; }
    if (p->precision != TRAJAM_FP64 && p->precision != TRAJAM_FP32) {
        why = "precision must be TRAJAM_FP64 or TRAJAM_FP32";
        return TRAJAM_ERR_INVALID;
    }
    return TRAJAM_OK;
}

// Inverse of the free block of a symmetric matrix M [dim x dim] over the index list
// `free`, padded into [ld x ld].
trajam_status free_inverse(const std::vector<double> &M, int dim, const std::vector<int> &free, int ld,
                           std::vector<double> &out, std::string &why)
{
    const int nf = (int)free.size();
    std::vector<double> Mf((size_t)nf * nf), inv;
    for (int i = 0; i < nf; ++i)
        for (int j = 0; j < nf; ++j) Mf[(size_t)i * nf + j] = M[(size_t)free[i] * dim + free[j]];
    if (!trajam::host_spd_inverse(nf, Mf, inv)) {
        why = "free block of a QP matrix is not positive definite";
        return TRAJAM_ERR_NUMERIC;
    }
    out.assign((size_t)ld * ld, 0.0);
    for (int i = 0; i < nf; ++i)
        for (int j = 0; j < nf; ++j) {
            const double v = inv[(size_t)i * nf + j];
            if (!std::isfinite(v)) { why = "non-finite QP operator"; return TRAJAM_ERR_NUMERIC; }
            out[(size_t)i * ld + j] = v;
        }
    return TRAJAM_OK;
}

void release(trajam_heading *h)
{
    for (void *p : {h->d_phi, h->d_xdes, h->d_obs, h->d_W, h->d_Wpsi})
        if (p) (void)hipFree(p);
    h->d_phi = h->d_xdes = h->d_obs = h->d_W = h->d_Wpsi = nullptr;
}

}  // namespace

extern "C" {

const char *trajam_heading_last_error(const trajam_heading *h) { return h ? h->err.c_str() : trajam_last_error(nullptr); }

void trajam_heading_destroy(trajam_heading *h)
{
    if (!h) return;
    release(h);
    delete h;
}

trajam_status trajam_heading_create(const trajam_heading_problem *p, trajam_heading **out)
{
    if (!out) return hfail(nullptr, TRAJAM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    std::string why;
    trajam_status st = validate(p, why);
    if (st != TRAJAM_OK) return hfail(nullptr, st, why);
    trajam_heading *h = new (std::nothrow) trajam_heading();
    if (!h) return hfail(nullptr, TRAJAM_ERR_DEVICE, "host allocation failed");
    h->prob = *p;
    const int n = p->degree, nv = n + 1, nt = p->n_steps;
    h->nv = nv;
    const double rho = p->rho;
    std::vector<double> P, Pd, Pdd;
    trajam::host_basis(n, nt, p->horizon, P, Pd, Pdd);
    auto gram = [&](const std::vector<double> &A) {
        std::vector<double> G((size_t)nv * nv, 0.0);
        for (int i = 0; i < nv; ++i)
            for (int j = 0; j < nv; ++j) {
                double s = 0.0;
                for (int k = 0; k < nt; ++k) s += A[(size_t)k * nv + i] * A[(size_t)k * nv + j];
                G[(size_t)i * nv + j] = s;
            }
        return G;
    };
    const std::vector<double> PP = gram(P), DD = gram(Pd), AA = gram(Pdd);
    double sr = 0.0, sr2 = 0.0;
    for (int m = 0; m < p->n_circles; ++m) {
        sr += p->radii[m];
        sr2 += p->radii[m] * p->radii[m];
    }
    const double no = p->n_obstacles, nc = p->n_circles;
    // Q + rho F'F of one position group, coefficients (x 0..n, c 0..n): the cost's
    // Pdd'Pdd + P'P on x; F's velocity and acceleration rows, n_o n_c collision rows
    // [P, r_m P] and the heading rows [0, P]
    const int dim = 2 * nv;
    std::vector<double> Q((size_t)dim * dim, 0.0);
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
            const size_t ij = (size_t)i * nv + j;
            Q[(size_t)i * dim + j] = AA[ij] + PP[ij] + rho * (DD[ij] + AA[ij] + no * nc * PP[ij]);
            Q[(size_t)i * dim + nv + j] = rho * no * sr * PP[ij];
            Q[(size_t)(nv + i) * dim + j] = rho * no * sr * PP[ij];
            Q[(size_t)(nv + i) * dim + nv + j] = rho * (no * sr2 + 1.0) * PP[ij];
        }
    std::vector<int> fx;
    for (int k = 3; k < n; ++k) fx.push_back(k);
    for (int k = 0; k < nv; ++k) fx.push_back(nv + k);
    std::vector<double> W, Wpsi;
    st = free_inverse(Q, dim, fx, kHF, W, why);
    if (st == TRAJAM_OK) {
        std::vector<double> Qp((size_t)nv * nv);
        for (size_t i = 0; i < Qp.size(); ++i) Qp[i] = AA[i] + rho * PP[i];
        std::vector<int> fp;
        for (int k = 1; k < n; ++k) fp.push_back(k);
        st = free_inverse(Qp, nv, fp, kHV, Wpsi, why);
    }
    if (st != TRAJAM_OK) {
        delete h;
        return hfail(nullptr, st, why);
    }
    std::vector<double> phi((size_t)3 * nt * kHV, 0.0);
    for (int k = 0; k < nt; ++k)
        for (int m = 0; m < nv; ++m) {
            phi[((size_t)0 * nt + k) * kHV + m] = P[(size_t)k * nv + m];
            phi[((size_t)1 * nt + k) * kHV + m] = Pd[(size_t)k * nv + m];
            phi[((size_t)2 * nt + k) * kHV + m] = Pdd[(size_t)k * nv + m];
        }
    const bool f64 = p->precision == TRAJAM_FP64;
    hipError_t e = put_prec(f64, &h->d_phi, phi);
    if (e == hipSuccess) e = put_prec(f64, &h->d_W, W);
    if (e == hipSuccess) e = put_prec(f64, &h->d_Wpsi, Wpsi);
    if (e == hipSuccess) e = put_prec(f64, &h->d_xdes, std::vector<double>((size_t)2 * nt, 0.0));
    if (e == hipSuccess) e = put_prec(f64, &h->d_obs, std::vector<double>((size_t)8 * p->n_obstacles, 0.0));
    if (e != hipSuccess) {
        trajam_heading_destroy(h);
        return hfail(nullptr, TRAJAM_ERR_DEVICE, std::string("heading tables: ") + hipGetErrorString(e));
    }
    trajam::HeadingArgs &a = h->args;
    a.phi = h->d_phi;
    a.x_des = h->d_xdes;
    a.obs = h->d_obs;
    a.W = h->d_W;
    a.Wpsi = h->d_Wpsi;
    for (int m = 0; m < trajam::kHeadingMaxCircles; ++m) a.radii[m] = m < p->n_circles ? p->radii[m] : 0.0;
    a.dt = p->horizon / (nt - 1);
    a.v_max = p->v_max;
    a.a_max = p->a_max;
    a.rho = rho;
    a.n_circles = p->n_circles;
    a.n_obs = p->n_obstacles;
    a.nv = nv;
    a.n_steps = nt;
    *out = h;
    return TRAJAM_OK;
}

trajam_status trajam_heading_set_scene(trajam_heading *h, const double *boundary, const double *x_des,
                                       const double *obstacles)
{
    if (!h) return TRAJAM_ERR_INVALID;
    h->err.clear();
    const trajam_heading_problem &p = h->prob;
    const int nt = p.n_steps, no = p.n_obstacles;
    if (!boundary || !x_des || (no > 0 && !obstacles)) return hfail(h, TRAJAM_ERR_INVALID, "NULL pointer");
    for (int i = 0; i < 10; ++i)
        if (!std::isfinite(boundary[i])) return hfail(h, TRAJAM_ERR_INVALID, "boundary rows must be finite");
    std::vector<double> xd(x_des, x_des + (size_t)2 * nt), ob((size_t)8 * no);
    for (double v : xd)
        if (!std::isfinite(v)) return hfail(h, TRAJAM_ERR_INVALID, "x_des must be finite");
    for (int j = 0; j < no; ++j) {
        const double *o = obstacles + (size_t)6 * j;
        for (int i = 0; i < 6; ++i)
            if (!std::isfinite(o[i])) return hfail(h, TRAJAM_ERR_INVALID, "obstacles must be finite");
        if (!(o[4] > 0.0) || !(o[5] > 0.0)) return hfail(h, TRAJAM_ERR_INVALID, "semi-axes must be > 0");
        for (int i = 0; i < 6; ++i) ob[(size_t)8 * j + i] = o[i];
        ob[(size_t)8 * j + 6] = 1.0 / o[4];
        ob[(size_t)8 * j + 7] = 1.0 / o[5];
    }
    trajam::HeadingArgs &a = h->args;
    for (int g = 0; g < 2; ++g) trajam::host_boundary_coeffs(p.degree, p.horizon, boundary + 4 * g, a.bcoef[g]);
    a.bpsi[0] = boundary[8];
    a.bpsi[1] = boundary[9];
    // the tables may be read by a projection still in flight on any stream
    hipError_t e = hipDeviceSynchronize();
    const bool f64 = p.precision == TRAJAM_FP64;
    if (e == hipSuccess) e = put_prec(f64, &h->d_xdes, xd);
    if (e == hipSuccess && no > 0) e = put_prec(f64, &h->d_obs, ob);
    if (e != hipSuccess) return hfail(h, TRAJAM_ERR_DEVICE, std::string("heading scene: ") + hipGetErrorString(e));
    h->scene = true;
    return TRAJAM_OK;
}

trajam_status trajam_heading_project(trajam_heading *h, int32_t batch, void *state, void *lambda, int32_t iters,
                                     void *res_trace, void *stream)
{
    if (!h) return TRAJAM_ERR_INVALID;
    h->err.clear();
    if (batch < 0 || iters < 0) return hfail(h, TRAJAM_ERR_INVALID, "batch and iters must be >= 0");
    if (batch > h->prob.max_batch) return hfail(h, TRAJAM_ERR_CAPACITY, "batch > max_batch");
    if (!h->scene) return hfail(h, TRAJAM_ERR_INVALID, "trajam_heading_set_scene has not been called");
    if (batch == 0) return TRAJAM_OK;
    if (!state || !lambda) return hfail(h, TRAJAM_ERR_INVALID, "NULL pointer");
    hipError_t e = trajam::launch_heading(h->prob.precision == TRAJAM_FP64, h->args, batch, iters, state, lambda,
                                          iters > 0 ? res_trace : nullptr, (hipStream_t)stream);
    if (e != hipSuccess) return hfail(h, TRAJAM_ERR_DEVICE, std::string("heading: ") + hipGetErrorString(e));
    return TRAJAM_OK;
}

trajam_status trajam_heading_shift(trajam_heading *h, int32_t batch, double delta, int32_t keep_lambda, void *state,
                                   void *lambda, void *stream)
{
    if (!h) return TRAJAM_ERR_INVALID;
    h->err.clear();
    if (batch < 0 || !std::isfinite(delta) || (keep_lambda != 0 && keep_lambda != 1))
        return hfail(h, TRAJAM_ERR_INVALID, "batch >= 0, finite delta, keep_lambda 0 or 1 required");
    if (batch > h->prob.max_batch) return hfail(h, TRAJAM_ERR_CAPACITY, "batch > max_batch");
    if (batch == 0) return TRAJAM_OK;
    if (!state || !lambda) return hfail(h, TRAJAM_ERR_INVALID, "NULL pointer");
    trajam::ShiftMatrix S;
    S.nv = h->nv;
    trajam::host_shift_matrix(h->prob.degree, delta / h->prob.horizon, S.s);
    // each row of a sample (x, c, y, s, psi) is read whole before it is written, so the
    // shift runs in place
    hipError_t e = trajam::launch_mpc_shift(h->prob.precision == TRAJAM_FP64, batch * 5, S, state, lambda, state,
                                            state, lambda, keep_lambda, (hipStream_t)stream);
    if (e != hipSuccess) return hfail(h, TRAJAM_ERR_DEVICE, std::string("heading shift: ") + hipGetErrorString(e));
    return TRAJAM_OK;
}

}  // extern "C"
