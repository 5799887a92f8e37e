// gfx950 kernel of the heading / multi-circle variant of the batch optimizer (thesis
// ch. 5, Paper II: a rectangular robot as n_c circles on its heading axis; eq
// reform_formulation and Alg 2).  Per sample the state is the Bernstein coefficients of
// x, c, y, s (c, s: slack copies of cos psi, sin psi) and psi, and the multipliers of
// the same five rows.
//
// One wave64 per sample, time step t on lanes t and t - 64 (n_t <= 128).  Both QPs are
// applied in delta form: with A xi = b already met, the step is
//     xi_f += W (lam + T(xi) - rho F'(F xi - g))_f
// (W: the inverse of the free block of Q + rho F'F, T(xi) = P'(x_des - x) - Pdd'Pdd xi
// on the position rows), and for the heading
//     psi_f += W_psi (lam_psi - Pdd'Pdd xi_psi + rho P'(psi_t - P xi_psi))_f,
// whose right-hand sides are contractions over time of per-step residuals, small near
// a fixed point, which keeps FP32 accurate.  F'(F xi - g) of the state after the polar
// step is at once the multiplier update and the next position step's residual.
// Coefficient vectors live in LDS (one slice per wave); the contractions over time are
// wave reductions; every exchange between the lanes of a wave orders LDS only.
#include <hip/hip_runtime.h>

#include "am_internal.h"

namespace trajam {
namespace {

constexpr int kHV = kHeadingMaxCoeffs;     // coefficient slots per row
constexpr int kHF = 2 * kHV - 4;           // free coefficients of one position group, padded

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Sum over the wave, the same value in every lane: within each row of 16 lanes by DPP
// (pairs, quads, half-row and row mirrors), then the four row sums read as scalars.
template <int C>
__device__ __forceinline__ float dpp(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), C, 0xF, 0xF, false));
}
template <int C>
__device__ __forceinline__ double dpp(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), C, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), C, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_value(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double lane_value(double v, int l)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    v += dpp<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp<0x141>(v);   // row_half_mirror
    v += dpp<0x140>(v);   // row_mirror
    return ((lane_value(v, 0) + lane_value(v, 16)) + lane_value(v, 32)) + lane_value(v, 48);
}

// (|w|, w / |w|) of w = (u, v), with (0, (1, 0)) at the origin (atan2(+0, +0) = 0).
// FP32 through the hardware reciprocal square root; FP64 by division.
__device__ __forceinline__ void norm_dir(float u, float v, float &rn, float &cu, float &sv)
{
    const float s2 = fmaf(u, u, v * v);
    const float ri = s2 > 0.0f ? __builtin_amdgcn_rsqf(s2) : 0.0f;
    rn = s2 * ri;
    cu = s2 > 0.0f ? u * ri : 1.0f;
    sv = v * ri;
}
__device__ __forceinline__ void norm_dir(double u, double v, double &rn, double &cu, double &sv)
{
    rn = sqrt(u * u + v * v);
    cu = rn > 0.0 ? u / rn : 1.0;
    sv = rn > 0.0 ? v / rn : 0.0;
}

__device__ __forceinline__ float unwrap_pi2(float) { return 6.28318530717958647692f; }
__device__ __forceinline__ double unwrap_pi2(double) { return 6.28318530717958647692; }

// Values of one time step.
template <typename T>
struct Step {
    T x, c, y, s, vx, vy, ax, ay, psi, psidd;
};

template <typename T>
__device__ __forceinline__ T dot_row(const T *row, const T *coef, int nv)
{
    T acc = 0;
#pragma unroll
    for (int k = 0; k < kHV; ++k)
        if (k < nv) acc = fma(row[k], coef[k], acc);
    return acc;
}

// Per-step residual pieces of F xi - g after the polar step (Alg 2 steps 3-4) and the
// tracking terms: rx/ry sum the collision rows, rc/rs add r_m times them and the
// heading rows; ev*/ea* the velocity / acceleration rows; sq their squares.
template <typename T>
struct Rows {
    T rx, rc, ry, rs, evx, evy, eax, eay, sq;
};

template <typename T>
__device__ __forceinline__ void ball_row(T vx, T vy, T bound, T &ex, T &ey)
{
    // target bound * min(1, |v| / bound) * (cos, sin)(atan2(vy, vx)); atan2(0, 0) = 0
    T n, cx, sy;
    norm_dir(vx, vy, n, cx, sy);
    const T d = n < bound ? n / bound : (T)1;
    ex = vx - bound * d * cx;
    ey = vy - bound * d * sy;
}

// The rows of a lane's two time steps together (two independent chains per obstacle).
template <typename T>
__device__ __forceinline__ void polar_rows2(const HeadingArgs &a, const Step<T> *p, const T *t, const T *cps,
                                            const T *sps, const bool *on, Rows<T> *r)
{
    const T *ob = (const T *)a.obs;
#pragma unroll
    for (int h = 0; h < 2; ++h) r[h] = Rows<T>{};
    for (int m = 0; m < a.n_circles; ++m) {
        const T rm = (T)a.radii[m];
        T px[2], py[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            px[h] = p[h].x + rm * cps[h];   // circle centre on the heading
            py[h] = p[h].y + rm * sps[h];
        }
        for (int j = 0; j < a.n_obs; ++j) {
            const T *o = ob + (size_t)j * 8;    // cx, cy, vx, vy, a, b, 1/a, 1/b
            {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const T xo = fma(o[2], t[h], o[0]), yo = fma(o[3], t[h], o[1]);
                    const T u = (px[h] - xo) * o[6], v = (py[h] - yo) * o[7];
                    T rn, ca, sa;
                    norm_dir(u, v, rn, ca, sa);
                    const T d = rn > (T)1 ? rn : (T)1;
                    // the row value F xi uses the slack: x + r_m c, y + r_m s
                    const T ex = fma(rm, p[h].c, p[h].x) - (xo + o[4] * d * ca);
                    const T ey = fma(rm, p[h].s, p[h].y) - (yo + o[5] * d * sa);
                    r[h].rx += ex;
                    r[h].ry += ey;
                    r[h].rc = fma(rm, ex, r[h].rc);
                    r[h].rs = fma(rm, ey, r[h].rs);
                    r[h].sq = fma(ex, ex, fma(ey, ey, r[h].sq));
                }
            }
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const T ec = p[h].c - cps[h], es = p[h].s - sps[h];
        r[h].rc += ec;
        r[h].rs += es;
        ball_row(p[h].vx, p[h].vy, (T)a.v_max, r[h].evx, r[h].evy);
        ball_row(p[h].ax, p[h].ay, (T)a.a_max, r[h].eax, r[h].eay);
        r[h].sq += ec * ec + es * es + r[h].evx * r[h].evx + r[h].evy * r[h].evy + r[h].eax * r[h].eax +
                   r[h].eay * r[h].eay;
        if (!on[h]) r[h] = Rows<T>{};
    }
}

template <typename T>
__global__ __launch_bounds__(256) void heading_kernel(HeadingArgs a, int batch, int iters, T *state, T *lam,
                                                      T *trace)
{
    __shared__ T lds[4][3][5][kHV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.x * 4 + wave;
    if (b >= batch) return;   // whole wave; no workgroup barrier below
    T(*XI)[kHV] = lds[wave][0];
    T(*LM)[kHV] = lds[wave][1];
    T(*V)[kHV] = lds[wave][2];
    const int nv = a.nv, nt = a.n_steps, n = nv - 1, nfp = nv - 4, nfx = 2 * nv - 4;
    const T rho = (T)a.rho;
    const T *phi = (const T *)a.phi;      // [3][n_t][kHV]: P, Pd, Pdd
    const T *xdes = (const T *)a.x_des;   // [2][n_t]

    for (int i = lane; i < 5 * kHV; i += 64) {
        const int r = i / kHV, k = i % kHV;
        XI[r][k] = k < nv ? state[((size_t)b * 5 + r) * nv + k] : (T)0;
        LM[r][k] = k < nv ? lam[((size_t)b * 5 + r) * nv + k] : (T)0;
        V[r][k] = 0;
    }
    wave_sync_lds();
    // the boundary rows fix coefficients 0, 1, 2, n of x and y and 0, n of psi
    if (lane < 2) {
        XI[2 * lane][0] = (T)a.bcoef[lane][0];
        XI[2 * lane][1] = (T)a.bcoef[lane][1];
        XI[2 * lane][2] = (T)a.bcoef[lane][2];
        XI[2 * lane][n] = (T)a.bcoef[lane][3];
    } else if (lane == 2) {
        XI[4][0] = (T)a.bpsi[0];
        XI[4][n] = (T)a.bpsi[1];
    }
    wave_sync_lds();

    // basis rows of this lane's (up to) two time steps
    T Pr[2][kHV], Pdr[2][kHV], Pddr[2][kHV], tt[2], xd[2], yd[2];
    bool on[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int t = lane + 64 * h;
        on[h] = t < nt;
        const int tc = on[h] ? t : 0;
#pragma unroll
        for (int k = 0; k < kHV; ++k) {
            Pr[h][k] = on[h] ? phi[((size_t)0 * nt + tc) * kHV + k] : (T)0;
            Pdr[h][k] = on[h] ? phi[((size_t)1 * nt + tc) * kHV + k] : (T)0;
            Pddr[h][k] = on[h] ? phi[((size_t)2 * nt + tc) * kHV + k] : (T)0;
        }
        tt[h] = (T)a.dt * (T)tc;
        xd[h] = on[h] ? xdes[tc] : (T)0;
        yd[h] = on[h] ? xdes[nt + tc] : (T)0;
    }

    Step<T> st[2];
    Rows<T> rw[2];
    T cps[2], sps[2];

    auto eval_pos = [&]() {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            st[h].x = dot_row(Pr[h], XI[0], nv);
            st[h].c = dot_row(Pr[h], XI[1], nv);
            st[h].y = dot_row(Pr[h], XI[2], nv);
            st[h].s = dot_row(Pr[h], XI[3], nv);
            st[h].vx = dot_row(Pdr[h], XI[0], nv);
            st[h].vy = dot_row(Pdr[h], XI[2], nv);
            st[h].ax = dot_row(Pddr[h], XI[0], nv);
            st[h].ay = dot_row(Pddr[h], XI[2], nv);
        }
    };
    auto eval_psi = [&]() {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            st[h].psi = dot_row(Pr[h], XI[4], nv);
            st[h].psidd = dot_row(Pddr[h], XI[4], nv);
            cps[h] = cos(st[h].psi);
            sps[h] = sin(st[h].psi);
        }
    };
    // polar step at the current state, then per coefficient k the contractions
    // F'(F xi - g) of both groups and the tracking terms; lane k keeps coefficient k.
    // With `update`, also lam -= rho F'(F xi - g) and lam_psi -= rho P'(psi - psi_t).
    // Writes V = lam + T - rho F'(F xi - g) (position groups).
    T dpsi[2] = {0, 0};
    auto polar_and_contract = [&](bool update, int k_iter) {
        polar_rows2(a, st, tt, cps, sps, on, rw);
        T sq = rw[0].sq + rw[1].sq;
        T sq2 = fma(dpsi[0], dpsi[0], dpsi[1] * dpsi[1]);
        // lane k keeps coefficient k's sums (selects, no branch), then updates once
        T cfx = 0, cfc = 0, cfy = 0, cfs = 0, ctx = 0, cty = 0, clp = 0;
#pragma unroll
        for (int k = 0; k < kHV; ++k) {
            if (k >= nv) continue;   // uniform
            T fx = 0, fc = 0, fy = 0, fs = 0, tx = 0, ty = 0, lp = 0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const T p = Pr[h][k], pd = Pdr[h][k], pdd = Pddr[h][k];
                fx = fma(p, rw[h].rx, fma(pd, rw[h].evx, fma(pdd, rw[h].eax, fx)));
                fy = fma(p, rw[h].ry, fma(pd, rw[h].evy, fma(pdd, rw[h].eay, fy)));
                fc = fma(p, rw[h].rc, fc);
                fs = fma(p, rw[h].rs, fs);
                if (on[h]) {
                    tx = fma(p, xd[h] - st[h].x, fma(-pdd, st[h].ax, tx));
                    ty = fma(p, yd[h] - st[h].y, fma(-pdd, st[h].ay, ty));
                }
                lp = fma(p, dpsi[h], lp);
            }
            fx = wave_sum(fx);
            fc = wave_sum(fc);
            fy = wave_sum(fy);
            fs = wave_sum(fs);
            tx = wave_sum(tx);
            ty = wave_sum(ty);
            if (update) lp = wave_sum(lp);
            const bool mine = lane == k;
            cfx = mine ? fx : cfx;
            cfc = mine ? fc : cfc;
            cfy = mine ? fy : cfy;
            cfs = mine ? fs : cfs;
            ctx = mine ? tx : ctx;
            cty = mine ? ty : cty;
            clp = mine ? lp : clp;
        }
        if (lane < nv) {
            const int k = lane;
            if (update) {
                LM[0][k] -= rho * cfx;
                LM[1][k] -= rho * cfc;
                LM[2][k] -= rho * cfy;
                LM[3][k] -= rho * cfs;
                LM[4][k] -= rho * clp;
            }
            V[0][k] = LM[0][k] + ctx - rho * cfx;
            V[1][k] = LM[1][k] - rho * cfc;
            V[2][k] = LM[2][k] + cty - rho * cfy;
            V[3][k] = LM[3][k] - rho * cfs;
        }
        if (trace && update) {
            sq = wave_sum(sq);
            sq2 = wave_sum(sq2);
            if (lane == 0) {
                trace[((size_t)k_iter * batch + b) * 2 + 0] = sqrt(sq);
                trace[((size_t)k_iter * batch + b) * 2 + 1] = sqrt(sq2);
            }
        }
        wave_sync_lds();
    };

    eval_pos();
    eval_psi();
    polar_and_contract(false, 0);

    // this lane's rows of both QP operators, held for the launch: W [kHF][kHF] (free x
    // coefficients 3..n-1, then c 0..n; row lane & 31), W_psi [kHV][kHV] (free psi
    // coefficients 1..n-1; row lane)
    T wrow[kHF], wprow[kHV];
    {
        const T *W = (const T *)a.W;
        const T *Wp = (const T *)a.Wpsi;
        const int i = lane & 31;
#pragma unroll
        for (int j = 0; j < kHF; ++j) wrow[j] = (i < nfx && j < nfx) ? W[(size_t)i * kHF + j] : (T)0;
#pragma unroll
        for (int j = 0; j < kHV; ++j) wprow[j] = (lane < n - 1 && j < n - 1) ? Wp[(size_t)lane * kHV + j] : (T)0;
    }
    const T two_pi = unwrap_pi2((T)0);
    for (int it = 0; it < iters; ++it) {
        // step 1: the position / slack QP of both groups (lanes 0..31: x, 32..63: y)
        {
            const int g = lane >> 5, i = lane & 31;
            T d = 0;
#pragma unroll
            for (int j = 0; j < kHF; ++j) {
                if (j < nfx) {   // uniform
                    const T vj = j < nfp ? V[2 * g][3 + j] : V[2 * g + 1][j - nfp];
                    d = fma(wrow[j], vj, d);
                }
            }
            wave_sync_lds();
            if (i < nfx) {
                if (i < nfp) XI[2 * g][3 + i] += d;
                else XI[2 * g + 1][i - nfp] += d;
            }
            wave_sync_lds();
        }
        // step 2: heading target and the surrogate QP
        eval_pos();
        T pt[2], cr = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const T th = atan2(st[h].s, st[h].c);
            pt[h] = on[h] ? th + two_pi * rint((st[h].psi - th) / two_pi) : (T)0;
        }
#pragma unroll
        for (int k = 0; k < kHV; ++k) {
            if (k < nv) {   // uniform
                T r = 0;
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    if (on[h]) r = fma(-Pddr[h][k], st[h].psidd, fma(rho * Pr[h][k], pt[h] - st[h].psi, r));
                r = wave_sum(r);
                cr = lane == k ? r : cr;
            }
        }
        if (lane < nv) V[4][lane] = LM[4][lane] + cr;
        wave_sync_lds();
        {
            T d = 0;
#pragma unroll
            for (int j = 0; j < kHV; ++j)
                if (j < n - 1) d = fma(wprow[j], V[4][1 + j], d);   // zero rows past n - 2
            wave_sync_lds();
            if (lane < n - 1) XI[4][1 + lane] += d;
            wave_sync_lds();
        }
        eval_psi();
#pragma unroll
        for (int h = 0; h < 2; ++h) dpsi[h] = on[h] ? st[h].psi - pt[h] : (T)0;
        // steps 3-5: polar step at the new state, multipliers, the next step's residual
        polar_and_contract(true, it);
    }

    for (int i = lane; i < 5 * nv; i += 64) {
        const int r = i / nv, k = i % nv;
        state[((size_t)b * 5 + r) * nv + k] = XI[r][k];
        lam[((size_t)b * 5 + r) * nv + k] = LM[r][k];
    }
}

}  // namespace

hipError_t launch_heading(bool fp64, const HeadingArgs &a, int batch, int iters, void *state, void *lam,
                          void *trace, hipStream_t st)
{
    if (batch <= 0) return hipSuccess;
    const dim3 grid((batch + 3) / 4), block(256);
    if (fp64)
        heading_kernel<double><<<grid, block, 0, st>>>(a, batch, iters, (double *)state, (double *)lam,
                                                        (double *)trace);
    else
        heading_kernel<float><<<grid, block, 0, st>>>(a, batch, iters, (float *)state, (float *)lam,
                                                      (float *)trace);
    return hipGetLastError();
}

}  // namespace trajam
