// gfx950 kernel of the heading / multi-circle variant of the batch optimizer (thesis
// ch. 5, Paper II: a rectangular robot as n_c circles on its heading axis; eq
// reform_formulation and Alg 2).  Per sample the state is the Bernstein coefficients of
// x, c, y, s (c, s: slack copies of cos psi, sin psi) and psi, and the multipliers of
// the same five rows.
//
// One workgroup of two wave64s per sample, time step t on thread t (n_t <= 128).  Both QPs are
// applied in delta form: with A xi = b already met, the step is
//     xi_f += W (lam + T(xi) - rho F'(F xi - g))_f
// (W: the inverse of the free block of Q + rho F'F, T(xi) = P'(x_des - x) - Pdd'Pdd xi
// on the position rows), and for the heading
//     psi_f += W_psi (lam_psi - Pdd'Pdd xi_psi + rho P'(psi_t - P xi_psi))_f,
// whose right-hand sides are contractions over time of per-step residuals, small near
// a fixed point, which keeps FP32 accurate.  F'(F xi - g) of the state after the polar
// step is at once the multiplier update and the next position step's residual.
// Coefficient vectors live in LDS; a contraction over time is a DPP sum in each wave,
// the two waves' sums added in a fixed order after a workgroup barrier.
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

// The rows of one time step.
template <typename T>
__device__ __forceinline__ Rows<T> polar_rows(const HeadingArgs &a, const Step<T> &p, T t, T cps, T sps)
{
    const T *ob = (const T *)a.obs;
    Rows<T> r{};
    for (int m = 0; m < a.n_circles; ++m) {
        const T rm = (T)a.radii[m];
        const T px = p.x + rm * cps, py = p.y + rm * sps;   // circle centre on the heading
        const T fx = fma(rm, p.c, p.x), fy = fma(rm, p.s, p.y);   // the row value F xi (slack)
        for (int j = 0; j < a.n_obs; ++j) {
            const T *o = ob + (size_t)j * 8;    // cx, cy, vx, vy, a, b, 1/a, 1/b
            const T xo = fma(o[2], t, o[0]), yo = fma(o[3], t, o[1]);
            const T u = (px - xo) * o[6], v = (py - yo) * o[7];
            T rn, ca, sa;
            norm_dir(u, v, rn, ca, sa);
            const T d = rn > (T)1 ? rn : (T)1;
            const T ex = fx - (xo + o[4] * d * ca);
            const T ey = fy - (yo + o[5] * d * sa);
            r.rx += ex;
            r.ry += ey;
            r.rc = fma(rm, ex, r.rc);
            r.rs = fma(rm, ey, r.rs);
            r.sq = fma(ex, ex, fma(ey, ey, r.sq));
        }
    }
    const T ec = p.c - cps, es = p.s - sps;
    r.rc += ec;
    r.rs += es;
    ball_row(p.vx, p.vy, (T)a.v_max, r.evx, r.evy);
    ball_row(p.ax, p.ay, (T)a.a_max, r.eax, r.eay);
    r.sq += ec * ec + es * es + r.evx * r.evx + r.evy * r.evy + r.eax * r.eax + r.eay * r.eay;
    return r;
}

__device__ __forceinline__ void block_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int kHThreads = 128;   // two waves, one time step each thread
constexpr int kParts = 8;        // contraction vectors per wave (7 used by the polar step, 1 by psi)

template <typename T>
__global__ __launch_bounds__(kHThreads) void heading_kernel(HeadingArgs a, int iters, int batch, T *state, T *lam,
                                                            T *trace)
{
    __shared__ T XI[5][kHV], LM[5][kHV], V[5][kHV];
    __shared__ T part[2][kParts][kHV];   // per wave: the sums its lanes k captured
    __shared__ T red[2][2];              // per wave: the squared residuals
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int b = blockIdx.x;            // the grid is the batch: no workgroup leaves early
    const int nv = a.nv, nt = a.n_steps, n = nv - 1, nfp = nv - 4, nfx = 2 * nv - 4;
    const T rho = (T)a.rho;
    const T *phi = (const T *)a.phi;      // [3][n_t][kHV]: P, Pd, Pdd
    const T *xdes = (const T *)a.x_des;   // [2][n_t]

    if (tid < 5 * kHV) {
        const int r = tid / kHV, k = tid % kHV;
        XI[r][k] = k < nv ? state[((size_t)b * 5 + r) * nv + k] : (T)0;
        LM[r][k] = k < nv ? lam[((size_t)b * 5 + r) * nv + k] : (T)0;
        V[r][k] = 0;
    }
    block_sync_lds();
    // the boundary rows fix coefficients 0, 1, 2, n of x and y and 0, n of psi
    if (tid < 2) {
        XI[2 * tid][0] = (T)a.bcoef[tid][0];
        XI[2 * tid][1] = (T)a.bcoef[tid][1];
        XI[2 * tid][2] = (T)a.bcoef[tid][2];
        XI[2 * tid][n] = (T)a.bcoef[tid][3];
    } else if (tid == 2) {
        XI[4][0] = (T)a.bpsi[0];
        XI[4][n] = (T)a.bpsi[1];
    }
    block_sync_lds();

    // this thread's time step and basis rows
    const bool on = tid < nt;
    const int tc = on ? tid : 0;
    T Pr[kHV], Pdr[kHV], Pddr[kHV];
#pragma unroll
    for (int k = 0; k < kHV; ++k) {
        Pr[k] = on ? phi[((size_t)0 * nt + tc) * kHV + k] : (T)0;
        Pdr[k] = on ? phi[((size_t)1 * nt + tc) * kHV + k] : (T)0;
        Pddr[k] = on ? phi[((size_t)2 * nt + tc) * kHV + k] : (T)0;
    }
    const T tt = (T)a.dt * (T)tc;
    const T xd = on ? xdes[tc] : (T)0, yd = on ? xdes[nt + tc] : (T)0;
    // this thread's rows of the QP operators, held for the launch: W [kHF][kHF] (free x
    // coefficients 3..n-1, then c 0..n; wave g applies group g, row lane), W_psi
    // [kHV][kHV] (free psi coefficients 1..n-1; wave 0, row lane)
    T wrow[kHF], wprow[kHV];
#pragma unroll
    for (int j = 0; j < kHF; ++j)
        wrow[j] = (lane < nfx && j < nfx) ? ((const T *)a.W)[(size_t)lane * kHF + j] : (T)0;
#pragma unroll
    for (int j = 0; j < kHV; ++j)
        wprow[j] = (wave == 0 && lane < n - 1 && j < n - 1) ? ((const T *)a.Wpsi)[(size_t)lane * kHV + j] : (T)0;

    Step<T> st;
    T cps = 1, sps = 0, dpsi = 0;
    auto eval_pos = [&]() {
        st.x = dot_row(Pr, XI[0], nv);
        st.c = dot_row(Pr, XI[1], nv);
        st.y = dot_row(Pr, XI[2], nv);
        st.s = dot_row(Pr, XI[3], nv);
        st.vx = dot_row(Pdr, XI[0], nv);
        st.vy = dot_row(Pdr, XI[2], nv);
        st.ax = dot_row(Pddr, XI[0], nv);
        st.ay = dot_row(Pddr, XI[2], nv);
    };
    auto eval_psi = [&]() {
        st.psi = dot_row(Pr, XI[4], nv);
        st.psidd = dot_row(Pddr, XI[4], nv);
        cps = cos(st.psi);
        sps = sin(st.psi);
    };
    // polar step at the current state, then per coefficient k the contractions
    // F'(F xi - g) of both groups and the tracking terms (lane k of each wave keeps its
    // wave's sums of coefficient k; thread k adds the two waves').  With `update`, also
    // lam -= rho F'(F xi - g) and lam_psi -= rho P'(psi - psi_t).  Writes
    // V = lam + T - rho F'(F xi - g) of the position groups.
    auto polar_and_contract = [&](bool update, int k_iter) {
        Rows<T> rw = on ? polar_rows(a, st, tt, cps, sps) : Rows<T>{};
        T c[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < kHV; ++k) {
            if (k >= nv) continue;   // uniform
            const T p = Pr[k], pd = Pdr[k], pdd = Pddr[k];
            T f[7];
            f[0] = wave_sum(fma(p, rw.rx, fma(pd, rw.evx, pdd * rw.eax)));
            f[1] = wave_sum(p * rw.rc);
            f[2] = wave_sum(fma(p, rw.ry, fma(pd, rw.evy, pdd * rw.eay)));
            f[3] = wave_sum(p * rw.rs);
            f[4] = wave_sum(on ? fma(p, xd - st.x, -pdd * st.ax) : (T)0);
            f[5] = wave_sum(on ? fma(p, yd - st.y, -pdd * st.ay) : (T)0);
            f[6] = update ? wave_sum(p * dpsi) : (T)0;
            const bool mine = lane == k;
#pragma unroll
            for (int q = 0; q < 7; ++q) c[q] = mine ? f[q] : c[q];
        }
        if (lane < nv) {
#pragma unroll
            for (int q = 0; q < 7; ++q) part[wave][q][lane] = c[q];
        }
        const T sq = wave_sum(rw.sq), sq2 = wave_sum(dpsi * dpsi);
        if (lane == 0) {
            red[wave][0] = sq;
            red[wave][1] = sq2;
        }
        block_sync_lds();
        if (tid < nv) {
            const int k = tid;
            T s[7];
#pragma unroll
            for (int q = 0; q < 7; ++q) s[q] = part[0][q][k] + part[1][q][k];
            if (update) {
                LM[0][k] -= rho * s[0];
                LM[1][k] -= rho * s[1];
                LM[2][k] -= rho * s[2];
                LM[3][k] -= rho * s[3];
                LM[4][k] -= rho * s[6];
            }
            V[0][k] = LM[0][k] + s[4] - rho * s[0];
            V[1][k] = LM[1][k] - rho * s[1];
            V[2][k] = LM[2][k] + s[5] - rho * s[2];
            V[3][k] = LM[3][k] - rho * s[3];
        }
        if (trace && update && tid == 0) {
            trace[((size_t)k_iter * batch + b) * 2 + 0] = sqrt(red[0][0] + red[1][0]);
            trace[((size_t)k_iter * batch + b) * 2 + 1] = sqrt(red[0][1] + red[1][1]);
        }
        block_sync_lds();
    };

    eval_pos();
    eval_psi();
    polar_and_contract(false, 0);

    const T two_pi = unwrap_pi2((T)0);
    for (int it = 0; it < iters; ++it) {
        // step 1: the position / slack QP (wave 0: group x, wave 1: group y)
        {
            const int g = wave;
            T d = 0;
#pragma unroll
            for (int j = 0; j < kHF; ++j) {
                if (j < nfx) {   // uniform
                    const T vj = j < nfp ? V[2 * g][3 + j] : V[2 * g + 1][j - nfp];
                    d = fma(wrow[j], vj, d);
                }
            }
            if (lane < nfx) {
                if (lane < nfp) XI[2 * g][3 + lane] += d;
                else XI[2 * g + 1][lane - nfp] += d;
            }
            block_sync_lds();
        }
        // step 2: heading target and the surrogate QP
        eval_pos();
        const T th = atan2(st.s, st.c);
        const T pt = on ? th + two_pi * rint((st.psi - th) / two_pi) : (T)0;
        {
            T c = 0;
#pragma unroll
            for (int k = 0; k < kHV; ++k) {
                if (k < nv) {   // uniform
                    const T r = wave_sum(on ? fma(-Pddr[k], st.psidd, rho * Pr[k] * (pt - st.psi)) : (T)0);
                    c = lane == k ? r : c;
                }
            }
            if (lane < nv) part[wave][7][lane] = c;
            block_sync_lds();
            if (wave == 0) {
                T d = 0;
#pragma unroll
                for (int j = 0; j < kHV; ++j)
                    if (j < n - 1) {   // zero rows past n - 2
                        const T vj = LM[4][1 + j] + part[0][7][1 + j] + part[1][7][1 + j];
                        d = fma(wprow[j], vj, d);
                    }
                if (lane < n - 1) XI[4][1 + lane] += d;
            }
            block_sync_lds();
        }
        eval_psi();
        dpsi = on ? st.psi - pt : (T)0;
        // steps 3-5: polar step at the new state, multipliers, the next step's residual
        polar_and_contract(true, it);
    }

    if (tid < 5 * nv) {
        const int r = tid / nv, k = tid % nv;
        state[((size_t)b * 5 + r) * nv + k] = XI[r][k];
        lam[((size_t)b * 5 + r) * nv + k] = LM[r][k];
    }
}

}  // namespace

hipError_t launch_heading(bool fp64, const HeadingArgs &a, int batch, int iters, void *state, void *lam,
                          void *trace, hipStream_t st)
{
    if (batch <= 0) return hipSuccess;
    const dim3 grid(batch), block(kHThreads);
    if (fp64)
        heading_kernel<double><<<grid, block, 0, st>>>(a, iters, batch, (double *)state, (double *)lam,
                                                        (double *)trace);
    else
        heading_kernel<float><<<grid, block, 0, st>>>(a, iters, batch, (float *)state, (float *)lam,
                                                      (float *)trace);
    return hipGetLastError();
}

}  // namespace trajam
