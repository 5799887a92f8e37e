// gfx950 kernels of the batched alternating-minimization (AM) projection of
// Bernstein trajectories (thesis ch. 6, eqs comp_alpha .. comp_zeta).
//
// Design (MI355X first):
//  * Samples are independent for the whole iteration, so one launch runs all K
//    iterations: each workgroup owns `tb` samples and keeps their state (xb in LDS,
//    lambda and xi in registers of the owning lanes) on chip from the first
//    iteration to the last.  HBM sees xi / xb / lambda once in and once out, plus
//    the residual trace: the kernel is bound by the VALU, not by memory.
//  * Lane layout: `tpad` lanes per sample (n_p rounded up to whole wave64s), lane t
//    owns time sample t.  Its rows of P, Pd, Pdd stay in registers for the whole
//    launch, so the waypoint map (eq parameter) and its transpose are register FMAs.
//  * The obstacle loop reads one packed obstacle record per step at a wave-uniform
//    address, which the compiler turns into scalar loads: obstacle data sits in
//    SGPRs and costs no VGPR, LDS or vector-memory traffic.
//  * The multiplier step needs F^T r, a sum over all time samples of every lane's
//    P-row times its residual.  Each wave reduces its D*NVP partial products with a
//    butterfly reduce-scatter (about one shuffle per value instead of log2(64) per
//    value); waves whose residuals are all zero (the common case near convergence)
//    skip it.
//  * The QP (eq affine_trans) uses the precomputed inverse of the free block of
//    I + rho F^T F in delta form (see trajam_api.cpp): the fixed matrix is applied to
//    the defect, which tends to zero, so reduced precision only perturbs the step.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <algorithm>

#include "am_internal.h"

namespace trajam {
namespace {

__device__ __forceinline__ float rsqrt_t(float x) { return rsqrtf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / sqrt(x); }

// ---- cross-lane exchanges (gfx950) ------------------------------------------
// v_permlane32_swap exchanges the upper 32 lanes of one VGPR with the lower 32 lanes
// of another; v_permlane16_swap does the same for the odd 16-lane rows of one and
// the even rows of the other.  DPP moves data inside 16-lane rows for free as an
// operand modifier of the consuming add.
__device__ __forceinline__ void swap32(float &a, float &b)
{
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap16(float &a, float &b)
{
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap32(double &a, double &b)
{
    const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
    auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
    auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
    b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
__device__ __forceinline__ void swap16(double &a, double &b)
{
    const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
    auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
    auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
    b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}

// DPP controls: rotate a 16-lane row by 8 (= lane ^ 8), mirror each 8-lane half row
// (lane i <-> 7 - i), and the quad permutations lane ^ 2, lane ^ 1.
constexpr int kDppRor8 = 0x128, kDppHalfMirror = 0x141, kDppXor2 = 0x4E, kDppXor1 = 0xB1;

template <int CTRL>
__device__ __forceinline__ float dpp(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double x)
{
    const long long u = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// One halving step inside 16-lane rows: lanes with `up` keep the upper half of the
// n values, their partner (selected by CTRL) keeps the lower half, and each adds
// the half it keeps from its partner.  The empty asm keeps the two candidates as
// register values so the select never becomes a runtime index into the array.
template <typename T, int CTRL>
__device__ __forceinline__ void halve_dpp(T *c, int n, bool up)
{
#pragma unroll
    for (int i = 0; i < n / 2; ++i) {
        T lo = c[i], hi = c[i + n / 2];
        asm volatile("" : "+v"(lo), "+v"(hi));
        const T keep = up ? hi : lo;
        const T send = up ? lo : hi;
        c[i] = keep + dpp<CTRL>(send);
    }
}

// Butterfly reduce-scatter over a wave64: on entry every lane holds V partial
// values c[0..V); on exit the lane returns the sum over all 64 lanes of
// c[lane >> (6 - log2 V)].  Step s halves the live values: the lanes whose lane bit
// (5 - s) is set keep the upper half.  About V exchanges in total instead of
// V log2(64).
template <typename T, int V>
__device__ __forceinline__ T reduce_scatter(T *c, int lane)
{
    static_assert(V >= 16 && V <= 64, "reduce-scatter width");
    int n = V;
#pragma unroll
    for (int i = 0; i < V / 2; ++i) {  // lane bit 5
        swap32(c[i], c[i + V / 2]);
        c[i] = c[i] + c[i + V / 2];
    }
    n = V / 2;
#pragma unroll
    for (int i = 0; i < V / 4; ++i) {  // lane bit 4
        swap16(c[i], c[i + V / 4]);
        c[i] = c[i] + c[i + V / 4];
    }
    n = V / 4;
    halve_dpp<T, kDppRor8>(c, n, (lane & 8) != 0);  // lane bit 3
    n /= 2;
    halve_dpp<T, kDppHalfMirror>(c, n, (lane & 4) != 0);  // lane bit 2
    n /= 2;
    T v;
    if (V == 16) {
        v = c[0];
        v += dpp<kDppXor2>(v);
        v += dpp<kDppXor1>(v);
    } else if (V == 32) {
        halve_dpp<T, kDppXor2>(c, n, (lane & 2) != 0);  // lane bit 1
        v = c[0];
        v += dpp<kDppXor1>(v);
    } else {
        halve_dpp<T, kDppXor2>(c, n, (lane & 2) != 0);
        halve_dpp<T, kDppXor1>(c, n / 2, (lane & 1) != 0);  // lane bit 0
        v = c[0];
    }
    return v;
}

// Sum / max over the 64 lanes of a wave, result in every lane: quad and row steps by
// DPP, then the two permlane swaps combine rows and halves.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    v += dpp<kDppXor1>(v);
    v += dpp<kDppXor2>(v);
    v += dpp<kDppHalfMirror>(v);
    v += dpp<kDppRor8>(v);
    T a = v, b = v;
    swap16(a, b);
    v = a + b;
    a = v;
    b = v;
    swap32(a, b);
    return a + b;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
    v = fmax(v, dpp<kDppXor1>(v));
    v = fmax(v, dpp<kDppXor2>(v));
    v = fmax(v, dpp<kDppHalfMirror>(v));
    v = fmax(v, dpp<kDppRor8>(v));
    T a = v, b = v;
    swap16(a, b);
    v = fmax(a, b);
    a = v;
    b = v;
    swap32(a, b);
    return fmax(a, b);
}

template <typename T>
__device__ __forceinline__ T wave_min(T v)
{
    v = fmin(v, dpp<kDppXor1>(v));
    v = fmin(v, dpp<kDppXor2>(v));
    v = fmin(v, dpp<kDppHalfMirror>(v));
    v = fmin(v, dpp<kDppRor8>(v));
    T a = v, b = v;
    swap16(a, b);
    v = fmin(a, b);
    a = v;
    b = v;
    swap32(a, b);
    return fmin(a, b);
}

// ---- the wave's bounding box in one packed reduction (FP32) --------------------
// Floats enter as order-preserving int32 images (an involution: a < b iff
// ord_i(a) < ord_i(b) for non-NaN values), so every step is an integer minimum,
// which needs no NaN canonicalisation and lets DPP fold into the v_min_i32.
__device__ __forceinline__ int ord_i(float x)
{
    const int b = __float_as_int(x);
    return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float ord_f(int k) { return __int_as_float(k ^ ((k >> 31) & 0x7fffffff)); }

__device__ __forceinline__ void swap32(int &a, int &b)
{
    auto r = __builtin_amdgcn_permlane32_swap((unsigned)a, (unsigned)b, false, false);
    a = (int)r[0];
    b = (int)r[1];
}
__device__ __forceinline__ void swap16(int &a, int &b)
{
    auto r = __builtin_amdgcn_permlane16_swap((unsigned)a, (unsigned)b, false, false);
    a = (int)r[0];
    b = (int)r[1];
}
template <int CTRL>
__device__ __forceinline__ int dpp_min_operand(int x)
{
    return __builtin_amdgcn_update_dpp(0x7fffffff, x, CTRL, 0xF, 0xF, false);
}

// Minimum over the 64 lanes of NV (4 or 8) int values at once: the permlane swaps
// halve the live values (lanes with lane bit 5, then 4, keep the upper half), for
// NV = 8 a DPP row rotation halves once more on lane bit 3, and DPP steps reduce the
// one value left inside its row.  Value j ends in every lane l with
// l / (64 / NV) == j.
template <int NV>
__device__ __forceinline__ int wave_min_multi(int (&c)[NV], int lane)
{
    static_assert(NV == 4 || NV == 8, "packed reduction width");
#pragma unroll
    for (int i = 0; i < NV / 2; ++i) {
        swap32(c[i], c[i + NV / 2]);
        c[i] = min(c[i], c[i + NV / 2]);
    }
#pragma unroll
    for (int i = 0; i < NV / 4; ++i) {
        swap16(c[i], c[i + NV / 4]);
        c[i] = min(c[i], c[i + NV / 4]);
    }
    int v;
    if constexpr (NV == 8) {
        int lo = c[0], hi = c[1];
        asm volatile("" : "+v"(lo), "+v"(hi));
        const bool up = (lane & 8) != 0;
        v = min(up ? hi : lo, dpp_min_operand<kDppRor8>(up ? lo : hi));
    } else {
        v = min(c[0], dpp_min_operand<kDppRor8>(c[0]));
    }
    v = min(v, dpp_min_operand<kDppHalfMirror>(v));
    v = min(v, dpp_min_operand<kDppXor2>(v));
    v = min(v, dpp_min_operand<kDppXor1>(v));
    return v;
}

// Box of the wave's points over lanes/points with ok (and their time range when DYN):
// minima of every coordinate and of the negated coordinates in one reduction.  A lane
// without points contributes +1e30 / -1e30, and NaN coordinates are dropped by the
// per-lane fmin / fmax, so the keys are never NaN.
template <int D, bool DYN, int NPT>
__device__ __forceinline__ void wave_box(const float (&tt)[NPT], const float (&p)[NPT][D], const bool (&ok)[NPT],
                                         float (&lo)[D], float (&hi)[D], float &tlo, float &thi)
{
    constexpr int NQ = D + (DYN ? 1 : 0);
    constexpr int NV = 2 * NQ <= 4 ? 4 : 8;
    const float big = 1e30f;
    int c[NV];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        float mn = big, mx = -big;
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const float x = q < D ? p[i][q < D ? q : 0] : tt[i];
            if (ok[i]) { mn = fminf(mn, x); mx = fmaxf(mx, x); }
        }
        c[q] = ord_i(mn);
        c[NQ + q] = ord_i(-mx);
    }
#pragma unroll
    for (int j = 2 * NQ; j < NV; ++j) c[j] = 0x7fffffff;
    const int v = wave_min_multi<NV>(c, threadIdx.x & 63);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const float mn = ord_f(__builtin_amdgcn_readlane(v, (64 / NV) * q));
        const float mx = -ord_f(__builtin_amdgcn_readlane(v, (64 / NV) * (NQ + q)));
        if (q < D) {
            lo[q < D ? q : 0] = mn;
            hi[q < D ? q : 0] = mx;
        } else {
            tlo = mn;
            thi = mx;
        }
    }
}

// Boxes of the four 16-lane rows of the wave (points with ok, coordinates and times):
// the same integer images reduced by the DPP steps inside a row only.  A row without
// points gets lo > hi.
template <int D, int NPT>
__device__ __forceinline__ void row_boxes(const float (&tt)[NPT], const float (&p)[NPT][D], const bool (&ok)[NPT],
                                          float (&lo)[4][D + 1], float (&hi)[4][D + 1])
{
    constexpr int NQ = D + 1;
    const float big = 1e30f;
    int c[2 * NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        float mn = big, mx = -big;
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const float x = q < D ? p[i][q < D ? q : 0] : tt[i];
            if (ok[i]) { mn = fminf(mn, x); mx = fmaxf(mx, x); }
        }
        c[q] = ord_i(mn);
        c[NQ + q] = ord_i(-mx);
    }
#pragma unroll
    for (int j = 0; j < 2 * NQ; ++j) {
        int v = c[j];
        v = min(v, dpp_min_operand<kDppRor8>(v));
        v = min(v, dpp_min_operand<kDppHalfMirror>(v));
        v = min(v, dpp_min_operand<kDppXor2>(v));
        v = min(v, dpp_min_operand<kDppXor1>(v));
        c[j] = v;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            lo[r][q] = ord_f(__builtin_amdgcn_readlane(c[q], 16 * r));
            hi[r][q] = -ord_f(__builtin_amdgcn_readlane(c[NQ + q], 16 * r));
        }
}

// Orders this wave's LDS writes before its later LDS reads (lanes of one wave
// exchanging data through LDS); no other wave takes part, so no block barrier.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Workgroup barrier that orders LDS only: inside the iteration loops the threads of a
// workgroup exchange data through LDS alone (the residual trace is written, never
// read back), so the barrier need not wait for outstanding global stores.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}


constexpr int pow2ceil(int x) { return x <= 1 ? 1 : 2 * pow2ceil((x + 1) / 2); }

// Obstacle data is read through the constant address space: the address is
// wave-uniform and the kernel never writes it, so the loads become scalar loads into
// SGPRs (no VGPR, LDS or vector-memory cost).
#define TRAJAM_CONST_AS __attribute__((address_space(4)))


// Inside-test data in groups: kGroupStore<T> obstacles per group, field-major, so
// that one scalar load brings one field of a whole (sub)group into SGPRs.  Groups
// are padded with sentinels far away that are never inside.
constexpr int kFCX = 0, kFWX = 3, kFIX = 6, kFNR2 = 9;

template <typename T, int G>
struct Lanes {
    T v[G];
};

// One field of a G-obstacle batch from the constant address space; adjacent
// uniform loads are merged into one wide scalar load.
template <typename T, int G>
__device__ __forceinline__ Lanes<T, G> load_field(const TRAJAM_CONST_AS T *p)
{
    Lanes<T, G> r;
#pragma unroll
    for (int u = 0; u < G; ++u) r.v[u] = p[u];
    return r;
}

// Obstacles tested per scalar-load batch: as many as fit ~48 SGPRs of fields.
template <typename T, int D, bool SPH, bool DYN>
constexpr int test_group()
{
    constexpr int fields = D + (DYN ? D : 0) + (SPH ? 1 : D);
    constexpr int g32 = fields <= 3 ? 16 : (fields <= 6 ? 8 : 4);
    return sizeof(T) == 4 ? g32 : g32 / 2;
}

// Residual of one obstacle for a lane known to be inside (rare path): the point is
// pushed onto the surface along the (scaled) ray from the centre, r = x~ (1 - 1/|u|);
// at the exact centre the angles are atan2(0, 0) = 0, i.e. the push is along +x (2D)
// or +z (3D), and r = -s along that axis.
template <typename T, int D, bool SPH, bool DYN>
__device__ __forceinline__ void obstacle_inside(const TRAJAM_CONST_AS T *o, const T (&p)[D], T tt,
                                                T (&R)[D], T &r2, T &rmax)
{
    T dx[D], nn = T(0);
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        dx[ax] = p[ax] - o[kOC + ax];
        if (DYN) dx[ax] = fma(o[kOW + ax], tt, dx[ax]);
        const T u = SPH ? dx[ax] : dx[ax] * o[kOI + ax];
        nn = fma(u, u, nn);
    }
    T r[D];
    if (nn > T(0)) {
        const T f = SPH ? (T(1) - o[kOR] * rsqrt_t(nn)) : (T(1) - rsqrt_t(nn));
#pragma unroll
        for (int ax = 0; ax < D; ++ax) r[ax] = dx[ax] * f;
    } else {
#pragma unroll
        for (int ax = 0; ax < D; ++ax) r[ax] = T(0);
        constexpr int push = (D == 2) ? 0 : 2;
        r[push] = SPH ? -o[kOR] : -o[kOS + push];
    }
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        R[ax] += r[ax];
        r2 = fma(r[ax], r[ax], r2);
        rmax = fmax(rmax, fabs(r[ax]));
    }
}

// The same residual as obstacle_inside from the offset dx = p - c(t) the inside test
// already formed (identical operations), with the obstacle's fields passed as
// wave-uniform values: rad the radius (spheres), iu the inverse semi-axes and s_push
// the semi-axis along the push direction (ellipsoids).
template <typename T, int D, bool SPH>
__device__ __forceinline__ void obstacle_residual_at(const T (&dx)[D], T rad, const T (&iu)[D], T s_push,
                                                     T (&R)[D], T &r2, T &rmax)
{
    T nn = T(0);
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        const T u = SPH ? dx[ax] : dx[ax] * iu[ax];
        nn = fma(u, u, nn);
    }
    T r[D];
    if (nn > T(0)) {
        const T f = SPH ? (T(1) - rad * rsqrt_t(nn)) : (T(1) - rsqrt_t(nn));
#pragma unroll
        for (int ax = 0; ax < D; ++ax) r[ax] = dx[ax] * f;
    } else {
#pragma unroll
        for (int ax = 0; ax < D; ++ax) r[ax] = T(0);
        constexpr int push = (D == 2) ? 0 : 2;
        r[push] = SPH ? -rad : -s_push;
    }
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        R[ax] += r[ax];
        r2 = fma(r[ax], r[ax], r2);
        rmax = fmax(rmax, fabs(r[ax]));
    }
}

// Obstacle polar step summed over all obstacles for NPT (sample, time) points of one
// lane (eqs collision_priest, zeta_2, compute_d_mij, d_max).  The residual
// r_j = p - e_j is zero outside obstacle j (d = |u| >= 1), so the loop evaluates the
// signed inside test q = |x~|^2 - r^2 (spheres) or |x~ ./ s|^2 - 1 (ellipsoids) for a
// batch of G obstacles whose fields sit in SGPRs, and enters the residual path only
// if a lane's point is inside one of them.  Points that must not contribute are
// placed far away (-1e30) by the caller and are never inside; the padding
// obstacles sit at +1e30.
template <typename T, int D, bool SPH, bool DYN, int NPT>
__device__ __forceinline__ void obstacle_loop(const TRAJAM_CONST_AS T *soa,
                                              const TRAJAM_CONST_AS T *aos, int n_o,
                                              const T (&tt)[NPT], const T (&p)[NPT][D],
                                              T (&R)[NPT][D], T &r2, T &rmax)
{
    constexpr int GS = kGroupStore<T>;
    constexpr int G0 = test_group<T, D, SPH, DYN>();
    constexpr int G = NPT > 2 ? (G0 >= 8 ? G0 / 2 : G0) : G0;
    using V = Lanes<T, G>;
    const int n_sub = ((n_o + GS - 1) / GS) * (GS / G);
    for (int sg = 0; sg < n_sub; ++sg) {
        const int g = sg / (GS / G), h = sg - g * (GS / G);
        const TRAJAM_CONST_AS T *base = soa + (size_t)g * kObstacleFields * GS + h * G;
        V c[D], w[D], is[D], nr2;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            c[ax] = load_field<T, G>(base + (kFCX + ax) * GS);
            if (DYN) w[ax] = load_field<T, G>(base + (kFWX + ax) * GS);
            if (!SPH) is[ax] = load_field<T, G>(base + (kFIX + ax) * GS);
        }
        if (SPH) nr2 = load_field<T, G>(base + kFNR2 * GS);
        T q[NPT][G];
        T qmin = T(1);
#pragma unroll
        for (int u = 0; u < G; ++u) {
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
                T dx[D];
#pragma unroll
                for (int ax = 0; ax < D; ++ax) {
                    dx[ax] = p[i][ax] - c[ax].v[u];
                    if (DYN) dx[ax] = fma(w[ax].v[u], tt[i], dx[ax]);
                }
                T acc;
                if (SPH) {
                    acc = fma(dx[D - 1], dx[D - 1], nr2.v[u]);
#pragma unroll
                    for (int ax = D - 2; ax >= 0; --ax) acc = fma(dx[ax], dx[ax], acc);
                } else {
                    acc = T(-1);
#pragma unroll
                    for (int ax = D - 1; ax >= 0; --ax) {
                        const T uu = dx[ax] * is[ax].v[u];
                        acc = fma(uu, uu, acc);
                    }
                }
                q[i][u] = acc;
                qmin = fmin(qmin, acc);
            }
        }
        if (qmin < T(0)) {
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int j = g * GS + h * G + u;  // padding sentinels are never inside;
                if (j >= n_o) break;               // the record array ends at n_o
                const TRAJAM_CONST_AS T *o = aos + (size_t)j * kObstacleRecord;
#pragma unroll
                for (int i = 0; i < NPT; ++i)
                    if (q[i][u] < T(0)) obstacle_inside<T, D, SPH, DYN>(o, p[i], tt[i], R[i], r2, rmax);
            }
        }
    }
}

template <typename T, int D, int NPT>
__device__ __forceinline__ void obstacle_residuals(const T *soa_g, const T *aos_g, int n_o,
                                                   int sphere, int dynamic, const T (&tt)[NPT],
                                                   const T (&p)[NPT][D], T (&R)[NPT][D], T &r2,
                                                   T &rmax)
{
    const TRAJAM_CONST_AS T *soa = (const TRAJAM_CONST_AS T *)soa_g;
    const TRAJAM_CONST_AS T *aos = (const TRAJAM_CONST_AS T *)aos_g;
    if (sphere) {
        if (dynamic) obstacle_loop<T, D, true, true, NPT>(soa, aos, n_o, tt, p, R, r2, rmax);
        else obstacle_loop<T, D, true, false, NPT>(soa, aos, n_o, tt, p, R, r2, rmax);
    } else {
        if (dynamic) obstacle_loop<T, D, false, true, NPT>(soa, aos, n_o, tt, p, R, r2, rmax);
        else obstacle_loop<T, D, false, false, NPT>(soa, aos, n_o, tt, p, R, r2, rmax);
    }
}

// Single-point form used by the multi-wave and residual kernels.
template <typename T, int D>
__device__ __forceinline__ void obstacle_residuals1(const T *soa_g, const T *aos_g, int n_o,
                                                    int sphere, int dynamic, T tt, const T (&p)[D],
                                                    T (&R)[D], T &r2, T &rmax)
{
    T tt1[1] = {tt};
    T p1[1][D], R1[1][D];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) { p1[0][ax] = p[ax]; R1[0][ax] = R[ax]; }
    obstacle_residuals<T, D, 1>(soa_g, aos_g, n_o, sphere, dynamic, tt1, p1, R1, r2, rmax);
#pragma unroll
    for (int ax = 0; ax < D; ++ax) R[ax] = R1[0][ax];
}

template <typename T>
__device__ __forceinline__ T readlane_t(T v, int l);
template <>
__device__ __forceinline__ float readlane_t<float>(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <>
__device__ __forceinline__ double readlane_t<double>(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename T>
__device__ __forceinline__ T shfl_t(T v, int src);
template <>
__device__ __forceinline__ float shfl_t<float>(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
template <>
__device__ __forceinline__ double shfl_t<double>(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The same obstacle polar step for the points of one wave, with exact culling: the
// wave's points span a small box (a stretch of one trajectory), and an obstacle
// whose bounding box -- swept over the wave's time range for moving obstacles, and
// widened by a margin far above the rounding of the inside test -- misses that box
// cannot contain any of the points, so its residual is zero.  Lane j of a chunk
// tests obstacle j against the box (one vector compare for 64 obstacles); the
// candidates' fields then come from v_readlane and get exactly the inside test of
// obstacle_loop, in obstacle order, so the result is bit-identical to testing every
// obstacle.  Every row stays in F and in H; only provably zero terms are skipped.
// Must be called by the whole wave (uniform control flow); points that must not
// contribute sit at -1e30 and are flagged false in `ok`.
// One 64-obstacle chunk of packed records, lane j holding obstacle base + j (zeros past
// n_o).  The first chunk is loaded once per launch, before the iteration loop.
template <typename T, int D>
struct ObsChunk {
    T c[D], w[D], is[D], s[D], nr2, r;
};

template <typename T, int D>
__device__ __forceinline__ ObsChunk<T, D> load_obs_chunk(const T *aos_g, int n_o, int base, int lane)
{
    ObsChunk<T, D> k;
    const int j = base + lane;
    const bool has = j < n_o;
    const T *o = aos_g + (size_t)(has ? j : 0) * kObstacleRecord;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        k.c[ax] = has ? o[kOC + ax] : T(0);
        k.w[ax] = has ? o[kOW + ax] : T(0);
        k.is[ax] = has ? o[kOI + ax] : T(0);
        k.s[ax] = has ? o[kOS + ax] : T(0);
    }
    k.nr2 = has ? o[kONR2] : T(0);
    k.r = has ? o[kOR] : T(0);
    return k;
}

// Obstacle fields staged in a wave's LDS (multi-agent kernels): per obstacle
// centre[D], -velocity[D], then -r^2 and r (spheres) or semi-axes[D] and their
// inverses[D] (ellipsoids), each field an array over the obstacles
// (stage_fields(D, sphere) arrays).

template <typename T, int D>
__device__ __forceinline__ void stage_obstacles(T *ol, const T *aos_g, int n_o, int sphere, int lane)
{
    for (int j = lane; j < n_o; j += 64) {
        const T *o = aos_g + (size_t)j * kObstacleRecord;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            ol[ax * n_o + j] = o[kOC + ax];
            ol[(D + ax) * n_o + j] = o[kOW + ax];
            if (!sphere) {
                ol[(2 * D + ax) * n_o + j] = o[kOS + ax];
                ol[(3 * D + ax) * n_o + j] = o[kOI + ax];
            }
        }
        if (sphere) {
            ol[2 * D * n_o + j] = o[kONR2];
            ol[(2 * D + 1) * n_o + j] = o[kOR];
        }
    }
    wave_lds_sync();
}

template <typename T, int D, bool SPH>
__device__ __forceinline__ ObsChunk<T, D> lds_obs_chunk(const T *ol, int n_o, int base, int lane)
{
    ObsChunk<T, D> k;
    const int j = base + lane;
    const int jj = j < n_o ? j : 0;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        k.c[ax] = ol[ax * n_o + jj];
        k.w[ax] = ol[(D + ax) * n_o + jj];
        k.s[ax] = SPH ? T(0) : ol[(2 * D + ax) * n_o + jj];
        k.is[ax] = SPH ? T(0) : ol[(3 * D + ax) * n_o + jj];
    }
    k.nr2 = SPH ? ol[2 * D * n_o + jj] : T(0);
    k.r = SPH ? ol[(2 * D + 1) * n_o + jj] : T(0);
    return k;
}

// Candidate masks of up to kCullCacheChunks obstacle chunks, kept across iterations.
// They were built against the wave's box grown by delta when every point of the wave
// was at pref; while no point has moved more than delta from there (max norm) each
// point still lies in that grown box, so the masks still hold every obstacle that can
// contain one of the wave's points, and the box reduction and chunk tests are skipped.
constexpr int kCullCacheChunks = 4;
// delta = kCullGrowFrac * (largest extent of the wave's box) + kCullGrowAbs: larger
// margins keep masks longer but admit more candidates (at config 2, 5 % of the extent
// grew the candidates from 2.0 to 3.4 per wave; 0.5 % rebuilt too often)
constexpr float kCullGrowFrac = 0.015f, kCullGrowAbs = 1e-3f;

template <typename T, int D, int NPT>
struct CullCache {
    bool valid = false;
    T delta = T(0);
    unsigned long long m0 = 0, m1 = 0, m2 = 0, m3 = 0;
    T pref[NPT][D] = {};
};

// Chunks of 64 obstacles (lane j: obstacle base + j) come from the LDS stage `ol`
// (STAGED) or from the packed records, the first one from `first`, loaded once per
// launch by the caller.
template <typename T, int D, bool SPH, bool DYN, int NPT, bool STAGED, bool CACHE, bool ROWSOK = false>
__device__ __forceinline__ void obstacle_cull_loop(const T *aos_g, const T *ol, int n_o, const ObsChunk<T, D> first,
                                                   const T (&tt)[NPT], const T (&p)[NPT][D], const bool (&ok)[NPT],
                                                   T (&R)[NPT][D], T &r2, T &rmax, CullCache<T, D, NPT> &cc)
{
    const T big = T(1e30);
    const bool cached = CACHE && n_o <= 64 * kCullCacheChunks;
    bool rebuild = true;
    if (cached && cc.valid) {
        bool moved = false;
#pragma unroll
        for (int i = 0; i < NPT; ++i)
#pragma unroll
            for (int ax = 0; ax < D; ++ax)
                moved = moved || (ok[i] && !(fabs(p[i][ax] - cc.pref[i][ax]) <= cc.delta));
        rebuild = __any(moved);
    }
    // moving obstacles are swept over a time range: against the four 16-lane rows'
    // boxes, each with its own shorter range, instead of the whole wave's
    constexpr bool ROWS = ROWSOK && DYN && !STAGED && sizeof(T) == sizeof(float);
    T lo[D], hi[D], tlo = T(0), thi = T(0);
    T rlo[4][D + 1], rhi[4][D + 1];
    if (!rebuild) {
        // masks from the cache below
    } else if constexpr (ROWS) {
        row_boxes<D, NPT>(tt, p, ok, rlo, rhi);
        // the wave's box is the union of the rows'
#pragma unroll
        for (int q = 0; q <= D; ++q) {
            T mn = rlo[0][q], mx = rhi[0][q];
#pragma unroll
            for (int r = 1; r < 4; ++r) {
                mn = fmin(mn, rlo[r][q]);
                mx = fmax(mx, rhi[r][q]);
            }
            if (q < D) {
                lo[q < D ? q : 0] = mn;
                hi[q < D ? q : 0] = mx;
            } else {
                tlo = mn;
                thi = mx;
            }
        }
    } else if constexpr (sizeof(T) == sizeof(float)) {
        wave_box<D, DYN, NPT>(tt, p, ok, lo, hi, tlo, thi);
    } else {
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            T mn = big, mx = -big;
#pragma unroll
            for (int i = 0; i < NPT; ++i)
                if (ok[i]) { mn = fmin(mn, p[i][ax]); mx = fmax(mx, p[i][ax]); }
            lo[ax] = wave_min(mn);
            hi[ax] = wave_max(mx);
        }
        if (DYN) {
            T mn = big, mx = -big;
#pragma unroll
            for (int i = 0; i < NPT; ++i)
                if (ok[i]) { mn = fmin(mn, tt[i]); mx = fmax(mx, tt[i]); }
            tlo = wave_min(mn);
            thi = wave_max(mx);
        }
    }
    if (rebuild) {
        if (!(lo[0] <= hi[0])) {  // no point of this wave takes part
            if (cached) cc.valid = false;
            return;
        }
        if (cached) {
            T ext = T(0);
#pragma unroll
            for (int ax = 0; ax < D; ++ax) ext = fmax(ext, hi[ax] - lo[ax]);
            const T dl = T(kCullGrowFrac) * ext + T(kCullGrowAbs);
            const T grow = fma(dl, T(1.0001), T(1e-5));  // also covers the rounding of p - pref
#pragma unroll
            for (int ax = 0; ax < D; ++ax) {
                lo[ax] -= grow;
                hi[ax] += grow;
            }
            if constexpr (ROWS) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int ax = 0; ax < D; ++ax) {
                        rlo[r][ax] -= grow;
                        rhi[r][ax] += grow;
                    }
            }
            cc.delta = dl;
#pragma unroll
            for (int i = 0; i < NPT; ++i)
#pragma unroll
                for (int ax = 0; ax < D; ++ax) cc.pref[i][ax] = p[i][ax];
            cc.valid = true;
        }
    }
    const int lane = threadIdx.x & 63;
    const T tabs = fmax(fabs(tlo), fabs(thi));
    for (int base = 0, ci = 0; base < n_o; base += 64, ++ci) {
        const ObsChunk<T, D> k = STAGED ? lds_obs_chunk<T, D, SPH>(ol, n_o, base, lane)
                                        : (base == 0 ? first : load_obs_chunk<T, D>(aos_g, n_o, base, lane));
        unsigned long long mask;
        if (rebuild) {
            bool cand = base + lane < n_o;
            if constexpr (ROWS) {
                // candidate if its box swept over some row's time range meets that row's box
                bool any = false;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (!(rlo[r][D] <= rhi[r][D])) continue;   // a row without points
                    const T ta = rlo[r][D], tb = rhi[r][D], tab = fmax(fabs(ta), fabs(tb));
                    bool cr = true;
#pragma unroll
                    for (int ax = 0; ax < D; ++ax) {
                        const T e = SPH ? k.r : k.s[ax];
                        const T c1 = fma(-k.w[ax], ta, k.c[ax]), c2 = fma(-k.w[ax], tb, k.c[ax]);
                        const T cmin = fmin(c1, c2), cmax = fmax(c1, c2);
                        const T m = fma(e, T(1.0001), T(1e-4)) + T(1e-5) * fabs(k.c[ax]) +
                                    T(1e-5) * (fabs(k.w[ax]) * tab + fabs(cmin) + fabs(cmax));
                        cr = cr && (cmin - m <= rhi[r][ax]) && (cmax + m >= rlo[r][ax]);
                    }
                    any = any || cr;
                }
                cand = cand && any;
            } else {
#pragma unroll
                for (int ax = 0; ax < D; ++ax) {
                    const T e = SPH ? k.r : k.s[ax];
                    T cmin = k.c[ax], cmax = k.c[ax], m = fma(e, T(1.0001), T(1e-4)) + T(1e-5) * fabs(k.c[ax]);
                    if (DYN) {
                        const T c1 = fma(-k.w[ax], tlo, k.c[ax]), c2 = fma(-k.w[ax], thi, k.c[ax]);
                        cmin = fmin(c1, c2);
                        cmax = fmax(c1, c2);
                        m += T(1e-5) * (fabs(k.w[ax]) * tabs + fabs(cmin) + fabs(cmax));
                    }
                    cand = cand && (cmin - m <= hi[ax]) && (cmax + m >= lo[ax]);
                }
            }
            mask = __ballot(cand);
            if (cached) {
                if (ci == 0) cc.m0 = mask;
                else if (ci == 1) cc.m1 = mask;
                else if (ci == 2) cc.m2 = mask;
                else cc.m3 = mask;
            }
        } else {
            mask = ci == 0 ? cc.m0 : ci == 1 ? cc.m1 : ci == 2 ? cc.m2 : cc.m3;
        }
        while (mask) {
            const int u = __builtin_ctzll(mask);
            mask &= mask - 1;
            T cu[D], wu[D], iu[D];
#pragma unroll
            for (int ax = 0; ax < D; ++ax) {
                cu[ax] = readlane_t<T>(k.c[ax], u);
                wu[ax] = DYN ? readlane_t<T>(k.w[ax], u) : T(0);
                iu[ax] = SPH ? T(0) : readlane_t<T>(k.is[ax], u);
            }
            const T nu = SPH ? readlane_t<T>(k.nr2, u) : T(0);
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
                T dx[D];
#pragma unroll
                for (int ax = 0; ax < D; ++ax) {
                    dx[ax] = p[i][ax] - cu[ax];
                    if (DYN) dx[ax] = fma(wu[ax], tt[i], dx[ax]);
                }
                T acc;
                if (SPH) {
                    acc = fma(dx[D - 1], dx[D - 1], nu);
#pragma unroll
                    for (int ax = D - 2; ax >= 0; --ax) acc = fma(dx[ax], dx[ax], acc);
                } else {
                    acc = T(-1);
#pragma unroll
                    for (int ax = D - 1; ax >= 0; --ax) {
                        const T uu = dx[ax] * iu[ax];
                        acc = fma(uu, uu, acc);
                    }
                }
                if (acc < T(0)) {
                    // inside: the residual from the chunk's registers (no record reload)
                    const T rad = SPH ? readlane_t<T>(k.r, u) : T(0);
                    const T sp = SPH ? T(0) : readlane_t<T>(k.s[D == 2 ? 0 : 2], u);
                    obstacle_residual_at<T, D, SPH>(dx, rad, iu, sp, R[i], r2, rmax);
                }
            }
        }
    }
}

// Obstacle motion of a kernel instance: static obstacles only, moving ones only, or
// either, chosen at run time (the ragged kernels, whose problems differ).
constexpr int kObsStatic = 0, kObsMoving = 1, kObsEither = 2;

template <typename T, int D, int NPT, int OM = kObsEither>
__device__ __forceinline__ void obstacle_residuals_culled(const T *aos_g, int n_o, int sphere, int dynamic,
                                                          const ObsChunk<T, D> first, const T (&tt)[NPT],
                                                          const T (&p)[NPT][D], const bool (&ok)[NPT],
                                                          T (&R)[NPT][D], T &r2, T &rmax, CullCache<T, D, NPT> &cc)
{
    // the cache's reference positions cost NPT * D registers a lane: FP64 launches with
    // more than two time samples a lane rebuild the masks every iteration instead
    constexpr bool C = sizeof(T) == sizeof(float) || NPT <= 2;
    const bool mov = OM == kObsMoving || (OM == kObsEither && dynamic);
    // row boxes only in the moving-obstacle instances: the either-motion (ragged)
    // kernels keep the smaller whole-wave test, their registers being at the limit
    constexpr bool RW = OM == kObsMoving;
    if (sphere) {
        if (OM != kObsStatic && mov) obstacle_cull_loop<T, D, true, true, NPT, false, C, RW>(aos_g, nullptr, n_o, first, tt, p, ok, R, r2, rmax, cc);
        else if (OM != kObsMoving) obstacle_cull_loop<T, D, true, false, NPT, false, C>(aos_g, nullptr, n_o, first, tt, p, ok, R, r2, rmax, cc);
    } else {
        if (OM != kObsStatic && mov) obstacle_cull_loop<T, D, false, true, NPT, false, C, RW>(aos_g, nullptr, n_o, first, tt, p, ok, R, r2, rmax, cc);
        else if (OM != kObsMoving) obstacle_cull_loop<T, D, false, false, NPT, false, C>(aos_g, nullptr, n_o, first, tt, p, ok, R, r2, rmax, cc);
    }
}

// The culled loop on obstacles staged in this wave's LDS (`ol`).
template <typename T, int D, int NPT>
__device__ __forceinline__ void obstacle_residuals_staged(const T *ol, const T *aos_g, int n_o, int sphere,
                                                          int dynamic, const T (&tt)[NPT], const T (&p)[NPT][D],
                                                          const bool (&ok)[NPT], T (&R)[NPT][D], T &r2, T &rmax)
{
    const ObsChunk<T, D> none{};
    CullCache<T, D, NPT> nc;  // unused: the staged loop rebuilds its masks every call
    if (sphere) {
        if (dynamic) obstacle_cull_loop<T, D, true, true, NPT, true, false>(aos_g, ol, n_o, none, tt, p, ok, R, r2, rmax, nc);
        else obstacle_cull_loop<T, D, true, false, NPT, true, false>(aos_g, ol, n_o, none, tt, p, ok, R, r2, rmax, nc);
    } else {
        if (dynamic) obstacle_cull_loop<T, D, false, true, NPT, true, false>(aos_g, ol, n_o, none, tt, p, ok, R, r2, rmax, nc);
        else obstacle_cull_loop<T, D, false, false, NPT, true, false>(aos_g, ol, n_o, none, tt, p, ok, R, r2, rmax, nc);
    }
}

// Velocity / acceleration polar step (eqs fv_priest, alpha_v, compute_dv): the
// residual is v (1 - bound / |v|) outside the ball of radius `bound`, else 0.
template <typename T, int D>
__device__ __forceinline__ void bound_residual(const T (&v)[D], T bound, T (&r)[D], T &r2,
                                               T &rmax)
{
    T vv = T(0);
#pragma unroll
    for (int ax = 0; ax < D; ++ax) vv = fma(v[ax], v[ax], vv);
    if (vv > bound * bound) {
        const T f = T(1) - bound * rsqrt_t(vv);
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            r[ax] = v[ax] * f;
            r2 = fma(r[ax], r[ax], r2);
            rmax = fmax(rmax, fabs(r[ax]));
        }
    } else {
#pragma unroll
        for (int ax = 0; ax < D; ++ax) r[ax] = T(0);
    }
}

// Workspace rows G = [-P; P] (Paper III, eq bound_con, and the slack step of its AM
// list): with the slack s = max(0, -G xb + tau) the residual of the row p <= hi is
// max(0, p - hi) and that of -p <= -lo is max(0, lo - p); G^T r adds their difference,
// p - clamp(p, lo, hi), to the position rows R, and their squares to r2.
// (BND: the bound arrays of the launch arguments, in whichever address space they sit)
template <typename T, int D, typename BND>
__device__ __forceinline__ void workspace_residual(const T (&p)[D], const BND &lo, const BND &hi, T (&R)[D], T &r2,
                                                   T &rmax)
{
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        const T r = p[ax] - fmin(fmax(p[ax], (T)lo[ax]), (T)hi[ax]);
        R[ax] += r;
        r2 = fma(r, r, r2);
        rmax = fmax(rmax, fabs(r));
    }
}

// ---- bf16 matrix-core QP step (TRAJAM_BF16_REFINE) ----------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_rn(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (short)(u >> 16);
}
__device__ __forceinline__ float bf16_f(short h) { return __uint_as_float(((unsigned)(unsigned short)h) << 16); }

// delta = W_ff v for one 16 x 16 tile on the matrix cores with both operands split
// into bf16 hi + lo parts: W v ~ Whi vhi + Whi vlo + Wlo vhi (the dropped Wlo vlo term
// is 2^-16 relative), accumulated in fp32.  Operand layout of
// v_mfma_f32_16x16x16_bf16: lane l holds A[l % 16][4 (l / 16) + i], B[4 (l / 16) + i][l % 16]
// and returns D[4 (l / 16) + i][l % 16], i = 0..3.
__device__ __forceinline__ f32x4 qp_mfma(bf16x4 ahi, bf16x4 alo, const float (&v)[4])
{
    bf16x4 bhi, blo;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const short h = bf16_rn(v[i]);
        bhi[i] = h;
        blo[i] = bf16_rn(v[i] - bf16_f(h));
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bhi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, blo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi, acc, 0, 0, 0);
    return acc;
}

// LDS of the matrix-core QP step (floats): y and delta tiles [16 columns][16 rows],
// H_ff [16][16] and H_fb [16][4] (boundary coefficients 0, 1, 2, n).
constexpr int kMqFloats = 256 + 256 + 256 + 64;

// Shared-memory carve-up of one AM workgroup (units of T).
template <int D, int NVP>
struct Lds {
    static constexpr int S = D * NVP;           // coefficients of one sample
    static constexpr int V = pow2ceil(D * NVP); // reduce-scatter width
    __host__ __device__ static int xbuf(int) { return 0; }
    __host__ __device__ static int gbuf(int tb) { return 2 * tb * S; }
    __host__ __device__ static int part(int tb) { return 3 * tb * S; }
    __host__ __device__ static int r2p(int tb, int wpt) { return part(tb) + tb * wpt * V; }
    __host__ __device__ static int wmat(int tb, int wpt) { return r2p(tb, wpt) + tb * wpt; }
    __host__ __device__ static int total(int tb, int wpt) { return wmat(tb, wpt) + NVP * NVP; }
};

// ----------------------------------------------------------------------------
// The fused AM kernel: `a.iters` iterations for `a.tb` samples per workgroup.
template <typename T, int D, int NVP, bool MQP, int OM>
__global__ __launch_bounds__(kMaxThreads) void am_project_kernel(AmArgs<T> a)
{
    using L = Lds<D, NVP>;
    constexpr int S = L::S;
    constexpr int V = L::V;
    constexpr int LOGV = (V >= 64) ? 6 : (V >= 32) ? 5 : (V >= 16) ? 4 : 3;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *smem = reinterpret_cast<T *>(smem_raw);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wpt = a.tpad >> 6;               // waves per sample
    const int ls = tid / a.tpad;               // local sample
    const int lt = tid - ls * a.tpad;          // lane within the sample (output index)
    const int wave_in_s = lt >> 6;
    const int sample = blockIdx.x * a.tb + ls;
    const bool live = sample < a.batch;
    // the time samples are split evenly over the sample's waves (equal boxes and
    // obstacle candidates per wave): wave w holds samples w * per_w + lane
    const int per_w = (a.n_p + wpt - 1) / wpt;
    const int ti = wave_in_s * per_w + lane;   // time sample of this lane
    const bool valid = live && lane < per_w && ti < a.n_p;
    const int nf = a.nv - 4;

    T *xbuf = smem + L::xbuf(a.tb);
    T *gbuf = smem + L::gbuf(a.tb);
    T *part = smem + L::part(a.tb);
    T *r2p = smem + L::r2p(a.tb, wpt);
    T *wmat = smem + L::wmat(a.tb, wpt);

    // Fixed QP operator into LDS (rows of free coefficients; zero padded).
    for (int i = tid; i < NVP * NVP; i += blockDim.x) {
        const int f = i / NVP, m = i - f * NVP;
        wmat[i] = (f < nf) ? a.W[f * NVP + m] : T(0);
    }
    // Matrix-core QP: W_ff hi/lo A operands in registers, H_ff and H_fb in LDS.
    float *mq = reinterpret_cast<float *>(smem + L::total(a.tb, wpt));
    bf16x4 ahi = {0, 0, 0, 0}, alo = {0, 0, 0, 0};
    if constexpr (MQP) {
        const int m = lane & 15, k0 = 4 * (lane >> 4);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ahi[i] = (short)a.Whi[m * 16 + k0 + i];
            alo[i] = (short)a.Wlo[m * 16 + k0 + i];
        }
        for (int i = tid; i < 256 + 64; i += blockDim.x) mq[512 + i] = a.Hmq[i];
    }
    // Basis rows of this lane's time sample stay in registers.
    T phi0[NVP], phi1[NVP], phi2[NVP];
#pragma unroll
    for (int m = 0; m < NVP; ++m) {
        phi0[m] = valid ? a.phi[(0 * a.n_p + ti) * NVP + m] : T(0);
        phi1[m] = valid ? a.phi[(1 * a.n_p + ti) * NVP + m] : T(0);
        phi2[m] = valid ? a.phi[(2 * a.n_p + ti) * NVP + m] : T(0);
    }
    const T tt = T(ti) * a.dt;

    // Output lanes: lane lt < S owns coefficient (axis, m) of its sample.
    const bool owner = live && lt < S;
    const int o_ax = lt / NVP, o_m = lt - (lt / NVP) * NVP;
    const bool o_real = owner && o_m < a.nv;
    const bool o_free = o_real && o_m >= 3 && o_m < a.nv - 1;
    const size_t gidx = (size_t)sample * D * a.nv + (size_t)o_ax * a.nv + o_m;
    T xi_o = T(0), lam_o = T(0), xb_o = T(0);
    if (o_real) {
        xi_o = a.xi[gidx];
        lam_o = a.lam[gidx];
        xb_o = a.xb[gidx];
    }
    T bnd_o = T(0);
    if (o_real && !o_free) {
        const int bi = (o_m == a.nv - 1) ? 3 : o_m;
        bnd_o = a.xiB[o_ax][bi];
    }
    if (lt < S && ls < a.tb) xbuf[ls * S + lt] = xb_o;  // buffer 0; padding entries are 0
    __syncthreads();

    const ObsChunk<T, D> oc0 = load_obs_chunk<T, D>(a.obs, a.n_o, 0, threadIdx.x & 63);
    CullCache<T, D, 1> ccache;     // obstacle candidates kept across iterations
    T res_first = T(0), res_last = T(0);
    bool nonfinite = false;
    const bool res_lane = live && lt == (wpt - 1) * 64;   // lane 0 of the sample's last wave
    int cur = 0;
    for (int k = 0; k < a.iters; ++k) {
        const T *xs = xbuf + (cur * a.tb + ls) * S;
        // ---- step (a): waypoints and polar steps (eqs parameter, comp_alpha..comp_d)
        T p[D], v[D], acc[D];
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
            for (int m = 0; m < NVP; ++m) {
                const T c = xs[ax * NVP + m];
                s0 = fma(phi0[m], c, s0);
                s1 = fma(phi1[m], c, s1);
                s2 = fma(phi2[m], c, s2);
            }
            p[ax] = s0; v[ax] = s1; acc[ax] = s2;
        }
        T R[D], rv[D], ra[D], r2 = T(0), rmax = T(0);
#pragma unroll
        for (int ax = 0; ax < D; ++ax) { R[ax] = T(0); rv[ax] = T(0); ra[ax] = T(0); }
        {
            const T tt1[1] = {tt};
            const bool ok1[1] = {valid};
            T p1[1][D], R1[1][D];
#pragma unroll
            for (int ax = 0; ax < D; ++ax) {
                p1[0][ax] = valid ? p[ax] : T(-1e30);
                R1[0][ax] = T(0);
            }
            obstacle_residuals_culled<T, D, 1, OM>(a.obs, a.n_o, a.sphere, a.dynamic, oc0, tt1, p1, ok1, R1, r2,
                                                   rmax, ccache);
#pragma unroll
            for (int ax = 0; ax < D; ++ax) R[ax] = R1[0][ax];
        }
        if (valid) {
            if (a.use_v) bound_residual<T, D>(v, a.vmax, rv, r2, rmax);
            if (a.use_a) bound_residual<T, D>(acc, a.amax, ra, r2, rmax);
            if (a.use_ws) workspace_residual(p, a.ws_lo, a.ws_hi, R, r2, rmax);
        }
        // ---- F^T r: each lane's rows times its residuals, reduced over the wave
        // each residual group (obstacle, velocity, acceleration) enters only when some
        // lane of the wave has it non-zero; a skipped group adds exact zeros
        bool nR = false, nV = false, nA = false;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            nR = nR || R[ax] != T(0);
            nV = nV || rv[ax] != T(0);
            nA = nA || ra[ax] != T(0);
        }
        const bool aR = __any(nR), aV = __any(nV), aA = __any(nA);
        T *mypart = part + (ls * wpt + wave_in_s) * V;
        if (aR || aV || aA) {
            T c[V];
#pragma unroll
            for (int i = 0; i < V; ++i) c[i] = T(0);
            if (aA)
#pragma unroll
                for (int ax = 0; ax < D; ++ax)
#pragma unroll
                    for (int m = 0; m < NVP; ++m) c[ax * NVP + m] = phi2[m] * ra[ax];
            if (aV)
#pragma unroll
                for (int ax = 0; ax < D; ++ax)
#pragma unroll
                    for (int m = 0; m < NVP; ++m) c[ax * NVP + m] = fma(phi1[m], rv[ax], c[ax * NVP + m]);
            if (aR)
#pragma unroll
                for (int ax = 0; ax < D; ++ax)
#pragma unroll
                    for (int m = 0; m < NVP; ++m) c[ax * NVP + m] = fma(phi0[m], R[ax], c[ax * NVP + m]);
            const T s = reduce_scatter<T, V>(c, lane);
            if ((lane & ((64 >> LOGV) - 1)) == 0) mypart[lane >> (6 - LOGV)] = s;
        } else if (lane < V) {
            mypart[lane] = T(0);
        }
        const T r2w = wave_sum(r2);
        if (lane == 0) r2p[ls * wpt + wave_in_s] = r2w;
        lds_barrier();

        // ---- step (c): multiplier (eq lag) and the QP right-hand side defect
        if (owner) {
            // the partials of the sample's waves (at most 4) are read together
            T pw[4];
#pragma unroll
            for (int w = 0; w < 4; ++w) pw[w] = w < wpt ? part[(ls * wpt + w) * V + lt] : T(0);
            T ftr = T(0);
#pragma unroll
            for (int w = 0; w < 4; ++w) ftr += pw[w];
            T gv = T(0);
            if (o_real) {
                lam_o = fma(-a.rho, ftr, lam_o);
                gv = o_free ? (xi_o - xb_o + lam_o - a.rho * ftr) : (bnd_o - xb_o);
            }
            gbuf[ls * S + lt] = gv;
        }
        // the residual norm is the last wave's: off the owners' path to the QP
        if (res_lane) {
            T rw[4];
#pragma unroll
            for (int w = 0; w < 4; ++w) rw[w] = w < wpt ? r2p[ls * wpt + w] : T(0);
            T rs = T(0);
#pragma unroll
            for (int w = 0; w < 4; ++w) rs += rw[w];
            rs = sqrt(rs);
            if (a.res) a.res[(size_t)k * a.batch + sample] = rs;
            if (k == 0) res_first = rs;
            res_last = rs;
            nonfinite = nonfinite || !isfinite(rs);
        }
        // ---- step (b): xb_free += W [g_free ; boundary defect]  (eq affine_trans)
        const int nxt = cur ^ 1;
        if constexpr (MQP) {
            lds_barrier();
            // y = g_f - H_fb Delta_b per (sample, axis) column; delta = W_ff y on the
            // matrix cores, then one refinement pass delta += W_ff (y - H_ff delta).
            float *yb = mq, *db = mq + 256;
            const float *hff = mq + 512, *hfb = mq + 768;
            const int cols = a.tb * D;
            for (int i = tid; i < 256; i += blockDim.x) {
                const int col = i >> 4, f = i & 15;
                float y = 0.f;
                if (col < cols && f < nf) {
                    const int sl = col / D, ax = col - sl * D;
                    const T *z = gbuf + sl * S + ax * NVP;
                    y = (float)z[3 + f] - (hfb[f * 4 + 0] * (float)z[0] + hfb[f * 4 + 1] * (float)z[1] +
                                           hfb[f * 4 + 2] * (float)z[2] + hfb[f * 4 + 3] * (float)z[a.nv - 1]);
                }
                yb[i] = y;
            }
            lds_barrier();
            const int cn = lane & 15, k0 = 4 * (lane >> 4);
            if (tid < 64) {
                float yv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) yv[i] = yb[cn * 16 + k0 + i];
                const f32x4 d0 = qp_mfma(ahi, alo, yv);
#pragma unroll
                for (int i = 0; i < 4; ++i) db[cn * 16 + k0 + i] = d0[i];
            }
            lds_barrier();
            if (tid < 64) {
                float rv[4], dv[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) dv[k] = db[cn * 16 + k];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float r = yb[cn * 16 + k0 + i];
#pragma unroll
                    for (int k = 0; k < 16; ++k) r = fmaf(-hff[(k0 + i) * 16 + k], dv[k], r);
                    rv[i] = r;
                }
                const f32x4 d1 = qp_mfma(ahi, alo, rv);
#pragma unroll
                for (int i = 0; i < 4; ++i) db[cn * 16 + k0 + i] = dv[k0 + i] + d1[i];
            }
            lds_barrier();
            if (owner) {
                if (o_free) xb_o += (T)db[(ls * D + o_ax) * 16 + (o_m - 3)];
                else if (o_real) xb_o = bnd_o;
                xbuf[(nxt * a.tb + ls) * S + lt] = xb_o;
            }
        } else {
            // The owners of a sample are lanes of one wave: their LDS writes of g are
            // visible to each other after a wavefront-scope fence, no block barrier.
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (owner) {
                if (o_free) {
                    const T *wr = wmat + (o_m - 3) * NVP;
                    const T *g = gbuf + ls * S + o_ax * NVP;
                    T d = T(0);
#pragma unroll
                    for (int m = 0; m < NVP; ++m) d = fma(wr[m], g[m], d);
                    xb_o += d;
                } else if (o_real) {
                    xb_o = bnd_o;
                }
                xbuf[(nxt * a.tb + ls) * S + lt] = xb_o;
            }
        }
        cur = nxt;
        lds_barrier();
    }

    if (o_real) {
        a.xb[gidx] = xb_o;
        a.lam[gidx] = lam_o;
        nonfinite = nonfinite || !isfinite(xb_o) || !isfinite(lam_o);
    }
    if (a.flags && a.iters > 0) {
        // the residual lane's bits reach the sample's first lane through LDS
        // (r2p is free after the loop's last barrier)
        if (res_lane) r2p[ls * wpt] = T((nonfinite ? 1 : 0) + (res_last > res_first ? 2 : 0));
        __syncthreads();
        const bool anyb = __any(nonfinite && owner);
        if (owner && lt == 0) {
            const int rb = (int)r2p[ls * wpt];
            uint32_t fl = (uint32_t)rb;
            if (anyb) fl |= 1u;
            a.flags[sample] = fl;
        }
    }
}


// ----------------------------------------------------------------------------
// One sample's whole projection on one wavefront: lane l owns time samples l,
// l + 64, ... (TPL of them).  The F^T r reduce-scatter leaves coefficient o's sum in
// lane o << (6 - log2 V), which is also its owner lane for the multiplier, the defect
// and the QP update, so the iteration needs no block barrier.  wmat [NVP][NVP] holds
// the QP operator, xs / gs [D*NVP] this wave's iterate and defect (LDS); db, hff,
// hfb and the A operands are used by the bf16 matrix-core QP only.
template <typename T, int D, int NVP, int TPL, bool MQP, typename A, int OM = kObsEither>
__device__ __forceinline__ void wave_sample(const A &a, const int sample, const int lane,
                                            const T *wmat, T *xs, T *gs, float *db,
                                            const float *hff, const float *hfb, bf16x4 ahi,
                                            bf16x4 alo)
{
    constexpr int S = D * NVP;
    constexpr int V = pow2ceil(S);
    constexpr int LOGV = (V >= 64) ? 6 : (V >= 32) ? 5 : (V >= 16) ? 4 : 3;
    constexpr int OSH = 6 - LOGV;
    const int nf = a.nv - 4;
    // This lane's time samples: the position rows of the basis in registers for the
    // launch.  In the plain FP32 kernel the derivative rows are read from the
    // (cache-resident) table where they are used, a row at a time, which keeps the
    // config-3 wave at two per SIMD; in FP64 and with the matrix-core QP they stay in
    // registers too (there the loads cost more than the occupancy they would buy).
    // Lanes past n_p read row 0 and discard what it gives.
    constexpr bool kHold = sizeof(T) == 8 || MQP;
    constexpr int HR = kHold ? TPL : 1;
    T tt[TPL], phi0[TPL][NVP], phi1[HR][NVP], phi2[HR][NVP];
    bool valid[TPL];
    const T *drow[TPL];   // the lane's first-derivative row; the second follows n_p rows later
#pragma unroll
    for (int i = 0; i < TPL; ++i) {
        const int t = lane + 64 * i;
        valid[i] = t < a.n_p;
        tt[i] = T(t) * a.dt;
        drow[i] = a.phi + (size_t)(1 * a.n_p + (valid[i] ? t : 0)) * NVP;
#pragma unroll
        for (int m = 0; m < NVP; ++m) phi0[i][m] = valid[i] ? a.phi[(0 * a.n_p + t) * NVP + m] : T(0);
    }
    const size_t d2 = (size_t)a.n_p * NVP;   // from a first-derivative row to its second
    if constexpr (kHold) {
#pragma unroll
        for (int i = 0; i < HR; ++i)
#pragma unroll
            for (int m = 0; m < NVP; ++m) {
                phi1[i][m] = valid[i] ? drow[i][m] : T(0);
                phi2[i][m] = valid[i] ? drow[i][d2 + m] : T(0);
            }
    }

    const int o = lane >> OSH;
    const bool owner = (lane & ((1 << OSH) - 1)) == 0 && o < S;
    const int o_ax = o / NVP, o_m = o - (o / NVP) * NVP;
    const bool o_real = owner && o_m < a.nv;
    const bool o_free = o_real && o_m >= 3 && o_m < a.nv - 1;
    const size_t gidx = (size_t)sample * D * a.nv + (size_t)o_ax * a.nv + o_m;
    T xi_o = T(0), lam_o = T(0), xb_o = T(0), bnd_o = T(0);
    if (o_real) {
        xi_o = a.xi[gidx];
        lam_o = a.lam[gidx];
        xb_o = a.xb[gidx];
        if (!o_free) bnd_o = a.xiB[o_ax][(o_m == a.nv - 1) ? 3 : o_m];
    }
    if (owner) xs[o] = xb_o;
    wave_lds_sync();

    const ObsChunk<T, D> oc0 = load_obs_chunk<T, D>(a.obs, a.n_o, 0, lane);
    CullCache<T, D, TPL> ccache;   // obstacle candidates kept across iterations
    T res_first = T(0), res_last = T(0);
    bool nonfinite = false;
    // Penalty continuation (thesis ch. 4 Alg 1, ch. 7): this sample's level on the
    // penalty ladder, the iterations since the last check and the residual then.  The
    // level's penalty enters the multiplier update and its QP operator the QP; after
    // each iteration the count rises, and every cont_window iterations the level goes
    // up by one when the residual is above cont_tol and above cont_stall times the
    // reference (0 before the first check).  All wave-uniform.
    const bool cont = a.cont_levels > 0;
    ContState *cst = cont ? reinterpret_cast<ContState *>(a.cont_state) + sample : nullptr;
    int c_lev = 0, c_cnt = 0;
    T c_ref = T(0);
    if (cont) {
        c_lev = cst->level;
        c_cnt = cst->count;
        c_ref = (T)cst->ref;
    }
    for (int k = 0; k < a.iters; ++k) {
        const T rho = cont ? a.cont_rho[c_lev] : a.rho;
        // ---- step (a): waypoints and polar steps
        T p[TPL][D], v[TPL][D], acc[TPL][D];
#pragma unroll
        for (int i = 0; i < TPL; ++i)
#pragma unroll
            for (int ax = 0; ax < D; ++ax) { p[i][ax] = T(0); v[i][ax] = T(0); acc[i][ax] = T(0); }
        if constexpr (kHold) {
#pragma unroll
            for (int ax = 0; ax < D; ++ax)
#pragma unroll
                for (int m = 0; m < NVP; ++m) {
                    const T c = xs[ax * NVP + m];
#pragma unroll
                    for (int i = 0; i < TPL; ++i) {
                        p[i][ax] = fma(phi0[i][m], c, p[i][ax]);
                        v[i][ax] = fma(phi1[i < HR ? i : 0][m], c, v[i][ax]);
                        acc[i][ax] = fma(phi2[i < HR ? i : 0][m], c, acc[i][ax]);
                    }
                }
        } else {
#pragma unroll
            for (int i = 0; i < TPL; ++i) {
                T r1[NVP], r2r[NVP];
#pragma unroll
                for (int m = 0; m < NVP; ++m) {
                    r1[m] = drow[i][m];
                    r2r[m] = drow[i][d2 + m];
                }
#pragma unroll
                for (int ax = 0; ax < D; ++ax)
#pragma unroll
                    for (int m = 0; m < NVP; ++m) {
                        const T c = xs[ax * NVP + m];
                        p[i][ax] = fma(phi0[i][m], c, p[i][ax]);
                        v[i][ax] = fma(r1[m], c, v[i][ax]);
                        acc[i][ax] = fma(r2r[m], c, acc[i][ax]);
                    }
                if (!valid[i])
#pragma unroll
                    for (int ax = 0; ax < D; ++ax) { v[i][ax] = T(0); acc[i][ax] = T(0); }
            }
        }
        // Lanes past n_p sit at -1e30: never inside an obstacle, and far from the
        // padding sentinels at +1e30 as well.
#pragma unroll
        for (int i = 0; i < TPL; ++i)
            if (!valid[i])
#pragma unroll
                for (int ax = 0; ax < D; ++ax) p[i][ax] = T(-1e30);
        T R[TPL][D], rv[TPL][D], ra[TPL][D], r2 = T(0), rmax = T(0);
#pragma unroll
        for (int i = 0; i < TPL; ++i)
#pragma unroll
            for (int ax = 0; ax < D; ++ax) { R[i][ax] = T(0); rv[i][ax] = T(0); ra[i][ax] = T(0); }
        obstacle_residuals_culled<T, D, TPL, OM>(a.obs, a.n_o, a.sphere, a.dynamic, oc0, tt, p, valid, R, r2, rmax,
                                                 ccache);
#pragma unroll
        for (int i = 0; i < TPL; ++i) {
            if (a.use_v) bound_residual<T, D>(v[i], a.vmax, rv[i], r2, rmax);
            if (a.use_a) bound_residual<T, D>(acc[i], a.amax, ra[i], r2, rmax);
            if (a.use_ws && valid[i]) workspace_residual(p[i], a.ws_lo, a.ws_hi, R[i], r2, rmax);
        }
        // ---- F^T r over the wave
        // residual groups enter only when some lane has them non-zero (exact zeros skipped)
        bool nR = false, nV = false, nA = false;
#pragma unroll
        for (int i = 0; i < TPL; ++i)
#pragma unroll
            for (int ax = 0; ax < D; ++ax) {
                nR = nR || R[i][ax] != T(0);
                nV = nV || rv[i][ax] != T(0);
                nA = nA || ra[i][ax] != T(0);
            }
        const bool aR = __any(nR), aV = __any(nV), aA = __any(nA);
        T ftr = T(0);
        if (aR || aV || aA) {
            T c[V];
#pragma unroll
            for (int j = 0; j < V; ++j) c[j] = T(0);
#pragma unroll
            for (int i = 0; i < TPL; ++i) {
                if constexpr (kHold) {
                    if (aA)
#pragma unroll
                        for (int ax = 0; ax < D; ++ax)
#pragma unroll
                            for (int m = 0; m < NVP; ++m)
                                c[ax * NVP + m] = fma(phi2[i < HR ? i : 0][m], ra[i][ax], c[ax * NVP + m]);
                    if (aV)
#pragma unroll
                        for (int ax = 0; ax < D; ++ax)
#pragma unroll
                            for (int m = 0; m < NVP; ++m)
                                c[ax * NVP + m] = fma(phi1[i < HR ? i : 0][m], rv[i][ax], c[ax * NVP + m]);
                } else {
                    if (aA) {
                        T row[NVP];
#pragma unroll
                        for (int m = 0; m < NVP; ++m) row[m] = drow[i][d2 + m];
#pragma unroll
                        for (int ax = 0; ax < D; ++ax)
#pragma unroll
                            for (int m = 0; m < NVP; ++m) c[ax * NVP + m] = fma(row[m], ra[i][ax], c[ax * NVP + m]);
                    }
                    if (aV) {
                        T row[NVP];
#pragma unroll
                        for (int m = 0; m < NVP; ++m) row[m] = drow[i][m];
#pragma unroll
                        for (int ax = 0; ax < D; ++ax)
#pragma unroll
                            for (int m = 0; m < NVP; ++m) c[ax * NVP + m] = fma(row[m], rv[i][ax], c[ax * NVP + m]);
                    }
                }
                if (aR)
#pragma unroll
                    for (int ax = 0; ax < D; ++ax)
#pragma unroll
                        for (int m = 0; m < NVP; ++m) c[ax * NVP + m] = fma(phi0[i][m], R[i][ax], c[ax * NVP + m]);
            }
            ftr = reduce_scatter<T, V>(c, lane);
        }
        const T r2w = wave_sum(r2);
        // ---- step (c): multiplier (eq lag) and the QP defect
        if (owner) {
            T gv = T(0);
            if (o_real) {
                lam_o = fma(-rho, ftr, lam_o);
                gv = o_free ? (xi_o - xb_o + lam_o - rho * ftr) : (bnd_o - xb_o);
            }
            gs[o] = gv;
        }
        if (lane == 0) {
            const T rs = sqrt(r2w);
            if (a.res) a.res[(size_t)k * a.batch + sample] = rs;
            if (k == 0) res_first = rs;
            res_last = rs;
            nonfinite = nonfinite || !isfinite(rs);
        }
        const int c_lev_k = c_lev;   // the level this iteration's QP uses
        if (cont) {
            // the check after the iteration decides the next one's penalty (lane 0's
            // residual, so the decision is uniform)
            const T rs = readlane_t<T>(sqrt(r2w), 0);
            if (++c_cnt >= a.cont_window) {
                if (rs > a.cont_tol && rs > a.cont_stall * c_ref && c_lev < a.cont_levels - 1)
                    ++c_lev;
                c_ref = rs;
                c_cnt = 0;
            }
        }
        wave_lds_sync();
        // ---- step (b): the fixed-matrix QP on the defect (eq affine_trans)
        if constexpr (MQP) {
            const int cn = lane & 15, k0 = 4 * (lane >> 4);
            float yv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int f = k0 + i;
                float y = 0.f;
                if (cn < D && f < nf) {
                    const T *z = gs + cn * NVP;
                    y = (float)z[3 + f] - (hfb[f * 4 + 0] * (float)z[0] + hfb[f * 4 + 1] * (float)z[1] +
                                           hfb[f * 4 + 2] * (float)z[2] + hfb[f * 4 + 3] * (float)z[a.nv - 1]);
                }
                yv[i] = y;
            }
            const f32x4 d0 = qp_mfma(ahi, alo, yv);
#pragma unroll
            for (int i = 0; i < 4; ++i) db[cn * 16 + k0 + i] = d0[i];
            wave_lds_sync();
            float dv[16], rv4[4];
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) dv[kk] = db[cn * 16 + kk];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float r = yv[i];
#pragma unroll
                for (int kk = 0; kk < 16; ++kk) r = fmaf(-hff[(k0 + i) * 16 + kk], dv[kk], r);
                rv4[i] = r;
            }
            const f32x4 d1 = qp_mfma(ahi, alo, rv4);
            wave_lds_sync();
#pragma unroll
            for (int i = 0; i < 4; ++i) db[cn * 16 + k0 + i] = d0[i] + d1[i];
            wave_lds_sync();
            if (o_free) xb_o += (T)db[o_ax * 16 + (o_m - 3)];
            else if (o_real) xb_o = bnd_o;
        } else {
            if (o_free) {
                const T *g = gs + o_ax * NVP;
                T d = T(0);
                if (cont) {   // the level's operator, from the (cached) table
                    const T *wr = a.cont_W + ((size_t)c_lev_k * NVP + (o_m - 3)) * NVP;
#pragma unroll
                    for (int m = 0; m < NVP; ++m) d = fma(wr[m], g[m], d);
                } else {
                    const T *wr = wmat + (o_m - 3) * NVP;
#pragma unroll
                    for (int m = 0; m < NVP; ++m) d = fma(wr[m], g[m], d);
                }
                xb_o += d;
            } else if (o_real) {
                xb_o = bnd_o;
            }
        }
        if (owner) xs[o] = xb_o;
        wave_lds_sync();
    }

    if (o_real) {
        a.xb[gidx] = xb_o;
        a.lam[gidx] = lam_o;
        nonfinite = nonfinite || !isfinite(xb_o) || !isfinite(lam_o);
    }
    if (cont && lane == 0) {
        cst->level = c_lev;
        cst->count = c_cnt;
        cst->ref = (double)c_ref;
    }
    if (a.flags && a.iters > 0) {
        const bool anyb = __any(nonfinite);
        if (lane == 0) {
            uint32_t fl = 0;
            if (anyb) fl |= 1u;
            if (res_last > res_first) fl |= 2u;
            a.flags[sample] = fl;
        }
    }
}

// Wave-per-sample AM kernel: `a.tb` samples per workgroup (= waves per workgroup),
// each wave independent of the others after the constant set-up.
template <typename T, int D, int NVP, int TPL, bool MQP, int OM>
__global__ __launch_bounds__(kMaxThreads) void am_wave_kernel(AmArgs<T> a)
{
    constexpr int S = D * NVP;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *smem = reinterpret_cast<T *>(smem_raw);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int sample = blockIdx.x * a.tb + wv;
    const int nf = a.nv - 4;

    T *wmat = smem;                                   // [NVP][NVP]
    T *xs = smem + NVP * NVP + wv * 2 * S;            // this wave's xb
    T *gs = xs + S;                                   // this wave's defect
    float *mqbase = reinterpret_cast<float *>(smem + NVP * NVP + a.tb * 2 * S);
    float *db = mqbase + wv * 256;                    // MQP: delta tile [16 cols][16 rows]
    float *hff = mqbase + a.tb * 256;                 // MQP: H_ff [16][16]
    float *hfb = hff + 256;                           // MQP: H_fb [16][4]

    for (int i = tid; i < NVP * NVP; i += blockDim.x) {
        const int f = i / NVP, m = i - f * NVP;
        wmat[i] = (f < nf) ? a.W[f * NVP + m] : T(0);
    }
    bf16x4 ahi = {0, 0, 0, 0}, alo = {0, 0, 0, 0};
    if constexpr (MQP) {
        const int m = lane & 15, k0 = 4 * (lane >> 4);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ahi[i] = (short)a.Whi[m * 16 + k0 + i];
            alo[i] = (short)a.Wlo[m * 16 + k0 + i];
        }
        for (int i = tid; i < 256 + 64; i += blockDim.x) hff[i] = a.Hmq[i];
    }
    __syncthreads();
    if (sample >= a.batch) return;  // waves are independent from here on
    wave_sample<T, D, NVP, TPL, MQP, AmArgs<T>, OM>(a, sample, lane, wmat, xs, gs, db, hff, hfb, ahi, alo);
}

// ----------------------------------------------------------------------------
// Multi-agent joint projection (thesis ch. 7, Paper IV, in the projection form of ch. 6).
// One wave per joint sample, lane a = agent a: each lane keeps its agent's
// coefficients, multiplier and F^T r in registers and walks the time samples; the
// basis rows and the obstacles are wave-uniform (scalar loads), and the other
// agents' positions at the current time come from v_readlane, so the pair rows need
// no LDS and no barrier.  A pair (a, b) is evaluated by both of its lanes on
// x~ = p_a - p_b resp. p_b - p_a; the residual of the exterior-of-a-sphere polar
// step (eqs sphere_proposed, com_alpha_i, com_beta_i, com_d_i) is an odd function of
// x~, so both lanes get the exact negatives of each other and each adds its own sign;
// only the exact tie x~ = 0 is not odd, and there the lower-index agent is pushed
// along +x (2D) / +z (3D) and the other one the opposite way.  The squared residual
// counts every pair once (lane a < b).
//
// Joint QP: with L = N I - 1 1^T the Gram of the pair rows, the free block of the
// joint Hessian is I (x) A + L (x) B (A = H_ff, B = rho (P^T P)_ff).  Splitting every
// agent's defect vector u_a (free defect, boundary shift) into the agent mean u_m and
// the deviation u_a - u_m diagonalizes it exactly: the mean moves by the single-robot
// operator W and each deviation by W2, the same operator built for H + N rho P^T P.

// Polar step of every (agent, obstacle), kinematic bound and pair row at time t for
// this lane's position p, velocity v, acceleration acc.  Adds the summed position
// residual to S and the velocity / acceleration residuals to rv / ra.
// px: this wave's LDS area of kAgentPosScalars for the agents' positions.  The lane
// serves agent `ag` of the half-wave `h` (h = 0 unless the wave's two halves take two
// time steps of one joint sample: then lane = 32 h + ag and every exchange between
// agents stays within the half).
template <typename T, int D, typename A>
__device__ __forceinline__ void agents_rows(const A &a, const T *ol, T *px, int lane, int ag, int h, bool active, T tt,
                                            const T (&p)[D], const T (&v)[D], const T (&acc)[D], T (&S)[D],
                                            T (&rv)[D], T (&ra)[D], T &r2, T &rmax)
{
    const int N = a.n_agents;
    {
        T p1[1][D], S1[1][D], tt1[1] = {tt};
        const bool ok1[1] = {active};
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            p1[0][ax] = active ? p[ax] : T(-1e30);
            S1[0][ax] = T(0);
        }
        // obstacles staged in LDS: only those whose box meets the agents' positions
        // at this time are tested (exactly; see obstacle_cull_loop)
        if (ol) obstacle_residuals_staged<T, D, 1>(ol, a.obs, a.n_o, a.sphere, a.dynamic, tt1, p1, ok1, S1, r2, rmax);
        else obstacle_residuals<T, D, 1>(a.obs_soa, a.obs, a.n_o, a.sphere, a.dynamic, tt1, p1, S1, r2, rmax);
#pragma unroll
        for (int ax = 0; ax < D; ++ax) S[ax] = S1[0][ax];
    }
#pragma unroll
    for (int ax = 0; ax < D; ++ax) { rv[ax] = T(0); ra[ax] = T(0); }
    if (active) {
        if (a.use_v) bound_residual<T, D>(v, a.vmax, rv, r2, rmax);
        if (a.use_a) bound_residual<T, D>(acc, a.amax, ra, r2, rmax);
        if (a.use_ws) workspace_residual(p, a.ws_lo, a.ws_hi, S, r2, rmax);
    }
    // Pair rows, each unordered pair evaluated once: at offset o = 1 .. N/2 lane a takes
    // partner b = (a + o) mod N, so every lane does about N/2 clearance tests instead
    // of N - 1.  The partner's row is the exact negation of lane a's (x_ba = -x_ab and
    // the same scale factor), handed over with a lane rotation by o when some pair at
    // this offset is near; at o = N/2 (N even) both lanes of a pair meet it, so each
    // keeps its own row.  Positions are published in LDS twice over (entries a and
    // a + N), so partner a + o needs no wrap, and read four offsets at a time.
    const T R = a.pair_r, R2 = R * R;
    const int e0 = 64 * h + ag;   // this agent's entry in the half's table
    if (active) {
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            px[4 * e0 + ax] = p[ax];
            px[4 * (e0 + N) + ax] = p[ax];
        }
    }
    wave_lds_sync();
    const int half = N >> 1;
    // agents past N are inactive: they read entry 64 h + ag + o < 128 (ag + o < 96 with
    // one half, < 48 with two), whatever it holds
    const T *pq = px + 4 * e0;
    for (int o0 = 1; o0 <= half; o0 += 4) {
        T x[4][D];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int o = min(o0 + j, half);   // past half: a repeated offset, skipped below
#pragma unroll
            for (int ax = 0; ax < D; ++ax) x[j][ax] = p[ax] - pq[4 * o + ax];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int o = o0 + j;
            if (o > half) break;
            T nn = T(0);
#pragma unroll
            for (int ax = 0; ax < D; ++ax) nn = fma(x[j][ax], x[j][ax], nn);
            const bool near = active && nn < R2;
            const bool mid = 2 * o == N;
            T r[D];
#pragma unroll
            for (int ax = 0; ax < D; ++ax) r[ax] = T(0);
            if (near) {
                const int b = ag + o < N ? ag + o : ag + o - N;
                if (nn > T(0)) {
                    const T f = T(1) - R * rsqrt_t(nn);
#pragma unroll
                    for (int ax = 0; ax < D; ++ax) r[ax] = x[j][ax] * f;
                } else {
                    // coincident agents: a fixed axis and the lane order give the direction
                    r[D == 2 ? 0 : 2] = ag < b ? -R : R;
                }
                T rr = T(0);
#pragma unroll
                for (int ax = 0; ax < D; ++ax) {
                    S[ax] += r[ax];
                    rr = fma(r[ax], r[ax], rr);
                    rmax = fmax(rmax, fabs(r[ax]));
                }
                if (!mid || ag < b) r2 += rr;
            }
            if (!mid && __any(near)) {
                // the lane whose partner at this offset is this lane
                int src = ag - o;
                src = src < 0 ? src + N : src;
                src = active ? 32 * h + src : lane;
#pragma unroll
                for (int ax = 0; ax < D; ++ax) {
                    const T g = shfl_t<T>(r[ax], src);
                    if (active) S[ax] -= g;
                }
            }
        }
    }
    wave_lds_sync();  // every lane has read the positions before the next time step
}

// One joint sample's whole projection on one wavefront (n_agents <= 64 lanes).
template <typename T, int D, int NVP, typename A>
__device__ __forceinline__ void agents_sample(const A &a, const int sample, const int lane, T *ol, T *px)
{
    if (ol) stage_obstacles<T, D>(ol, a.obs, a.n_o, a.sphere, lane);
    const int N = a.n_agents, nv = a.nv, n_p = a.n_p;
    // N <= 32: the wave's halves take the even and the odd time steps of the sample
    // (lane 32 h + ag serves agent ag at times 2 s + h); both halves hold the agent's
    // whole state and apply the same QP step
    const bool split = N <= 32;
    const int h = split ? (lane >> 5) : 0;
    const int ag = split ? (lane & 31) : lane;
    const bool active = ag < N;
    const TRAJAM_CONST_AS T *phi = (const TRAJAM_CONST_AS T *)a.phi;
    const TRAJAM_CONST_AS T *W1 = (const TRAJAM_CONST_AS T *)a.W;
    const TRAJAM_CONST_AS T *W2 = (const TRAJAM_CONST_AS T *)a.W2;
    T xi[D][NVP], xb[D][NVP], lam[D][NVP], bnd[D][4];
    const size_t base = ((size_t)sample * N + (active ? ag : 0)) * D * nv;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
#pragma unroll
        for (int m = 0; m < NVP; ++m) {
            const bool real = active && m < nv;
            xi[ax][m] = real ? a.xi[base + ax * nv + m] : T(0);
            xb[ax][m] = real ? a.xb[base + ax * nv + m] : T(0);
            lam[ax][m] = real ? a.lam[base + ax * nv + m] : T(0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) bnd[ax][i] = active ? a.xiB_ag[((active ? ag : 0) * D + ax) * 4 + i] : T(0);
    }
    T res_first = T(0), res_last = T(0);
    bool nonfinite = false;
    for (int k = 0; k < a.iters; ++k) {
        T ftr[D][NVP];
#pragma unroll
        for (int ax = 0; ax < D; ++ax)
#pragma unroll
            for (int m = 0; m < NVP; ++m) ftr[ax][m] = T(0);
        T r2 = T(0), rmax = T(0);
        for (int t0 = 0; t0 < n_p; t0 += split ? 2 : 1) {
            const int t = t0 + h;
            const bool on = active && t < n_p;
            // basis rows of the wave's time steps (uniform: scalar loads, SGPR operands)
            const int t1 = (split && t0 + 1 < n_p) ? t0 + 1 : t0;
            T ph[3][NVP], pk[3][NVP];
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int m = 0; m < NVP; ++m) {
                    ph[d][m] = phi[(size_t)(d * n_p + t0) * NVP + m];
                    pk[d][m] = phi[(size_t)(d * n_p + t1) * NVP + m];
                }
            T p[D], v[D], acc[D];
#pragma unroll
            for (int ax = 0; ax < D; ++ax) {
                T sp = T(0), sv = T(0), sa = T(0);
#pragma unroll
                for (int m = 0; m < NVP; ++m) {
                    sp = fma(ph[0][m], xb[ax][m], sp);
                    sv = fma(ph[1][m], xb[ax][m], sv);
                    sa = fma(ph[2][m], xb[ax][m], sa);
                }
                if (split) {   // the odd half's step
                    T qp = T(0), qv = T(0), qa = T(0);
#pragma unroll
                    for (int m = 0; m < NVP; ++m) {
                        qp = fma(pk[0][m], xb[ax][m], qp);
                        qv = fma(pk[1][m], xb[ax][m], qv);
                        qa = fma(pk[2][m], xb[ax][m], qa);
                    }
                    sp = h ? qp : sp;
                    sv = h ? qv : sv;
                    sa = h ? qa : sa;
                }
                p[ax] = sp;
                v[ax] = sv;
                acc[ax] = sa;
            }
            T S[D], rv[D], ra[D];
            agents_rows<T, D, A>(a, ol, px, lane, ag, h, on, T(t) * a.dt, p, v, acc, S, rv, ra, r2, rmax);
            if (split) {   // each half adds its own step's rows
#pragma unroll
                for (int ax = 0; ax < D; ++ax) {
                    const T s0 = h ? T(0) : S[ax], v0 = h ? T(0) : rv[ax], a0 = h ? T(0) : ra[ax];
                    const T s1 = h ? S[ax] : T(0), v1 = h ? rv[ax] : T(0), a1 = h ? ra[ax] : T(0);
#pragma unroll
                    for (int m = 0; m < NVP; ++m)
                        ftr[ax][m] = fma(ph[0][m], s0, fma(ph[1][m], v0, fma(ph[2][m], a0,
                                     fma(pk[0][m], s1, fma(pk[1][m], v1, fma(pk[2][m], a1, ftr[ax][m]))))));
                }
            } else {
#pragma unroll
                for (int ax = 0; ax < D; ++ax)
#pragma unroll
                    for (int m = 0; m < NVP; ++m)
                        ftr[ax][m] = fma(ph[0][m], S[ax], fma(ph[1][m], rv[ax], fma(ph[2][m], ra[ax], ftr[ax][m])));
            }
        }
        if (split) {   // F^T r over both halves' time steps, the same sum in both halves
#pragma unroll
            for (int ax = 0; ax < D; ++ax)
#pragma unroll
                for (int m = 0; m < NVP; ++m) ftr[ax][m] += shfl_t<T>(ftr[ax][m], lane ^ 32);
        }
        const T r2w = wave_sum(r2);
        if (lane == 0) {
            const T rs = sqrt(r2w);
            if (a.res) a.res[(size_t)k * a.batch + sample] = rs;
            if (k == 0) res_first = rs;
            res_last = rs;
            nonfinite = nonfinite || !isfinite(rs);
        }
        // step (c): multiplier; then the defect u of every coefficient
        T u[D][NVP];
#pragma unroll
        for (int ax = 0; ax < D; ++ax)
#pragma unroll
            for (int m = 0; m < NVP; ++m) {
                T uv = T(0);
                if (active && m < nv) {
                    lam[ax][m] = fma(-a.rho, ftr[ax][m], lam[ax][m]);
                    const int bi = (m == nv - 1) ? 3 : m;
                    uv = (m >= 3 && m < nv - 1) ? (xi[ax][m] - xb[ax][m] + lam[ax][m] - a.rho * ftr[ax][m])
                                                : (bnd[ax][bi] - xb[ax][m]);
                }
                u[ax][m] = uv;
            }
        // step (b): agent mean by the single-robot operator, deviations by W2
        const T invN = T(1) / T(N);
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            T um[NVP];
#pragma unroll
            for (int m = 0; m < NVP; ++m) um[m] = (m < nv) ? wave_sum(h ? T(0) : u[ax][m]) * invN : T(0);
#pragma unroll
            for (int f = 0; f < NVP - 4; ++f) {
                if (f < nv - 4) {
                    T d = T(0);
#pragma unroll
                    for (int m = 0; m < NVP; ++m)
                        d = fma(W1[f * NVP + m], um[m], fma(W2[f * NVP + m], u[ax][m] - um[m], d));
                    if (active) xb[ax][3 + f] += d;
                }
            }
            if (active) {
                xb[ax][0] = bnd[ax][0];
                xb[ax][1] = bnd[ax][1];
                xb[ax][2] = bnd[ax][2];
#pragma unroll
                for (int m = 3; m < NVP; ++m)
                    if (m == nv - 1) xb[ax][m] = bnd[ax][3];
            }
        }
    }
    if (active && h == 0) {
#pragma unroll
        for (int ax = 0; ax < D; ++ax)
#pragma unroll
            for (int m = 0; m < NVP; ++m)
                if (m < nv) {
                    a.xb[base + ax * nv + m] = xb[ax][m];
                    a.lam[base + ax * nv + m] = lam[ax][m];
                    nonfinite = nonfinite || !isfinite(xb[ax][m]) || !isfinite(lam[ax][m]);
                }
    }
    if (a.flags && a.iters > 0) {
        const bool anyb = __any(nonfinite);
        if (lane == 0) {
            uint32_t fl = 0;
            if (anyb) fl |= 1u;
            if (res_last > res_first) fl |= 2u;
            a.flags[sample] = fl;
        }
    }
}

// Residual only, at the given joint coefficients: res[sample] = 2-norm, res_max.
template <typename T, int D, int NVP, typename A>
__device__ __forceinline__ void agents_residual(const A &a, const int sample, const int lane, T *ol, T *px)
{
    if (ol) stage_obstacles<T, D>(ol, a.obs, a.n_o, a.sphere, lane);
    const int N = a.n_agents, nv = a.nv, n_p = a.n_p;
    const bool active = lane < N;
    const TRAJAM_CONST_AS T *phi = (const TRAJAM_CONST_AS T *)a.phi;
    T xb[D][NVP];
    const size_t base = ((size_t)sample * N + (active ? lane : 0)) * D * nv;
#pragma unroll
    for (int ax = 0; ax < D; ++ax)
#pragma unroll
        for (int m = 0; m < NVP; ++m) xb[ax][m] = (active && m < nv) ? a.xb[base + ax * nv + m] : T(0);
    T r2 = T(0), rmax = T(0);
    for (int t = 0; t < n_p; ++t) {
        T p[D], v[D], acc[D];
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            T sp = T(0), sv = T(0), sa = T(0);
#pragma unroll
            for (int m = 0; m < NVP; ++m) {
                sp = fma(phi[(size_t)(0 * n_p + t) * NVP + m], xb[ax][m], sp);
                sv = fma(phi[(size_t)(1 * n_p + t) * NVP + m], xb[ax][m], sv);
                sa = fma(phi[(size_t)(2 * n_p + t) * NVP + m], xb[ax][m], sa);
            }
            p[ax] = sp;
            v[ax] = sv;
            acc[ax] = sa;
        }
        T S[D], rv[D], ra[D];
        agents_rows<T, D, A>(a, ol, px, lane, lane, 0, active, T(t) * a.dt, p, v, acc, S, rv, ra, r2, rmax);
    }
    const T r2w = wave_sum(r2), mx = wave_max(rmax);
    if (lane == 0) {
        a.res[sample] = sqrt(r2w);
        if (a.res_max) a.res_max[sample] = mx;
    }
}

// Per-wave LDS of the multi-agent kernels: a.cull_lds scalars of obstacle stage (0 =
// no culling), then kAgentPosScalars for the agents' positions.
template <typename T, int D, int NVP>
__global__ __launch_bounds__(kMaxThreads) void am_agents_kernel(AmArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int sample = blockIdx.x * a.tb + (threadIdx.x >> 6);
    if (sample >= a.batch) return;  // whole waves leave together
    T *slot = reinterpret_cast<T *>(smem_raw) + (threadIdx.x >> 6) * (a.cull_lds + kAgentPosScalars);
    agents_sample<T, D, NVP, AmArgs<T>>(a, sample, threadIdx.x & 63, a.cull_lds ? slot : nullptr, slot + a.cull_lds);
}

template <typename T, int D, int NVP>
__global__ __launch_bounds__(kMaxThreads) void am_agents_residual_kernel(AmArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int sample = blockIdx.x * a.tb + (threadIdx.x >> 6);
    if (sample >= a.batch) return;
    T *slot = reinterpret_cast<T *>(smem_raw) + (threadIdx.x >> 6) * (a.cull_lds + kAgentPosScalars);
    agents_residual<T, D, NVP, AmArgs<T>>(a, sample, threadIdx.x & 63, a.cull_lds ? slot : nullptr,
                                          slot + a.cull_lds);
}

// ----------------------------------------------------------------------------
// Ragged persistent launch: many independent problems (each its own fixed matrices,
// obstacles, batch) in one launch; single-robot and multi-agent problems go to two
// instantiations (their register budgets differ by a wave per SIMD).  Every wave repeatedly takes the next work unit
// (problem, sample) from a device counter and runs that sample's whole projection;
// problems are ordered longest-first on the host, so the expensive units start first
// and the short ones fill the tail.  Every wave exits once the counter passes the
// last unit.  FP32; per unit the kernel dispatches to the (dims, padded coefficients,
// time samples per lane) instantiation of the problem.
constexpr int kRaggedWaveLds = 16 * 16 + 2 * 3 * 16;  // floats per wave: W, xb, defect

using RaggedArgs = TRAJAM_CONST_AS AmArgs<float>;

template <int D, int NVP, int TPL>
__device__ __forceinline__ void ragged_unit(const RaggedArgs &a, int sample, int lane, float *wl)
{
    constexpr int S = D * NVP;
    const int nf = a.nv - 4;
    for (int i = lane; i < NVP * NVP; i += 64) {
        const int f = i / NVP, m = i - f * NVP;
        wl[i] = (f < nf) ? a.W[f * NVP + m] : 0.f;
    }
    wave_lds_sync();
    const bf16x4 z = {0, 0, 0, 0};
    float *xs = wl + 256;
    wave_sample<float, D, NVP, TPL, false, RaggedArgs>(a, sample, lane, wl, xs, xs + S, nullptr, nullptr, nullptr,
                                                       z, z);
    wave_lds_sync();  // this wave's LDS is reused by its next unit
}

template <bool AGENTS>
__global__ __launch_bounds__(kMaxThreads) void am_ragged_kernel(const AmArgs<float> *__restrict__ probs_g,
                                                                const int *__restrict__ offsets_g, int n_probs,
                                                                int total, int *__restrict__ counter, int wave_lds)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *wl = reinterpret_cast<float *>(smem_raw) + (threadIdx.x >> 6) * wave_lds;
    const int lane = threadIdx.x & 63;
    // The table and the offsets are read-only for the launch: constant address space,
    // so with a wave-uniform unit index every field is a scalar load.
    const RaggedArgs *probs = (const RaggedArgs *)probs_g;
    const TRAJAM_CONST_AS int *offsets = (const TRAJAM_CONST_AS int *)offsets_g;
    for (;;) {
        int u = 0;
        if (lane == 0) u = atomicAdd(counter, 1);
        u = __builtin_amdgcn_readfirstlane(__shfl(u, 0));
        if (u >= total) break;
        int lo = 0, hi = n_probs;  // largest lo with offsets[lo] <= u
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (offsets[mid] <= u) lo = mid;
            else hi = mid;
        }
        const RaggedArgs &a = probs[lo];
        const int sample = u - offsets[lo];
        const int nvp = a.nv <= 8 ? 8 : 12;
        const int tpl = (a.n_p + 63) >> 6;
        if constexpr (AGENTS) {
            // this wave's LDS slot: the obstacle stage (cull_lds floats, at most the
            // plan's largest), the agents' positions at the slot's end
            float *ol = a.cull_lds ? wl : nullptr;
            float *px = wl + wave_lds - kAgentPosScalars;
            if (a.dims == 2) { if (nvp == 8) agents_sample<float, 2, 8, RaggedArgs>(a, sample, lane, ol, px); else agents_sample<float, 2, 12, RaggedArgs>(a, sample, lane, ol, px); }
            else             { if (nvp == 8) agents_sample<float, 3, 8, RaggedArgs>(a, sample, lane, ol, px); else agents_sample<float, 3, 12, RaggedArgs>(a, sample, lane, ol, px); }
            wave_lds_sync();  // the next unit restages
            continue;
        } else {
        if (a.dims == 2) {
            if (nvp == 8) { if (tpl == 1) ragged_unit<2, 8, 1>(a, sample, lane, wl); else ragged_unit<2, 8, 2>(a, sample, lane, wl); }
            else          { if (tpl == 1) ragged_unit<2, 12, 1>(a, sample, lane, wl); else ragged_unit<2, 12, 2>(a, sample, lane, wl); }
        } else {
            if (nvp == 8) { if (tpl == 1) ragged_unit<3, 8, 1>(a, sample, lane, wl); else ragged_unit<3, 8, 2>(a, sample, lane, wl); }
            else          { if (tpl == 1) ragged_unit<3, 12, 1>(a, sample, lane, wl); else ragged_unit<3, 12, 2>(a, sample, lane, wl); }
        }
        }
    }
}

__global__ void zero_counter_kernel(int *counter) { *counter = 0; }

// Residual only: steps (a) and the residual norms at the given coefficients.
template <typename T, int D, int NVP, int OM>
__global__ __launch_bounds__(kMaxThreads) void am_residual_kernel(AmArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *smem = reinterpret_cast<T *>(smem_raw);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wpt = a.tpad >> 6;
    const int ls = tid / a.tpad;
    const int lt = tid - ls * a.tpad;
    const int sample = blockIdx.x * a.tb + ls;
    const bool valid = sample < a.batch && lt < a.n_p;
    T *r2p = smem;                  // [tb][wpt]
    T *rmp = smem + a.tb * wpt;     // [tb][wpt]
    T p[D], v[D], acc[D];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) { p[ax] = T(0); v[ax] = T(0); acc[ax] = T(0); }
    if (valid) {
        const T *x = a.xb + (size_t)sample * D * a.nv;
        for (int m = 0; m < a.nv; ++m) {
            const T f0 = a.phi[(0 * a.n_p + lt) * NVP + m];
            const T f1 = a.phi[(1 * a.n_p + lt) * NVP + m];
            const T f2 = a.phi[(2 * a.n_p + lt) * NVP + m];
#pragma unroll
            for (int ax = 0; ax < D; ++ax) {
                const T c = x[ax * a.nv + m];
                p[ax] = fma(f0, c, p[ax]);
                v[ax] = fma(f1, c, v[ax]);
                acc[ax] = fma(f2, c, acc[ax]);
            }
        }
    }
    T R[D], rv[D], ra[D], r2 = T(0), rmax = T(0);
#pragma unroll
    for (int ax = 0; ax < D; ++ax) R[ax] = T(0);
    if constexpr (OM == kObsStatic) {
        // static obstacles: the projection's culled loop (few candidates per wave),
        // called by every lane of the wave, lanes without a point passing one far away
        const ObsChunk<T, D> oc0 = load_obs_chunk<T, D>(a.obs, a.n_o, 0, lane);
        CullCache<T, D, 1> cc;
        const T tt1[1] = {T(lt) * a.dt};
        const bool ok1[1] = {valid};
        T p1[1][D], R1[1][D];
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            p1[0][ax] = valid ? p[ax] : T(-1e30);
            R1[0][ax] = T(0);
        }
        obstacle_residuals_culled<T, D, 1, kObsStatic>(a.obs, a.n_o, a.sphere, 0, oc0, tt1, p1, ok1, R1, r2, rmax,
                                                       cc);
#pragma unroll
        for (int ax = 0; ax < D; ++ax) R[ax] = R1[0][ax];
    } else {
        // moving obstacles swept over a wave's time range leave most of them candidates:
        // every obstacle is tested from its fields in scalar registers instead
        if (valid) obstacle_residuals1<T, D>(a.obs_soa, a.obs, a.n_o, a.sphere, a.dynamic, T(lt) * a.dt, p, R, r2, rmax);
    }
    if (valid) {
        if (a.use_v) bound_residual<T, D>(v, a.vmax, rv, r2, rmax);
        if (a.use_a) bound_residual<T, D>(acc, a.amax, ra, r2, rmax);
        if (a.use_ws) workspace_residual(p, a.ws_lo, a.ws_hi, R, r2, rmax);
    }
    const T s = wave_sum(r2);
    const T mx = wave_max(rmax);
    if (lane == 0) {
        r2p[ls * wpt + (lt >> 6)] = s;
        rmp[ls * wpt + (lt >> 6)] = mx;
    }
    __syncthreads();
    if (lt == 0 && sample < a.batch) {
        T rs = T(0), rm = T(0);
        for (int w = 0; w < wpt; ++w) {
            rs += r2p[ls * wpt + w];
            rm = fmax(rm, rmp[ls * wpt + w]);
        }
        a.res[sample] = sqrt(rs);
        if (a.res_max) a.res_max[sample] = rm;
    }
}

// Packs the caller's obstacle arrays.  (1) One 16-slot record per obstacle:
// centre[3], -velocity[3], 1/semi-axes[3], semi-axes[3], -radius^2, radius (radius =
// first semi-axis, used by the sphere model).  (2) The inside-test fields in groups of
// kGroupStore obstacles, field-major: centre[3], -velocity[3], 1/semi-axes[3],
// -radius^2.  Slots past n_o hold a sentinel (centre 1e30, unit scale, zero radius)
// whose test value is +inf or huge, so it is never inside.
template <typename T, int D>
__global__ void pack_obstacles_kernel(int n_o, int n_pad, const T *__restrict__ c,
                                      const T *__restrict__ w, const T *__restrict__ s,
                                      T *__restrict__ out, T *__restrict__ soa)
{
    constexpr int REC = kObstacleRecord;
    constexpr int GS = kGroupStore<T>;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_pad) return;
    T f[kObstacleFields];
    if (j < n_o) {
        T *o = out + (size_t)j * REC;
#pragma unroll
        for (int i = 0; i < REC; ++i) o[i] = T(0);
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            o[kOC + ax] = c[j * D + ax];
            o[kOW + ax] = w ? -w[j * D + ax] : T(0);
            o[kOI + ax] = T(1) / s[j * D + ax];
            o[kOS + ax] = s[j * D + ax];
        }
        o[kONR2] = -s[j * D] * s[j * D];
        o[kOR] = s[j * D];
#pragma unroll
        for (int i = 0; i < kObstacleFields; ++i) f[i] = T(0);
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            f[kFCX + ax] = o[kOC + ax];
            f[kFWX + ax] = o[kOW + ax];
            f[kFIX + ax] = o[kOI + ax];
        }
        f[kFNR2] = o[kONR2];
    } else {
#pragma unroll
        for (int i = 0; i < kObstacleFields; ++i) f[i] = T(0);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            f[kFCX + ax] = T(1e30);
            f[kFIX + ax] = T(1);
        }
    }
    const int g = j / GS, u = j - g * GS;
#pragma unroll
    for (int i = 0; i < kObstacleFields; ++i) soa[((size_t)g * kObstacleFields + i) * GS + u] = f[i];
}

template <typename T, int D, int NVP, bool MQP>
hipError_t launch_project_t(const AmArgs<T> &a, hipStream_t st)
{
    using L = Lds<D, NVP>;
    const int wpt = a.tpad / 64;
    const size_t lds = sizeof(T) * (size_t)L::total(a.tb, wpt) + (MQP ? sizeof(float) * kMqFloats : 0);
    const int threads = a.tb * a.tpad;
    const int blocks = (a.batch + a.tb - 1) / a.tb;
    if (a.tb < 1 || threads > kMaxThreads) return hipErrorInvalidValue;
    if (MQP && (a.tb * D > 16 || a.nv - 4 > 16)) return hipErrorInvalidValue;
    // separate instances for static and moving obstacles: each carries one obstacle loop
    if (a.dynamic)
        hipLaunchKernelGGL((am_project_kernel<T, D, NVP, MQP, kObsMoving>), dim3(blocks), dim3(threads), lds, st, a);
    else
        hipLaunchKernelGGL((am_project_kernel<T, D, NVP, MQP, kObsStatic>), dim3(blocks), dim3(threads), lds, st, a);
    return hipGetLastError();
}
template <typename T, int D, int NVP, bool MQP>
hipError_t launch_wave_t(const AmArgs<T> &a, hipStream_t st)
{
    const size_t lds = sizeof(T) * (size_t)(NVP * NVP + a.tb * 2 * D * NVP) +
                       (MQP ? sizeof(float) * (size_t)(a.tb * 256 + 320) : 0);
    const int threads = a.tb * 64;
    const int blocks = (a.batch + a.tb - 1) / a.tb;
    const int tpl = (a.n_p + 63) / 64;
    if (a.tb < 1 || threads > kMaxThreads) return hipErrorInvalidValue;
#define TRAJAM_WAVE_LAUNCH(OMV)                                                                                 \
    switch (tpl) {                                                                                             \
    case 1: hipLaunchKernelGGL((am_wave_kernel<T, D, NVP, 1, MQP, OMV>), dim3(blocks), dim3(threads), lds, st, a); break; \
    case 2: hipLaunchKernelGGL((am_wave_kernel<T, D, NVP, 2, MQP, OMV>), dim3(blocks), dim3(threads), lds, st, a); break; \
    case 3: hipLaunchKernelGGL((am_wave_kernel<T, D, NVP, 3, MQP, OMV>), dim3(blocks), dim3(threads), lds, st, a); break; \
    case 4: hipLaunchKernelGGL((am_wave_kernel<T, D, NVP, 4, MQP, OMV>), dim3(blocks), dim3(threads), lds, st, a); break; \
    default: return hipErrorInvalidValue;                                                                      \
    }
    if (a.dynamic) {
        TRAJAM_WAVE_LAUNCH(kObsMoving)
    } else {
        TRAJAM_WAVE_LAUNCH(kObsStatic)
    }
#undef TRAJAM_WAVE_LAUNCH
    return hipGetLastError();
}
template <typename T, int D, int NVP>
hipError_t launch_wave_plain(const AmArgs<T> &a, hipStream_t st) { return launch_wave_t<T, D, NVP, false>(a, st); }
template <typename T, int D, int NVP>
hipError_t launch_wave_mqp(const AmArgs<T> &a, hipStream_t st) { return launch_wave_t<T, D, NVP, true>(a, st); }
template <typename T, int D, int NVP>
hipError_t launch_project_plain(const AmArgs<T> &a, hipStream_t st) { return launch_project_t<T, D, NVP, false>(a, st); }
template <typename T, int D, int NVP>
hipError_t launch_project_mqp(const AmArgs<T> &a, hipStream_t st) { return launch_project_t<T, D, NVP, true>(a, st); }

template <typename T, int D, int NVP>
hipError_t launch_residual_t(const AmArgs<T> &a, hipStream_t st)
{
    const int wpt = a.tpad / 64;
    const size_t lds = sizeof(T) * 2 * (size_t)a.tb * wpt;
    const int threads = a.tb * a.tpad;
    const int blocks = (a.batch + a.tb - 1) / a.tb;
    if (a.tb < 1 || threads > kMaxThreads) return hipErrorInvalidValue;
    if (a.dynamic)
        hipLaunchKernelGGL((am_residual_kernel<T, D, NVP, kObsMoving>), dim3(blocks), dim3(threads), lds, st, a);
    else
        hipLaunchKernelGGL((am_residual_kernel<T, D, NVP, kObsStatic>), dim3(blocks), dim3(threads), lds, st, a);
    return hipGetLastError();
}


template <typename T, template <typename, int, int> class F>
struct Dispatch;

#define TRAJAM_DISPATCH(FN, T, dims, nvp, ...)                                          \
    do {                                                                                \
        if ((dims) == 2) {                                                              \
            if ((nvp) == 8) return FN<T, 2, 8>(__VA_ARGS__);                            \
            if ((nvp) == 12) return FN<T, 2, 12>(__VA_ARGS__);                          \
            if ((nvp) == 16) return FN<T, 2, 16>(__VA_ARGS__);                          \
        } else if ((dims) == 3) {                                                       \
            if ((nvp) == 8) return FN<T, 3, 8>(__VA_ARGS__);                            \
            if ((nvp) == 12) return FN<T, 3, 12>(__VA_ARGS__);                          \
            if ((nvp) == 16) return FN<T, 3, 16>(__VA_ARGS__);                          \
        }                                                                               \
        return hipErrorInvalidValue;                                                    \
    } while (0)

}  // namespace

template <typename T>
hipError_t launch_agents_t(int dims, int nvp, const AmArgs<T> &a, bool residual, hipStream_t st)
{
    if (a.batch <= 0) return hipSuccess;
    if (a.n_agents < 1 || a.n_agents > 64 || a.tb < 1 || a.tb > kMaxThreads / 64) return hipErrorInvalidValue;
    // the obstacle stages of a workgroup's waves stay within 64 KiB of LDS
    if (a.cull_lds < 0 || (size_t)a.cull_lds * sizeof(T) * a.tb > (size_t)kStageMaxFloats * sizeof(float) * 4)
        return hipErrorInvalidValue;
    const dim3 grid((a.batch + a.tb - 1) / a.tb), block(64 * a.tb);
    const size_t lds = sizeof(T) * (size_t)(a.cull_lds + kAgentPosScalars) * a.tb;
#define TRAJAM_AGENTS(DD, NN)                                                                            \
    if (dims == DD && nvp == NN) {                                                                       \
        if (residual) hipLaunchKernelGGL((am_agents_residual_kernel<T, DD, NN>), grid, block, lds, st, a); \
        else hipLaunchKernelGGL((am_agents_kernel<T, DD, NN>), grid, block, lds, st, a);                   \
        return hipGetLastError();                                                                        \
    }
    TRAJAM_AGENTS(2, 8)
    TRAJAM_AGENTS(2, 12)
    TRAJAM_AGENTS(3, 8)
    TRAJAM_AGENTS(3, 12)
#undef TRAJAM_AGENTS
    return hipErrorInvalidValue;
}

hipError_t launch_agents_f64(int dims, int nvp, const AmArgs<double> &a, hipStream_t st)
{
    return launch_agents_t<double>(dims, nvp, a, false, st);
}
hipError_t launch_agents_f32(int dims, int nvp, const AmArgs<float> &a, hipStream_t st)
{
    return launch_agents_t<float>(dims, nvp, a, false, st);
}
hipError_t launch_agents_residual_f64(int dims, int nvp, const AmArgs<double> &a, hipStream_t st)
{
    return launch_agents_t<double>(dims, nvp, a, true, st);
}
hipError_t launch_agents_residual_f32(int dims, int nvp, const AmArgs<float> &a, hipStream_t st)
{
    return launch_agents_t<float>(dims, nvp, a, true, st);
}

hipError_t launch_ragged(const AmArgs<float> *probs, const int *offsets, int n_probs, int total, int *counter,
                         int blocks, bool agents, int agent_stage, hipStream_t st)
{
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, st, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (agents) {
        if (agent_stage < 0 || agent_stage > kStageMaxFloats) return hipErrorInvalidValue;
        const int wave_lds = agent_stage + kAgentPosScalars;
        const size_t lds = sizeof(float) * (size_t)wave_lds * (kMaxThreads / 64);
        hipLaunchKernelGGL(am_ragged_kernel<true>, dim3(blocks), dim3(kMaxThreads), lds, st, probs, offsets, n_probs,
                           total, counter, wave_lds);
    } else {
        const size_t lds = sizeof(float) * (size_t)kRaggedWaveLds * (kMaxThreads / 64);
        hipLaunchKernelGGL(am_ragged_kernel<false>, dim3(blocks), dim3(kMaxThreads), lds, st, probs, offsets,
                           n_probs, total, counter, kRaggedWaveLds);
    }
    return hipGetLastError();
}

size_t project_lds_bytes(int dims, int nvp, int tpad, int tb, size_t scalar)
{
    const int S = dims * nvp;
    const int V = pow2ceil(S);
    const int wpt = tpad / 64;
    return scalar * (size_t)(3 * tb * S + tb * wpt * V + tb * wpt + nvp * nvp);
}

hipError_t launch_project_f64(int dims, int nvp, int variant, const AmArgs<double> &a,
                              hipStream_t st)
{
    if (variant == kVariantWave) TRAJAM_DISPATCH(launch_wave_plain, double, dims, nvp, a, st);
    TRAJAM_DISPATCH(launch_project_plain, double, dims, nvp, a, st);
}

hipError_t launch_project_f32(int dims, int nvp, int variant, bool mfma_qp, const AmArgs<float> &a,
                              hipStream_t st)
{
    if (variant == kVariantWave) {
        if (mfma_qp) TRAJAM_DISPATCH(launch_wave_mqp, float, dims, nvp, a, st);
        TRAJAM_DISPATCH(launch_wave_plain, float, dims, nvp, a, st);
    }
    if (mfma_qp) TRAJAM_DISPATCH(launch_project_mqp, float, dims, nvp, a, st);
    TRAJAM_DISPATCH(launch_project_plain, float, dims, nvp, a, st);
}

hipError_t launch_residual_f64(int dims, int nvp, const AmArgs<double> &a, hipStream_t st)
{
    TRAJAM_DISPATCH(launch_residual_t, double, dims, nvp, a, st);
}

hipError_t launch_residual_f32(int dims, int nvp, const AmArgs<float> &a, hipStream_t st)
{
    TRAJAM_DISPATCH(launch_residual_t, float, dims, nvp, a, st);
}


template <typename T>
static hipError_t pack_t(int dims, int n_o, const T *c, const T *w, const T *s, T *out, T *soa,
                         hipStream_t st)
{
    if (n_o <= 0) return hipSuccess;
    const int n_pad = obstacle_groups(n_o, sizeof(T)) * (int)group_store(sizeof(T));
    const int threads = 64, blocks = (n_pad + threads - 1) / threads;
    if (dims == 2)
        hipLaunchKernelGGL((pack_obstacles_kernel<T, 2>), dim3(blocks), dim3(threads), 0, st, n_o,
                           n_pad, c, w, s, out, soa);
    else
        hipLaunchKernelGGL((pack_obstacles_kernel<T, 3>), dim3(blocks), dim3(threads), 0, st, n_o,
                           n_pad, c, w, s, out, soa);
    return hipGetLastError();
}

hipError_t launch_pack_obstacles_f64(int dims, int n_o, const double *c, const double *w,
                                     const double *s, double *out, double *soa, hipStream_t st)
{
    return pack_t<double>(dims, n_o, c, w, s, out, soa, st);
}

hipError_t launch_pack_obstacles_f32(int dims, int n_o, const float *c, const float *w,
                                     const float *s, float *out, float *soa, hipStream_t st)
{
    return pack_t<float>(dims, n_o, c, w, s, out, soa, st);
}

}  // namespace trajam
