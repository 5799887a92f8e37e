// gfx950 kernel of the materialised polar variables (trajam_polar): alpha, beta, d of
// every (sample, obstacle, time step) and the kinematic blocks' polar variables,
// written to HBM as unpadded rows.  Bound by the HBM write stream and the per-element
// VALU work (two arctangents in 3D).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "am_internal.h"

namespace trajam {
namespace {

// Angle and norm of the materialised polar variables.  FP32: atan2 from the ratio of
// the smaller to the larger magnitude (in [0, 1]), its arctangent by an odd polynomial
// a P(a^2) whose coefficients were fitted for this kernel (least squares on Chebyshev
// nodes reweighted towards equal ripple on [0, 1]; in float arithmetic the largest
// error on [0, 1] is 1.3e-7 rad with a correctly rounded reciprocal and 1.9e-7 with
// the hardware reciprocal's 1-ulp error), then the octant and quadrant corrections
// (rounding pi - r to float: at most 3.7e-7 rad over the whole circle) and the sign
// of y (so atan2(-0, x < 0) = -pi, as IEEE atan2).  The larger magnitude is kept at
// least FLT_MIN, so atan2(0, 0) = 0 without a branch (vectors shorter than FLT_MIN,
// i.e. denormal, get the angle of a distorted ratio).  The square root is the
// hardware one (1 ulp).  FP64: the library functions.
__device__ __forceinline__ float polar_atan_poly(float a)
{
    const float s = a * a;
    float q = -0.004054564982652664f;
    q = fmaf(q, s, 0.021862955763936043f);
    q = fmaf(q, s, -0.055912334471940994f);
    q = fmaf(q, s, 0.0964219868183136f);
    q = fmaf(q, s, -0.1390863060951233f);
    q = fmaf(q, s, 0.19946566224098206f);
    q = fmaf(q, s, -0.33329859375953674f);
    q = fmaf(q, s, 0.9999993443489075f);
    return a * q;
}
// atan2(y, x) for y >= 0 (no sign step): the polar angle beta in [0, pi]
__device__ __forceinline__ float polar_atan2_up(float y, float x)
{
    const float ax = fabsf(x);
    const float a = fminf(ax, y) * __builtin_amdgcn_rcpf(fmaxf(fmaxf(ax, y), 1.17549435e-38f));
    float r = polar_atan_poly(a);
    r = y > ax ? 1.5707963267948966f - r : r;
    return x < 0.f ? 3.14159265358979323f - r : r;
}
__device__ __forceinline__ float polar_atan2(float y, float x)
{
    return __builtin_copysignf(polar_atan2_up(fabsf(y), x), y);
}
__device__ __forceinline__ double polar_atan2_up(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ double polar_atan2(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ float polar_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double polar_sqrt(double x) { return sqrt(x); }

// Raw buffer stores: a per-workgroup base in scalar registers, a 32-bit lane offset,
// and the hardware's bounds check (an offset at or past num_records, a negative one
// included, is dropped), non-temporal (written once, never read back here).
constexpr int kBufferWord3 = 0x00020000;  // raw buffer, 32-bit data (gfx9 family)
constexpr int kNonTemporal = 2;           // cache-policy bit NT
struct RowStore {
    __amdgpu_buffer_rsrc_t r;
    bool on;
};
__device__ __forceinline__ RowStore row_store(void *base, unsigned bytes)
{
    RowStore s;
    s.on = base != nullptr;
    s.r = __builtin_amdgcn_make_buffer_rsrc(s.on ? base : (void *)nullptr, (short)0, (int)bytes, kBufferWord3);
    return s;
}
__device__ __forceinline__ void put(const RowStore &s, float v, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), s.r, (int)off, 0, kNonTemporal);
}
typedef unsigned polar_u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void put(const RowStore &s, double v, unsigned off)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const polar_u32x2 w = {(unsigned)b, (unsigned)(b >> 32)};
    __builtin_amdgcn_raw_buffer_store_b64(w, s.r, (int)off, 0, kNonTemporal);
}

// Materialised polar variables at given coefficients, as unpadded rows
// [batch][n_o][n_p] (eqs comp_alpha, comp_beta, comp_d, with the angles taken in
// semi-axis-scaled coordinates): per (obstacle, time step) alpha = atan2(u_y, u_x),
// beta = atan2(|u_xy|, u_z) (pi/2 in 2D) and d = max(1, |u|) of u = (p(t) - c(t)) ./ s,
// and per time step the kinematic blocks' (alpha, beta, min(1, |v| / bound))
// (eqs alpha_v, compute_dv, alpha_a, compute_da) as [batch][6][n_p].
// Grid (batch, parts): the `parts` workgroups of a sample each take a contiguous range
// [e0, e1) of its n_o * n_p elements.  A workgroup first maps the sample's coefficients
// to (p(t), t) records in LDS (part 0 also writes the kinematic rows) and stages one
// record per obstacle (centre, -velocity, 1 / semi-axis; 1 / radius on every axis for
// the sphere model) in LDS when they fit.  Then its threads stride through the range,
// consecutive lanes taking consecutive elements and four elements a pass (their LDS
// reads overlap).  The lanes are laid on the outputs' global element index so that
// each wave's store covers 64 elements starting on a multiple of 64 -- whole cache
// lines, whatever row or sample they belong to -- and the lanes that fall outside the
// range (at most one partial chunk at each end) are dropped by the buffer stores'
// bounds check.  Each thread tracks its (obstacle, step) pair incrementally.
template <typename T, int D>
struct PolarLds {
    static constexpr int kPos = 4;                  // p[D], t (and a pad in 2D)
    static constexpr int kObs = D == 3 ? 12 : 8;    // c[D], -w[D], 1/s[D], pads
};

template <typename T, int D, bool STAGED>
__device__ __forceinline__ void polar_fields(const T *of, const AmArgs<T> &a, int j, int sc, T (&c)[D], T (&w)[D],
                                             T (&is)[D])
{
    if constexpr (STAGED) {
        const T *o = of + j * PolarLds<T, D>::kObs;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            c[ax] = o[ax];
            w[ax] = o[D + ax];
            is[ax] = o[2 * D + ax];
        }
    } else {
        const T *o = a.obs + (size_t)j * kObstacleRecord;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            c[ax] = o[kOC + ax];
            w[ax] = o[kOW + ax];
            is[ax] = o[kOI + sc * ax];
        }
    }
}

template <typename T, int D>
__device__ __forceinline__ void polar_element(const T (&c)[D], const T (&w)[D], const T (&is)[D], const T *pr,
                                              unsigned off, const RowStore &sal, const RowStore &sbe,
                                              const RowStore &sdd)
{
    const T tt = pr[3];
    T u[D];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) u[ax] = fma(w[ax], tt, pr[ax] - c[ax]) * is[ax];
    const T rxy2 = fma(u[1], u[1], u[0] * u[0]);
    const T nn = D == 3 ? fma(u[D - 1], u[D - 1], rxy2) : rxy2;
    if (sal.on) put(sal, polar_atan2(u[1], u[0]), off);
    if (sbe.on) put(sbe, D == 3 ? polar_atan2_up(polar_sqrt(rxy2), u[D - 1]) : T(1.5707963267948966), off);
    if (sdd.on) put(sdd, fmax(polar_sqrt(nn), T(1)), off);
}

template <typename T, int D, int NVP, bool STAGED>
__global__ __launch_bounds__(512) void am_polar_kernel(AmArgs<T> a, int per_part, T *__restrict__ oal,
                                                       T *__restrict__ obe, T *__restrict__ odd,
                                                       T *__restrict__ kin)
{
    using L = PolarLds<T, D>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *pos = reinterpret_cast<T *>(smem_raw);   // [n_p][kPos]: p(t), t
    T *of = pos + L::kPos * a.n_p + L::kObs;    // STAGED: [-1 .. n_o - 1][kObs] (record -1 is zero)
    const int sample = blockIdx.x, part = blockIdx.y;
    const int n_p = a.n_p, n_o = a.n_o;
    const T half_pi = T(1.5707963267948966);
    const T *x = a.xb + (size_t)sample * D * a.nv;
    const bool do_kin = kin && part == 0;
    // this sample's coefficients (zero past n_v, like the basis rows)
    T xc[D][NVP];
#pragma unroll
    for (int ax = 0; ax < D; ++ax)
#pragma unroll
        for (int m = 0; m < NVP; ++m) xc[ax][m] = m < a.nv ? x[ax * a.nv + m] : T(0);
    for (int t = threadIdx.x; t < n_p; t += blockDim.x) {
        T q[3][D];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int ax = 0; ax < D; ++ax) q[k][ax] = T(0);
            if (k > 0 && !do_kin) continue;
            const T *ph = a.phi + ((size_t)k * n_p + t) * NVP;
#pragma unroll
            for (int m = 0; m < NVP; ++m) {
                const T f = ph[m];
#pragma unroll
                for (int ax = 0; ax < D; ++ax) q[k][ax] = fma(f, xc[ax][m], q[k][ax]);
            }
        }
        T *pr = pos + t * L::kPos;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) pr[ax] = q[0][ax];
        if (D == 2) pr[2] = T(0);
        pr[3] = T(t) * a.dt;
        if (do_kin) {
            T *kr = kin + (size_t)sample * 6 * n_p;
#pragma unroll
            for (int k = 1; k < 3; ++k) {
                const T bound = k == 1 ? a.vmax : a.amax;
                T al = T(0), be = T(0), dv = T(0);
                if (bound > T(0)) {
                    T nn = T(0);
#pragma unroll
                    for (int ax = 0; ax < D; ++ax) nn = fma(q[k][ax], q[k][ax], nn);
                    al = polar_atan2(q[k][1], q[k][0]);
                    be = D == 3 ? polar_atan2_up(polar_sqrt(fma(q[k][0], q[k][0], q[k][1] * q[k][1])), q[k][D - 1])
                                : half_pi;
                    dv = fmin(polar_sqrt(nn) / bound, T(1));
                }
                kr[(3 * (k - 1) + 0) * n_p + t] = al;
                kr[(3 * (k - 1) + 1) * n_p + t] = be;
                kr[(3 * (k - 1) + 2) * n_p + t] = dv;
            }
        }
    }
    if (!oal && !obe && !odd) return;
    // the sphere model scales every axis by 1 / radius (the first semi-axis; the
    // caller's other entries are ignored and may be anything, zero included)
    const int sc = a.sphere ? 0 : 1;
    if constexpr (STAGED) {
        if (threadIdx.x < L::kObs) of[(int)threadIdx.x - L::kObs] = T(0);
        for (int j = threadIdx.x; j < n_o; j += blockDim.x) {
            const T *o = a.obs + (size_t)j * kObstacleRecord;
            T *d = of + j * L::kObs;
#pragma unroll
            for (int ax = 0; ax < D; ++ax) {
                d[ax] = o[kOC + ax];
                d[D + ax] = o[kOW + ax];
                d[2 * D + ax] = o[kOI + sc * ax];
            }
#pragma unroll
            for (int k = 3 * D; k < L::kObs; ++k) d[k] = T(0);
        }
    }
    __syncthreads();
    const int total = n_o * n_p;
    const int e0 = part * per_part, e1 = min(total, e0 + per_part);
    const size_t g0 = (size_t)sample * total + e0;   // global element index of e0
    const unsigned bytes = (unsigned)(sizeof(T) * (size_t)(e1 - e0));
    const RowStore sal = row_store(oal ? oal + g0 : nullptr, bytes);
    const RowStore sbe = row_store(obe ? obe + g0 : nullptr, bytes);
    const RowStore sdd = row_store(odd ? odd + g0 : nullptr, bytes);
    // first pass starts at the multiple of 64 (global index) at or below e0; lanes
    // before e0 (negative offsets) or at / past e1 are dropped by the bounds check
    const int step = blockDim.x, qj = step / n_p, qt = step - qj * n_p;
    int e = e0 - (int)(g0 & 63) + threadIdx.x;
    int j, t;
    if (e >= 0) {
        j = e / n_p;
        t = e - j * n_p;
    } else {   // floor division for the lanes before the sample's first element
        j = -1 - (-e - 1) / n_p;
        t = e - j * n_p;
    }
    auto advance = [&](int &jj, int &tv) {
        tv += qt;
        jj += qj;
        if (tv >= n_p) {
            tv -= n_p;
            ++jj;
        }
    };
    // the dropped lanes before e0 read obstacle -1 (a zero record in LDS; clamped for
    // the packed records); elements below e1 have obstacles below n_o
    auto jc = [&](int jj) { return STAGED ? jj : max(jj, 0); };
    constexpr int U = 4;
    for (; e + (U - 1) * step < e1; e += U * step) {
        int jj[U], tv[U];
        jj[0] = j;
        tv[0] = t;
#pragma unroll
        for (int u = 1; u < U; ++u) {
            jj[u] = jj[u - 1];
            tv[u] = tv[u - 1];
            advance(jj[u], tv[u]);
        }
        T c[U][D], w[U][D], is[U][D], pr[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            polar_fields<T, D, STAGED>(of, a, jc(jj[u]), sc, c[u], w[u], is[u]);
#pragma unroll
            for (int k = 0; k < 4; ++k) pr[u][k] = pos[tv[u] * L::kPos + k];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            polar_element<T, D>(c[u], w[u], is[u], pr[u], (unsigned)((e + u * step - e0) * (int)sizeof(T)), sal,
                                sbe, sdd);
        j = jj[U - 1];
        t = tv[U - 1];
        advance(j, t);
    }
    for (; e < e1; e += step) {
        T c[D], w[D], is[D], pr[4];
        polar_fields<T, D, STAGED>(of, a, jc(j), sc, c, w, is);
#pragma unroll
        for (int k = 0; k < 4; ++k) pr[k] = pos[t * L::kPos + k];
        polar_element<T, D>(c, w, is, pr, (unsigned)((e - e0) * (int)sizeof(T)), sal, sbe, sdd);
        advance(j, t);
    }
}

template <typename T, int D, int NVP>
hipError_t launch_polar_t(const AmArgs<T> &a, void *al, void *be, void *dd, void *kin, hipStream_t st)
{
    using L = PolarLds<T, D>;
    constexpr int kThreads = 512;   // measured: 512 > 256 > 1024 > 128 threads at config 3
    // obstacle records in LDS up to 48 KiB (with the p(t) records); read from the
    // packed records beyond
    const size_t pos_bytes = sizeof(T) * (L::kPos * (size_t)a.n_p + L::kObs);   // + the zero record
    const size_t obs_bytes = sizeof(T) * L::kObs * (size_t)a.n_o;
    const bool staged = pos_bytes + obs_bytes <= 48 * 1024;
    const size_t lds = pos_bytes + (staged ? obs_bytes : 0);
    // enough workgroups to fill the chip (>= 4096 in all), each with at least 16
    // elements a thread, so p(t) and the obstacle stage are amortised
    const long total = (long)a.n_o * a.n_p;
    long parts = (4096 + a.batch - 1) / a.batch;
    const long max_parts = std::max(1L, total / (16L * kThreads));
    parts = std::max(1L, std::min(parts, max_parts));
    const int per_part = (int)((total + parts - 1) / parts);
    const dim3 grid(a.batch, (unsigned)parts);
    if (staged)
        hipLaunchKernelGGL((am_polar_kernel<T, D, NVP, true>), grid, dim3(kThreads), lds, st, a, per_part, (T *)al,
                           (T *)be, (T *)dd, (T *)kin);
    else
        hipLaunchKernelGGL((am_polar_kernel<T, D, NVP, false>), grid, dim3(kThreads), lds, st, a, per_part,
                           (T *)al, (T *)be, (T *)dd, (T *)kin);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch_polar(int dims, int nvp, const AmArgs<T> &a, void *al, void *be, void *dd, void *kin,
                          hipStream_t st)
{
    if (dims == 2) {
        if (nvp == 8) return launch_polar_t<T, 2, 8>(a, al, be, dd, kin, st);
        if (nvp == 12) return launch_polar_t<T, 2, 12>(a, al, be, dd, kin, st);
        if (nvp == 16) return launch_polar_t<T, 2, 16>(a, al, be, dd, kin, st);
    } else if (dims == 3) {
        if (nvp == 8) return launch_polar_t<T, 3, 8>(a, al, be, dd, kin, st);
        if (nvp == 12) return launch_polar_t<T, 3, 12>(a, al, be, dd, kin, st);
        if (nvp == 16) return launch_polar_t<T, 3, 16>(a, al, be, dd, kin, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_polar_f64(int dims, int nvp, const AmArgs<double> &a, void *al, void *be, void *dd, void *kin,
                            hipStream_t st)
{
    return dispatch_polar<double>(dims, nvp, a, al, be, dd, kin, st);
}

hipError_t launch_polar_f32(int dims, int nvp, const AmArgs<float> &a, void *al, void *be, void *dd, void *kin,
                            hipStream_t st)
{
    return dispatch_polar<float>(dims, nvp, a, al, be, dd, kin, st);
}

}  // namespace trajam
