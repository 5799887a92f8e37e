// gfx950 kernels of the projection-guided sampling loop (thesis ch. 6, Alg 3):
// Gaussian sampling from (mu, L), the augmented cost and residual key, top-k
// selection by rank with lexicographic keys, and the weighted mean / covariance
// update (eqs update_mean, update_covariance) with the Cholesky factor
// for the next draw.  The projection between sampling and cost is the AM kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "am_internal.h"

namespace trajam {
namespace {

// xi[i][r] = mu[r] + sum_{c <= r} L[r][c] z[i][c]; optionally the cold start of the
// projection, xb = xi and lam = 0, from the same thread.
template <typename T>
__global__ void cem_sample_kernel(int n, int dim, const T *__restrict__ mu,
                                  const T *__restrict__ L, const T *__restrict__ z,
                                  T *__restrict__ xi, T *__restrict__ xb, T *__restrict__ lam)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n * dim) return;
    const int i = gid / dim, r = gid - (gid / dim) * dim;
    T acc = mu[r];
    for (int c = 0; c <= r; ++c) acc = fma(L[r * dim + c], z[(size_t)i * dim + c], acc);
    xi[gid] = acc;
    if (xb) xb[gid] = acc;
    if (lam) lam[gid] = T(0);
}

template <typename T>
__device__ __forceinline__ T wave_sum64(T v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// One wave per sample: c_1 = sum_t |Pdd xb(t)|^2, c_aug = c_1 + r, and the residual
// key floor(r / quantum) (clamped to int32).
template <typename T>
__global__ void cem_cost_kernel(int n, int dims, int nv, int n_p, int nvp,
                                const T *__restrict__ pdd, const T *__restrict__ xb,
                                const T *__restrict__ res, T inv_quantum, T *__restrict__ caug,
                                int32_t *__restrict__ rkey)
{
    const int wv = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wv >= n) return;
    const T *x = xb + (size_t)wv * dims * nv;
    T acc = T(0);
    for (int t = lane; t < n_p; t += 64)
        for (int ax = 0; ax < dims; ++ax) {
            T a = T(0);
            for (int m = 0; m < nv; ++m) a = fma(pdd[(size_t)t * nvp + m], x[ax * nv + m], a);
            acc = fma(a, a, acc);
        }
    acc = wave_sum64(acc);
    if (lane == 0) {
        const T r = res[wv];
        caug[wv] = acc + r;
        const T q = floor(r * inv_quantum);
        rkey[wv] = q >= T(2147483647) ? 2147483647 : (int32_t)q;
    }
}

// Order-preserving unsigned images of the sort keys: a < b as numbers iff
// ord(a) < ord(b).  -0 maps to +0 and every NaN to the largest image, so NaNs sort
// after +inf and tie among themselves (then by index), as a stable lexicographic
// sort of the numbers does.
__device__ __forceinline__ uint32_t ord_key(int32_t v) { return (uint32_t)v ^ 0x80000000u; }

__device__ __forceinline__ uint64_t ord_key(float v)
{
    if (v != v) return 0xffffffffull;
    const uint32_t b = __float_as_uint(v == 0.f ? 0.f : v);
    return (b & 0x80000000u) ? (uint64_t)(~b) : (uint64_t)(b | 0x80000000u);
}

__device__ __forceinline__ uint64_t ord_key(double v)
{
    if (v != v) return ~0ull;
    const uint64_t b = (uint64_t)__double_as_longlong(v == 0.0 ? 0.0 : v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

constexpr int kRankThreads = 256, kRankSub = 16, kRankPerBlock = kRankThreads / kRankSub;

// Selection by rank.  Keys are unique (the index breaks every tie), so the rank of
// element i, the number of keys below its key, is its position in the sorted order;
// an element whose rank is below n_keep writes its index to out[rank].  Every block
// stages all n keys in LDS and ranks kRankPerBlock elements, kRankSub threads per
// element each counting a strided slice of the keys.
//   SUBSET = false: element i has key (rkey[i], caug[i], i).
//   SUBSET = true : element e is list[e] with key (caug[list[e]], list[e]).
template <typename T, bool SUBSET>
__global__ __launch_bounds__(kRankThreads) void cem_rank_kernel(int n, const int32_t *__restrict__ rkey,
                                                               const T *__restrict__ caug,
                                                               const int32_t *__restrict__ list, int n_keep,
                                                               int32_t *__restrict__ out)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    uint64_t *k2 = reinterpret_cast<uint64_t *>(smem_raw);   // [n] caug image
    uint32_t *k1 = reinterpret_cast<uint32_t *>(k2 + n);     // [n] rkey image, or the index
#pragma unroll 4
    for (int j = threadIdx.x; j < n; j += kRankThreads) {
        if (SUBSET) {
            const int32_t p = list[j];
            k2[j] = ord_key(caug[p]);
            k1[j] = (uint32_t)p;
        } else {
            k2[j] = ord_key(caug[j]);
            k1[j] = ord_key(rkey[j]);
        }
    }
    __syncthreads();
    const int e = blockIdx.x * kRankPerBlock + (int)(threadIdx.x / kRankSub);
    const int sub = threadIdx.x & (kRankSub - 1);
    const int ee = e < n ? e : n - 1;
    const uint32_t a1 = k1[ee];
    const uint64_t a2 = k2[ee];
    int cnt = 0;
#pragma unroll 4
    for (int j = sub; j < n; j += kRankSub) {
        const uint32_t b1 = k1[j];
        const uint64_t b2 = k2[j];
        bool lt;
        if (SUBSET) lt = b2 < a2 || (b2 == a2 && b1 < a1);            // (caug, index)
        else lt = b1 < a1 || (b1 == a1 && (b2 < a2 || (b2 == a2 && j < ee)));  // (rkey, caug, index)
        cnt += lt ? 1 : 0;
    }
#pragma unroll
    for (int off = kRankSub / 2; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
    if (sub == 0 && e < n && cnt < n_keep) out[cnt] = SUBSET ? (int32_t)a1 : e;
}

enum class Red { kSum, kMin };

template <typename T>
__device__ __forceinline__ T red_op(T a, T b, Red op) { return op == Red::kMin ? fmin(a, b) : a + b; }

// Workgroup-wide sum or minimum; every thread gets the result.
template <typename T>
__device__ T block_reduce(T v, T *scratch, Red op)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = red_op(v, __shfl_xor(v, off), op);
    __syncthreads();
    if (lane == 0) scratch[wv] = v;
    __syncthreads();
    T r = scratch[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = red_op(r, scratch[w], op);
    return r;
}

// Orders the LDS accesses of one wave around this point (the wave's lanes exchange
// values through LDS; no other wave takes part).
__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

constexpr int kUpdThreads = 256;
constexpr size_t kUpdLds = 65536;

// LDS layout of cem_update_kernel: wgt[n_elite] | mun[MAXD] | part[256] | scratch[16] |
// X[rows][MAXD] (a chunk of elite rows, later the matrix to factor).  Rows are padded
// to MAXD columns so that the unrolled loops over a row need no bounds tests.
template <typename T>
__host__ __device__ inline size_t upd_fixed_bytes(int n_elite, int maxd)
{
    return sizeof(T) * ((size_t)n_elite + maxd + kUpdThreads + 16);
}

// One workgroup: weights, new mean and covariance (eqs update_mean,
// update_covariance) and L = chol(Sigma + eps I).  Elite rows are staged in LDS in
// chunks of `rows` (all of them when they fit); the mean is a sum of per-thread
// strided partials, each lower-triangle covariance entry is one thread's sum over
// the elites (SL entries per thread), and the factor is computed by one wave with
// row r in lane r's registers (dim <= MAXD <= 64).
template <typename T, int MAXD, int SL>
__global__ __launch_bounds__(kUpdThreads) void cem_update_kernel(int n_elite, int dim, int rows,
                                                                 const int32_t *__restrict__ elite,
                                                                 const T *__restrict__ xb,
                                                                 const T *__restrict__ caug, T sigma, T gamma,
                                                                 T eps, T *__restrict__ mu,
                                                                 T *__restrict__ Sigma, T *__restrict__ L)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *wgt = reinterpret_cast<T *>(smem_raw);   // [n_elite]
    T *mun = wgt + n_elite;                      // [MAXD], zero past dim
    T *part = mun + MAXD;                        // [256]
    T *scratch = part + kUpdThreads;             // [16]
    T *X = scratch + 16;                         // [rows][MAXD], then [MAXD][MAXD]
    const int tid = threadIdx.x;
    const bool resident = rows >= n_elite;
    // row e of the elite set -> X[e - c0][:]; one thread per row so that a row costs
    // one round trip of independent loads (columns past dim repeat the last one)
    auto load_rows = [&](int c0, int cn) {
        for (int e = tid; e < cn; e += kUpdThreads) {
            const T *src = xb + (size_t)elite[c0 + e] * dim;
            T v[MAXD];
#pragma unroll
            for (int c = 0; c < MAXD; ++c) v[c] = src[min(c, dim - 1)];
#pragma unroll
            for (int c = 0; c < MAXD; ++c) X[e * MAXD + c] = v[c];
        }
    };
    T mn = T(INFINITY), s = T(0);
#pragma unroll 4
    for (int e = tid; e < n_elite; e += kUpdThreads) {
        const T c = caug[elite[e]];
        wgt[e] = c;
        mn = fmin(mn, c);
        s += c;
    }
    if (resident) load_rows(0, n_elite);
    // delta = min c_aug, spread = population std over the elite set
    const T delta = block_reduce(mn, scratch, Red::kMin);
    const T mean = block_reduce(s, scratch, Red::kSum) / T(n_elite);
    T v = T(0);
    for (int e = tid; e < n_elite; e += kUpdThreads) {
        const T d = wgt[e] - mean;
        v = fma(d, d, v);
    }
    const T spread = sqrt(block_reduce(v, scratch, Red::kSum) / T(n_elite));
    const T scale = spread > T(0) ? gamma * spread : T(1);
    T sw = T(0);
    for (int e = tid; e < n_elite; e += kUpdThreads) {
        const T wv = exp(-(wgt[e] - delta) / scale);
        wgt[e] = wv;
        sw += wv;
    }
    const T wsum = block_reduce(sw, scratch, Red::kSum);  // ends with a barrier: wgt[] complete

    // mean: thread (r, sl) sums elites sl, sl + S, ... of every chunk for coordinate r
    const int S = kUpdThreads / dim;
    const int mr = tid % dim, msl = tid / dim;
    T macc = T(0);
    for (int c0 = 0; c0 < n_elite; c0 += rows) {
        const int cn = min(rows, n_elite - c0);
        if (!resident) load_rows(c0, cn);
        __syncthreads();
        if (msl < S)
#pragma unroll 4
            for (int e = msl; e < cn; e += S) macc = fma(wgt[c0 + e], X[e * MAXD + mr], macc);
        __syncthreads();
    }
    if (msl < S) part[tid] = macc;
    __syncthreads();
    if (tid < MAXD) {
        T m = T(0);
        if (tid < dim) {
            T a = T(0);
            for (int k = 0; k < S; ++k) a += part[k * dim + tid];
            m = (T(1) - sigma) * mu[tid] + sigma * a / wsum;
            mu[tid] = m;
        }
        mun[tid] = m;
    }
    // covariance: slot k of thread tid holds lower-triangle entry q = tid + 256 k,
    // q = r (r + 1) / 2 + c; slots past the triangle accumulate entry (0, 0) and are
    // dropped, so the elite loop has no per-lane branches
    const int n_ent = dim * (dim + 1) / 2;
    int er[SL], ec[SL];
    T cacc[SL];
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int q = tid + k * kUpdThreads;
        int r = (int)((sqrtf(8.f * (float)q + 1.f) - 1.f) * 0.5f);
        while (r * (r + 1) / 2 > q) --r;
        while ((r + 1) * (r + 2) / 2 <= q) ++r;
        const bool on = q < n_ent;
        er[k] = on ? r : 0;
        ec[k] = on ? q - r * (r + 1) / 2 : 0;
        cacc[k] = T(0);
    }
    for (int c0 = 0; c0 < n_elite; c0 += rows) {
        const int cn = min(rows, n_elite - c0);
        if (!resident) load_rows(c0, cn);
        __syncthreads();   // chunk loaded; mun[] visible
        for (int e = tid; e < cn; e += kUpdThreads)
#pragma unroll
            for (int c = 0; c < MAXD; ++c) X[e * MAXD + c] -= mun[c];
        __syncthreads();
#pragma unroll 4
        for (int e = 0; e < cn; ++e) {
            const T w = wgt[c0 + e];
            const T *x = X + e * MAXD;
#pragma unroll
            for (int k = 0; k < SL; ++k) cacc[k] = fma(w * x[er[k]], x[ec[k]], cacc[k]);
        }
        __syncthreads();
    }
    // Sigma' = (1 - sigma) Sigma + sigma C / wsum from the lower triangle, mirrored;
    // A = Sigma' + eps I overwrites the staged rows
    T *A = X;
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        if (tid + k * kUpdThreads >= n_ent) continue;
        const int r = er[k], c = ec[k];
        const T sn = (T(1) - sigma) * Sigma[r * dim + c] + sigma * cacc[k] / wsum;
        Sigma[r * dim + c] = sn;
        Sigma[c * dim + r] = sn;
        A[r * MAXD + c] = sn + (r == c ? eps : T(0));
    }
    __syncthreads();
    if (tid >= 64) return;
    // right-looking Cholesky by one wave, row r in lane r's registers; column j's
    // scaled entries L[.][j] reach the other lanes through LDS (part[] is free now).
    // Entries above the diagonal, and rows and columns past dim, carry values that
    // are never read back nor stored, so the unrolled update needs no masks.
    const int r = tid;
    T *col = part;
    T a[MAXD];
#pragma unroll
    for (int c = 0; c < MAXD; ++c) a[c] = (r < dim && c <= r) ? A[r * MAXD + c] : T(0);
#pragma unroll
    for (int j = 0; j < MAXD; ++j) {
        if (j < dim) {
            if (r == j) col[0] = a[j];
            wave_sync_lds();
            const T d = sqrt(col[0]);
            const T l = r == j ? d : a[j] / d;
            a[j] = l;
            col[1 + r] = l;
            wave_sync_lds();
#pragma unroll
            for (int c = j + 1; c < MAXD; ++c) a[c] = fma(-l, col[1 + c], a[c]);
            wave_sync_lds();
        }
    }
    // rows back through LDS, then L written coalesced (zero above the diagonal)
    if (r < dim)
#pragma unroll
        for (int c = 0; c < MAXD; ++c) A[r * MAXD + c] = a[c];
    wave_sync_lds();
    for (int i = r; i < dim * dim; i += 64) {
        const int rr = i / dim, cc = i - rr * dim;
        L[i] = cc <= rr ? A[rr * MAXD + cc] : T(0);
    }
}

template <typename T, int MAXD, int SL>
hipError_t update_launch(int n_elite, int dim, const int32_t *elite, const void *xb, const void *caug,
                         double sigma, double gamma, double eps, void *mu, void *Sigma, void *L, hipStream_t st)
{
    const size_t fixed = upd_fixed_bytes<T>(n_elite, MAXD);
    const size_t row_bytes = (size_t)MAXD * sizeof(T);
    if (fixed + (size_t)MAXD * row_bytes > kUpdLds) return hipErrorInvalidValue;
    const int rows = (int)std::min<size_t>((size_t)n_elite, (kUpdLds - fixed) / row_bytes);
    const size_t lds = fixed + (size_t)std::max(rows, MAXD) * row_bytes;
    hipLaunchKernelGGL((cem_update_kernel<T, MAXD, SL>), dim3(1), dim3(kUpdThreads), lds, st, n_elite, dim, rows,
                       elite, (const T *)xb, (const T *)caug, (T)sigma, (T)gamma, (T)eps, (T *)mu, (T *)Sigma,
                       (T *)L);
    return hipGetLastError();
}

template <typename T>
hipError_t sample_t(int n, int dim, const void *mu, const void *L, const void *z, void *xi, void *xb,
                    void *lam, hipStream_t st)
{
    const int total = n * dim, threads = 256;
    hipLaunchKernelGGL(cem_sample_kernel<T>, dim3((total + threads - 1) / threads), dim3(threads), 0, st,
                       n, dim, (const T *)mu, (const T *)L, (const T *)z, (T *)xi, (T *)xb, (T *)lam);
    return hipGetLastError();
}

template <typename T>
hipError_t cost_t(int n, int dims, int nv, int n_p, int nvp, const void *phi, const void *xb,
                  const void *res, double quantum, void *caug, int32_t *rkey, hipStream_t st)
{
    const int threads = 256, blocks = (n * 64 + threads - 1) / threads;
    const T *pdd = (const T *)phi + (size_t)2 * n_p * nvp;
    hipLaunchKernelGGL(cem_cost_kernel<T>, dim3(blocks), dim3(threads), 0, st, n, dims, nv, n_p, nvp, pdd,
                       (const T *)xb, (const T *)res, (T)(1.0 / quantum), (T *)caug, rkey);
    return hipGetLastError();
}

template <typename T>
hipError_t select_t(int n, const int32_t *rkey, const void *caug, int n_proj, int n_elite,
                    int32_t *proj, int32_t *elite, hipStream_t st)
{
    // first the n_proj smallest (rkey, caug, index), then among those the n_elite
    // smallest (caug, index); the second launch ranks the first one's output
    const size_t lds1 = (size_t)n * (sizeof(uint64_t) + sizeof(uint32_t));
    hipLaunchKernelGGL((cem_rank_kernel<T, false>), dim3((n + kRankPerBlock - 1) / kRankPerBlock),
                       dim3(kRankThreads), lds1, st, n, rkey, (const T *)caug, (const int32_t *)nullptr, n_proj,
                       proj);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds2 = (size_t)n_proj * (sizeof(uint64_t) + sizeof(uint32_t));
    hipLaunchKernelGGL((cem_rank_kernel<T, true>), dim3((n_proj + kRankPerBlock - 1) / kRankPerBlock),
                       dim3(kRankThreads), lds2, st, n_proj, (const int32_t *)nullptr, (const T *)caug,
                       (const int32_t *)proj, n_elite, elite);
    return hipGetLastError();
}

template <typename T>
hipError_t update_t(int n_elite, int dim, const int32_t *elite, const void *xb, const void *caug,
                    double sigma, double gamma, double eps, void *mu, void *Sigma, void *L,
                    hipStream_t st)
{
    // instances (MAXD, SL): dim <= MAXD and dim (dim + 1) / 2 <= 256 SL
    if (dim < 1 || dim > 48) return hipErrorInvalidValue;
    if (dim <= 16) return update_launch<T, 16, 1>(n_elite, dim, elite, xb, caug, sigma, gamma, eps, mu, Sigma, L, st);
    if (dim <= 22) return update_launch<T, 24, 1>(n_elite, dim, elite, xb, caug, sigma, gamma, eps, mu, Sigma, L, st);
    if (dim <= 24) return update_launch<T, 24, 2>(n_elite, dim, elite, xb, caug, sigma, gamma, eps, mu, Sigma, L, st);
    if (dim <= 32) return update_launch<T, 32, 3>(n_elite, dim, elite, xb, caug, sigma, gamma, eps, mu, Sigma, L, st);
    return update_launch<T, 48, 5>(n_elite, dim, elite, xb, caug, sigma, gamma, eps, mu, Sigma, L, st);
}

// ---- counter-based draws (Philox4x64-10, Salmon et al. SC 2011; Box-Muller) ----
// Block b of the stream (key, counter): the 256-bit counter (counter + b mod 2^64, 0, 0,
// 0) under the key (key, 0), ten rounds; its four words give uniforms
// (floor(x / 2^11) + 1/2) 2^-53 and, in pairs, four standard normals (FP64 arithmetic,
// stored in the output's precision).
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull, kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull, kPhiloxW1 = 0xBB67AE8584CAA73Bull;

template <typename T>
__global__ __launch_bounds__(256) void normals_kernel(long count, uint64_t key, uint64_t counter, T *__restrict__ z)
{
    const long b = (long)blockIdx.x * 256 + threadIdx.x;
    if (4 * b >= count) return;
    uint64_t c0 = counter + (uint64_t)b, c1 = 0, c2 = 0, c3 = 0, k0 = key, k1 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t hi0 = __umul64hi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
        const uint64_t hi1 = __umul64hi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    const uint64_t w[4] = {c0, c1, c2, c3};
    double zz[4];
#pragma unroll
    for (int j = 0; j < 4; j += 2) {
        const double u0 = ((double)(w[j] >> 11) + 0.5) * 0x1p-53;
        const double u1 = ((double)(w[j + 1] >> 11) + 0.5) * 0x1p-53;
        const double r = sqrt(-2.0 * log(u0));
        double sn, cs;
        sincos(2.0 * M_PI * u1, &sn, &cs);
        zz[j] = r * cs;
        zz[j + 1] = r * sn;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (4 * b + j < count) z[4 * b + j] = (T)zz[j];
}

}  // namespace

hipError_t launch_normals(bool f64, long count, uint64_t key, uint64_t counter, void *z, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const long blocks = (count + 3) / 4;
    const dim3 grid((unsigned)((blocks + 255) / 256));
    if (f64) hipLaunchKernelGGL(normals_kernel<double>, grid, dim3(256), 0, st, count, key, counter, (double *)z);
    else hipLaunchKernelGGL(normals_kernel<float>, grid, dim3(256), 0, st, count, key, counter, (float *)z);
    return hipGetLastError();
}

hipError_t launch_cem_sample(bool f64, int n, int dim, const void *mu, const void *L, const void *z,
                             void *xi, void *xb, void *lam, hipStream_t st)
{
    return f64 ? sample_t<double>(n, dim, mu, L, z, xi, xb, lam, st)
               : sample_t<float>(n, dim, mu, L, z, xi, xb, lam, st);
}

hipError_t launch_cem_cost(bool f64, int n, int dims, int nv, int n_p, int nvp, const void *phi,
                           const void *xb, const void *res, double quantum, void *caug, int32_t *rkey,
                           hipStream_t st)
{
    return f64 ? cost_t<double>(n, dims, nv, n_p, nvp, phi, xb, res, quantum, caug, rkey, st)
               : cost_t<float>(n, dims, nv, n_p, nvp, phi, xb, res, quantum, caug, rkey, st);
}

hipError_t launch_cem_select(bool f64, int n, const int32_t *rkey, const void *caug, int n_proj,
                             int n_elite, int32_t *proj, int32_t *elite, hipStream_t st)
{
    return f64 ? select_t<double>(n, rkey, caug, n_proj, n_elite, proj, elite, st)
               : select_t<float>(n, rkey, caug, n_proj, n_elite, proj, elite, st);
}

hipError_t launch_cem_update(bool f64, int n_elite, int dim, const int32_t *elite, const void *xb,
                             const void *caug, double sigma, double gamma, double eps, void *mu,
                             void *Sigma, void *L, hipStream_t st)
{
    return f64 ? update_t<double>(n_elite, dim, elite, xb, caug, sigma, gamma, eps, mu, Sigma, L, st)
               : update_t<float>(n_elite, dim, elite, xb, caug, sigma, gamma, eps, mu, Sigma, L, st);
}

}  // namespace trajam
