// gfx950 kernels of the projection-guided sampling loop (thesis ch. 6, Alg 3):
// Gaussian sampling from (mu, L), the augmented cost and residual key, a one-
// workgroup bitonic top-k with lexicographic keys, and the weighted mean /
// covariance update (eqs update_mean, update_covariance) with the Cholesky factor
// for the next draw.  The projection between sampling and cost is the AM kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "am_internal.h"

namespace trajam {
namespace {

// xi[i][r] = mu[r] + sum_{c <= r} L[r][c] z[i][c]
template <typename T>
__global__ void cem_sample_kernel(int n, int dim, const T *__restrict__ mu,
                                  const T *__restrict__ L, const T *__restrict__ z,
                                  T *__restrict__ xi)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n * dim) return;
    const int i = gid / dim, r = gid - (gid / dim) * dim;
    T acc = mu[r];
    for (int c = 0; c <= r; ++c) acc = fma(L[r * dim + c], z[(size_t)i * dim + c], acc);
    xi[gid] = acc;
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

// Lexicographic (k1, k2, idx) comparison.
template <typename T>
__device__ __forceinline__ bool key_less(int32_t a1, T a2, int32_t ai, int32_t b1, T b2, int32_t bi)
{
    if (a1 != b1) return a1 < b1;
    if (a2 != b2) return a2 < b2;
    return ai < bi;
}

template <typename T>
__device__ void bitonic_sort(int32_t *k1, T *k2, int32_t *id, int len)
{
    for (int size = 2; size <= len; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < len / 2; t += blockDim.x) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool up = ((lo & size) == 0);
                const bool lt = key_less(k1[hi], k2[hi], id[hi], k1[lo], k2[lo], id[lo]);
                if (lt == up) {
                    int32_t a = k1[lo]; k1[lo] = k1[hi]; k1[hi] = a;
                    T b = k2[lo]; k2[lo] = k2[hi]; k2[hi] = b;
                    int32_t c = id[lo]; id[lo] = id[hi]; id[hi] = c;
                }
            }
            __syncthreads();
        }
    }
}

// One workgroup: the n_proj smallest (rkey, caug, index) and, among those, the
// n_elite smallest (caug, index).  len = n rounded up to a power of two (<= 4096).
template <typename T>
__global__ void cem_select_kernel(int n, int len, const int32_t *__restrict__ rkey,
                                  const T *__restrict__ caug, int n_proj, int n_elite,
                                  int32_t *__restrict__ proj_idx, int32_t *__restrict__ elite_idx)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *k2 = reinterpret_cast<T *>(smem_raw);
    int32_t *k1 = reinterpret_cast<int32_t *>(k2 + len);
    int32_t *id = k1 + len;
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
        const bool real = i < n;
        k1[i] = real ? rkey[i] : 2147483647;
        k2[i] = real ? caug[i] : T(INFINITY);
        id[i] = real ? i : 2147483647;
    }
    __syncthreads();
    bitonic_sort<T>(k1, k2, id, len);
    for (int i = threadIdx.x; i < n_proj; i += blockDim.x) proj_idx[i] = id[i];
    __syncthreads();
    // second stage: the ConstraintEliteSet by (caug, index)
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
        const bool real = i < n_proj;
        k1[i] = real ? 0 : 2147483647;
        if (!real) { k2[i] = T(INFINITY); id[i] = 2147483647; }
    }
    __syncthreads();
    bitonic_sort<T>(k1, k2, id, len);
    for (int i = threadIdx.x; i < n_elite; i += blockDim.x) elite_idx[i] = id[i];
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

// One workgroup: weights, new mean and covariance, and L = chol(Sigma + eps I).
template <typename T>
__global__ void cem_update_kernel(int n_elite, int dim, const int32_t *__restrict__ elite,
                                  const T *__restrict__ xb, const T *__restrict__ caug, T sigma,
                                  T gamma, T eps, T *__restrict__ mu, T *__restrict__ Sigma,
                                  T *__restrict__ L)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *wgt = reinterpret_cast<T *>(smem_raw);       // [n_elite]
    T *mun = wgt + n_elite;                          // [dim]
    T *A = mun + dim;                                // [dim][dim]
    T *scratch = A + dim * dim;                      // [16]
    const int tid = threadIdx.x;
    // delta = min c_aug, spread = population std over the elite set
    T mn = T(INFINITY), s = T(0);
    for (int e = tid; e < n_elite; e += blockDim.x) {
        const T c = caug[elite[e]];
        mn = fmin(mn, c);
        s += c;
    }
    const T delta = block_reduce(mn, scratch, Red::kMin);
    const T mean = block_reduce(s, scratch, Red::kSum) / T(n_elite);
    T v = T(0);
    for (int e = tid; e < n_elite; e += blockDim.x) {
        const T d = caug[elite[e]] - mean;
        v = fma(d, d, v);
    }
    const T spread = sqrt(block_reduce(v, scratch, Red::kSum) / T(n_elite));
    const T scale = spread > T(0) ? gamma * spread : T(1);
    T sw = T(0);
    for (int e = tid; e < n_elite; e += blockDim.x) {
        const T wv = exp(-(caug[elite[e]] - delta) / scale);
        wgt[e] = wv;
        sw += wv;
    }
    const T wsum = block_reduce(sw, scratch, Red::kSum);
    __syncthreads();
    for (int r = tid; r < dim; r += blockDim.x) {
        T acc = T(0);
        for (int e = 0; e < n_elite; ++e) acc = fma(wgt[e], xb[(size_t)elite[e] * dim + r], acc);
        mun[r] = (T(1) - sigma) * mu[r] + sigma * acc / wsum;
    }
    __syncthreads();
    for (int i = tid; i < dim * dim; i += blockDim.x) {
        const int r = i / dim, c = i - (i / dim) * dim;
        T acc = T(0);
        for (int e = 0; e < n_elite; ++e) {
            const T *x = xb + (size_t)elite[e] * dim;
            acc = fma(wgt[e] * (x[r] - mun[r]), x[c] - mun[c], acc);
        }
        const T sn = (T(1) - sigma) * Sigma[i] + sigma * acc / wsum;
        Sigma[i] = sn;
        A[i] = sn + (r == c ? eps : T(0));
    }
    for (int r = tid; r < dim; r += blockDim.x) mu[r] = mun[r];
    __syncthreads();
    // right-looking Cholesky in LDS: column j, then the trailing update
    for (int j = 0; j < dim; ++j) {
        if (tid == 0) A[j * dim + j] = sqrt(A[j * dim + j]);
        __syncthreads();
        for (int r = j + 1 + tid; r < dim; r += blockDim.x) A[r * dim + j] /= A[j * dim + j];
        __syncthreads();
        for (int i = tid; i < dim * dim; i += blockDim.x) {
            const int r = i / dim, c = i - (i / dim) * dim;
            if (r > j && c > j && c <= r) A[i] = fma(-A[r * dim + j], A[c * dim + j], A[i]);
        }
        __syncthreads();
    }
    for (int i = tid; i < dim * dim; i += blockDim.x) {
        const int r = i / dim, c = i - (i / dim) * dim;
        L[i] = c <= r ? A[i] : T(0);
    }
}

template <typename T>
hipError_t sample_t(int n, int dim, const void *mu, const void *L, const void *z, void *xi,
                    hipStream_t st)
{
    const int total = n * dim, threads = 256;
    hipLaunchKernelGGL(cem_sample_kernel<T>, dim3((total + threads - 1) / threads), dim3(threads), 0, st,
                       n, dim, (const T *)mu, (const T *)L, (const T *)z, (T *)xi);
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
    int len = 1;
    while (len < n) len <<= 1;
    if (len < 2) len = 2;
    const size_t lds = (size_t)len * (sizeof(T) + 2 * sizeof(int32_t));
    hipLaunchKernelGGL(cem_select_kernel<T>, dim3(1), dim3(1024), lds, st, n, len, rkey, (const T *)caug,
                       n_proj, n_elite, proj, elite);
    return hipGetLastError();
}

template <typename T>
hipError_t update_t(int n_elite, int dim, const int32_t *elite, const void *xb, const void *caug,
                    double sigma, double gamma, double eps, void *mu, void *Sigma, void *L,
                    hipStream_t st)
{
    const size_t lds = sizeof(T) * ((size_t)n_elite + dim + (size_t)dim * dim + 16);
    hipLaunchKernelGGL(cem_update_kernel<T>, dim3(1), dim3(256), lds, st, n_elite, dim, elite,
                       (const T *)xb, (const T *)caug, (T)sigma, (T)gamma, (T)eps, (T *)mu,
                       (T *)Sigma, (T *)L);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cem_sample(bool f64, int n, int dim, const void *mu, const void *L, const void *z,
                             void *xi, hipStream_t st)
{
    return f64 ? sample_t<double>(n, dim, mu, L, z, xi, st) : sample_t<float>(n, dim, mu, L, z, xi, st);
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
