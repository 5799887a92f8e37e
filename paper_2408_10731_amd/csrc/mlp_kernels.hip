// gfx950 kernels of the learned warm start: a fully connected ReLU network trained
// and evaluated on the GPU (forward, backward, MSE, Adam), plus the kernels that
// turn its prediction into a warm start (xi_bar0, lambda0) with a cold fallback.
//
// All products go through one strided tiled GEMM, C[m][n] = sum_k A(m,k) B(k,n) with
// A(m,k) = A[m*sam + k*sak] and B(k,n) = B[k*sbk + n*sbn], so the forward product
// (x W^T), the weight gradient (d^T a) and the input gradient (d W) are the same
// kernel with different strides.  64 x 64 output tile per workgroup, K staged through
// LDS in steps of 16.  FP32 mode: 4 x 4 outputs per thread on the VALU.  BF16 mode:
// four waves, each a 32 x 32 sub-tile of v_mfma_f32_16x16x16_bf16 (operands rounded
// to bf16 when read from LDS, fp32 accumulation).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "am_internal.h"

namespace trajam {
namespace {

constexpr int BM = 64, BN = 64, BK = 16;

typedef short mlp_bf16x4 __attribute__((ext_vector_type(4)));
typedef float mlp_f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

enum Epi { kEpiNone = 0, kEpiBiasRelu = 1, kEpiBias = 2, kEpiMask = 3 };

template <bool BF16>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, const float *__restrict__ A,
                                                   long sam, long sak, const float *__restrict__ B,
                                                   long sbk, long sbn, float *__restrict__ C, int ldc,
                                                   int epi, const float *__restrict__ bias,
                                                   const float *__restrict__ mask, int ldm)
{
    __shared__ float As[BK][BM + 4];
    __shared__ float Bs[BK][BN + 4];
    const int tid = threadIdx.x;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    float acc[4][4] = {};
    mlp_f32x4 macc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) macc[i][j] = mlp_f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = tid + 256 * r;
            const int ml = e & (BM - 1), kl = e / BM;
            const int m = m0 + ml, k = k0 + kl;
            As[kl][ml] = (m < M && k < K) ? A[(long)m * sam + (long)k * sak] : 0.f;
            const int n = n0 + ml;
            Bs[kl][ml] = (n < N && k < K) ? B[(long)k * sbk + (long)n * sbn] : 0.f;
        }
        __syncthreads();
        if constexpr (!BF16) {
            const int ty = tid >> 4, tx = tid & 15;
#pragma unroll
            for (int k = 0; k < BK; ++k) {
                float a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) { a[i] = As[k][ty * 4 + i]; b[i] = Bs[k][tx * 4 + i]; }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
            }
        } else {
            const int lane = tid & 63, wv = tid >> 6;
            const int rb = (wv >> 1) * 32, cb = (wv & 1) * 32;
            const int r16 = lane & 15, kq = 4 * (lane >> 4);
            mlp_bf16x4 av[2], bv[2];
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    av[t][i] = to_bf16(As[kq + i][rb + t * 16 + r16]);
                    bv[t][i] = to_bf16(Bs[kq + i][cb + t * 16 + r16]);
                }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    macc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[i], bv[j], macc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    auto store = [&](int m, int n, float v) {
        if (m >= M || n >= N) return;
        if (epi == kEpiBiasRelu) v = fmaxf(v + bias[n], 0.f);
        else if (epi == kEpiBias) v = v + bias[n];
        else if (epi == kEpiMask) v = mask[(long)m * ldm + n] > 0.f ? v : 0.f;
        C[(long)m * ldc + n] = v;
    };
    if constexpr (!BF16) {
        const int ty = tid >> 4, tx = tid & 15;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) store(m0 + ty * 4 + i, n0 + tx * 4 + j, acc[i][j]);
    } else {
        const int lane = tid & 63, wv = tid >> 6;
        const int rb = (wv >> 1) * 32, cb = (wv & 1) * 32;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    store(m0 + rb + i * 16 + 4 * (lane >> 4) + q, n0 + cb + j * 16 + (lane & 15), macc[i][j][q]);
    }
}

// db[n] = sum_b d[b][n] (fixed summation order)
__global__ void colsum_kernel(int rows, int cols, const float *__restrict__ d, float *__restrict__ out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= cols) return;
    float s = 0.f;
    for (int b = 0; b < rows; ++b) s += d[(long)b * cols + n];
    out[n] = s;
}

// dy = 2 (y - t) / count; loss = mean (y - t)^2 (one workgroup, fixed order)
__global__ void mse_kernel(long count, const float *__restrict__ y, const float *__restrict__ t,
                           float *__restrict__ dy, float *__restrict__ loss)
{
    __shared__ float part[1024];
    float s = 0.f;
    const float inv = 1.f / (float)count;
    for (long i = threadIdx.x; i < count; i += blockDim.x) {
        const float d = y[i] - t[i];
        dy[i] = 2.f * d * inv;
        s = fmaf(d, d, s);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = part[0] * inv;
}

__global__ void adam_kernel(long n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// X[b] = [scene features, (xi[b] - line) * inv_scale]
__global__ void warm_features_kernel(int batch, int dim, int n_scene, const float *__restrict__ scene,
                                     const float *__restrict__ xi, const float *__restrict__ line,
                                     float inv_scale, float *__restrict__ X)
{
    const int width = n_scene + dim;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)batch * width) return;
    const int b = (int)(i / width), f = (int)(i - (long)b * width);
    X[i] = f < n_scene ? scene[f] : (xi[(long)b * dim + (f - n_scene)] - line[f - n_scene]) * inv_scale;
}

// One thread per sample: delta = y * out_scale; xb0 = xi + delta on the free
// coefficients and the exact boundary coefficients on the others (when given);
// lambda0 = delta on the free coefficients (the converged multiplier of a fixed point
// equals xb - xi there) and 0 on the boundary ones; non-finite predictions fall back
// cold.
__global__ void warm_apply_kernel(int batch, int dims, int nv, const float *__restrict__ y,
                                  const float *__restrict__ xi, float out_scale, WarmBoundary bc,
                                  float *__restrict__ xb0, float *__restrict__ lam0, uint32_t *__restrict__ flags)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const int dim = dims * nv;
    bool finite = true;
    for (int r = 0; r < dim; ++r) finite = finite && isfinite(y[(long)b * dim + r]);
    for (int r = 0; r < dim; ++r) {
        const long i = (long)b * dim + r;
        const int m = r % nv;
        const bool bnd = m <= 2 || m == nv - 1;
        const float d = finite ? y[i] * out_scale : 0.f;
        xb0[i] = (finite && bnd && bc.set) ? bc.c[r / nv][m == nv - 1 ? 3 : m] : xi[i] + d;
        lam0[i] = bnd ? 0.f : d;
    }
    if (flags) flags[b] = finite ? 0u : 4u;
}

// Per-sample fallback: when the warm start's residual exceeds the cold start's, the
// sample restarts cold (xb0 = xi, lambda0 = 0) and is flagged.
__global__ void warm_fallback_kernel(int batch, int dim, const float *__restrict__ rw,
                                     const float *__restrict__ rc, const float *__restrict__ xi,
                                     float *__restrict__ xb0, float *__restrict__ lam0,
                                     uint32_t *__restrict__ flags)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    if (!(rw[b] <= rc[b])) {
        for (int r = 0; r < dim; ++r) {
            xb0[(long)b * dim + r] = xi[(long)b * dim + r];
            lam0[(long)b * dim + r] = 0.f;
        }
        if (flags) flags[b] |= 4u;
    }
}

}  // namespace

hipError_t launch_gemm(bool bf16, int M, int N, int K, const float *A, long sam, long sak, const float *B,
                       long sbk, long sbn, float *C, int ldc, int epi, const float *bias, const float *mask,
                       int ldm, hipStream_t st)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM);
    if (bf16)
        hipLaunchKernelGGL(gemm_kernel<true>, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc,
                           epi, bias, mask, ldm);
    else
        hipLaunchKernelGGL(gemm_kernel<false>, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc,
                           epi, bias, mask, ldm);
    return hipGetLastError();
}

hipError_t launch_colsum(int rows, int cols, const float *d, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(colsum_kernel, dim3((cols + 255) / 256), dim3(256), 0, st, rows, cols, d, out);
    return hipGetLastError();
}

hipError_t launch_mse(long count, const float *y, const float *t, float *dy, float *loss, hipStream_t st)
{
    hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(1024), 0, st, count, y, t, dy, loss);
    return hipGetLastError();
}

hipError_t launch_adam(long n, float *p, const float *g, float *m, float *v, int step, float lr, float b1,
                       float b2, float eps, hipStream_t st)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, p, g, m, v, lr, b1,
                       b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_warm_features(int batch, int dim, int n_scene, const float *scene, const float *xi,
                                const float *line, float inv_scale, float *X, hipStream_t st)
{
    const long total = (long)batch * (n_scene + dim);
    hipLaunchKernelGGL(warm_features_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, batch, dim,
                       n_scene, scene, xi, line, inv_scale, X);
    return hipGetLastError();
}

hipError_t launch_warm_apply(int batch, int dims, int nv, const float *y, const float *xi, float out_scale,
                             const WarmBoundary &bc, float *xb0, float *lam0, uint32_t *flags, hipStream_t st)
{
    hipLaunchKernelGGL(warm_apply_kernel, dim3((batch + 255) / 256), dim3(256), 0, st, batch, dims, nv, y, xi,
                       out_scale, bc, xb0, lam0, flags);
    return hipGetLastError();
}

hipError_t launch_warm_fallback(int batch, int dim, const float *rw, const float *rc, const float *xi,
                                float *xb0, float *lam0, uint32_t *flags, hipStream_t st)
{
    hipLaunchKernelGGL(warm_fallback_kernel, dim3((batch + 255) / 256), dim3(256), 0, st, batch, dim, rw, rc, xi,
                       xb0, lam0, flags);
    return hipGetLastError();
}

}  // namespace trajam
