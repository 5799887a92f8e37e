// gfx950 kernels of the learned warm start: a fully connected ReLU network trained
// and evaluated on the GPU (forward, backward, MSE, Adam), plus the kernels that
// turn its prediction into a warm start (xi_bar0, lambda0) with a cold fallback.
//
// All products go through one strided GEMM, C[m][n] = sum_k A(m,k) B(k,n) with
// A(m,k) = A[m*sam + k*sak] and B(k,n) = B[k*sbk + n*sbn], so the forward product
// (x W^T), the weight gradient (d^T a) and the input gradient (d W) are the same
// kernel with different strides, optionally split over K into slices whose partial
// products are added in slice order by a second kernel (the weight gradient, whose K
// is the batch, would otherwise run on a handful of workgroups).
//  - FP32 mode: 64 x 64 output tile per workgroup, K staged through LDS in steps of
//    16, 4 x 4 outputs per thread on the VALU.
//  - BF16 mode (matrix cores): 128 x 128 output tile per workgroup of four waves, each
//    a 64 x 64 block of 4 x 4 v_mfma_f32_16x16x32_bf16 tiles; K in steps of 32 through
//    two LDS buffers (one barrier per step) holding the operands already rounded to
//    bf16, k-contiguous per row so that a lane's fragment is one 16-byte read; fp32
//    accumulation.  Tiles are numbered so that the tiles of one XCD share their rows
//    of A in that XCD's L2, and the weight gradient's bias gradient (the row sums of
//    A = d^T) is taken from the fp32 values while they are staged.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "../../include/trajam.h"
#include "am_internal.h"

namespace trajam {
namespace {

constexpr int BM = 64, BN = 64, BK = 16;

typedef short mlp_bf16x4 __attribute__((ext_vector_type(4)));
typedef float mlp_f32x4 __attribute__((ext_vector_type(4)));

// Round to nearest even; a NaN stays a (quiet) NaN instead of carrying into the sign.
__device__ __forceinline__ short to_bf16(float x)
{
    unsigned u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (short)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

enum Epi { kEpiNone = 0, kEpiBiasRelu = 1, kEpiBias = 2, kEpiMask = 3 };

// FP32 mode; blockIdx.z is the K slice [z k_chunk, min(K, (z+1) k_chunk)), whose
// product goes to C + z c_slice.
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, const float *__restrict__ A,
                                                   long sam, long sak, const float *__restrict__ B,
                                                   long sbk, long sbn, float *__restrict__ C, int ldc,
                                                   int epi, const float *__restrict__ bias,
                                                   const float *__restrict__ mask, int ldm, int k_chunk,
                                                   long c_slice)
{
    __shared__ float As[BK][BM + 4];
    __shared__ float Bs[BK][BN + 4];
    const int tid = threadIdx.x;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int kb = blockIdx.z * k_chunk, ke = min(K, kb + k_chunk);
    C += (long)blockIdx.z * c_slice;
    float acc[4][4] = {};
    // Global -> register tile loads, mapped so that consecutive threads read
    // consecutive addresses whichever stride of the operand is 1, with the next tile
    // prefetched into registers while the current one is multiplied out of LDS.
    const bool a_k = sak == 1, b_k = sbk == 1;
    float ra[4], rb[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = tid + 256 * r;
            const int ma = a_k ? (e >> 4) : (e & (BM - 1)), ka = a_k ? (e & (BK - 1)) : (e >> 6);
            const int m = m0 + ma, k = k0 + ka;
            ra[r] = (m < M && k < ke) ? A[(long)m * sam + (long)k * sak] : 0.f;
            const int nb = b_k ? (e >> 4) : (e & (BN - 1)), kq = b_k ? (e & (BK - 1)) : (e >> 6);
            const int n = n0 + nb, kk = k0 + kq;
            rb[r] = (n < N && kk < ke) ? B[(long)kk * sbk + (long)n * sbn] : 0.f;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = tid + 256 * r;
            As[a_k ? (e & (BK - 1)) : (e >> 6)][a_k ? (e >> 4) : (e & (BM - 1))] = ra[r];
            Bs[b_k ? (e & (BK - 1)) : (e >> 6)][b_k ? (e >> 4) : (e & (BN - 1))] = rb[r];
        }
    };
    fetch(kb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
        stash();
        if (k0 + BK < ke) fetch(k0 + BK);
        __syncthreads();
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
        __syncthreads();
    }
    const int ty = tid >> 4, tx = tid & 15;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = m0 + ty * 4 + i, n = n0 + tx * 4 + j;
            if (m >= M || n >= N) continue;
            float v = acc[i][j];
            if (epi == kEpiBiasRelu) v = fmaxf(v + bias[n], 0.f);
            else if (epi == kEpiBias) v = v + bias[n];
            else if (epi == kEpiMask) v = mask[(long)m * ldm + n] > 0.f ? v : 0.f;
            C[(long)m * ldc + n] = v;
        }
}

// ---------------------------------------------------------------- BF16 GEMM
typedef __bf16 gm_bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short gm_u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short gm_u16x4 __attribute__((ext_vector_type(4)));

struct MfmaGemm {
    int M, N, K;
    const float *A;
    long sam, sak;
    const float *B;
    long sbk, sbn;
    float *C;
    int ldc;
    long c_slice;      // C offset of K slice z: z * c_slice
    int k_chunk;       // K range of one slice (a multiple of the K step, or >= K)
    int epi;
    const float *bias, *mask;
    int ldm;
    float *rowsum;     // optional: rowsum[z rs_slice + m] = sum over the slice's k of A(m, k)
    long rs_slice;
    int tiles_m, tiles_n;
    int c_vec;         // ldc, c_slice multiples of 4 and C 16-byte aligned: float4 stores
};

// How an operand tile is read from HBM.
enum OpMode {
    kRows = 0,   // rows consecutive in memory (stride 1 between rows): coalesced across rows
    kKc = 1,     // k-contiguous rows, scalar loads
    kKcVec = 2,  // k-contiguous rows, row stride and K multiples of 4, 16-byte aligned: float4 loads
};

// The thread's share of an R_T-row x KT-k operand tile X(r, k) = X[r sr + k sk]: one
// row and V = R_T KT / 256 consecutive k.  With k-contiguous rows the P = KT / V
// neighbouring threads of a row take its parts (whole 128-byte segments of the row);
// otherwise R_T consecutive threads take R_T consecutive rows at one k.  In LDS the
// tile is stored as bf16, k-contiguous per row with a pitch of KT + 8.
template <int R_T, int KT, int MODE>
struct TileOp {
    static constexpr int V = R_T * KT / 256, P = KT / V, KP = KT + 8;
    static constexpr bool KC = MODE != kRows;
    static_assert(V % 4 == 0 && V <= 32, "4 to 32 values per thread");
    __device__ static __forceinline__ int row(int tid) { return KC ? tid / P : tid % R_T; }
    __device__ static __forceinline__ int part(int tid) { return KC ? tid % P : tid / R_T; }

    // Every thread issues the same loads, at indices clamped into the operand (also
    // past the last step), and nothing is selected here, so the loads stay in flight
    // until the values are stashed.  A clamped row only feeds outputs (or row sums)
    // beyond M or N, which are never stored; k beyond ke is zeroed by `stash`.  In
    // kKcVec mode a group of four is wholly inside or wholly outside [kb, ke).
    __device__ static __forceinline__ void fetch(const float *__restrict__ X, long sr, long sk, int R, int r0, int kb,
                                                 int ke, float v[V])
    {
        const int tid = threadIdx.x;
        const int r = min(r0 + row(tid), R - 1), k = kb + V * part(tid);
        const float *p = X + (long)r * sr;
        if constexpr (MODE == kKcVec) {
#pragma unroll
            for (int q = 0; q < V / 4; ++q) {
                const float4 f = *reinterpret_cast<const float4 *>(p + min(k + 4 * q, ke - 4));
                v[4 * q] = f.x;
                v[4 * q + 1] = f.y;
                v[4 * q + 2] = f.z;
                v[4 * q + 3] = f.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < V; ++i) v[i] = p[(long)min(k + i, ke - 1) * sk];
        }
    }

    // zero k >= ke, round to bf16 and store the thread's share; returns the fp32 sum of
    // its (zeroed) values for the row sums
    __device__ static __forceinline__ float stash(unsigned short *__restrict__ S, const float v[V], int kb, int ke)
    {
        const int tid = threadIdx.x;
        const int k = kb + V * part(tid);
        float w[V], sum = 0.f;
#pragma unroll
        for (int i = 0; i < V; ++i) {
            w[i] = k + i < ke ? v[i] : 0.f;
            sum += w[i];
        }
        unsigned short *d = S + row(tid) * KP + V * part(tid);
        if constexpr (V >= 8) {
#pragma unroll
            for (int c = 0; c < V / 8; ++c) {
                gm_u16x8 u;
#pragma unroll
                for (int i = 0; i < 8; ++i) u[i] = (unsigned short)to_bf16(w[8 * c + i]);
                *reinterpret_cast<gm_u16x8 *>(d + 8 * c) = u;
            }
        } else {
            gm_u16x4 u;
#pragma unroll
            for (int i = 0; i < 4; ++i) u[i] = (unsigned short)to_bf16(w[i]);
            *reinterpret_cast<gm_u16x4 *>(d) = u;
        }
        return sum;
    }
};

// BM x BN output tile per workgroup of four waves in a 2 x 2 grid, each wave
// (BM/2) x (BN/2) in 16 x 16 matrix-core tiles, K in steps of KT.  The operands of
// step kt are loaded into register set kt & 1 two steps ahead of their use and
// stashed into LDS buffer kt & 1 one step ahead (one barrier per step).
template <int BM_, int BN_, int KT, int AMODE, int BMODE>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(MfmaGemm g)
{
    using OA = TileOp<BM_, KT, AMODE>;
    using OB = TileOp<BN_, KT, BMODE>;
    constexpr int MI = BM_ / 32, NJ = BN_ / 32, KP = KT + 8;
    __shared__ __attribute__((aligned(16))) unsigned short smem[2][(BM_ + BN_) * KP];
    __shared__ float rs_part[OA::P][BM_];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // XCD-aware numbering: workgroup i runs on XCD i mod 8, so give each XCD a
    // contiguous run of tiles (consecutive tiles share their row block of A)
    const int T = g.tiles_m * g.tiles_n;
    int t = blockIdx.x;
    if ((T & 7) == 0) t = (t & 7) * (T >> 3) + (t >> 3);
    const int mb = t / g.tiles_n, nb = t - mb * g.tiles_n;
    const int m0 = mb * BM_, n0 = nb * BN_;
    const int z = blockIdx.y;
    const int kb = z * g.k_chunk, ke = min(g.K, kb + g.k_chunk);
    const int nk = (ke - kb + KT - 1) / KT;   // >= 1: the launcher makes no empty slice
    const bool do_rs = g.rowsum != nullptr && nb == 0;
    const int wm = (wv >> 1) * (BM_ / 2), wn = (wv & 1) * (BN_ / 2);
    const int fr = lane & 15, fk = 8 * (lane >> 4);
    mlp_f32x4 acc[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = mlp_f32x4{0.f, 0.f, 0.f, 0.f};
    float va0[OA::V], vb0[OB::V], va1[OA::V], vb1[OB::V], rs = 0.f;

#define GEMM_FETCH(VA, VB, K0)                                          \
    OA::fetch(g.A, g.sam, g.sak, g.M, m0, (K0), ke, VA);               \
    OB::fetch(g.B, g.sbn, g.sbk, g.N, n0, (K0), ke, VB);
#define GEMM_STASH(BUF, VA, VB, K0)                                     \
    {                                                                   \
        const float sa_ = OA::stash(smem[BUF], VA, (K0), ke);           \
        OB::stash(smem[BUF] + BM_ * KP, VB, (K0), ke);                  \
        if (do_rs) rs += sa_;                                           \
    }
#define GEMM_MMA(BUF)                                                                                        \
    {                                                                                                        \
        const unsigned short *As_ = smem[BUF], *Bs_ = smem[BUF] + BM_ * KP;                                  \
        _Pragma("unroll") for (int ks = 0; ks < KT; ks += 32)                                                \
        {                                                                                                    \
            gm_bf16x8 af[MI], bf[NJ];                                                                        \
            _Pragma("unroll") for (int i = 0; i < MI; ++i) af[i] = __builtin_bit_cast(                       \
                gm_bf16x8, *reinterpret_cast<const gm_u16x8 *>(As_ + (wm + 16 * i + fr) * KP + ks + fk));    \
            _Pragma("unroll") for (int j = 0; j < NJ; ++j) bf[j] = __builtin_bit_cast(                       \
                gm_bf16x8, *reinterpret_cast<const gm_u16x8 *>(Bs_ + (wn + 16 * j + fr) * KP + ks + fk));    \
            _Pragma("unroll") for (int i = 0; i < MI; ++i)                                                   \
                _Pragma("unroll") for (int j = 0; j < NJ; ++j) acc[i][j] =                                   \
                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);               \
        }                                                                                                    \
    }

    GEMM_FETCH(va0, vb0, kb)
    GEMM_FETCH(va1, vb1, kb + KT)
    GEMM_STASH(0, va0, vb0, kb)
    __syncthreads();
    for (int kt = 0; kt < nk; kt += 2) {
        GEMM_FETCH(va0, vb0, kb + (kt + 2) * KT)
        GEMM_MMA(0)
        if (kt + 1 < nk) GEMM_STASH(1, va1, vb1, kb + (kt + 1) * KT)
        __syncthreads();
        if (kt + 1 >= nk) break;
        GEMM_FETCH(va1, vb1, kb + (kt + 3) * KT)
        GEMM_MMA(1)
        if (kt + 2 < nk) GEMM_STASH(0, va0, vb0, kb + (kt + 2) * KT)
        __syncthreads();
    }
#undef GEMM_FETCH
#undef GEMM_STASH
#undef GEMM_MMA
    if (do_rs) {
        rs_part[OA::part(tid)][OA::row(tid)] = rs;
        __syncthreads();
        if (tid < BM_ && m0 + tid < g.M) {
            float s = 0.f;
#pragma unroll
            for (int p = 0; p < OA::P; ++p) s += rs_part[p][tid];
            g.rowsum[(long)z * g.rs_slice + m0 + tid] = s;
        }
    }
    // Epilogue through LDS: the tile is laid out row-major there and written with
    // consecutive threads on consecutive 16-byte pieces of a row, so every store
    // instruction covers whole cache lines.
    constexpr int CP = BN_ + 4;
    static_assert(BM_ * CP * 4 <= 2 * (BM_ + BN_) * KP * 2, "C tile fits in the operand buffers");
    float *Cs = reinterpret_cast<float *>(&smem[0][0]);
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                Cs[(wm + 16 * i + 4 * (lane >> 4) + q) * CP + wn + 16 * j + (lane & 15)] = acc[i][j][q];
    __syncthreads();
    float *C = g.C + (long)z * g.c_slice;
    constexpr int Q = BN_ / 4;  // float4 pieces per tile row
    for (int e = tid; e < BM_ * Q; e += 256) {
        const int r = e / Q, c = 4 * (e - r * Q);
        const int m = m0 + r, n = n0 + c;
        if (m >= g.M || n >= g.N) continue;
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = Cs[r * CP + c + q];
        const bool full = n + 4 <= g.N;
        if (g.epi == kEpiBiasRelu || g.epi == kEpiBias) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float b = (full || n + q < g.N) ? g.bias[n + q] : 0.f;
                v[q] = g.epi == kEpiBiasRelu ? fmaxf(v[q] + b, 0.f) : v[q] + b;
            }
        } else if (g.epi == kEpiMask) {
            const float *mr = g.mask + (long)m * g.ldm + n;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (full || n + q < g.N) v[q] = mr[q] > 0.f ? v[q] : 0.f;
        }
        float *cr = C + (long)m * g.ldc + n;
        if (full && g.c_vec) {
            *reinterpret_cast<float4 *>(cr) = make_float4(v[0], v[1], v[2], v[3]);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (n + q < g.N) cr[q] = v[q];
        }
    }
}

// out[i] = sum over z = 0 .. S-1, in that order, of part[z stride + i]
__global__ __launch_bounds__(256) void slice_sum_kernel(long n, int S, const float *__restrict__ part, long stride,
                                                        float *__restrict__ out)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    int z = 0;
    for (; z + 8 <= S; z += 8) {
        float v[8];   // eight loads in flight, added in order
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = part[(long)(z + q) * stride + i];
#pragma unroll
        for (int q = 0; q < 8; ++q) s += v[q];
    }
    for (; z < S; ++z) s += part[(long)z * stride + i];
    out[i] = s;
}

// db[n] = sum_b d[b][n] (fixed summation order)
// out[n] = sum_b d[b][n]: 64 columns per workgroup and 16 row slices of one wave each
// (coalesced 256-byte row segments, loads unrolled); the slices' partials are added
// in slice order, so the result does not depend on timing.
__global__ __launch_bounds__(1024) void colsum_kernel(int rows, int cols, const float *__restrict__ d,
                                                      float *__restrict__ out)
{
    __shared__ float part[16][64];
    const int col = blockIdx.x * 64 + (threadIdx.x & 63);
    const int sl = threadIdx.x >> 6;
    float s = 0.f;
    if (col < cols) {
#pragma unroll 8
        for (int b = sl; b < rows; b += 16) s += d[(long)b * cols + col];
    }
    part[sl][threadIdx.x & 63] = s;
    __syncthreads();
    if (sl == 0 && col < cols) {
        float t = 0.f;
#pragma unroll
        for (int k = 0; k < 16; ++k) t += part[k][threadIdx.x];
        out[col] = t;
    }
}

// dy = 2 (y - t) / count over a grid-stride range; each workgroup's sum of (y - t)^2
// goes to part[blockIdx.x] (fixed order within the workgroup)
__global__ __launch_bounds__(256) void mse_part_kernel(long count, const float *__restrict__ y,
                                                       const float *__restrict__ t, float *__restrict__ dy,
                                                       float *__restrict__ part)
{
    __shared__ float red[256];
    float s = 0.f;
    const float inv = 1.f / (float)count;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long)gridDim.x * 256) {
        const float d = y[i] - t[i];
        dy[i] = 2.f * d * inv;
        s = fmaf(d, d, s);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// loss[0] = (sum of the n partial sums, fixed order) / count
__global__ __launch_bounds__(256) void mse_final_kernel(int n, long count, const float *__restrict__ part,
                                                        float *__restrict__ loss)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] / (float)count;
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

// Fused inference: the whole network for kInferSamples samples per workgroup, the
// activations of one layer kept in LDS as act[k][s] (the samples of one input feature
// contiguous, read as one 128-bit broadcast), the weights read from L2 in the packed
// layout (per layer W^T [in][out], then the bias), so that the lanes of a wave read
// consecutive outputs of one input; eight weights are loaded before they are used.
// An output is computed by g lanes that split its inputs (g = 256 / out rounded down
// to a power of two, at most 64), combined by a butterfly over the g lanes, so thin
// layers keep the workgroup busy.  fp32 products, the same sums as the layer-by-layer
// forward up to their order.
constexpr int kInferSamples = 8;
constexpr int kInferMaxWidth = 512;

struct InferShape {
    int n_layers;
    int width[9];
};

__device__ __forceinline__ void infer_fma(float (&acc)[kInferSamples], float wv, const float *a)
{
    const float4 a0 = *reinterpret_cast<const float4 *>(a);
    const float4 a1 = *reinterpret_cast<const float4 *>(a + 4);
    acc[0] = fmaf(wv, a0.x, acc[0]);
    acc[1] = fmaf(wv, a0.y, acc[1]);
    acc[2] = fmaf(wv, a0.z, acc[2]);
    acc[3] = fmaf(wv, a0.w, acc[3]);
    acc[4] = fmaf(wv, a1.x, acc[4]);
    acc[5] = fmaf(wv, a1.y, acc[5]);
    acc[6] = fmaf(wv, a1.z, acc[6]);
    acc[7] = fmaf(wv, a1.w, acc[7]);
}

__global__ __launch_bounds__(256) void mlp_infer_kernel(InferShape sh, int batch, const float *__restrict__ packed,
                                                         const float *__restrict__ x, float *__restrict__ y)
{
    constexpr int SB = kInferSamples;
    __shared__ __align__(16) float act[2][kInferMaxWidth][SB];
    const int tid = threadIdx.x;
    const int s0 = blockIdx.x * SB;
    const int ns = min(SB, batch - s0);
    const int w0 = sh.width[0];
    for (int e = tid; e < w0 * SB; e += 256) {
        const int s = e / w0, k = e - s * w0;
        act[0][k][s] = s < ns ? x[(long)(s0 + s) * w0 + k] : 0.f;
    }
    __syncthreads();
    const float *p = packed;
    int cur = 0;
    for (int l = 0; l < sh.n_layers; ++l) {
        const int in = sh.width[l], out = sh.width[l + 1];
        const float *Wt = p, *bias = p + (long)out * in;
        p += (long)out * in + out;
        const bool last = l == sh.n_layers - 1;
        int g = 1;
        while (g < 64 && g * 2 * out <= 256) g *= 2;
        const int part = tid & (g - 1);
        for (int o0 = 0; o0 < out * g; o0 += 256) {
            const int o = (o0 + tid) / g;
            const bool live = (o0 + tid) < out * g;
            float acc[SB];
#pragma unroll
            for (int s = 0; s < SB; ++s) acc[s] = 0.f;
            if (live) {
                const float *wc = Wt + o;
                int k = part;
                for (; k + 7 * g < in; k += 8 * g) {
                    float wv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) wv[u] = wc[(long)(k + u * g) * out];
#pragma unroll
                    for (int u = 0; u < 8; ++u) infer_fma(acc, wv[u], &act[cur][k + u * g][0]);
                }
                for (; k < in; k += g) infer_fma(acc, wc[(long)k * out], &act[cur][k][0]);
            }
            for (int m = 1; m < g; m *= 2)
#pragma unroll
                for (int s = 0; s < SB; ++s) acc[s] += __shfl_xor(acc[s], m);
            if (live && part == 0) {
                const float bo = bias[o];
#pragma unroll
                for (int s = 0; s < SB; ++s) {
                    const float v = acc[s] + bo;
                    act[cur ^ 1][o][s] = last ? v : fmaxf(v, 0.f);
                }
            }
        }
        __syncthreads();
        cur ^= 1;
    }
    const int wl = sh.width[sh.n_layers];
    for (int e = tid; e < wl * SB; e += 256) {
        const int s = e / wl, o = e - s * wl;
        if (s < ns) y[(long)(s0 + s) * wl + o] = act[cur][o][s];
    }
}

// Packed inference layout of one layer: W [out][in] -> W^T [in][out], bias copied.
__global__ void mlp_pack_layer_kernel(int in, int out, const float *__restrict__ src, float *__restrict__ dst)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long nw = (long)in * out;
    if (i >= nw + out) return;
    if (i < nw) {
        const int o = (int)(i / in), k = (int)(i - (long)o * in);
        dst[(long)k * out + o] = src[i];
    } else {
        dst[i] = src[i];
    }
}

// Probe features: X[b] = [(xb[b] - xi[b]), lam[b]] * inv_scale, each [dim].
__global__ void warm_features_kernel(int batch, int dim, const float *__restrict__ xi, const float *__restrict__ xb,
                                     const float *__restrict__ lam, float inv_scale, float *__restrict__ X)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)batch * 2 * dim) return;
    const int b = (int)(i / (2 * dim)), f = (int)(i - (long)b * 2 * dim);
    const long e = (long)b * dim + (f < dim ? f : f - dim);
    X[i] = (f < dim ? xb[e] - xi[e] : lam[e]) * inv_scale;
}

// Jump: y[b] = d_xb [dim] / out_scale.  xb_out = xb + d_xb on the free coefficients
// (the boundary ones are already exact); the multiplier of a free coefficient is set
// to xb_out - xi, the value it has at a fixed point of the iteration, and the
// boundary ones keep the probe's.  One thread per coefficient.
__global__ void warm_apply_kernel(int batch, int dims, int nv, const float *__restrict__ y, float out_scale,
                                  const float *__restrict__ xi, const float *__restrict__ xb,
                                  const float *__restrict__ lam, float *__restrict__ xbo, float *__restrict__ lamo)
{
    const int dim = dims * nv;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)batch * dim) return;
    const int m = (int)(i % nv);
    const bool bnd = m <= 2 || m == nv - 1;
    const float xn = bnd ? xb[i] : fmaf(y[i], out_scale, xb[i]);
    xbo[i] = xn;
    lamo[i] = bnd ? lam[i] : xn - xi[i];
}

// Per-sample fallback, one wave per sample: where the jumped state's residual is not
// below the probe's (or is NaN), or the jumped state is not finite, the sample keeps
// the probe state (xb_src, lam_src) and is flagged.
__global__ void warm_fallback_kernel(int batch, int dim, const float *__restrict__ rw, const float *__restrict__ rc,
                                     const float *__restrict__ xs, const float *__restrict__ ls,
                                     float *__restrict__ xb, float *__restrict__ lam, uint32_t *__restrict__ flags)
{
    const int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (b >= batch) return;  // whole waves
    bool finite = true;
    for (int r = lane; r < dim; r += 64) {
        const long e = (long)b * dim + r;
        finite = finite && isfinite(xb[e]) && isfinite(lam[e]);
    }
    const bool bad = __any(!finite) || !(rw[b] <= rc[b]);
    if (bad)
        for (int r = lane; r < dim; r += 64) {
            const long e = (long)b * dim + r;
            xb[e] = xs[e];
            lam[e] = ls[e];
        }
    if (lane == 0 && flags) flags[b] = bad ? 4u : 0u;
}

// ---- fused warm jump on the matrix cores -----------------------------------------
// Features, the whole network and the jump for 16 samples per workgroup in one launch:
// X = [(xb - xi), lam] * in_scale (bf16) in LDS, each layer a row of 16 x 16 output
// tiles of v_mfma_f32_16x16x16_bf16 (the workgroup's 4 waves take the tiles round
// robin; fp32 accumulation, bias and ReLU in the epilogue, the hidden activations back
// to LDS as bf16), the linear output y kept in fp32, then xb_out = xb + out_scale * y on
// the free coefficients with lam_out = xb_out - xi there, boundary coefficients and
// their multipliers unchanged (as trajam_warm_apply).  Weights come pre-packed in the
// MFMA B-operand order (trajam_warm_pack_mfma): one 8-byte load per lane and tile step.
constexpr int kJumpRows = 16;       // samples per workgroup (one MFMA row tile)
constexpr int kJumpMaxWidth = 256;  // every width, padded to 16
constexpr int kJumpMaxLayers = 4;

struct JumpShape {
    int n_layers;
    int width[kJumpMaxLayers + 1];
    long woff[kJumpMaxLayers];  // byte offsets of each layer's packed weights
    long boff[kJumpMaxLayers];  // byte offsets of each layer's bias (fp32, padded to 16)
};

__host__ __device__ constexpr int ceil16(int x) { return (x + 15) / 16; }

// Pack layer l of the flat fp32 parameters (W [out][in] row-major, then b [out]) into the
// B-operand order: tile (nt, kt), lane, 4 bf16 (rows k = kt*16 + 4(lane/16) + i of
// column n = nt*16 + lane%16), zero outside the matrix; bias padded with zeros.
__global__ void warm_pack_layer_kernel(int in, int out, const float *__restrict__ src, short *__restrict__ wdst,
                                       float *__restrict__ bdst)
{
    const int KT = ceil16(in), NT = ceil16(out);
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long nw = (long)NT * KT * 64 * 4;
    if (i < nw) {
        const int q = (int)(i & 3), lane = (int)((i >> 2) & 63);
        const long tile = i >> 8;
        const int kt = (int)(tile % KT), nt = (int)(tile / KT);
        const int n = nt * 16 + (lane & 15), k = kt * 16 + 4 * (lane >> 4) + q;
        wdst[i] = to_bf16((n < out && k < in) ? src[(long)n * in + k] : 0.f);
    } else if (i < nw + NT * 16) {
        const int n = (int)(i - nw);
        bdst[n] = n < out ? src[(long)out * in + n] : 0.f;
    }
}

__global__ __launch_bounds__(256) void warm_jump_kernel(JumpShape sh, int batch, int dims, int nv,
                                                        const unsigned char *__restrict__ packed, float in_scale,
                                                        float out_scale, const float *__restrict__ xi,
                                                        const float *__restrict__ xb, const float *__restrict__ lam,
                                                        float *__restrict__ xbo, float *__restrict__ lamo)
{
    constexpr int R = kJumpRows, LD = kJumpMaxWidth + 8;   // +8 bf16: rows on distinct banks
    __shared__ __align__(16) short act[2][R][LD];
    __shared__ float yout[R][kJumpMaxWidth];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int s0 = blockIdx.x * R;
    const int dim = dims * nv, w0 = sh.width[0];
    for (int e = tid; e < R * ceil16(w0) * 16; e += 256) {
        const int s = e / (ceil16(w0) * 16), f = e - s * ceil16(w0) * 16;
        float v = 0.f;
        if (s0 + s < batch && f < w0 && f < 2 * dim) {
            const long g = (long)(s0 + s) * dim + (f < dim ? f : f - dim);
            v = (f < dim ? xb[g] - xi[g] : lam[g]) * in_scale;
        }
        act[0][s][f] = to_bf16(v);
    }
    __syncthreads();
    int cur = 0;
    const int r16 = lane & 15, kq = 4 * (lane >> 4);
    for (int l = 0; l < sh.n_layers; ++l) {
        const int in = sh.width[l], out = sh.width[l + 1];
        const int KT = ceil16(in), NT = ceil16(out);
        const bool last = l == sh.n_layers - 1;
        const mlp_bf16x4 *W = reinterpret_cast<const mlp_bf16x4 *>(packed + sh.woff[l]);
        const float *bias = reinterpret_cast<const float *>(packed + sh.boff[l]);
        for (int nt = wv; nt < NT; nt += 4) {
            mlp_f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            const mlp_bf16x4 *Wt = W + (long)nt * KT * 64 + lane;
            for (int kt = 0; kt < KT; ++kt) {
                const mlp_bf16x4 a = *reinterpret_cast<const mlp_bf16x4 *>(&act[cur][r16][kt * 16 + kq]);
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, Wt[kt * 64], acc, 0, 0, 0);
            }
            const int n = nt * 16 + r16;
            const float bn = bias[n];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = kq + q;
                const float v = acc[q] + bn;
                if (last) yout[m][n] = v;
                else act[cur ^ 1][m][n] = to_bf16(n < out ? fmaxf(v, 0.f) : 0.f);
            }
        }
        __syncthreads();
        cur ^= 1;
    }
    for (int e = tid; e < R * dim; e += 256) {
        const int s = e / dim, c = e - s * dim;
        if (s0 + s >= batch) continue;
        const long g = (long)(s0 + s) * dim + c;
        const int m = c % nv;
        const bool bnd = m <= 2 || m == nv - 1;
        const float x = xb[g];
        const float xn = bnd ? x : fmaf(yout[s][c], out_scale, x);
        xbo[g] = xn;
        lamo[g] = bnd ? lam[g] : xn - xi[g];
    }
}

// Matrix-core tile shapes (BM x BN x K step) and the choice among them, from timings
// of the network's products on MI355X (batch 16384, widths 22 to 256): 64 x 64 x 32
// for the large-M products; a narrow output (N <= 32) or a weight gradient with few
// rows (M <= 32) takes the matching half-width tile with a 64-deep K step.
constexpr int kMfmaTiles[][3] = {{64, 64, 32}, {64, 32, 64}, {32, 64, 64}};

int mfma_tile_cfg(int M, int N)
{
    if (N <= 32) return 1;
    if (M <= 32) return 2;
    return 0;
}

template <int BM_, int BN_, int KT, int AM, int BMD>
hipError_t launch_mfma_tiles(MfmaGemm g, int slices, hipStream_t st)
{
    g.tiles_m = (g.M + BM_ - 1) / BM_, g.tiles_n = (g.N + BN_ - 1) / BN_;
    gemm_mfma_kernel<BM_, BN_, KT, AM, BMD><<<dim3((unsigned)(g.tiles_m * g.tiles_n), slices), dim3(256), 0, st>>>(g);
    return hipGetLastError();
}

template <int BM_, int BN_, int KT>
hipError_t launch_mfma_modes(const MfmaGemm &g, int am, int bm, int slices, hipStream_t st)
{
    switch (am * 3 + bm) {
    case 0: return launch_mfma_tiles<BM_, BN_, KT, kRows, kRows>(g, slices, st);
    case 1: return launch_mfma_tiles<BM_, BN_, KT, kRows, kKc>(g, slices, st);
    case 2: return launch_mfma_tiles<BM_, BN_, KT, kRows, kKcVec>(g, slices, st);
    case 3: return launch_mfma_tiles<BM_, BN_, KT, kKc, kRows>(g, slices, st);
    case 4: return launch_mfma_tiles<BM_, BN_, KT, kKc, kKc>(g, slices, st);
    case 5: return launch_mfma_tiles<BM_, BN_, KT, kKc, kKcVec>(g, slices, st);
    case 6: return launch_mfma_tiles<BM_, BN_, KT, kKcVec, kRows>(g, slices, st);
    case 7: return launch_mfma_tiles<BM_, BN_, KT, kKcVec, kKc>(g, slices, st);
    case 8: return launch_mfma_tiles<BM_, BN_, KT, kKcVec, kKcVec>(g, slices, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mfma_cfg(int cfg, const MfmaGemm &g, int am, int bm, int slices, hipStream_t st)
{
    switch (cfg) {
    case 0: return launch_mfma_modes<64, 64, 32>(g, am, bm, slices, st);
    case 1: return launch_mfma_modes<64, 32, 64>(g, am, bm, slices, st);
    case 2: return launch_mfma_modes<32, 64, 64>(g, am, bm, slices, st);
    default: return hipErrorInvalidValue;
    }
}

int op_mode(const float *X, long sr, long sk, int K)
{
    if (sk != 1) return kRows;
    return (sr % 4 == 0 && K % 4 == 0 && ((uintptr_t)X & 15) == 0) ? kKcVec : kKc;
}

}  // namespace

int gemm_plan_slices(bool bf16, int M, int N, int K, long space, int *k_chunk)
{
    const int cfg = mfma_tile_cfg(M, N);
    const int tm = bf16 ? kMfmaTiles[cfg][0] : BM, tn = bf16 ? kMfmaTiles[cfg][1] : BN;
    const int tk = bf16 ? kMfmaTiles[cfg][2] : BK;
    const long tiles = (long)((M + tm - 1) / tm) * ((N + tn - 1) / tn);
    // about 512 workgroups, at least 256 of K per slice, partials within the space
    long S = std::max(1L, (512 + tiles - 1) / tiles);
    S = std::min(S, (long)(K / 256));
    const long per = (long)M * N + (bf16 ? M : 0);
    S = std::min(S, space / per);
    if (S <= 1) {
        *k_chunk = K;
        return 1;
    }
    const long kc = ((K + S - 1) / S + tk - 1) / tk * tk;
    *k_chunk = (int)kc;
    return (int)((K + kc - 1) / kc);
}

hipError_t launch_gemm(bool bf16, int M, int N, int K, const float *A, long sam, long sak, const float *B,
                       long sbk, long sbn, float *C, int ldc, int epi, const float *bias, const float *mask,
                       int ldm, hipStream_t st, int slices, int k_chunk, long c_slice, float *rowsum,
                       long rs_slice)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    if (slices < 1 || (slices > 1 && (epi != kEpiNone || (long)(slices - 1) * k_chunk >= K)))
        return hipErrorInvalidValue;
    if (slices == 1) k_chunk = K;
    if (!bf16) {
        if (rowsum) return hipErrorInvalidValue;
        dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, slices);
        hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, epi,
                           bias, mask, ldm, k_chunk, c_slice);
        return hipGetLastError();
    }
    const int cfg = mfma_tile_cfg(M, N);
    if (slices > 1 && k_chunk % kMfmaTiles[cfg][2]) return hipErrorInvalidValue;
    MfmaGemm g;
    g.M = M, g.N = N, g.K = K;
    g.A = A, g.sam = sam, g.sak = sak;
    g.B = B, g.sbk = sbk, g.sbn = sbn;
    g.C = C, g.ldc = ldc, g.c_slice = c_slice, g.k_chunk = k_chunk;
    g.epi = epi, g.bias = bias, g.mask = mask, g.ldm = ldm;
    g.rowsum = rowsum, g.rs_slice = rs_slice;
    g.c_vec = ldc % 4 == 0 && c_slice % 4 == 0 && ((uintptr_t)C & 15) == 0;
    return launch_mfma_cfg(cfg, g, op_mode(A, sam, sak, K), op_mode(B, sbn, sbk, K), slices, st);
}

hipError_t launch_slice_sum(long n, int slices, const float *part, long stride, float *out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(slice_sum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, slices, part,
                       stride, out);
    return hipGetLastError();
}

hipError_t launch_colsum(int rows, int cols, const float *d, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(colsum_kernel, dim3((cols + 63) / 64), dim3(1024), 0, st, rows, cols, d, out);
    return hipGetLastError();
}

hipError_t launch_mse(long count, const float *y, const float *t, float *dy, float *loss, hipStream_t st)
{
    const int parts = (int)std::min<long>(TRAJAM_MLP_MSE_LOSS_FLOATS - 1, (count + 2047) / 2048);
    hipLaunchKernelGGL(mse_part_kernel, dim3(parts), dim3(256), 0, st, count, y, t, dy, loss + 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(256), 0, st, parts, count, loss + 1, loss);
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

hipError_t launch_mlp_pack_infer(int n_layers, const int *width, const float *params, float *packed, hipStream_t st)
{
    long off = 0;
    for (int l = 0; l < n_layers; ++l) {
        const long n = (long)width[l] * width[l + 1] + width[l + 1];
        hipLaunchKernelGGL(mlp_pack_layer_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, width[l],
                           width[l + 1], params + off, packed + off);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        off += n;
    }
    return hipSuccess;
}

hipError_t launch_mlp_infer(int n_layers, const int *width, int batch, const float *params, const float *x,
                            float *y, hipStream_t st)
{
    if (n_layers < 1 || n_layers > 8) return hipErrorInvalidValue;
    InferShape sh{};
    sh.n_layers = n_layers;
    for (int l = 0; l <= n_layers; ++l) {
        if (width[l] < 1 || width[l] > kInferMaxWidth) return hipErrorInvalidValue;
        sh.width[l] = width[l];
    }
    hipLaunchKernelGGL(mlp_infer_kernel, dim3((batch + kInferSamples - 1) / kInferSamples), dim3(256), 0, st, sh,
                       batch, params, x, y);
    return hipGetLastError();
}

hipError_t launch_warm_features(int batch, int dim, const float *xi, const float *xb, const float *lam,
                                float inv_scale, float *X, hipStream_t st)
{
    const long total = (long)batch * 2 * dim;
    hipLaunchKernelGGL(warm_features_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, batch, dim,
                       xi, xb, lam, inv_scale, X);
    return hipGetLastError();
}

hipError_t launch_warm_apply(int batch, int dims, int nv, const float *y, float out_scale, const float *xi,
                             const float *xb, const float *lam, float *xbo, float *lamo, hipStream_t st)
{
    const long total = (long)batch * dims * nv;
    hipLaunchKernelGGL(warm_apply_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, batch, dims, nv,
                       y, out_scale, xi, xb, lam, xbo, lamo);
    return hipGetLastError();
}

// Byte layout of the packed jump parameters (host): per layer the B-operand tiles
// (NT * KT * 64 * 4 bf16), then the bias (NT * 16 fp32), each 16-byte aligned.
static long jump_layout(int n_layers, const int *width, JumpShape &sh)
{
    long off = 0;
    sh.n_layers = n_layers;
    for (int l = 0; l <= n_layers; ++l) sh.width[l] = width[l];
    for (int l = 0; l < n_layers; ++l) {
        const long KT = ceil16(width[l]), NT = ceil16(width[l + 1]);
        sh.woff[l] = off;
        off += NT * KT * 64 * 4 * 2;
        off = (off + 15) / 16 * 16;
        sh.boff[l] = off;
        off += NT * 16 * 4;
        off = (off + 15) / 16 * 16;
    }
    return off;
}

long warm_jump_packed_bytes(int n_layers, const int *width)
{
    if (n_layers < 1 || n_layers > kJumpMaxLayers) return -1;
    for (int l = 0; l <= n_layers; ++l)
        if (width[l] < 1 || width[l] > kJumpMaxWidth) return -1;
    JumpShape sh{};
    return jump_layout(n_layers, width, sh);
}

hipError_t launch_warm_pack_mfma(int n_layers, const int *width, const float *params, void *packed, hipStream_t st)
{
    JumpShape sh{};
    jump_layout(n_layers, width, sh);
    long poff = 0;
    for (int l = 0; l < n_layers; ++l) {
        const int in = width[l], out = width[l + 1];
        const long n = (long)ceil16(out) * ceil16(in) * 256 + ceil16(out) * 16;
        hipLaunchKernelGGL(warm_pack_layer_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out,
                           params + poff, reinterpret_cast<short *>((unsigned char *)packed + sh.woff[l]),
                           reinterpret_cast<float *>((unsigned char *)packed + sh.boff[l]));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        poff += (long)in * out + out;
    }
    return hipSuccess;
}

hipError_t launch_warm_jump(int n_layers, const int *width, int batch, int dims, int nv, const void *packed,
                            float in_scale, float out_scale, const float *xi, const float *xb, const float *lam,
                            float *xbo, float *lamo, hipStream_t st)
{
    JumpShape sh{};
    jump_layout(n_layers, width, sh);
    hipLaunchKernelGGL(warm_jump_kernel, dim3((batch + kJumpRows - 1) / kJumpRows), dim3(256), 0, st, sh, batch,
                       dims, nv, (const unsigned char *)packed, in_scale, out_scale, xi, xb, lam, xbo, lamo);
    return hipGetLastError();
}

hipError_t launch_warm_fallback(int batch, int dim, const float *rw, const float *rc, const float *xs,
                                const float *ls, float *xb, float *lam, uint32_t *flags, hipStream_t st)
{
    hipLaunchKernelGGL(warm_fallback_kernel, dim3((batch + 3) / 4), dim3(256), 0, st, batch, dim, rw, rc, xs, ls, xb,
                       lam, flags);
    return hipGetLastError();
}

// Workspace of trajam_mlp_backward_noalloc: the two ping-pong buffers of the input
// gradients, in a file-scope device array instead of caller memory, for callers that
// cannot allocate.  Every GPU the library runs on holds its own copy until the process
// ends.  In host code `scratch` names a host-side stand-in, so the device address is
// looked up once per device (with that device current) and only that address is ever
// passed to kernels.
constexpr size_t kNoallocScratchFloats = size_t(1) << 21;  // 8 MiB
static __device__ __align__(256) float scratch[kNoallocScratchFloats];

hipError_t noalloc_scratch(float **ptr, size_t *n_floats)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static float *dev_ptr[kMaxDevices] = {};
    int d = -1;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return e;
    if (d < 0 || d >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!dev_ptr[d]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        dev_ptr[d] = static_cast<float *>(p);
    }
    *ptr = dev_ptr[d];
    *n_floats = kNoallocScratchFloats;
    return hipSuccess;
}

}  // namespace trajam
