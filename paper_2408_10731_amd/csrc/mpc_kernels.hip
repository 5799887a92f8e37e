// gfx950 kernel of the receding-horizon loop (thesis ch. 5, Paper II, Implementation
// Details: each control cycle starts from the preceding cycle's solution): every
// sample's coefficients re-expressed on the window shifted by the elapsed time, and
// the multipliers carried over or cleared.
#include <hip/hip_runtime.h>

#include "am_internal.h"

namespace trajam {
namespace {

// One thread per (sample, [agent,] axis) row of n_v coefficients: the row is read
// whole into registers before it is written, so the outputs may alias the inputs.
template <typename T>
__global__ __launch_bounds__(256) void mpc_shift_kernel(int rows, ShiftMatrix S, const T *xb, const T *lam,
                                                        T *xi_next, T *xb_next, T *lam_next, int keep_lambda)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    const int nv = S.nv;
    const size_t base = (size_t)r * nv;
    double x[kShiftMaxCoeffs], l[kShiftMaxCoeffs];
#pragma unroll
    for (int m = 0; m < kShiftMaxCoeffs; ++m) {
        x[m] = m < nv ? (double)xb[base + m] : 0.0;
        l[m] = (m < nv && keep_lambda) ? (double)lam[base + m] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kShiftMaxCoeffs; ++j) {
        if (j >= nv) break;
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < kShiftMaxCoeffs; ++m) acc = fma(S.s[j * kShiftMaxCoeffs + m], x[m], acc);
        xi_next[base + j] = (T)acc;
        xb_next[base + j] = (T)acc;
        lam_next[base + j] = (T)l[j];
    }
}

}  // namespace

hipError_t launch_mpc_shift(bool fp64, int rows, const ShiftMatrix &S, const void *xb, const void *lam,
                            void *xi_next, void *xb_next, void *lam_next, int keep_lambda, hipStream_t st)
{
    if (rows <= 0) return hipSuccess;
    const dim3 grid((rows + 255) / 256);
    if (fp64)
        hipLaunchKernelGGL(mpc_shift_kernel<double>, grid, dim3(256), 0, st, rows, S, (const double *)xb,
                           (const double *)lam, (double *)xi_next, (double *)xb_next, (double *)lam_next,
                           keep_lambda);
    else
        hipLaunchKernelGGL(mpc_shift_kernel<float>, grid, dim3(256), 0, st, rows, S, (const float *)xb,
                           (const float *)lam, (float *)xi_next, (float *)xb_next, (float *)lam_next,
                           keep_lambda);
    return hipGetLastError();
}

}  // namespace trajam
