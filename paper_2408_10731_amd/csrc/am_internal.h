// Internal interface between the C-ABI layer (trajam_api.cpp) and the gfx950
// kernels (am_kernels.hip).  Not installed; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trajam {

// Largest workgroup the AM kernels are built for (four wave64s).
constexpr int kMaxThreads = 256;
// Largest Bernstein degree + 1 supported (coefficient registers are sized for it).
constexpr int kMaxCoeffs = 16;

// Everything one fused AM launch needs.  T is double (FP64) or float (FP32 and
// BF16_REFINE).  Passed by value as kernel arguments.
template <typename T>
struct AmArgs {
    int batch;       // samples in this call
    int dims;        // 2 or 3 (read by the ragged kernel's dispatch)
    int n_p;         // time samples
    int nv;          // coefficients per axis (degree + 1)
    int n_o;         // obstacles
    int iters;       // AM iterations in this launch
    int tpad;        // threads per trajectory: n_p rounded up to a multiple of 64
    int tb;          // trajectories per workgroup
    int use_v, use_a;
    int sphere;      // obstacles are spheres/circles of radius axes[j][0]
    int dynamic;     // obstacles move (velocity given)
    T rho, vmax, amax, dt;  // dt = T / (n_p - 1)
    T xiB[3][4];            // closed-form boundary coefficients (xi_0, xi_1, xi_2, xi_n) per axis
    const T *phi;           // [3][n_p][NVP]: rows of P, Pd, Pdd, zero padded to NVP
    const T *W;             // [NVP - 4 rows used: nv - 4][NVP] QP update operator
    const T *obs;           // packed obstacle records [n_o][kObstacleRecord]
    const T *obs_soa;       // grouped inside-test fields [groups][kObstacleFields][group]
    const T *xi;            // [batch][D][nv]
    T *xb;                  // [batch][D][nv] in/out
    T *lam;                 // [batch][D][nv] in/out
    T *res;                 // [iters][batch] or null
    uint32_t *flags;        // [batch] or null
    T *res_max;             // residual-only launches: [batch] or null
    // BF16_REFINE: the QP operator split into bf16 hi and lo parts, and H_ff for the
    // refinement pass (only read when the launch uses the matrix-core QP step).
    const uint16_t *Whi;    // [16][16] bf16 bits of W_ff = H_ff^-1 (zero padded)
    const uint16_t *Wlo;    // [16][16] bf16 bits of W_ff - Whi
    const float *Hmq;       // H_ff [16][16] then H_fb [16][4] (coefficients 0, 1, 2, n), fp32
    // Multi-agent problems (n_agents > 1): samples are joint samples of n_agents
    // trajectories, xi / xb / lam are [batch][n_agents][D][nv].
    int n_agents;
    int cull_lds;           // multi-agent: floats of the per-wave LDS obstacle stage, 0 = none
    T pair_r;               // combined radius of a pair (twice the agent radius)
    const T *W2;            // [NVP][NVP] QP operator of H + n_agents rho P^T P (agent deviations)
    const T *xiB_ag;        // [n_agents][D][4] boundary coefficients per agent
    // Penalty continuation (single robot, wave-per-sample kernel; cont_levels = 0: off):
    // per-level penalties and QP operators, and the per-sample state ContState[batch].
    int cont_levels, cont_window;
    T cont_stall, cont_tol;
    const T *cont_rho;      // [levels]
    const T *cont_W;        // [levels][NVP][NVP]
    void *cont_state;       // [batch] ContState, in/out
    // Workspace bounds (rows G = [-P; P]): use_ws = 0 when the problem has none.
    int use_ws;
    T ws_lo[3], ws_hi[3];
};

// Per-sample state of the penalty continuation (the C ABI's trajam_cont_state).
struct ContState {
    int32_t level;   // index into the penalty ladder
    int32_t count;   // iterations since the last check
    double ref;      // residual at the last check (0 before the first)
};

// Obstacle fields per obstacle in the multi-agent kernels' LDS stage, and the largest
// stage per wave (floats) for which the stage is used (4 waves x 16 KiB).
__host__ __device__ constexpr int stage_fields(int dims, bool sphere) { return sphere ? 2 * dims + 2 : 4 * dims; }
constexpr int kStageMaxFloats = 4096;

// Per-wave LDS scalars of the multi-agent kernels' position exchange (128 entries x
// 4: every agent's position at entries a and a + N).
constexpr int kAgentPosScalars = 512;

// Packed obstacle record length (scalars), any dims.
constexpr int kObstacleRecord = 16;
// Field offsets in the packed record: centre, -velocity, 1/semi-axes, semi-axes,
// -radius^2, radius.
constexpr int kOC = 0, kOW = 3, kOI = 6, kOS = 9, kONR2 = 12, kOR = 13;
// Inside-test fields per obstacle in the grouped layout, and obstacles per group
// (one 64-byte scalar load per field and group in float, 64 bytes in double).
constexpr int kObstacleFields = 10;
template <typename T>
constexpr int kGroupStore = sizeof(T) == 4 ? 16 : 8;
constexpr size_t group_store(size_t scalar) { return scalar == 4 ? 16 : 8; }
inline int obstacle_groups(int n_o, size_t scalar) { return (n_o + (int)group_store(scalar) - 1) / (int)group_store(scalar); }

// Launchers.  Return the HIP error of the launch.  `nvp` is the padded coefficient
// count (8, 12 or 16); `mfma_qp` selects the bf16 matrix-core QP step.
// Kernel variants: several waves per sample (one lane per time sample, tb samples
// per workgroup) or one wave per sample (ceil(n_p / 64) time samples per lane, tb
// samples = waves per workgroup).
constexpr int kVariantMultiWave = 0;
constexpr int kVariantWave = 1;
hipError_t launch_project_f64(int dims, int nvp, int variant, const AmArgs<double> &a,
                              hipStream_t st);
hipError_t launch_project_f32(int dims, int nvp, int variant, bool mfma_qp,
                              const AmArgs<float> &a, hipStream_t st);
hipError_t launch_residual_f64(int dims, int nvp, const AmArgs<double> &a, hipStream_t st);
// Multi-agent joint projection / residuals: one wave per joint sample, one lane per
// agent (n_agents <= 64, nvp 8 or 12), a.tb joint samples per workgroup.
hipError_t launch_agents_f64(int dims, int nvp, const AmArgs<double> &a, hipStream_t st);
hipError_t launch_agents_f32(int dims, int nvp, const AmArgs<float> &a, hipStream_t st);
hipError_t launch_agents_residual_f64(int dims, int nvp, const AmArgs<double> &a, hipStream_t st);
hipError_t launch_agents_residual_f32(int dims, int nvp, const AmArgs<float> &a, hipStream_t st);
hipError_t launch_residual_f32(int dims, int nvp, const AmArgs<float> &a, hipStream_t st);
hipError_t launch_polar_f64(int dims, int nvp, const AmArgs<double> &a, void *al, void *be, void *dd, void *kin,
                            hipStream_t st);
hipError_t launch_polar_f32(int dims, int nvp, const AmArgs<float> &a, void *al, void *be, void *dd, void *kin,
                            hipStream_t st);
hipError_t launch_pack_obstacles_f64(int dims, int n_o, const double *c, const double *w,
                                     const double *s, double *out, double *soa, hipStream_t st);
hipError_t launch_pack_obstacles_f32(int dims, int n_o, const float *c, const float *w,
                                     const float *s, float *out, float *soa, hipStream_t st);

// Sampling-loop kernels (cem_kernels.hip).
hipError_t launch_cem_sample(bool f64, int n, int dim, const void *mu, const void *L, const void *z,
                             void *xi, void *xb, void *lam, hipStream_t st);
hipError_t launch_cem_cost(bool f64, int n, int dims, int nv, int n_p, int nvp, const void *phi,
                           const void *xb, const void *res, double quantum, void *caug, int32_t *rkey,
                           hipStream_t st);
hipError_t launch_cem_select(bool f64, int n, const int32_t *rkey, const void *caug, int n_proj,
                             int n_elite, int32_t *proj, int32_t *elite, hipStream_t st);
hipError_t launch_cem_update(bool f64, int n_elite, int dim, const int32_t *elite, const void *xb,
                             const void *caug, double sigma, double gamma, double eps, void *mu,
                             void *Sigma, void *L, hipStream_t st);

// Receding-horizon window shift (mpc_kernels.hip): S[j][m] row-major, padded to
// kShiftMaxCoeffs; passed by value.
constexpr int kShiftMaxCoeffs = 16;
struct ShiftMatrix {
    double s[kShiftMaxCoeffs * kShiftMaxCoeffs];
    int nv;
};
hipError_t launch_mpc_shift(bool fp64, int rows, const ShiftMatrix &S, const void *xb, const void *lam,
                            void *xi_next, void *xb_next, void *lam_next, int keep_lambda, hipStream_t st);

// Counter-based standard normals (cem_kernels.hip): Philox4x64-10 and Box-Muller.
hipError_t launch_normals(bool f64, long count, uint64_t key, uint64_t counter, void *z, hipStream_t st);

// Warm-start network kernels (mlp_kernels.hip).
// Split of a product over K: the number of slices (1 = no split) whose partial products
// fit in `space` floats (M N each, plus M row sums in bf16 mode), and the K range of
// one slice.
int gemm_plan_slices(bool bf16, int M, int N, int K, long space, int *k_chunk);
// C = A B (epilogue epi on the last slice only when slices == 1); with slices > 1 the
// product of K slice z goes to C + z c_slice.  rowsum (bf16 mode only, may be NULL):
// rowsum[z rs_slice + m] = sum over slice z's k of A(m, k), in fp32.
hipError_t launch_gemm(bool bf16, int M, int N, int K, const float *A, long sam, long sak, const float *B,
                       long sbk, long sbn, float *C, int ldc, int epi, const float *bias, const float *mask,
                       int ldm, hipStream_t st, int slices = 1, int k_chunk = 0, long c_slice = 0,
                       float *rowsum = nullptr, long rs_slice = 0);
hipError_t launch_slice_sum(long n, int slices, const float *part, long stride, float *out, hipStream_t st);
hipError_t launch_colsum(int rows, int cols, const float *d, float *out, hipStream_t st);
hipError_t launch_mse(long count, const float *y, const float *t, float *dy, float *loss, hipStream_t st);
hipError_t launch_adam(long n, float *p, const float *g, float *m, float *v, int step, float lr, float b1,
                       float b2, float eps, hipStream_t st);
hipError_t launch_warm_features(int batch, int dim, const float *xi, const float *xb, const float *lam,
                                float inv_scale, float *X, hipStream_t st);
hipError_t launch_warm_apply(int batch, int dims, int nv, const float *y, float out_scale, const float *xi,
                             const float *xb, const float *lam, float *xbo, float *lamo, hipStream_t st);
hipError_t launch_mlp_infer(int n_layers, const int *width, int batch, const float *packed, const float *x,
                            float *y, hipStream_t st);
hipError_t launch_mlp_pack_infer(int n_layers, const int *width, const float *params, float *packed, hipStream_t st);
hipError_t launch_warm_fallback(int batch, int dim, const float *rw, const float *rc, const float *xs,
                                const float *ls, float *xb, float *lam, uint32_t *flags, hipStream_t st);
// Fused warm jump on the matrix cores (features, network, jump; mlp_kernels.hip).
long warm_jump_packed_bytes(int n_layers, const int *width);
hipError_t launch_warm_pack_mfma(int n_layers, const int *width, const float *params, void *packed, hipStream_t st);
hipError_t launch_warm_jump(int n_layers, const int *width, int batch, int dims, int nv, const void *packed,
                            float in_scale, float out_scale, const float *xi, const float *xb, const float *lam,
                            float *xbo, float *lamo, hipStream_t st);
// Device address (on the current device) and size in floats of the backward pass's
// static workspace; looked up once per device.
hipError_t noalloc_scratch(float **ptr, size_t *n_floats);

// Ragged persistent launch (FP32): zeroes the counter, then runs the work queue.
hipError_t launch_ragged(const AmArgs<float> *probs, const int *offsets, int n_probs, int total, int *counter,
                         int blocks, bool agents, int agent_stage, hipStream_t st);

// Dynamic LDS bytes of one AM workgroup.
size_t project_lds_bytes(int dims, int nvp, int tpad, int tb, size_t scalar);

// Heading / multi-circle variant (heading_kernels.hip).  Device tables in the
// solver's precision: phi [3][n_steps][kHeadingMaxCoeffs] (P, Pd, Pdd), x_des
// [2][n_steps], obs [n_obs][8] (cx, cy, vx, vy, a, b, 1/a, 1/b), W [2 kHeadingMaxCoeffs
// - 4]^2 (inverse of the free block of one position group's Q + rho F'F: free x
// coefficients 3..n-1, then c 0..n), Wpsi [kHeadingMaxCoeffs]^2 (free psi coefficients
// 1..n-1).
constexpr int kHeadingMaxCoeffs = 12;
constexpr int kHeadingMaxCircles = 8;
struct HeadingArgs {
    const void *phi, *x_des, *obs, *W, *Wpsi;
    double radii[kHeadingMaxCircles];
    double bcoef[2][4];   // coefficients 0, 1, 2, n of x and y fixed by the boundary rows
    double bpsi[2];       // coefficients 0, n of psi
    double dt, v_max, a_max, rho;
    int n_circles, n_obs, nv, n_steps;
};
hipError_t launch_heading(bool fp64, const HeadingArgs &a, int batch, int iters, void *state, void *lam,
                          void *trace, hipStream_t st);

}  // namespace trajam
