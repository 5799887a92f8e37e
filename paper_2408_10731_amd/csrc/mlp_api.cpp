// C-ABI of the warm-start network and the warm-start kernels (no solver handle;
// errors are reported through the thread-local message of trajam_last_error(NULL)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "../../include/trajam.h"
#include "am_internal.h"

namespace trajam {
void set_thread_error(const std::string &msg);  // trajam_api.cpp
}

namespace {

trajam_status fail(trajam_status st, const std::string &m)
{
    trajam::set_thread_error(m);
    return st;
}

trajam_status dev(hipError_t e, const char *what)
{
    if (e == hipSuccess) return TRAJAM_OK;
    return fail(TRAJAM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool shape_ok(const trajam_mlp_shape *s)
{
    if (!s || s->n_layers < 1 || s->n_layers > TRAJAM_MLP_MAX_LAYERS) return false;
    for (int l = 0; l <= s->n_layers; ++l)
        if (s->width[l] < 1 || s->width[l] > 65536) return false;
    return true;
}

int64_t count_params(const trajam_mlp_shape *s)
{
    int64_t n = 0;
    for (int l = 0; l < s->n_layers; ++l) n += (int64_t)s->width[l + 1] * s->width[l] + s->width[l + 1];
    return n;
}

}  // namespace

extern "C" trajam_status trajam_mlp_param_count(const trajam_mlp_shape *shape, int64_t *n)
{
    if (!shape_ok(shape) || !n) return fail(TRAJAM_ERR_INVALID, "invalid network shape");
    *n = count_params(shape);
    return TRAJAM_OK;
}

extern "C" trajam_status trajam_mlp_forward(const trajam_mlp_shape *s, int32_t batch, int32_t precision,
                                            const float *params, const float *x, float *acts, float *y,
                                            void *stream)
{
    if (!shape_ok(s)) return fail(TRAJAM_ERR_INVALID, "invalid network shape");
    if (batch < 0 || (precision != 0 && precision != 1)) return fail(TRAJAM_ERR_INVALID, "batch >= 0, precision 0 or 1");
    if (batch == 0) return TRAJAM_OK;
    if (!params || !x || !y || (s->n_layers > 1 && !acts)) return fail(TRAJAM_ERR_INVALID, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    const float *a = x, *p = params;
    float *act = acts;
    for (int l = 0; l < s->n_layers; ++l) {
        const int in = s->width[l], out = s->width[l + 1];
        const float *W = p, *b = p + (int64_t)out * in;
        const bool last = l == s->n_layers - 1;
        float *dst = last ? y : act;
        trajam_status r = dev(trajam::launch_gemm(precision == 1, batch, out, in, a, in, 1, W, 1, in, dst, out,
                                                  last ? 2 : 1, b, nullptr, 0, st),
                              "mlp forward");
        if (r != TRAJAM_OK) return r;
        a = dst;
        if (!last) act += (int64_t)batch * out;
        p += (int64_t)out * in + out;
    }
    return TRAJAM_OK;
}

extern "C" trajam_status trajam_mlp_pack_infer(const trajam_mlp_shape *s, const float *params, float *packed,
                                               void *stream)
{
    if (!shape_ok(s)) return fail(TRAJAM_ERR_INVALID, "invalid network shape");
    if (!params || !packed || params == packed) return fail(TRAJAM_ERR_INVALID, "distinct non-NULL pointers");
    return dev(trajam::launch_mlp_pack_infer(s->n_layers, s->width, params, packed, (hipStream_t)stream),
               "mlp pack");
}

extern "C" trajam_status trajam_mlp_infer(const trajam_mlp_shape *s, int32_t batch, const float *params,
                                          const float *x, float *y, void *stream)
{
    if (!shape_ok(s)) return fail(TRAJAM_ERR_INVALID, "invalid network shape");
    for (int l = 0; l <= s->n_layers; ++l)
        if (s->width[l] > 512) return fail(TRAJAM_ERR_UNSUPPORTED, "trajam_mlp_infer: widths <= 512");
    if (batch < 0) return fail(TRAJAM_ERR_INVALID, "batch >= 0");
    if (batch == 0) return TRAJAM_OK;
    if (!params || !x || !y) return fail(TRAJAM_ERR_INVALID, "NULL pointer");
    return dev(trajam::launch_mlp_infer(s->n_layers, s->width, batch, params, x, y, (hipStream_t)stream), "mlp infer");
}

extern "C" trajam_status trajam_mlp_backward(const trajam_mlp_shape *s, int32_t batch, int32_t precision,
                                             const float *params, const float *x, const float *acts,
                                             const float *dy, float *grads, float *scratch, void *stream)
{
    if (!shape_ok(s)) return fail(TRAJAM_ERR_INVALID, "invalid network shape");
    if (batch < 1 || (precision != 0 && precision != 1)) return fail(TRAJAM_ERR_INVALID, "batch >= 1, precision 0 or 1");
    if (!params || !x || !dy || !grads || (s->n_layers > 1 && (!acts || !scratch)))
        return fail(TRAJAM_ERR_INVALID, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    const int L = s->n_layers;
    // offsets of each layer's parameters and activations
    int64_t poff[TRAJAM_MLP_MAX_LAYERS + 1], aoff[TRAJAM_MLP_MAX_LAYERS + 1];
    poff[0] = 0;
    aoff[1] = 0;
    int maxw = 1;
    for (int l = 0; l < L; ++l) poff[l + 1] = poff[l] + (int64_t)s->width[l + 1] * s->width[l] + s->width[l + 1];
    for (int l = 1; l < L; ++l) {
        aoff[l + 1] = aoff[l] + (int64_t)batch * s->width[l];
        maxw = std::max(maxw, s->width[l]);
    }
    const float *d = dy;
    float *bufs[2] = {scratch, scratch ? scratch + (int64_t)batch * maxw : nullptr};
    // the idle input-gradient buffer (batch * maxw floats) takes the partial products
    // of a weight gradient split over the batch (none for a single-layer network)
    const long space = (L > 1 && scratch) ? (long)batch * maxw : 0;
    const bool bf = precision == 1;
    int which = 0;
    for (int l = L - 1; l >= 0; --l) {
        const int in = s->width[l], out = s->width[l + 1];
        const float *a_prev = (l == 0) ? x : acts + aoff[l];
        float *gW = grads + poff[l], *gb = gW + (int64_t)out * in;
        // dW = d^T a_prev  (M = out, N = in, K = batch); in bf16 mode the bias gradient
        // (the sum of d over the batch) comes out of the same pass over d
        int k_chunk = batch;
        const int S = trajam::gemm_plan_slices(bf, out, in, batch, space, &k_chunk);
        trajam_status r;
        if (S == 1) {
            r = dev(trajam::launch_gemm(bf, out, in, batch, d, 1, out, a_prev, in, 1, gW, in, 0, nullptr, nullptr, 0,
                                        st, 1, batch, 0, bf ? gb : nullptr, 0),
                    "mlp weight gradient");
        } else {
            float *part = bufs[which], *rpart = part + (long)S * out * in;
            r = dev(trajam::launch_gemm(bf, out, in, batch, d, 1, out, a_prev, in, 1, part, in, 0, nullptr, nullptr,
                                        0, st, S, k_chunk, (long)out * in, bf ? rpart : nullptr, out),
                    "mlp weight gradient");
            if (r == TRAJAM_OK)
                r = dev(trajam::launch_slice_sum((long)out * in, S, part, (long)out * in, gW, st),
                        "mlp weight gradient sum");
            if (r == TRAJAM_OK && bf)
                r = dev(trajam::launch_slice_sum(out, S, rpart, out, gb, st), "mlp bias gradient sum");
        }
        if (r != TRAJAM_OK) return r;
        if (!bf) {
            r = dev(trajam::launch_colsum(batch, out, d, gb, st), "mlp bias gradient");
            if (r != TRAJAM_OK) return r;
        }
        if (l > 0) {
            // d_prev = (d W) * [a_prev > 0]  (M = batch, N = in, K = out)
            float *dn = bufs[which];
            which ^= 1;
            const float *W = params + poff[l];
            r = dev(trajam::launch_gemm(precision == 1, batch, in, out, d, out, 1, W, in, 1, dn, in, 3, nullptr,
                                        a_prev, in, st),
                    "mlp input gradient");
            if (r != TRAJAM_OK) return r;
            d = dn;
        }
    }
    return TRAJAM_OK;
}

extern "C" trajam_status trajam_mlp_backward_noalloc(const trajam_mlp_shape *s, int32_t batch,
                                                     int32_t precision, const float *params,
                                                     const float *x, const float *acts, const float *dy,
                                                     float *grads, void *stream)
{
    if (!shape_ok(s)) return fail(TRAJAM_ERR_INVALID, "invalid network shape");
    if (batch < 1 || (precision != 0 && precision != 1)) return fail(TRAJAM_ERR_INVALID, "batch >= 1, precision 0 or 1");
    int64_t maxw = 1;
    for (int l = 1; l < s->n_layers; ++l) maxw = std::max<int64_t>(maxw, s->width[l]);
    const int64_t need = s->n_layers > 1 ? 2 * (int64_t)batch * maxw : 0;
    if (need > (int64_t)TRAJAM_MLP_NOALLOC_SCRATCH_FLOATS)
        return fail(TRAJAM_ERR_CAPACITY, "mlp backward without allocation: 2 * batch * largest hidden width = " +
                                             std::to_string(need) + " floats exceeds the static workspace of " +
                                             std::to_string((int64_t)TRAJAM_MLP_NOALLOC_SCRATCH_FLOATS));
    float *ws = nullptr;
    size_t cap = 0;
    trajam_status r = dev(trajam::noalloc_scratch(&ws, &cap), "mlp backward workspace address");
    if (r != TRAJAM_OK) return r;
    if ((int64_t)cap < (int64_t)TRAJAM_MLP_NOALLOC_SCRATCH_FLOATS)
        return fail(TRAJAM_ERR_DEVICE, "mlp backward workspace smaller than declared");
    // the kernels write every workspace entry they read, so nothing needs clearing
    return trajam_mlp_backward(s, batch, precision, params, x, acts, dy, grads, ws, stream);
}

extern "C" trajam_status trajam_mlp_mse(int64_t count, const float *y, const float *t, float *dy, float *loss,
                                        void *stream)
{
    if (count < 1 || !y || !t || !dy || !loss) return fail(TRAJAM_ERR_INVALID, "count >= 1 and non-NULL pointers");
    return dev(trajam::launch_mse(count, y, t, dy, loss, (hipStream_t)stream), "mse");
}

extern "C" trajam_status trajam_mlp_adam(int64_t n, float *p, const float *g, float *m, float *v, int32_t step,
                                         float lr, float b1, float b2, float eps, void *stream)
{
    if (n < 1 || step < 1 || !p || !g || !m || !v || !(lr > 0.f) || !(b1 >= 0.f && b1 < 1.f) ||
        !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
        return fail(TRAJAM_ERR_INVALID, "invalid Adam arguments");
    return dev(trajam::launch_adam(n, p, g, m, v, step, lr, b1, b2, eps, (hipStream_t)stream), "adam");
}

extern "C" trajam_status trajam_warm_features(int32_t batch, int32_t dims, int32_t nv, const float *xi,
                                              const float *xb, const float *lam, float inv_scale, float *x,
                                              void *stream)
{
    if (batch < 0 || dims < 1 || nv < 1 || !xi || !xb || !lam || !x)
        return fail(TRAJAM_ERR_INVALID, "invalid warm-start feature arguments");
    if (batch == 0) return TRAJAM_OK;
    return dev(trajam::launch_warm_features(batch, dims * nv, xi, xb, lam, inv_scale, x, (hipStream_t)stream),
               "warm features");
}

extern "C" trajam_status trajam_warm_apply(int32_t batch, int32_t dims, int32_t nv, const float *y, float out_scale,
                                           const float *xi, const float *xb, const float *lam, float *xb_out,
                                           float *lam_out, void *stream)
{
    if (batch < 0 || dims < 1 || nv < 4 || !y || !xi || !xb || !lam || !xb_out || !lam_out)
        return fail(TRAJAM_ERR_INVALID, "invalid warm-start apply arguments");
    if (batch == 0) return TRAJAM_OK;
    return dev(trajam::launch_warm_apply(batch, dims, nv, y, out_scale, xi, xb, lam, xb_out, lam_out,
                                         (hipStream_t)stream),
               "warm apply");
}

extern "C" trajam_status trajam_warm_pack_mfma(const trajam_mlp_shape *s, const float *params, void *packed,
                                               int64_t *packed_bytes, void *stream)
{
    if (!shape_ok(s) || !packed_bytes) return fail(TRAJAM_ERR_INVALID, "invalid network shape or NULL size");
    const long need = trajam::warm_jump_packed_bytes(s->n_layers, s->width);
    if (need < 0) return fail(TRAJAM_ERR_UNSUPPORTED, "warm jump: 1..4 layers, every width <= 256");
    *packed_bytes = need;
    if (!packed) return TRAJAM_OK;   // size query
    if (!params) return fail(TRAJAM_ERR_INVALID, "NULL parameters");
    return dev(trajam::launch_warm_pack_mfma(s->n_layers, s->width, params, packed, (hipStream_t)stream),
               "warm pack");
}

extern "C" trajam_status trajam_warm_jump(const trajam_mlp_shape *s, int32_t batch, int32_t dims, int32_t nv,
                                          const void *packed, float in_scale, float out_scale, const float *xi,
                                          const float *xb, const float *lam, float *xb_out, float *lam_out,
                                          void *stream)
{
    if (!shape_ok(s)) return fail(TRAJAM_ERR_INVALID, "invalid network shape");
    if (trajam::warm_jump_packed_bytes(s->n_layers, s->width) < 0)
        return fail(TRAJAM_ERR_UNSUPPORTED, "warm jump: 1..4 layers, every width <= 256");
    if (batch < 0 || dims < 2 || dims > 3 || nv < 4) return fail(TRAJAM_ERR_INVALID, "batch >= 0, dims 2 or 3, nv >= 4");
    if (s->width[0] != 2 * dims * nv || s->width[s->n_layers] != dims * nv)
        return fail(TRAJAM_ERR_INVALID, "warm jump: widths must be 2 dims nv in and dims nv out");
    if (batch == 0) return TRAJAM_OK;
    if (!packed || !xi || !xb || !lam || !xb_out || !lam_out) return fail(TRAJAM_ERR_INVALID, "NULL pointer");
    if (xb_out == xb || lam_out == lam) return fail(TRAJAM_ERR_INVALID, "outputs must not alias xb or lam");
    return dev(trajam::launch_warm_jump(s->n_layers, s->width, batch, dims, nv, packed, in_scale, out_scale, xi, xb,
                                        lam, xb_out, lam_out, (hipStream_t)stream),
               "warm jump");
}

extern "C" trajam_status trajam_warm_fallback(int32_t batch, int32_t dims, int32_t nv, const float *rw,
                                              const float *rc, const float *xb_src, const float *lam_src,
                                              float *xb, float *lam, uint32_t *flags, void *stream)
{
    if (batch < 0 || dims < 1 || nv < 1 || !rw || !rc || !xb_src || !lam_src || !xb || !lam)
        return fail(TRAJAM_ERR_INVALID, "invalid warm-start fallback arguments");
    if (batch == 0) return TRAJAM_OK;
    return dev(trajam::launch_warm_fallback(batch, dims * nv, rw, rc, xb_src, lam_src, xb, lam, flags,
                                            (hipStream_t)stream),
               "warm fallback");
}
