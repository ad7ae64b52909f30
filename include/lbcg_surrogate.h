/*
 * lbcg_surrogate.h -- C ABI of the learned surrogate's gfx950 kernels: a 3D
 * convolutional U-Net trained on snapshots of the colour-gradient LB solver
 * (include/lbcg.h) to predict the phase field rho^N and the velocity u a fixed
 * number of steps ahead, with the LB step as its fallback and judge.
 *
 * Tensors.  Activations are channels-last (N, D, H, W, C) arrays; a view
 * names a channel slice [coff, coff + c) of an array with ctot channels per
 * position, so skip connections can concatenate channels without copies
 * (sg_up2_cat_fwd instead writes a concatenation in whole rows, which is
 * faster where the two parts would otherwise be written as partial lines).
 * Activations are BF16 (MFMA operands), gradients FP32.  Convolution
 * weights are [co][k^3 * ci] (tap-major, channel-minor, tap = (dz+1)*9 +
 * (dy+1)*3 + (dx+1) for k = 3); k is 1 or 3; stride 1; padding 1 for k = 3,
 * periodic along the axes set in periodic_mask (bit 0 x, 1 y, 2 z) and zero
 * elsewhere.  Requirements (else SG_EINVAL): ci, ctot and coff multiples of 8
 * for BF16 views read by the MFMA kernels; co a multiple of 16 in weights
 * (rows beyond the output view's c are computed and dropped).
 *
 * All pointers are caller-owned DEVICE memory; every call is asynchronous on
 * hip_stream (NULL = default stream) and returns 0 or a negative code.
 */
#ifndef LBCG_SURROGATE_H
#define LBCG_SURROGATE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SG_OK 0
#define SG_EINVAL (-1)
#define SG_EDEVICE (-3)

typedef struct sg_view {
    void *p;                      /* base of the (N, D, H, W, ctot) array */
    int32_t n, d, h, w;
    int32_t ctot, coff, c;        /* channel slice of the view */
    int32_t reserved;
} sg_view;

/* y = act(conv(x, W) + bias).  x: BF16 view with c == ci.  w: BF16 [co][k^3 ci].
 * bias: FP32 with at least max(y.c, y32.c) entries, or NULL.  y: BF16 view (c <= co), or NULL.  y32: FP32 view
 * (c <= co), or NULL.  relu: 1 applies max(0, .) to the stored outputs.
 * accumulate (FP32 output only): 1 adds into y32. */
int sg_conv3d_fwd(const sg_view *x, const void *w, const float *bias, int32_t co, int32_t k,
                  int32_t periodic_mask, int32_t relu, const sg_view *y, const sg_view *y32,
                  int32_t accumulate, void *hip_stream);

/* Weight preparation after an optimiser step: FP32 master [co][k^3 ci] ->
 * BF16 [co_pad][k^3 ci] (rows beyond co zero) and the BF16 flipped transpose
 * [ci_pad][k^3 co8] (co8 = co rounded up to 8; taps mirrored) used by the data
 * gradient: the adjoint convolution is sg_conv3d_fwd with these weights. */
int sg_weight_prep(const float *w32, int32_t co, int32_t ci, int32_t k, void *w_bf16, void *wt_bf16,
                   int32_t co_pad, int32_t ci_pad, void *hip_stream);

/* Weight and bias gradients: dw[co][k^3 ci] = sum_p dy[p][co] x[p + tap][ci],
 * db[co] = sum_p dy[p][co] (FP32, overwritten).  x, dy: BF16 views.  ws: FP32
 * workspace of sg_conv3d_bwd_weight_ws() bytes. */
int64_t sg_conv3d_bwd_weight_ws(const sg_view *dy, int32_t ci, int32_t k);
int sg_conv3d_bwd_weight(const sg_view *x, const sg_view *dy, int32_t k, int32_t periodic_mask,
                         float *dw, float *db, float *ws, int64_t ws_bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the weight and
 * bias gradients of sg_conv3d_bwd_weight, computed by the same kernels with
 * the same partial-sum plan (so the results are equal bit for bit), but with
 * the partial sums in a scratch array inside the library instead of a
 * caller workspace.  The scratch holds SG_NOALLOC_SCRATCH_BYTES (96 MiB) per
 * GPU, reserved when the library's surrogate code is first loaded on that GPU
 * and held until the process ends; the call allocates nothing.  A problem
 * whose sg_conv3d_bwd_weight_ws() exceeds that size returns SG_EINVAL, as do
 * the argument errors of sg_conv3d_bwd_weight.  hip_stream must belong to the
 * calling thread's current device (the scratch of that device is used).  All
 * calls on one GPU share its scratch: calls that overlap in time on that GPU
 * (on different streams, or from different threads) race and give wrong
 * gradients; calls in order on one stream are safe.  Every scratch entry that
 * is read is first written by the same call, so nothing needs clearing. */
#define SG_NOALLOC_SCRATCH_BYTES ((int64_t)96 << 20)
int sg_conv3d_bwd_weight_noalloc(const sg_view *x, const sg_view *dy, int32_t k, int32_t periodic_mask,
                                 float *dw, float *db, void *hip_stream);

/* dyb = BF16(dx * [y > 0]) (mask only when y != NULL): the gradient through
 * a ReLU, cast to the MFMA operand type.  dx: FP32 view, y: BF16 view, dyb:
 * BF16 view, all with the same shape. */
int sg_relu_bwd_cast(const sg_view *dx, const sg_view *y, const sg_view *dyb, void *hip_stream);

/* 2x2x2 average pooling (BF16 -> BF16) and its adjoint (FP32 -> FP32,
 * accumulate optional); nearest 2x upsampling (BF16 -> BF16) and its adjoint
 * (sum of the 8 children, FP32 -> FP32, accumulate optional). */
int sg_pool2_fwd(const sg_view *x, const sg_view *y, void *hip_stream);
int sg_pool2_bwd(const sg_view *dy, const sg_view *dx, int32_t accumulate, void *hip_stream);
int sg_up2_fwd(const sg_view *x, const sg_view *y, void *hip_stream);
int sg_up2_bwd(const sg_view *dy, const sg_view *dx, int32_t accumulate, void *hip_stream);

/* Upsampling into a concatenation: y (BF16, fine) receives in its first x->c
 * channels the nearest 2x upsampling of x (BF16, coarse) and in the next
 * skip->c channels a copy of skip (BF16, y's positions); y->c must equal
 * x->c + skip->c.  Adjacent threads write adjacent 16-byte chunks of y's
 * rows, so a y that interleaves the two parts per position is still written
 * in whole lines.  Channel counts, strides and offsets multiples of 8; y's
 * 8-channel chunk count below 2^31.  SG_EINVAL otherwise. */
int sg_up2_cat_fwd(const sg_view *x, const sg_view *skip, const sg_view *y, void *hip_stream);

/* Mean-squared error of an FP32 view against an FP32 target of the same
 * shape: grad = 2 (out - target) / count into an FP32 view.  loss: device
 * array of 257 doubles; loss[0] receives the mean square, loss[1..256] are
 * per-workgroup partial sums (summed in a fixed order). */
int sg_mse(const sg_view *out, const sg_view *target, const sg_view *grad, double *loss, void *hip_stream);

/* Adam on FP32 master weights (step counts from 1). */
int sg_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float beta1, float beta2,
            float eps, int64_t step, void *hip_stream);

/* Fields <-> network tensors.  pack: planar FP32 fields f[c][node] (node
 * x-fastest over an nx*ny*nz box) from the sub-box starting at (x0,y0,z0)
 * with periodic wrap, divided by scale[c] (host array of nf <= 8 nonzero
 * values, NULL = 1) -> BF16 view (batch item b, channels [0, nf), the rest of
 * the view's channels zeroed) and, if y32 != NULL, the same values into an
 * FP32 view.  unpack: FP32 view (batch item b) times scale[c] -> planar FP32
 * fields of the view's box. */
int sg_pack(const float *f, int32_t nf, int32_t nx, int32_t ny, int32_t nz, int32_t x0, int32_t y0,
            int32_t z0, const float *scale, const sg_view *y, const sg_view *y32, int32_t b, void *hip_stream);
int sg_unpack(const sg_view *x32, int32_t b, const float *scale, float *f, int32_t nf, void *hip_stream);

/* Lift the surrogate's prediction to the fields lbcg_set_fields takes.
 * pred: planar FP32 (rho^N, u_x, u_y, u_z), 4 n values.  out: planar FP64
 * (rho_R, rho_B, u_x, u_y, u_z), 5 n values.  The colour densities are the
 * ones whose phase field (rho^N as defined below Eq. 8, each colour scaled by
 * its initial density) is the predicted rho^N clipped to [-1, 1], and whose
 * pressure p = rho_R cs2R + rho_B cs2B (the colour pressures p_k of Eq. 6)
 * equals the local pressure of the state before the jump, taken from
 * rhoR_prev and rhoB_prev (FP32, n values each), or p_in everywhere when both
 * are NULL.  With the initial densities in pressure balance
 * (rho_R^in cs2R = rho_B^in cs2B) this gives rho_R = p (1 + rho^N) / (2 cs2R),
 * rho_B = p (1 - rho^N) / (2 cs2B).  cs2k = (1 - alpha_k)/2 > 0.
 * Device pointers; SG_EINVAL on a NULL buffer, n <= 0, a non-positive cs2 or
 * p_in, or only one of the two previous-density pointers. */
int sg_lift(const float *pred, int64_t n, const float *rhoR_prev, const float *rhoB_prev, double cs2R, double cs2B,
            double p_in, double *out, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBCG_SURROGATE_H */
