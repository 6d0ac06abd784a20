/*
 * ctmi_unet -- BF16 kernels of the learned prior used plug-and-play inside
 * CGLS (libctmi.so, gfx950).
 *
 * The paper's discussion of data-driven methods notes that trained networks
 * call the projection operators; it defines no network.  The denoiser here
 * is the builder's: a 3-D residual U-Net with 4 levels of (16, 32, 64, 128)
 * channels, two [3x3x3 conv, zero padding 1, + bias, ReLU] per level, 2x2x2
 * average pooling down, stride-2 2x2x2 transposed convolution (+ bias) up,
 * skip connections by channel concatenation (upsampled channels first), and
 * a 1x1x1 head added to the input.  Weights and activations are BF16 (round
 * to nearest, ties to even), every sum is accumulated in FP32, master
 * weights are FP32 and training uses MSE and Adam.
 *
 * Conventions:
 *   - BF16 values are passed as uint16_t bit patterns;
 *   - activation tensors are channels-last: element (b, z, y, x, c) of a
 *     tensor with row length `ld` sits at ((((b d + z) h + y) w + x) ld + c);
 *     a call uses channels [0, C) of each row, so a slice of a wider tensor
 *     (for example one half of a concatenation) is a pointer offset plus its
 *     `ld`.  ld must be a multiple of 8 and at least C; tensor pointers must
 *     be 16-byte aligned;
 *   - 3x3x3 weights are [cout][27][cin] with tap t = 9 kz + 3 ky + kx reading
 *     the input at (z + kz - 1, y + ky - 1, x + kx - 1), zero outside;
 *     transposed-convolution weights are [cout][8][cin] with sub-position
 *     s = 4 a + 2 b + c writing output voxel (2z + a, 2y + b, 2x + c);
 *   - all pointers are device pointers owned by the caller; outputs must not
 *     overlap inputs; calls are asynchronous on `stream`; return codes are
 *     those of ctmi.h, and argument checks happen before anything is
 *     enqueued.
 */
#ifndef CTMI_UNET_H
#define CTMI_UNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 3x3x3 convolution, forward: out[v][co] = bf16(act(bias[co] +
 * sum_t sum_ci in[v + t][ci] wt[co][t][ci])) over the channel concatenation
 * in = [in0 (c0 channels), in1 (c1 channels)]; in1 may be NULL with c1 = 0.
 * act = ReLU when relu != 0.  c0, c1: multiples of 16; cout in {16, 32, 64,
 * 128}; bias: FP32 [cout] or NULL.  Volume n x d x h x w, any sizes. */
int ctmi_conv3d_bf16_fwd(int n, int d, int h, int w, const uint16_t* in0, int c0, int ld0, const uint16_t* in1,
                         int c1, int ld1, const uint16_t* wt, const float* bias, int cout, int relu, uint16_t* out,
                         int ldo, void* stream);

/* Data gradient of the convolution (its adjoint in the input):
 * dx[u][ci] = bf16(m[u][ci] * sum_t sum_co dz[u - t][co] w[co][t][ci]),
 * m = (mask > 0) when mask is not NULL (the ReLU derivative of the layer that
 * produced the input), else 1.  wd: the flipped, transposed weights
 * wd[ci][26 - t][co] written by ctmi_conv3d_pack_weights.  cin in
 * {16, 32, 64, 128}; cout a multiple of 16. */
int ctmi_conv3d_bf16_dgrad(int n, int d, int h, int w, const uint16_t* dz, int cout, int ldz, const uint16_t* wd,
                           int cin, const uint16_t* mask, int ldm, uint16_t* dx, int ldx, void* stream);

/* Device workspace (bytes) of ctmi_conv3d_bf16_wgrad for these sizes. */
size_t ctmi_conv3d_wgrad_workspace_bytes(int n, int d, int h, int w, int cin, int cout);

/* Weight gradient: dw[co][t][ci] (FP32) = sum_v dz[v][co] in[v + t][ci]
 * and, when db is not NULL, db[co] = sum_v dz[v][co]; added to dw / db when
 * accumulate != 0.  Summation order is fixed (deterministic). */
int ctmi_conv3d_bf16_wgrad(int n, int d, int h, int w, const uint16_t* in0, int c0, int ld0, const uint16_t* in1,
                           int c1, int ld1, const uint16_t* dz, int cout, int ldz, float* dw, float* db,
                           int accumulate, void* ws, size_t ws_bytes, void* stream);

/* FP32 master weights [cout][27][cin] -> BF16 forward weights wf (same
 * layout) and, when wd is not NULL, BF16 data-gradient weights
 * wd[ci][26 - t][co]. */
int ctmi_conv3d_pack_weights(const float* w, int cout, int cin, uint16_t* wf, uint16_t* wd, void* stream);

/* Network input: FP32 volume (nvox values) -> BF16 16-channel rows with
 * channel 0 = bf16(x) and channels 1..15 = 0, so that the first 1-channel
 * convolution runs on the same kernel with zero weights beyond channel 0. */
int ctmi_unet_pack_input(const float* x, int64_t nvox, uint16_t* out, void* stream);

/* 2x2x2 average pooling: out (n x d x h x w) from in (n x 2d x 2h x 2w),
 * c channels (multiple of 8). */
int ctmi_pool2(int n, int d, int h, int w, int c, const uint16_t* in, int ldi, uint16_t* out, int ldo, void* stream);

/* Gradient at a skip tensor e (n x d x h x w, even sizes) that feeds both a
 * pooling and a concatenation: out = bf16((e > 0) * (dp[parent] / 8 + dcat)),
 * dp the gradient at the pooled tensor (n x d/2 x h/2 x w/2), dcat the
 * concatenation gradient's slice for e. */
int ctmi_pool2_skip_grad(int n, int d, int h, int w, int c, const uint16_t* e, int lde, const uint16_t* dp, int ldp,
                         const uint16_t* dcat, int ldc, uint16_t* out, int ldo, void* stream);

/* Stride-2 2x2x2 transposed convolution from x (n x d x h x w, cin
 * channels) to out (n x 2d x 2h x 2w, cout channels):
 * out[2v + s][co] = bf16(bias[co] + sum_ci x[v][ci] wt[co][s][ci]).
 * cin, cout multiples of 8; bias FP32 or NULL. */
int ctmi_upsample2(int n, int d, int h, int w, const uint16_t* x, int cin, int ldx, const uint16_t* wt,
                   const float* bias, int cout, uint16_t* out, int ldo, void* stream);

/* Its data gradient, with the ReLU mask of its input:
 * dx[v][ci] = bf16((below[v][ci] > 0) * sum_s sum_co g[2v + s][co] wt[co][s][ci]);
 * below may be NULL (no mask). */
int ctmi_upsample2_dgrad(int n, int d, int h, int w, const uint16_t* g, int cout, int ldg, const uint16_t* wt, int cin,
                         const uint16_t* below, int ldb, uint16_t* dx, int ldx, void* stream);

/* Device workspace (bytes) of ctmi_upsample2_wgrad. */
size_t ctmi_upsample2_wgrad_workspace_bytes(int n, int d, int h, int w, int cin, int cout);

/* Its weight gradient: dw[co][s][ci] = sum_v g[2v + s][co] x[v][ci] and
 * db[co] = sum g[.][co] (db may be NULL), FP32, deterministic; cin and cout
 * multiples of 16. */
int ctmi_upsample2_wgrad(int n, int d, int h, int w, const uint16_t* x, int cin, int ldx, const uint16_t* g, int cout,
                         int ldg, float* dw, float* db, int accumulate, void* ws, size_t ws_bytes, void* stream);

/* Residual head: out[v] = x_in[v] + hb[0] + sum_c hw[c] act[v][c], FP32
 * output; hw: BF16 [c]; hb: FP32 [1]. */
int ctmi_unet_head(int64_t nvox, const float* xin, const uint16_t* act, int c, int lda, const uint16_t* hw,
                   const float* hb, float* out, void* stream);

/* Device workspace (bytes) of ctmi_unet_head_mse_bwd. */
size_t ctmi_unet_head_workspace_bytes(void);

/* MSE loss L = mean((out - target)^2) through a 16-channel head: with
 * g = 2 (out - target) / nvox, writes dz[v][c] = bf16((act > 0) g hw[c]) and
 * sums[0..15] = sum_v g act[v][c] (the head weight gradient), sums[16] =
 * sum g (the head bias gradient), sums[17] = sum (out - target)^2, all FP64
 * (device doubles), deterministic.  When dhead is not NULL, sums[0..16] are
 * also written there as FP32 (the head's slice of a gradient buffer). */
int ctmi_unet_head_mse_bwd(int64_t nvox, const float* out, const float* target, const uint16_t* act, int lda,
                           const uint16_t* hw, uint16_t* dz, int ldz, double* sums, float* dhead, void* ws,
                           size_t ws_bytes, void* stream);

/* Adam (Kingma & Ba 2015) on FP32 arrays of n values, step t >= 1 (the
 * bias corrections use t): m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
 * w -= (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps). */
int ctmi_adam_step(float* w, float* m, float* v, const float* g, int64_t n, float lr, float beta1, float beta2,
                   float eps, int64_t t, void* stream);

/* out[i] = bf16(a[i]), round to nearest even. */
int ctmi_to_bf16(const float* a, int64_t n, uint16_t* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* CTMI_UNET_H */
