/*
 * splotch_nn.h -- C ABI of the learned x4 upscaler kernels (gfx950 BF16
 * matrix cores, FP32 accumulation).
 *
 * The upscaler is not part of the paper: it reconstructs a full-resolution
 * render from a render at a quarter of the resolution per side.  Network:
 * six 3x3 convolutions (4 -> 32, four 32 -> 32, 32 -> 48; ReLU after all but
 * the last) on the low-resolution input [optical depth R, G, B,
 * log1p(centre count)], a x4 pixel shuffle of the 48 = 3 x 16 output
 * channels, the x4 bilinear upsample of the low-resolution optical depth
 * added as a residual, and the resolve I = 1 - exp(-L) (Eq. 1 with E = A).
 *
 * Conventions:
 *  - Device pointers, NHWC tensors, bf16 = IEEE bfloat16 (2 bytes,
 *    round-to-nearest-even conversions).
 *  - Weights of a layer: bf16 [cout][3][3][cin] (cross-correlation, zero
 *    padding 1, stride 1); bias float [cout].
 *  - Calls queue work on hip_stream (a hipStream_t, NULL = default) and
 *    return without synchronising.  Errors are returned before any launch.
 *  - Channel counts: convolutions take cout in {16, 32, 48} and cin in
 *    1..64 (forward; cin > 32 needs cout <= 32) or 1..32 (weight gradient);
 *    other counts give SPLOTCH_ERR_UNSUPPORTED.  n, h, w >= 1 and
 *    n*h*w < 2^31 (the head and the consistency check: n*16*h*w < 2^31).
 *  - Alignment: tensors whose channel count is a multiple of 8, and all
 *    conv outputs, start on a 16-byte boundary (SPLOTCH_ERR_INVALID_ARG
 *    otherwise); the packed input on an 8-byte boundary.
 */
#ifndef SPLOTCH_NN_H
#define SPLOTCH_NN_H

#include <stddef.h>
#include <stdint.h>

#include "splotch.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * y = conv3x3(x * [mask > 0], w) + bias, then ReLU if relu != 0.
 * x: bf16 [n][h][w][cin].  mask: optional bf16 [n][h][w][cin]; where given,
 * input elements whose mask value is not > 0 count as zero (the ReLU
 * derivative when this call computes a data gradient).  bias: optional
 * float [cout].  y: [n][h][w][cout], float when out_f32 != 0, else bf16.
 */
splotch_status splotch_nn_conv3x3_fwd(const void* x, const void* w, const float* bias,
                                      const void* mask, void* y, int32_t n, int32_t h, int32_t w_,
                                      int32_t cin, int32_t cout, int32_t relu, int32_t out_f32,
                                      void* hip_stream);

/* wt[ci][2-ky][2-kx][co] = w[co][ky][kx][ci] (bf16): the weights with which
 * splotch_nn_conv3x3_fwd computes the data gradient dx from dy. */
splotch_status splotch_nn_flip_weights(const void* w, void* wt, int32_t cin, int32_t cout,
                                       void* hip_stream);

/*
 * Weight and bias gradients, ACCUMULATED into dw (float [cout][3][3][cin])
 * and db (float [cout], may be NULL): dw += sum over pixels of
 * dy'[p][co] x[p + (ky-1, kx-1)][ci], db += sum of dy'[p][co], where
 * dy' = dy * [mask > 0] (mask: optional bf16 [n][h][w][cout], the layer's
 * ReLU output).  x: bf16 [n][h][w][cin]; dy: bf16 [n][h][w][cout].
 */
splotch_status splotch_nn_conv3x3_bwd_weight(const void* x, const void* dy, const void* mask,
                                             float* dw, float* db, int32_t n, int32_t h,
                                             int32_t w_, int32_t cin, int32_t cout,
                                             void* hip_stream);

/* Network input: x[p] = bf16(log1p(L_R), log1p(L_G), log1p(L_B),
 * log1p(count)) from a render's log_accum (float [n][h][w][3]) and
 * center_count (int32 [n][h][w]). */
splotch_status splotch_nn_pack_input(const float* log_accum, const int32_t* center_count,
                                     void* x, int32_t n, int32_t h, int32_t w_,
                                     void* hip_stream);

/*
 * Output head at full resolution H = 4h, W = 4w:
 *   L[n][Y][X][c] = max(0, conv6[n][Y/4][X/4][16c + 4(Y%4) + X%4]
 *                        + bilinear_x4(L_low)[n][Y][X][c])
 *                   (bilinear: half-pixel centres, sources clamped to the
 *                   image; an optical depth is never negative)
 *   rgb = 1 - exp(-L).
 * conv6: float [n][h][w][48]; L_low: float [n][h][w][3]; rgb: float
 * [n][H][W][3]; L_full: optional float [n][H][W][3].  With target (float
 * [n][H][W][3]) given: loss_sum (float, ACCUMULATED) += sum (rgb-target)^2
 * and dconv6 (bf16 [n][h][w][48], optional) = d(mean squared error)/d conv6
 * (zero where the clamp is active).
 */
splotch_status splotch_nn_head(const float* conv6, const float* L_low, float* rgb, float* L_full,
                               const float* target, float* loss_sum, void* dconv6, int32_t n,
                               int32_t h, int32_t w_, void* hip_stream);

/* Adam step on count float parameters (bias-corrected, step >= 1). */
splotch_status splotch_nn_adam(float* p, const float* g, float* m, float* v, int64_t count,
                               float lr, float beta1, float beta2, float eps, int32_t step,
                               void* hip_stream);

/* dst (bf16) = round-to-nearest-even(src (float)), count elements. */
splotch_status splotch_nn_to_bf16(const float* src, void* dst, int64_t count, void* hip_stream);

/*
 * Consistency of a prediction with its low-resolution render: sum over
 * low-resolution pixels p and channels c (ACCUMULATED into *sum_sq) of
 * (exp(-L_low) - exp(-Lc))^2 with Lc the mean of L_full over the 2x2 central
 * full-resolution pixels of p's 4x4 block.  The RMS is
 * sqrt(sum_sq / (3 n h w)).  L_full: float [n][4h][4w][3].
 */
splotch_status splotch_nn_consistency(const float* L_full, const float* L_low, float* sum_sq,
                                      int32_t n, int32_t h, int32_t w_, void* hip_stream);

/* Weights of the six layers: w[k] bf16 [cout][3][3][cin] (16-byte aligned),
 * b[k] float [cout], with (cin, cout) = (4, 32), (32, 32) x 4, (32, 48). */
typedef struct splotch_nn_weights {
  const void* w[6];
  const float* b[6];
} splotch_nn_weights;

/*
 * The consistency check and fallback decision per region of one image (the
 * learned path's plain-render fallback taken region by region).  For each
 * square region of `region` full-resolution pixels (region/4 low-resolution
 * pixels per side; region a multiple of 4, at most 4096), row-major over
 * ceil(4w/region) x ceil(4h/region) regions: m = sqrt(mean over the
 * region's low-resolution pixels p inside the image and channels c of
 * (exp(-L_low) - exp(-Lc))^2), Lc as in splotch_nn_consistency.
 * mask[r] = 1 where m > theta or m is NaN, else 0 (uint8, device);
 * *n_marked (device int32, ACCUMULATED) += the number of marked regions;
 * metric (optional, float per region) receives m.  The mask is laid out as
 * splotch_image.region_mask with region_size = region.
 * L_full: float [4h][4w][3]; L_low: float [h][w][3].
 */
splotch_status splotch_nn_region_check(const float* L_full, const float* L_low, int32_t h,
                                      int32_t w_, int32_t region, float theta, float* metric,
                                      uint8_t* mask, int32_t* n_marked, void* hip_stream);

/* Workspace bytes of splotch_nn_upscale for n images of h x w low-resolution
 * pixels: the packed input and two activation buffers (bf16), the last
 * layer's output (float) and the partial sums of the consistency check. */
splotch_status splotch_nn_upscale_workspace_size(int32_t n, int32_t h, int32_t w_,
                                                 size_t* bytes);

/*
 * The whole network on a low-resolution render, in one call: pack the input
 * from log_accum (float [n][h][w][3]) and center_count (int32 [n][h][w]),
 * run the six convolutions, and write the full-resolution image rgb (float
 * [n][4h][4w][3]) and, if given, its optical depth L_full (same shape).
 * With check_sum_sq given (device float; L_full then required) the call sets
 * it to the consistency sum of squares of splotch_nn_consistency, summed in
 * a fixed order (the same inputs give the same bits).  ws: caller
 * workspace (16-byte aligned) of at least splotch_nn_upscale_workspace_size
 * bytes, SPLOTCH_ERR_WORKSPACE if smaller.  The host pointer wts is read
 * during the call only.
 */
splotch_status splotch_nn_upscale(const splotch_nn_weights* wts, const float* log_accum,
                                  const int32_t* center_count, int32_t n, int32_t h, int32_t w_,
                                  float* rgb, float* L_full, float* check_sum_sq, void* ws,
                                  size_t ws_bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SPLOTCH_NN_H */
