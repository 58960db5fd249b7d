/* cgh_net.h -- C ABI of the learned initialiser's network kernels (gfx950).
 *
 * A U-Net (Ronneberger, Fischer and Brox 2015) maps a target intensity to the
 * parameters of a lattice of Gaussians, the starting point of the paper's
 * optimisation (Sec. 3.2, Alg. 1; the paper itself starts from random
 * parameters, Sec. 4).  Its layers are 3x3 convolutions with zero padding,
 * ReLU, 2x2 average pooling and nearest 2x upsampling with skip
 * concatenation.  Precision: weights and the activations a convolution reads
 * are BF16 (round to nearest, ties to even), sums are FP32 on the matrix
 * cores (v_mfma_f32_32x32x8 bf16).
 *
 * Layouts: activations NHWC with batch 1, [H][W][C] contiguous; convolution
 * weights [Co][3][3][Ci] with out[y][x][co] = b[co] + sum_{ky,kx,ci}
 * in[y + ky - 1][x + kx - 1][ci] w[co][ky][kx][ci] (in = 0 outside the image).
 * All pointers are device pointers owned by the caller, 16-byte aligned; every
 * call only enqueues work on `stream` and allocates nothing.  Argument errors
 * return CGH_ERR_INVALID_ARG before any launch; cgh_last_error() describes
 * them.
 */
#ifndef CGH_NET_H
#define CGH_NET_H

#include <stddef.h>
#include <stdint.h>

#include "cgh.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef uint16_t cgh_bf16; /* the upper 16 bits of an IEEE binary32 */

/* 3x3 convolution of in = [up(x1) if up else x1, x2] (channels concatenated,
 * x1 first; up repeats each pixel of x1, which is then H/2 x W/2, over a 2x2
 * block).  x1: c1 channels, x2: c2 channels (x2 may be NULL with c2 = 0);
 * c1, c2 multiples of 8; cout a multiple of 8; H, W >= 1 (even when up).
 * w: [cout][3][3][c1 + c2] BF16; bias: [cout] FP32 or NULL.
 * out32 (FP32 [H][W][cout], may be NULL) receives the sum plus bias; out16
 * (BF16, may be NULL) receives the same, after ReLU when relu != 0.  With
 * weights from cgh_net_flip_weights this is also the adjoint of a
 * convolution with respect to its input. */
cgh_status cgh_net_conv3x3(const cgh_bf16 *x1, int32_t c1, int32_t up, const cgh_bf16 *x2,
                           int32_t c2, int32_t H, int32_t W, const cgh_bf16 *w,
                           const float *bias, int32_t cout, int32_t relu, float *out32,
                           cgh_bf16 *out16, void *stream);

/* w_t[ci][ky][kx][co] = w[co][2 - ky][2 - kx][ci]: the weights of the adjoint
 * (input gradient) of the convolution with w ([cout][3][3][cin], BF16). */
cgh_status cgh_net_flip_weights(const cgh_bf16 *w, int32_t cout, int32_t cin, cgh_bf16 *w_t,
                                void *stream);

/* Bytes of scratch cgh_net_conv3x3_wgrad needs for this shape: FP32 partial
 * sums over pixel ranges, and channel-major BF16 copies of dL/dout and of the
 * input (three column-shifted, zero-padded copies). */
size_t cgh_net_wgrad_workspace(int32_t H, int32_t W, int32_t cin, int32_t cout);

/* Weight and bias gradients of the convolution above for dL/dout = gy
 * (BF16 [H][W][cout]): gw[co][ky][kx][ci] = sum_p gy[p][co] in[p + k - 1][ci]
 * and gb[co] = sum_p gy[p][co] (FP32; gb may be NULL), in = [up(x1), x2] as in
 * cgh_net_conv3x3 (same restrictions).  Partial sums over pixel ranges go to
 * `workspace` (>= cgh_net_wgrad_workspace bytes, else CGH_ERR_WORKSPACE;
 * 16-byte aligned, as gy must be) and are added in a fixed order, so the
 * result is deterministic. */
cgh_status cgh_net_conv3x3_wgrad(const cgh_bf16 *x1, int32_t c1, int32_t up, const cgh_bf16 *x2,
                                 int32_t c2, int32_t H, int32_t W, const cgh_bf16 *gy,
                                 int32_t cout, float *gw, float *gb, void *workspace,
                                 size_t workspace_bytes, void *stream);

/* out[i] = BF16(x[i]) (round to nearest, ties to even), i < count. */
cgh_status cgh_net_cast_bf16(const float *x, int64_t count, cgh_bf16 *out, void *stream);

/* Gradient through ReLU into the BF16 input of a convolution's adjoints:
 * out[i] = BF16(g[i] * (a[i] > 0)), where a is the stored (BF16) activation;
 * a == NULL: no ReLU (out = BF16(g)). */
cgh_status cgh_net_relu_grad(const float *g, const cgh_bf16 *a, int64_t count, cgh_bf16 *out,
                             void *stream);

/* 2x2 average pooling, BF16 [H][W][C] -> BF16 [H/2][W/2][C] (H, W even). */
cgh_status cgh_net_pool2(const cgh_bf16 *x, int32_t H, int32_t W, int32_t C, cgh_bf16 *out,
                         void *stream);

/* Adjoint of the upsampling inside a convolution's input: out[y][x][c] =
 * sum_{i,j < 2} g[2y + i][2x + j][c] for the first C channels of g (FP32
 * [H][W][stride]); out: FP32 [H/2][W/2][C]. */
cgh_status cgh_net_up_adjoint(const float *g, int32_t H, int32_t W, int32_t stride, int32_t C,
                              float *out, void *stream);

/* Gradient of an encoder output that feeds both the pooling and a skip:
 * out[y][x][c] = gp[y/2][x/2][c] / 4 + gs[y][x][off + c] (gs rows of `stride`
 * channels); FP32, out [H][W][C]. */
cgh_status cgh_net_grad_combine(const float *gp, const float *gs, int32_t stride, int32_t off,
                                int32_t H, int32_t W, int32_t C, float *out, void *stream);

/* Lattice of gy x gx Gaussians on an H x W canvas with C colour channels:
 * Gaussian k = i gx + j sits at ((j + 1/2) W / gx, (i + 1/2) H / gy) and reads
 * the network output `net` (FP32 [H][W][8 C], one block of 8 per colour) at
 * the pixel containing that point.  Block 0 holds the shared geometry:
 * channels 0, 1 move the mean (pixels, clipped to (1e-3, size - 1e-3)), 2, 3
 * are log-scales minus ln 2, 4 the rotation, 7 the opacity logit plus 1/2;
 * block c holds colour c: 8 c + 5 the amplitude minus 1/2, 8 c + 6 the phase.
 * params: the library's flat layout (cgh.h) for n = gy gx.  Computed in FP64.
 * Requires gy <= H and gx <= W (one pixel per Gaussian), 1 <= C <= 4. */
cgh_status cgh_net_lattice_gather(const float *net, int32_t H, int32_t W, int32_t gy,
                                  int32_t gx, int32_t C, float *params, void *stream);

/* Adjoint of cgh_net_lattice_gather: g_net (FP32 [H][W][8 C], overwritten,
 * zero where no Gaussian reads) from dL/dparams (flat layout). */
cgh_status cgh_net_lattice_scatter(const float *net, const float *grads, int32_t H, int32_t W,
                                   int32_t gy, int32_t gx, int32_t C, float *g_net,
                                   void *stream);

/* The network's input.  cgh_net_sqrt_field: field[i] = sqrt(max(T[i], 0)) + 0 j
 * (complex64, `count` elements), the amplitude whose propagation by -z
 * (cgh_propagate on a context with that distance) gives `back`.
 * cgh_net_features: target and back planar [C][count] (count = H W); out (BF16
 * [H][W][8 C]) holds, in block c of each pixel, [T, sqrt(T), Re back, Im back,
 * |back|, 0, 0, 0] of colour c. */
cgh_status cgh_net_sqrt_field(const float *target, int64_t count, cgh_c64 *field, void *stream);
cgh_status cgh_net_features(const float *target, const cgh_c64 *back, int64_t count, int32_t C,
                            cgh_bf16 *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif
