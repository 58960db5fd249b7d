/*
 * cgh.h -- C ABI of the MI355X (gfx950) library for complex-valued 2D Gaussian
 * computer-generated holography: differentiable rasterization of N complex 2D
 * Gaussians into the SLM-plane field, band-limited angular-spectrum (BLASM)
 * propagation, the MSE loss on |u|^2, their adjoints, and an Adam step.
 *
 * The calls follow the paper's optimisation loop (Alg. 1): ComplexRasterize2D
 * -> ZeroPad -> MultiPlanePropagate -> loss -> optimiser step, with the
 * problem statement of Sec. 3 (target I in R^{C x H x W}, hologram in
 * C^{C x H x W}).
 *
 * Conventions shared by every entry point
 *  - Memory: every buffer pointer is a DEVICE pointer owned by the caller and
 *    must stay valid until the work queued on `stream` has finished.  The
 *    library allocates no device memory: all scratch lives in the caller's
 *    workspace (size from cgh_workspace_size), so peak memory is the caller's.
 *    Pointers must be 16-byte aligned.
 *  - Streams: `stream` is a hipStream_t (NULL = legacy default stream).  Every
 *    call only enqueues work on it and returns without waiting, except
 *    cgh_create (which builds its tables on the stream and waits for them)
 *    and cgh_read_status (which waits for the stream).
 *  - Errors: argument errors are detected on the host before anything is
 *    enqueued and return a non-zero cgh_status; cgh_last_error() then returns
 *    a message (thread-local).  Launch failures return CGH_ERR_DEVICE.
 *    Pair-list overflow is detected on the device and reported by
 *    cgh_read_status.  No C++ exception crosses this interface.
 *  - Threads: a context may be used by one host thread at a time.
 *  - Batches: a context may hold B = cgh_config.batch holograms of one size
 *    (each with its own Gaussians, target and optics; every kernel then runs
 *    over all of them in one launch).  With B > 1 the arrays below gain a
 *    hologram dimension: parameters and gradients [B][n (6 + 2C)] (each
 *    hologram's block in the layout below), field [B][C][H][W], and every
 *    per-plane array [L][B][C][H][W] (for each plane, the holograms act as
 *    further channels of the propagation); masks [L][B][H][W]; loss [B][2].
 *    B = 1 is the single-hologram layout.
 *
 * Layouts
 *  - Complex values are interleaved float pairs (re, im), cgh_c64 below --
 *    the layout of torch.complex64.
 *  - Field:     [C][H][W] complex, row-major, x (column) fastest.
 *  - Intensity: [L][C][H][W] float.  Target: same layout.
 *  - Parameters (pre-activation, Sec. 3.1 and the supplementary activation
 *    functions), one flat float array of n * (6 + 2C) values holding, in this
 *    order, contiguous blocks:
 *        mean_pre [n][2]  (x~: mean = (tanh(x~) + 1)/2 * [W, H], pixels)
 *        log_scale[n][2]  (s~: scale = exp(s~) + 0.1)
 *        rotation [n]     (theta, radians)
 *        amplitude[n][C]  (c, unconstrained)
 *        phase    [n][C]  (phi, radians)
 *        opacity  [n]     (alpha~: alpha = sigmoid(alpha~))
 *    Gradients use the same layout.  Pixel (i, j) sits at the point (i, j)
 *    of the same frame as the mean (0-based, i = column).
 */
#ifndef CGH_H
#define CGH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  float re, im;
} cgh_c64;

typedef enum {
  CGH_OK = 0,
  CGH_ERR_INVALID_ARG = 1, /* bad size, null or misaligned pointer, unsupported value */
  CGH_ERR_WORKSPACE = 2,   /* workspace smaller than cgh_workspace_size            */
  CGH_ERR_CAPACITY = 3,    /* pair list overflowed (see cgh_read_status)            */
  CGH_ERR_DEVICE = 4,      /* HIP runtime error                                     */
  CGH_ERR_UNSUPPORTED = 5, /* valid request the library does not implement          */
  CGH_ERR_STATE = 6,       /* call order violated (e.g. adjoint before rasterize)   */
  CGH_ERR_NONFINITE = 7    /* NaN or Inf met by a CGH_CHECK_FINITE context          */
} cgh_status;

#define CGH_MAX_CHANNELS 4
#define CGH_MAX_PLANES 8
#define CGH_MAX_BATCH 64

/* Geometry and optics of one hologram problem. */
typedef struct {
  int32_t height, width;         /* H, W: SLM pixels (1 .. 8192 each)                     */
  int32_t channels;              /* C: 1 .. CGH_MAX_CHANNELS, one wavelength each          */
  int32_t pad_height, pad_width; /* padded FFT grid Hp >= H, Wp >= W; each must factor     */
                                 /* into 2, 3, 5 and be <= 8192 (0 = 2H, 2W)               */
  double pitch_m;                /* pixel pitch (square pixels), metres                   */
  double wavelength_m[CGH_MAX_CHANNELS]; /* lambda per channel, metres                   */
  int32_t num_planes;            /* L: propagation distances, 1 <= L <= CGH_MAX_PLANES    */
  double z_m[CGH_MAX_PLANES];    /* propagation distance per plane, metres (any sign)     */
  float support_sigma;           /* k: a Gaussian covers the pixels with Mahalanobis      */
                                 /* distance q <= k^2 (k <= 0: every pixel)               */
  int32_t max_gaussians;         /* capacity for n (per hologram)                         */
  int64_t max_pairs;             /* capacity of the (tile, Gaussian) list (0: default     */
                                 /* K B max_gaussians + 65536, K = 16 for 8 x 8 tiles,    */
                                 /* else 8)                                               */
  int32_t flags;                 /* 0, or CGH_FULL_LOSS, CGH_PAPER_ALPHA, CGH_CHECK_FINITE */
  double aperture;               /* circular aperture of Alg. 3 in the frequency plane:   */
                                 /* keep the bins of the padded grid with                 */
                                 /* kx^2 + ky^2 < aperture^2 (signed bin indices, centred */
                                 /* on the zero frequency); 0: none                       */
  int32_t tile_w, tile_h;        /* rasterizer tile in pixels: 16 x 16, 32 x 8, 16 x 8 or */
                                 /* 8 x 8 (0, 0: 16 x 16).  Results do not depend on it   */
                                 /* beyond FP32 rounding (pixel offsets are formed from   */
                                 /* the tile origin; the adjoint's partial sums per tile) */
  int32_t batch;                 /* B: holograms of this size in the context, 1 .. 64     */
                                 /* (0: 1); wavelength_m and z_m give every hologram's    */
                                 /* optics at creation (cgh_set_hologram_optics changes   */
                                 /* one); needs flags without CGH_FULL_LOSS when B > 1    */
} cgh_config;

/* cgh_config.flags: reserve the workspace of cgh_backward_full (the SSIM term:
 * intensity, propagated field and three coefficient maps per plane and
 * channel, about 24 bytes per element of [L][C][H][W]); needs H, W >= 11. */
#define CGH_FULL_LOSS 1
/* cgh_config.flags: the weight of Alg. 2 instead of the coherent-sum equations
 * of Sec. 3.1 and the supplementary rendering: a Gaussian contributes
 * c_{n,c} w exp(j phi_{n,c}) with w = min(0.99, alpha_n G_n), and nothing where
 * alpha_n G_n < 1/255 (on top of the k-sigma support).  Forward and every
 * adjoint follow it (w does not depend on alpha or the geometry where the
 * 0.99 clamp is active).  Costs 8 bytes per Gaussian of workspace. */
#define CGH_PAPER_ALPHA 2
/* cgh_config.flags: check for NaN and Inf on the device: the parameters read by
 * cgh_rasterize and cgh_rasterize_lists, the gradients written by every
 * backward and rasterizer adjoint, and the loss.  A non-finite value sets a
 * sticky device word that cgh_read_status reports as CGH_ERR_NONFINITE (and
 * then clears).  Costs one compare per value and no extra launch. */
#define CGH_CHECK_FINITE 4

typedef struct cgh_ctx cgh_ctx;

/* Bytes of device workspace a context with this configuration needs: the FFT
 * twiddle tables, the FP64-built transfer functions (Sec. 2 equation for H;
 * Alg. 3), the column-tiled propagation buffers of the padded grid (Alg. 1
 * ZeroPad), the Gaussian records and (tile, Gaussian) lists of Alg. 2, and the
 * rasterizer adjoint's per-pair partial sums.  Host-only; validates the
 * configuration (CGH_ERR_INVALID_ARG on a bad one, CGH_ERR_UNSUPPORTED on a
 * valid one this library does not implement). */
cgh_status cgh_workspace_size(const cgh_config *cfg, size_t *bytes);

/* Creates a context over a caller-owned device workspace (>= cgh_workspace_size
 * bytes, 256-byte aligned).  Builds, on `stream`, the FFT twiddle tables and the
 * band-limited transfer function H(fx, fy; lambda_c, z_l) of every channel and
 * plane in FP64 (Sec. 2 equation for H; supplementary "Spatial Frequency
 * Computation", "Bandlimit Computation", "Transfer Function Evaluation"), rounds
 * it to complex64, and waits for the stream.  *out receives a host handle. */
cgh_status cgh_create(const cgh_config *cfg, void *workspace, size_t workspace_bytes,
                      void *stream, cgh_ctx **out);

/* Releases the host handle (the workspace stays the caller's).  For a context
 * of cgh_create_static: frees the device's static workspace for the next one
 * (work still queued with that context must have finished). */
cgh_status cgh_destroy(cgh_ctx *ctx);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): cgh_create
 * with the library's static workspace, a device array of
 * CGH_STATIC_WORKSPACE_BYTES that each GPU the library runs on holds until the
 * process ends, instead of a caller workspace.  Calls no allocating routine.
 * The context then works with every entry point as any other.
 *  - One static context per device at a time: while one exists on the current
 *    device, another call returns CGH_ERR_STATE (cgh_destroy frees the slot).
 *  - A configuration whose cgh_workspace_size exceeds the array returns
 *    CGH_ERR_WORKSPACE before any device work.
 *  - The array keeps what the last context left in it; creation rebuilds the
 *    tables and clears the status words, as cgh_create does, and nothing else
 *    needs to start at zero.  Work of a destroyed static context that is still
 *    running when the next one is created on the same device races with that
 *    creation: synchronise its stream before cgh_destroy.
 * Builds the tables on `stream` and waits for them (as cgh_create). */
#define CGH_STATIC_WORKSPACE_BYTES (64u << 20)
cgh_status cgh_create_static(const cgh_config *cfg, void *stream, cgh_ctx **out);

/* ComplexRasterize2D (Alg. 2; Sec. 3.1 coherent sum; supplementary Forward
 * Pass): field[c][j][i] = sum_n alpha_n c_{n,c} G_n(i, j) exp(j phi_{n,c}) over
 * the Gaussians whose k-sigma ellipse contains (i, j), with
 * G = exp(max(-q/2, -50)) (alpha_n G_n replaced as documented at
 * CGH_PAPER_ALPHA when that flag is set).  params: n * (6 + 2C) floats (layout above),
 * 0 <= n <= max_gaussians (per hologram; B blocks with a batch).  field:
 * [C][H][W] complex ([B][C][H][W]), overwritten.
 * Keeps the per-tile Gaussian lists in the workspace for the adjoint and
 * advances the context's list generation (cgh_generation). */
cgh_status cgh_rasterize(cgh_ctx *ctx, const float *params, int32_t n, cgh_c64 *field,
                         void *stream);

/* Render path (Alg. 1 ZeroPad + MultiPlanePropagate): for each plane l and
 * channel c, u = crop(IFFT2(H(lambda_c, z_l) . FFT2(pad(field_c)))), where pad
 * embeds the field centred in the Hp x Wp grid and crop takes the same window.
 * intensity: [L][C][H][W] = |u|^2 (may be NULL); field_out: [L][C][H][W] complex
 * u (may be NULL).  field is not modified. */
cgh_status cgh_propagate(cgh_ctx *ctx, const cgh_c64 *field, float *intensity,
                         cgh_c64 *field_out, void *stream);

/* Fused loss and adjoint of one optimisation step (Sec. 3.2 L_MSE; supplementary
 * BLASM Backward Pass and rasterizer Backward Pass): propagates `field` (the
 * output of cgh_rasterize for these params), evaluates
 *   L = (1 / (L C H W)) sum (|u|^2 - target)^2,
 * and back-propagates it through |.|^2, the conjugate transfer function with the
 * same band limit, and the rasterizer.
 *   target   : [L][C][H][W] float.
 *   loss     : device double[2] <- {L, 10 log10(1 / L)} (may be NULL).
 *   grad_field: [C][H][W] complex <- dL/dRe(U0) + j dL/dIm(U0) (may be NULL:
 *              the workspace holds it).
 *   grads    : n * (6 + 2C) floats <- dL/dparams (pre-activation; layout above).
 * Precondition: the last cgh_rasterize on this context used the same n and
 * params (CGH_ERR_STATE if n differs). */
cgh_status cgh_backward(cgh_ctx *ctx, const float *params, int32_t n, const cgh_c64 *field,
                        const float *target, double *loss, cgh_c64 *grad_field, float *grads,
                        void *stream);

/* One whole optimisation step after cgh_rasterize: cgh_backward followed by the
 * Adam update of cgh_step (uniform learning rate), fused: the per-Gaussian
 * stage of the rasterizer adjoint applies Adam (Kingma & Ba, Algorithm 1) to
 * each Gaussian's 6 + 2C parameters as it produces their gradients, so the
 * gradients make no round trip through memory before the update.  The results
 * (params, m, v, loss, grad_field and grads) are bitwise those of cgh_backward
 * and then cgh_step with lr_groups = NULL.
 *   params : n * (6 + 2C) floats, updated in place (read first, as cgh_backward).
 *   grads  : dL/dparams as cgh_backward, or NULL (not stored).
 *   m, v   : the Adam moments, same layout, updated in place (zero before t = 1).
 *   t, lr, beta1, beta2, eps: as cgh_step.
 * Other arguments, outputs and preconditions as cgh_backward; the Adam
 * arguments are checked as in cgh_step (CGH_ERR_INVALID_ARG). */
cgh_status cgh_backward_step(cgh_ctx *ctx, float *params, int32_t n, const cgh_c64 *field,
                             const float *target, double *loss, cgh_c64 *grad_field,
                             float *grads, float *m, float *v, int32_t t, float lr, float beta1,
                             float beta2, float eps, void *stream);

/* cgh_backward with the reconstruction loss of Sec. 3.2 (L_recon) in place of
 * L_MSE: per plane l the sum of ||I_l - T_l||^2, ||I_l M_l - T_l M_l||^2 and
 * ||I_l T_l - T_l T_l||^2, averaged over planes; as for L_MSE each squared norm
 * is taken as a mean over its C H W elements, so
 *   L = (1 / (L C H W)) sum (|u|^2 - target)^2 (1 + mask^2 + target^2).
 *   mask : [L][H][W] float, the per-plane depth mask M_l (binary in the paper;
 *          any real weight is accepted), shared by the channels.
 * Other arguments, outputs and preconditions as cgh_backward; loss[1] is
 * 10 log10(1 / L).  The SSIM term of the paper's final loss is in
 * cgh_backward_full. */
cgh_status cgh_backward_recon(cgh_ctx *ctx, const float *params, int32_t n,
                              const cgh_c64 *field, const float *target, const float *mask,
                              double *loss, cgh_c64 *grad_field, float *grads, void *stream);

/* The paper's final training loss (Sec. 3.2, L = L_recon + lambda_1 L_SSIM, the
 * paper uses lambda_1 = 0.005) and its adjoint: L_recon as cgh_backward_recon
 * (L_MSE when mask is NULL) plus ssim_weight * L_SSIM, with
 * L_SSIM = 1 - (mean SSIM over planes, channels and window positions).  SSIM
 * is the structural similarity of Wang, Bovik, Sheikh and Simoncelli (2004)
 * between I_l and the target of the same plane and channel: an 11 x 11
 * Gaussian window (standard deviation 1.5, normalised to sum 1) at every
 * position fully inside the H x W image, C1 = 0.01^2, C2 = 0.03^2 (intensities
 * in [0, 1]).  loss[0] = L; loss[1] = 10 log10(1 / MSE) with the plain MSE
 * between I and the target (the reported PSNR).
 * Needs a context created with CGH_FULL_LOSS (else CGH_ERR_STATE) and
 * ssim_weight >= 0 and finite (else CGH_ERR_INVALID_ARG).  Other arguments,
 * outputs and preconditions as cgh_backward_recon, except that mask may be
 * NULL. */
cgh_status cgh_backward_full(cgh_ctx *ctx, const float *params, int32_t n,
                             const cgh_c64 *field, const float *target, const float *mask,
                             float ssim_weight, double *loss, cgh_c64 *grad_field,
                             float *grads, void *stream);

/* Adjoint of cgh_propagate's intensity for an arbitrary loss (supplementary
 * BLASM Backward Pass: the same zero padding, FFT and band limit with the
 * conjugate transfer function, then the crop's adjoint): given
 * grad_intensity = dL/dI ([L][C][H][W]) at I = |u(field)|^2, writes
 * grad_field = dL/dRe(field) + j dL/dIm(field) = sum_l P_l^H (2 dL/dI_l u_l)
 * ([C][H][W]).  Recomputes u from field instead of storing it. */
cgh_status cgh_propagate_adjoint(cgh_ctx *ctx, const cgh_c64 *field,
                                 const float *grad_intensity, cgh_c64 *grad_field,
                                 void *stream);

/* Adjoint of cgh_propagate's field output for an arbitrary seed: given
 * grad_u = dL/dRe(u) + j dL/dIm(u) ([L][C][H][W]), writes grad_field =
 * sum_l P_l^H grad_u[l] ([C][H][W]), the conjugate transfer function with the
 * same band limit (supplementary BLASM Backward Pass).  Used where the loss is
 * not a function of the intensity alone (the Random POH's L_extract). */
cgh_status cgh_propagate_field_adjoint(cgh_ctx *ctx, const cgh_c64 *grad_u, cgh_c64 *grad_field,
                                       void *stream);

/* Adjoint of cgh_rasterize (supplementary rasterizer Backward Pass, items 1-7):
 * grads <- dL/dparams from grad_field = dL/dRe(U0) + j dL/dIm(U0) ([C][H][W]).
 * Recomputes every pixel's Gaussian response from the tile lists instead of
 * storing it.  Same precondition as cgh_backward: the lists must be those of
 * these params (a caller that cannot guarantee it compares cgh_generation
 * with the value after its own rasterize, and on a mismatch rebuilds them
 * with cgh_rasterize_lists first). */
cgh_status cgh_rasterize_adjoint(cgh_ctx *ctx, const float *params, int32_t n,
                                 const cgh_c64 *grad_field, float *grads, void *stream);

/* The list-building part of ComplexRasterize2D (Alg. 2: preprocess, duplicate
 * each Gaussian to the tiles its support box touches, sort by tile) without
 * the per-pixel sum: rebuilds the context's tile lists for `params` so that a
 * rasterizer adjoint can follow, and advances the generation.  The
 * recomputation step of a deferred adjoint (e.g. after other rasterize calls
 * on the same context).  Arguments as cgh_rasterize. */
cgh_status cgh_rasterize_lists(cgh_ctx *ctx, const float *params, int32_t n, void *stream);

/* *generation <- the number of cgh_rasterize / cgh_rasterize_lists calls made
 * on ctx so far (host counter; no device work).  The tile lists in the
 * workspace are those of the call that set the current value. */
cgh_status cgh_generation(cgh_ctx *ctx, int64_t *generation);

/* Adam step (Kingma & Ba, Algorithm 1) over `count` floats, in place:
 *   m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
 *   p <- p - lr / (1 - b1^t) * m / (sqrt(v) / sqrt(1 - b2^t) + eps).
 * t >= 1 is the step number.  lr_groups: optional HOST array of 6 learning
 * rates for the six parameter blocks of the layout above (then count must be
 * n * (6 + 2C) with n = count / (6 + 2 * channels)); NULL: `lr` everywhere.
 * channels is used only with lr_groups. */
cgh_status cgh_step(float *params, const float *grads, float *m, float *v, int64_t count,
                    int32_t t, float lr, float beta1, float beta2, float eps,
                    const float *lr_groups, int32_t channels, void *stream);

/* Adan step (Xie et al., "Adan: Adaptive Nesterov Momentum Algorithm", Algorithm
 * 1, with bias-corrected moments; the optimiser of Sec. 4) over `count` floats,
 * in place, in the decay-rate convention (betas close to 1; the Adan paper's
 * defaults are 0.98, 0.92, 0.99).  With diff = g - prev_grads (0 at t = 1):
 *   m <- b1 m + (1 - b1) g;  d <- b2 d + (1 - b2) diff;
 *   s <- b3 s + (1 - b3) (g + b2 diff)^2;
 *   p <- p (1 - lr wd) - lr (m / (1 - b1^t) + b2 d / (1 - b2^t)) / (sqrt(s / (1 - b3^t)) + eps);
 *   prev_grads <- g.
 * m, d, s, prev_grads: caller-owned state of `count` floats (any contents at
 * t = 1 except that m, d, s must be zero).  lr_groups / channels as cgh_step:
 * per-block learning rates (e.g. the paper's position / scale / rotation /
 * amplitude / phase / opacity rates, cosine-annealed by the caller). */
cgh_status cgh_step_adan(float *params, const float *grads, float *m, float *d, float *s,
                         float *prev_grads, int64_t count, int32_t t, float lr, float beta1,
                         float beta2, float beta3, float eps, float weight_decay,
                         const float *lr_groups, int32_t channels, void *stream);

/* Copies the transfer function of (channel, plane) into `out` (with a batch,
 * channel b C + c is colour c of hologram b), a device array of
 * (Hp/2 + 1) x (Wp/2 + 1) complex: entry [qy][qx] is H at |fy| = qy / (Hp pitch),
 * |fx| = qx / (Wp pitch) (H depends on the frequency only through |fx|, |fy|). */
cgh_status cgh_get_transfer(cgh_ctx *ctx, int32_t channel, int32_t plane, cgh_c64 *out,
                            void *stream);

/* Waits for `stream`, then reports the device-side status of the last
 * rasterize: *pairs <- number of (tile, Gaussian) pairs it needed (may be NULL).
 * Returns CGH_ERR_CAPACITY if that exceeded max_pairs (the field and gradients of
 * that call are then incomplete), or if any rasterize since the previous
 * cgh_read_status on this context did (a solve graph runs many; this part is
 * reported once and then cleared); else CGH_ERR_NONFINITE if a
 * CGH_CHECK_FINITE context met a NaN or Inf since the previous read (the
 * message says where: parameters, gradients or loss; reported once, then
 * cleared); CGH_OK otherwise. */
cgh_status cgh_read_status(cgh_ctx *ctx, void *stream, int64_t *pairs);

/* Kernel classes for cgh_profile_begin. */
#define CGH_KERNEL_PREPROCESS 1         /* FP64 per-Gaussian preprocess                 */
#define CGH_KERNEL_BINNING 2            /* scan, emit, radix sort, tile ranges          */
#define CGH_KERNEL_RASTER 3             /* forward rasterizer                           */
#define CGH_KERNEL_ROW_FFT 4            /* first forward and last adjoint row pass      */
#define CGH_KERNEL_COL_PASS 5           /* column passes (H and conj H)                 */
#define CGH_KERNEL_ROW_LOSS 6           /* middle row pass: |u|^2, loss, adjoint seed   */
#define CGH_KERNEL_LOSS 7               /* loss reduction                               */
#define CGH_KERNEL_RASTER_ADJOINT 8     /* rasterizer adjoint, tile stage               */
#define CGH_KERNEL_PREPROCESS_ADJOINT 9 /* rasterizer adjoint, per-Gaussian FP64 stage  */

/* Timing of one kernel class: after cgh_profile_begin, every launch of that
 * class on this context is bracketed by two HIP events recorded on the stream
 * of the call (at most 256 launches).  cgh_profile_end waits for `stream`
 * and returns the summed event time in ms and the number of launches timed,
 * then stops timing.  Other classes are unaffected; the events add no device
 * work beyond the two timestamps. */
cgh_status cgh_profile_begin(cgh_ctx *ctx, int32_t kernel_class);
cgh_status cgh_profile_end(cgh_ctx *ctx, void *stream, double *total_ms, int32_t *launches);

/* Replaces the wavelengths and propagation distances of an existing context
 * and rebuilds its transfer functions H(fx, fy; lambda_c, z_l) in FP64 on
 * `stream`, the same tables cgh_create builds, so that one context and its
 * workspace serve holograms of one size under different optics.
 *   wavelength_m: HOST array of C values (> 0, finite), metres;
 *   z_m         : HOST array of L values (finite), metres.
 * Stream-ordered: work enqueued earlier on `stream` still reads the old
 * tables; work on other streams must be ordered against this call by the
 * caller.  Argument errors leave the context unchanged.  Does not wait. */
cgh_status cgh_set_optics(cgh_ctx *ctx, const double *wavelength_m, const double *z_m,
                          void *stream);

/* cgh_set_optics for hologram `hologram` (0 .. B - 1) of a batched context
 * only: its C wavelengths and L distances (HOST arrays), its transfer tables
 * rebuilt in FP64 on `stream`.  cgh_set_optics sets every hologram's. */
cgh_status cgh_set_hologram_optics(cgh_ctx *ctx, int32_t hologram, const double *wavelength_m,
                                   const double *z_m, void *stream);

/* A plain-optimiser solve (Alg. 1 with L_MSE and Adam) captured once as a HIP
 * graph, so that one launch replaces the host's per-kernel launches of every
 * step.  Each launch of the graph first zeroes m and v, then, for
 * t = 1 .. steps, runs exactly the kernels of
 *   cgh_rasterize(ctx, params, n, field);
 *   cgh_backward_step(ctx, params, n, field, target, loss_log + 2 (t - 1), NULL, grads,
 *                     m, v, t, lr, beta1, beta2, eps)
 * which give bit for bit the results of cgh_backward and then
 * cgh_step(params, grads, m, v, count, t, lr, beta1, beta2, eps, NULL, C)
 * (count = n (6 + 2C)); grads receives the last step's gradients only.  The graph binds
 * the pointers given here: a launch optimises from whatever params and target
 * hold when it starts and leaves the optimised parameters in params;
 * loss_log (device double[2 steps]) receives {L, 10 log10(1 / L)} before each
 * step.  Buffers and their layouts as in those calls; grads, m and v hold
 * count floats.  steps: 1 .. 10000.  stream must not be NULL (the legacy
 * stream cannot be captured); cgh_solve_create records the graph without
 * running it and returns CGH_ERR_STATE while kernel timing
 * (cgh_profile_begin) is active on ctx.  The context, its workspace and the
 * bound buffers must outlive the solve, and nothing else may use the context
 * while a launch runs (launches on one stream are ordered; across streams the
 * caller orders them). */
typedef struct cgh_solve cgh_solve;
cgh_status cgh_solve_create(cgh_ctx *ctx, float *params, int32_t n, const float *target,
                            cgh_c64 *field, float *grads, float *m, float *v, double *loss_log,
                            int32_t steps, float lr, float beta1, float beta2, float eps,
                            void *stream, cgh_solve **out);
/* Enqueues one launch of the solve's graph on `stream` (not NULL). */
cgh_status cgh_solve_launch(cgh_solve *solve, void *stream);
/* Releases the graph (the buffers stay the caller's). */
cgh_status cgh_solve_destroy(cgh_solve *solve);

/* Message for the last non-OK status returned on this thread. */
const char *cgh_last_error(void);

/* ABI version of this header (CGH_ABI_VERSION). */
#define CGH_ABI_VERSION 4
int32_t cgh_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CGH_H */
