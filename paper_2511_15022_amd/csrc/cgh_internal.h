// Internal declarations shared by the HIP translation units of libcgh.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "cgh.h"

namespace cgh {

constexpr int kTile = 16;          // default rasterizer tile edge, pixels
constexpr int kMaxBatch = CGH_MAX_BATCH;
constexpr int kMaxStages = 16;     // radix stages per FFT length
constexpr int kMaxFft = 8192;      // longest supported FFT
constexpr int kSortBits = 8;       // bits per radix-sort pass
constexpr int kSortItems = 2048;   // keys per radix-sort block (256 threads x 8)
constexpr int kScanItems = 2048;   // elements per scan block (256 threads x 8)

// Mixed-radix (2, 3, 4, 5, 8) Stockham plan for one transform length.
// Stage s has radix r[s]; ns[s] is the product of the radices before it;
// magic[s] = ceil(2^32 / ns[s]) divides exactly for indices < 2^13;
// tws[s] = n / (ns[s] r[s]) is the stride into the length-n twiddle table.
struct FftPlan {
  int n;
  int nstages;
  int radix[kMaxStages];
  int ns[kMaxStages];
  uint32_t magic[kMaxStages];
  int tws[kMaxStages];
};

bool make_plan(int n, FftPlan *plan);
bool smooth235(int n);

// Column-pass limits: even Hp runs as two Hp/2-point chains (Hp/2 <= 1152 in a
// 77 KB LDS block, <= 2400 in 150 KB); odd Hp runs one Hp-point transform
// (<= 2400).  1024-thread workgroups.
constexpr int kColHalfSmall = 1152;
constexpr int kColHalfMax = 2400;
constexpr int kColFullMax = 2400;
bool col_supported(int Hp);
constexpr int kTwTable = 256;      // float2 slots reserved per two-level twiddle table

// Record of one Gaussian for the rasterizer (FP32, written by the FP64
// preprocess).  Offsets within a record of rec_stride floats:
enum RecField {
  R_MIX = 0,   // floor(mean_x), stored as int bits
  R_MIY = 1,   // floor(mean_y), int bits
  R_MFX = 2,   // mean_x - floor(mean_x)
  R_MFY = 3,
  R_A = 4,     // -0.5 log2(e) inv00
  R_B = 5,     // -log2(e) inv01
  R_C = 6,     // -0.5 log2(e) inv11   (log2 G = a dx^2 + b dx dy + c dy^2)
  R_RX = 7,    // k sqrt(Sigma00): half-width of the support box, pixels
  R_RY = 8,    // k sqrt(Sigma11)
  R_AMP = 9    // then alpha c_c cos(phi_c), alpha c_c sin(phi_c) for c < C
};
// After the amplitudes (padded to 4 floats) four more: the exponent along a pixel
// row, log2 G = kappa dy^2 - (ra (dx - s dy))^2, with
enum RecExt {
  RX_S = 0,      // s = Sigma01 / Sigma11 (x offset of the row maximum per unit dy)
  RX_KAPPA = 1,  // kappa = -log2(e) / (2 Sigma11)
  RX_RA = 2      // ra = sqrt(log2(e) inv00 / 2)  (a = -ra^2)
};
inline int rec_ext(int C) { return ((R_AMP + 2 * C) + 3) & ~3; }
inline int rec_stride(int C) { return rec_ext(C) + 4; }
inline int partial_stride(int C) { return ((2 * C + 5) + 3) & ~3; }

// One Adam update (Kingma & Ba, Algorithm 1) of a parameter p with gradient g:
// lr_scaled = lr / (1 - b1^t), inv_sqrt_bc2 = 1 / sqrt(1 - b2^t).
__device__ __forceinline__ void adam_one(float &p, float g, float &m, float &v, float lr_scaled,
                                         float b1, float b2, float eps, float inv_sqrt_bc2) {
  m = fmaf(b1, m, (1.0f - b1) * g);
  v = fmaf(b2, v, (1.0f - b2) * g * g);
  const float denom = sqrtf(v) * inv_sqrt_bc2 + eps;
  p -= lr_scaled * m / denom;
}

// Adam applied by the preprocess adjoint as it produces each Gaussian's
// gradients (cgh_backward_step): the parameters p and moments m, v in the
// parameter layout, with the step's scalars.
struct AdamFuse {
  float *p, *m, *v;
  float lr_scaled, b1, b2, eps, inv_sqrt_bc2;
};

// Bits of the sticky non-finite word (status[3]) of a CGH_CHECK_FINITE context.
constexpr uint32_t kNonFiniteParams = 1u, kNonFiniteGrads = 2u, kNonFiniteLoss = 4u;

struct Ctx {
  cgh_config cfg;
  int H, W, C, L, Hp, Wp, Hq, Wq;   // Hq, Wq: quarter-table extents Hp/2+1, Wp/2+1
  int B;                            // holograms in the context
  int CF;                           // B C: channels of the propagation (hologram-major)
  int Wt;                           // column tiles of 8 in the propagation buffer
  int tile_w, tile_h;               // rasterizer tile, pixels
  int tiles_x, tiles_y;             // tiles of one hologram per row / column
  int tiles_per;                    // tiles_x tiles_y
  int num_tiles, sort_passes;       // num_tiles = B tiles_per (sort keys b tiles_per + tile)
  int64_t gen;                      // rasterize / rasterize_lists calls so far
  double lam[kMaxBatch][CGH_MAX_CHANNELS];  // wavelength of (hologram, colour)
  double zd[kMaxBatch][CGH_MAX_PLANES];     // distance of (hologram, plane)
  int64_t pair_cap;
  int sort_blocks;                  // radix-sort grid (covers pair_cap)
  int rec_stride, part_stride;
  FftPlan plan_x, plan_y, plan_m;   // lengths Wp, Hp, Hp/2 (plan_m unused for odd Hp)
  int last_n;                       // n of the last rasterize (-1: none)
  int num_cu;                       // compute units of the device the context was created on
  // workspace carve (device pointers)
  float2 *tw_x, *tw_y, *tw_m;       // two-level twiddle tables for Wp, Hp, Hp/2
  float2 *twf_x, *twf_m;            // full twiddle tables for Wp and Hp/2 (Hp if odd)
  float2 *htab;                     // [B C][L][Hq][Wq]
  float2 *htab_t;                   // [B C][L][Wq][Hq] (column-major copy), wave column pass only
  float2 *twf_y;                    // full twiddle table for Hp, wave column pass only
  float2 *spec;                     // [B C][Wt][H][8] column-tiled propagation buffer
  float2 *spec_plane;               // per-plane column-pass output (spec itself when L = 1)
  float2 *spec_acc;                 // adjoint sum over planes (spec itself when L = 1)
  float2 *field_tmp;                // [B C][H][W]
  float2 *gfield_tmp;               // [B C][H][W]
  float *rec;                       // [B max_gaussians + 1][rec_stride]; the last is all zeros
  float2 *alim;                     // CGH_PAPER_ALPHA only, else null: [B max_gaussians + 1]
                                    // (lo, hi) exponent limits, log2 G in [lo, .) kept,
                                    // clamped at hi (the last entry (0, 0))
  uint2 *rect;                      // [B max_gaussians] tile rectangles (x0|x1<<16, y0|y1<<16)
  uint32_t *counts;                 // [B max_gaussians]
  uint32_t *offsets;                // [B max_gaussians + 1]
  uint32_t *keys[2], *vals[2];      // [pair_cap] ping-pong (tile id, Gaussian id)
  uint2 *ranges;                    // [num_tiles] [start, end) into the sorted list
  uint32_t *hist;                   // digit-major block histograms: [256 * max(sort_blocks,
                                    // preprocess workgroups)]
  uint32_t *hist_chunks;            // chunk sums of the histogram scans
  uint32_t *scan_tmp;               // partial sums for scans
  float *partials;                  // [pair_cap][part_stride] raster-adjoint partials
  double *loss_part;                // [L][row-pass workgroups] FP64 loss partials (the
                                    // workgroups of hologram b contiguous in each plane)
  // cgh_backward_full only (CGH_FULL_LOSS), else null
  float *ssim_I;                    // [L][C][H][W] intensity
  float2 *ssim_u;                   // [L][C][H][W] propagated field, then 2 dL/dI u
  float *ssim_abc;                  // [3][L][C][H - 10][W - 10] SSIM gradient coefficients
  double *ssim_part;                // [L][C][position tiles] sums of SSIM
  double *mse_part;                 // [L][C][pixel tiles] sums of (I - T)^2
  uint32_t *status;                 // [0] overflow flag, [1] pair total, [2] sticky overflow,
                                    // [3] sticky non-finite bits (kNonFinite*)
  uint32_t *finite_flag;            // status + 3 with CGH_CHECK_FINITE, else null
  int sorted;                       // which ping-pong buffer holds the sorted pairs
  // kernel-class timing (cgh_profile_begin / _end)
  int prof_class;                   // 0: off
  int prof_n;                       // launches recorded
  hipEvent_t *prof_ev;              // 2 * kMaxProf events, created on first use
  int static_dev;                   // device whose static workspace this context uses
                                    // (cgh_create_static), -1 otherwise
};
constexpr int kMaxProf = 256;

cgh_status create_into(const cgh_config *cfg, void *workspace, size_t workspace_bytes,
                       hipStream_t s, Ctx *out);

size_t carve(Ctx *c, char *base);   // returns bytes used (base may be null)
cgh_status report(cgh_status st, const char *fmt, ...);  // sets cgh_last_error()

// The column pass runs one wave per column chain, four chains per column
// (k_col_wave4), for Hp = 4 M with H <= 2 M and M one of the chain lengths it is
// built for (4K: 1080; 1080p: 540; 1024^2 .. 4096^2 pads: 256, 384, 512, 1024); it
// reads the column-major transfer table.  col_wave4_m returns M, or 0 where it does
// not apply.
inline int col_wave4_m(const Ctx &c) {
  if (c.Hp % 4 != 0 || 2 * c.H > c.Hp || c.Wp % 8 != 0) return 0;
  const int M = c.Hp / 4;
  return (M == 1080 || M == 1024 || M == 540 || M == 512 || M == 384 || M == 256) ? M : 0;
}
inline bool col_wave4(const Ctx &c) { return col_wave4_m(c) != 0; }

// ---- launchers (all enqueue on `s`; return hipSuccess or the launch error) ----
hipError_t launch_build_twiddles(float2 *tw, int n, hipStream_t s);
hipError_t launch_build_twiddles_full(float2 *tw, int n, hipStream_t s);
int row_group_rows(const Ctx &c);   // rows per row-pass workgroup
// transfer tables of holograms [b0, b1) from c.lam, c.zd
hipError_t launch_build_transfer(const Ctx &c, int b0, int b1, hipStream_t s);
hipError_t launch_row_fwd(const Ctx &c, const float2 *field, float2 *dst, hipStream_t s);
hipError_t launch_row_inv(const Ctx &c, const float2 *src, float2 *out, hipStream_t s);
// column pass of plane `plane`: src -> dst (may alias); acc adds into dst
hipError_t launch_col_pass(const Ctx &c, int conj_h, int plane, const float2 *src, float2 *dst,
                           int acc, hipStream_t s);
// mask (optional, [L][H][W]): the L_recon weight 1 + mask^2 + target^2
hipError_t launch_row_loss(const Ctx &c, int plane, float2 *buf, const float *target,
                           const float *grad_intensity, const float *mask, float *intensity,
                           float2 *u_out, int make_grad, hipStream_t s);
hipError_t launch_loss_finalize(const Ctx &c, double *loss, hipStream_t s);

// SSIM term of the full loss over the [L][C] images in c.ssim_I against target
int ssim_pos_tiles(const Ctx &c);   // position tiles per image (k_ssim_fwd)
int ssim_pix_tiles(const Ctx &c);   // pixel tiles per image (k_ssim_bwd)
hipError_t launch_ssim_fwd(const Ctx &c, const float *target, hipStream_t s);
// c.ssim_u <- 2 (dL_recon/dI + ssim_weight dL_SSIM/dI) u, and the MSE partials
hipError_t launch_ssim_bwd(const Ctx &c, const float *target, const float *mask,
                           float ssim_weight, hipStream_t s);
hipError_t launch_full_loss_finalize(const Ctx &c, float ssim_weight, double *loss,
                                     hipStream_t s);

// the number of Gaussians of all holograms: B n
inline int64_t total_gaussians(const Ctx &c, int n) { return (int64_t)c.B * n; }
hipError_t launch_preprocess(const Ctx &c, const float *params, int n, hipStream_t s);
hipError_t launch_zero_record(const Ctx &c, hipStream_t s);
hipError_t launch_zero_status(const Ctx &c, hipStream_t s);
hipError_t launch_binning(Ctx &c, int n, hipStream_t s);  // sets c.sorted
hipError_t launch_raster_fwd(const Ctx &c, float2 *field, hipStream_t s);
hipError_t launch_raster_adjoint(const Ctx &c, const float2 *grad_field, hipStream_t s);
// grads may be null when adam is given (the fused Adam step)
hipError_t launch_preprocess_adjoint(const Ctx &c, const float *params, int n, float *grads,
                                     hipStream_t s, const AdamFuse *adam = nullptr);

hipError_t launch_adan(float *p, const float *g, float *m, float *d, float *s, float *gprev,
                       int64_t count, int t, float lr, float b1, float b2, float b3, float eps,
                       float wd, const float *lr_groups, int n, int C, hipStream_t st);
hipError_t launch_zero_pair(float *a, float *b, int64_t count, hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t count, float lr,
                       float step_size_scale, float beta1, float beta2, float eps,
                       float inv_sqrt_bc2, const float *lr_groups, int n, int C,
                       hipStream_t s);

}  // namespace cgh

// the host handle of a context
struct cgh_ctx {
  cgh::Ctx c;
};

namespace cgh {
// frees the static workspace of a cgh_create_static context for the next one
void release_static(cgh_ctx *ctx);
}  // namespace cgh
