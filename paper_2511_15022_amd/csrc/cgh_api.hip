// C ABI of libcgh: argument validation, workspace carving, and the sequence of
// kernel launches behind each entry point.  No device allocation happens here:
// every buffer is the caller's or lives in the caller's workspace.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "cgh_internal.h"

namespace {

thread_local char g_err[512] = "";

cgh_status fail(cgh_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

cgh_status device_fail(hipError_t e, const char *where) {
  return fail(CGH_ERR_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

// the error channel of cgh_last_error() for the other source files of the library
cgh_status cgh::report(cgh_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

namespace {

#define CGH_CHECK_LAUNCH(expr, where)              \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return device_fail(e_, where); \
  } while (0)

// Validates cfg and fills the derived sizes of ctx (no pointers).
cgh_status setup(const cgh_config *cfg, cgh::Ctx *c) {
  using namespace cgh;
  if (!cfg) return fail(CGH_ERR_INVALID_ARG, "config is NULL");
  const cgh_config &f = *cfg;
  if (f.height < 1 || f.width < 1 || f.height > kMaxFft || f.width > kMaxFft)
    return fail(CGH_ERR_INVALID_ARG, "height/width must be in [1, %d] (got %d x %d)", kMaxFft,
                f.height, f.width);
  if (f.channels < 1 || f.channels > CGH_MAX_CHANNELS)
    return fail(CGH_ERR_INVALID_ARG, "channels must be in [1, %d] (got %d)", CGH_MAX_CHANNELS,
                f.channels);
  if (f.num_planes < 1 || f.num_planes > CGH_MAX_PLANES)
    return fail(CGH_ERR_INVALID_ARG, "num_planes must be in [1, %d] (got %d)", CGH_MAX_PLANES,
                f.num_planes);
  const int Hp = f.pad_height ? f.pad_height : 2 * f.height;
  const int Wp = f.pad_width ? f.pad_width : 2 * f.width;
  if (Hp < f.height || Wp < f.width)
    return fail(CGH_ERR_INVALID_ARG, "padded grid %d x %d smaller than the SLM %d x %d", Hp, Wp,
                f.height, f.width);
  if (!smooth235(Hp) || !smooth235(Wp) || Hp > kMaxFft || Wp > kMaxFft)
    return fail(CGH_ERR_INVALID_ARG,
                "padded grid %d x %d: each side must factor into 2, 3, 5 and be <= %d", Hp, Wp,
                kMaxFft);
  if (!col_supported(Hp))
    return fail(CGH_ERR_UNSUPPORTED,
                "padded height %d: the library supports even values up to %d and odd values "
                "up to %d", Hp, 2 * kColHalfMax, kColFullMax);
  if (!(f.pitch_m > 0.0) || !std::isfinite(f.pitch_m))
    return fail(CGH_ERR_INVALID_ARG, "pitch must be positive and finite");
  for (int ch = 0; ch < f.channels; ++ch)
    if (!(f.wavelength_m[ch] > 0.0) || !std::isfinite(f.wavelength_m[ch]))
      return fail(CGH_ERR_INVALID_ARG, "wavelength of channel %d must be positive", ch);
  for (int l = 0; l < f.num_planes; ++l)
    if (!std::isfinite(f.z_m[l])) return fail(CGH_ERR_INVALID_ARG, "z of plane %d not finite", l);
  if (!(f.aperture >= 0.0) || !std::isfinite(f.aperture))
    return fail(CGH_ERR_INVALID_ARG, "aperture must be >= 0 and finite");
  if (!std::isfinite(f.support_sigma))
    return fail(CGH_ERR_INVALID_ARG, "support_sigma must be finite");
  if (f.max_gaussians < 0 || f.max_gaussians > (1 << 28))
    return fail(CGH_ERR_INVALID_ARG, "max_gaussians must be in [0, 2^28]");
  if (f.max_pairs < 0 || f.max_pairs > 0x7fffffffLL)
    return fail(CGH_ERR_INVALID_ARG, "max_pairs must be in [0, 2^31)");
  const int32_t known = CGH_FULL_LOSS | CGH_PAPER_ALPHA | CGH_CHECK_FINITE;
  if (f.flags & ~known)
    return fail(CGH_ERR_INVALID_ARG, "flags: unknown bits 0x%x", f.flags & ~known);
  if ((f.flags & CGH_FULL_LOSS) && (f.height < 11 || f.width < 11))
    return fail(CGH_ERR_INVALID_ARG, "CGH_FULL_LOSS needs height, width >= 11 (the SSIM window)");
  const int tw = f.tile_w ? f.tile_w : kTile, th = f.tile_h ? f.tile_h : kTile;
  if ((f.tile_w == 0) != (f.tile_h == 0))
    return fail(CGH_ERR_INVALID_ARG, "tile_w and tile_h must both be 0 or both be set");
  if (!((tw == 16 && th == 16) || (tw == 32 && th == 8) || (tw == 16 && th == 8) ||
        (tw == 8 && th == 8)))
    return fail(CGH_ERR_UNSUPPORTED,
                "tile %d x %d: the rasterizer supports 16 x 16, 32 x 8, 16 x 8 and 8 x 8", tw, th);
  const int B = f.batch ? f.batch : 1;
  if (B < 1 || B > CGH_MAX_BATCH)
    return fail(CGH_ERR_INVALID_ARG, "batch must be in [1, %d] (got %d)", CGH_MAX_BATCH, f.batch);
  if (B > 1 && (f.flags & CGH_FULL_LOSS))
    return fail(CGH_ERR_UNSUPPORTED, "CGH_FULL_LOSS needs a context of one hologram");
  if ((int64_t)B * f.max_gaussians > (1 << 28))
    return fail(CGH_ERR_INVALID_ARG, "batch * max_gaussians must be <= 2^28");

  c->cfg = f;
  c->cfg.pad_height = Hp;
  c->cfg.pad_width = Wp;
  c->H = f.height;
  c->W = f.width;
  c->C = f.channels;
  c->L = f.num_planes;
  c->Hp = Hp;
  c->Wp = Wp;
  c->Hq = Hp / 2 + 1;
  c->Wq = Wp / 2 + 1;
  c->cfg.tile_w = tw;
  c->cfg.tile_h = th;
  c->cfg.batch = B;
  c->B = B;
  c->CF = B * f.channels;
  c->Wt = (Wp + 7) / 8;
  c->tile_w = tw;
  c->tile_h = th;
  c->tiles_x = (f.width + tw - 1) / tw;
  c->tiles_y = (f.height + th - 1) / th;
  c->tiles_per = c->tiles_x * c->tiles_y;
  if ((int64_t)B * c->tiles_per > (1LL << 30))
    return fail(CGH_ERR_INVALID_ARG, "too many tiles (%lld)", (long long)B * c->tiles_per);
  c->num_tiles = B * c->tiles_per;
  int bits = 0;
  while ((1 << bits) < c->num_tiles) ++bits;
  // at least one pass: the last pass also writes the tile ranges
  c->sort_passes = std::max(1, (bits + kSortBits - 1) / kSortBits);
  // about 3 (16 x 16) to 7 (8 x 8) tiles per Gaussian at the synthetic scales
  const int64_t per = tw * th <= 64 ? 16 : 8;
  int64_t cap = f.max_pairs ? f.max_pairs : per * B * f.max_gaussians + 65536;
  if (cap > 0x7fffffffLL) cap = 0x7fffffffLL;
  c->pair_cap = cap;
  c->sort_blocks = (int)((cap + kSortItems - 1) / kSortItems);
  c->rec_stride = rec_stride(c->C);
  c->part_stride = partial_stride(c->C);
  c->last_n = -1;
  c->gen = 0;
  for (int b = 0; b < B; ++b) {
    for (int ch = 0; ch < f.channels; ++ch) c->lam[b][ch] = f.wavelength_m[ch];
    for (int l = 0; l < f.num_planes; ++l) c->zd[b][l] = f.z_m[l];
  }
  c->sorted = 0;
  c->num_cu = 1;
  c->prof_class = 0;
  c->prof_n = 0;
  c->prof_ev = nullptr;
  c->static_dev = -1;
  if (!make_plan(Wp, &c->plan_x) || !make_plan(Hp, &c->plan_y) ||
      !make_plan(Hp % 2 == 0 ? Hp / 2 : Hp, &c->plan_m))
    return fail(CGH_ERR_INVALID_ARG, "cannot plan FFTs of %d and %d", Wp, Hp);
  return CGH_OK;
}

// Brackets the launches of one kernel class with HIP events while that class
// is being profiled (cgh_profile_begin); a no-op otherwise.
struct ProfScope {
  cgh::Ctx &c;
  hipStream_t s;
  bool on;
  ProfScope(cgh::Ctx &c_, int cls, hipStream_t s_) : c(c_), s(s_) {
    on = c.prof_ev && c.prof_class == cls && c.prof_n < cgh::kMaxProf;
    // a launch whose events cannot be recorded is simply not timed
    if (on && hipEventRecord(c.prof_ev[2 * c.prof_n], s) != hipSuccess) on = false;
  }
  ~ProfScope() {
    if (on && hipEventRecord(c.prof_ev[2 * c.prof_n + 1], s) == hipSuccess) ++c.prof_n;
  }
};

}  // namespace

namespace cgh {

size_t carve(Ctx *c, char *base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char * {
    off = (off + 255) & ~(size_t)255;
    char *p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const size_t N = (size_t)c->B * c->cfg.max_gaussians;  // Gaussians of all holograms
  const size_t cap = (size_t)c->pair_cap;
  const size_t HW = (size_t)c->H * c->W;
  c->tw_x = (float2 *)take(sizeof(float2) * kTwTable);
  c->tw_y = (float2 *)take(sizeof(float2) * kTwTable);
  c->tw_m = (float2 *)take(sizeof(float2) * kTwTable);
  // full tables of Wp and Hp entries, each followed (when its length is a
  // multiple of 4) by the contiguous table of the quarter length, the twiddles
  // of the four-chain row and column passes
  c->twf_x = (float2 *)take(sizeof(float2) * (c->Wp + (c->Wp % 4 ? 0 : c->Wp / 4)));
  c->twf_m = (float2 *)take(sizeof(float2) * c->plan_m.n);
  c->htab = (float2 *)take(sizeof(float2) * c->CF * c->L * (size_t)c->Hq * c->Wq);
  const bool wave_cols = col_wave4(*c);
  c->htab_t = wave_cols ? (float2 *)take(sizeof(float2) * c->CF * c->L * (size_t)c->Hq * c->Wq)
                        : nullptr;
  c->twf_y = wave_cols ? (float2 *)take(sizeof(float2) * (c->Hp + c->Hp / 4)) : nullptr;
  const size_t spec_len = (size_t)c->CF * c->Wt * c->H * 8;
  c->spec = (float2 *)take(sizeof(float2) * spec_len);
  // with several planes the shared row spectrum stays in spec; each plane's
  // column pass writes spec_plane, and the adjoint sums the planes in spec_acc
  c->spec_plane = c->L > 1 ? (float2 *)take(sizeof(float2) * spec_len) : c->spec;
  c->spec_acc = c->L > 1 ? (float2 *)take(sizeof(float2) * spec_len) : c->spec;
  c->field_tmp = (float2 *)take(sizeof(float2) * c->CF * HW);
  c->gfield_tmp = (float2 *)take(sizeof(float2) * c->CF * HW);
  c->rec = (float *)take(sizeof(float) * c->rec_stride * (N + 1));
  c->alim = (c->cfg.flags & CGH_PAPER_ALPHA) ? (float2 *)take(sizeof(float2) * (N + 1)) : nullptr;
  c->rect = (uint2 *)take(sizeof(uint2) * (N ? N : 1));
  c->counts = (uint32_t *)take(sizeof(uint32_t) * (N ? N : 1));
  c->offsets = (uint32_t *)take(sizeof(uint32_t) * (N + 1));
  for (int b = 0; b < 2; ++b) {
    c->keys[b] = (uint32_t *)take(sizeof(uint32_t) * cap);
    c->vals[b] = (uint32_t *)take(sizeof(uint32_t) * cap);
  }
  c->ranges = (uint2 *)take(sizeof(uint2) * c->num_tiles);
  // the first sort pass counts per preprocess workgroup (256 Gaussians), the
  // later passes per sort block
  const size_t hist_blocks = std::max((size_t)c->sort_blocks, (N + 255) / 256);
  c->hist = (uint32_t *)take(sizeof(uint32_t) * 256 * hist_blocks);
  const size_t scan_len = std::max(N + 1, (size_t)256 * hist_blocks);
  c->hist_chunks = (uint32_t *)take(sizeof(uint32_t) * (scan_len / kScanItems + 2));
  // chunk sums: per kScanItems of a scan, or per preprocess workgroup (256 Gaussians)
  c->scan_tmp = (uint32_t *)take(sizeof(uint32_t) *
                                 std::max(scan_len / kScanItems + 2, (N + 255) / 256 + 2));
  c->partials = (float *)take(sizeof(float) * c->part_stride * cap);
  const int rg = row_group_rows(*c);  // one loss partial per row-pass workgroup
  c->loss_part = (double *)take(sizeof(double) * c->L * c->CF * (size_t)((c->H + rg - 1) / rg));
  c->status = (uint32_t *)take(sizeof(uint32_t) * 4);
  c->finite_flag = (c->cfg.flags & CGH_CHECK_FINITE) && c->status ? c->status + 3 : nullptr;
  c->ssim_I = nullptr;
  c->ssim_u = nullptr;
  c->ssim_abc = nullptr;
  c->ssim_part = nullptr;
  c->mse_part = nullptr;
  if (c->cfg.flags & CGH_FULL_LOSS) {
    const size_t LC = (size_t)c->L * c->C;
    const size_t valid = (size_t)(c->H - 10) * (c->W - 10);
    c->ssim_I = (float *)take(sizeof(float) * LC * HW);
    c->ssim_u = (float2 *)take(sizeof(float2) * LC * HW);
    c->ssim_abc = (float *)take(sizeof(float) * 3 * LC * valid);
    c->ssim_part = (double *)take(sizeof(double) * LC * ssim_pos_tiles(*c));
    c->mse_part = (double *)take(sizeof(double) * LC * ssim_pix_tiles(*c));
  }
  return (off + 255) & ~(size_t)255;
}

}  // namespace cgh

using cgh::Ctx;

extern "C" {

int32_t cgh_abi_version(void) { return CGH_ABI_VERSION; }

const char *cgh_last_error(void) { return g_err; }

cgh_status cgh_workspace_size(const cgh_config *cfg, size_t *bytes) {
  if (!bytes) return fail(CGH_ERR_INVALID_ARG, "bytes is NULL");
  Ctx c;
  cgh_status st = setup(cfg, &c);
  if (st != CGH_OK) return st;
  *bytes = cgh::carve(&c, nullptr);
  return CGH_OK;
}

}  // extern "C"

// Validates cfg, carves the workspace, builds the tables on the stream and
// waits for them; *out receives the context (no host or device allocation).
cgh_status cgh::create_into(const cgh_config *cfg, void *workspace, size_t workspace_bytes,
                            hipStream_t s, Ctx *out) {
  Ctx c;
  cgh_status st = setup(cfg, &c);
  if (st != CGH_OK) return st;
  const size_t need = cgh::carve(&c, nullptr);
  if (!workspace) return fail(CGH_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)workspace & 255u) != 0)
    return fail(CGH_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (workspace_bytes < need)
    return fail(CGH_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
  cgh::carve(&c, (char *)workspace);
  {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c.num_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return device_fail(e, "cgh_create");
    if (c.num_cu < 1) c.num_cu = 1;
  }
  CGH_CHECK_LAUNCH(cgh::launch_build_twiddles(c.tw_x, c.Wp, s), "twiddles");
  CGH_CHECK_LAUNCH(cgh::launch_build_twiddles(c.tw_y, c.Hp, s), "twiddles");
  CGH_CHECK_LAUNCH(cgh::launch_build_twiddles(c.tw_m, c.plan_m.n, s), "twiddles");
  CGH_CHECK_LAUNCH(cgh::launch_build_twiddles_full(c.twf_x, c.Wp, s), "twiddles");
  if (c.Wp % 4 == 0)
    CGH_CHECK_LAUNCH(cgh::launch_build_twiddles_full(c.twf_x + c.Wp, c.Wp / 4, s), "twiddles");
  CGH_CHECK_LAUNCH(cgh::launch_build_twiddles_full(c.twf_m, c.plan_m.n, s), "twiddles");
  if (c.twf_y) {
    CGH_CHECK_LAUNCH(cgh::launch_build_twiddles_full(c.twf_y, c.Hp, s), "twiddles");
    CGH_CHECK_LAUNCH(cgh::launch_build_twiddles_full(c.twf_y + c.Hp, c.Hp / 4, s), "twiddles");
  }
  CGH_CHECK_LAUNCH(cgh::launch_build_transfer(c, 0, c.B, s), "transfer function");
  CGH_CHECK_LAUNCH(cgh::launch_zero_record(c, s), "zero record");
  CGH_CHECK_LAUNCH(cgh::launch_zero_status(c, s), "zero status");
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return device_fail(e, "cgh_create");
  *out = c;
  return CGH_OK;
}

extern "C" {

cgh_status cgh_create(const cgh_config *cfg, void *workspace, size_t workspace_bytes,
                      void *stream, cgh_ctx **out) {
  if (!out) return fail(CGH_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  Ctx c;
  cgh_status st = cgh::create_into(cfg, workspace, workspace_bytes, (hipStream_t)stream, &c);
  if (st != CGH_OK) return st;
  cgh_ctx *h = new (std::nothrow) cgh_ctx;
  if (!h) return fail(CGH_ERR_INVALID_ARG, "host allocation failed");
  h->c = c;
  *out = h;
  return CGH_OK;
}

cgh_status cgh_destroy(cgh_ctx *ctx) {
  if (ctx && ctx->c.prof_ev) {
    // teardown: a failure to destroy an event leaves nothing to recover
    for (int i = 0; i < 2 * cgh::kMaxProf; ++i) (void)hipEventDestroy(ctx->c.prof_ev[i]);
    delete[] ctx->c.prof_ev;
    ctx->c.prof_ev = nullptr;
  }
  if (ctx && ctx->c.static_dev >= 0) {
    cgh::release_static(ctx);  // the library's own handle: not deleted
    return CGH_OK;
  }
  delete ctx;
  return CGH_OK;
}

static cgh_status check_n(const Ctx &c, int32_t n) {
  if (n < 0 || n > c.cfg.max_gaussians)
    return fail(CGH_ERR_INVALID_ARG, "n = %d outside [0, max_gaussians = %d]", n,
                c.cfg.max_gaussians);
  return CGH_OK;
}

// preprocess and binning of Alg. 2: the tile lists of params, a new generation
static cgh_status build_lists(Ctx &c, const float *params, int32_t n, hipStream_t s) {
  {
    ProfScope p(c, CGH_KERNEL_PREPROCESS, s);
    CGH_CHECK_LAUNCH(cgh::launch_preprocess(c, params, n, s), "preprocess");
  }
  {
    ProfScope p(c, CGH_KERNEL_BINNING, s);
    CGH_CHECK_LAUNCH(cgh::launch_binning(c, n, s), "binning");
  }
  c.last_n = n;
  ++c.gen;
  return CGH_OK;
}

cgh_status cgh_rasterize(cgh_ctx *ctx, const float *params, int32_t n, cgh_c64 *field,
                         void *stream) {
  if (!ctx) return fail(CGH_ERR_INVALID_ARG, "ctx is NULL");
  Ctx &c = ctx->c;
  cgh_status st = check_n(c, n);
  if (st != CGH_OK) return st;
  if ((n > 0 && !params) || !field) return fail(CGH_ERR_INVALID_ARG, "params/field is NULL");
  if (!aligned16(field)) return fail(CGH_ERR_INVALID_ARG, "field must be 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  st = build_lists(c, params, n, s);
  if (st != CGH_OK) return st;
  ProfScope p(c, CGH_KERNEL_RASTER, s);
  CGH_CHECK_LAUNCH(cgh::launch_raster_fwd(c, reinterpret_cast<float2 *>(field), s), "raster");
  return CGH_OK;
}

cgh_status cgh_rasterize_lists(cgh_ctx *ctx, const float *params, int32_t n, void *stream) {
  if (!ctx) return fail(CGH_ERR_INVALID_ARG, "ctx is NULL");
  Ctx &c = ctx->c;
  cgh_status st = check_n(c, n);
  if (st != CGH_OK) return st;
  if (n > 0 && !params) return fail(CGH_ERR_INVALID_ARG, "params is NULL");
  return build_lists(c, params, n, (hipStream_t)stream);
}

cgh_status cgh_generation(cgh_ctx *ctx, int64_t *generation) {
  if (!ctx || !generation) return fail(CGH_ERR_INVALID_ARG, "ctx/generation is NULL");
  *generation = ctx->c.gen;
  return CGH_OK;
}

// F1: field -> row spectrum in c.spec (shared by every plane)
static cgh_status row_spectrum(Ctx &c, const cgh_c64 *field, hipStream_t s) {
  ProfScope p(c, CGH_KERNEL_ROW_FFT, s);
  CGH_CHECK_LAUNCH(cgh::launch_row_fwd(c, reinterpret_cast<const float2 *>(field), c.spec, s),
                   "row fft");
  return CGH_OK;
}

// F2 of plane l: c.spec -> c.spec_plane (in place when L = 1)
static cgh_status plane_spectrum(Ctx &c, int l, hipStream_t s) {
  ProfScope p(c, CGH_KERNEL_COL_PASS, s);
  CGH_CHECK_LAUNCH(cgh::launch_col_pass(c, 0, l, c.spec, c.spec_plane, 0, s), "column pass");
  return CGH_OK;
}

// B1 of plane l: the adjoint seed in c.spec_plane -> c.spec_acc (summed over
// planes: the first plane writes, the others add)
static cgh_status plane_adjoint(Ctx &c, int l, hipStream_t s) {
  ProfScope p(c, CGH_KERNEL_COL_PASS, s);
  CGH_CHECK_LAUNCH(cgh::launch_col_pass(c, 1, l, c.spec_plane, c.spec_acc, l > 0, s),
                   "adjoint column pass");
  return CGH_OK;
}

// rasterizer adjoint: tile stage, then the FP64 per-Gaussian stage
static cgh_status raster_adjoint(Ctx &c, const float *params, int n, const float2 *gf,
                                 float *grads, hipStream_t s,
                                 const cgh::AdamFuse *adam = nullptr) {
  {
    ProfScope p(c, CGH_KERNEL_RASTER_ADJOINT, s);
    CGH_CHECK_LAUNCH(cgh::launch_raster_adjoint(c, gf, s), "raster adjoint");
  }
  {
    ProfScope p(c, CGH_KERNEL_PREPROCESS_ADJOINT, s);
    CGH_CHECK_LAUNCH(cgh::launch_preprocess_adjoint(c, params, n, grads, s, adam),
                     "preprocess adjoint");
  }
  return CGH_OK;
}

// B2: c.spec_acc -> dL/dU0
static cgh_status adjoint_rows(Ctx &c, float2 *grad_field, hipStream_t s) {
  ProfScope p(c, CGH_KERNEL_ROW_FFT, s);
  CGH_CHECK_LAUNCH(cgh::launch_row_inv(c, c.spec_acc, grad_field, s), "adjoint row fft");
  return CGH_OK;
}

cgh_status cgh_propagate(cgh_ctx *ctx, const cgh_c64 *field, float *intensity,
                         cgh_c64 *field_out, void *stream) {
  if (!ctx) return fail(CGH_ERR_INVALID_ARG, "ctx is NULL");
  Ctx &c = ctx->c;
  if (!field) return fail(CGH_ERR_INVALID_ARG, "field is NULL");
  if (!aligned16(field) || !aligned16(intensity) || !aligned16(field_out))
    return fail(CGH_ERR_INVALID_ARG, "buffers must be 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  cgh_status st = row_spectrum(c, field, s);
  if (st != CGH_OK) return st;
  for (int l = 0; l < c.L; ++l) {
    st = plane_spectrum(c, l, s);
    if (st != CGH_OK) return st;
    ProfScope p(c, CGH_KERNEL_ROW_LOSS, s);
    CGH_CHECK_LAUNCH(cgh::launch_row_loss(c, l, c.spec_plane, nullptr, nullptr, nullptr,
                                          intensity, reinterpret_cast<float2 *>(field_out), 0,
                                          s),
                     "intensity row pass");
  }
  return CGH_OK;
}

// the fused loss and adjoint of cgh_backward / cgh_backward_recon
static cgh_status backward_impl(cgh_ctx *ctx, const float *params, int32_t n,
                                const cgh_c64 *field, const float *target, const float *mask,
                                double *loss, cgh_c64 *grad_field, float *grads,
                                void *stream, const cgh::AdamFuse *adam = nullptr) {
  if (!ctx) return fail(CGH_ERR_INVALID_ARG, "ctx is NULL");
  Ctx &c = ctx->c;
  cgh_status st = check_n(c, n);
  if (st != CGH_OK) return st;
  if (n != c.last_n)
    return fail(CGH_ERR_STATE, "backward with n = %d after rasterize with n = %d", n, c.last_n);
  if (!field || !target || (n > 0 && (!params || (!grads && !adam))))
    return fail(CGH_ERR_INVALID_ARG, "field/target/params/grads is NULL");
  if (!aligned16(field) || !aligned16(grad_field) || ((uintptr_t)loss & 7u))
    return fail(CGH_ERR_INVALID_ARG, "misaligned buffer");
  hipStream_t s = (hipStream_t)stream;
  float2 *gf = grad_field ? reinterpret_cast<float2 *>(grad_field) : c.gfield_tmp;
  st = row_spectrum(c, field, s);
  if (st != CGH_OK) return st;
  for (int l = 0; l < c.L; ++l) {
    st = plane_spectrum(c, l, s);
    if (st != CGH_OK) return st;
    {
      ProfScope p(c, CGH_KERNEL_ROW_LOSS, s);
      CGH_CHECK_LAUNCH(cgh::launch_row_loss(c, l, c.spec_plane, target, nullptr, mask, nullptr,
                                            nullptr, 1, s),
                       "loss row pass");
    }
    st = plane_adjoint(c, l, s);
    if (st != CGH_OK) return st;
  }
  if (loss) {
    ProfScope p(c, CGH_KERNEL_LOSS, s);
    CGH_CHECK_LAUNCH(cgh::launch_loss_finalize(c, loss, s), "loss");
  }
  st = adjoint_rows(c, gf, s);
  if (st != CGH_OK) return st;
  return raster_adjoint(c, params, n, gf, grads, s, adam);
}

// checks of the Adam arguments shared by cgh_step and cgh_backward_step; fills
// the step's scalars
static cgh_status adam_scalars(int32_t t, float lr, float beta1, float beta2, float eps,
                               float *lr_scaled, float *inv_sqrt_bc2) {
  if (t < 1) return fail(CGH_ERR_INVALID_ARG, "step number t must be >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f))
    return fail(CGH_ERR_INVALID_ARG, "betas must be in [0, 1) and eps >= 0");
  const double bc1 = 1.0 - std::pow((double)beta1, (double)t);
  const double bc2 = 1.0 - std::pow((double)beta2, (double)t);
  *lr_scaled = (float)(1.0 / bc1);
  *inv_sqrt_bc2 = (float)(1.0 / std::sqrt(bc2));
  return CGH_OK;
}

cgh_status cgh_backward(cgh_ctx *ctx, const float *params, int32_t n, const cgh_c64 *field,
                        const float *target, double *loss, cgh_c64 *grad_field, float *grads,
                        void *stream) {
  return backward_impl(ctx, params, n, field, target, nullptr, loss, grad_field, grads, stream);
}

cgh_status cgh_backward_step(cgh_ctx *ctx, float *params, int32_t n, const cgh_c64 *field,
                             const float *target, double *loss, cgh_c64 *grad_field,
                             float *grads, float *m, float *v, int32_t t, float lr, float beta1,
                             float beta2, float eps, void *stream) {
  if (n > 0 && (!m || !v)) return fail(CGH_ERR_INVALID_ARG, "m/v is NULL");
  if (!aligned16(params) || !aligned16(grads) || !aligned16(m) || !aligned16(v))
    return fail(CGH_ERR_INVALID_ARG, "buffers must be 16-byte aligned");
  float scale = 0.f, isb = 0.f;
  cgh_status st = adam_scalars(t, lr, beta1, beta2, eps, &scale, &isb);
  if (st != CGH_OK) return st;
  // the same FP32 scalars as cgh_step: lr_scaled = lr * (1 / (1 - b1^t))
  const cgh::AdamFuse adam{params, m, v, lr * scale, beta1, beta2, eps, isb};
  return backward_impl(ctx, params, n, field, target, nullptr, loss, grad_field, grads, stream,
                       &adam);
}

cgh_status cgh_backward_recon(cgh_ctx *ctx, const float *params, int32_t n,
                              const cgh_c64 *field, const float *target, const float *mask,
                              double *loss, cgh_c64 *grad_field, float *grads, void *stream) {
  if (!mask) return fail(CGH_ERR_INVALID_ARG, "mask is NULL");
  return backward_impl(ctx, params, n, field, target, mask, loss, grad_field, grads, stream);
}

cgh_status cgh_backward_full(cgh_ctx *ctx, const float *params, int32_t n,
                             const cgh_c64 *field, const float *target, const float *mask,
                             float ssim_weight, double *loss, cgh_c64 *grad_field,
                             float *grads, void *stream) {
  if (!ctx) return fail(CGH_ERR_INVALID_ARG, "ctx is NULL");
  Ctx &c = ctx->c;
  if (!(c.cfg.flags & CGH_FULL_LOSS))
    return fail(CGH_ERR_STATE, "cgh_backward_full needs a context created with CGH_FULL_LOSS");
  if (!(ssim_weight >= 0.f) || !std::isfinite(ssim_weight))
    return fail(CGH_ERR_INVALID_ARG, "ssim_weight must be >= 0 and finite");
  cgh_status st = check_n(c, n);
  if (st != CGH_OK) return st;
  if (n != c.last_n)
    return fail(CGH_ERR_STATE, "backward with n = %d after rasterize with n = %d", n, c.last_n);
  if (!field || !target || (n > 0 && (!params || !grads)))
    return fail(CGH_ERR_INVALID_ARG, "field/target/params/grads is NULL");
  if (!aligned16(field) || !aligned16(grad_field) || ((uintptr_t)loss & 7u))
    return fail(CGH_ERR_INVALID_ARG, "misaligned buffer");
  hipStream_t s = (hipStream_t)stream;
  float2 *gf = grad_field ? reinterpret_cast<float2 *>(grad_field) : c.gfield_tmp;
  // forward: every plane's intensity, field and L_recon partials
  st = row_spectrum(c, field, s);
  if (st != CGH_OK) return st;
  for (int l = 0; l < c.L; ++l) {
    st = plane_spectrum(c, l, s);
    if (st != CGH_OK) return st;
    ProfScope p(c, CGH_KERNEL_ROW_LOSS, s);
    CGH_CHECK_LAUNCH(cgh::launch_row_loss(c, l, c.spec_plane, target, nullptr, mask, c.ssim_I,
                                          c.ssim_u, 0, s),
                     "loss row pass");
  }
  // SSIM and dL/dI over all planes; ssim_u becomes 2 (dL/dI) u
  {
    ProfScope p(c, CGH_KERNEL_LOSS, s);
    CGH_CHECK_LAUNCH(cgh::launch_ssim_fwd(c, target, s), "ssim");
    CGH_CHECK_LAUNCH(cgh::launch_ssim_bwd(c, target, mask, ssim_weight, s), "ssim adjoint");
    if (loss) CGH_CHECK_LAUNCH(cgh::launch_full_loss_finalize(c, ssim_weight, loss, s), "loss");
  }
  // adjoint of the propagation from the intensity gradient, plane by plane
  for (int l = 0; l < c.L; ++l) {
    {
      ProfScope p(c, CGH_KERNEL_ROW_FFT, s);
      CGH_CHECK_LAUNCH(cgh::launch_row_fwd(c, c.ssim_u + (size_t)l * c.C * c.H * c.W,
                                           c.spec_plane, s),
                       "adjoint seed row fft");
    }
    st = plane_adjoint(c, l, s);
    if (st != CGH_OK) return st;
  }
  st = adjoint_rows(c, gf, s);
  if (st != CGH_OK) return st;
  return raster_adjoint(c, params, n, gf, grads, s);
}

cgh_status cgh_propagate_field_adjoint(cgh_ctx *ctx, const cgh_c64 *grad_u, cgh_c64 *grad_field,
                                       void *stream) {
  if (!ctx) return fail(CGH_ERR_INVALID_ARG, "ctx is NULL");
  Ctx &c = ctx->c;
  if (!grad_u || !grad_field) return fail(CGH_ERR_INVALID_ARG, "grad_u/grad_field is NULL");
  if (!aligned16(grad_u) || !aligned16(grad_field))
    return fail(CGH_ERR_INVALID_ARG, "buffers must be 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const float2 *g = reinterpret_cast<const float2 *>(grad_u);
  for (int l = 0; l < c.L; ++l) {
    {
      ProfScope p(c, CGH_KERNEL_ROW_FFT, s);
      CGH_CHECK_LAUNCH(cgh::launch_row_fwd(c, g + (size_t)l * c.CF * c.H * c.W, c.spec_plane, s),
                       "adjoint seed row fft");
    }
    cgh_status st = plane_adjoint(c, l, s);
    if (st != CGH_OK) return st;
  }
  return adjoint_rows(c, reinterpret_cast<float2 *>(grad_field), s);
}

cgh_status cgh_propagate_adjoint(cgh_ctx *ctx, const cgh_c64 *field,
                                 const float *grad_intensity, cgh_c64 *grad_field,
                                 void *stream) {
  if (!ctx) return fail(CGH_ERR_INVALID_ARG, "ctx is NULL");
  Ctx &c = ctx->c;
  if (!field || !grad_intensity || !grad_field)
    return fail(CGH_ERR_INVALID_ARG, "field/grad_intensity/grad_field is NULL");
  if (!aligned16(field) || !aligned16(grad_field))
    return fail(CGH_ERR_INVALID_ARG, "misaligned buffer");
  hipStream_t s = (hipStream_t)stream;
  cgh_status st = row_spectrum(c, field, s);
  if (st != CGH_OK) return st;
  for (int l = 0; l < c.L; ++l) {
    st = plane_spectrum(c, l, s);
    if (st != CGH_OK) return st;
    {
      ProfScope p(c, CGH_KERNEL_ROW_LOSS, s);
      CGH_CHECK_LAUNCH(cgh::launch_row_loss(c, l, c.spec_plane, nullptr, grad_intensity,
                                            nullptr, nullptr, nullptr, 1, s),
                       "adjoint seed row pass");
    }
    st = plane_adjoint(c, l, s);
    if (st != CGH_OK) return st;
  }
  return adjoint_rows(c, reinterpret_cast<float2 *>(grad_field), s);
}

cgh_status cgh_rasterize_adjoint(cgh_ctx *ctx, const float *params, int32_t n,
                                 const cgh_c64 *grad_field, float *grads, void *stream) {
  if (!ctx) return fail(CGH_ERR_INVALID_ARG, "ctx is NULL");
  Ctx &c = ctx->c;
  cgh_status st = check_n(c, n);
  if (st != CGH_OK) return st;
  if (n != c.last_n)
    return fail(CGH_ERR_STATE, "adjoint with n = %d after rasterize with n = %d", n, c.last_n);
  if (!grad_field || (n > 0 && (!params || !grads)))
    return fail(CGH_ERR_INVALID_ARG, "grad_field/params/grads is NULL");
  if (!aligned16(grad_field)) return fail(CGH_ERR_INVALID_ARG, "misaligned grad_field");
  return raster_adjoint(c, params, n, reinterpret_cast<const float2 *>(grad_field), grads,
                        (hipStream_t)stream);
}

cgh_status cgh_step_adan(float *params, const float *grads, float *m, float *d, float *s,
                         float *prev_grads, int64_t count, int32_t t, float lr, float beta1,
                         float beta2, float beta3, float eps, float weight_decay,
                         const float *lr_groups, int32_t channels, void *stream) {
  if (count < 0) return fail(CGH_ERR_INVALID_ARG, "count < 0");
  if (count == 0) return CGH_OK;
  if (!params || !grads || !m || !d || !s || !prev_grads)
    return fail(CGH_ERR_INVALID_ARG, "NULL buffer");
  if (!aligned16(params) || !aligned16(grads) || !aligned16(m) || !aligned16(d) ||
      !aligned16(s) || !aligned16(prev_grads))
    return fail(CGH_ERR_INVALID_ARG, "buffers must be 16-byte aligned");
  if (t < 1) return fail(CGH_ERR_INVALID_ARG, "step number t must be >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && beta3 >= 0.f &&
        beta3 < 1.f && eps >= 0.f && weight_decay >= 0.f))
    return fail(CGH_ERR_INVALID_ARG, "betas must be in [0, 1), eps and weight_decay >= 0");
  int n = 0;
  if (lr_groups) {
    if (channels < 1 || channels > CGH_MAX_CHANNELS)
      return fail(CGH_ERR_INVALID_ARG, "channels must be in [1, %d]", CGH_MAX_CHANNELS);
    const int64_t per = 6 + 2 * channels;
    if (count % per) return fail(CGH_ERR_INVALID_ARG, "count not a multiple of 6 + 2C");
    n = (int)(count / per);
  }
  CGH_CHECK_LAUNCH(cgh::launch_adan(params, grads, m, d, s, prev_grads, count, t, lr, beta1,
                                    beta2, beta3, eps, weight_decay, lr_groups, n, channels,
                                    (hipStream_t)stream),
                   "adan");
  return CGH_OK;
}

cgh_status cgh_step(float *params, const float *grads, float *m, float *v, int64_t count,
                    int32_t t, float lr, float beta1, float beta2, float eps,
                    const float *lr_groups, int32_t channels, void *stream) {
  if (count < 0) return fail(CGH_ERR_INVALID_ARG, "count < 0");
  if (count == 0) return CGH_OK;
  if (!params || !grads || !m || !v) return fail(CGH_ERR_INVALID_ARG, "NULL buffer");
  if (!aligned16(params) || !aligned16(grads) || !aligned16(m) || !aligned16(v))
    return fail(CGH_ERR_INVALID_ARG, "buffers must be 16-byte aligned");
  float scale = 0.f, isb = 0.f;
  cgh_status st = adam_scalars(t, lr, beta1, beta2, eps, &scale, &isb);
  if (st != CGH_OK) return st;
  int n = 0;
  if (lr_groups) {
    if (channels < 1 || channels > CGH_MAX_CHANNELS)
      return fail(CGH_ERR_INVALID_ARG, "channels must be in [1, %d]", CGH_MAX_CHANNELS);
    const int64_t per = 6 + 2 * channels;
    if (count % per) return fail(CGH_ERR_INVALID_ARG, "count not a multiple of 6 + 2C");
    n = (int)(count / per);
  }
  CGH_CHECK_LAUNCH(cgh::launch_adam(params, grads, m, v, count, lr, scale, beta1, beta2, eps,
                                    isb, lr_groups, n, channels, (hipStream_t)stream),
                   "adam");
  return CGH_OK;
}

cgh_status cgh_get_transfer(cgh_ctx *ctx, int32_t channel, int32_t plane, cgh_c64 *out,
                            void *stream) {
  if (!ctx || !out) return fail(CGH_ERR_INVALID_ARG, "ctx/out is NULL");
  Ctx &c = ctx->c;
  if (channel < 0 || channel >= c.CF || plane < 0 || plane >= c.L)
    return fail(CGH_ERR_INVALID_ARG, "channel/plane out of range");
  const size_t elems = (size_t)c.Hq * c.Wq;
  hipError_t e = hipMemcpyAsync(out, c.htab + ((size_t)channel * c.L + plane) * elems,
                                elems * sizeof(float2), hipMemcpyDeviceToDevice,
                                (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "cgh_get_transfer");
  return CGH_OK;
}

cgh_status cgh_profile_begin(cgh_ctx *ctx, int32_t kernel_class) {
  if (!ctx) return fail(CGH_ERR_INVALID_ARG, "ctx is NULL");
  if (kernel_class < CGH_KERNEL_PREPROCESS || kernel_class > CGH_KERNEL_PREPROCESS_ADJOINT)
    return fail(CGH_ERR_INVALID_ARG, "unknown kernel class %d", kernel_class);
  Ctx &c = ctx->c;
  if (!c.prof_ev) {
    hipEvent_t *ev = new (std::nothrow) hipEvent_t[2 * cgh::kMaxProf];
    if (!ev) return fail(CGH_ERR_INVALID_ARG, "host allocation failed");
    for (int i = 0; i < 2 * cgh::kMaxProf; ++i) {
      hipError_t e = hipEventCreate(&ev[i]);
      if (e != hipSuccess) {
        for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
        delete[] ev;
        return device_fail(e, "cgh_profile_begin");
      }
    }
    c.prof_ev = ev;
  }
  c.prof_class = kernel_class;
  c.prof_n = 0;
  return CGH_OK;
}

cgh_status cgh_profile_end(cgh_ctx *ctx, void *stream, double *total_ms, int32_t *launches) {
  if (!ctx) return fail(CGH_ERR_INVALID_ARG, "ctx is NULL");
  Ctx &c = ctx->c;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "cgh_profile_end");
  double sum = 0.0;
  for (int i = 0; i < c.prof_n; ++i) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, c.prof_ev[2 * i], c.prof_ev[2 * i + 1]);
    if (e != hipSuccess) return device_fail(e, "cgh_profile_end");
    sum += ms;
  }
  if (total_ms) *total_ms = sum;
  if (launches) *launches = c.prof_n;
  c.prof_class = 0;
  c.prof_n = 0;
  return CGH_OK;
}

// new optics for holograms [b0, b1) of ctx; validated before anything changes
static cgh_status set_optics_range(cgh_ctx *ctx, int b0, int b1, const double *wavelength_m,
                                   const double *z_m, void *stream) {
  if (!ctx || !wavelength_m || !z_m) return fail(CGH_ERR_INVALID_ARG, "ctx/wavelength/z is NULL");
  Ctx &c = ctx->c;
  for (int ch = 0; ch < c.C; ++ch)
    if (!(wavelength_m[ch] > 0.0) || !std::isfinite(wavelength_m[ch]))
      return fail(CGH_ERR_INVALID_ARG, "wavelength of channel %d must be positive", ch);
  for (int l = 0; l < c.L; ++l)
    if (!std::isfinite(z_m[l])) return fail(CGH_ERR_INVALID_ARG, "z of plane %d not finite", l);
  for (int b = b0; b < b1; ++b) {
    for (int ch = 0; ch < c.C; ++ch) c.lam[b][ch] = wavelength_m[ch];
    for (int l = 0; l < c.L; ++l) c.zd[b][l] = z_m[l];
  }
  if (b0 == 0 && b1 == c.B) {
    for (int ch = 0; ch < c.C; ++ch) c.cfg.wavelength_m[ch] = wavelength_m[ch];
    for (int l = 0; l < c.L; ++l) c.cfg.z_m[l] = z_m[l];
  }
  CGH_CHECK_LAUNCH(cgh::launch_build_transfer(c, b0, b1, (hipStream_t)stream),
                   "transfer function");
  return CGH_OK;
}

cgh_status cgh_set_optics(cgh_ctx *ctx, const double *wavelength_m, const double *z_m,
                          void *stream) {
  return set_optics_range(ctx, 0, ctx ? ctx->c.B : 0, wavelength_m, z_m, stream);
}

cgh_status cgh_set_hologram_optics(cgh_ctx *ctx, int32_t hologram, const double *wavelength_m,
                                   const double *z_m, void *stream) {
  if (!ctx) return fail(CGH_ERR_INVALID_ARG, "ctx is NULL");
  if (hologram < 0 || hologram >= ctx->c.B)
    return fail(CGH_ERR_INVALID_ARG, "hologram %d outside [0, %d)", hologram, ctx->c.B);
  return set_optics_range(ctx, hologram, hologram + 1, wavelength_m, z_m, stream);
}

}  // extern "C"

struct cgh_solve {
  hipGraphExec_t exec;
};

namespace {

// The kernels of one solve, enqueued on s (which is capturing).
cgh_status record_solve(cgh_ctx *ctx, float *params, int32_t n, const float *target,
                        cgh_c64 *field, float *grads, float *m, float *v, double *loss_log,
                        int32_t steps, float lr, float beta1, float beta2, float eps,
                        hipStream_t s) {
  const int64_t count = cgh::total_gaussians(ctx->c, n) * (6 + 2 * ctx->c.C);
  CGH_CHECK_LAUNCH(cgh::launch_zero_pair(m, v, count, s), "solve: zero moments");
  for (int32_t t = 1; t <= steps; ++t) {
    cgh_status st = cgh_rasterize(ctx, params, n, field, s);
    if (st == CGH_OK)
      st = cgh_backward_step(ctx, params, n, field, target,
                             loss_log + 2 * (int64_t)ctx->c.B * (t - 1), nullptr,
                             t == steps ? grads : nullptr, m, v, t, lr, beta1, beta2, eps, s);
    if (st != CGH_OK) return st;
  }
  return CGH_OK;
}

}  // namespace

extern "C" {

cgh_status cgh_solve_create(cgh_ctx *ctx, float *params, int32_t n, const float *target,
                            cgh_c64 *field, float *grads, float *m, float *v, double *loss_log,
                            int32_t steps, float lr, float beta1, float beta2, float eps,
                            void *stream, cgh_solve **out) {
  if (!out) return fail(CGH_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(CGH_ERR_INVALID_ARG, "ctx is NULL");
  if (!stream) return fail(CGH_ERR_INVALID_ARG, "the NULL stream cannot be captured");
  cgh_status st = check_n(ctx->c, n);
  if (st != CGH_OK) return st;
  if (n < 1) return fail(CGH_ERR_INVALID_ARG, "a solve needs n >= 1");
  if (steps < 1 || steps > 10000) return fail(CGH_ERR_INVALID_ARG, "steps must be in [1, 10000]");
  if (!params || !target || !field || !grads || !m || !v || !loss_log)
    return fail(CGH_ERR_INVALID_ARG, "NULL buffer");
  if (!aligned16(params) || !aligned16(grads) || !aligned16(m) || !aligned16(v) ||
      !aligned16(field) || ((uintptr_t)loss_log & 7u))
    return fail(CGH_ERR_INVALID_ARG, "misaligned buffer");
  if (!(lr >= 0.f) || !std::isfinite(lr) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f))
    return fail(CGH_ERR_INVALID_ARG, "lr must be >= 0, betas in [0, 1), eps >= 0");
  if (ctx->c.prof_class)
    return fail(CGH_ERR_STATE, "kernel timing is active on this context");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return device_fail(e, "cgh_solve_create: begin capture");
  st = record_solve(ctx, params, n, target, field, grads, m, v, loss_log, steps, lr, beta1, beta2,
                    eps, s);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(s, &graph);
  if (st != CGH_OK) {
    if (graph) (void)hipGraphDestroy(graph);  // the recorded error is the one to report
    return st;
  }
  if (e != hipSuccess) return device_fail(e, "cgh_solve_create: end capture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);  // the executable graph no longer needs it
  if (e != hipSuccess) return device_fail(e, "cgh_solve_create: instantiate");
  cgh_solve *h = new (std::nothrow) cgh_solve;
  if (!h) {
    (void)hipGraphExecDestroy(exec);
    return fail(CGH_ERR_INVALID_ARG, "host allocation failed");
  }
  h->exec = exec;
  *out = h;
  return CGH_OK;
}

cgh_status cgh_solve_launch(cgh_solve *solve, void *stream) {
  if (!solve) return fail(CGH_ERR_INVALID_ARG, "solve is NULL");
  if (!stream) return fail(CGH_ERR_INVALID_ARG, "stream is NULL");
  hipError_t e = hipGraphLaunch(solve->exec, (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "cgh_solve_launch");
  return CGH_OK;
}

cgh_status cgh_solve_destroy(cgh_solve *solve) {
  if (!solve) return CGH_OK;
  hipError_t e = hipGraphExecDestroy(solve->exec);
  delete solve;
  if (e != hipSuccess) return device_fail(e, "cgh_solve_destroy");
  return CGH_OK;
}

cgh_status cgh_read_status(cgh_ctx *ctx, void *stream, int64_t *pairs) {
  if (!ctx) return fail(CGH_ERR_INVALID_ARG, "ctx is NULL");
  Ctx &c = ctx->c;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "cgh_read_status");
  uint32_t st[4] = {0, 0, 0, 0};
  e = hipMemcpy(st, c.status, sizeof(st), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return device_fail(e, "cgh_read_status");
  if (pairs) *pairs = (int64_t)st[1];
  if (st[2] || st[3]) {
    // an overflow or a non-finite value since the last read: report it once
    const uint32_t zero[2] = {0u, 0u};
    e = hipMemcpy(c.status + 2, zero, sizeof(zero), hipMemcpyHostToDevice);
    if (e != hipSuccess) return device_fail(e, "cgh_read_status");
  }
  if (st[0])
    return fail(CGH_ERR_CAPACITY, "pair list needed %u entries, capacity is %lld", st[1],
                (long long)c.pair_cap);
  if (st[2])
    return fail(CGH_ERR_CAPACITY,
                "a rasterize since the last status read overflowed the pair list (capacity "
                "%lld; the last one needed %u entries)", (long long)c.pair_cap, st[1]);
  if (st[3])
    return fail(CGH_ERR_NONFINITE, "non-finite values since the last status read in:%s%s%s",
                (st[3] & cgh::kNonFiniteParams) ? " parameters" : "",
                (st[3] & cgh::kNonFiniteGrads) ? " gradients" : "",
                (st[3] & cgh::kNonFiniteLoss) ? " loss" : "");
  return CGH_OK;
}

}  // extern "C"
