// Complex 2D Gaussian rasterizer on gfx950 (Alg. 2; Sec. 3.1 coherent sum;
// supplementary Forward and Backward Pass).
//
//   preprocess (FP64)  activations, covariance, inverse, support box, tile
//                      rectangle; writes one FP32 record per Gaussian
//   binning            exclusive scan of tile counts -> emit (tile, gaussian)
//                      pairs in Gaussian order -> stable LSD radix sort on the
//                      tile id -> [start, end) per tile.  Deterministic: each
//                      tile lists its Gaussians in increasing index.
//   forward            one tile (16x16, 32x8, 16x8 or 8x8 pixels) per
//                      workgroup, one 8x8 sub-block per wavefront; Gaussians
//                      culled per sub-block with a ballot, summed per pixel in
//                      FP32 in list order
//   adjoint            per tile, the tile's dL/dU0 staged in LDS; one lane per
//                      (tile, Gaussian) pair walks the pair's pixels and keeps
//                      its 2C + 5 partial sums in registers (no per-pixel
//                      storage, no atomics); the per-pair partials are summed in
//                      a fixed order per Gaussian by the FP64 preprocess adjoint
// A context may hold B holograms of one size: Gaussian g belongs to hologram
// g / n (its parameters are that hologram's block of the [B][n (6 + 2C)]
// array), and tile t to hologram t / tiles_per, so one launch of each kernel
// covers all of them.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "cgh_internal.h"

namespace cgh {

constexpr double kLog2e = 1.4426950408889634074;
constexpr float kPowerFloor2 = -50.0f * 1.4426950408889634f;  // clamp of the exponent, base 2

constexpr int rec_ext_c(int C) { return ((R_AMP + 2 * C) + 3) & ~3; }
constexpr int rec_stride_c(int C) { return rec_ext_c(C) + 4; }
constexpr int part_stride_c(int C) { return ((2 * C + 5) + 3) & ~3; }

// ----------------------------------------------------------------------------
// Preprocess: supplementary "Parameter Activation Functions", "2D Covariance
// Matrix Computation", "2D Covariance Matrix Inversion".  The mean's
// activation runs in FP64 (its fraction of a pixel is stored, and FP32 would
// round a position near x = 1920 to 1.2e-4 px); the rest in FP32.  Sigma is
// R diag(l0, l1) R^T with l0 = s_x^2 + eps_Sigma, l1 = s_y^2 + eps_Sigma (the
// regularised covariance), so its inverse is R diag(1 / l0, 1 / l1) R^T, with
// no cancellation however elongated the Gaussian, and det = l0 l1 >= 0.0121:
// the determinant clamp never applies.
// ----------------------------------------------------------------------------
struct Geom {
  double mx, my;
  float sx, sy, ct, st, s00, s01, s11, i00, i01, i11, alpha;
};

__device__ __forceinline__ Geom geometry(const float *__restrict__ params, int n, int C, int g,
                                         int W, int H) {
  const float *mp = params;
  const float *ls = params + 2 * (size_t)n;
  const float *rot = params + 4 * (size_t)n;
  const float *op = params + (size_t)(5 + 2 * C) * n;
  Geom q;
  q.mx = 0.5 * (tanh((double)mp[2 * g]) + 1.0) * (double)W;
  q.my = 0.5 * (tanh((double)mp[2 * g + 1]) + 1.0) * (double)H;
  q.sx = expf(ls[2 * g]) + 0.1f;
  q.sy = expf(ls[2 * g + 1]) + 0.1f;
  sincosf(rot[g], &q.st, &q.ct);
  const float c = q.ct, s = q.st;
  const float sx2 = q.sx * q.sx, sy2 = q.sy * q.sy;
  q.s00 = sx2 * c * c + sy2 * s * s + 0.1f;
  q.s01 = (sx2 - sy2) * c * s;
  q.s11 = sx2 * s * s + sy2 * c * c + 0.1f;
  const float e0 = 1.0f / (sx2 + 0.1f), e1 = 1.0f / (sy2 + 0.1f);
  q.i00 = c * c * e0 + s * s * e1;
  q.i01 = c * s * (e0 - e1);
  q.i11 = s * s * e0 + c * c * e1;
  q.alpha = 1.0f / (1.0f + expf(-op[g]));
  return q;
}

// true if the 6 + 2C parameters of Gaussian g (of n) are all finite
template <int C>
__device__ __forceinline__ bool params_finite(const float *__restrict__ params, int n, int g) {
  bool ok = isfinite(params[2 * g]) && isfinite(params[2 * g + 1]) &&
            isfinite(params[2 * (size_t)n + 2 * g]) &&
            isfinite(params[2 * (size_t)n + 2 * g + 1]) && isfinite(params[4 * (size_t)n + g]) &&
            isfinite(params[(size_t)(5 + 2 * C) * n + g]);
#pragma unroll
  for (int c = 0; c < C; ++c)
    ok = ok && isfinite(params[5 * (size_t)n + (size_t)g * C + c]) &&
         isfinite(params[(size_t)(5 + C) * n + (size_t)g * C + c]);
  return ok;
}

// Gaussian g of all B n: hologram b = g / n, index gl within it, and the base
// of that hologram's parameter (or gradient) block
struct GaussIdx {
  int b, gl;
  size_t base;
};
template <int C>
__device__ __forceinline__ GaussIdx gauss_idx(int g, int n) {
  GaussIdx r;
  r.b = g / n;
  r.gl = g - r.b * n;
  r.base = (size_t)r.b * n * (6 + 2 * C);
  return r;
}

// Scans over one workgroup of 256 threads.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// block-wide exclusive scan of one value per thread (256 threads); returns the
// thread's exclusive prefix, *total gets the block sum
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *total) {
  __shared__ uint32_t wsum[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t incl = wave_inclusive_scan(v);
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t off = 0;
  for (int w = 0; w < wave; ++w) off += wsum[w];
  *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  __syncthreads();
  return off + incl - v;
}

// Gaussian g of all B n: its record, tile rectangle and tile count (returned);
// tile shape (1 << tlx) x (1 << tly) pixels
template <int C>
__device__ __forceinline__ uint32_t preprocess_one(const float *__restrict__ params_all, int n,
                                                   int g, int W, int H, float k, int tlx,
                                                   int tly, float *__restrict__ rec,
                                                   uint2 *__restrict__ rect,
                                                   uint32_t *__restrict__ counts, float thr,
                                                   float2 *__restrict__ alim,
                                                   uint32_t *__restrict__ finite_flag,
                                                   uint2 &rc_out) {
  constexpr int RS = rec_stride_c(C);
  const GaussIdx gi = gauss_idx<C>(g, n);
  const float *params = params_all + gi.base;
  if (finite_flag && !params_finite<C>(params, n, gi.gl)) atomicOr(finite_flag, kNonFiniteParams);
  const Geom q = geometry(params, n, C, gi.gl, W, H);
  const float *amp = params + 5 * (size_t)n + (size_t)gi.gl * C;
  const float *ph = params + (size_t)(5 + C) * n + (size_t)gi.gl * C;
  float r[RS];
#pragma unroll
  for (int i = 0; i < RS; ++i) r[i] = 0.f;
  const double fx = floor(q.mx), fy = floor(q.my);
  r[R_MIX] = __int_as_float((int)fx);
  r[R_MIY] = __int_as_float((int)fy);
  r[R_MFX] = (float)(q.mx - fx);
  r[R_MFY] = (float)(q.my - fy);
  constexpr float kL2e = (float)kLog2e;
  r[R_A] = -0.5f * kL2e * q.i00;
  r[R_B] = -kL2e * q.i01;
  r[R_C] = -0.5f * kL2e * q.i11;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    float s, co;
    sincosf(ph[c], &s, &co);
    const float a = q.alpha * amp[c];
    r[R_AMP + 2 * c] = a * co;
    r[R_AMP + 2 * c + 1] = a * s;
  }
  // support box (k sqrt(Sigma00), k sqrt(Sigma11)) -> inclusive pixel range
  uint32_t cnt = 0;
  uint2 rc = make_uint2(0u, 0u);
  double i0, i1, j0, j1;
  if (k > 0.f) {
    const float rxf = k * sqrtf(q.s00), ryf = k * sqrtf(q.s11);
    const double rx = rxf, ry = ryf;
    r[R_RX] = rxf;
    r[R_RY] = ryf;
    const double pad = 1e-3;  // keeps every pixel the FP32 predicate could accept
    i0 = fmax(0.0, ceil(q.mx - rx - pad));
    i1 = fmin((double)(W - 1), floor(q.mx + rx + pad));
    j0 = fmax(0.0, ceil(q.my - ry - pad));
    j1 = fmin((double)(H - 1), floor(q.my + ry + pad));
  } else {
    r[R_RX] = 1e30f;
    r[R_RY] = 1e30f;
    i0 = 0; i1 = W - 1; j0 = 0; j1 = H - 1;
  }
  if (i0 <= i1 && j0 <= j1) {
    const uint32_t tx0 = (uint32_t)i0 >> tlx, tx1 = (uint32_t)i1 >> tlx;
    const uint32_t ty0 = (uint32_t)j0 >> tly, ty1 = (uint32_t)j1 >> tly;
    cnt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
    rc = make_uint2(tx0 | (tx1 << 16), ty0 | (ty1 << 16));
  }
  // row form of the exponent (completing the square in dx):
  //   i00 dx^2 + 2 i01 dx dy + i11 dy^2 = i00 (dx - s dy)^2 + dy^2 / Sigma11,
  //   s = -i01 / i00 = Sigma01 / Sigma11
  r[rec_ext_c(C) + RX_S] = q.s01 / q.s11;
  r[rec_ext_c(C) + RX_KAPPA] = -0.5f * kL2e / q.s11;
  r[rec_ext_c(C) + RX_RA] = sqrtf(0.5f * kL2e * q.i00);
  float4 *dst = reinterpret_cast<float4 *>(rec + (size_t)g * RS);
#pragma unroll
  for (int i = 0; i < RS / 4; ++i) dst[i] = make_float4(r[4 * i], r[4 * i + 1], r[4 * i + 2], r[4 * i + 3]);
  counts[g] = cnt;
  rect[g] = rc;
  rc_out = rc;
  if (alim) {
    // Alg. 2 weight w = min(0.99, alpha G), kept where alpha G >= 1/255: in the
    // exponent p = log2 G, kept for p >= max(support threshold, log2(1/(255 alpha)))
    // and clamped at log2(0.99 / alpha)
    const float lo = -log2f(255.0f * q.alpha), hi = log2f(0.99f / q.alpha);
    alim[g] = make_float2(fmaxf(thr, lo), hi);
  }
  return cnt;
}

// The preprocess of 256 Gaussians per workgroup, which also starts the
// binning: the workgroup's exclusive scan of its tile counts goes to
// offsets[g] and its total to chunk_sums[workgroup] (the emit adds the totals
// of the workgroups before its own), the histogram of the first sort digit
// (tile id & 255) over the workgroup's pairs to hist1[digit * workgroups +
// workgroup], every tile range is set to (0xffffffff, 0) (the last sort pass
// narrows them with atomic min / max), and workgroup 0 clears the overflow
// flag of this rasterize (*overflow).
template <int C>
__global__ __launch_bounds__(256) void k_preprocess(const float *__restrict__ params_all, int n,
                                                    int total, int W, int H, float k, int tlx,
                                                    int tly, float *__restrict__ rec,
                                                    uint2 *__restrict__ rect,
                                                    uint32_t *__restrict__ counts, float thr,
                                                    float2 *__restrict__ alim,
                                                    uint32_t *__restrict__ finite_flag,
                                                    uint32_t *__restrict__ offsets,
                                                    uint32_t *__restrict__ chunk_sums,
                                                    uint32_t *__restrict__ overflow,
                                                    int tiles_x, int tiles_per,
                                                    uint32_t *__restrict__ hist1,
                                                    uint2 *__restrict__ ranges, int num_tiles) {
  __shared__ uint32_t h1[256];
  const int tid = threadIdx.x;
  const int g = blockIdx.x * blockDim.x + tid;
  for (int t = blockIdx.x * blockDim.x + tid; t < num_tiles; t += gridDim.x * blockDim.x)
    ranges[t] = make_uint2(0xffffffffu, 0u);
  h1[tid] = 0u;
  uint32_t cnt = 0;
  uint2 rc = make_uint2(0u, 0u);
  if (g < total)
    cnt = preprocess_one<C>(params_all, n, g, W, H, k, tlx, tly, rec, rect, counts, thr, alim,
                            finite_flag, rc);
  uint32_t sum;
  const uint32_t pre = block_exclusive_scan(cnt, &sum);  // every thread takes part
  if (g < total) offsets[g] = pre;
  if (tid == 0) chunk_sums[blockIdx.x] = sum;
  if (g == 0) *overflow = 0u;
  // (the scan's barriers order the clearing of h1 before the counting)
  if (cnt) {
    const uint32_t tx0 = rc.x & 0xffffu, tx1 = rc.x >> 16, ty0 = rc.y & 0xffffu;
    const uint32_t kb = (uint32_t)(g / n) * (uint32_t)tiles_per;
    uint32_t tx = tx0, ty = ty0;
    for (uint32_t t = 0; t < cnt; ++t) {
      atomicAdd(&h1[(kb + ty * (uint32_t)tiles_x + tx) & 255u], 1u);
      if (++tx > tx1) { tx = tx0; ++ty; }
    }
  }
  __syncthreads();
  hist1[(size_t)tid * gridDim.x + blockIdx.x] = h1[tid];
}

static float support_threshold(float k) {
  // log2 G >= -k^2/2 log2(e)  <=>  q <= k^2 ; k <= 0: everything
  if (k <= 0.f) return -INFINITY;
  return (float)(-0.5 * (double)k * (double)k * kLog2e);
}

static int log2i(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

hipError_t launch_preprocess(const Ctx &c, const float *params, int n, hipStream_t s) {
  const int total = (int)total_gaussians(c, n);
  if (total <= 0) return hipSuccess;
  dim3 grid((total + 255) / 256), block(256);
  const float k = c.cfg.support_sigma, thr = support_threshold(k);
  const int tlx = log2i(c.tile_w), tly = log2i(c.tile_h);
#define CGH_PRE(CC)                                                                           \
  hipLaunchKernelGGL(k_preprocess<CC>, grid, block, 0, s, params, n, total, c.W, c.H, k, tlx, \
                     tly, c.rec, c.rect, c.counts, thr, c.alim, c.finite_flag, c.offsets,     \
                     c.scan_tmp, c.status, c.tiles_x, c.tiles_per, c.hist, c.ranges,          \
                     c.num_tiles)
  switch (c.C) {
    case 1: CGH_PRE(1); break;
    case 2: CGH_PRE(2); break;
    case 3: CGH_PRE(3); break;
    default: CGH_PRE(4); break;
  }
#undef CGH_PRE
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Exclusive scan of u32 (three kernels: per-block scan, scan of block sums,
// add).
// ----------------------------------------------------------------------------
// per-block exclusive scans of kScanItems elements and the block sums; also
// clears *zero_word (if given), which lets the binning skip a launch
__global__ __launch_bounds__(256) void k_scan_local(const uint32_t *__restrict__ in,
                                                    uint32_t *__restrict__ out, int len,
                                                    uint32_t *__restrict__ block_sums,
                                                    uint32_t *__restrict__ zero_word) {
  if (zero_word && blockIdx.x == 0 && threadIdx.x == 0) *zero_word = 0u;
  const int base = blockIdx.x * kScanItems + threadIdx.x * 8;
  uint32_t v[8];
  uint32_t s = 0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const uint32_t x = base + e < len ? in[base + e] : 0u;
    v[e] = s;
    s += x;
  }
  uint32_t total;
  const uint32_t off = block_exclusive_scan(s, &total);
#pragma unroll
  for (int e = 0; e < 8; ++e)
    if (base + e < len) out[base + e] = v[e] + off;
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// exclusive scan of the block sums in one block; writes the grand total to
// total_out[0] (and total_out[1] if total_out2 is set)
__global__ __launch_bounds__(256) void k_scan_sums(uint32_t *__restrict__ sums, int nb,
                                                   uint32_t *__restrict__ total_out,
                                                   uint32_t *__restrict__ total_out2) {
  uint32_t carry = 0;
  for (int base = 0; base < nb; base += 256) {
    const int i = base + threadIdx.x;
    const uint32_t x = i < nb ? sums[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(x, &tot);
    if (i < nb) sums[i] = ex + carry;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    if (total_out) *total_out = carry;
    if (total_out2) *total_out2 = carry;
  }
}

__global__ __launch_bounds__(256) void k_scan_add(uint32_t *__restrict__ out, int len,
                                                  const uint32_t *__restrict__ sums) {
  const int base = blockIdx.x * kScanItems + threadIdx.x * 8;
  const uint32_t add = sums[blockIdx.x];
#pragma unroll
  for (int e = 0; e < 8; ++e)
    if (base + e < len) out[base + e] += add;
}

static hipError_t scan_u32(const uint32_t *in, uint32_t *out, int len, uint32_t *tmp,
                           uint32_t *total, uint32_t *total2, hipStream_t s) {
  const int nb = (len + kScanItems - 1) / kScanItems;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(256), 0, s, in, out, len, tmp, nullptr);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, tmp, nb, total, total2);
  hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(256), 0, s, out, len, tmp);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Binning: emit (tile, gaussian) pairs, stable radix sort, tile ranges.
// ----------------------------------------------------------------------------
__device__ __forceinline__ uint32_t pair_count(const uint32_t *status, int64_t cap) {
  const uint64_t total = status[1];
  return (uint32_t)((int64_t)total < cap ? total : cap);
}

// Per-block digit histograms, digit-major: hist[d * nblocks + b].  Each thread
// loads its 16 keys before counting them.
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t *__restrict__ keys,
                                                    const uint32_t *__restrict__ status,
                                                    int64_t cap, int shift,
                                                    uint32_t *__restrict__ hist, int nblocks) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const uint32_t count = pair_count(status, cap);
  const uint32_t base = blockIdx.x * kSortItems;
  if (base < count) {
    constexpr int PER = kSortItems / 256;
    uint32_t k[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) k[j] = keys[min(base + j * 256 + tid, count - 1)];
#pragma unroll
    for (int j = 0; j < PER; ++j)
      if (base + j * 256 + tid < count) atomicAdd(&h[(k[j] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(size_t)tid * nblocks + blockIdx.x] = h[tid];
}

// Stable scatter of one 8-bit digit.  Wave w of block b owns the kSortItems / 4
// keys from kSortItems b + (kSortItems / 4) w, taken in index order 64 at a
// time; a key's rank among equal digits of its wave is (the wave's running
// count of the digit) + (earlier lanes of its round with that digit, from
// ballots over the digit bits).  The block then orders its keys by digit in
// LDS (digit, then wave, then rank) and writes them out in that order, so
// consecutive threads store consecutive positions of one digit's run and the
// stores coalesce.  The global position of the key at local index i with
// digit d is (exclusive scan of the digit-major histogram at (d, b)) +
// (i - the block's first local index of d): equal keys keep their order.
// hist_scan holds the digit-major histogram scanned either globally
// (chunk_sums == nullptr) or per chunk of kScanItems, with the chunk sums in
// chunk_sums (at most kMaxScanChunks); then each block scans the chunk sums.
// With ranges != nullptr (the last pass, up to kMaxAtomicRangeTiles tiles) no
// keys are written: a block's keys, in the order it writes them, are sorted
// (its input is sorted on the lower digits), so each run of one tile id in it
// is a piece of that tile's final list, and the block takes the tile's range
// to the piece's first and last positions with atomic min / max (every
// tile's range starts as (0xffffffff, 0)).  A block holds about one piece per
// value of its digit, so with many tiles the atomics cost more than a
// separate ranges kernel (k_ranges).
constexpr int kMaxScanChunks = 1024;
constexpr int kMaxAtomicRangeTiles = 16384;

__global__ __launch_bounds__(256) void k_radix_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
    const uint32_t *__restrict__ status, int64_t cap, int shift,
    const uint32_t *__restrict__ hist_scan, int nblocks,
    const uint32_t *__restrict__ chunk_sums, int nchunks, uint2 *__restrict__ ranges,
    uint32_t num_tiles) {
  constexpr int R = kSortItems / 256;  // rounds of 64 keys per wave
  __shared__ uint32_t wcnt[4][256];    // per-wave digit counts, then local offsets
  __shared__ uint32_t gofs[256];       // global position of local index 0 of each digit
  __shared__ uint32_t cpre[kMaxScanChunks];
  __shared__ uint32_t skey[kSortItems], sval[kSortItems];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t count = pair_count(status, cap);
  const uint32_t base = blockIdx.x * kSortItems;
  if (base >= count) return;  // the whole block is past the end (uniform)
  const uint32_t nvalid = min((uint32_t)kSortItems, count - base);
#pragma unroll
  for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
  const uint32_t first = base + (uint32_t)(kSortItems / 4) * wave + lane;
  uint32_t key[R], val[R], rank[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = min(first + 64u * r, count - 1);
    key[r] = kin[i];
    val[r] = vin[i];
  }
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool valid = first + 64u * r < count;
    const uint32_t d = (key[r] >> shift) & 255u;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const uint64_t bb = __ballot(on);
      m &= on ? bb : ~bb;
    }
    const uint32_t before = __popcll(m & lt);
    const uint32_t prev = wcnt[wave][d];
    rank[r] = prev + before;
    // the lowest lane of each digit group advances the wave's count; this
    // wave's LDS accesses complete in order, so the next round reads it
    if (valid && before == 0) wcnt[wave][d] = prev + (uint32_t)__popcll(m);
  }
  if (chunk_sums) {
    // exclusive scan of the chunk sums, four per thread
    uint32_t c4[4], sum = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = tid * 4 + e;
      c4[e] = sum;
      sum += i < nchunks ? chunk_sums[i] : 0u;
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(sum, &tot);
#pragma unroll
    for (int e = 0; e < 4; ++e) cpre[tid * 4 + e] = ex + c4[e];
  }
  __syncthreads();
  {
    // thread tid = digit d: the block's local offsets of d per wave, and the
    // global position of d's local index 0
    uint32_t c[4], tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) { c[w] = wcnt[w][tid]; tot += c[w]; }
    uint32_t all;
    const uint32_t lbase = block_exclusive_scan(tot, &all);
    uint32_t run = lbase;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      wcnt[w][tid] = run;
      run += c[w];
    }
    const size_t e = (size_t)tid * nblocks + blockIdx.x;
    gofs[tid] = hist_scan[e] + (chunk_sums ? cpre[e / kScanItems] : 0u) - lbase;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (first + 64u * r < count) {
      const uint32_t d = (key[r] >> shift) & 255u;
      const uint32_t lp = wcnt[wave][d] + rank[r];
      if (lp < (uint32_t)kSortItems) {  // always true for consistent counts; guards the write
        skey[lp] = key[r];
        sval[lp] = val[r];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = (uint32_t)tid + 256u * r;
    if (i < nvalid) {
      const uint32_t k = skey[i];
      const uint32_t pos = gofs[(k >> shift) & 255u] + i;
      if (pos < count) {  // always true for a consistent histogram; guards the write
        vout[pos] = sval[i];
        if (!ranges) {
          kout[pos] = k;
        } else if (k < num_tiles) {  // keys are tile ids; guards the atomics
          if (i == 0 || skey[i - 1] != k) atomicMin(&ranges[k].x, pos);
          if (i + 1 == nvalid || skey[i + 1] != k) atomicMax(&ranges[k].y, pos + 1u);
        }
      }
    }
  }
}

// Tile ranges from the sorted keys, for contexts with more than
// kMaxAtomicRangeTiles tiles; each tile without pairs gets an empty range
// from the thread at the gap it falls in (every tile is written once).
// A grid-stride loop: the grid is sized for the pair capacity's worth of
// blocks at most, far fewer than one thread per pair.
__global__ void k_ranges(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ status,
                         int64_t cap, uint2 *__restrict__ ranges, uint32_t num_tiles) {
  const uint32_t count = pair_count(status, cap);
  const uint32_t i0 = blockIdx.x * blockDim.x + threadIdx.x;
  if (count == 0) return;  // every range is still the preprocess's empty (0xffffffff, 0)
  for (uint32_t i = i0; i < count; i += gridDim.x * blockDim.x) {
    const uint32_t k = keys[i];
    if (k >= num_tiles) continue;  // keys are tile ids; guards the writes
    if (i == 0 || keys[i - 1] != k) {
      ranges[k].x = i;
      const uint32_t prev = i == 0 ? 0u : keys[i - 1] + 1u;
      for (uint32_t t = prev; t < k; ++t) ranges[t] = make_uint2(0u, 0u);
    }
    if (i + 1 == count || keys[i + 1] != k) {
      ranges[k].y = i + 1;
      if (i + 1 == count)
        for (uint32_t t = k + 1; t < num_tiles; ++t) ranges[t] = make_uint2(0u, 0u);
    }
  }
}

// The emit fused with the first sort pass.  Gaussian g's pairs own the pair
// slots [offset(g), offset(g) + count(g)) in row-major tile order (the adjoint
// writes its partial sums there); the key of tile (tx, ty) of hologram
// b = g / n_per is b tiles_per + ty tiles_x + tx.  offsets[] holds the
// exclusive scans within the preprocess workgroups (256 Gaussians, the same as
// a workgroup here) and chunk_sums their totals: each workgroup adds the
// totals of the workgroups before its own and writes the offsets back, and
// workgroup 0 writes the grand total to offsets[n] and to the pair total
// status[1] (and flags an overflow of the pair capacity).  The workgroup then
// lays its pairs out in LDS in slot order, kEmitChunk at a time, and sorts
// them on the first digit exactly as k_radix_scatter does, with the
// preprocess's digit histogram of the workgroup (hist_scan: scanned, digit-
// major over the workgroups; per chunk of kScanItems with the chunk sums in
// hchunk_sums, or globally when hchunk_sums is null).  A pair's position is
// below the pair total, and positions at or past the capacity are dropped.
// ranges != nullptr: this is also the last pass (one digit covers every tile
// id), and it narrows the tile ranges as the last pass of k_radix_scatter does.
constexpr int kEmitChunk = 1024;  // 8 workgroups per CU fit in LDS

__global__ __launch_bounds__(256) void k_emit_sort(
    int n, int n_per, int tiles_per, const uint32_t *__restrict__ counts,
    uint32_t *__restrict__ offsets, const uint32_t *__restrict__ chunk_sums, int nchunks,
    const uint2 *__restrict__ rect, int tiles_x, int64_t cap,
    const uint32_t *__restrict__ hist_scan, const uint32_t *__restrict__ hchunk_sums,
    int hnchunks, uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
    uint32_t *__restrict__ status, uint2 *__restrict__ ranges, uint32_t num_tiles) {
  constexpr int R = kEmitChunk / 256;  // rounds of 64 pairs per wave
  __shared__ uint32_t wcnt[4][256];    // per-wave digit counts, then local offsets
  __shared__ uint32_t dnext[256];      // global position of the workgroup's next pair of each digit
  __shared__ uint32_t gofs[256];       // global position of local index 0 of each digit
  // the pairs of a chunk (keys, then values); before the first chunk, the
  // scanned chunk sums of the histogram
  __shared__ uint32_t spair[2 * kEmitChunk];
  static_assert(2 * kEmitChunk >= kMaxScanChunks, "room for the chunk sums");
  uint32_t *skey = spair, *sval = spair + kEmitChunk, *cpre = spair;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nb = gridDim.x;
  const int upto = blockIdx.x == 0 ? nchunks : (int)blockIdx.x;
  uint32_t part = 0;
  for (int k = tid; k < upto; k += 256) part += chunk_sums[k];
  uint32_t total;
  block_exclusive_scan(part, &total);  // every thread of the workgroup takes part
  const uint32_t prefix = blockIdx.x == 0 ? 0u : total;
  if (blockIdx.x == 0 && tid == 0) {
    offsets[n] = total;
    status[1] = total;
    if ((int64_t)total > cap) {
      status[0] |= 1u;  // this rasterize
      status[2] |= 1u;  // sticky until the next status read
    }
  }
  const uint32_t npairs = chunk_sums[blockIdx.x];  // this workgroup's pairs
  const int g = blockIdx.x * 256 + tid;
  uint32_t cnt = 0, loc = 0, tx0 = 0, tx1 = 0, ty0 = 0, kb = 0;
  if (g < n) {
    cnt = counts[g];
    loc = offsets[g];
    offsets[g] = loc + prefix;
    const uint2 rc = rect[g];
    tx0 = rc.x & 0xffffu; tx1 = rc.x >> 16; ty0 = rc.y & 0xffffu;
    kb = (uint32_t)(g / n_per) * (uint32_t)tiles_per;
  }
  if (hchunk_sums) {
    // exclusive scan of the histogram's chunk sums, four per thread
    uint32_t c4[4], sum = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = tid * 4 + e;
      c4[e] = sum;
      sum += i < hnchunks ? hchunk_sums[i] : 0u;
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(sum, &tot);
#pragma unroll
    for (int e = 0; e < 4; ++e) cpre[tid * 4 + e] = ex + c4[e];
    __syncthreads();
  }
  {
    const size_t e = (size_t)tid * nb + blockIdx.x;
    dnext[tid] = hist_scan[e] + (hchunk_sums ? cpre[e / kScanItems] : 0u);
  }
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint32_t w = tx1 - tx0 + 1;
  for (uint32_t c0 = 0; c0 < npairs; c0 += kEmitChunk) {  // uniform
    const uint32_t nvalid = min((uint32_t)kEmitChunk, npairs - c0);
    __syncthreads();  // the previous chunk's LDS reads are done
    // this Gaussian's pairs whose slots fall in [c0, c0 + nvalid), in slot order
    if (cnt && loc < c0 + nvalid && loc + cnt > c0) {
      const uint32_t t0 = c0 > loc ? c0 - loc : 0u, t1 = min(cnt, c0 + nvalid - loc);
      uint32_t ty = ty0 + t0 / w, tx = tx0 + t0 % w;
      for (uint32_t t = t0; t < t1; ++t) {
        skey[loc + t - c0] = kb + ty * (uint32_t)tiles_x + tx;
        sval[loc + t - c0] = (uint32_t)g;
        if (++tx > tx1) { tx = tx0; ++ty; }
      }
    }
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) wcnt[ww][tid] = 0;
    __syncthreads();
    // ranks: wave w owns local indices 64 q w + (0 .. 64 q - 1), 64 at a time in
    // index order, with q = ceil(nvalid / 256) <= R rounds per wave
    const uint32_t q = (nvalid + 255u) / 256u;
    const uint32_t first = 64u * q * wave + lane;
    uint32_t key[R], val[R], rank[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      key[r] = 0u;
      val[r] = 0u;
      rank[r] = 0u;
      if ((uint32_t)r >= q) continue;  // uniform
      const uint32_t i = first + 64u * r;
      const bool valid = i < nvalid;
      key[r] = valid ? skey[i] : 0u;
      val[r] = valid ? sval[i] : 0u;
      const uint32_t d = key[r] & 255u;
      uint64_t m = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const bool on = (d >> bit) & 1u;
        const uint64_t bb = __ballot(on);
        m &= on ? bb : ~bb;
      }
      const uint32_t before = __popcll(m & lt);
      const uint32_t prev = wcnt[wave][d];
      rank[r] = prev + before;
      // the lowest lane of each digit group advances the wave's count; this
      // wave's LDS accesses complete in order, so the next round reads it
      if (valid && before == 0) wcnt[wave][d] = prev + (uint32_t)__popcll(m);
    }
    __syncthreads();
    {
      // thread tid = digit d: the chunk's local offsets of d per wave, and the
      // global position of d's local index 0
      uint32_t c[4], tot = 0;
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) { c[ww] = wcnt[ww][tid]; tot += c[ww]; }
      uint32_t all;
      const uint32_t lbase = block_exclusive_scan(tot, &all);
      uint32_t run = lbase;
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        wcnt[ww][tid] = run;
        run += c[ww];
      }
      gofs[tid] = dnext[tid] - lbase;
      dnext[tid] += tot;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if ((uint32_t)r < q && first + 64u * r < nvalid) {
        const uint32_t lp = wcnt[wave][key[r] & 255u] + rank[r];
        if (lp < (uint32_t)kEmitChunk) {  // always true for consistent counts; guards the write
          skey[lp] = key[r];
          sval[lp] = val[r];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = (uint32_t)tid + 256u * r;
      if ((uint32_t)r < q && i < nvalid) {
        const uint32_t k = skey[i];
        const uint32_t pos = gofs[k & 255u] + i;
        if ((int64_t)pos < cap) {  // drops what is past the capacity
          vout[pos] = sval[i];
          if (!ranges) {
            kout[pos] = k;
          } else if (k < num_tiles) {  // keys are tile ids; guards the atomics
            if (i == 0 || skey[i - 1] != k) atomicMin(&ranges[k].x, pos);
            if (i + 1 == nvalid || skey[i + 1] != k) atomicMax(&ranges[k].y, pos + 1u);
          }
        }
      }
    }
  }
}

// the record after the last Gaussian slot: all zeros (zero amplitude), used to
// pad per-wave lists in the forward rasterizer
__global__ void k_zero_record(float *rec, int slot, int rs, float2 *alim) {
  if ((int)threadIdx.x < rs) rec[(size_t)slot * rs + threadIdx.x] = 0.f;
  if (alim && threadIdx.x == 0) alim[slot] = make_float2(0.f, 0.f);  // G = 1 times amplitude 0
}

hipError_t launch_zero_record(const Ctx &c, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_record, dim3(1), dim3(64), 0, s, c.rec,
                     (int)total_gaussians(c, c.cfg.max_gaussians), c.rec_stride, c.alim);
  return hipGetLastError();
}


__global__ void k_zero_u32(uint32_t *p, int len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) p[i] = 0u;
}

// the status words: overflow of the last rasterize, its pair total, and the
// overflow flag that stays set until cgh_read_status reads it
hipError_t launch_zero_status(const Ctx &c, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, c.status, 4);
  return hipGetLastError();
}

hipError_t launch_binning(Ctx &c, int n, hipStream_t s) {
  // status[0] (overflow) and status[1] (pair total) restart: the preprocess
  // clears the flag and the emit writes the total
  const int total = (int)total_gaussians(c, n);
  if (total <= 0) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, c.status, 2);
    const int words = 2 * c.num_tiles;  // every range empty: (0, 0)
    hipLaunchKernelGGL(k_zero_u32, dim3((words + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<uint32_t *>(c.ranges), words);
    c.sorted = 0;
    return hipGetLastError();
  }
  // scans of the digit-major histograms: per chunk of kScanItems, each sort
  // workgroup scanning the chunk sums itself, or globally for long histograms
  auto scan_hist = [&](int hlen, const uint32_t **chunks, int *nchunks) -> hipError_t {
    *nchunks = (hlen + kScanItems - 1) / kScanItems;
    *chunks = nullptr;
    if (*nchunks <= kMaxScanChunks) {
      hipLaunchKernelGGL(k_scan_local, dim3(*nchunks), dim3(256), 0, s, c.hist, c.hist, hlen,
                         c.hist_chunks, nullptr);
      *chunks = c.hist_chunks;
      return hipGetLastError();
    }
    return scan_u32(c.hist, c.hist, hlen, c.hist_chunks, nullptr, nullptr, s);
  };
  // first pass: the preprocess counted the first digit per workgroup of 256
  // Gaussians; the emit sorts each workgroup's pairs on it
  const int nb = (total + 255) / 256;
  const uint32_t *chunks;
  int nchunks;
  hipError_t e = scan_hist(256 * nb, &chunks, &nchunks);
  if (e != hipSuccess) return e;
  const bool atomic_ranges = c.num_tiles <= kMaxAtomicRangeTiles;
  bool last = c.sort_passes == 1 && atomic_ranges;
  hipLaunchKernelGGL(k_emit_sort, dim3(nb), dim3(256), 0, s, total, n, c.tiles_per, c.counts,
                     c.offsets, c.scan_tmp, nb, c.rect, c.tiles_x, c.pair_cap, c.hist, chunks,
                     nchunks, last ? nullptr : c.keys[1], c.vals[1], c.status,
                     last ? c.ranges : nullptr, (uint32_t)c.num_tiles);
  int cur = 1;
  for (int pass = 1; pass < c.sort_passes; ++pass) {
    const int shift = pass * kSortBits;
    hipLaunchKernelGGL(k_radix_hist, dim3(c.sort_blocks), dim3(256), 0, s, c.keys[cur],
                       c.status, c.pair_cap, shift, c.hist, c.sort_blocks);
    e = scan_hist(256 * c.sort_blocks, &chunks, &nchunks);
    if (e != hipSuccess) return e;
    last = pass + 1 == c.sort_passes && atomic_ranges;
    hipLaunchKernelGGL(k_radix_scatter, dim3(c.sort_blocks), dim3(256), 0, s, c.keys[cur],
                       c.vals[cur], last ? nullptr : c.keys[cur ^ 1], c.vals[cur ^ 1], c.status,
                       c.pair_cap, shift, c.hist, c.sort_blocks, chunks, nchunks,
                       last ? c.ranges : nullptr, (uint32_t)c.num_tiles);
    cur ^= 1;
  }
  c.sorted = cur;
  if (!atomic_ranges) {
    const int64_t grid = std::min<int64_t>((c.pair_cap + 255) / 256, (int64_t)c.num_cu * 8);
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)grid), dim3(256), 0, s, c.keys[cur], c.status,
                       c.pair_cap, c.ranges, (uint32_t)c.num_tiles);
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Forward: U_c(p) = sum over the tile's Gaussians with log2 G(p) >= -k^2/2 log2 e
// of G(p) (alpha c cos phi + j alpha c sin phi).
// Each wave owns an 8x8 sub-block: it culls the tile's Gaussians against its
// sub-block (one Gaussian per lane), writes the survivors to a per-wave list
// together with the sub-block origin's offset from their mean, and walks the
// list two Gaussians at a time.  The list entries and records are wave-uniform,
// so they come in through scalar registers; per pixel and Gaussian only
// d = (pixel offset in the sub-block) + (origin offset) is left to compute.
// Slot kBatch pads the list to even length with the all-zero record.
// ----------------------------------------------------------------------------
constexpr int kBatch = 256;

// CLAMP: the support threshold lies at or below the exponent clamp (unbounded
// support), so the clamp has to be applied; otherwise every exponent that
// passes the threshold is above the clamp already.
// PA: the Alg. 2 weight (CGH_PAPER_ALPHA): G = 2^min(p, hi) where p >= lo, else 0
template <int C, bool CLAMP, bool PA>
__device__ __forceinline__ void accumulate(const float *r, float offx, float offy, float flx,
                                           float fly, float thr, float lo, float hi, float *ar,
                                           float *ai) {
  const float dx = flx + offx, dy = fly + offy;
  const float p2 = fmaf(dx, fmaf(r[R_A], dx, r[R_B] * dy), r[R_C] * dy * dy);
  float G;
  if (PA)
    G = p2 >= lo ? __builtin_amdgcn_exp2f(fminf(p2, hi)) : 0.f;
  else
    G = p2 >= thr ? __builtin_amdgcn_exp2f(CLAMP ? fmaxf(p2, kPowerFloor2) : p2) : 0.f;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    ar[c] = fmaf(G, r[R_AMP + 2 * c], ar[c]);
    ai[c] = fmaf(G, r[R_AMP + 2 * c + 1], ai[c]);
  }
}

// zero_id: index of an all-zero record (after the last Gaussian slot).
// The tile is SBX x SBY sub-blocks of 8 x 8 pixels, one wave each.
template <int C, bool CLAMP, bool PA, int SBX, int SBY>
__global__ __launch_bounds__(64 * SBX * SBY) void k_raster_fwd(
    const float *__restrict__ rec, const uint32_t *__restrict__ vals,
    const uint2 *__restrict__ ranges, int W, int H, int tiles_x, int tiles_per, float thr,
    uint32_t zero_id, const float2 *__restrict__ alim, float2 *__restrict__ field_all) {
  constexpr int RS = rec_stride_c(C);
  constexpr int NW = SBX * SBY;
  // (Gaussian id, origin offset x, origin offset y) of the surviving Gaussians
  __shared__ uint4 list[NW][kBatch + 2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tile = blockIdx.x;
  const int hb = tile / tiles_per, ltile = tile - hb * tiles_per;  // hologram, its tile
  float2 *field = field_all + (size_t)hb * C * H * W;
  const int tx = ltile % tiles_x, ty = ltile / tiles_x;
  const int Xt = tx * (8 * SBX), Yt = ty * (8 * SBY);  // tile origin
  const int sx = (wave % SBX) * 8, sy = (wave / SBX) * 8;  // sub-block origin in the tile
  const int X0 = Xt + sx, Y0 = Yt + sy;
  const int lx = lane & 7, ly = lane >> 3;
  // pixel offsets from the tile origin: d = (x - Xt) + ((Xt - floor(mean)) - frac(mean)),
  // the same FP32 operations as the adjoint's
  const float flx = (float)(sx + lx), fly = (float)(sy + ly);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  float ar[C], ai[C];
#pragma unroll
  for (int c = 0; c < C; ++c) { ar[c] = 0.f; ai[c] = 0.f; }
  const uint2 rg = ranges[tile];
  for (uint32_t base = rg.x; base < rg.y; base += kBatch) {
    const int cnt = (int)min((uint32_t)kBatch, rg.y - base);
    // cull the batch against this wave's sub-block (one Gaussian per lane per
    // round); the ids of the survivors go to list[wave], in list order
    // the ids of all rounds are loaded first, then the records they name
    // (one latency each rather than two per round)
    constexpr int QD = kBatch / 64;
    uint32_t gid[QD];
#pragma unroll
    for (int qd = 0; qd < QD; ++qd) {
      const int idx = qd * 64 + lane;
      gid[qd] = idx < cnt ? vals[base + idx] : zero_id;
    }
    float4 r0[QD], r1[QD];
    float ryv[QD];
#pragma unroll
    for (int qd = 0; qd < QD; ++qd) {
      // r0 = (mix, miy, mfx, mfy), r1 = (a, b, c, rx); ry is element 8
      const float *rg0 = rec + (size_t)gid[qd] * RS;
      r0[qd] = reinterpret_cast<const float4 *>(rg0)[0];
      r1[qd] = reinterpret_cast<const float4 *>(rg0)[1];
      ryv[qd] = rg0[R_RY];
    }
    int n = 0;
#pragma unroll
    for (int qd = 0; qd < QD; ++qd) {
      const int idx = qd * 64 + lane;
      // offsets of the tile origin from the mean (kept in the list), and of
      // the sub-block's pixels: dx in [ex0, ex0 + 7], dy in [ey0, ey0 + 7]
      // (to rounding; the culling test below has a margin)
      const float ext = (float)(Xt - __float_as_int(r0[qd].x)) - r0[qd].z;
      const float eyt = (float)(Yt - __float_as_int(r0[qd].y)) - r0[qd].w;
      const float ex0 = ext + (float)sx, ey0 = eyt + (float)sy;
      const float rx = r1[qd].w + 0.01f, ry = ryv[qd] + 0.01f;
      bool hit = idx < cnt && (ex0 <= rx) && (ex0 + 7.f >= -rx) && (ey0 <= ry) &&
                 (ey0 + 7.f >= -ry);
      if (hit && thr > -INFINITY) {
        // the support box touches the sub-block; keep the Gaussian only if the
        // maximum of the (concave) exponent over the sub-block's rectangle
        // reaches the threshold (with a margin for rounding)
        const float a = r1[qd].x, b = r1[qd].y, c = r1[qd].z;
        const float ex1 = ex0 + 7.f, ey1 = ey0 + 7.f;
        const bool inside = ex0 <= 0.f && ex1 >= 0.f && ey0 <= 0.f && ey1 >= 0.f;
        const float ka = -0.5f * b / a, kc = -0.5f * b / c;
        auto on_x = [&](float e) {  // edge dx = e: maximise over dy
          const float t = fminf(fmaxf(kc * e, ey0), ey1);
          return e * (a * e + b * t) + c * t * t;
        };
        auto on_y = [&](float f) {  // edge dy = f: maximise over dx
          const float t = fminf(fmaxf(ka * f, ex0), ex1);
          return t * (a * t + b * f) + c * f * f;
        };
        const float best = fmaxf(fmaxf(on_x(ex0), on_x(ex1)), fmaxf(on_y(ey0), on_y(ey1)));
        hit = inside || best >= thr - 1e-3f * (1.f - thr);
      }
      const uint64_t m = __ballot(hit);
      if (hit)
        list[wave][n + __popcll(m & lt)] =
            make_uint4(gid[qd], __float_as_uint(ext), __float_as_uint(eyt), 0u);
      n += __popcll(m);
    }
    if (lane == 0) list[wave][n] = make_uint4(zero_id, 0u, 0u, 0u);  // pad to even length
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // walk the list two at a time: the record addresses are wave-uniform, so
    // the records come in through scalar loads and feed the VALU as scalar
    // operands; both pairs of loads are issued before either is used.  The
    // offsets stay in (uniform) vector registers: the adds take them as they are.
    for (int k = 0; k < n; k += 2) {
      const uint4 e0 = list[wave][k], e1 = list[wave][k + 1];
      const uint32_t g0 = __builtin_amdgcn_readfirstlane(e0.x);
      const uint32_t g1 = __builtin_amdgcn_readfirstlane(e1.x);
      const float ox0 = __uint_as_float(e0.y), oy0 = __uint_as_float(e0.z);
      const float ox1 = __uint_as_float(e1.y), oy1 = __uint_as_float(e1.z);
      const float *s0 = rec + (size_t)g0 * RS;
      const float *s1 = rec + (size_t)g1 * RS;
      float r0[R_AMP + 2 * C], r1[R_AMP + 2 * C];
#pragma unroll
      for (int i = R_A; i < R_AMP + 2 * C; ++i) { r0[i] = s0[i]; r1[i] = s1[i]; }
      float2 l0 = make_float2(0.f, 0.f), l1 = make_float2(0.f, 0.f);
      if (PA) { l0 = alim[g0]; l1 = alim[g1]; }
      accumulate<C, CLAMP, PA>(r0, ox0, oy0, flx, fly, thr, l0.x, l0.y, ar, ai);
      accumulate<C, CLAMP, PA>(r1, ox1, oy1, flx, fly, thr, l1.x, l1.y, ar, ai);
    }
    __builtin_amdgcn_wave_barrier();
  }
  const int px = X0 + lx, py = Y0 + ly;
  if (px < W && py < H) {
#pragma unroll
    for (int c = 0; c < C; ++c) field[((size_t)c * H + py) * W + px] = make_float2(ar[c], ai[c]);
  }
}

// ----------------------------------------------------------------------------
// Forward, row-segment form (tiles 16 or 32 pixels wide, without the Alg. 2
// weight).  The tile is cut into segments of 16 pixels of one row, and a wave
// owns four segments, one per DPP row of 16 lanes: lane i of row g is pixel i
// of segment 4 wave + g.  Along a pixel row the exponent is
//   log2 G = kappa dy^2 - (ra (dx - s dy))^2          (dx, dy = pixel - mean)
// (the record's row form), so with u = x - (segment centre) in [-7.5, 7.5]
//   w = ra u + m,   log2 G = qmax - w^2,
//   m = ra ((segment centre - mean_x) - s dy),   qmax = kappa dy^2
// per (Gaussian, segment).  The largest exponent over the segment is
// qmax - max(0, |m| - 7.5 ra)^2, and a Gaussian is listed for the segment only
// where that reaches the support threshold, so no pixel row outside the
// support is walked.  The walk takes sixteen listed Gaussians per row at a
// time, one per lane (m, qmax, ra from the list, amplitudes from the record),
// and broadcasts them across the row one after another with DPP row_newbcast:
// the four rows of a wave step through four different lists in one
// instruction stream, and each listed Gaussian costs 7 + 2C instructions per
// 16 pixels.  Lists keep the tile-list order, so the sums are reproducible.
// ----------------------------------------------------------------------------
constexpr int kSegBatch = 128;  // Gaussians culled per batch (two per lane of each wave)

#define CGH_NB(j) " row_newbcast:" #j " row_mask:0xf bank_mask:0xf\n"
// two steps (lanes ja, jb of each row): exponents into pa, pb
#define CGH_P2(ja, jb)                                  \
  "v_mov_b32_dpp %[wa], %[m]" CGH_NB(ja)                \
  "v_mov_b32_dpp %[wb], %[m]" CGH_NB(jb)                \
  "v_fmac_f32_dpp %[wa], %[ra], %[u]" CGH_NB(ja)        \
  "v_fmac_f32_dpp %[wb], %[ra], %[u]" CGH_NB(jb)        \
  "v_mul_f32_e32 %[wa], %[wa], %[wa]\n"                 \
  "v_mul_f32_e32 %[wb], %[wb], %[wb]\n"                 \
  "v_sub_f32_dpp %[pa], %[qm], %[wa]" CGH_NB(ja)        \
  "v_sub_f32_dpp %[pb], %[qm], %[wb]" CGH_NB(jb)
// G = 2^p where p >= thr, else 0 (into wa, wb).  The comparisons are issued
// first: a lane mask written by a VALU compare needs two wait states before
// v_cndmask reads it, and a v_exp result one.
#define CGH_G                                           \
  "v_cmp_le_f32_e32 vcc, %[thr], %[pa]\n"               \
  "v_cmp_le_f32_e64 %[sb], %[thr], %[pb]\n"             \
  "v_exp_f32_e32 %[wa], %[pa]\n"                        \
  "v_exp_f32_e32 %[wb], %[pb]\n"                        \
  "v_cndmask_b32_e32 %[wa], 0, %[wa], vcc\n"            \
  "v_cndmask_b32_e64 %[wb], 0, %[wb], %[sb]\n"
// the same with the exponent clamped at fl from below (unbounded support)
#define CGH_G_CLAMP                                     \
  "v_cmp_le_f32_e32 vcc, %[thr], %[pa]\n"               \
  "v_cmp_le_f32_e64 %[sb], %[thr], %[pb]\n"             \
  "v_max_f32_e32 %[pa], %[fl], %[pa]\n"                 \
  "v_max_f32_e32 %[pb], %[fl], %[pb]\n"                 \
  "v_exp_f32_e32 %[wa], %[pa]\n"                        \
  "v_exp_f32_e32 %[wb], %[pb]\n"                        \
  "v_cndmask_b32_e32 %[wa], 0, %[wa], vcc\n"            \
  "v_cndmask_b32_e64 %[wb], 0, %[wb], %[sb]\n"
#define CGH_ACC(j, g, k) "v_fmac_f32_dpp %[a" #k "], %[c" #k "], %[" g "]" CGH_NB(j)
#define CGH_ACC1(j, g) CGH_ACC(j, g, 0) CGH_ACC(j, g, 1)
#define CGH_ACC2(j, g) CGH_ACC1(j, g) CGH_ACC(j, g, 2) CGH_ACC(j, g, 3)
#define CGH_ACC3(j, g) CGH_ACC2(j, g) CGH_ACC(j, g, 4) CGH_ACC(j, g, 5)
#define CGH_ACC4(j, g) CGH_ACC3(j, g) CGH_ACC(j, g, 6) CGH_ACC(j, g, 7)
// four steps, lanes j0..j3.  The s_nop gives the two wait states a DPP source
// needs after a VALU write (the sources are not written inside the block).
#define CGH_STEP4(ACC, GEXP, j0, j1, j2, j3)                                       \
  "s_nop 1\n" CGH_P2(j0, j1) GEXP ACC(j0, "wa") ACC(j1, "wb") CGH_P2(j2, j3) GEXP \
      ACC(j2, "wa") ACC(j3, "wb")

// accumulators a[2C] (re, im per channel), amplitudes c[2C] of the lane's
// listed Gaussian; runs steps 4 q .. 4 q + 3
#define CGH_OPS_COMMON                                                          \
  [wa] "=&v"(wa), [wb] "=&v"(wb), [pa] "=&v"(pa), [pb] "=&v"(pb), [sb] "=&s"(sb)
template <int C, bool CLAMP, int Q>
__device__ __forceinline__ void seg_steps(float (&a)[2 * C], const float (&cv)[2 * C], float m,
                                          float ra, float qm, float u, float thr, float fl) {
  float wa, wb, pa, pb;
  uint64_t sb;
#define CGH_IN [m] "v"(m), [ra] "v"(ra), [qm] "v"(qm), [u] "v"(u), [thr] "s"(thr), [fl] "s"(fl)
#define CGH_RUN(N, GEXP, j0, j1, j2, j3)                                           \
  asm volatile(CGH_STEP4(CGH_ACC##N, GEXP, j0, j1, j2, j3)                           \
               : CGH_OPS_COMMON, CGH_O##N                                           \
               : CGH_IN, CGH_I##N                                                   \
               : "vcc")
#define CGH_O1 [a0] "+v"(a[0]), [a1] "+v"(a[1])
#define CGH_O2 CGH_O1, [a2] "+v"(a[2]), [a3] "+v"(a[3])
#define CGH_O3 CGH_O2, [a4] "+v"(a[4]), [a5] "+v"(a[5])
#define CGH_O4 CGH_O3, [a6] "+v"(a[6]), [a7] "+v"(a[7])
#define CGH_I1 [c0] "v"(cv[0]), [c1] "v"(cv[1])
#define CGH_I2 CGH_I1, [c2] "v"(cv[2]), [c3] "v"(cv[3])
#define CGH_I3 CGH_I2, [c4] "v"(cv[4]), [c5] "v"(cv[5])
#define CGH_I4 CGH_I3, [c6] "v"(cv[6]), [c7] "v"(cv[7])
#define CGH_BY_Q(N, GEXP)                                     \
  if constexpr (Q == 0) CGH_RUN(N, GEXP, 0, 1, 2, 3);         \
  else if constexpr (Q == 1) CGH_RUN(N, GEXP, 4, 5, 6, 7);    \
  else if constexpr (Q == 2) CGH_RUN(N, GEXP, 8, 9, 10, 11);  \
  else CGH_RUN(N, GEXP, 12, 13, 14, 15)
#define CGH_BY_G(N)                                             \
  if constexpr (CLAMP) { CGH_BY_Q(N, CGH_G_CLAMP); } else { CGH_BY_Q(N, CGH_G); }
  if constexpr (C == 1) { CGH_BY_G(1); }
  else if constexpr (C == 2) { CGH_BY_G(2); }
  else if constexpr (C == 3) { CGH_BY_G(3); }
  else { CGH_BY_G(4); }
#undef CGH_IN
#undef CGH_RUN
#undef CGH_O1
#undef CGH_O2
#undef CGH_O3
#undef CGH_O4
#undef CGH_I1
#undef CGH_I2
#undef CGH_I3
#undef CGH_I4
#undef CGH_BY_Q
#undef CGH_BY_G
}

template <int C, bool CLAMP, int TW, int TH>
__global__ __launch_bounds__(TW * TH) void k_raster_seg(
    const float *__restrict__ rec, const uint32_t *__restrict__ vals,
    const uint2 *__restrict__ ranges, int W, int H, int tiles_x, int tiles_per, float thr,
    uint32_t zero_id, float2 *__restrict__ field_all) {
  constexpr int RS = rec_stride_c(C), RX = rec_ext_c(C);
  constexpr int SPR = TW / 16;  // segments per pixel row
  constexpr int NW = SPR * TH / 4;
  static_assert(TW % 16 == 0 && (SPR * TH) % 4 == 0, "tile shape");
  // (Gaussian id bits, m, qmax, ra) of the listed Gaussians of each segment
  __shared__ float4 list[NW][4][kSegBatch];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = blockIdx.x;
  const int hb = tile / tiles_per, ltile = tile - hb * tiles_per;  // hologram, its tile
  float2 *field = field_all + (size_t)hb * C * H * W;
  const int tx = ltile % tiles_x, ty = ltile / tiles_x;
  const int Xt = tx * TW, Yt = ty * TH;  // tile origin
  // this lane's pixel: row rg = lane / 16 of the wave, pixel lane % 16 of segment
  // 4 wave + rg
  const int rg = lane >> 4, seg = 4 * wave + rg;
  const int sr = seg / SPR, sc = seg % SPR;
  const int px = Xt + 16 * sc + (lane & 15), py = Yt + sr;
  const float u = (float)(lane & 15) - 7.5f;
  const float fl = kPowerFloor2;
  const float cull = thr - 1e-3f * (1.f - thr);  // margin for rounding
  float acc[2 * C];
#pragma unroll
  for (int k = 0; k < 2 * C; ++k) acc[k] = 0.f;
  const uint2 rng = ranges[tile];
  // a batch's Gaussian ids and record heads; the next batch's ids are loaded
  // before this batch is culled and its records before this batch is walked
  constexpr int QD = kSegBatch / 64;
  uint32_t ngid[QD];
  float4 nr0[QD], nrx[QD];
  auto load_ids = [&](uint32_t b) {
#pragma unroll
    for (int qd = 0; qd < QD; ++qd) {
      const uint32_t idx = b + qd * 64 + lane;
      ngid[qd] = idx < rng.y ? vals[idx] : zero_id;
    }
  };
  auto load_heads = [&] {
#pragma unroll
    for (int qd = 0; qd < QD; ++qd) {
      const float *g0 = rec + (size_t)ngid[qd] * RS;
      nr0[qd] = reinterpret_cast<const float4 *>(g0)[0];       // mix, miy, mfx, mfy
      nrx[qd] = reinterpret_cast<const float4 *>(g0 + RX)[0];  // s, kappa, ra
    }
  };
  if (rng.x < rng.y) {
    load_ids(rng.x);
    load_heads();
  }
  for (uint32_t base = rng.x; base < rng.y; base += kSegBatch) {
    const int cnt = (int)min((uint32_t)kSegBatch, rng.y - base);
    // ---- cull: each lane takes one Gaussian per round against the wave's
    // four segments; survivors are appended to the segment lists in order
    uint32_t gid[QD];
    float4 r0[QD], rx[QD];
#pragma unroll
    for (int qd = 0; qd < QD; ++qd) {
      gid[qd] = ngid[qd];
      r0[qd] = nr0[qd];
      rx[qd] = nrx[qd];
    }
    const bool more = base + kSegBatch < rng.y;  // uniform
    if (more) load_ids(base + kSegBatch);
    int nl[4] = {0, 0, 0, 0};  // list lengths (wave-uniform)
#pragma unroll
    for (int qd = 0; qd < QD; ++qd) {
      if (qd * 64 >= cnt) break;  // uniform
      // lanes past the batch end: a scalar mask, so that each segment's ballot
      // takes its comparison's lane mask as it is
      const int nv = min(64, cnt - qd * 64);
      const uint64_t vmask = nv >= 64 ? ~0ull : ((1ull << nv) - 1ull);
      const bool in_batch = lane < nv;
      const float oxt = (float)(Xt - __float_as_int(r0[qd].x)) - r0[qd].z;
      const float eyt = (float)(Yt - __float_as_int(r0[qd].y)) - r0[qd].w;
      const float s = rx[qd].x, kap = rx[qd].y, ra = rx[qd].z;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int sg = 4 * wave + g;
        const float dy = eyt + (float)(sg / SPR);
        const float oxc = oxt + (float)(16 * (sg % SPR)) + 7.5f;
        const float qm = kap * dy * dy;
        const float m = ra * fmaf(-s, dy, oxc);
        const float d = fmaxf(fmaf(-7.5f, ra, fabsf(m)), 0.f);
        const bool pass = fmaf(-d, d, qm) >= cull;
        const uint64_t bm = __builtin_amdgcn_ballot_w64(pass) & vmask;
        if (pass && in_batch) {
          const int pos = nl[g] + (int)__builtin_amdgcn_mbcnt_hi(
                                      (uint32_t)(bm >> 32),
                                      __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u));
          list[wave][g][pos] = make_float4(__uint_as_float(gid[qd]), m, qm, ra);
        }
        nl[g] += __popcll(bm);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (more) load_heads();
    // ---- walk: sixteen entries of each row's list per round; the entries
    // and amplitudes of the next round are loaded while this one runs
    const int nmax = max(max(nl[0], nl[1]), max(nl[2], nl[3]));
    const int nmine = rg == 0 ? nl[0] : rg == 1 ? nl[1] : rg == 2 ? nl[2] : nl[3];
    auto fetch = [&](int b0, float4 &e, float (&cv)[2 * C]) {
      const int j = b0 + (lane & 15);
      e = list[wave][rg][min(j, kSegBatch - 1)];
      if (j >= nmine) e = make_float4(__uint_as_float(zero_id), 0.f, 0.f, 0.f);
      const float *amp = rec + (size_t)__float_as_uint(e.x) * RS + R_AMP;
#pragma unroll
      for (int k = 0; k < 2 * C; ++k) cv[k] = amp[k];
    };
    auto walk_round = [&](int b0, const float4 &e, const float (&cv)[2 * C]) {
      const int left = nmax - b0;
      seg_steps<C, CLAMP, 0>(acc, cv, e.y, e.w, e.z, u, thr, fl);
      if (left > 4) seg_steps<C, CLAMP, 1>(acc, cv, e.y, e.w, e.z, u, thr, fl);
      if (left > 8) seg_steps<C, CLAMP, 2>(acc, cv, e.y, e.w, e.z, u, thr, fl);
      if (left > 12) seg_steps<C, CLAMP, 3>(acc, cv, e.y, e.w, e.z, u, thr, fl);
    };
    // two rounds per iteration with the two entry sets in alternate roles, so
    // no registers are copied between rounds; the next round's fetch is
    // issued on every round (past the end it reads zero entries), so the wait
    // before the steps covers only this round's loads
    float4 ea, eb;
    float ca[2 * C], cb[2 * C];
    if (nmax > 0) fetch(0, ea, ca);
    for (int b0 = 0; b0 < nmax; b0 += 32) {
      fetch(b0 + 16, eb, cb);
      walk_round(b0, ea, ca);
      if (b0 + 16 >= nmax) break;
      fetch(b0 + 32, ea, ca);
      walk_round(b0 + 16, eb, cb);
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (px < W && py < H) {
#pragma unroll
    for (int c = 0; c < C; ++c)
      field[((size_t)c * H + py) * W + px] = make_float2(acc[2 * c], acc[2 * c + 1]);
  }
}
#undef CGH_NB
#undef CGH_P2
#undef CGH_G
#undef CGH_G_CLAMP
#undef CGH_ACC
#undef CGH_ACC1
#undef CGH_ACC2
#undef CGH_ACC3
#undef CGH_ACC4
#undef CGH_STEP4
#undef CGH_OPS_COMMON

// calls f(integral_constant<TW>, integral_constant<TH>) for the context's tile
template <class F>
static void with_tile(const Ctx &c, F &&f) {
  using std::integral_constant;
  if (c.tile_w == 32 && c.tile_h == 8) f(integral_constant<int, 32>{}, integral_constant<int, 8>{});
  else if (c.tile_w == 16 && c.tile_h == 8) f(integral_constant<int, 16>{}, integral_constant<int, 8>{});
  else if (c.tile_w == 8 && c.tile_h == 8) f(integral_constant<int, 8>{}, integral_constant<int, 8>{});
  else f(integral_constant<int, 16>{}, integral_constant<int, 16>{});
}

template <class F>
static void with_channels(int C, F &&f) {
  using std::integral_constant;
  switch (C) {
    case 1: f(integral_constant<int, 1>{}); break;
    case 2: f(integral_constant<int, 2>{}); break;
    case 3: f(integral_constant<int, 3>{}); break;
    default: f(integral_constant<int, 4>{}); break;
  }
}

hipError_t launch_raster_fwd(const Ctx &c, float2 *field, hipStream_t s) {
  const float thr = support_threshold(c.cfg.support_sigma);
  // the zero record, after the last Gaussian slot of every hologram
  const uint32_t zid = (uint32_t)((int64_t)c.B * c.cfg.max_gaussians);
  const uint32_t *vals = c.vals[c.sorted];
  const bool clamp = !(thr > kPowerFloor2);
  const bool pa = c.alim != nullptr;  // the clamp of the exponent never binds there
  with_tile(c, [&](auto tw, auto th) {
    constexpr int SBX = decltype(tw)::value / 8, SBY = decltype(th)::value / 8;
    with_channels(c.C, [&](auto cc) {
      constexpr int CC = decltype(cc)::value;
      dim3 grid(c.num_tiles), block(64 * SBX * SBY);
      auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, block, 0, s, c.rec, vals, c.ranges, c.W, c.H, c.tiles_x,
                           c.tiles_per, thr, zid, c.alim, field);
      };
      constexpr int TW = decltype(tw)::value, TH = decltype(th)::value;
      auto go_seg = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(TW * TH), 0, s, c.rec, vals, c.ranges, c.W,
                           c.H, c.tiles_x, c.tiles_per, thr, zid, field);
      };
      if (pa) go(k_raster_fwd<CC, false, true, SBX, SBY>);
      else if constexpr (TW >= 16) {
        if (clamp) go_seg(k_raster_seg<CC, true, TW, TH>);
        else go_seg(k_raster_seg<CC, false, TW, TH>);
      } else if (clamp) go(k_raster_fwd<CC, true, false, SBX, SBY>);
      else go(k_raster_fwd<CC, false, false, SBX, SBY>);
    });
  });
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Adjoint, tile stage.  For a pair (tile, Gaussian) and every pixel of the
// tile inside the Gaussian's support, with g = dL/dU0 (per channel) and
// w = dL/dpower = G sum_c (g_re P_c + g_im Q_c)  (P + jQ = alpha c e^{j phi}):
//   S[2c] += G g_re, S[2c+1] += G g_im           (dL/dP_c, dL/dQ_c)
//   S[2C] += w dx, S[2C+1] += w dy                (-> dL/dmean)
//   S[2C+2] += w dx^2, S[2C+3] += w dx dy, S[2C+4] += w dy^2   (-> dL/dSigma^{-1})
// with dx, dy = pixel - mean.  The clamped exponent has zero derivative.
//
// Work balance.  A workgroup of three waves owns a tile: the tile's dL/dU0 is
// staged in LDS once, the pair list is cut into three equal parts, and each
// wave takes its part in batches of 64 with a pair table of its own in LDS
// (three waves per tile rather than one keep more waves resident per CU,
// since the staged tile is shared).  Each pair's pixel box is cut into segments of 8 pixels (the last one
// padded), the segments of a batch are laid end to end, and the segment range
// is cut into 64 equal contiguous pieces, one per lane, so every lane walks
// the same number of pixels whatever the mix of box sizes.  A lane can move to
// its next pair only at a segment boundary, so that bookkeeping runs once per
// 8 pixels.  A pair that lies inside one lane's piece is written straight to
// its partial slot.  A pair cut by piece boundaries is finished by the lane
// where it starts: that lane adds, in lane order, the first part of each
// following lane the pair reaches (shuffled across the wave).  The cut points
// depend only on the box areas, so the result is bitwise reproducible.
// ----------------------------------------------------------------------------
constexpr int kAdjBatch = 64;
constexpr int kAdjSeg = 8;    // pixels per segment
constexpr int kAdjRowPad = 1;  // float2 of padding after each staged tile row (bank spread)
constexpr int kAdjWaves = 3;  // waves per tile; wave w takes part w of kAdjWaves of the list

// per-pair quantities kept in LDS for the walk (floats):
//   0-1 offx, offy (tile origin - floor(mean) - frac(mean))
//   2-4 a, b, c;  5.. amplitude (2C);  then box, first segment, slot (int bits)
// The stride N is a multiple of 4 floats (16-byte reads) with N / 4 odd: lanes
// reading different pairs then spread their 16-byte reads over all LDS banks.
// PA (CGH_PAPER_ALPHA) adds the exponent limits (lo, hi) of the pair's Gaussian
template <int C, bool PA> struct AdjQ {
  static constexpr int AMP = 5;
  static constexpr int BOX = 5 + 2 * C, START = BOX + 1, SLOT = BOX + 2;
  static constexpr int LO = SLOT + 1, HI = SLOT + 2;
  static constexpr int N4 = ((SLOT + 1 + (PA ? 2 : 0)) + 3) & ~3;
  static constexpr int N = (N4 / 4) % 2 ? N4 : N4 + 4;
};

// Pair partials: dP_c, dQ_c (2C), sum w d (2), sum w d d^T (3); with PA one more,
// the sum of G gp over the pixels where the 0.99 clamp is active (their
// weight does not depend on alpha), in the slot that the stride leaves spare.
template <int C, bool CLAMP, bool PA, int TW, int TH>
__global__ __launch_bounds__(64 * kAdjWaves) void k_raster_adj(
    const float *__restrict__ rec, const uint32_t *__restrict__ vals,
    const uint2 *__restrict__ ranges, const uint2 *__restrict__ rect,
    const uint32_t *__restrict__ offsets, int W, int H, int tiles_x, int tiles_per, float thr,
    const float2 *__restrict__ alim, const float2 *__restrict__ gfield_all, int64_t cap,
    float *__restrict__ partials) {
  constexpr int RS = rec_stride_c(C), RX = rec_ext_c(C);
  constexpr int PS = part_stride_c(C);
  constexpr int NS = 2 * C + 5 + (PA ? 1 : 0);
  static_assert(NS <= PS, "the clamped-pixel sum needs a spare partial slot");
  using Q = AdjQ<C, PA>;
  constexpr int TP = TW * TH;  // pixels of the tile
  static_assert(TP % 64 == 0 && TW * C <= 64 * 4, "tile shape");
  // dL/dU0 of the tile, plus one row of zeros (row TH) that the padding
  // pixels of a pair's last segment read when they run past the tile's last
  // row; pixel (x, y) channel c at float2 y RS2 + x C + c (RS2: the row
  // stride, kAdjRowPad float2 longer than a row).  One LDS block, so that the
  // staged tile starts at LDS address 0 and the walk's reads take their
  // offsets as immediates.
  constexpr int RS2 = TW * C + kAdjRowPad;
  constexpr int kSg4 = ((TH + 1) * RS2 * 2 + 3) / 4, kSq4 = kAdjBatch * Q::N / 4;
  __shared__ float4 lds4[kSg4 + kAdjWaves * kSq4];
  float2 *sg = reinterpret_cast<float2 *>(lds4);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // each wave's own pair table: after the tile's dL/dU0 is staged, the waves
  // share nothing, and a wave's LDS operations execute in issue order
  float *sq = reinterpret_cast<float *>(lds4 + kSg4 + wave * kSq4);
  auto wave_sync = [] {
    if constexpr (kAdjWaves == 1) __syncthreads();
    else asm volatile("" ::: "memory");
  };
  const int tile = blockIdx.x;
  const int hb = tile / tiles_per, ltile = tile - hb * tiles_per;  // hologram, its tile
  const float2 *gfield = gfield_all + (size_t)hb * C * H * W;
  const int tx = ltile % tiles_x, ty = ltile / tiles_x;
  const int X0 = tx * TW, Y0 = ty * TH;
  {
    // all loads of a thread are issued before the first is stored
    constexpr int NT = 64 * kAdjWaves, K = (C * TP + NT - 1) / NT;
    const int tid = threadIdx.x;
    float2 v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = min(tid + NT * k, C * TP - 1), c = i / TP, p = i % TP;
      const int x = X0 + (p % TW), y = Y0 + (p / TW);
      v[k] = gfield[((size_t)c * H + min(y, H - 1)) * W + min(x, W - 1)];
      if (x >= W || y >= H) v[k] = make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + NT * k;
      if ((C * TP) % NT == 0 || i < C * TP) {
        const int p = i % TP;
        sg[(p / TW) * RS2 + (p % TW) * C + i / TP] = v[k];
      }
    }
    for (int i = tid; i < TW * C; i += NT) sg[TH * RS2 + i] = make_float2(0.f, 0.f);
  }
  if constexpr (kAdjWaves > 1) __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint2 rg = ranges[tile];
  {
    // a tile without pairs has the range (0xffffffff, 0)
    const uint32_t len = rg.y > rg.x ? rg.y - rg.x : 0u;
    rg = make_uint2(rg.x + (uint32_t)(((uint64_t)len * wave) / kAdjWaves),
                    rg.x + (uint32_t)(((uint64_t)len * (wave + 1)) / kAdjWaves));
  }
  for (uint32_t base = rg.x; base < rg.y; base += kAdjBatch) {
    // ---- set-up: one pair per lane --------------------------------------
    const int cnt = (int)min((uint32_t)kAdjBatch, rg.y - base);
    int area = 0;
    int xa = 0, xb = -1, ya = 0, yb = -1;
    uint32_t slot = 0xffffffffu;
    float r[RX];
#pragma unroll
    for (int k = 0; k < RX; ++k) r[k] = 0.f;
    if (lane < cnt) {
      const uint32_t g = vals[base + lane];
      const float4 *src = reinterpret_cast<const float4 *>(rec + (size_t)g * RS);
#pragma unroll
      for (int k = 0; k < RX / 4; ++k) {
        const float4 v = src[k];
        r[4 * k] = v.x; r[4 * k + 1] = v.y; r[4 * k + 2] = v.z; r[4 * k + 3] = v.w;
      }
      const int mix = __float_as_int(r[R_MIX]), miy = __float_as_int(r[R_MIY]);
      // pixel box of the support inside this tile (local coordinates)
      const float rx = fminf(r[R_RX], 1e6f) + 0.01f, ry = fminf(r[R_RY], 1e6f) + 0.01f;
      const float cx = (float)(mix - X0) + r[R_MFX], cy = (float)(miy - Y0) + r[R_MFY];
      xa = max(0, (int)ceilf(fmaxf(cx - rx, -1.f)));
      xb = min(TW - 1, (int)floorf(fminf(cx + rx, (float)TW)));
      ya = max(0, (int)ceilf(fmaxf(cy - ry, -1.f)));
      yb = min(TH - 1, (int)floorf(fminf(cy + ry, (float)TH)));
      if (xb >= xa && yb >= ya) area = (xb - xa + 1) * (yb - ya + 1);
      const uint2 rc = rect[g];
      const uint32_t tx0 = rc.x & 0xffffu, tx1 = rc.x >> 16, ty0 = rc.y & 0xffffu;
      const uint64_t pos = (uint64_t)offsets[g] + (uint64_t)(ty - (int)ty0) * (tx1 - tx0 + 1) +
                           (uint64_t)(tx - (int)tx0);
      if ((int64_t)pos < cap) slot = (uint32_t)pos;
      if (area == 0 && slot != 0xffffffffu) {  // nothing of the support in this tile
        float4 *dst = reinterpret_cast<float4 *>(partials + (size_t)slot * PS);
#pragma unroll
        for (int k = 0; k < PS / 4; ++k) dst[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    // exclusive scan of the segment counts (lane order); the non-empty pairs
    // are compacted to the front of the LDS table in the same order
    const int segs = (area + kAdjSeg - 1) / kAdjSeg;
    int incl = segs;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int v = __shfl_up(incl, d);
      if (lane >= d) incl += v;
    }
    const int start = incl - segs;
    const int total = __shfl(incl, 63);
    const uint64_t nem = __ballot(area > 0);
    const int np = __popcll(nem);
    if (area > 0) {
      const int j = __popcll(nem & lt);
      float *q = sq + j * Q::N;
      const int mix = __float_as_int(r[R_MIX]), miy = __float_as_int(r[R_MIY]);
      // same FP32 operations as the forward: d = (pixel offset in the tile)
      // + ((tile origin - floor(mean)) - frac(mean))
      q[0] = (float)(X0 - mix) - r[R_MFX];
      q[1] = (float)(Y0 - miy) - r[R_MFY];
      q[2] = r[R_A]; q[3] = r[R_B]; q[4] = r[R_C];
#pragma unroll
      for (int k = 0; k < 2 * C; ++k) q[Q::AMP + k] = r[R_AMP + k];
      q[Q::BOX] = __int_as_float(xa | (xb << 8) | (ya << 16) | (yb << 24));
      q[Q::START] = __int_as_float(start);
      q[Q::SLOT] = __uint_as_float(slot);
      if (PA) {
        const float2 l = alim[vals[base + lane]];
        q[Q::LO] = l.x;
        q[Q::HI] = l.y;
      }
    }
    wave_sync();
    if (total > 0) {
      // ---- walk: this lane owns segments [s0, s1) of the concatenated boxes
      const int chunk = (total + 63) / 64;
      const int s0 = min(total, lane * chunk), s1 = min(total, s0 + chunk);
      // first pair whose segments contain s0: the last j with start_j <= s0
      int j = 0;
      for (int step = 32; step > 0; step >>= 1) {
        const int t = j + step;
        if (t < np && __float_as_int(sq[t * Q::N + Q::START]) <= s0) j = t;
      }
      float offx, offy, qa, qb, qc, amp[2 * C], plo = 0.f, phi = 0.f;
      // the walk's pixel: tile-local column and row as exact FP32 integers, the
      // LDS byte offset of its dL/dU0, and the box's first and last column
      float fx, fy, fxa, fxb;
      uint32_t la, lwrap;  // lwrap: the offset step from a box row's end to the next row
      int bxa, bxb, bya, sj, left, span = 0;
      auto set_pixel = [&](int x, int y) {
        fx = (float)x;
        fy = (float)y;
        la = (uint32_t)(y * RS2 + x * C) * (uint32_t)sizeof(float2);
      };
      auto load_pair = [&](int jj) {
        const float *q = sq + jj * Q::N;
        offx = q[0]; offy = q[1];
        qa = q[2]; qb = q[3]; qc = q[4];
        if (PA) { plo = q[Q::LO]; phi = q[Q::HI]; }
#pragma unroll
        for (int k = 0; k < 2 * C; ++k) amp[k] = q[Q::AMP + k];
        const int bx = __float_as_int(q[Q::BOX]);
        bxa = bx & 0xff; bxb = (bx >> 8) & 0xff;
        bya = (bx >> 16) & 0xff;
        const int byb = (bx >> 24) & 0xff;
        sj = __float_as_int(q[Q::START]);
        left = ((bxb - bxa + 1) * (byb - bya + 1) + kAdjSeg - 1) / kAdjSeg;
        fxa = (float)bxa;
        fxb = (float)bxb;
        lwrap = (uint32_t)(RS2 - (bxb - bxa) * C) * (uint32_t)sizeof(float2);
        set_pixel(bxa, bya);
      };
      auto flush_global = [&](int jj, const float *v) {
        const uint32_t sl = __float_as_uint(sq[jj * Q::N + Q::SLOT]);
        if (sl != 0xffffffffu) {
          float4 *dst = reinterpret_cast<float4 *>(partials + (size_t)sl * PS);
          float o[PS];
#pragma unroll
          for (int k = 0; k < PS; ++k) o[k] = k < NS ? v[k] : 0.f;
#pragma unroll
          for (int k = 0; k < PS / 4; ++k)
            dst[k] = make_float4(o[4 * k], o[4 * k + 1], o[4 * k + 2], o[4 * k + 3]);
        }
      };
      float S[NS], F[NS];  // running sums; F: the first part when it began before s0
#pragma unroll
      for (int k = 0; k < NS; ++k) { S[k] = 0.f; F[k] = 0.f; }
      if (s0 < s1) {
        load_pair(j);
        bool head = sj < s0;
        {
          const int skip = s0 - sj, o = skip * kAdjSeg, wb = bxb - bxa + 1;
          const int oy = o / wb;
          set_pixel(bxa + (o - oy * wb), bya + oy);
          left -= skip;
        }
        for (int s = s0; s < s1; ++s) {
          if (left == 0) {
            // the previous pair ended with the previous segment
            if (head) {
#pragma unroll
              for (int k = 0; k < NS; ++k) F[k] = S[k];
            } else {
              flush_global(j, S);
            }
#pragma unroll
            for (int k = 0; k < NS; ++k) S[k] = 0.f;
            head = false;
            load_pair(++j);
          }
#pragma unroll
          for (int u = 0; u < kAdjSeg; ++u) {
            // The last segment of a pair is padded: its padding pixels run on
            // along the box rows, below the box (outside the support, so G = 0)
            // or below the tile (every offset from the zero row on reads the
            // zero row, so every term is 0).
            const float dy = fy + offy, dx = fx + offx;
            const float p2 = fmaf(dx, fmaf(qa, dx, qb * dy), qc * dy * dy);
            float G;
            if (PA)
              G = p2 >= plo ? __builtin_amdgcn_exp2f(fminf(p2, phi)) : 0.f;
            else
              G = p2 >= thr ? __builtin_amdgcn_exp2f(CLAMP ? fmaxf(p2, kPowerFloor2) : p2)
                            : 0.f;
            const float2 *gv = reinterpret_cast<const float2 *>(
                reinterpret_cast<const char *>(sg) +
                min(la, (uint32_t)(TH * RS2 * sizeof(float2))));
            float gp = 0.f;
#pragma unroll
            for (int c = 0; c < C; ++c) {
              const float2 v = gv[c];
              gp = fmaf(v.x, amp[2 * c], fmaf(v.y, amp[2 * c + 1], gp));
              S[2 * c] = fmaf(G, v.x, S[2 * c]);
              S[2 * c + 1] = fmaf(G, v.y, S[2 * c + 1]);
            }
            // without the clamp, G > 0 implies p2 >= thr > the clamp; with PA the
            // weight is constant (0.99) where p2 > hi, so only alpha's sum sees it
            float w;
            if constexpr (PA) {
              const bool clamped = p2 > phi;
              w = clamped ? 0.f : gp * G;
              S[2 * C + 5] += clamped ? gp * G : 0.f;
            } else {
              w = (!CLAMP || p2 > kPowerFloor2) ? gp * G : 0.f;
            }
            const float wx = w * dx, wy = w * dy;
            S[2 * C] += wx;
            S[2 * C + 1] += wy;
            S[2 * C + 2] = fmaf(wx, dx, S[2 * C + 2]);
            S[2 * C + 3] = fmaf(wx, dy, S[2 * C + 3]);
            S[2 * C + 4] = fmaf(wy, dy, S[2 * C + 4]);
            const float fx1 = fx + 1.f;
            const bool wrap = fx1 > fxb;
            fx = wrap ? fxa : fx1;
            fy = wrap ? fy + 1.f : fy;
            la += wrap ? lwrap : (uint32_t)(C * sizeof(float2));
          }
          --left;
        }
        if (left == 0) {  // the piece ends exactly where the pair ends
          if (head) {
#pragma unroll
            for (int k = 0; k < NS; ++k) F[k] = S[k];
          } else {
            flush_global(j, S);
          }
        } else if (head) {  // a pair that covers this whole piece
#pragma unroll
          for (int k = 0; k < NS; ++k) F[k] = S[k];
        } else {
          // this lane started the pair and finishes it: it reaches the lanes
          // lane+1 .. (last segment of the pair) / chunk
          span = (s1 + left - 1) / chunk - lane;
        }
      }
      // ---- pairs cut by piece boundaries: add the parts in lane order ------
      for (int d = 1; __any(d <= span); ++d) {
        const int src = min(63, lane + d);
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const float v = __shfl(F[k], src);
          if (d <= span) S[k] += v;
        }
      }
      if (span > 0) flush_global(j, S);
    }
    wave_sync();
  }
}

// ----------------------------------------------------------------------------
// Adjoint, Gaussian stage (FP64): sum the pair partials of each Gaussian in a
// fixed order, then chain rule through the preprocess (supplementary Backward
// Pass items 1-7):
//   dL/dc_c   = alpha (cos phi dP_c + sin phi dQ_c)
//   dL/dphi_c = alpha c (-sin phi dP_c + cos phi dQ_c)
//   dL/dalpha = sum_c c (cos phi dP_c + sin phi dQ_c) (minus, with CGH_PAPER_ALPHA, the
//               part of the pixels where the 0.99 clamp is active);
//               dalpha/dalpha~ = alpha (1 - alpha)
//   dL/dmean  = Sigma^{-1} (sum w d);  dmean/dx~ = [W, H]/2 (1 - tanh^2 x~)
//   dL/dSigma^{-1} entries (inv00, inv01 stored once, inv11) = -(1/2, 1, 1/2) sum w d d
//   dL/dSigma = -Sigma^{-1} G Sigma^{-1} (G the symmetric gradient matrix), off-
//   diagonal counted twice for the single stored Sigma01; clamped determinant:
//   inv = adj(Sigma) / eps_d
//   Sigma -> (s_x, s_y, theta) and s = exp(s~) + eps_s.
// ----------------------------------------------------------------------------
// the 2C + 5 partial sums of a pair, plus the clamped-pixel sum with CGH_PAPER_ALPHA
template <int C, bool PA>
constexpr int kPairSums = 2 * C + 5 + (PA ? 1 : 0);
constexpr int kPairChunk = 512;  // pairs per LDS chunk of the per-Gaussian reduction

// FP64 sums of the pair partials of Gaussian g0 + threadIdx.x, for the 256
// Gaussians g0 .. g0 + 255 of a workgroup (all threads must call it).  A
// Gaussian's pairs own the slots offset .. offset + count - 1 and the offsets
// are the scan of the counts, so the workgroup's pairs are one contiguous run
// of slots: it is read into LDS kPairChunk pairs at a time with every thread
// on consecutive 16-byte words, and each thread adds its own pairs from LDS in
// slot order (the same order, so the same sums, as reading them one by one).
template <int C, bool PA>
__device__ __forceinline__ void pair_sums_block(int g0, int total,
                                                const uint32_t *__restrict__ counts,
                                                const uint32_t *__restrict__ offsets, int64_t cap,
                                                const float *__restrict__ partials,
                                                float4 *__restrict__ chunk4,
                                                double (&S)[kPairSums<C, PA>]) {
  constexpr int PS = part_stride_c(C), NP = kPairSums<C, PA>;
  static_assert(NP <= PS, "spare partial slot");
  constexpr int NF4 = kPairChunk * PS / 4, KF = NF4 / 256;
  static_assert(NF4 % 256 == 0, "chunk of whole float4 rounds");
  const int tid = threadIdx.x, gg = g0 + tid;
  const int last = min(total, g0 + 256) - 1;
#pragma unroll
  for (int k = 0; k < NP; ++k) S[k] = 0.0;
  uint64_t off = 0, end = 0;
  if (gg < total) {
    off = offsets[gg];
    end = min(off + counts[gg], (uint64_t)cap);
  }
  const uint64_t run0 = offsets[g0];
  const uint64_t run1 = min((uint64_t)offsets[last] + counts[last], (uint64_t)cap);
  const float4 *src4 = reinterpret_cast<const float4 *>(partials);
  for (uint64_t c0 = run0; c0 < run1; c0 += kPairChunk) {
    const uint64_t c1 = min(c0 + kPairChunk, run1);
    const int nf4 = (int)(c1 - c0) * (PS / 4);
    float4 v[KF];
#pragma unroll
    for (int k = 0; k < KF; ++k) {
      const int i = tid + 256 * k;
      v[k] = i < nf4 ? src4[c0 * (PS / 4) + i] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();  // every thread is done with the previous chunk
#pragma unroll
    for (int k = 0; k < KF; ++k) chunk4[tid + 256 * k] = v[k];
    __syncthreads();
    const uint64_t p1 = min(end, c1);
    for (uint64_t p = max(off, c0); p < p1; ++p) {
      const float *r = reinterpret_cast<const float *>(chunk4) + (p - c0) * PS;
#pragma unroll
      for (int k = 0; k < NP; ++k) S[k] += (double)r[k];
    }
  }
}

// The 6 + 2C gradients of Gaussian gg (of all B n) in the order mean (2),
// log-scale (2), rotation, amplitude (C), phase (C), opacity, from the sums of
// its pair partials and its parameters.
template <int C, bool PA>
__device__ __forceinline__ void gaussian_grads(const float *params_all, int n, int W, int H, int gg,
                                               const double (&S)[kPairSums<C, PA>],
                                               float (&gv)[6 + 2 * C]) {
  // partial slots are indexed by the Gaussian's index among all B n; its
  // parameters by its index g in its hologram's block
  const GaussIdx gi = gauss_idx<C>(gg, n);
  const float *params = params_all + gi.base;
  const int g = gi.gl;
  const Geom q = geometry(params, n, C, g, W, H);
  const float *amp = params + 5 * (size_t)n;
  const float *ph = params + (size_t)(5 + C) * n;
  // the 6 + 2C gradients of this Gaussian: mean (2), log-scale (2), rotation,
  // amplitude (C), phase (C), opacity; the sums above are FP64, the chain rule
  // FP32
  float gm[2], gs[2], gr, ga[C], gph[C], go;
  float dalpha = 0.f;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    float sn, cs;
    sincosf(ph[(size_t)g * C + c], &sn, &cs);
    const float cc = amp[(size_t)g * C + c];
    const float dP = (float)S[2 * c], dQ = (float)S[2 * c + 1];
    const float proj = cs * dP + sn * dQ;
    ga[c] = q.alpha * proj;
    gph[c] = q.alpha * cc * (-sn * dP + cs * dQ);
    dalpha += cc * proj;
  }
  // pixels where the Alg. 2 clamp is active contribute 0.99 c e^{j phi}, which
  // does not depend on alpha: their part of the amplitude sums comes off here
  if constexpr (PA) dalpha -= (float)S[2 * C + 5] / q.alpha;
  go = dalpha * q.alpha * (1.0f - q.alpha);
  const float W1 = (float)S[2 * C], W2 = (float)S[2 * C + 1], W3 = (float)S[2 * C + 2],
              W4 = (float)S[2 * C + 3], W5 = (float)S[2 * C + 4];
  const float dmx = q.i00 * W1 + q.i01 * W2;
  const float dmy = q.i01 * W1 + q.i11 * W2;
  // d tanh(x) / dx = 1 - tanh^2 x = 4 / (e^x + e^-x)^2, without the cancellation
  auto sech2 = [](float x) {
    const float e = expf(-fabsf(x)), d = 1.0f + e * e;
    return 4.0f * e * e / (d * d);
  };
  gm[0] = dmx * 0.5f * (float)W * sech2(params[2 * g]);
  gm[1] = dmy * 0.5f * (float)H * sech2(params[2 * g + 1]);
  // gradient w.r.t. the stored inverse entries
  const float g00 = -0.5f * W3, g01 = -W4, g11 = -0.5f * W5;
  // dL/dSigma = -M Gm M with M = Sigma^{-1} and the symmetric gradient matrix
  // Gm = [[g00, g01/2], [g01/2, g11]] (the stored off-diagonal counted twice)
  const float h01 = 0.5f * g01;
  const float t00 = q.i00 * g00 + q.i01 * h01, t01 = q.i00 * h01 + q.i01 * g11;
  const float t10 = q.i01 * g00 + q.i11 * h01, t11 = q.i01 * h01 + q.i11 * g11;
  const float d00 = -(t00 * q.i00 + t01 * q.i01);
  const float d11 = -(t10 * q.i01 + t11 * q.i11);
  const float d01 = -2.0f * (t00 * q.i01 + t01 * q.i11);
  const float c = q.ct, s = q.st, sx = q.sx, sy = q.sy;
  const float dsx = 2.0f * sx * (c * c * d00 + c * s * d01 + s * s * d11);
  const float dsy = 2.0f * sy * (s * s * d00 - c * s * d01 + c * c * d11);
  const float dth = 2.0f * (sy * sy - sx * sx) * c * s * d00 +
                    (sx * sx - sy * sy) * (c * c - s * s) * d01 +
                    2.0f * (sx * sx - sy * sy) * c * s * d11;
  gs[0] = dsx * (sx - 0.1f);      // d s / d s~ = exp(s~)
  gs[1] = dsy * (sy - 0.1f);
  gr = dth;
  gv[0] = gm[0]; gv[1] = gm[1]; gv[2] = gs[0]; gv[3] = gs[1]; gv[4] = gr;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    gv[5 + c] = ga[c];
    gv[5 + C + c] = gph[c];
  }
  gv[5 + 2 * C] = go;
}

// offset of parameter k (in the order of gaussian_grads) of Gaussian g in its
// hologram's block
template <int C>
__device__ __forceinline__ size_t param_offset(int k, int g, int n) {
  if (k < 2) return 2 * (size_t)g + k;
  if (k < 4) return 2 * (size_t)n + 2 * (size_t)g + (k - 2);
  if (k == 4) return 4 * (size_t)n + g;
  if (k < 5 + C) return 5 * (size_t)n + (size_t)g * C + (k - 5);
  if (k < 5 + 2 * C) return (size_t)(5 + C) * n + (size_t)g * C + (k - 5 - C);
  return (size_t)(5 + 2 * C) * n + g;
}

// the 6 + 2C parameters of Gaussian gg, as the parameter block of a single
// Gaussian (n = 1), so that they can be loaded before they are needed
template <int C>
__device__ __forceinline__ void load_one_gaussian(const float *params_all, int n, int gg,
                                                  float (&lp)[6 + 2 * C]) {
  const GaussIdx gi = gauss_idx<C>(gg, n);
#pragma unroll
  for (int k = 0; k < 6 + 2 * C; ++k) lp[k] = params_all[gi.base + param_offset<C>(k, gi.gl, n)];
}

template <int C, bool PA>
__global__ __launch_bounds__(256) void k_preprocess_adj(
    const float *__restrict__ params_all, int n, int total, int W, int H,
    const uint32_t *__restrict__ counts, const uint32_t *__restrict__ offsets, int64_t cap,
    const float *__restrict__ partials, float *__restrict__ grads_all,
    uint32_t *__restrict__ finite_flag) {
  __shared__ float4 chunk4[kPairChunk * part_stride_c(C) / 4];
  const int g0 = blockIdx.x * 256, gg = g0 + threadIdx.x;
  float lp[6 + 2 * C];
  if (gg < total) load_one_gaussian<C>(params_all, n, gg, lp);
  double S[kPairSums<C, PA>];
  pair_sums_block<C, PA>(g0, total, counts, offsets, cap, partials, chunk4, S);
  if (gg >= total) return;
  float gv[6 + 2 * C];
  gaussian_grads<C, PA>(lp, 1, W, H, 0, S, gv);
  const GaussIdx gi = gauss_idx<C>(gg, n);
  bool finite = true;
#pragma unroll
  for (int k = 0; k < 6 + 2 * C; ++k) {
    finite = finite && isfinite(gv[k]);
    grads_all[gi.base + param_offset<C>(k, gi.gl, n)] = gv[k];
  }
  if (finite_flag && !finite) atomicOr(finite_flag, kNonFiniteGrads);
}

// The same, followed by one Adam update of the workgroup's parameters
// (cgh_backward_step).  The 256 Gaussians of a workgroup own, in each of the six
// parameter blocks, one contiguous run (two where the workgroup straddles two
// holograms); their gradients go through LDS so that the update then walks
// those runs with consecutive threads on consecutive parameters.  grads_all
// may be null.
template <int C, bool PA>
__global__ __launch_bounds__(256) void k_preprocess_adj_adam(
    float *params_all, int n, int total, int W, int H,
    const uint32_t *__restrict__ counts, const uint32_t *__restrict__ offsets, int64_t cap,
    const float *__restrict__ partials, float *__restrict__ grads_all,
    uint32_t *__restrict__ finite_flag, AdamFuse adam) {
  constexpr int NPAR = 6 + 2 * C;
  __shared__ float sgv[NPAR][256];
  __shared__ float4 chunk4[kPairChunk * part_stride_c(C) / 4];
  const int tid = threadIdx.x;
  const int g0 = blockIdx.x * 256;
  const int gg = g0 + tid;
  float lp[NPAR];
  if (gg < total) load_one_gaussian<C>(params_all, n, gg, lp);
  double S[kPairSums<C, PA>];
  pair_sums_block<C, PA>(g0, total, counts, offsets, cap, partials, chunk4, S);
  const int cnt = min(256, total - g0);
  // element e of the workgroup's share of parameter block a (per-Gaussian
  // width w_a: 2, 2, 1, C, C, 1) is component e % w_a of Gaussian e / w_a;
  // with cnt <= 256 a thread takes elements tid + 256 r, r < w_a, of block a:
  // NPAR in all, whose parameters and moments are all loaded before the chain
  // rule, which hides their latency
  constexpr int wid[6] = {2, 2, 1, C, C, 1};
  size_t off[NPAR];
  float pk[NPAR], mk[NPAR], vk[NPAR], gk[NPAR];
  bool ok[NPAR];
  {
    int kbase = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      const int w = wid[a];
#pragma unroll
      for (int r = 0; r < w; ++r) {
        const int sl = kbase + r, e = tid + 256 * r;
        ok[sl] = e < cnt * w;
        off[sl] = 0;
        pk[sl] = mk[sl] = vk[sl] = 0.f;
        if (ok[sl]) {
          const int j = e / w, comp = e - j * w;
          const GaussIdx gi = gauss_idx<C>(g0 + j, n);
          off[sl] = gi.base + param_offset<C>(kbase + comp, gi.gl, n);
          pk[sl] = params_all[off[sl]];
          mk[sl] = adam.m[off[sl]];
          vk[sl] = adam.v[off[sl]];
        }
      }
      kbase += w;
    }
  }
  if (gg < total) {
    float gv[NPAR];
    gaussian_grads<C, PA>(lp, 1, W, H, 0, S, gv);
    bool finite = true;
#pragma unroll
    for (int k = 0; k < NPAR; ++k) {
      finite = finite && isfinite(gv[k]);
      sgv[k][tid] = gv[k];
    }
    if (finite_flag && !finite) atomicOr(finite_flag, kNonFiniteGrads);
  }
  __syncthreads();  // every thread reaches it: no early return above
  {
    int kbase = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      const int w = wid[a];
#pragma unroll
      for (int r = 0; r < w; ++r) {
        const int sl = kbase + r, e = tid + 256 * r;
        const int j = e / w, comp = e - j * w;
        gk[sl] = ok[sl] ? sgv[kbase + comp][j] : 0.f;
      }
      kbase += w;
    }
  }
#pragma unroll
  for (int sl = 0; sl < NPAR; ++sl) {
    if (ok[sl]) {
      adam_one(pk[sl], gk[sl], mk[sl], vk[sl], adam.lr_scaled, adam.b1, adam.b2, adam.eps,
               adam.inv_sqrt_bc2);
      params_all[off[sl]] = pk[sl];
      adam.m[off[sl]] = mk[sl];
      adam.v[off[sl]] = vk[sl];
      if (grads_all) grads_all[off[sl]] = gk[sl];
    }
  }
}

hipError_t launch_raster_adjoint(const Ctx &c, const float2 *grad_field, hipStream_t s) {
  const float thr = support_threshold(c.cfg.support_sigma);
  const uint32_t *vals = c.vals[c.sorted];
  const bool clamp = !(thr > kPowerFloor2);
  const bool pa = c.alim != nullptr;
  with_tile(c, [&](auto tw, auto th) {
    constexpr int TW = decltype(tw)::value, TH = decltype(th)::value;
    with_channels(c.C, [&](auto cc) {
      constexpr int CC = decltype(cc)::value;
      auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(c.num_tiles), dim3(64 * kAdjWaves), 0, s, c.rec, vals, c.ranges,
                           c.rect, c.offsets, c.W, c.H, c.tiles_x, c.tiles_per, thr, c.alim,
                           grad_field, c.pair_cap, c.partials);
      };
      if (pa) go(k_raster_adj<CC, false, true, TW, TH>);
      else if (clamp) go(k_raster_adj<CC, true, false, TW, TH>);
      else go(k_raster_adj<CC, false, false, TW, TH>);
    });
  });
  return hipGetLastError();
}

hipError_t launch_preprocess_adjoint(const Ctx &c, const float *params, int n, float *grads,
                                     hipStream_t s, const AdamFuse *adam) {
  const int total = (int)total_gaussians(c, n);
  if (total <= 0) return hipSuccess;
  dim3 g2((total + 255) / 256), block(256);
  const bool pa = c.alim != nullptr;
  with_channels(c.C, [&](auto cc) {
    constexpr int CC = decltype(cc)::value;
    if (adam) {
      auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, g2, block, 0, s, adam->p, n, total, c.W, c.H, c.counts,
                           c.offsets, c.pair_cap, c.partials, grads, c.finite_flag, *adam);
      };
      if (pa) go(k_preprocess_adj_adam<CC, true>);
      else go(k_preprocess_adj_adam<CC, false>);
    } else {
      auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, g2, block, 0, s, params, n, total, c.W, c.H, c.counts,
                           c.offsets, c.pair_cap, c.partials, grads, c.finite_flag);
      };
      if (pa) go(k_preprocess_adj<CC, true>);
      else go(k_preprocess_adj<CC, false>);
    }
  });
  return hipGetLastError();
}

}  // namespace cgh
