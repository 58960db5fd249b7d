// SSIM term of the paper's final training loss (Sec. 3.2: L = L_recon +
// lambda_1 L_SSIM) and its adjoint, over the [L][C] intensity images.
//
// SSIM (Wang, Bovik, Sheikh and Simoncelli 2004) at window position p (the
// 11 x 11 window with top-left pixel p, fully inside the image) from the
// window-weighted sums mu_x = sum w x, e_xx = sum w x^2, e_xy = sum w x y (and
// the same for y): sigma_x^2 = e_xx - mu_x^2, sigma_xy = e_xy - mu_x mu_y,
//   S = (2 mu_x mu_y + C1)(2 sigma_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)).
// The window is separable, w_ij = w_i w_j (Gaussian, standard deviation 1.5).
// S depends on x(q) only through those sums, so
//   dS(p)/dx(q) = w_(q-p) [A(p) + 2 x(q) B(p) + y(q) Cc(p)]
// with B = dS/dsigma_x^2, Cc = dS/dsigma_xy and A = dS/dmu_x (at fixed
// sigmas) - 2 mu_x B - mu_y Cc.  k_ssim_fwd filters the moments of a tile of
// positions and writes A, B, Cc and the tile's sum of S; k_ssim_bwd filters
// A, B, Cc back onto a tile of pixels (the same weights: the window is
// symmetric), adds the elementwise L_recon gradient, and writes
// g = 2 (dL/dI) u, the row-pass input of the adjoint.
#include <algorithm>
#include <cmath>

#include "cgh_internal.h"

namespace cgh {

constexpr int kSsimWin = 11;
constexpr int kTX = 32, kTY = 64;          // positions (or pixels) per tile: columns, rows
constexpr int kSX = kTX + kSsimWin - 1;    // 42 staged columns
constexpr int kSY = kTY + kSsimWin - 1;    // 74 staged rows
constexpr int kLd = 44;                    // staged row stride: four float4 reads per group
constexpr int kHG = 4;                     // horizontal outputs per thread (one float4)
constexpr int kVR = 8;                     // vertical outputs per thread
constexpr int kHItems = kSY * (kTX / kHG); // 592 horizontal work items
constexpr int kStage = (kSY * kLd + 255) / 256;  // staged values per thread
constexpr float kSsimC1 = 0.01f * 0.01f, kSsimC2 = 0.03f * 0.03f;
static_assert(kTX / kHG * kHG == kTX && 4 * 4 <= kLd && kHG * (kTX / kHG - 1) + 16 <= kLd,
              "a group reads 16 staged columns from 4 g");
static_assert((kTX * kTY) / kVR == 256, "one vertical item per thread");

struct SsimWin {
  float w[kSsimWin];
};

static SsimWin ssim_window() {
  SsimWin r;
  double s = 0.0, v[kSsimWin];
  for (int i = 0; i < kSsimWin; ++i) {
    const double d = i - kSsimWin / 2;
    v[i] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    s += v[i];
  }
  for (int i = 0; i < kSsimWin; ++i) r.w[i] = (float)(v[i] / s);
  return r;
}

static int tiles_x(int n) { return (n + kTX - 1) / kTX; }
static int tiles_y(int n) { return (n + kTY - 1) / kTY; }
int ssim_pos_tiles(const Ctx &c) {
  return tiles_x(c.W - kSsimWin + 1) * tiles_y(c.H - kSsimWin + 1);
}
int ssim_pix_tiles(const Ctx &c) { return tiles_x(c.W) * tiles_y(c.H); }

// fixed-order FP64 sum over a 256-thread block; the result is valid in every thread
__device__ double block_sum_f64(double v, double *red) {
  for (int d = 32; d > 0; d >>= 1) v += __shfl_down(v, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// 16 consecutive staged values from column 4 g of row r (four 16-byte reads;
// the 8 lanes of one LDS cycle read 128 contiguous bytes)
__device__ inline void read16(const float (*plane)[kLd], int r, int g, float *v) {
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const float4 q = *reinterpret_cast<const float4 *>(&plane[r][kHG * g + 4 * m]);
    v[4 * m] = q.x;
    v[4 * m + 1] = q.y;
    v[4 * m + 2] = q.z;
    v[4 * m + 3] = q.w;
  }
}

// Tile t of a [images][tiles_y][tiles_x] grid; every block walks tiles t, t + G, ...
// (G blocks) and prefetches the next tile's staged span into registers while it
// filters the current one.
struct TileGrid {
  int nx, ny, total;
  __device__ void at(int t, int &img, int &bx, int &by) const {
    img = t / (nx * ny);
    const int rem = t - img * nx * ny;
    by = rem / nx;
    bx = rem - by * nx;
  }
};

// horizontal window sums of x, y, x^2, y^2, x y over the staged span, 4
// consecutive outputs per item, into hm[5][74][32]
__device__ inline void ssim_fwd_rows(const float (*sx)[kLd], const float (*sy)[kLd],
                                     float (*hm)[kSY][kTX], const SsimWin &wt, int tid) {
  for (int it = tid; it < kHItems; it += 256) {
    const int r = it / (kTX / kHG), g = it - r * (kTX / kHG);
    float x[16], y[16];
    read16(sx, r, g, x);
    read16(sy, r, g, y);
    float m[5][kHG];
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
      for (int o = 0; o < kHG; ++o) m[q][o] = 0.f;
#pragma unroll
    for (int j = 0; j < kHG + kSsimWin - 1; ++j) {
      const float xx = x[j] * x[j], yy = y[j] * y[j], xy = x[j] * y[j];
#pragma unroll
      for (int o = 0; o < kHG; ++o) {
        const int k = j - o;
        if (k < 0 || k >= kSsimWin) continue;
        const float w = wt.w[k];
        m[0][o] = fmaf(w, x[j], m[0][o]);
        m[1][o] = fmaf(w, y[j], m[1][o]);
        m[2][o] = fmaf(w, xx, m[2][o]);
        m[3][o] = fmaf(w, yy, m[3][o]);
        m[4][o] = fmaf(w, xy, m[4][o]);
      }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q)
      *reinterpret_cast<float4 *>(&hm[q][r][kHG * g]) =
          make_float4(m[q][0], m[q][1], m[q][2], m[q][3]);
  }
}

// G blocks of 256 threads over the position tiles of all L C images
__global__ __launch_bounds__(256) void k_ssim_fwd(const float *__restrict__ I,
                                                  const float *__restrict__ T, int H, int W,
                                                  TileGrid tg, SsimWin wt,
                                                  float *__restrict__ abc, size_t abc_plane,
                                                  double *__restrict__ part) {
  __shared__ __align__(16) float sx[kSY][kLd];
  __shared__ __align__(16) float sy[kSY][kLd];
  __shared__ __align__(16) float hm[5][kSY][kTX];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int Hv = H - kSsimWin + 1, Wv = W - kSsimWin + 1;
  float vx[kStage], vy[kStage];
  // the span [py0, py0 + 74) x [px0, px0 + 44) of tile t, zero outside the image
  auto fetch = [&](int t) {
    int img, bx, by;
    tg.at(t, img, bx, by);
    const float *Ii = I + (size_t)img * H * W, *Ti = T + (size_t)img * H * W;
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int i = min(tid + 256 * k, kSY * kLd - 1), r = i / kLd, c = i - r * kLd;
      const int y = by * kTY + r, x = bx * kTX + c;
      const size_t o = (size_t)min(y, H - 1) * W + min(x, W - 1);
      const bool in = y < H && x < W;
      vx[k] = in ? Ii[o] : 0.f;
      vy[k] = in ? Ti[o] : 0.f;
    }
  };
  int t = blockIdx.x;
  if (t < tg.total) fetch(t);
  for (; t < tg.total; t += gridDim.x) {
    // sx, sy were last read before the previous tile's second barrier; hm is
    // written only after the barrier below, when every thread has left the
    // previous tile's vertical pass
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int i = tid + 256 * k, r = i / kLd, c = i - r * kLd;
      if (i < kSY * kLd) {
        sx[r][c] = vx[k];
        sy[r][c] = vy[k];
      }
    }
    __syncthreads();
    if (t + (int)gridDim.x < tg.total) fetch(t + gridDim.x);
    ssim_fwd_rows(sx, sy, hm, wt, tid);
    __syncthreads();
    // vertical sums: column c, rows r0 .. r0 + 7 of the tile
    int img, bx, by;
    tg.at(t, img, bx, by);
    const int c = tid % kTX, r0 = kVR * (tid / kTX);
    float acc[5][kVR];
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
      for (int o = 0; o < kVR; ++o) acc[q][o] = 0.f;
#pragma unroll
    for (int j = 0; j < kVR + kSsimWin - 1; ++j) {
      float v[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) v[q] = hm[q][r0 + j][c];
#pragma unroll
      for (int o = 0; o < kVR; ++o) {
        const int k = j - o;
        if (k < 0 || k >= kSsimWin) continue;
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[q][o] = fmaf(wt.w[k], v[q], acc[q][o]);
      }
    }
    double sum = 0.0;
    const int px = bx * kTX + c;
#pragma unroll
    for (int o = 0; o < kVR; ++o) {
      const int py = by * kTY + r0 + o;
      if (py >= Hv || px >= Wv) continue;
      const float mx = acc[0][o], my = acc[1][o];
      const float sxx = acc[2][o] - mx * mx, syy = acc[3][o] - my * my;
      const float sxy = acc[4][o] - mx * my;
      const float n1 = 2.f * mx * my + kSsimC1, n2 = 2.f * sxy + kSsimC2;
      // d1 >= C1 and d2 >= C2 (up to rounding of the variances): no zero divisors
      const float i1 = __builtin_amdgcn_rcpf(mx * mx + my * my + kSsimC1);
      const float i2 = __builtin_amdgcn_rcpf(sxx + syy + kSsimC2);
      const float inv = i1 * i2;
      const float S = n1 * n2 * inv;
      const float B = -S * i2, Cc = 2.f * n1 * inv;
      const float dmx = 2.f * my * n2 * inv - 2.f * mx * S * i1;  // dS/dmu_x at fixed sigmas
      const size_t at = ((size_t)img * Hv + py) * Wv + px;
      abc[at] = dmx - 2.f * mx * B - my * Cc;
      abc[abc_plane + at] = B;
      abc[2 * abc_plane + at] = Cc;
      sum += (double)S;
    }
    // red is rewritten only after two more barriers
    const double s = block_sum_f64(sum, red);
    if (tid == 0) part[t] = s;
  }
}

// G blocks of 256 threads over the pixel tiles of all L C images.  coef =
// -ssim_weight / (number of positions over all images); inv_n = 1 / (L C H W).
__global__ __launch_bounds__(256) void k_ssim_bwd(
    const float *__restrict__ I, const float *__restrict__ T, const float *__restrict__ mask,
    const float *__restrict__ abc, size_t abc_plane, float2 *__restrict__ u, int H, int W,
    int C, TileGrid tg, SsimWin wt, float coef, float inv_n, double *__restrict__ part) {
  __shared__ __align__(16) float sa[3][kSY][kLd];
  __shared__ __align__(16) float hm[3][kSY][kTX];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int Hv = H - kSsimWin + 1, Wv = W - kSsimWin + 1;
  float va[3][kStage];
  // coefficients at positions [qy0 - 10, qy0 + 64) x [qx0 - 10, qx0 + 34), zero
  // outside the valid positions
  auto fetch = [&](int t) {
    int img, bx, by;
    tg.at(t, img, bx, by);
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int i = min(tid + 256 * k, kSY * kLd - 1), r = i / kLd, cc = i - r * kLd;
      const int py = by * kTY - (kSsimWin - 1) + r, px = bx * kTX - (kSsimWin - 1) + cc;
      const bool in = py >= 0 && py < Hv && px >= 0 && px < Wv;
      const size_t o =
          ((size_t)img * Hv + min(max(py, 0), Hv - 1)) * Wv + min(max(px, 0), Wv - 1);
#pragma unroll
      for (int q = 0; q < 3; ++q) va[q][k] = in ? abc[q * abc_plane + o] : 0.f;
    }
  };
  int t = blockIdx.x;
  if (t < tg.total) fetch(t);
  for (; t < tg.total; t += gridDim.x) {
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int i = tid + 256 * k, r = i / kLd, cc = i - r * kLd;
      if (i < kSY * kLd)
#pragma unroll
        for (int q = 0; q < 3; ++q) sa[q][r][cc] = va[q][k];
    }
    __syncthreads();
    if (t + (int)gridDim.x < tg.total) fetch(t + gridDim.x);
    int img, bx, by;
    tg.at(t, img, bx, by);
    const int c = tid % kTX, r0 = kVR * (tid / kTX);
    // per-pixel inputs of this thread, fetched before the filters so that their
    // latency overlaps them
    const float *Ii = I + (size_t)img * H * W, *Ti = T + (size_t)img * H * W;
    const float *Mi = mask ? mask + (size_t)(img / C) * H * W : nullptr;
    float2 *ui = u + (size_t)img * H * W;
    const int x = bx * kTX + c;
    float pi[kVR], pt[kVR], pm[kVR];
    float2 pu[kVR];
#pragma unroll
    for (int o = 0; o < kVR; ++o) {
      const size_t at = (size_t)min(by * kTY + r0 + o, H - 1) * W + min(x, W - 1);
      pi[o] = Ii[at];
      pt[o] = Ti[at];
      pm[o] = Mi ? Mi[at] : 0.f;
      pu[o] = ui[at];
    }
    // pixel x gathers positions x - 10 .. x with weights w[10 - j] = w[j]
    for (int it = tid; it < kHItems; it += 256) {
      const int r = it / (kTX / kHG), g = it - r * (kTX / kHG);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        float a[16];
        read16(sa[q], r, g, a);
        float m[kHG] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < kHG + kSsimWin - 1; ++j)
#pragma unroll
          for (int o = 0; o < kHG; ++o) {
            const int k = j - o;
            if (k >= 0 && k < kSsimWin) m[o] = fmaf(wt.w[k], a[j], m[o]);
          }
        *reinterpret_cast<float4 *>(&hm[q][r][kHG * g]) = make_float4(m[0], m[1], m[2], m[3]);
      }
    }
    __syncthreads();
    float acc[3][kVR];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int o = 0; o < kVR; ++o) acc[q][o] = 0.f;
#pragma unroll
    for (int j = 0; j < kVR + kSsimWin - 1; ++j) {
      float v[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) v[q] = hm[q][r0 + j][c];
#pragma unroll
      for (int o = 0; o < kVR; ++o) {
        const int k = j - o;
        if (k < 0 || k >= kSsimWin) continue;
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[q][o] = fmaf(wt.w[k], v[q], acc[q][o]);
      }
    }
    double sum = 0.0;
#pragma unroll
    for (int o = 0; o < kVR; ++o) {
      const int y = by * kTY + r0 + o;
      if (y >= H || x >= W) continue;
      const float xi = pi[o], ti = pt[o];
      const float d = xi - ti;
      // L_recon weight 1 + m^2 + t^2 (plain MSE without a mask)
      const float w = Mi ? 1.f + pm[o] * pm[o] + ti * ti : 1.f;
      const float dI =
          2.f * w * d * inv_n + coef * (acc[0][o] + 2.f * xi * acc[1][o] + ti * acc[2][o]);
      ui[(size_t)y * W + x] = make_float2(2.f * dI * pu[o].x, 2.f * dI * pu[o].y);
      sum += (double)d * (double)d;
    }
    const double s = block_sum_f64(sum, red);
    if (tid == 0) part[t] = s;
  }
}

// persistent grid: two blocks per compute unit (the LDS of each kernel allows two)
static int ssim_blocks(const Ctx &c, int tiles) { return std::min(tiles, 2 * c.num_cu); }

hipError_t launch_ssim_fwd(const Ctx &c, const float *target, hipStream_t s) {
  const int Hv = c.H - kSsimWin + 1, Wv = c.W - kSsimWin + 1;
  const TileGrid tg{tiles_x(Wv), tiles_y(Hv), tiles_x(Wv) * tiles_y(Hv) * c.L * c.C};
  hipLaunchKernelGGL(k_ssim_fwd, dim3(ssim_blocks(c, tg.total)), dim3(256), 0, s, c.ssim_I,
                     target, c.H, c.W, tg, ssim_window(), c.ssim_abc,
                     (size_t)c.L * c.C * Hv * Wv, c.ssim_part);
  return hipGetLastError();
}

hipError_t launch_ssim_bwd(const Ctx &c, const float *target, const float *mask,
                           float ssim_weight, hipStream_t s) {
  const int Hv = c.H - kSsimWin + 1, Wv = c.W - kSsimWin + 1;
  const double npos = (double)c.L * c.C * Hv * Wv;
  const double n_el = (double)c.L * c.C * c.H * c.W;
  const TileGrid tg{tiles_x(c.W), tiles_y(c.H), tiles_x(c.W) * tiles_y(c.H) * c.L * c.C};
  hipLaunchKernelGGL(k_ssim_bwd, dim3(ssim_blocks(c, tg.total)), dim3(256), 0, s, c.ssim_I,
                     target, mask, c.ssim_abc, (size_t)c.L * c.C * Hv * Wv, c.ssim_u, c.H,
                     c.W, c.C, tg, ssim_window(),
                     (float)(-(double)ssim_weight / npos), (float)(1.0 / n_el), c.mse_part);
  return hipGetLastError();
}

// loss[0] = L_recon + w (1 - mean SSIM), loss[1] = 10 log10(1 / MSE); one block,
// fixed-order sums
__global__ __launch_bounds__(256) void k_full_loss_finalize(
    const double *__restrict__ recon, int n_recon, const double *__restrict__ ssim, int n_ssim,
    const double *__restrict__ mse, int n_mse, double inv_n, double inv_pos, double weight,
    double *__restrict__ out) {
  __shared__ double red[4];
  // four independent chains per thread and sum, each in a fixed order
  auto chain = [](const double *__restrict__ v, int n) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    int i = threadIdx.x;
    for (; i + 3 * 256 < n; i += 4 * 256) {
      s[0] += v[i];
      s[1] += v[i + 256];
      s[2] += v[i + 512];
      s[3] += v[i + 768];
    }
    if (i < n) s[0] += v[i];
    if (i + 256 < n) s[1] += v[i + 256];
    if (i + 512 < n) s[2] += v[i + 512];
    return (s[0] + s[1]) + (s[2] + s[3]);
  };
  const double a = chain(recon, n_recon), b = chain(ssim, n_ssim), m = chain(mse, n_mse);
  const double sa = block_sum_f64(a, red);
  __syncthreads();
  const double sb = block_sum_f64(b, red);
  __syncthreads();
  const double sm = block_sum_f64(m, red);
  if (threadIdx.x == 0) {
    out[0] = sa * inv_n + weight * (1.0 - sb * inv_pos);
    out[1] = 10.0 * log10(1.0 / (sm * inv_n));
  }
}

hipError_t launch_full_loss_finalize(const Ctx &c, float ssim_weight, double *loss,
                                     hipStream_t s) {
  const int Hv = c.H - kSsimWin + 1, Wv = c.W - kSsimWin + 1;
  const int LC = c.L * c.C;
  const int rows = c.C * ((c.H + row_group_rows(c) - 1) / row_group_rows(c));
  hipLaunchKernelGGL(k_full_loss_finalize, dim3(1), dim3(256), 0, s, c.loss_part, c.L * rows,
                     c.ssim_part, LC * ssim_pos_tiles(c), c.mse_part, LC * ssim_pix_tiles(c),
                     1.0 / ((double)LC * c.H * c.W), 1.0 / ((double)LC * Hv * Wv),
                     (double)ssim_weight, loss);
  return hipGetLastError();
}

}  // namespace cgh
