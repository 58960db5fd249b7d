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
#include <cmath>

#include "cgh_internal.h"

namespace cgh {

constexpr int kSsimWin = 11;
constexpr int kSsimTile = 32;                         // positions (or pixels) per tile side
constexpr int kSsimSpan = kSsimTile + kSsimWin - 1;  // 42: tile plus window
constexpr float kSsimC1 = 0.01f * 0.01f, kSsimC2 = 0.03f * 0.03f;

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

static int tiles_of(int n) { return (n + kSsimTile - 1) / kSsimTile; }
int ssim_pos_tiles(const Ctx &c) { return tiles_of(c.W - kSsimWin + 1) * tiles_of(c.H - kSsimWin + 1); }
int ssim_pix_tiles(const Ctx &c) { return tiles_of(c.W) * tiles_of(c.H); }

// fixed-order FP64 sum over a 256-thread block; the result is valid in thread 0
__device__ double block_sum_f64(double v, double *red) {
  for (int d = 32; d > 0; d >>= 1) v += __shfl_down(v, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// grid (position tiles x, y; image l C + c), 256 threads
__global__ __launch_bounds__(256) void k_ssim_fwd(const float *__restrict__ I,
                                                  const float *__restrict__ T, int H, int W,
                                                  SsimWin wt, float *__restrict__ abc,
                                                  size_t abc_plane, double *__restrict__ part) {
  __shared__ float sx[kSsimSpan][kSsimSpan + 1], sy[kSsimSpan][kSsimSpan + 1];
  __shared__ float h[5][kSsimSpan][kSsimTile + 1];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int Hv = H - kSsimWin + 1, Wv = W - kSsimWin + 1;
  const int px0 = blockIdx.x * kSsimTile, py0 = blockIdx.y * kSsimTile, img = blockIdx.z;
  const float *Ii = I + (size_t)img * H * W, *Ti = T + (size_t)img * H * W;
  for (int i = tid; i < kSsimSpan * kSsimSpan; i += 256) {
    const int r = i / kSsimSpan, c = i - r * kSsimSpan, y = py0 + r, x = px0 + c;
    const bool in = y < H && x < W;
    const size_t o = (size_t)min(y, H - 1) * W + min(x, W - 1);
    sx[r][c] = in ? Ii[o] : 0.f;
    sy[r][c] = in ? Ti[o] : 0.f;
  }
  __syncthreads();
  for (int i = tid; i < kSsimSpan * kSsimTile; i += 256) {
    const int r = i / kSsimTile, c = i - r * kSsimTile;
    float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
    for (int k = 0; k < kSsimWin; ++k) {
      const float x = sx[r][c + k], y = sy[r][c + k], wk = wt.w[k];
      a = fmaf(wk, x, a);
      b = fmaf(wk, y, b);
      aa = fmaf(wk * x, x, aa);
      bb = fmaf(wk * y, y, bb);
      ab = fmaf(wk * x, y, ab);
    }
    h[0][r][c] = a; h[1][r][c] = b; h[2][r][c] = aa; h[3][r][c] = bb; h[4][r][c] = ab;
  }
  __syncthreads();
  double acc = 0.0;
  for (int i = tid; i < kSsimTile * kSsimTile; i += 256) {
    const int r = i / kSsimTile, c = i - r * kSsimTile, py = py0 + r, px = px0 + c;
    if (py >= Hv || px >= Wv) continue;
    float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < kSsimWin; ++k)
#pragma unroll
      for (int q = 0; q < 5; ++q) m[q] = fmaf(wt.w[k], h[q][r + k][c], m[q]);
    const float mx = m[0], my = m[1];
    const float sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
    const float n1 = 2.f * mx * my + kSsimC1, n2 = 2.f * sxy + kSsimC2;
    const float d1 = mx * mx + my * my + kSsimC1, d2 = sxx + syy + kSsimC2;
    const float inv = 1.f / (d1 * d2);
    const float S = n1 * n2 * inv;
    const float dmx = 2.f * my * n2 * inv - 2.f * mx * S / d1;  // at fixed sigmas
    const float B = -S / d2, Cc = 2.f * n1 * inv;
    const size_t o = ((size_t)img * Hv + py) * Wv + px;
    abc[o] = dmx - 2.f * mx * B - my * Cc;
    abc[abc_plane + o] = B;
    abc[2 * abc_plane + o] = Cc;
    acc += (double)S;
  }
  const double s = block_sum_f64(acc, red);
  if (tid == 0) part[(size_t)img * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// grid (pixel tiles x, y; image l C + c), 256 threads.  coef = -ssim_weight / (number
// of positions over all images); inv_n = 1 / (L C H W).
__global__ __launch_bounds__(256) void k_ssim_bwd(
    const float *__restrict__ I, const float *__restrict__ T, const float *__restrict__ mask,
    const float *__restrict__ abc, size_t abc_plane, float2 *__restrict__ u, int H, int W,
    int C, SsimWin wt, float coef, float inv_n, double *__restrict__ part) {
  __shared__ float sa[3][kSsimSpan][kSsimSpan + 1];
  __shared__ float h[3][kSsimSpan][kSsimTile + 1];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int Hv = H - kSsimWin + 1, Wv = W - kSsimWin + 1;
  const int qx0 = blockIdx.x * kSsimTile, qy0 = blockIdx.y * kSsimTile, img = blockIdx.z;
  const int plane = img / C;
  // coefficients at positions [qy0 - 10, qy0 + 32) x [qx0 - 10, qx0 + 32), zero
  // outside the valid positions
  for (int i = tid; i < kSsimSpan * kSsimSpan; i += 256) {
    const int r = i / kSsimSpan, c = i - r * kSsimSpan;
    const int py = qy0 - (kSsimWin - 1) + r, px = qx0 - (kSsimWin - 1) + c;
    const bool in = py >= 0 && py < Hv && px >= 0 && px < Wv;
    const size_t o = ((size_t)img * Hv + min(max(py, 0), Hv - 1)) * Wv + min(max(px, 0), Wv - 1);
#pragma unroll
    for (int q = 0; q < 3; ++q) sa[q][r][c] = in ? abc[q * abc_plane + o] : 0.f;
  }
  __syncthreads();
  for (int i = tid; i < kSsimSpan * kSsimTile; i += 256) {
    const int r = i / kSsimTile, c = i - r * kSsimTile;
    float v[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < kSsimWin; ++k)
#pragma unroll
      for (int q = 0; q < 3; ++q) v[q] = fmaf(wt.w[k], sa[q][r][c + k], v[q]);
#pragma unroll
    for (int q = 0; q < 3; ++q) h[q][r][c] = v[q];
  }
  __syncthreads();
  const float *Ii = I + (size_t)img * H * W, *Ti = T + (size_t)img * H * W;
  const float *Mi = mask ? mask + (size_t)plane * H * W : nullptr;
  float2 *ui = u + (size_t)img * H * W;
  double acc = 0.0;
  for (int i = tid; i < kSsimTile * kSsimTile; i += 256) {
    const int r = i / kSsimTile, c = i - r * kSsimTile, y = qy0 + r, x = qx0 + c;
    if (y >= H || x >= W) continue;
    float v[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < kSsimWin; ++k)
#pragma unroll
      for (int q = 0; q < 3; ++q) v[q] = fmaf(wt.w[k], h[q][r + k][c], v[q]);
    const size_t o = (size_t)y * W + x;
    const float xi = Ii[o], ti = Ti[o];
    const float d = xi - ti;
    // L_recon weight 1 + m^2 + t^2 (plain MSE without a mask)
    const float w = Mi ? 1.f + Mi[o] * Mi[o] + ti * ti : 1.f;
    const float dI = 2.f * w * d * inv_n + coef * (v[0] + 2.f * xi * v[1] + ti * v[2]);
    const float2 uu = ui[o];
    ui[o] = make_float2(2.f * dI * uu.x, 2.f * dI * uu.y);
    acc += (double)d * (double)d;
  }
  const double s = block_sum_f64(acc, red);
  if (tid == 0) part[(size_t)img * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] = s;
}

hipError_t launch_ssim_fwd(const Ctx &c, const float *target, hipStream_t s) {
  const int Hv = c.H - kSsimWin + 1, Wv = c.W - kSsimWin + 1;
  const dim3 grid(tiles_of(Wv), tiles_of(Hv), c.L * c.C);
  hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, s, c.ssim_I, target, c.H, c.W,
                     ssim_window(), c.ssim_abc, (size_t)c.L * c.C * Hv * Wv, c.ssim_part);
  return hipGetLastError();
}

hipError_t launch_ssim_bwd(const Ctx &c, const float *target, const float *mask,
                           float ssim_weight, hipStream_t s) {
  const int Hv = c.H - kSsimWin + 1, Wv = c.W - kSsimWin + 1;
  const double npos = (double)c.L * c.C * Hv * Wv;
  const double n_el = (double)c.L * c.C * c.H * c.W;
  const dim3 grid(tiles_of(c.W), tiles_of(c.H), c.L * c.C);
  hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, s, c.ssim_I, target, mask, c.ssim_abc,
                     (size_t)c.L * c.C * Hv * Wv, c.ssim_u, c.H, c.W, c.C, ssim_window(),
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
  double a = 0.0, b = 0.0, m = 0.0;
  for (int i = threadIdx.x; i < n_recon; i += 256) a += recon[i];
  for (int i = threadIdx.x; i < n_ssim; i += 256) b += ssim[i];
  for (int i = threadIdx.x; i < n_mse; i += 256) m += mse[i];
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
