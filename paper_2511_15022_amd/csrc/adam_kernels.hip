// Fused optimiser updates over the flat parameter array, FP32, one pass each:
// Adam (Kingma & Ba, Algorithm 1) and Adan (Xie et al., Adan: adaptive
// Nesterov momentum, Algorithm 1, with bias-corrected moments), the
// optimiser the paper trains with (Sec. 4).
#include <algorithm>
#include <cmath>

#include "cgh_internal.h"

namespace cgh {

// lr_scaled = lr / (1 - b1^t) (uniform), or per parameter block when
// group_lr != nullptr (six blocks of the layout mean, scale, rotation,
// amplitude, phase, opacity with sizes 2n, 2n, n, Cn, Cn, n).
struct GroupLr {
  float lr[6];
  int64_t end[6];
};

__global__ __launch_bounds__(256) void k_adam(float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v,
                                              int64_t count, float lr_scaled, float b1,
                                              float b2, float eps, float inv_sqrt_bc2,
                                              GroupLr groups, int use_groups) {
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= count) return;
  if (i0 + 4 <= count && !use_groups) {
    float4 pp = *reinterpret_cast<float4 *>(p + i0);
    const float4 gg = *reinterpret_cast<const float4 *>(g + i0);
    float4 mm = *reinterpret_cast<float4 *>(m + i0);
    float4 vv = *reinterpret_cast<float4 *>(v + i0);
    adam_one(pp.x, gg.x, mm.x, vv.x, lr_scaled, b1, b2, eps, inv_sqrt_bc2);
    adam_one(pp.y, gg.y, mm.y, vv.y, lr_scaled, b1, b2, eps, inv_sqrt_bc2);
    adam_one(pp.z, gg.z, mm.z, vv.z, lr_scaled, b1, b2, eps, inv_sqrt_bc2);
    adam_one(pp.w, gg.w, mm.w, vv.w, lr_scaled, b1, b2, eps, inv_sqrt_bc2);
    *reinterpret_cast<float4 *>(p + i0) = pp;
    *reinterpret_cast<float4 *>(m + i0) = mm;
    *reinterpret_cast<float4 *>(v + i0) = vv;
    return;
  }
  for (int64_t i = i0; i < i0 + 4 && i < count; ++i) {
    float lr = lr_scaled;
    if (use_groups) {
      int k = 0;
      while (k < 5 && i >= groups.end[k]) ++k;
      lr = groups.lr[k];
    }
    float pi = p[i], mi = m[i], vi = v[i];
    adam_one(pi, g[i], mi, vi, lr, b1, b2, eps, inv_sqrt_bc2);
    p[i] = pi;
    m[i] = mi;
    v[i] = vi;
  }
}

// Adan, decay-rate convention (beta close to 1).  With diff = g - g_prev
// (zero at the first step):
//   m = b1 m + (1 - b1) g
//   d = b2 d + (1 - b2) diff
//   s = b3 s + (1 - b3) (g + b2 diff)^2      (Nesterov-corrected gradient)
//   p = p (1 - lr wd) - lr (m / bc1 + b2 d / bc2) / (sqrt(s / bc3) + eps)
// with bc_i = 1 - b_i^t; g_prev <- g.
struct AdanArgs {
  float b1, b2, b3, eps, wd;
  float inv_bc1, inv_bc2, inv_sqrt_bc3;
  int first;
};

__device__ __forceinline__ void adan_one(float &p, float g, float &m, float &d, float &s,
                                         float &gp, float lr, const AdanArgs &a) {
  const float diff = a.first ? 0.f : g - gp;
  m = fmaf(a.b1, m, (1.0f - a.b1) * g);
  d = fmaf(a.b2, d, (1.0f - a.b2) * diff);
  const float u = fmaf(a.b2, diff, g);
  s = fmaf(a.b3, s, (1.0f - a.b3) * u * u);
  gp = g;
  const float denom = sqrtf(s) * a.inv_sqrt_bc3 + a.eps;
  const float step = fmaf(a.b2 * a.inv_bc2, d, m * a.inv_bc1) / denom;
  p = fmaf(p, -lr * a.wd, p) - lr * step;
}

__global__ __launch_bounds__(256) void k_adan(float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ d,
                                              float *__restrict__ s, float *__restrict__ gprev,
                                              int64_t count, float lr, AdanArgs a,
                                              GroupLr groups, int use_groups) {
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= count) return;
  if (i0 + 4 <= count && !use_groups) {
    float4 pp = *reinterpret_cast<float4 *>(p + i0);
    const float4 gg = *reinterpret_cast<const float4 *>(g + i0);
    float4 mm = *reinterpret_cast<float4 *>(m + i0);
    float4 dd = *reinterpret_cast<float4 *>(d + i0);
    float4 ss = *reinterpret_cast<float4 *>(s + i0);
    float4 qq = *reinterpret_cast<float4 *>(gprev + i0);
    adan_one(pp.x, gg.x, mm.x, dd.x, ss.x, qq.x, lr, a);
    adan_one(pp.y, gg.y, mm.y, dd.y, ss.y, qq.y, lr, a);
    adan_one(pp.z, gg.z, mm.z, dd.z, ss.z, qq.z, lr, a);
    adan_one(pp.w, gg.w, mm.w, dd.w, ss.w, qq.w, lr, a);
    *reinterpret_cast<float4 *>(p + i0) = pp;
    *reinterpret_cast<float4 *>(m + i0) = mm;
    *reinterpret_cast<float4 *>(d + i0) = dd;
    *reinterpret_cast<float4 *>(s + i0) = ss;
    *reinterpret_cast<float4 *>(gprev + i0) = qq;
    return;
  }
  for (int64_t i = i0; i < i0 + 4 && i < count; ++i) {
    float lri = lr;
    if (use_groups) {
      int k = 0;
      while (k < 5 && i >= groups.end[k]) ++k;
      lri = groups.lr[k];
    }
    float pi = p[i], mi = m[i], di = d[i], si = s[i], qi = gprev[i];
    adan_one(pi, g[i], mi, di, si, qi, lri, a);
    p[i] = pi;
    m[i] = mi;
    d[i] = di;
    s[i] = si;
    gprev[i] = qi;
  }
}

static GroupLr group_lrs(const float *lr_groups, int n, int C, int *use) {
  GroupLr gr{};
  *use = 0;
  if (lr_groups) {
    *use = 1;
    const int64_t sizes[6] = {2LL * n, 2LL * n, n, (int64_t)C * n, (int64_t)C * n, n};
    int64_t acc = 0;
    for (int k = 0; k < 6; ++k) {
      acc += sizes[k];
      gr.end[k] = acc;
      gr.lr[k] = lr_groups[k];
    }
  }
  return gr;
}

hipError_t launch_adan(float *p, const float *g, float *m, float *d, float *s, float *gprev,
                       int64_t count, int t, float lr, float b1, float b2, float b3, float eps,
                       float wd, const float *lr_groups, int n, int C, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  AdanArgs a;
  a.b1 = b1; a.b2 = b2; a.b3 = b3; a.eps = eps; a.wd = wd;
  a.inv_bc1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)t)));
  // the difference moment is zero at t = 1, so its correction only matters later
  const double bc2 = 1.0 - std::pow((double)b2, (double)t);
  a.inv_bc2 = bc2 > 0.0 ? (float)(1.0 / bc2) : 0.f;
  a.inv_sqrt_bc3 = (float)(1.0 / std::sqrt(1.0 - std::pow((double)b3, (double)t)));
  a.first = t == 1;
  int use = 0;
  const GroupLr gr = group_lrs(lr_groups, n, C, &use);
  const int64_t threads = (count + 3) / 4;
  hipLaunchKernelGGL(k_adan, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, p, g, m,
                     d, s, gprev, count, lr, a, gr, use);
  return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t count, float lr,
                       float step_size_scale, float beta1, float beta2, float eps,
                       float inv_sqrt_bc2, const float *lr_groups, int n, int C,
                       hipStream_t s) {
  if (count <= 0) return hipSuccess;
  GroupLr gr{};
  int use = 0;
  if (lr_groups) {
    use = 1;
    const int64_t sizes[6] = {2LL * n, 2LL * n, n, (int64_t)C * n, (int64_t)C * n, n};
    int64_t acc = 0;
    for (int k = 0; k < 6; ++k) {
      acc += sizes[k];
      gr.end[k] = acc;
      gr.lr[k] = lr_groups[k] * step_size_scale;
    }
  }
  const int64_t threads = (count + 3) / 4;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, p, g, m,
                     v, count, lr * step_size_scale, beta1, beta2, eps, inv_sqrt_bc2, gr, use);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero_pair(float *__restrict__ a, float *__restrict__ b,
                                                   int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += stride) {
    a[i] = 0.f;
    b[i] = 0.f;
  }
}

// a[0 .. count) = b[0 .. count) = 0 by a kernel (no memset node when captured)
hipError_t launch_zero_pair(float *a, float *b, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero_pair, dim3((unsigned)blocks), dim3(256), 0, s, a, b, count);
  return hipGetLastError();
}

}  // namespace cgh
