// Fused Adam update (Kingma & Ba, Algorithm 1) over the flat parameter array,
// FP32, one pass: read p, g, m, v; write p, m, v.
#include "cgh_internal.h"

namespace cgh {

__device__ __forceinline__ void adam_one(float &p, float g, float &m, float &v, float lr_scaled,
                                         float b1, float b2, float eps, float inv_sqrt_bc2) {
  m = fmaf(b1, m, (1.0f - b1) * g);
  v = fmaf(b2, v, (1.0f - b2) * g * g);
  const float denom = sqrtf(v) * inv_sqrt_bc2 + eps;
  p -= lr_scaled * m / denom;
}

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

}  // namespace cgh
