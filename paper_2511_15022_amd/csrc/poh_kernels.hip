// Phase-only hologram conversion (include/cgh_poh.h): double-phase coding of
// the Smooth POH and the elementwise parts of the Random POH's joint
// optimisation (the L_extract seed of the two adjoint propagations, exp(j phi)
// and the phase gradient).
#include <cmath>

#include "cgh_internal.h"
#include "cgh_poh.h"

namespace cgh {
namespace {

unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

__global__ void k_zero_f32(float *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// per-channel max of |field|: block reduction, then an atomic max on the bits
// (non-negative floats order as their unsigned bit patterns)
__global__ __launch_bounds__(256) void k_absmax(const float2 *__restrict__ f, int64_t count,
                                                float *__restrict__ amax) {
  __shared__ float red[4];
  const int c = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float v = 0.f;
  if (i < count) {
    const float2 z = f[(size_t)c * count + i];
    v = sqrtf(z.x * z.x + z.y * z.y);
  }
  for (int d = 32; d > 0; d >>= 1) v = fmaxf(v, __shfl_down(v, d, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    atomicMax(reinterpret_cast<unsigned int *>(amax + c), __float_as_uint(m));
  }
}

__global__ void k_dpac(const float2 *__restrict__ f, int64_t count, int W,
                       const float *__restrict__ amax, float *__restrict__ phase) {
  const int c = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float2 z = f[(size_t)c * count + i];
  const float m = amax[c];
  const float a = m > 0.f ? fminf(sqrtf(z.x * z.x + z.y * z.y) / m, 1.f) : 0.f;
  const float phi = atan2f(z.y, z.x), d = acosf(a);
  const int64_t y = i / W, x = i - y * W;
  phase[(size_t)c * count + i] = ((x + y) & 1) ? phi - d : phi + d;
}

__global__ void k_expj(const float *__restrict__ phase, int64_t n, float2 *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s, co;
  sincosf(phase[i], &s, &co);
  out[i] = make_float2(co, s);
}

__global__ void k_phase_grad(const float *__restrict__ phase, const float2 *__restrict__ g,
                             int64_t n, float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s, co;
  sincosf(phase[i], &s, &co);
  const float2 v = g[i];
  out[i] = v.y * co - v.x * s;  // Im(conj(e^{j phi}) g)
}

__device__ __forceinline__ float sgn(float v) { return v > 0.f ? 1.f : (v < 0.f ? -1.f : 0.f); }

// one element per thread; FP64 partial per 256-thread block
__global__ __launch_bounds__(256) void k_extract(
    const float2 *__restrict__ u, const float2 *__restrict__ ur, const float *__restrict__ T,
    const float *__restrict__ mask, int C, int HW, int64_t n, float inv_n, float lc, float lf,
    float2 *__restrict__ gu, float2 *__restrict__ gur, double *__restrict__ part) {
  __shared__ double red[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double acc = 0.0;
  if (i < n) {
    const float2 a = u[i], b = ur[i];
    const float t = T[i];
    // focal mask of the element's plane, shared by the channels: [L][H][W]
    const int64_t plane = i / ((int64_t)C * HW), px = i % HW;
    const float m = mask ? mask[plane * HW + px] : 0.f;
    const float w = mask ? 1.f + m * m + t * t : 1.f;
    const float I = a.x * a.x + a.y * a.y, Ir = b.x * b.x + b.y * b.y;
    const float r = I - t, rr = Ir - t, dI = I - Ir;
    const float dx = a.x - b.x, dy = a.y - b.y;
    acc = (double)w * ((double)r * r + (double)rr * rr) + (double)lc * (double)dI * dI +
          (double)lf * (double)(fabsf(dx) + fabsf(dy));
    // d/dI of w r^2 / n and of lc dI^2 / n; the chain to u is 2 u
    const float gI = 2.f * inv_n * (w * r + lc * dI), gIr = 2.f * inv_n * (w * rr - lc * dI);
    const float fx = lf * inv_n * sgn(dx), fy = lf * inv_n * sgn(dy);
    gu[i] = make_float2(2.f * gI * a.x + fx, 2.f * gI * a.y + fy);
    gur[i] = make_float2(2.f * gIr * b.x - fx, 2.f * gIr * b.y - fy);
  }
  for (int d = 32; d > 0; d >>= 1) acc += __shfl_down(acc, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_extract_finalize(const double *__restrict__ part, int64_t k,
                                                          double inv_n, double *__restrict__ loss) {
  __shared__ double red[4];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < k; i += 256) a += part[i];
  for (int d = 32; d > 0; d >>= 1) a += __shfl_down(a, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) loss[0] = ((red[0] + red[1]) + (red[2] + red[3])) * inv_n;
}

}  // namespace
}  // namespace cgh

using namespace cgh;

#define POH_CHECK(cond, ...) \
  do {                       \
    if (!(cond)) return report(CGH_ERR_INVALID_ARG, __VA_ARGS__); \
  } while (0)
#define POH_LAUNCHED(where)                                                           \
  do {                                                                                \
    const hipError_t e_ = hipGetLastError();                                          \
    if (e_ != hipSuccess) return report(CGH_ERR_DEVICE, "%s: %s", where, hipGetErrorString(e_)); \
  } while (0)

extern "C" {

cgh_status cgh_poh_dpac(const cgh_c64 *field, int32_t C, int32_t H, int32_t W, float *amax,
                        float *phase, void *stream) {
  POH_CHECK(field && amax && phase && C >= 1 && C <= CGH_MAX_CHANNELS && H >= 1 && W >= 1,
            "bad arguments");
  const int64_t count = (int64_t)H * W;
  hipStream_t s = (hipStream_t)stream;
  const float2 *f = reinterpret_cast<const float2 *>(field);
  hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, amax, C);
  hipLaunchKernelGGL(k_absmax, dim3(nblocks(count, 256), C), dim3(256), 0, s, f, count, amax);
  hipLaunchKernelGGL(k_dpac, dim3(nblocks(count, 256), C), dim3(256), 0, s, f, count, W, amax,
                     phase);
  POH_LAUNCHED("poh_dpac");
  return CGH_OK;
}

cgh_status cgh_poh_field(const float *phase, int64_t count, cgh_c64 *field, void *stream) {
  POH_CHECK(phase && field && count > 0, "bad arguments");
  hipLaunchKernelGGL(k_expj, dim3(nblocks(count, 256)), dim3(256), 0, (hipStream_t)stream, phase,
                     count, reinterpret_cast<float2 *>(field));
  POH_LAUNCHED("poh_field");
  return CGH_OK;
}

cgh_status cgh_poh_phase_grad(const float *phase, const cgh_c64 *grad_field, int64_t count,
                              float *grad_phase, void *stream) {
  POH_CHECK(phase && grad_field && grad_phase && count > 0, "bad arguments");
  hipLaunchKernelGGL(k_phase_grad, dim3(nblocks(count, 256)), dim3(256), 0, (hipStream_t)stream,
                     phase, reinterpret_cast<const float2 *>(grad_field), count, grad_phase);
  POH_LAUNCHED("poh_phase_grad");
  return CGH_OK;
}

int64_t cgh_poh_extract_partials(int64_t count) { return count > 0 ? (count + 255) / 256 : 0; }

cgh_status cgh_poh_extract_seed(const cgh_c64 *u, const cgh_c64 *u_rand, const float *target,
                                const float *mask, int32_t L, int32_t C, int32_t H, int32_t W,
                                float l_comp, float l_field, cgh_c64 *grad_u,
                                cgh_c64 *grad_u_rand, double *partials, double *loss,
                                void *stream) {
  POH_CHECK(u && u_rand && target && grad_u && grad_u_rand && partials, "NULL buffer");
  POH_CHECK(L >= 1 && C >= 1 && H >= 1 && W >= 1, "bad sizes");
  POH_CHECK(l_comp >= 0.f && l_field >= 0.f && std::isfinite(l_comp) && std::isfinite(l_field),
            "weights must be >= 0 and finite");
  const int64_t n = (int64_t)L * C * H * W;
  const int64_t k = cgh_poh_extract_partials(n);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_extract, dim3((unsigned)k), dim3(256), 0, s,
                     reinterpret_cast<const float2 *>(u), reinterpret_cast<const float2 *>(u_rand),
                     target, mask, C, H * W, n, (float)(1.0 / (double)n), l_comp, l_field,
                     reinterpret_cast<float2 *>(grad_u), reinterpret_cast<float2 *>(grad_u_rand),
                     partials);
  POH_LAUNCHED("poh_extract_seed");
  if (loss) {
    hipLaunchKernelGGL(k_extract_finalize, dim3(1), dim3(256), 0, s, partials, k, 1.0 / (double)n,
                       loss);
    POH_LAUNCHED("poh_extract_finalize");
  }
  return CGH_OK;
}

}  // extern "C"
