// Band-limited angular-spectrum propagation on gfx950: mixed-radix Stockham
// FFTs held in LDS, the transfer-function multiply fused into the column
// pass, and intensity / MSE / adjoint seed fused into the middle row pass.
//
// The propagation of one channel is u = crop(IFFT2(H . FFT2(pad(U0))))
// (Sec. 2; Alg. 1 ZeroPad + MultiPlanePropagate).  Because FFT2 -> H -> IFFT2
// is a circular convolution, padding the field at the start of each row and
// column (instead of centring it) and cropping the same leading window gives
// the same u; the kernels use that placement so rows and columns never touch
// the zero padding in memory:
//   F1  row FFT:    U0 [C][H][W] -> X [C][H][Wp]           (rows zero-extended)
//   F2  column pass X: FFT over Hp (zero-extended), x H/(Hp Wp), IFFT, keep H rows
//   F3  row pass:   IFFT, crop W -> u; I = |u|^2; loss; g = dL/du; zero-extend; FFT
//   B1  column pass with conj(H) (the adjoint, supplementary BLASM Backward Pass)
//   B2  row IFFT, crop W -> dL/dU0
#include <cmath>

#include "cgh_internal.h"

namespace cgh {

// ----------------------------------------------------------------------------
// complex helpers
// ----------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// multiply by DIR * i  (DIR = -1: forward kernel e^{-i}, +1: inverse)
template <int DIR>
__device__ __forceinline__ float2 rot90(float2 a) {
  return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ----------------------------------------------------------------------------
// small DFTs: y_k = sum_q x_q exp(DIR 2 pi i q k / R)
// ----------------------------------------------------------------------------
template <int R, int DIR>
struct Dft;

template <int DIR>
struct Dft<2, DIR> {
  static __device__ __forceinline__ void run(float2 *x) {
    float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <int DIR>
struct Dft<3, DIR> {
  static __device__ __forceinline__ void run(float2 *x) {
    const float h = 0.86602540378443864676f;  // sin(2 pi / 3)
    float2 s = cadd(x[1], x[2]), d = csub(x[1], x[2]);
    float2 t = make_float2(x[0].x - 0.5f * s.x, x[0].y - 0.5f * s.y);
    float2 r = rot90<DIR>(cscale(d, h));
    x[0] = cadd(x[0], s);
    x[1] = cadd(t, r);
    x[2] = csub(t, r);
  }
};

template <int DIR>
struct Dft<4, DIR> {
  static __device__ __forceinline__ void run(float2 *x) {
    float2 a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
    float2 c = cadd(x[1], x[3]), d = rot90<DIR>(csub(x[1], x[3]));
    x[0] = cadd(a, c);
    x[2] = csub(a, c);
    x[1] = cadd(b, d);
    x[3] = csub(b, d);
  }
};

template <int DIR>
struct Dft<5, DIR> {
  static __device__ __forceinline__ void run(float2 *x) {
    const float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
    const float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
    const float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
    const float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
    float2 s14 = cadd(x[1], x[4]), d14 = csub(x[1], x[4]);
    float2 s23 = cadd(x[2], x[3]), d23 = csub(x[2], x[3]);
    float2 x0 = x[0];
    float2 ta = make_float2(x0.x + c1 * s14.x + c2 * s23.x, x0.y + c1 * s14.y + c2 * s23.y);
    float2 tb = make_float2(x0.x + c2 * s14.x + c1 * s23.x, x0.y + c2 * s14.y + c1 * s23.y);
    float2 tc = rot90<DIR>(make_float2(s1 * d14.x + s2 * d23.x, s1 * d14.y + s2 * d23.y));
    float2 td = rot90<DIR>(make_float2(s2 * d14.x - s1 * d23.x, s2 * d14.y - s1 * d23.y));
    x[0] = cadd(x0, cadd(s14, s23));
    x[1] = cadd(ta, tc);
    x[4] = csub(ta, tc);
    x[2] = cadd(tb, td);
    x[3] = csub(tb, td);
  }
};

template <int DIR>
struct Dft<8, DIR> {
  static __device__ __forceinline__ void run(float2 *x) {
    const float r = 0.70710678118654752440f;
    float2 e[4] = {x[0], x[2], x[4], x[6]};
    float2 o[4] = {x[1], x[3], x[5], x[7]};
    Dft<4, DIR>::run(e);
    Dft<4, DIR>::run(o);
    // twiddles w8^k = exp(DIR 2 pi i k / 8)
    float2 o1 = cscale(cadd(o[1], rot90<DIR>(o[1])), r);
    float2 o2 = rot90<DIR>(o[2]);
    float2 o3 = cscale(csub(rot90<DIR>(o[3]), o[3]), r);
    x[0] = cadd(e[0], o[0]);
    x[4] = csub(e[0], o[0]);
    x[1] = cadd(e[1], o1);
    x[5] = csub(e[1], o1);
    x[2] = cadd(e[2], o2);
    x[6] = csub(e[2], o2);
    x[3] = cadd(e[3], o3);
    x[7] = csub(e[3], o3);
  }
};

// ----------------------------------------------------------------------------
// One Stockham stage over B interleaved transforms held in LDS:
// element (index r, transform b) lives at buf[r * B + b].  Butterfly j of
// transform b reads r = j + q n/R (q < R), twiddles by exp(DIR 2 pi i q k /
// (Ns R)) with k = j mod Ns, and writes to (j / Ns) Ns R + k + q Ns.  All
// reads of a stage complete (barrier) before its writes, so one buffer
// suffices; each thread keeps its butterflies in registers across the barrier.
// ----------------------------------------------------------------------------
template <int R, int DIR, int B, int T, int MAXN>
__device__ __forceinline__ void fft_stage(float2 *__restrict__ buf, int n, int Ns,
                                          uint32_t magic, int tws,
                                          const float2 *__restrict__ tw, int tid) {
  constexpr int MAXIT = (B * ((MAXN + R - 1) / R) + T - 1) / T;
  const int nb = n / R;
  const int items = nb * B;
  float2 v[MAXIT][R];
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int i = tid + it * T;
    if (i < items) {
      const int b = i % B, j = i / B;
#pragma unroll
      for (int q = 0; q < R; ++q) v[it][q] = buf[(j + q * nb) * B + b];
      if (Ns > 1) {
        const int grp = (int)__umulhi((uint32_t)j, magic);
        const int e = (j - grp * Ns) * tws;
#pragma unroll
        for (int q = 1; q < R; ++q) {
          float2 w = tw[q * e];
          if (DIR > 0) w.y = -w.y;
          v[it][q] = cmul(v[it][q], w);
        }
      }
      Dft<R, DIR>::run(v[it]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int i = tid + it * T;
    if (i < items) {
      const int b = i % B, j = i / B;
      const int grp = Ns > 1 ? (int)__umulhi((uint32_t)j, magic) : j;
      const int base = grp * Ns * R + (j - grp * Ns);
#pragma unroll
      for (int q = 0; q < R; ++q) buf[(base + q * Ns) * B + b] = v[it][q];
    }
  }
  __syncthreads();
}

template <int DIR, int B, int T, int MAXN>
__device__ void fft_lds(float2 *__restrict__ buf, const FftPlan &p,
                        const float2 *__restrict__ tw, int tid) {
  for (int s = 0; s < p.nstages; ++s) {
    const int r = p.radix[s];
    if (r == 8)
      fft_stage<8, DIR, B, T, MAXN>(buf, p.n, p.ns[s], p.magic[s], p.tws[s], tw, tid);
    else if (r == 4)
      fft_stage<4, DIR, B, T, MAXN>(buf, p.n, p.ns[s], p.magic[s], p.tws[s], tw, tid);
    else if (r == 3)
      fft_stage<3, DIR, B, T, MAXN>(buf, p.n, p.ns[s], p.magic[s], p.tws[s], tw, tid);
    else if (r == 5)
      fft_stage<5, DIR, B, T, MAXN>(buf, p.n, p.ns[s], p.magic[s], p.tws[s], tw, tid);
    else
      fft_stage<2, DIR, B, T, MAXN>(buf, p.n, p.ns[s], p.magic[s], p.tws[s], tw, tid);
  }
}

// ----------------------------------------------------------------------------
// Host-side planning
// ----------------------------------------------------------------------------
bool smooth235(int n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

bool make_plan(int n, FftPlan *plan) {
  if (!smooth235(n) || n > kMaxFft) return false;
  int rad[kMaxStages];
  int ns = 0, m = n, twos = 0;
  while (m % 2 == 0) { m /= 2; ++twos; }
  // powers of two as radix 8 where possible, leftovers as 4 (or one 2)
  while (twos >= 3 && !(twos == 4)) { rad[ns++] = 8; twos -= 3; }
  while (twos >= 2) { rad[ns++] = 4; twos -= 2; }
  if (twos == 1) rad[ns++] = 2;
  while (m % 3 == 0) { rad[ns++] = 3; m /= 3; }
  while (m % 5 == 0) { rad[ns++] = 5; m /= 5; }
  if (ns > kMaxStages) return false;
  plan->n = n;
  plan->nstages = ns;
  int prod = 1;
  for (int s = 0; s < ns; ++s) {
    plan->radix[s] = rad[s];
    plan->ns[s] = prod;
    plan->magic[s] = prod > 1 ? (uint32_t)((((uint64_t)1 << 32) + prod - 1) / prod) : 0u;
    plan->tws[s] = n / (prod * rad[s]);
    prod *= rad[s];
  }
  for (int s = ns; s < kMaxStages; ++s) {
    plan->radix[s] = 0; plan->ns[s] = 0; plan->magic[s] = 0; plan->tws[s] = 0;
  }
  return true;
}

// ----------------------------------------------------------------------------
// Tables (FP64 on the device, rounded to FP32 once)
// ----------------------------------------------------------------------------
__global__ void k_twiddles(float2 *tw, int n) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s, c;
  sincospi(2.0 * (double)k / (double)n, &s, &c);
  tw[k] = make_float2((float)c, (float)(-s));  // exp(-2 pi i k / n)
}

hipError_t launch_build_twiddles(float2 *tw, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles, dim3((n + 255) / 256), dim3(256), 0, s, tw, n);
  return hipGetLastError();
}

// Band-limited angular-spectrum transfer function (Sec. 2; supplementary
// "Spatial Frequency Computation", "Bandlimit Computation", "Transfer Function
// Evaluation"), quarter table indexed by |fx| = qx / (Wp dx), |fy| = qy / (Hp dx).
// L_x, L_y are the extents of the padded grid.  Evanescent frequencies get 0.
__global__ void k_transfer(float2 *out, int Hq, int Wq, int Hp, int Wp, double pitch,
                           double lambda, double z) {
  int qx = blockIdx.x * blockDim.x + threadIdx.x;
  int qy = blockIdx.y;
  if (qx >= Wq) return;
  const double Lx = Wp * pitch, Ly = Hp * pitch;
  const double fx = qx / Lx, fy = qy / Ly;
  const double ax = 2.0 * z / Lx, ay = 2.0 * z / Ly;
  const double fxmax = 1.0 / (lambda * sqrt(ax * ax + 1.0));
  const double fymax = 1.0 / (lambda * sqrt(ay * ay + 1.0));
  const double arg = 1.0 / (lambda * lambda) - fx * fx - fy * fy;
  float2 h = make_float2(0.f, 0.f);
  if (fx < fxmax && fy < fymax && arg >= 0.0) {
    const double ph = 6.283185307179586476925 * z * sqrt(arg);  // 2 pi z sqrt(arg)
    double sn, cs;
    sincos(ph, &sn, &cs);
    h = make_float2((float)cs, (float)sn);
  }
  out[(size_t)qy * Wq + qx] = h;
}

hipError_t launch_build_transfer(const Ctx &c, hipStream_t s) {
  for (int ch = 0; ch < c.C; ++ch)
    for (int l = 0; l < c.L; ++l) {
      float2 *dst = c.htab + ((size_t)ch * c.L + l) * c.Hq * c.Wq;
      hipLaunchKernelGGL(k_transfer, dim3((c.Wq + 255) / 256, c.Hq), dim3(256), 0, s, dst,
                         c.Hq, c.Wq, c.Hp, c.Wp, c.cfg.pitch_m, c.cfg.wavelength_m[ch],
                         c.cfg.z_m[l]);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

// ----------------------------------------------------------------------------
// Row transform: load in_len values of a row (zero-extend to n), transform,
// store the first out_len values.  One workgroup per row, row in LDS.
// ----------------------------------------------------------------------------
constexpr int kRowThreads = 256;

template <int DIR>
__global__ __launch_bounds__(kRowThreads) void k_row_fft(const float2 *__restrict__ in,
                                                         int in_len, long in_stride,
                                                         float2 *__restrict__ out,
                                                         int out_len, long out_stride,
                                                         FftPlan p,
                                                         const float2 *__restrict__ tw) {
  extern __shared__ float2 sbuf[];
  const int tid = threadIdx.x;
  const int n = p.n;
  const float2 *src = in + (size_t)blockIdx.x * in_stride;
  for (int i = tid; i < n; i += kRowThreads) sbuf[i] = i < in_len ? src[i] : make_float2(0.f, 0.f);
  __syncthreads();
  fft_lds<DIR, 1, kRowThreads, kMaxFft>(sbuf, p, tw, tid);
  float2 *dst = out + (size_t)blockIdx.x * out_stride;
  for (int i = tid; i < out_len; i += kRowThreads) dst[i] = sbuf[i];
}

hipError_t launch_row_fft(const Ctx &c, const float2 *in, int in_len, long in_stride,
                          float2 *out, int out_len, long out_stride, int rows, int inverse,
                          hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const size_t lds = (size_t)c.plan_x.n * sizeof(float2);
  if (inverse)
    hipLaunchKernelGGL(k_row_fft<+1>, dim3(rows), dim3(kRowThreads), lds, s, in, in_len,
                       in_stride, out, out_len, out_stride, c.plan_x, c.tw_x);
  else
    hipLaunchKernelGGL(k_row_fft<-1>, dim3(rows), dim3(kRowThreads), lds, s, in, in_len,
                       in_stride, out, out_len, out_stride, c.plan_x, c.tw_x);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Column pass: B adjacent columns of one channel.  Load H rows (zero-extend
// to Hp), FFT, multiply by H (or conj H) / (Hp Wp), IFFT, store H rows back in
// place.  The columns are disjoint between workgroups, so in place is safe.
// ----------------------------------------------------------------------------
constexpr int kColThreads = 1024;
constexpr int kColLdsElems = 19200;  // 150 KiB of float2

template <int B>
__global__ __launch_bounds__(kColThreads) void k_col_pass(float2 *__restrict__ data, int H,
                                                          int Wp, FftPlan py,
                                                          const float2 *__restrict__ tw,
                                                          const float2 *__restrict__ htab,
                                                          int Hq, int Wq, int L, int conj_h,
                                                          float scale) {
  constexpr int MAXN = kColLdsElems / B;
  __shared__ float2 sbuf[B * MAXN];
  const int tid = threadIdx.x;
  const int ch = blockIdx.y;
  const int col0 = blockIdx.x * B;
  const int Hp = py.n;
  float2 *base = data + (size_t)ch * H * Wp + col0;
  const int total = Hp * B;
  for (int i = tid; i < total; i += kColThreads) {
    const int r = i / B, b = i % B;
    float2 v = make_float2(0.f, 0.f);
    if (r < H && col0 + b < Wp) v = base[(size_t)r * Wp + b];
    sbuf[i] = v;
  }
  __syncthreads();
  fft_lds<-1, B, kColThreads, MAXN>(sbuf, py, tw, tid);
  const float2 *hc = htab + (size_t)ch * L * Hq * Wq;  // plane 0
  for (int i = tid; i < total; i += kColThreads) {
    const int r = i / B, b = i % B;
    const int kx = col0 + b;
    float2 v = make_float2(0.f, 0.f);
    if (kx < Wp) {
      const int qx = min(kx, Wp - kx), qy = min(r, Hp - r);
      float2 h = hc[(size_t)qy * Wq + qx];
      if (conj_h) h.y = -h.y;
      v = cscale(cmul(sbuf[i], h), scale);
    }
    sbuf[i] = v;
  }
  __syncthreads();
  fft_lds<+1, B, kColThreads, MAXN>(sbuf, py, tw, tid);
  const int keep = H * B;
  for (int i = tid; i < keep; i += kColThreads) {
    const int r = i / B, b = i % B;
    if (col0 + b < Wp) base[(size_t)r * Wp + b] = sbuf[i];
  }
}

static int col_batch(int Hp) {
  // widest column batch whose Hp x B block fits the LDS budget (B <= 16)
  for (int b : {16, 8, 4, 2})
    if (Hp * b <= kColLdsElems) return b;
  return 0;
}

hipError_t launch_col_pass(const Ctx &c, float2 *data, int conj_h, hipStream_t s) {
  const int B = col_batch(c.Hp);
  const float scale = (float)(1.0 / ((double)c.Hp * (double)c.Wp));
  dim3 grid((c.Wp + B - 1) / B, c.C);
  switch (B) {
    case 16:
      hipLaunchKernelGGL(k_col_pass<16>, grid, dim3(kColThreads), 0, s, data, c.H, c.Wp,
                         c.plan_y, c.tw_y, c.htab, c.Hq, c.Wq, c.L, conj_h, scale);
      break;
    case 8:
      hipLaunchKernelGGL(k_col_pass<8>, grid, dim3(kColThreads), 0, s, data, c.H, c.Wp,
                         c.plan_y, c.tw_y, c.htab, c.Hq, c.Wq, c.L, conj_h, scale);
      break;
    case 4:
      hipLaunchKernelGGL(k_col_pass<4>, grid, dim3(kColThreads), 0, s, data, c.H, c.Wp,
                         c.plan_y, c.tw_y, c.htab, c.Hq, c.Wq, c.L, conj_h, scale);
      break;
    default:
      hipLaunchKernelGGL(k_col_pass<2>, grid, dim3(kColThreads), 0, s, data, c.H, c.Wp,
                         c.plan_y, c.tw_y, c.htab, c.Hq, c.Wq, c.L, conj_h, scale);
      break;
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Middle row pass (F3): IFFT a row of the column-pass output, crop the first W
// values -> u, I = |u|^2 (optionally stored, with u), and if make_grad:
//   dL/dI = 2 (I - T) / M (MSE, Sec. 3.2) or the caller's dL/dI,
//   g = 2 dL/dI u = dL/dRe(u) + j dL/dIm(u),
// zero-extend g and FFT it back into the row (seed of the adjoint pass).
// Per-row FP64 partial sums of (I - T)^2 go to loss_part.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kRowThreads) void k_row_loss(
    float2 *__restrict__ data, int W, int Wp, FftPlan px, const float2 *__restrict__ tw,
    const float *__restrict__ target, const float *__restrict__ grad_I,
    float *__restrict__ intensity, float2 *__restrict__ u_out, double *__restrict__ loss_part,
    float gscale, int make_grad) {
  extern __shared__ float2 sbuf[];
  __shared__ double red[kRowThreads];
  const int tid = threadIdx.x;
  const size_t row = blockIdx.x;
  float2 *rp = data + row * Wp;
  for (int i = tid; i < Wp; i += kRowThreads) sbuf[i] = rp[i];
  __syncthreads();
  fft_lds<+1, 1, kRowThreads, kMaxFft>(sbuf, px, tw, tid);
  double acc = 0.0;
  for (int i = tid; i < Wp; i += kRowThreads) {
    if (i < W) {
      const float2 u = sbuf[i];
      const float I = u.x * u.x + u.y * u.y;
      const size_t o = row * W + i;
      if (intensity) intensity[o] = I;
      if (u_out) u_out[o] = u;
      if (make_grad) {
        float f;
        if (target) {
          const float d = I - target[o];
          acc += (double)d * (double)d;
          f = gscale * d;  // 4 (I - T) / M
        } else {
          f = 2.0f * grad_I[o];
        }
        sbuf[i] = make_float2(f * u.x, f * u.y);
      } else if (target) {
        const float d = I - target[o];
        acc += (double)d * (double)d;
      }
    } else if (make_grad) {
      sbuf[i] = make_float2(0.f, 0.f);
    }
  }
  if (target) {
    red[tid] = acc;
    __syncthreads();
    for (int w = kRowThreads / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) loss_part[row] = red[0];
  }
  if (make_grad) {
    __syncthreads();
    fft_lds<-1, 1, kRowThreads, kMaxFft>(sbuf, px, tw, tid);
    for (int i = tid; i < Wp; i += kRowThreads) rp[i] = sbuf[i];
  }
}

hipError_t launch_row_loss(const Ctx &c, float2 *data, const float *target,
                           const float *grad_intensity, float *intensity, float2 *u_out,
                           int make_grad, hipStream_t s) {
  const int rows = c.L * c.C * c.H;
  const double M = (double)c.L * c.C * c.H * c.W;
  const float gscale = (float)(4.0 / M);
  const size_t lds = (size_t)c.Wp * sizeof(float2);
  hipLaunchKernelGGL(k_row_loss, dim3(rows), dim3(kRowThreads), lds, s, data, c.W, c.Wp,
                     c.plan_x, c.tw_x, target, grad_intensity, intensity, u_out, c.loss_part,
                     gscale, make_grad);
  return hipGetLastError();
}

// loss = sum(loss_part) / M, psnr = 10 log10(1 / loss): one block, fixed order.
__global__ __launch_bounds__(256) void k_loss_finalize(const double *__restrict__ part,
                                                       int rows, double inv_m,
                                                       double *__restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < rows; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double loss = red[0] * inv_m;
    out[0] = loss;
    out[1] = 10.0 * log10(1.0 / loss);
  }
}

hipError_t launch_loss_finalize(const Ctx &c, double *loss, hipStream_t s) {
  const int rows = c.L * c.C * c.H;
  const double inv_m = 1.0 / ((double)c.L * c.C * c.H * c.W);
  hipLaunchKernelGGL(k_loss_finalize, dim3(1), dim3(256), 0, s, c.loss_part, rows, inv_m, loss);
  return hipGetLastError();
}

}  // namespace cgh
