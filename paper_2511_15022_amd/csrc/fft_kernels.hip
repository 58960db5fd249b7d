// Band-limited angular-spectrum propagation on gfx950: mixed-radix Stockham
// FFTs held in LDS, the transfer-function multiply fused into the column
// pass, and intensity / MSE / adjoint seed fused into the middle row pass.
//
// The propagation of one channel is u = crop(IFFT2(H . FFT2(pad(U0))))
// (Sec. 2; Alg. 1 ZeroPad + MultiPlanePropagate).  Because FFT2 -> H -> IFFT2
// is a circular convolution, padding the field at the start of each row and
// column (instead of centring it) and cropping the same leading window gives
// the same u; the kernels use that placement so the zero padding never exists
// in memory:
//   F1  row FFT:    U0 [C][H][W] -> S (rows zero-extended to Wp)
//   F2  column pass on S: FFT over Hp (zero-extended), x H/(Hp Wp), IFFT, keep H rows
//   F3  row pass:   IFFT, crop W -> u; I = |u|^2; loss; g = dL/du; zero-extend; FFT
//   B1  column pass with conj(H) (the adjoint, supplementary BLASM Backward Pass)
//   B2  row IFFT, crop W -> dL/dU0
// S is column-tiled: [C][ceil(Wp/8)][H][8] complex, so a column workgroup
// reads and writes one contiguous block and a row workgroup (two rows) moves
// whole 128-byte lines.
//
// Column pass for even Hp = 2M: the input occupies rows [0, H) and only rows
// [0, H) of the output are kept, so the Hp-point transform splits into two
// M-point chains (radix-2 first and last stages done in registers):
//   even chain: FFT_M(x[n] + x[n+M])             -> x H(ky = 2m)   -> IFFT_M -> e
//   odd chain:  FFT_M((x[n] - x[n+M]) w^n)       -> x H(ky = 2m+1) -> IFFT_M -> o
//   y[n] = e[n] + w^-n o[n],  y[n+M] = e[n] - w^-n o[n],   w = exp(-2 pi i / Hp)
// which halves the LDS footprint of a column block.
#include <cmath>

#include <type_traits>

#include "cgh_internal.h"
#include "fft_reg.h"

namespace cgh {

// ----------------------------------------------------------------------------
// Twiddles w^e = exp(-2 pi i e / n) from a two-level table kept in LDS:
// hi[j] = w^{64 j} (j <= n/64), lo[j] = w^j (j < 64); w^e = hi[e >> 6] lo[e & 63].
// The global copy of a table is kTwEntries float2: hi at [0, 129), lo at [129, 193).
// ----------------------------------------------------------------------------
constexpr int kTwHi = 129;
constexpr int kTwEntries = kTwHi + 64;

struct TwLds {
  float2 hi[kTwHi];
  float2 lo[64];
};

// Element i of an array at a wave-uniform base, addressed with a 32-bit byte
// offset (so the access takes the scalar-base form, with no 64-bit address add).
template <class T>
__device__ __forceinline__ T &at32(T *base, uint32_t i) {
  return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ const T &at32(const T *base, uint32_t i) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                      i * (uint32_t)sizeof(T));
}

__device__ __forceinline__ float2 tw_at(const TwLds &t, int e) {
  return cmul(t.hi[e >> 6], t.lo[e & 63]);
}

template <int T>
__device__ __forceinline__ void load_tw(TwLds &dst, const float2 *__restrict__ src, int tid) {
  for (int i = tid; i < kTwEntries; i += T) {
    if (i < kTwHi) dst.hi[i] = src[i];
    else dst.lo[i - kTwHi] = src[i];
  }
}

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
                                          uint32_t magic, int tws, const TwLds &tw,
                                          int tid) {
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
        float2 w1 = tw_at(tw, (j - grp * Ns) * tws);
        if (DIR > 0) w1.y = -w1.y;
        float2 w = w1;
        v[it][1] = cmul(v[it][1], w);
#pragma unroll
        for (int q = 2; q < R; ++q) {
          w = cmul(w, w1);
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
__device__ void fft_lds(float2 *__restrict__ buf, const FftPlan &p, const TwLds &tw, int tid) {
  for (int s = 0; s < p.nstages; ++s) {
    const int r = p.radix[s];
    // An opaque per-stage copy of the thread index: without it the compiler
    // hoists every radix variant's per-butterfly index math out of this loop
    // and keeps it all live (about 2x the registers).
    int ts = tid;
    asm volatile("" : "+v"(ts));
    if (r == 8)
      fft_stage<8, DIR, B, T, MAXN>(buf, p.n, p.ns[s], p.magic[s], p.tws[s], tw, ts);
    else if (r == 4)
      fft_stage<4, DIR, B, T, MAXN>(buf, p.n, p.ns[s], p.magic[s], p.tws[s], tw, ts);
    else if (r == 3)
      fft_stage<3, DIR, B, T, MAXN>(buf, p.n, p.ns[s], p.magic[s], p.tws[s], tw, ts);
    else if (r == 5)
      fft_stage<5, DIR, B, T, MAXN>(buf, p.n, p.ns[s], p.magic[s], p.tws[s], tw, ts);
    else
      fft_stage<2, DIR, B, T, MAXN>(buf, p.n, p.ns[s], p.magic[s], p.tws[s], tw, ts);
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
  while (twos >= 3 && twos != 4) { rad[ns++] = 8; twos -= 3; }
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

bool col_supported(int Hp) {
  if (Hp % 2 == 0) return Hp / 2 <= kColHalfMax;
  return Hp <= kColFullMax;
}

// ----------------------------------------------------------------------------
// Tables (FP64 on the device, rounded to FP32 once)
// ----------------------------------------------------------------------------
__global__ void k_twiddles(float2 *tw, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kTwEntries) return;
  const long e = j < kTwHi ? (64L * j) % n : (long)(j - kTwHi) % n;
  double s, c;
  sincospi(2.0 * (double)e / (double)n, &s, &c);
  tw[j] = make_float2((float)c, (float)(-s));  // exp(-2 pi i e / n)
}

hipError_t launch_build_twiddles(float2 *tw, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles, dim3(1), dim3(256), 0, s, tw, n);
  return hipGetLastError();
}

// full table tw[e] = exp(-2 pi i e / n), e < n
__global__ void k_twiddles_full(float2 *tw, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double s, c;
  sincospi(2.0 * (double)e / (double)n, &s, &c);
  tw[e] = make_float2((float)c, (float)(-s));
}

hipError_t launch_build_twiddles_full(float2 *tw, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles_full, dim3((n + 255) / 256), dim3(256), 0, s, tw, n);
  return hipGetLastError();
}

// Band-limited angular-spectrum transfer function (Sec. 2; supplementary
// "Spatial Frequency Computation", "Bandlimit Computation", "Transfer Function
// Evaluation"), quarter table indexed by |fx| = qx / (Wp dx), |fy| = qy / (Hp dx).
// L_x, L_y are the extents of the padded grid.  Evanescent frequencies get 0.
// out_t (optional) receives the same table column-major, [Wq][Hq], times
// t_scale (the 1 / (Hp Wp) of the inverse transform, applied in FP64).
// aperture > 0: the circular aperture of Alg. 3, centred on the zero frequency
// (bins with qx^2 + qy^2 >= aperture^2 are zeroed).
__global__ void k_transfer(float2 *out, float2 *out_t, double t_scale, int Hq, int Wq, int Hp,
                           int Wp, double pitch, double lambda, double z, double aperture) {
  int qx = blockIdx.x * blockDim.x + threadIdx.x;
  int qy = blockIdx.y;
  if (qx >= Wq) return;
  const double Lx = Wp * pitch, Ly = Hp * pitch;
  const double fx = qx / Lx, fy = qy / Ly;
  const double ax = 2.0 * z / Lx, ay = 2.0 * z / Ly;
  const double fxmax = 1.0 / (lambda * sqrt(ax * ax + 1.0));
  const double fymax = 1.0 / (lambda * sqrt(ay * ay + 1.0));
  const double arg = 1.0 / (lambda * lambda) - fx * fx - fy * fy;
  double sn = 0.0, cs = 0.0;
  const bool open = aperture <= 0.0 || (double)qx * qx + (double)qy * qy < aperture * aperture;
  if (fx < fxmax && fy < fymax && arg >= 0.0 && open) {
    const double ph = 6.283185307179586476925 * z * sqrt(arg);  // 2 pi z sqrt(arg)
    sincos(ph, &sn, &cs);
  }
  out[(size_t)qy * Wq + qx] = make_float2((float)cs, (float)sn);
  if (out_t)
    out_t[(size_t)qx * Hq + qy] = make_float2((float)(cs * t_scale), (float)(sn * t_scale));
}

hipError_t launch_build_transfer(const Ctx &c, int b0, int b1, hipStream_t s) {
  for (int b = b0; b < b1; ++b)
    for (int ch = 0; ch < c.C; ++ch)
      for (int l = 0; l < c.L; ++l) {
        // propagation channel b C + ch: colour ch of hologram b
        const size_t at = (((size_t)b * c.C + ch) * c.L + l) * c.Hq * c.Wq;
        hipLaunchKernelGGL(k_transfer, dim3((c.Wq + 255) / 256, c.Hq), dim3(256), 0, s,
                           c.htab + at, c.htab_t ? c.htab_t + at : nullptr,
                           1.0 / ((double)c.Hp * (double)c.Wp), c.Hq, c.Wq, c.Hp, c.Wp,
                           c.cfg.pitch_m, c.lam[b][ch], c.zd[b][l], c.cfg.aperture);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
  return hipSuccess;
}

// ----------------------------------------------------------------------------
// Row passes: two rows (y0, y0+1) of one channel per workgroup, interleaved in
// LDS as element (x, b) at sbuf[2 x + b].  Column-tiled global layout:
//   S[c][x / 8][y][x % 8]
// so sixteen consecutive threads move one 128-byte line (rows y0, y0+1 of a tile).
// ----------------------------------------------------------------------------
constexpr int kRowThreads = 512;

__device__ __forceinline__ size_t tiled(int c, int y, int x, int H, int Wt) {
  return (((size_t)c * Wt + (x >> 3)) * H + y) * 8 + (x & 7);
}

// Global -> LDS copy of n elements with G loads in flight per thread: every load
// of a group is issued (at a clamped, always valid index) before the first one
// is stored, so their latencies overlap instead of adding up.  ld(i) must be
// callable for every 0 <= i < n; st(i, v) stores element i.
template <int T, int G, class LD, class ST>
__device__ __forceinline__ void staged_copy(int n, int tid, LD ld, ST st) {
  for (int i0 = tid; i0 < n; i0 += T * G) {
    float2 v[G];
#pragma unroll
    for (int g = 0; g < G; ++g) v[g] = ld(min(i0 + g * T, n - 1));
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (i0 + g * T < n) st(i0 + g * T, v[g]);
  }
}

// row b (< ROWS) and column x of element i of ROWS consecutive rows of length w
template <int ROWS>
__device__ __forceinline__ int row_of(int i, int w) {
  int b = 0;
#pragma unroll
  for (int r = 1; r < ROWS; ++r) b += i >= r * w;
  return b;
}

// load the two rows of S into LDS (zero beyond Wp or H)
__device__ __forceinline__ void load_rows_tiled(float2 *sbuf, const float2 *__restrict__ S,
                                                int c, int y0, int H, int Wp, int Wt,
                                                int tid) {
  staged_copy<kRowThreads, 8>(
      Wt * 16, tid,
      [&](int i) {
        const int b = (i >> 3) & 1, x = (i >> 4) * 8 + (i & 7);
        const float2 v = S[tiled(c, min(y0 + b, H - 1), x, H, Wt)];
        return y0 + b < H ? v : make_float2(0.f, 0.f);
      },
      [&](int i, float2 v) {
        const int b = (i >> 3) & 1, x = (i >> 4) * 8 + (i & 7);
        if (x < Wp) sbuf[2 * x + b] = v;
      });
}

// rows y0, y0+1 of the field, zero-extended to n, into LDS (interleaved)
__device__ __forceinline__ void load_field_rows(float2 *sbuf, const float2 *__restrict__ field,
                                                int c, int y0, int H, int W, int n, int tid) {
  staged_copy<kRowThreads, 8>(
      2 * W, tid,
      [&](int i) {
        const int b = row_of<2>(i, W), x = i - b * W;
        const float2 v = field[((size_t)c * H + min(y0 + b, H - 1)) * W + x];
        return y0 + b < H ? v : make_float2(0.f, 0.f);
      },
      [&](int i, float2 v) {
        const int b = row_of<2>(i, W), x = i - b * W;
        sbuf[2 * x + b] = v;
      });
  for (int i = tid; i < 2 * (n - W); i += kRowThreads) sbuf[2 * W + i] = make_float2(0.f, 0.f);
}

__device__ __forceinline__ void store_rows_tiled(const float2 *sbuf, float2 *__restrict__ S,
                                                 int c, int y0, int H, int Wp, int Wt,
                                                 int tid) {
  for (int i = tid; i < Wt * 16; i += kRowThreads) {
    const int t = i >> 4, b = (i >> 3) & 1, x = t * 8 + (i & 7);
    if (x < Wp && y0 + b < H) S[tiled(c, y0 + b, x, H, Wt)] = sbuf[2 * x + b];
  }
}

// F1: field rows (zero-extended to Wp) -> forward FFT -> S
template <int MAXN>
__global__ __launch_bounds__(kRowThreads) void k_row_fwd(const float2 *__restrict__ field,
                                                         int H, int W, int Wt, FftPlan p,
                                                         const float2 *__restrict__ twx,
                                                         float2 *__restrict__ S) {
  extern __shared__ float2 sbuf[];
  __shared__ TwLds tw;
  const int tid = threadIdx.x, n = p.n;
  const int pairs = (H + 1) >> 1;
  const int c = blockIdx.x / pairs, y0 = 2 * (blockIdx.x % pairs);
  load_tw<kRowThreads>(tw, twx, tid);
  load_field_rows(sbuf, field, c, y0, H, W, n, tid);
  __syncthreads();
  fft_lds<-1, 2, kRowThreads, MAXN>(sbuf, p, tw, tid);
  store_rows_tiled(sbuf, S, c, y0, H, n, Wt, tid);
}

// B2: S -> inverse FFT -> first W values of each row -> grad field
template <int MAXN>
__global__ __launch_bounds__(kRowThreads) void k_row_inv(const float2 *__restrict__ S, int H,
                                                         int W, int Wt, FftPlan p,
                                                         const float2 *__restrict__ twx,
                                                         float2 *__restrict__ out) {
  extern __shared__ float2 sbuf[];
  __shared__ TwLds tw;
  const int tid = threadIdx.x, n = p.n;
  const int pairs = (H + 1) >> 1;
  const int c = blockIdx.x / pairs, y0 = 2 * (blockIdx.x % pairs);
  load_tw<kRowThreads>(tw, twx, tid);
  load_rows_tiled(sbuf, S, c, y0, H, n, Wt, tid);
  __syncthreads();
  fft_lds<+1, 2, kRowThreads, MAXN>(sbuf, p, tw, tid);
  for (int b = 0; b < 2; ++b) {
    if (y0 + b >= H) break;
    float2 *dst = out + ((size_t)c * H + y0 + b) * W;
    for (int x = tid; x < W; x += kRowThreads) dst[x] = sbuf[2 * x + b];
  }
}

// F3: S -> inverse FFT -> u (first W values) -> I = |u|^2 (optionally stored,
// with u); if make_grad: dL/dI = 2 (I - T) / M (MSE, Sec. 3.2) or the caller's
// dL/dI, g = 2 dL/dI u = dL/dRe(u) + j dL/dIm(u), zero-extended, forward FFT,
// back into S.  FP64 partial sums of (I - T)^2 per workgroup into loss_part.
template <int MAXN>
__global__ __launch_bounds__(kRowThreads) void k_row_loss(
    float2 *__restrict__ S, int H, int W, int Wt, FftPlan p, const float2 *__restrict__ twx,
    const float *__restrict__ target, const float *__restrict__ grad_I,
    const float *__restrict__ mask, int mcg, float *__restrict__ intensity, float2 *__restrict__ u_out,
    double *__restrict__ loss_part, float gscale, int make_grad) {
  extern __shared__ float2 sbuf[];
  __shared__ TwLds tw;
  __shared__ double red[kRowThreads / 64];
  const int tid = threadIdx.x, n = p.n;
  const int pairs = (H + 1) >> 1;
  const int c = blockIdx.x / pairs, y0 = 2 * (blockIdx.x % pairs);
  load_tw<kRowThreads>(tw, twx, tid);
  if (mask) mask += (size_t)(c / mcg) * H * W;
  load_rows_tiled(sbuf, S, c, y0, H, n, Wt, tid);
  __syncthreads();
  fft_lds<+1, 2, kRowThreads, MAXN>(sbuf, p, tw, tid);
  double acc = 0.0;
  for (int i = tid; i < 2 * n; i += kRowThreads) {
    const int b = i >= n, x = i - b * n;
    const int y = y0 + b;
    if (x < W && y < H) {
      const float2 u = sbuf[2 * x + b];
      const float I = u.x * u.x + u.y * u.y;
      const size_t o = ((size_t)c * H + y) * W + x;
      if (intensity) intensity[o] = I;
      if (u_out) u_out[o] = u;
      float f = 0.f;
      if (target) {
        const float t = target[o], d = I - t;
        // L_recon weight 1 + m^2 + t^2 (plain MSE without a mask)
        const float w = mask ? 1.f + mask[(size_t)y * W + x] * mask[(size_t)y * W + x] + t * t
                             : 1.f;
        acc += (double)d * (double)d * (double)w;
        f = gscale * d * w;  // 4 w (I - T) / M
      } else if (grad_I) {
        f = 2.0f * grad_I[o];
      }
      if (make_grad) sbuf[2 * x + b] = make_float2(f * u.x, f * u.y);
    } else if (make_grad) {
      sbuf[2 * x + b] = make_float2(0.f, 0.f);
    }
  }
  if (target) {
    // wave sums, then a fixed-order sum over the waves
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_down(acc, d, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < kRowThreads / 64; ++w) s += red[w];
      loss_part[blockIdx.x] = s;
    }
  }
  if (make_grad) {
    __syncthreads();
    fft_lds<-1, 2, kRowThreads, MAXN>(sbuf, p, tw, tid);
    store_rows_tiled(sbuf, S, c, y0, H, n, Wt, tid);
  }
}

// ----------------------------------------------------------------------------
// Size-specialised row passes: compile-time plan (three large-radix stages for
// the workload lengths), ROWS rows per workgroup, full twiddle table in LDS.
// ----------------------------------------------------------------------------
template <int N, int ROWS, int T>
__device__ __forceinline__ void load_rows_c(float2 *sbuf, const float2 *__restrict__ S, int c,
                                            int y0, int H, int Wt, int tid) {
  constexpr int NT = (N + 7) / 8 * 8 * ROWS, G = (NT + T - 1) / T;
  staged_copy<T, G>(
      Wt * 8 * ROWS, tid,
      [&](int i) {
        const int t = i / (8 * ROWS), r = i % (8 * ROWS), b = r >> 3, x = t * 8 + (r & 7);
        const float2 v = S[tiled(c, min(y0 + b, H - 1), x, H, Wt)];
        return y0 + b < H ? v : make_float2(0.f, 0.f);
      },
      [&](int i, float2 v) {
        const int t = i / (8 * ROWS), r = i % (8 * ROWS), b = r >> 3, x = t * 8 + (r & 7);
        if (x < N) sbuf[ROWS * x + b] = v;
      });
}

template <int N, int ROWS, int T>
__device__ __forceinline__ void store_rows_c(const float2 *sbuf, float2 *__restrict__ S, int c,
                                             int y0, int H, int Wt, int tid) {
  for (int i = tid; i < Wt * 8 * ROWS; i += T) {
    const int t = i / (8 * ROWS), r = i % (8 * ROWS), b = r >> 3, x = t * 8 + (r & 7);
    if (x < N && y0 + b < H) S[tiled(c, y0 + b, x, H, Wt)] = sbuf[ROWS * x + b];
  }
}

template <int N, int T>
__device__ __forceinline__ void load_table(float2 *tw, const float2 *__restrict__ src, int tid) {
  for (int i = tid; i < N; i += T) tw[i] = src[i];
}

// Twiddles of a specialised row pass: the full length-N table when it fits in
// LDS beside the rows (FULL), otherwise the two-level table.
template <int N, bool FULL>
struct RowTw;
template <int N>
struct RowTw<N, true> {
  float2 t[N];
  template <int T>
  __device__ __forceinline__ void load(const float2 *full, const float2 *, int tid) { load_table<N, T>(t, full, tid); }
  template <int DIR, int B, int T>
  __device__ __forceinline__ void fft(float2 *buf, int tid) const { cfft<DIR, B, T, N>(buf, t, tid); }
};
template <int N>
struct RowTw<N, false> {
  TwLds t;
  template <int T>
  __device__ __forceinline__ void load(const float2 *, const float2 *two, int tid) { load_tw<T>(t, two, tid); }
  template <int DIR, int B, int T>
  __device__ __forceinline__ void fft(float2 *buf, int tid) const { cfft2<DIR, B, T, N>(buf, t, tid); }
};

template <int N, int ROWS, int T, bool FULL>
__global__ __launch_bounds__(T) void k_row_fwd_c(const float2 *__restrict__ field, int H, int W,
                                                 int Wt, const float2 *__restrict__ twf,
                                                 const float2 *__restrict__ tw2,
                                                 float2 *__restrict__ S) {
  __shared__ float2 sbuf[ROWS * N];
  __shared__ RowTw<N, FULL> tw;
  const int tid = threadIdx.x;
  const int groups = (H + ROWS - 1) / ROWS;
  const int c = blockIdx.x / groups, y0 = ROWS * (blockIdx.x % groups);
  tw.template load<T>(twf, tw2, tid);
  staged_copy<T, (ROWS * N + T - 1) / T>(
      ROWS * W, tid,
      [&](int i) {
        const int b = row_of<ROWS>(i, W), x = i - b * W;
        const float2 v = field[((size_t)c * H + min(y0 + b, H - 1)) * W + x];
        return y0 + b < H ? v : make_float2(0.f, 0.f);
      },
      [&](int i, float2 v) {
        const int b = row_of<ROWS>(i, W), x = i - b * W;
        sbuf[ROWS * x + b] = v;
      });
  for (int i = tid; i < ROWS * (N - W); i += T) sbuf[ROWS * W + i] = make_float2(0.f, 0.f);
  __syncthreads();
  tw.template fft<-1, ROWS, T>(sbuf, tid);
  store_rows_c<N, ROWS, T>(sbuf, S, c, y0, H, Wt, tid);
}

template <int N, int ROWS, int T, bool FULL>
__global__ __launch_bounds__(T) void k_row_inv_c(const float2 *__restrict__ S, int H, int W,
                                                 int Wt, const float2 *__restrict__ twf,
                                                 const float2 *__restrict__ tw2,
                                                 float2 *__restrict__ out) {
  __shared__ float2 sbuf[ROWS * N];
  __shared__ RowTw<N, FULL> tw;
  const int tid = threadIdx.x;
  const int groups = (H + ROWS - 1) / ROWS;
  const int c = blockIdx.x / groups, y0 = ROWS * (blockIdx.x % groups);
  tw.template load<T>(twf, tw2, tid);
  load_rows_c<N, ROWS, T>(sbuf, S, c, y0, H, Wt, tid);
  __syncthreads();
  tw.template fft<+1, ROWS, T>(sbuf, tid);
  for (int b = 0; b < ROWS; ++b) {
    if (y0 + b >= H) break;
    float2 *dst = out + ((size_t)c * H + y0 + b) * W;
    for (int x = tid; x < W; x += T) dst[x] = sbuf[ROWS * x + b];
  }
}

template <int N, int ROWS, int T, bool FULL>
__global__ __launch_bounds__(T) void k_row_loss_c(
    float2 *__restrict__ S, int H, int W, int Wt, const float2 *__restrict__ twf,
    const float2 *__restrict__ tw2, const float *__restrict__ target,
    const float *__restrict__ grad_I, const float *__restrict__ mask, int mcg,
    float *__restrict__ intensity, float2 *__restrict__ u_out, double *__restrict__ loss_part,
    float gscale, int make_grad) {
  __shared__ float2 sbuf[ROWS * N];
  __shared__ RowTw<N, FULL> tw;
  __shared__ double red[T / 64];
  constexpr int KT = (ROWS * N + T - 1) / T;  // cropped elements per thread (W <= N)
  const int tid = threadIdx.x;
  const int groups = (H + ROWS - 1) / ROWS;
  const int c = blockIdx.x / groups, y0 = ROWS * (blockIdx.x % groups);
  const int nw = ROWS * W;  // element i: row y0 + i / W, column i % W
  if (mask) mask += (size_t)(c / mcg) * H * W;
  tw.template load<T>(twf, tw2, tid);
  load_rows_c<N, ROWS, T>(sbuf, S, c, y0, H, Wt, tid);
  // the target (or the caller's dL/dI) of this thread's elements, fetched
  // before the transform (whose barriers do not wait for global loads) so
  // that the loads overlap it
  const float *tsrc = target ? target : grad_I;
  float tv[KT], mv[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int i = min(tid + k * T, nw - 1);
    const int b = row_of<ROWS>(i, W), x = i - b * W, y = min(y0 + b, H - 1);
    tv[k] = tsrc ? tsrc[((size_t)c * H + y) * W + x] : 0.f;
    mv[k] = mask ? mask[(size_t)y * W + x] : 0.f;
  }
  lds_sync();
  tw.template fft<+1, ROWS, T>(sbuf, tid);
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int i = tid + k * T;
    if (i < nw) {
      const int b = row_of<ROWS>(i, W), x = i - b * W, y = y0 + b;
      if (y < H) {
        const float2 u = sbuf[ROWS * x + b];
        const float I = u.x * u.x + u.y * u.y;
        const size_t o = ((size_t)c * H + y) * W + x;
        if (intensity) intensity[o] = I;
        if (u_out) u_out[o] = u;
        float f = 0.f;
        if (target) {
          // L_recon weight 1 + m^2 + t^2 (plain MSE without a mask)
          const float d = I - tv[k], w = mask ? 1.f + mv[k] * mv[k] + tv[k] * tv[k] : 1.f;
          acc += (double)d * (double)d * (double)w;
          f = gscale * d * w;  // 4 w (I - T) / M
        } else if (grad_I) {
          f = 2.0f * tv[k];
        }
        if (make_grad) sbuf[ROWS * x + b] = make_float2(f * u.x, f * u.y);
      } else if (make_grad) {
        sbuf[ROWS * x + b] = make_float2(0.f, 0.f);
      }
    }
  }
  if (make_grad)
    for (int i = tid; i < ROWS * (N - W); i += T) sbuf[ROWS * W + i] = make_float2(0.f, 0.f);
  if (target) {
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_down(acc, d, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
      for (int w = 0; w < T / 64; ++w) sum += red[w];
      loss_part[blockIdx.x] = sum;
    }
  }
  if (make_grad) {
    __syncthreads();
    tw.template fft<-1, ROWS, T>(sbuf, tid);
    store_rows_c<N, ROWS, T>(sbuf, S, c, y0, H, Wt, tid);
  }
}

// ----------------------------------------------------------------------------
// Quarter-length row passes, for Wp = 4M with W <= 2M (7680: M = 1920).  With
// the samples at n < 2M, bin 4m + p of the forward is FFT_M of
// w^{pn}(x[n] + (-i)^p x[n + M]) (n < M), and the inverse cropped to n < 2M is
// u[n + M j] = sum_p w^{-pn} i^{pj} z_p[n] for j = 0, 1, with z_p the M-point
// inverse of bins p mod 4 (w = exp(-2 pi i / Wp)).  A 512-thread workgroup
// takes one row: four interleaved M-point chains, chain p at buf[4 m + p],
// which is the row in natural bin order.  Blocks b and b + 8, which run on one
// XCD, take rows 2k and 2k + 1, so the two halves of each 128-byte line of the
// column-tiled spectrum meet in one L2.
// ----------------------------------------------------------------------------
__device__ __forceinline__ int quarter_row(int b, int rows) {
  if (b >= (rows & ~15)) return b;
  return (b & ~15) + 2 * (b & 7) + ((b >> 3) & 1);
}

// M-entry table exp(-2 pi i e / M) (every fourth entry of the Wp = 4 M table),
// stored contiguously after that table
template <int M, int T>
__device__ __forceinline__ void load_quarter_table(float2 *tw, const float2 *__restrict__ twf_x,
                                                   int tid) {
  constexpr int KT = (M + T - 1) / T;
  float2 tv[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) tv[k] = at32(twf_x, 4 * M + min(tid + k * T, M - 1));
#pragma unroll
  for (int k = 0; k < KT; ++k)
    if (KT * T == M || tid + k * T < M) tw[tid + k * T] = tv[k];
}

// one row y of channel base Sc (column-tiled [Wp / 8][H][8]) <-> buf in natural order
template <int M, int T>
__device__ __forceinline__ void load_quarter_row(float2 *buf, const float2 *Sc, int H, int y,
                                                 int tid) {
  constexpr int n = 4 * M, K = (n + T - 1) / T;
  float2 v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int x = min(tid + k * T, n - 1);
    v[k] = at32(Sc, ((x >> 3) * H + y) * 8 + (x & 7));
  }
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (K * T == n || tid + k * T < n) buf[tid + k * T] = v[k];
}

template <int M, int T>
__device__ __forceinline__ void store_quarter_row(const float2 *buf, float2 *Sc, int H, int y,
                                                  int tid) {
  constexpr int n = 4 * M, K = (n + T - 1) / T;
  float2 v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = buf[min(tid + k * T, n - 1)];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int x = tid + k * T;
    if (K * T == n || x < n) at32(Sc, ((x >> 3) * H + y) * 8 + (x & 7)) = v[k];
  }
}

// the four chain inputs at m = n from the samples a = x[n], b = x[n + M]
__device__ __forceinline__ void quarter_inputs(float2 *buf, int n, float2 a, float2 b,
                                               float2 w1) {
  const float2 w2 = cmul(w1, w1), w3 = cmul(w2, w1);
  buf[4 * n] = cadd(a, b);
  buf[4 * n + 1] = cmul(make_float2(a.x + b.y, a.y - b.x), w1);  // (a - i b) w^n
  buf[4 * n + 2] = cmul(csub(a, b), w2);                         // (a - b) w^{2n}
  buf[4 * n + 3] = cmul(make_float2(a.x - b.y, a.y + b.x), w3);  // (a + i b) w^{3n}
}

// u[n] and u[n + M] from the four chain outputs at m = n
__device__ __forceinline__ void quarter_outputs(const float2 *buf, int n, float2 w1, float2 &u0,
                                                float2 &u1) {
  const float2 w2 = cmul(w1, w1), w3 = cmul(w2, w1);
  const float2 z0 = buf[4 * n];
  const float2 z1 = cmul(cconj(w1), buf[4 * n + 1]);
  const float2 z2 = cmul(cconj(w2), buf[4 * n + 2]);
  const float2 z3 = cmul(cconj(w3), buf[4 * n + 3]);
  u0 = cadd(cadd(z0, z1), cadd(z2, z3));
  const float2 e = csub(z0, z2), o = csub(z1, z3);
  u1 = make_float2(e.x - o.y, e.y + o.x);  // z0 + i z1 - z2 - i z3
}

template <int M>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_row_fwd_q(
    const float2 *__restrict__ field, int H, int W, int rows, const float2 *__restrict__ twf_x,
    float2 *__restrict__ S) {
  constexpr int T = 512, K = (M + T - 1) / T, Wt = M / 2;
  __shared__ float2 buf[4 * M];
  __shared__ float2 tw[M];
  const int tid = threadIdx.x;
  const int R = quarter_row(blockIdx.x, rows), c = R / H, y = R - c * H;
  load_quarter_table<M, T>(tw, twf_x, tid);
  {
    const float2 *f = field + ((size_t)c * H + y) * W;
    float2 av[K], bv[K], wv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int n = min(tid + k * T, M - 1);
      av[k] = at32(f, min(n, W - 1));
      bv[k] = at32(f, min(n + M, W - 1));
      wv[k] = at32(twf_x, n);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int n = tid + k * T;
      if (K * T == M || n < M) {
        const float2 a = n < W ? av[k] : make_float2(0.f, 0.f);
        const float2 b = n + M < W ? bv[k] : make_float2(0.f, 0.f);
        quarter_inputs(buf, n, a, b, wv[k]);
      }
    }
  }
  __syncthreads();
  cfft<-1, 4, T, M>(buf, tw, tid);
  store_quarter_row<M, T>(buf, S + (size_t)c * Wt * H * 8, H, y, tid);
}

template <int M>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_row_inv_q(
    const float2 *__restrict__ S, int H, int W, int rows, const float2 *__restrict__ twf_x,
    float2 *__restrict__ out) {
  constexpr int T = 512, K = (M + T - 1) / T, Wt = M / 2;
  __shared__ float2 buf[4 * M];
  __shared__ float2 tw[M];
  const int tid = threadIdx.x;
  const int R = quarter_row(blockIdx.x, rows), c = R / H, y = R - c * H;
  load_quarter_table<M, T>(tw, twf_x, tid);
  load_quarter_row<M, T>(buf, S + (size_t)c * Wt * H * 8, H, y, tid);
  float2 wv[K];
#pragma unroll
  for (int k = 0; k < K; ++k) wv[k] = at32(twf_x, min(tid + k * T, M - 1));
  lds_sync();
  cfft<+1, 4, T, M>(buf, tw, tid);
  float2 *o = out + ((size_t)c * H + y) * W;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int n = tid + k * T;
    if ((K * T == M || n < M) && n < W) {
      float2 u0, u1;
      quarter_outputs(buf, n, wv[k], u0, u1);
      o[n] = u0;
      if (n + M < W) o[n + M] = u1;
    }
  }
}

template <int M>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_row_loss_q(
    float2 *__restrict__ S, int H, int W, int rows, const float2 *__restrict__ twf_x,
    const float *__restrict__ target, const float *__restrict__ grad_I,
    const float *__restrict__ mask, int mcg, float *__restrict__ intensity, float2 *__restrict__ u_out,
    double *__restrict__ loss_part, float gscale, int make_grad) {
  constexpr int T = 512, K = (M + T - 1) / T, Wt = M / 2;
  __shared__ float2 buf[4 * M];
  __shared__ float2 tw[M];
  __shared__ double red[T / 64];
  const int tid = threadIdx.x;
  const int R = quarter_row(blockIdx.x, rows), c = R / H, y = R - c * H;
  float2 *Sc = S + (size_t)c * Wt * H * 8;
  load_quarter_table<M, T>(tw, twf_x, tid);
  load_quarter_row<M, T>(buf, Sc, H, y, tid);
  if (mask) mask += (size_t)(c / mcg) * H * W;
  // per-element inputs at n and n + M, fetched before the transform so that
  // their latency overlaps it
  const float *tsrc = target ? target : grad_I;
  const size_t row = ((size_t)c * H + y) * W;
  float tv0[K], tv1[K], mv0[K], mv1[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int n = min(tid + k * T, M - 1);
    const int n0 = min(n, W - 1), n1 = min(n + M, W - 1);
    tv0[k] = tsrc ? tsrc[row + n0] : 0.f;
    tv1[k] = tsrc ? tsrc[row + n1] : 0.f;
    mv0[k] = mask ? mask[(size_t)y * W + n0] : 0.f;
    mv1[k] = mask ? mask[(size_t)y * W + n1] : 0.f;
  }
  lds_sync();
  cfft<+1, 4, T, M>(buf, tw, tid);
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int n = tid + k * T;
    if (K * T == M || n < M) {
      const float2 w1 = at32(twf_x, n);
      float2 u[2];
      quarter_outputs(buf, n, w1, u[0], u[1]);
      float f[2] = {0.f, 0.f};
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int x = n + j * M;
        if (x >= W) continue;
        const float t = j ? tv1[k] : tv0[k], m = j ? mv1[k] : mv0[k];
        const float I = u[j].x * u[j].x + u[j].y * u[j].y;
        if (intensity) intensity[row + x] = I;
        if (u_out) u_out[row + x] = u[j];
        if (target) {
          // L_recon weight 1 + m^2 + t^2 (plain MSE without a mask)
          const float d = I - t, w = mask ? 1.f + m * m + t * t : 1.f;
          acc += (double)d * (double)d * (double)w;
          f[j] = gscale * d * w;  // 4 w (I - T) / M
        } else if (grad_I) {
          f[j] = 2.0f * t;
        }
      }
      if (make_grad)
        quarter_inputs(buf, n, make_float2(f[0] * u[0].x, f[0] * u[0].y),
                       make_float2(f[1] * u[1].x, f[1] * u[1].y), w1);
    }
  }
  if (target) {
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_down(acc, d, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
      for (int w = 0; w < T / 64; ++w) sum += red[w];
      loss_part[R] = sum;
    }
  }
  if (make_grad) {
    __syncthreads();
    cfft<-1, 4, T, M>(buf, tw, tid);
    store_quarter_row<M, T>(buf, Sc, H, y, tid);
  }
}

// rows per row-pass workgroup (specialised lengths use 4, the runtime path 2)
static bool row_specialised(int Wp) { return Wp == 3840 || Wp == 512; }
// the half-length row passes take Wp = 3840 (1080p) and 7680 (4K) with W <= Wp / 2
// the quarter-length row passes take Wp = 4 M with W <= Wp / 2, one row per workgroup,
// for the chain lengths they are built for (4K: 1920; 1080p: 960; 1024 .. 4096 pads:
// 256, 512, 1024);
// quarter_m returns M, or 0 where they do not apply
static int quarter_m(const Ctx &c) {
  if (c.Wp % 4 != 0 || 2 * c.W > c.Wp) return 0;
  const int M = c.Wp / 4;
  return (M == 1920 || M == 1024 || M == 960 || M == 512 || M == 256) ? M : 0;
}
static bool row_quarter(const Ctx &c) { return quarter_m(c) != 0; }
// calls f(std::integral_constant<int, M>) for the quarter length of c
template <class F>
static void with_quarter(const Ctx &c, F &&f) {
  switch (quarter_m(c)) {
    case 1920: f(std::integral_constant<int, 1920>{}); break;
    case 1024: f(std::integral_constant<int, 1024>{}); break;
    case 960: f(std::integral_constant<int, 960>{}); break;
    case 512: f(std::integral_constant<int, 512>{}); break;
    default: f(std::integral_constant<int, 256>{}); break;
  }
}
int row_group_rows(const Ctx &c) {
  return c.Wp == 512 ? 4 : (row_quarter(c) ? 1 : 2);
}
static int row_blocks(const Ctx &c) {
  const int r = row_group_rows(c);
  return c.CF * ((c.H + r - 1) / r);
}
static size_t row_lds(const Ctx &c) { return (size_t)2 * c.Wp * sizeof(float2); }

hipError_t launch_row_fwd(const Ctx &c, const float2 *field, float2 *dst, hipStream_t s) {
  if (row_quarter(c))
    with_quarter(c, [&](auto mc) {
      hipLaunchKernelGGL(k_row_fwd_q<decltype(mc)::value>, dim3(row_blocks(c)), dim3(512), 0, s,
                         field, c.H, c.W, row_blocks(c), c.twf_x, dst);
    });
  else if (c.Wp == 3840)
    hipLaunchKernelGGL((k_row_fwd_c<3840, 2, 512, false>), dim3(row_blocks(c)), dim3(512), 0, s,
                       field, c.H, c.W, c.Wt, c.twf_x, c.tw_x, dst);
  else if (c.Wp == 512)
    hipLaunchKernelGGL((k_row_fwd_c<512, 4, 256, true>), dim3(row_blocks(c)), dim3(256), 0, s,
                       field, c.H, c.W, c.Wt, c.twf_x, c.tw_x, dst);
  else if (c.Wp <= 4096)
    hipLaunchKernelGGL(k_row_fwd<4096>, dim3(row_blocks(c)), dim3(kRowThreads), row_lds(c), s,
                       field, c.H, c.W, c.Wt, c.plan_x, c.tw_x, dst);
  else
    hipLaunchKernelGGL(k_row_fwd<8192>, dim3(row_blocks(c)), dim3(kRowThreads), row_lds(c), s,
                       field, c.H, c.W, c.Wt, c.plan_x, c.tw_x, dst);
  return hipGetLastError();
}

hipError_t launch_row_inv(const Ctx &c, const float2 *src, float2 *out, hipStream_t s) {
  if (row_quarter(c))
    with_quarter(c, [&](auto mc) {
      hipLaunchKernelGGL(k_row_inv_q<decltype(mc)::value>, dim3(row_blocks(c)), dim3(512), 0, s,
                         src, c.H, c.W, row_blocks(c), c.twf_x, out);
    });
  else if (c.Wp == 3840)
    hipLaunchKernelGGL((k_row_inv_c<3840, 2, 512, false>), dim3(row_blocks(c)), dim3(512), 0, s,
                       src, c.H, c.W, c.Wt, c.twf_x, c.tw_x, out);
  else if (c.Wp == 512)
    hipLaunchKernelGGL((k_row_inv_c<512, 4, 256, true>), dim3(row_blocks(c)), dim3(256), 0, s,
                       src, c.H, c.W, c.Wt, c.twf_x, c.tw_x, out);
  else if (c.Wp <= 4096)
    hipLaunchKernelGGL(k_row_inv<4096>, dim3(row_blocks(c)), dim3(kRowThreads), row_lds(c), s,
                       src, c.H, c.W, c.Wt, c.plan_x, c.tw_x, out);
  else
    hipLaunchKernelGGL(k_row_inv<8192>, dim3(row_blocks(c)), dim3(kRowThreads), row_lds(c), s,
                       src, c.H, c.W, c.Wt, c.plan_x, c.tw_x, out);
  return hipGetLastError();
}

hipError_t launch_row_loss(const Ctx &c, int plane, float2 *buf, const float *target,
                           const float *grad_intensity, const float *mask, float *intensity,
                           float2 *u_out, int make_grad, hipStream_t s) {
  // the loss of each hologram is its own mean over L C H W
  const double M = (double)c.L * c.C * c.H * c.W;
  const float gscale = (float)(4.0 / M);
  // plane l of the [L][B C][H][W] arrays; its loss partials after those of planes < l
  const size_t po = (size_t)plane * c.CF * c.H * c.W;
  if (target) target += po;
  if (grad_intensity) grad_intensity += po;
  if (intensity) intensity += po;
  if (u_out) u_out += po;
  // [L][B][H][W]: propagation channel ch reads the mask of hologram ch / C
  if (mask) mask += (size_t)plane * c.B * c.H * c.W;
  const int mcg = c.C;
  double *lp = c.loss_part + (size_t)plane * row_blocks(c);
  if (row_quarter(c))
    with_quarter(c, [&](auto mc) {
      hipLaunchKernelGGL(k_row_loss_q<decltype(mc)::value>, dim3(row_blocks(c)), dim3(512), 0, s,
                         buf, c.H, c.W, row_blocks(c), c.twf_x, target, grad_intensity, mask, mcg,
                         intensity, u_out, lp, gscale, make_grad);
    });
  else if (c.Wp == 3840)
    hipLaunchKernelGGL((k_row_loss_c<3840, 2, 512, false>), dim3(row_blocks(c)), dim3(512), 0, s,
                       buf, c.H, c.W, c.Wt, c.twf_x, c.tw_x, target, grad_intensity, mask, mcg, intensity,
                       u_out, lp, gscale, make_grad);
  else if (c.Wp == 512)
    hipLaunchKernelGGL((k_row_loss_c<512, 4, 256, true>), dim3(row_blocks(c)), dim3(256), 0, s,
                       buf, c.H, c.W, c.Wt, c.twf_x, c.tw_x, target, grad_intensity, mask, mcg, intensity,
                       u_out, lp, gscale, make_grad);
  else if (c.Wp <= 4096)
    hipLaunchKernelGGL(k_row_loss<4096>, dim3(row_blocks(c)), dim3(kRowThreads), row_lds(c), s,
                       buf, c.H, c.W, c.Wt, c.plan_x, c.tw_x, target, grad_intensity, mask, mcg,
                       intensity, u_out, lp, gscale, make_grad);
  else
    hipLaunchKernelGGL(k_row_loss<8192>, dim3(row_blocks(c)), dim3(kRowThreads), row_lds(c), s,
                       buf, c.H, c.W, c.Wt, c.plan_x, c.tw_x, target, grad_intensity, mask, mcg,
                       intensity, u_out, lp, gscale, make_grad);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Column passes over one 8-column tile of one channel (a contiguous block of
// H x 8 complex in S), in place.
// ----------------------------------------------------------------------------
// Source, destination and transfer table of one column pass.  src and dst
// may be the same buffer (in place).  acc: add the result to dst instead of
// overwriting it (the adjoint's sum over planes).  htab points at the table
// of the pass's plane for channel 0; channel ch is at htab + ch * hstride.
struct ColIO {
  const float2 *src;
  float2 *dst;
  const float2 *htab;
  size_t hstride;
  int acc;
};

__device__ __forceinline__ void col_store(const ColIO &io, size_t i, float2 v) {
  io.dst[i] = io.acc ? cadd(io.dst[i], v) : v;
}

__device__ __forceinline__ float2 transfer_at(const float2 *__restrict__ hc, int ky, int kx,
                                              int Hp, int Wp, int Wq, int conj_h, float scale) {
  const int qx = min(kx, Wp - kx), qy = min(ky, Hp - ky);
  float2 h = hc[(size_t)qy * Wq + qx];
  if (conj_h) h.y = -h.y;
  return cscale(h, scale);
}

// X[i] *= H(2 (i >> 3) + parity, 8 t + (i & 7)) over one column block of M rows:
// all table loads of a thread are issued before the first is used, so their
// latencies overlap.
template <int M, int T>
__device__ __forceinline__ void apply_transfer(float2 *X, const float2 *__restrict__ hc,
                                               int parity, int t, int Wp, int Wq, int conj_h,
                                               float scale, int tid) {
  constexpr int total = 8 * M, K = (total + T - 1) / T, G = 3;
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += G) {
    float2 hv[G];
#pragma unroll
    for (int k = k0; k < k0 + G && k < K; ++k) {
      const int i = tid + k * T;
      hv[k - k0] = make_float2(0.f, 0.f);
      if (total % T == 0 || i < total) {
        const int kx = t * 8 + (i & 7), ky = 2 * (i >> 3) + parity;
        const int qx = min(kx, Wp - kx), qy = min(ky, 2 * M - ky);
        if (kx < Wp) hv[k - k0] = hc[(uint32_t)(qy * Wq + qx)];
      }
    }
#pragma unroll
    for (int k = k0; k < k0 + G && k < K; ++k) {
      const int i = tid + k * T;
      if (total % T == 0 || i < total) {
        float2 h = hv[k - k0];
        if (conj_h) h.y = -h.y;
        X[i] = cmul(X[i], cscale(h, scale));
      }
    }
  }
}

// even Hp = 2M: two M-point chains (see the file header)
template <int MAXM, int T>
__global__ __launch_bounds__(T, 2048 / T) void k_col_half(ColIO io, int H, int Wp, int Wt,
                                                FftPlan pm, const float2 *__restrict__ twm,
                                                const float2 *__restrict__ twh, int Wq,
                                                int conj_h, float scale) {
  __shared__ float2 sbuf[8 * MAXM];
  __shared__ TwLds tm, th;
  constexpr int K = (8 * MAXM + T - 1) / T;
  const int tid = threadIdx.x;
  const int M = pm.n, Hp = 2 * M;
  const int t = blockIdx.x, ch = blockIdx.y;
  const size_t off = ((size_t)ch * Wt + t) * H * 8;
  const float2 *base = io.src + off;
  const float2 *hc = io.htab + ch * io.hstride;
  const int total = 8 * M;
  load_tw<T>(tm, twm, tid);
  load_tw<T>(th, twh, tid);
  __syncthreads();
  float2 keep[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tid + k * T;
    keep[k] = make_float2(0.f, 0.f);
    if (i < total) {
      const int n = i >> 3, kx = t * 8 + (i & 7);
      float2 x0 = make_float2(0.f, 0.f), x1 = x0;
      if (kx < Wp) {
        if (n < H) x0 = base[i];
        if (n + M < H) x1 = base[i + 8 * M];
      }
      sbuf[i] = cadd(x0, x1);
      keep[k] = cmul(csub(x0, x1), tw_at(th, n));
    }
  }
  __syncthreads();
  for (int parity = 0; parity < 2; ++parity) {
    fft_lds<-1, 8, T, MAXM>(sbuf, pm, tm, tid);
    for (int i = tid; i < total; i += T) {
      const int m = i >> 3, kx = t * 8 + (i & 7);
      sbuf[i] = kx < Wp ? cmul(sbuf[i], transfer_at(hc, 2 * m + parity, kx, Hp, Wp, Wq, conj_h,
                                                     scale))
                        : make_float2(0.f, 0.f);
    }
    __syncthreads();
    fft_lds<+1, 8, T, MAXM>(sbuf, pm, tm, tid);
    if (parity == 0) {
      // even result to registers, odd-chain input to LDS (each thread its own slots)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = tid + k * T;
        if (i < total) {
          const float2 e = sbuf[i];
          sbuf[i] = keep[k];
          keep[k] = e;
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tid + k * T;
    if (i < total) {
      const int n = i >> 3, kx = t * 8 + (i & 7);
      if (kx < Wp) {
        const float2 wo = cmul(cconj(tw_at(th, n)), sbuf[i]);
        if (n < H) col_store(io, off + i, cadd(keep[k], wo));
        if (n + M < H) col_store(io, off + i + 8 * M, csub(keep[k], wo));
      }
    }
  }
}

// odd Hp: one Hp-point transform per column
template <int MAXN, int T>
__global__ __launch_bounds__(T) void k_col_full(ColIO io, int H, int Wp, int Wt, FftPlan py,
                                                const float2 *__restrict__ twy, int Wq,
                                                int conj_h, float scale) {
  __shared__ float2 sbuf[8 * MAXN];
  __shared__ TwLds ty;
  const int tid = threadIdx.x;
  const int Hp = py.n;
  const int t = blockIdx.x, ch = blockIdx.y;
  const size_t off = ((size_t)ch * Wt + t) * H * 8;
  const float2 *base = io.src + off;
  const float2 *hc = io.htab + ch * io.hstride;
  const int total = 8 * Hp;
  load_tw<T>(ty, twy, tid);
  for (int i = tid; i < total; i += T) {
    const int r = i >> 3, kx = t * 8 + (i & 7);
    sbuf[i] = (r < H && kx < Wp) ? base[i] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  fft_lds<-1, 8, T, MAXN>(sbuf, py, ty, tid);
  for (int i = tid; i < total; i += T) {
    const int r = i >> 3, kx = t * 8 + (i & 7);
    sbuf[i] = kx < Wp ? cmul(sbuf[i], transfer_at(hc, r, kx, Hp, Wp, Wq, conj_h, scale))
                      : make_float2(0.f, 0.f);
  }
  __syncthreads();
  fft_lds<+1, 8, T, MAXN>(sbuf, py, ty, tid);
  for (int i = tid; i < 8 * H; i += T) {
    const int kx = t * 8 + (i & 7);
    if (kx < Wp) col_store(io, off + i, sbuf[i]);
  }
}

// size-specialised even/odd column pass: compile-time M-point plan, full
// M-entry twiddle table in LDS (the Hp-point pre/post twiddles use the small
// two-level table)
template <int M, int T>
__global__ __launch_bounds__(T) void k_col_half_c(ColIO io, int H, int Wp, int Wt,
                                                  const float2 *__restrict__ twf_m,
                                                  const float2 *__restrict__ twh, int Wq,
                                                  int conj_h, float scale) {
  __shared__ float2 sbuf[8 * M];
  __shared__ float2 tw[M];
  __shared__ TwLds th;
  constexpr int K = (8 * M + T - 1) / T;
  constexpr int total = 8 * M;
  constexpr int Hp = 2 * M;
  const int tid = threadIdx.x;
  const int t = blockIdx.x, ch = blockIdx.y;
  const size_t off = ((size_t)ch * Wt + t) * H * 8;
  const float2 *base = io.src + off;
  const float2 *hc = io.htab + ch * io.hstride;
  load_table<M, T>(tw, twf_m, tid);
  load_tw<T>(th, twh, tid);
  __syncthreads();
  float2 keep[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tid + k * T;
    keep[k] = make_float2(0.f, 0.f);
    if (total % T == 0 || i < total) {
      const int n = i >> 3, kx = t * 8 + (i & 7);
      float2 x0 = make_float2(0.f, 0.f), x1 = x0;
      if (kx < Wp) {
        if (n < H) x0 = base[i];
        if (n + M < H) x1 = base[i + 8 * M];
      }
      sbuf[i] = cadd(x0, x1);
      keep[k] = cmul(csub(x0, x1), tw_at(th, n));
    }
  }
  __syncthreads();
  for (int parity = 0; parity < 2; ++parity) {
    cfft<-1, 8, T, M>(sbuf, tw, tid);
    apply_transfer<M, T>(sbuf, hc, parity, t, Wp, Wq, conj_h, scale, tid);
    __syncthreads();
    cfft<+1, 8, T, M>(sbuf, tw, tid);
    if (parity == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = tid + k * T;
        if (total % T == 0 || i < total) {
          const float2 e = sbuf[i];
          sbuf[i] = keep[k];
          keep[k] = e;
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tid + k * T;
    if (total % T == 0 || i < total) {
      const int n = i >> 3, kx = t * 8 + (i & 7);
      if (kx < Wp) {
        const float2 wo = cmul(cconj(tw_at(th, n)), sbuf[i]);
        if (n < H) col_store(io, off + i, cadd(keep[k], wo));
        if (n + M < H) col_store(io, off + i + 8 * M, csub(keep[k], wo));
      }
    }
  }
}

// ----------------------------------------------------------------------------
// Column pass for Hp = 4 M with H <= 2 M, one wave per chain, M = R0 R1 R2
// (1080 = 9 6 20 at 4K, 540 = 12 5 9 at 1080p); CONJ: multiply by conj(H)
// (the adjoint pass).
// Output bin 4 m + p of the padded column is bin m of the M-point transform
// of w^{p n} (x[n] + (-i)^p x[n + M]) (n < M; w = e^{-2 pi i / Hp}), so a
// column is four M-point chains; the inverse gives u[n + M j] = sum_p
// w^{-p n} i^{p j} z_p[n] for j = 0, 1.  A workgroup takes two columns of a
// quarter tile; wave 4 c + p runs chain p of column c in its own M-element
// LDS buffer, so the stages of a chain need no workgroup barrier: only
// loading the columns and combining the chains are workgroup steps.  The
// forward plan is R0, R1, R2; its last stage leaves lane j < M / R2 holding
// spectrum entries j + (M / R2) q (q < R2), exactly the input of a first
// inverse stage of radix R2, so the transfer multiply and that stage run in
// registers; the inverse plan is R2, R1, R0.  The transfer table is read
// column-major ([Wq][Hq]); the eight quarter tiles of a mirror pair of tiles
// (t, Wt - 1 - t), whose columns need the same table columns, are blocks
// b + 8 s (s < 8), which share an XCD.
// ----------------------------------------------------------------------------
template <int R0, int R1, int R2, bool CONJ>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_col_wave4(
    ColIO io, const float2 *__restrict__ htab_t, int Hq, int H, int Wp, int Wt, int C,
    const float2 *__restrict__ twf_y) {
  constexpr int M = R0 * R1 * R2;
  constexpr int NB2 = M / R2;
  static_assert(NB2 <= 64, "the fused stage takes one butterfly per lane");
  constexpr int T = 512, NI = 2 * M, K = (NI + T - 1) / T, KT = (M + T - 1) / T;
  __shared__ float2 buf[8 * M];
  __shared__ float2 tw[M];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: scalar addressing
  const int b = blockIdx.x;
  const int slot = (b >> 3) & 7, pi = (b >> 6) * 8 + (b & 7);
  const int hp = (Wt + 1) >> 1;
  if (pi >= C * hp) return;
  const int ch = pi / hp, pp = pi - ch * hp;
  const int t = slot < 4 ? pp : Wt - 1 - pp;
  if (slot >= 4 && t == pp) return;  // the middle tile of an odd count has no mirror
  const int part = slot & 3;
  const size_t off = ((size_t)ch * Wt + t) * H * 8 + part * 2;
  const float2 *src = io.src + off;
  float2 *dst = io.dst + off;
  {
    // item i: row n = i / 2 of column c = i % 2; every global load of this
    // phase is issued before the first LDS store
    float2 av[K], bv[K], w1[K], tv[KT];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + k * T, n = min(i >> 1, M - 1), c = i & 1;
      av[k] = at32(src, min(n, H - 1) * 8 + c);
      bv[k] = at32(src, min(n + M, H - 1) * 8 + c);
      w1[k] = at32(twf_y, n);
    }
#pragma unroll
    for (int k = 0; k < KT; ++k) tv[k] = at32(twf_y, 4 * M + min(tid + k * T, M - 1));  // w_M^k
#pragma unroll
    for (int k = 0; k < KT; ++k)
      if (tid + k * T < M) tw[tid + k * T] = tv[k];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + k * T, n = i >> 1, c = i & 1;
      if (K * T == NI || i < NI) {
        const float2 a = n < H ? av[k] : make_float2(0.f, 0.f);
        const float2 bb = n + M < H ? bv[k] : make_float2(0.f, 0.f);
        const float2 s0 = cadd(a, bb), s2 = csub(a, bb);
        const float2 s1 = make_float2(a.x + bb.y, a.y - bb.x);  // a - i b
        const float2 s3 = make_float2(a.x - bb.y, a.y + bb.x);  // a + i b
        const float2 w2 = cmul(w1[k], w1[k]), w3 = cmul(w2, w1[k]);  // w^{2n}, w^{3n}
        buf[(4 * c) * M + n] = s0;
        buf[(4 * c + 1) * M + n] = cmul(s1, w1[k]);
        buf[(4 * c + 2) * M + n] = cmul(s2, w2);
        buf[(4 * c + 3) * M + n] = cmul(s3, w3);
      }
    }
  }
  __syncthreads();
  {
    const int c = wave >> 2, p = wave & 3;
    float2 *wb = buf + wave * M;
    const int kx = t * 8 + part * 2 + c;
    const int qx = min(kx, Wp - kx);
    const float2 *hcol = htab_t + (size_t)ch * io.hstride + (size_t)qx * Hq;
    // transfer values for ky = 4 (j + NB2 q) + p, issued before the forward stages
    float2 hv[R2];
    {
      const int j = min(lane, NB2 - 1);
      static_for<0, R2>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const int ky = 4 * (j + NB2 * q) + p;
        hv[q] = at32(hcol, min(ky, 4 * M - ky));
      });
    }
    wstage<R0, -1, M, 1>(wb, tw, lane);
    wstage<R1, -1, M, R0>(wb, tw, lane);
    float2 v[R2];
    if (lane < NB2) {
      static_for<0, R2>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        v[q] = wb[lane + q * NB2];
      });
      static_for<1, R2>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        v[q] = cmul(v[q], tw[q * lane]);  // last forward stage: Ns = NB2, unit twiddle step
      });
      RFft<R2, -1>::run(v);
      static_for<0, R2>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        v[q] = cmul(v[q], CONJ ? cconj(hv[q]) : hv[q]);  // the table carries 1 / (Hp Wp)
      });
      RFft<R2, +1>::run(v);  // first inverse stage: Ns = 1, no twiddles
    }
    wave_lds_order();
    if (lane < NB2) {
      static_for<0, R2>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        wb[lane * R2 + q] = v[q];
      });
    }
    wave_lds_order();
    wstage<R1, +1, M, R2>(wb, tw, lane);
    wstage<R0, +1, M, R2 * R1>(wb, tw, lane);
  }
  {
    float2 w1[K];
#pragma unroll
    for (int k = 0; k < K; ++k) w1[k] = at32(twf_y, min((tid + k * T) >> 1, M - 1));
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + k * T, n = i >> 1, c = i & 1;
      if ((K * T == NI || i < NI) && n < H) {
        const float2 w2 = cmul(w1[k], w1[k]), w3 = cmul(w2, w1[k]);
        const float2 z0 = buf[(4 * c) * M + n];
        const float2 z1 = cmul(cconj(w1[k]), buf[(4 * c + 1) * M + n]);
        const float2 z2 = cmul(cconj(w2), buf[(4 * c + 2) * M + n]);
        const float2 z3 = cmul(cconj(w3), buf[(4 * c + 3) * M + n]);
        const float2 y0 = cadd(cadd(z0, z1), cadd(z2, z3));
        float2 &d0 = at32(dst, n * 8 + c);
        d0 = io.acc ? cadd(d0, y0) : y0;
        if (n + M < H) {
          // z0 + i z1 - z2 - i z3
          const float2 e = csub(z0, z2), o = csub(z1, z3);
          const float2 y1 = make_float2(e.x - o.y, e.y + o.x);
          float2 &d1 = at32(dst, (n + M) * 8 + c);
          d1 = io.acc ? cadd(d1, y1) : y1;
        }
      }
    }
  }
}

hipError_t launch_col_pass(const Ctx &c, int conj_h, int plane, const float2 *src, float2 *dst,
                           int acc, hipStream_t s) {
  const float scale = (float)(1.0 / ((double)c.Hp * (double)c.Wp));
  const size_t tab = (size_t)c.Hq * c.Wq;
  const ColIO io{src, dst, c.htab + (size_t)plane * tab, (size_t)c.L * tab, acc};
  dim3 grid(c.Wt, c.CF);
  if (col_wave4(c)) {
    const int pairs = c.CF * ((c.Wt + 1) / 2);
    const float2 *ht = c.htab_t + (size_t)plane * tab;
    const dim3 grid4((pairs + 7) / 8 * 64);
    // M = R0 R1 R2 with M / R2 <= 64 (one fused butterfly per lane)
    auto go = [&](auto r0, auto r1, auto r2) {
      constexpr int R0 = decltype(r0)::value, R1 = decltype(r1)::value, R2 = decltype(r2)::value;
      if (conj_h)
        hipLaunchKernelGGL((k_col_wave4<R0, R1, R2, true>), grid4, dim3(512), 0, s, io, ht, c.Hq,
                           c.H, c.Wp, c.Wt, c.CF, c.twf_y);
      else
        hipLaunchKernelGGL((k_col_wave4<R0, R1, R2, false>), grid4, dim3(512), 0, s, io, ht,
                           c.Hq, c.H, c.Wp, c.Wt, c.CF, c.twf_y);
    };
    using std::integral_constant;
    switch (col_wave4_m(c)) {
      case 1080: go(integral_constant<int, 9>{}, integral_constant<int, 6>{}, integral_constant<int, 20>{}); break;
      case 1024: go(integral_constant<int, 8>{}, integral_constant<int, 8>{}, integral_constant<int, 16>{}); break;
      case 540: go(integral_constant<int, 12>{}, integral_constant<int, 5>{}, integral_constant<int, 9>{}); break;
      case 512: go(integral_constant<int, 8>{}, integral_constant<int, 8>{}, integral_constant<int, 8>{}); break;
      case 384: go(integral_constant<int, 6>{}, integral_constant<int, 8>{}, integral_constant<int, 8>{}); break;
      default: go(integral_constant<int, 4>{}, integral_constant<int, 8>{}, integral_constant<int, 8>{}); break;
    }
  } else if (c.Hp == 2160) {
    hipLaunchKernelGGL((k_col_half_c<1080, 1024>), grid, dim3(1024), 0, s, io, c.H, c.Wp, c.Wt,
                       c.twf_m, c.tw_y, c.Wq, conj_h, scale);
  } else if (c.Hp == 512) {
    hipLaunchKernelGGL((k_col_half_c<256, 256>), grid, dim3(256), 0, s, io, c.H, c.Wp, c.Wt,
                       c.twf_m, c.tw_y, c.Wq, conj_h, scale);
  } else if (c.Hp % 2 == 0) {
    const int M = c.Hp / 2;
    if (M <= kColHalfSmall)
      hipLaunchKernelGGL((k_col_half<kColHalfSmall, 512>), grid, dim3(512), 0, s, io, c.H, c.Wp,
                         c.Wt, c.plan_m, c.tw_m, c.tw_y, c.Wq, conj_h, scale);
    else
      hipLaunchKernelGGL((k_col_half<kColHalfMax, 1024>), grid, dim3(1024), 0, s, io, c.H, c.Wp,
                         c.Wt, c.plan_m, c.tw_m, c.tw_y, c.Wq, conj_h, scale);
  } else {
    hipLaunchKernelGGL((k_col_full<kColFullMax, 1024>), grid, dim3(1024), 0, s, io, c.H, c.Wp,
                       c.Wt, c.plan_y, c.tw_y, c.Wq, conj_h, scale);
  }
  return hipGetLastError();
}

// Per hologram b: loss = sum of its loss partials / M, psnr = 10 log10(1 / loss);
// one block per hologram, fixed order.  The partials of plane l are
// part[l * rows_per_plane + r]; hologram b owns r in [b span, (b + 1) span).
__global__ __launch_bounds__(256) void k_loss_finalize(const double *__restrict__ part,
                                                       int planes, int rows_per_plane, int span,
                                                       double inv_m, double *__restrict__ out,
                                                       uint32_t *__restrict__ finite_flag) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  double acc = 0.0;
  for (int l = 0; l < planes; ++l) {
    const double *p = part + (size_t)l * rows_per_plane + (size_t)b * span;
    for (int i = threadIdx.x; i < span; i += 256) acc += p[i];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double loss = red[0] * inv_m;
    out[2 * b] = loss;
    out[2 * b + 1] = 10.0 * log10(1.0 / loss);
    if (finite_flag && !isfinite(loss)) atomicOr(finite_flag, kNonFiniteLoss);
  }
}

hipError_t launch_loss_finalize(const Ctx &c, double *loss, hipStream_t s) {
  const double inv_m = 1.0 / ((double)c.L * c.C * c.H * c.W);
  const int rows = row_blocks(c);
  hipLaunchKernelGGL(k_loss_finalize, dim3(c.B), dim3(256), 0, s, c.loss_part, c.L, rows,
                     rows / c.B, inv_m, loss, c.finite_flag);
  return hipGetLastError();
}

}  // namespace cgh
