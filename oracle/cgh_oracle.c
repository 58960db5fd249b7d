/*
 * cgh_oracle.c -- plain FP64 CPU oracle for complex-valued 2D Gaussian CGH.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * statement of what the GPU path computes.  It shares no code, header,
 * table or constant with the HIP library; only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.
 *
 * Every routine states the passage of the paper it writes out:
 *   - Supplementary "Forward Pass": parameter activations, 2D covariance,
 *     2x2 inversion with the determinant clamp, Gaussian evaluation with the
 *     power clamp, complex field rendering (coherent, order-independent sum);
 *   - Supplementary "Backward Pass": the per-parameter gradient formulas;
 *   - Sec. 2 (free-space propagation) and the supplementary BLASM section:
 *     spatial frequencies, band limit, transfer function, conjugate adjoint.
 *
 * Readings taken where the paper is silent (each is listed in the design
 * notes): pixel (i, j) sits at the integer point (i, j) in the frame of the
 * mean (0-based); the support of a Gaussian is the ellipse q <= k^2 of its
 * regularised covariance (k <= 0: unbounded); the FFT is unnormalised forward
 * with kernel exp(-2 pi i k n / N) and 1/N on the inverse; the transfer
 * function is laid out in natural FFT order (equivalent to the paper's
 * shift / multiply / unshift); evanescent frequencies get H = 0.
 *
 * Precision: every quantity is FP64.  The callers widen the FP32 arrays the
 * GPU receives to FP64 exactly, so both sides start from identical values.
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define TWO_PI 6.283185307179586476925286766559


#define EPS_SCALE 0.1   /* scale regulariser epsilon_s (Suppl. notation)        */
#define EPS_COV 0.1     /* covariance regulariser epsilon_c (Suppl. notation)   */
#define EPS_DET 1e-10   /* determinant clamp epsilon_d (Suppl. notation)        */
#define POWER_FLOOR -50.0 /* clamp on the Gaussian exponent (Suppl. "Gaussian Evaluation") */

#define FLAG_PAPER_ALPHA 2 /* alpha_eff = min(0.99, alpha G), skip below 1/255 (Alg. 2) */

/* ------------------------------------------------------------------------- */
/* Per-Gaussian geometry (Suppl. "Parameter Activation Functions",           */
/* "2D Covariance Matrix Computation", "2D Covariance Matrix Inversion").    */
/* ------------------------------------------------------------------------- */
typedef struct {
  double mx, my;          /* activated mean, pixels                           */
  double sx, sy;          /* activated scales                                 */
  double ct, st;          /* cos(theta), sin(theta)                           */
  double s00, s01, s11;   /* covariance with epsilon_c on the diagonal        */
  double det;             /* s00 s11 - s01^2 (unclamped)                      */
  double dsafe;           /* max(det, epsilon_d)                              */
  double i00, i01, i11;   /* stored inverse entries                           */
  double alpha;           /* sigmoid(alpha_pre)                               */
} geom_t;

static void geometry(int n, int W, int H, const double *mean_pre, const double *log_scale,
                     const double *rotation, const double *opacity_pre, geom_t *g) {
  for (int i = 0; i < n; ++i) {
    double xt = mean_pre[2 * i], yt = mean_pre[2 * i + 1];
    g[i].mx = 0.5 * (tanh(xt) + 1.0) * (double)W;
    g[i].my = 0.5 * (tanh(yt) + 1.0) * (double)H;
    g[i].sx = exp((double)log_scale[2 * i]) + EPS_SCALE;
    g[i].sy = exp((double)log_scale[2 * i + 1]) + EPS_SCALE;
    double th = rotation[i];
    g[i].ct = cos(th);
    g[i].st = sin(th);
    double sx2 = g[i].sx * g[i].sx, sy2 = g[i].sy * g[i].sy;
    double c = g[i].ct, s = g[i].st;
    g[i].s00 = sx2 * c * c + sy2 * s * s + EPS_COV;
    g[i].s01 = (sx2 - sy2) * c * s;
    g[i].s11 = sx2 * s * s + sy2 * c * c + EPS_COV;
    g[i].det = g[i].s00 * g[i].s11 - g[i].s01 * g[i].s01;
    g[i].dsafe = g[i].det > EPS_DET ? g[i].det : EPS_DET;
    g[i].i00 = g[i].s11 / g[i].dsafe;
    g[i].i01 = -g[i].s01 / g[i].dsafe;
    g[i].i11 = g[i].s00 / g[i].dsafe;
    g[i].alpha = 1.0 / (1.0 + exp(-(double)opacity_pre[i]));
  }
}

/* Exported so tests can pin the activations and covariance directly.
 * out[n][12] = mx, my, sx, sy, s00, s01, s11, det, i00, i01, i11, alpha. */
void orc_geometry(int n, int W, int H, const double *mean_pre, const double *log_scale,
                  const double *rotation, const double *opacity_pre, double *out) {
  geom_t *g = (geom_t *)malloc(sizeof(geom_t) * (size_t)(n > 0 ? n : 1));
  geometry(n, W, H, mean_pre, log_scale, rotation, opacity_pre, g);
  for (int i = 0; i < n; ++i) {
    double *o = out + 12 * (size_t)i;
    o[0] = g[i].mx; o[1] = g[i].my; o[2] = g[i].sx; o[3] = g[i].sy;
    o[4] = g[i].s00; o[5] = g[i].s01; o[6] = g[i].s11; o[7] = g[i].det;
    o[8] = g[i].i00; o[9] = g[i].i01; o[10] = g[i].i11; o[11] = g[i].alpha;
  }
  free(g);
}

/* Mahalanobis distance q = d^T Sigma^{-1} d with the stored inverse entries
 * (Suppl. "Gaussian Evaluation"). */
static double mahal(const geom_t *g, double dx, double dy) {
  return dx * dx * g->i00 + 2.0 * dx * dy * g->i01 + dy * dy * g->i11;
}

/* Support predicate: pixel inside the k-sigma ellipse of the (support)
 * geometry.  k <= 0 means every pixel is in support. */
static int in_support(const geom_t *gs, double px, double py, double k) {
  if (k <= 0.0) return 1;
  return mahal(gs, px - gs->mx, py - gs->my) <= k * k;
}

/* Inclusive pixel range of the support's axis-aligned box, widened by one
 * pixel so that rounding in the box never drops a pixel the predicate keeps. */
static void support_box(const geom_t *gs, double k, int W, int H, int *i0, int *i1, int *j0,
                        int *j1) {
  if (k <= 0.0) { *i0 = 0; *i1 = W - 1; *j0 = 0; *j1 = H - 1; return; }
  double rx = k * sqrt(gs->s00), ry = k * sqrt(gs->s11);
  double a = floor(gs->mx - rx) - 1.0, b = ceil(gs->mx + rx) + 1.0;
  double c = floor(gs->my - ry) - 1.0, d = ceil(gs->my + ry) + 1.0;
  *i0 = a < 0.0 ? 0 : (a > W - 1 ? W : (int)a);
  *i1 = b > W - 1 ? W - 1 : (b < 0.0 ? -1 : (int)b);
  *j0 = c < 0.0 ? 0 : (c > H - 1 ? H : (int)c);
  *j1 = d > H - 1 ? H - 1 : (d < 0.0 ? -1 : (int)d);
}

/* Contribution weight of Gaussian g at pixel p: returns the real factor w
 * such that the pixel receives c_{n,c} * w * exp(j phi_{n,c}); 0 if skipped.
 * Default: w = alpha G with G = exp(max(-q/2, -50)) (Suppl. "Complex Field
 * Rendering").  FLAG_PAPER_ALPHA follows Alg. 2 instead:
 * w = min(0.99, alpha G), skipped when below 1/255. */
static double pixel_weight(const geom_t *g, double dx, double dy, int flags, double *G_out,
                           int *clamped_power, int *clamped_alpha) {
  double q = mahal(g, dx, dy);
  double power = -0.5 * q;
  *clamped_power = power < POWER_FLOOR;
  if (power < POWER_FLOOR) power = POWER_FLOOR;
  double G = exp(power);
  *G_out = G;
  *clamped_alpha = 0;
  if (flags & FLAG_PAPER_ALPHA) {
    double ae = g->alpha * G;
    if (ae > 0.99) { ae = 0.99; *clamped_alpha = 1; }
    if (ae < 1.0 / 255.0) return 0.0;
    return ae;
  }
  return g->alpha * G;
}

/* ------------------------------------------------------------------------- */
/* Rasterization: U_c(p) = sum_n c_{n,c} alpha_n G_n(p) exp(j phi_{n,c})     */
/* (Sec. 3.1 coherent sum; Suppl. "Complex Field Rendering").                */
/* ------------------------------------------------------------------------- */

/* Brute force: every pixel against every Gaussian.  `sup_*` (optional, may be
 * NULL) give a second parameter set whose geometry decides the support
 * predicate -- used to hold the support fixed for finite differences. */
static void raster_impl(int brute, int n, int C, int W, int H, double k, int flags,
                        const double *mean_pre, const double *log_scale, const double *rotation,
                        const double *amplitude, const double *phase, const double *opacity_pre,
                        const double *sup_mean_pre, const double *sup_log_scale,
                        const double *sup_rotation, double *out_re, double *out_im) {
  geom_t *g = (geom_t *)malloc(sizeof(geom_t) * (size_t)(n > 0 ? n : 1));
  geom_t *gs = (geom_t *)malloc(sizeof(geom_t) * (size_t)(n > 0 ? n : 1));
  int *box = (int *)malloc(sizeof(int) * 4 * (size_t)(n > 0 ? n : 1));
  geometry(n, W, H, mean_pre, log_scale, rotation, opacity_pre, g);
  if (sup_mean_pre)
    geometry(n, W, H, sup_mean_pre, sup_log_scale, sup_rotation, opacity_pre, gs);
  else
    memcpy(gs, g, sizeof(geom_t) * (size_t)n);
  for (int i = 0; i < n; ++i)
    support_box(&gs[i], k, W, H, &box[4 * i], &box[4 * i + 1], &box[4 * i + 2], &box[4 * i + 3]);

  #pragma omp parallel for schedule(dynamic, 1)
  for (int j = 0; j < H; ++j) {
    for (int i = 0; i < W; ++i)
      for (int c = 0; c < C; ++c) {
        out_re[((size_t)c * H + j) * W + i] = 0.0;
        out_im[((size_t)c * H + j) * W + i] = 0.0;
      }
    for (int m = 0; m < n; ++m) {
      int i0 = 0, i1 = W - 1;
      if (!brute) {
        if (j < box[4 * m + 2] || j > box[4 * m + 3]) continue;
        i0 = box[4 * m];
        i1 = box[4 * m + 1];
      }
      for (int i = i0; i <= i1; ++i) {
        if (!in_support(&gs[m], (double)i, (double)j, k)) continue;
        double G;
        int cp, ca;
        double w = pixel_weight(&g[m], (double)i - g[m].mx, (double)j - g[m].my, flags, &G,
                                &cp, &ca);
        if (w == 0.0) continue;
        for (int c = 0; c < C; ++c) {
          double a = (double)amplitude[(size_t)m * C + c] * w;
          double ph = phase[(size_t)m * C + c];
          out_re[((size_t)c * H + j) * W + i] += a * cos(ph);
          out_im[((size_t)c * H + j) * W + i] += a * sin(ph);
        }
      }
    }
  }
  free(g);
  free(gs);
  free(box);
}

void orc_raster_brute(int n, int C, int W, int H, double k, int flags, const double *mean_pre,
                      const double *log_scale, const double *rotation, const double *amplitude,
                      const double *phase, const double *opacity_pre, double *out_re,
                      double *out_im) {
  raster_impl(1, n, C, W, H, k, flags, mean_pre, log_scale, rotation, amplitude, phase,
              opacity_pre, NULL, NULL, NULL, out_re, out_im);
}

/* Same sum, but each Gaussian only visits the pixels of its support box (the
 * predicate still decides).  Identical by definition to the brute force for
 * k > 0; used where the brute force would take minutes. */
void orc_raster(int n, int C, int W, int H, double k, int flags, const double *mean_pre,
                const double *log_scale, const double *rotation, const double *amplitude,
                const double *phase, const double *opacity_pre, const double *sup_mean_pre,
                const double *sup_log_scale, const double *sup_rotation, double *out_re,
                double *out_im) {
  raster_impl(0, n, C, W, H, k, flags, mean_pre, log_scale, rotation, amplitude, phase,
              opacity_pre, sup_mean_pre, sup_log_scale, sup_rotation, out_re, out_im);
}

/* Pairs whose Mahalanobis distance lies within a relative band of the
 * support boundary k^2: their in/out decision depends on rounding, so the
 * parity tests exclude the pixels they touch.  With FLAG_PAPER_ALPHA the
 * Alg. 2 skip (alpha G < 1/255, i.e. q > 2 ln(255 alpha)) is a second such
 * boundary, with a jump of c/255 in the contribution, and pairs within the
 * same band of it count too.  Writes 1 into mask[j*W+i] for every such pixel
 * and returns the number of such pairs. */
long orc_ambiguous_pixels(int n, int W, int H, double k, double rel_band, int flags,
                          const double *mean_pre, const double *log_scale,
                          const double *rotation, const double *opacity_pre,
                          unsigned char *mask) {
  if (k <= 0.0) return 0;
  geom_t *g = (geom_t *)malloc(sizeof(geom_t) * (size_t)(n > 0 ? n : 1));
  geometry(n, W, H, mean_pre, log_scale, rotation, opacity_pre, g);
  long count = 0;
  memset(mask, 0, (size_t)W * H);
  double k2 = k * k;
  for (int m = 0; m < n; ++m) {
    int i0, i1, j0, j1;
    support_box(&g[m], k, W, H, &i0, &i1, &j0, &j1);
    for (int j = j0; j <= j1; ++j)
      for (int i = i0; i <= i1; ++i) {
        double q = mahal(&g[m], (double)i - g[m].mx, (double)j - g[m].my);
        int near = fabs(q - k2) <= rel_band * k2;
        if ((flags & FLAG_PAPER_ALPHA) && q <= k2)
          near |= fabs(q - 2.0 * log(255.0 * g[m].alpha)) <= rel_band * k2;
        if (near) {
          mask[(size_t)j * W + i] = 1;
          ++count;
        }
      }
  }
  free(g);
  return count;
}

/* ------------------------------------------------------------------------- */
/* Discrete Fourier transform.  Forward: X[k] = sum_n x[n] e^{-2 pi i k n/N}, */
/* unnormalised; inverse: e^{+2 pi i k n / N} with 1/N.                       */
/* Mixed-radix Cooley-Tukey by recursion on the smallest prime factor; a     */
/* prime length falls through to the direct sum.                             */
/* ------------------------------------------------------------------------- */
static cplx root_of_unity(long num, long den, int sign) {
  /* exp(sign * 2 pi i num / den) with the angle reduced exactly first */
  long r = num % den;
  if (r < 0) r += den;
  double ang = TWO_PI * (double)r / (double)den;
  return cos(ang) + (double)sign * sin(ang) * I;
}

static int smallest_factor(int n) {
  for (int p = 2; p * p <= n; ++p)
    if (n % p == 0) return p;
  return n;
}

/* out[0..n) = DFT of in[0], in[stride], ..., in[(n-1) stride] */
static void dft_rec(const cplx *in, long stride, cplx *out, int n, int sign) {
  if (n == 1) { out[0] = in[0]; return; }
  int p = smallest_factor(n);
  int m = n / p;
  /* sub-transforms of the p decimated sequences x[r + p t], t < m */
  for (int r = 0; r < p; ++r) dft_rec(in + r * stride, stride * p, out + (size_t)r * m, m, sign);
  cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)n);
  for (int kk = 0; kk < m; ++kk)
    for (int q = 0; q < p; ++q) {
      long k = kk + (long)m * q;
      cplx s = 0.0;
      for (int r = 0; r < p; ++r) s += root_of_unity((long)r * k, n, sign) * out[(size_t)r * m + kk];
      tmp[k] = s;
    }
  memcpy(out, tmp, sizeof(cplx) * (size_t)n);
  free(tmp);
}

/* 1-D transform of contiguous complex data (interleaved re, im), in place.
 * inverse != 0 selects the +i kernel and the 1/N factor. */
void orc_fft1(int n, double *data, int inverse) {
  cplx *x = (cplx *)data;
  cplx *y = (cplx *)malloc(sizeof(cplx) * (size_t)n);
  dft_rec(x, 1, y, n, inverse ? +1 : -1);
  double s = inverse ? 1.0 / n : 1.0;
  for (int i = 0; i < n; ++i) x[i] = y[i] * s;
  free(y);
}

/* 2-D transform of an [ny][nx] complex array: rows, then columns. */
void orc_fft2(int ny, int nx, double *data, int inverse) {
  cplx *x = (cplx *)data;
  int sign = inverse ? +1 : -1;
  #pragma omp parallel
  {
    cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)(nx > ny ? nx : ny));
    cplx *col = (cplx *)malloc(sizeof(cplx) * (size_t)ny);
    #pragma omp for schedule(static)
    for (int j = 0; j < ny; ++j) {
      dft_rec(x + (size_t)j * nx, 1, buf, nx, sign);
      memcpy(x + (size_t)j * nx, buf, sizeof(cplx) * (size_t)nx);
    }
    #pragma omp for schedule(static)
    for (int i = 0; i < nx; ++i) {
      for (int j = 0; j < ny; ++j) col[j] = x[(size_t)j * nx + i];
      dft_rec(col, 1, buf, ny, sign);
      for (int j = 0; j < ny; ++j) x[(size_t)j * nx + i] = buf[j];
    }
    free(buf);
    free(col);
  }
  if (inverse) {
    double s = 1.0 / ((double)nx * ny);
    for (size_t t = 0; t < (size_t)nx * ny; ++t) x[t] *= s;
  }
}

/* ------------------------------------------------------------------------- */
/* Band-limited angular spectrum transfer function (Sec. 2 equation for H;  */
/* supplementary "Spatial Frequency Computation", "Bandlimit Computation",  */
/* "Transfer Function Evaluation").  Laid out in natural FFT order: index k */
/* carries the frequency ((k + N/2) mod N - N/2) / (N dx), i.e. the         */
/* paper's centred grid without the shift.  aperture > 0: the circular     */
/* aperture of Alg. 3, read as centred on the zero frequency: bins with     */
/* kx^2 + ky^2 >= aperture^2 (signed bin indices) are zeroed.               */
/* ------------------------------------------------------------------------- */
static double signed_index(int k, int n) { return (double)(((k + n / 2) % n) - n / 2); }

void orc_transfer(int ny, int nx, double pitch, double lambda, double z, double aperture,
                  double *out) {
  double Lx = nx * pitch, Ly = ny * pitch;
  double fxmax = 1.0 / (lambda * sqrt((2.0 * z / Lx) * (2.0 * z / Lx) + 1.0));
  double fymax = 1.0 / (lambda * sqrt((2.0 * z / Ly) * (2.0 * z / Ly) + 1.0));
  cplx *h = (cplx *)out;
  for (int ky = 0; ky < ny; ++ky)
    for (int kx = 0; kx < nx; ++kx) {
      double fx = signed_index(kx, nx) / Lx;
      double fy = signed_index(ky, ny) / Ly;
      double arg = 1.0 / (lambda * lambda) - fx * fx - fy * fy;
      cplx v = 0.0;
      double ix = signed_index(kx, nx), iy = signed_index(ky, ny);
      int open = aperture <= 0.0 || ix * ix + iy * iy < aperture * aperture;
      if (fabs(fx) < fxmax && fabs(fy) < fymax && arg >= 0.0 && open) {
        double ph = TWO_PI * z * sqrt(arg);
        v = cos(ph) + sin(ph) * I;
      }
      h[(size_t)ky * nx + kx] = v;
    }
}

/* ------------------------------------------------------------------------- */
/* Propagation of a [C][H][W] field to planes z_l: zero-pad (centred),      */
/* FFT2, multiply by H(lambda_c, z_l), IFFT2, crop the same window          */
/* (Alg. 1 ZeroPad + MultiPlanePropagate; Sec. 3.2).                         */
/* adjoint != 0 applies the conjugate transfer function (supplementary      */
/* "Backward Pass" of BLASM) and sums over planes into a [C][H][W] result.  */
/* ------------------------------------------------------------------------- */
static void propagate_one(int H, int W, int Hp, int Wp, double pitch, double lambda, double z,
                          double aperture, int conj_h, const cplx *in, cplx *out) {
  int oy = (Hp - H) / 2, ox = (Wp - W) / 2;
  cplx *P = (cplx *)calloc((size_t)Hp * Wp, sizeof(cplx));
  cplx *Ht = (cplx *)malloc(sizeof(cplx) * (size_t)Hp * Wp);
  for (int j = 0; j < H; ++j)
    for (int i = 0; i < W; ++i) P[(size_t)(j + oy) * Wp + (i + ox)] = in[(size_t)j * W + i];
  orc_fft2(Hp, Wp, (double *)P, 0);
  orc_transfer(Hp, Wp, pitch, lambda, z, aperture, (double *)Ht);
  for (size_t t = 0; t < (size_t)Hp * Wp; ++t) P[t] *= conj_h ? conj(Ht[t]) : Ht[t];
  orc_fft2(Hp, Wp, (double *)P, 1);
  for (int j = 0; j < H; ++j)
    for (int i = 0; i < W; ++i) out[(size_t)j * W + i] = P[(size_t)(j + oy) * Wp + (i + ox)];
  free(P);
  free(Ht);
}

/* field: [C][H][W] complex -> out: [L][C][H][W] complex */
void orc_propagate(int C, int H, int W, int Hp, int Wp, double pitch, const double *lambdas,
                   int L, const double *zs, double aperture, const double *field, double *out) {
  for (int l = 0; l < L; ++l)
    for (int c = 0; c < C; ++c)
      propagate_one(H, W, Hp, Wp, pitch, lambdas[c], zs[l], aperture, 0,
                    (const cplx *)field + (size_t)c * H * W,
                    (cplx *)out + ((size_t)l * C + c) * H * W);
}

/* grad_u: [L][C][H][W] complex -> grad_field: [C][H][W] complex (sum over l) */
void orc_propagate_adjoint(int C, int H, int W, int Hp, int Wp, double pitch,
                           const double *lambdas, int L, const double *zs, double aperture,
                           const double *grad_u, double *grad_field) {
  cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)H * W);
  cplx *gf = (cplx *)grad_field;
  memset(gf, 0, sizeof(cplx) * (size_t)C * H * W);
  for (int l = 0; l < L; ++l)
    for (int c = 0; c < C; ++c) {
      propagate_one(H, W, Hp, Wp, pitch, lambdas[c], zs[l], aperture, 1,
                    (const cplx *)grad_u + ((size_t)l * C + c) * H * W, tmp);
      for (size_t t = 0; t < (size_t)H * W; ++t) gf[(size_t)c * H * W + t] += tmp[t];
    }
  free(tmp);
}

/* ------------------------------------------------------------------------- */
/* Rasterizer adjoint (Supplementary "Backward Pass", items 1-7).           */
/* grad_field holds dL/dreal + j dL/dimag per channel and pixel, [C][H][W]. */
/* Outputs (pre-activation parameters, same layouts as the inputs):         */
/*   g_mean [N][2], g_log_scale [N][2], g_rotation [N], g_amplitude [N][C],  */
/*   g_phase [N][C], g_opacity [N].                                          */
/* ------------------------------------------------------------------------- */
void orc_raster_adjoint(int n, int C, int W, int H, double k, int flags, const double *mean_pre,
                        const double *log_scale, const double *rotation, const double *amplitude,
                        const double *phase, const double *opacity_pre, const double *grad_field,
                        double *g_mean, double *g_log_scale, double *g_rotation,
                        double *g_amplitude, double *g_phase, double *g_opacity) {
  geom_t *gg = (geom_t *)malloc(sizeof(geom_t) * (size_t)(n > 0 ? n : 1));
  geometry(n, W, H, mean_pre, log_scale, rotation, opacity_pre, gg);
  const cplx *gf = (const cplx *)grad_field;

  #pragma omp parallel for schedule(dynamic, 64)
  for (int m = 0; m < n; ++m) {
    const geom_t *g = &gg[m];
    int i0, i1, j0, j1;
    support_box(g, k, W, H, &i0, &i1, &j0, &j1);
    double dL_dmx = 0, dL_dmy = 0, dL_di00 = 0, dL_di01 = 0, dL_di11 = 0, dL_dalpha = 0;
    double dL_dc[4] = {0, 0, 0, 0}, dL_dphi[4] = {0, 0, 0, 0};
    for (int j = j0; j <= j1; ++j)
      for (int i = i0; i <= i1; ++i) {
        if (!in_support(g, (double)i, (double)j, k)) continue;
        double dx = (double)i - g->mx, dy = (double)j - g->my;
        double G;
        int cp, ca;
        double w = pixel_weight(g, dx, dy, flags, &G, &cp, &ca);
        if (w == 0.0) continue;
        /* dL/dw where the pixel receives sum_c c_c w e^{j phi_c} */
        double dL_dw = 0.0;
        for (int c = 0; c < C; ++c) {
          cplx gc = gf[((size_t)c * H + j) * W + i];
          double cc = amplitude[(size_t)m * C + c], ph = phase[(size_t)m * C + c];
          double cs = cos(ph), sn = sin(ph);
          double proj = creal(gc) * cs + cimag(gc) * sn;   /* Re(conj(g) e^{j phi}) */
          double rot = -creal(gc) * sn + cimag(gc) * cs;   /* Re(conj(g) j e^{j phi}) */
          dL_dc[c] += w * proj;                            /* item 1 */
          dL_dphi[c] += cc * w * rot;                      /* item 2 */
          dL_dw += cc * proj;
        }
        /* w = alpha G (default) or min(0.99, alpha G) (paper alpha) */
        double dL_dG;
        if (ca) { dL_dG = 0.0; }
        else {
          dL_dalpha += dL_dw * G;                          /* item 3 */
          dL_dG = dL_dw * g->alpha;
        }
        if (!cp) {
          /* G = exp(-q/2): dG/dq = -G/2 (items 4, 5) */
          double dL_dq = dL_dG * (-0.5 * G);
          dL_dmx += dL_dq * (-2.0 * (dx * g->i00 + dy * g->i01));
          dL_dmy += dL_dq * (-2.0 * (dx * g->i01 + dy * g->i11));
          dL_di00 += dL_dq * dx * dx;
          dL_di01 += dL_dq * 2.0 * dx * dy;
          dL_di11 += dL_dq * dy * dy;
        }
      }
    /* pre-activation chain: tanh for the mean (item 4) */
    double tx = tanh((double)mean_pre[2 * m]), ty = tanh((double)mean_pre[2 * m + 1]);
    g_mean[2 * m] = dL_dmx * 0.5 * W * (1.0 - tx * tx);
    g_mean[2 * m + 1] = dL_dmy * 0.5 * H * (1.0 - ty * ty);
    /* sigmoid for the opacity (item 3) */
    g_opacity[m] = dL_dalpha * g->alpha * (1.0 - g->alpha);
    /* w already carries alpha (items 1, 2) */
    for (int c = 0; c < C; ++c) {
      g_amplitude[(size_t)m * C + c] = dL_dc[c];
      g_phase[(size_t)m * C + c] = dL_dphi[c];
    }
    /* inverse entries -> covariance entries: quotient rule on inv = adj / D */
    double s00 = g->s00, s01 = g->s01, s11 = g->s11, D = g->dsafe;
    double dL_ds00, dL_ds01, dL_ds11;
    if (g->det > EPS_DET) {
      double D2 = D * D;
      /* d inv00 / d(s00, s01, s11) etc. with dD = s11 ds00 + s00 ds11 - 2 s01 ds01 */
      double i00_s00 = -s11 * s11 / D2, i00_s01 = 2.0 * s01 * s11 / D2,
             i00_s11 = 1.0 / D - s11 * s00 / D2;
      double i01_s00 = s01 * s11 / D2, i01_s01 = -1.0 / D - 2.0 * s01 * s01 / D2,
             i01_s11 = s01 * s00 / D2;
      double i11_s00 = 1.0 / D - s00 * s11 / D2, i11_s01 = 2.0 * s01 * s00 / D2,
             i11_s11 = -s00 * s00 / D2;
      dL_ds00 = dL_di00 * i00_s00 + dL_di01 * i01_s00 + dL_di11 * i11_s00;
      dL_ds01 = dL_di00 * i00_s01 + dL_di01 * i01_s01 + dL_di11 * i11_s01;
      dL_ds11 = dL_di00 * i00_s11 + dL_di01 * i01_s11 + dL_di11 * i11_s11;
    } else {
      /* clamped determinant: inv = adj / eps_d, no dependence through D */
      dL_ds00 = dL_di11 / D;
      dL_ds01 = -dL_di01 / D;
      dL_ds11 = dL_di00 / D;
    }
    /* covariance -> (s_x, s_y, theta) (items 6, 7) */
    double sx = g->sx, sy = g->sy, c = g->ct, s = g->st;
    double dL_dsx = 2.0 * sx * (c * c * dL_ds00 + c * s * dL_ds01 + s * s * dL_ds11);
    double dL_dsy = 2.0 * sy * (s * s * dL_ds00 - c * s * dL_ds01 + c * c * dL_ds11);
    double dL_dth = 2.0 * (sy * sy - sx * sx) * c * s * dL_ds00 +
                    (sx * sx - sy * sy) * (c * c - s * s) * dL_ds01 +
                    2.0 * (sx * sx - sy * sy) * c * s * dL_ds11;
    g_log_scale[2 * m] = dL_dsx * exp((double)log_scale[2 * m]);
    g_log_scale[2 * m + 1] = dL_dsy * exp((double)log_scale[2 * m + 1]);
    g_rotation[m] = dL_dth;
  }
  free(gg);
}
