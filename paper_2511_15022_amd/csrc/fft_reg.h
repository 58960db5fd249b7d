// Register-resident DFTs of compile-time length and compile-time Stockham
// plans: the building blocks of the size-specialised propagation kernels.
//
// RFft<N, DIR> transforms N complex values held in registers (natural order in
// and out), y_k = sum_n x_n exp(DIR 2 pi i n k / N), by splitting N = N1 N2
// (N1 a base radix 2, 3, 4, 5 or 8): N2 DFTs of length N1, a multiply by the
// compile-time twiddles exp(DIR 2 pi i n2 k1 / N), then N1 DFTs of length N2.
// All twiddles are constants evaluated at compile time in double precision.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

// arithmetic helpers are host-callable too, so the transforms can be checked on a CPU
#define CGH_HD __host__ __device__ __forceinline__

namespace cgh {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
CGH_HD float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
CGH_HD float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
CGH_HD float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
CGH_HD float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
CGH_HD float2 cneg(float2 a) { return make_float2(-a.x, -a.y); }
CGH_HD float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// multiply by DIR * i
template <int DIR>
CGH_HD float2 rot90(float2 a) {
  return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// compile-time unit roots exp(2 pi i m / n): exact integer reduction to an
// angle in [0, pi/4], then Taylor series in double
// ---------------------------------------------------------------------------
struct CDouble {
  double re, im;
};

constexpr double kPiD = 3.14159265358979323846264338327950288;

constexpr double sin_series(double x) {
  double x2 = x * x, t = x, s = x;
  for (int i = 1; i < 14; ++i) {
    t *= -x2 / ((2.0 * i) * (2.0 * i + 1.0));
    s += t;
  }
  return s;
}

constexpr double cos_series(double x) {
  double x2 = x * x, t = 1.0, s = 1.0;
  for (int i = 1; i < 14; ++i) {
    t *= -x2 / ((2.0 * i - 1.0) * (2.0 * i));
    s += t;
  }
  return s;
}

constexpr CDouble unit_root(long m, long n) {
  m %= n;
  if (m < 0) m += n;
  const long q = (4 * m) / n;      // quarter turns
  const long r = 4 * m - q * n;    // remainder, angle (pi/2) r / n in [0, pi/2)
  const bool comp = 2 * r > n;
  const double a = comp ? (kPiD / 2) * (double)(n - r) / (double)n : (kPiD / 2) * (double)r / (double)n;
  double c = cos_series(a), s = sin_series(a);
  if (comp) {
    const double t = c;
    c = s;
    s = t;
  }
  CDouble v{c, s};
  for (long i = 0; i < q; ++i) v = CDouble{-v.im, v.re};
  return v;
}

// ---------------------------------------------------------------------------
// compile-time loop
// ---------------------------------------------------------------------------
template <int I, int E, class F>
CGH_HD void static_for(F &&f) {
  if constexpr (I < E) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, E>(f);
  }
}

// x * exp(DIR 2 pi i M / N) with M, N compile-time
template <int N, int DIR, int M>
CGH_HD float2 twiddle_const(float2 x) {
  constexpr int m = ((M % N) + N) % N;
  if constexpr (m == 0) {
    return x;
  } else if constexpr (4 * m == N) {
    return rot90<DIR>(x);
  } else if constexpr (2 * m == N) {
    return cneg(x);
  } else if constexpr (4 * m == 3 * N) {
    return rot90<-DIR>(x);
  } else {
    constexpr CDouble w = unit_root((long)DIR * m, N);
    return cmul(x, make_float2((float)w.re, (float)w.im));
  }
}

// ---------------------------------------------------------------------------
// base DFTs: y_k = sum_q x_q exp(DIR 2 pi i q k / R)
// ---------------------------------------------------------------------------
template <int R, int DIR>
struct Dft;

template <int DIR>
struct Dft<2, DIR> {
  static CGH_HD void run(float2 *x) {
    float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <int DIR>
struct Dft<3, DIR> {
  static CGH_HD void run(float2 *x) {
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
  static CGH_HD void run(float2 *x) {
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
  static CGH_HD void run(float2 *x) {
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
  static CGH_HD void run(float2 *x) {
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

// ---------------------------------------------------------------------------
// composite register DFT
// ---------------------------------------------------------------------------
constexpr bool is_base_radix(int n) { return n == 2 || n == 3 || n == 4 || n == 5 || n == 8; }

constexpr int base_factor(int n) {
  // first factor of a composite length: a power-of-two part up to 8 if present,
  // otherwise 5, then 3
  if (n % 8 == 0 && n != 8) return 8;
  if (n % 4 == 0 && n != 4) return 4;
  if (n % 2 == 0 && n != 2) return 2;
  if (n % 5 == 0 && n != 5) return 5;
  return 3;
}

constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }
// multiplicative inverse of a modulo m (m > 1, gcd(a, m) = 1)
constexpr int inv_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 0;
}

template <int N, int DIR>
struct RFft {
  static CGH_HD void run(float2 *x) {
    if constexpr (N == 1) {
    } else if constexpr (is_base_radix(N)) {
      Dft<N, DIR>::run(x);
    } else if constexpr (gcd_c(base_factor(N), N / base_factor(N)) == 1) {
      // coprime factors: prime-factor (Good-Thomas) split, no twiddles.
      // Input n = (N2 n1 + N1 n2) mod N; output k = (N2 a k1 + N1 b k2) mod N
      // with a = N2^-1 mod N1, b = N1^-1 mod N2; then exp(2 pi i n k / N)
      // factors into exp(2 pi i n1 k1 / N1) exp(2 pi i n2 k2 / N2).
      constexpr int N1 = base_factor(N);
      constexpr int N2 = N / N1;
      constexpr int A = inv_mod(N2 % N1, N1), B = inv_mod(N1 % N2, N2);
      float2 t[N];
      static_for<0, N1>([&](auto n1c) {
        constexpr int n1 = decltype(n1c)::value;
        float2 u[N2];
        static_for<0, N2>([&](auto n2c) {
          constexpr int n2 = decltype(n2c)::value;
          u[n2] = x[(N2 * n1 + N1 * n2) % N];
        });
        RFft<N2, DIR>::run(u);
        static_for<0, N2>([&](auto k2c) {
          constexpr int k2 = decltype(k2c)::value;
          t[n1 * N2 + k2] = u[k2];
        });
      });
      static_for<0, N2>([&](auto k2c) {
        constexpr int k2 = decltype(k2c)::value;
        float2 v[N1];
        static_for<0, N1>([&](auto n1c) {
          constexpr int n1 = decltype(n1c)::value;
          v[n1] = t[n1 * N2 + k2];
        });
        RFft<N1, DIR>::run(v);
        static_for<0, N1>([&](auto k1c) {
          constexpr int k1 = decltype(k1c)::value;
          x[(N2 * A * k1 + N1 * B * k2) % N] = v[k1];
        });
      });
    } else {
      constexpr int N1 = base_factor(N);
      constexpr int N2 = N / N1;
      float2 t[N];
      static_for<0, N2>([&](auto n2c) {
        constexpr int n2 = decltype(n2c)::value;
        float2 s[N1];
        static_for<0, N1>([&](auto n1c) {
          constexpr int n1 = decltype(n1c)::value;
          s[n1] = x[N2 * n1 + n2];
        });
        Dft<N1, DIR>::run(s);
        static_for<0, N1>([&](auto k1c) {
          constexpr int k1 = decltype(k1c)::value;
          t[k1 * N2 + n2] = twiddle_const<N, DIR, n2 * k1>(s[k1]);
        });
      });
      static_for<0, N1>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        float2 u[N2];
        static_for<0, N2>([&](auto n2c) {
          constexpr int n2 = decltype(n2c)::value;
          u[n2] = t[k1 * N2 + n2];
        });
        RFft<N2, DIR>::run(u);
        static_for<0, N2>([&](auto k2c) {
          constexpr int k2 = decltype(k2c)::value;
          x[k1 + N1 * k2] = u[k2];
        });
      });
    }
  }
};

// ---------------------------------------------------------------------------
// compile-time Stockham plan: radices chosen greedily from the list below
// (fewest LDS passes with at most 16 values per butterfly), then ordered odd
// radices first: the first stage writes at stride R, and an odd stride
// spreads those writes over the LDS banks where a power of two would not.
// ---------------------------------------------------------------------------
constexpr int pick_radix(int n) {
  constexpr int cand[] = {16, 15, 12, 10, 9, 8, 6, 5, 4, 3, 2};
  for (int r : cand)
    if (n % r == 0) return r;
  return n;
}

// Measured plans that replace the greedy one for some lengths (n = 0: none).
// With four chains over 512 threads a stage of radix R has 4 N / R
// butterflies, one or more per thread.  For 960 the greedy 15 16 4 has a
// radix-16 stage with 240 butterflies (half the threads idle) and two
// radix-4 passes; 15 8 8 (256, 480, 480 butterflies) shortens the chain each
// thread runs between barriers (row passes 36.7 -> 35.6 us, loss row pass
// 65.3 -> 61.8 us at 1080p; 12 8 10, 8 12 10 and 10 12 8 were in between).
template <int N>
struct CPlanFixed {
  static constexpr int n = 0;
  static constexpr int r[1] = {1};
};
template <>
struct CPlanFixed<960> {
  static constexpr int n = 3;
  static constexpr int r[3] = {15, 8, 8};
};
// The serving pads' quarter rows (1024, 512, 256) likewise: greedy 16 16 4,
// 16 16 2 and 16 16 leave 3/4 to 7/8 of the threads idle in their radix-16
// stages; 8 8 16, 8 8 8 and 4 8 8 cut the batched solves of the 512^2,
// 768x1024 and 1024^2 classes by 8, 7 and 3 %.
template <>
struct CPlanFixed<1024> {
  static constexpr int n = 3;
  static constexpr int r[3] = {8, 8, 16};
};
template <>
struct CPlanFixed<512> {
  static constexpr int n = 3;
  static constexpr int r[3] = {8, 8, 8};
};
template <>
struct CPlanFixed<256> {
  static constexpr int n = 3;
  static constexpr int r[3] = {4, 8, 8};
};

template <int N>
struct CPlan {
  static constexpr int greedy(int s) {
    int n = N;
    for (int i = 0; i < s; ++i) n /= pick_radix(n);
    return pick_radix(n);
  }
  static constexpr int stages() {
    if (CPlanFixed<N>::n) return CPlanFixed<N>::n;
    int n = N, s = 0;
    while (n > 1) {
      n /= pick_radix(n);
      ++s;
    }
    return s;
  }
  // s-th radix after moving the odd radices (in greedy order) to the front
  static constexpr int radix(int s) {
    if (CPlanFixed<N>::n) return CPlanFixed<N>::r[s];
    int k = 0;
    for (int i = 0; i < stages(); ++i)
      if (greedy(i) % 2 == 1 && k++ == s) return greedy(i);
    for (int i = 0; i < stages(); ++i)
      if (greedy(i) % 2 == 0 && k++ == s) return greedy(i);
    return 1;
  }
  static constexpr int ns(int s) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= radix(i);
    return p;
  }
};

// Workgroup barrier that orders LDS only: wait for this wave's LDS operations,
// then s_barrier.  Unlike __syncthreads() it does not wait for outstanding
// global memory operations (such as a prefetch streaming into another LDS
// buffer, or stores that nothing in the workgroup reads back).
__device__ __forceinline__ void lds_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// One compile-time Stockham stage over B interleaved transforms in LDS
// (element (r, b) at buf[r * B + b]); stage twiddles exp(DIR 2 pi i q k / (Ns R))
// read from the full length-N table tw[e] = exp(-2 pi i e / N) in LDS.
template <int R, int DIR, int B, int T, int N, int NS>
__device__ __forceinline__ void cstage(float2 *__restrict__ buf, const float2 *__restrict__ tw,
                                       int tid) {
  constexpr int NB = N / R;
  constexpr int ITEMS = NB * B;
  constexpr int MAXIT = (ITEMS + T - 1) / T;
  constexpr int TWS = N / (NS * R);
  float2 v[MAXIT][R];
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int i = tid + it * T;
    if (ITEMS % T == 0 || i < ITEMS) {
      const int b = i % B, j = i / B;
      static_for<0, R>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        v[it][q] = buf[(j + q * NB) * B + b];
      });
      if constexpr (NS > 1) {
        const int e = (j % NS) * TWS;
        static_for<1, R>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          float2 w = tw[q * e];
          if constexpr (DIR > 0) w.y = -w.y;
          v[it][q] = cmul(v[it][q], w);
        });
      }
      RFft<R, DIR>::run(v[it]);
    }
  }
  lds_sync();
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int i = tid + it * T;
    if (ITEMS % T == 0 || i < ITEMS) {
      const int b = i % B, j = i / B;
      const int base = (j / NS) * NS * R + (j % NS);
      static_for<0, R>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        buf[(base + q * NS) * B + b] = v[it][q];
      });
    }
  }
  lds_sync();
}

// Same stage with twiddles from a two-level table (hi[e >> 6] lo[e & 63]),
// for lengths whose full table does not fit beside the data.
template <int R, int DIR, int B, int T, int N, int NS, class TW>
__device__ __forceinline__ void cstage2(float2 *__restrict__ buf, const TW &tw, int tid) {
  constexpr int NB = N / R;
  constexpr int ITEMS = NB * B;
  constexpr int MAXIT = (ITEMS + T - 1) / T;
  constexpr int TWS = N / (NS * R);
  float2 v[MAXIT][R];
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int i = tid + it * T;
    if (ITEMS % T == 0 || i < ITEMS) {
      const int b = i % B, j = i / B;
      static_for<0, R>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        v[it][q] = buf[(j + q * NB) * B + b];
      });
      if constexpr (NS > 1) {
        const int e = (j % NS) * TWS;
        static_for<1, R>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          const int eq = q * e;
          float2 w = cmul(tw.hi[eq >> 6], tw.lo[eq & 63]);
          if constexpr (DIR > 0) w.y = -w.y;
          v[it][q] = cmul(v[it][q], w);
        });
      }
      RFft<R, DIR>::run(v[it]);
    }
  }
  lds_sync();
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int i = tid + it * T;
    if (ITEMS % T == 0 || i < ITEMS) {
      const int b = i % B, j = i / B;
      const int base = (j / NS) * NS * R + (j % NS);
      static_for<0, R>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        buf[(base + q * NS) * B + b] = v[it][q];
      });
    }
  }
  lds_sync();
}

// Orders this wave's LDS accesses before and after it (compiler barrier only):
// LDS operations of one wave execute in issue order, so a wave that alone owns
// a buffer needs no workgroup barrier between the stages of its transform.
__device__ __forceinline__ void wave_lds_order() { asm volatile("" ::: "memory"); }

// One Stockham stage of a length-N transform owned by a single wave: the
// buffer buf[0, N) is contiguous in LDS and lane l takes butterflies
// j = l, l + 64, ...  Same index scheme and twiddles as cstage with B = 1.
// The stage input element i comes from ld(i) (the buffer itself, or global
// memory for a first stage); the output goes to the buffer.
template <int R, int DIR, int N, int NS, class LD>
__device__ __forceinline__ void wstage_ld(float2 *__restrict__ buf, const float2 *__restrict__ tw,
                                          int lane, LD &&ld) {
  constexpr int NB = N / R;
  constexpr int IT = (NB + 63) / 64;
  constexpr int TWS = N / (NS * R);
  float2 v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int j = lane + 64 * it;
    if ((it + 1) * 64 <= NB || j < NB) {
      static_for<0, R>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        v[it][q] = ld(j + q * NB);
      });
      if constexpr (NS > 1) {
        const int e = (j % NS) * TWS;
        static_for<1, R>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          float2 w = tw[q * e];
          if constexpr (DIR > 0) w.y = -w.y;
          v[it][q] = cmul(v[it][q], w);
        });
      }
      RFft<R, DIR>::run(v[it]);
    }
  }
  wave_lds_order();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int j = lane + 64 * it;
    if ((it + 1) * 64 <= NB || j < NB) {
      const int k = j % NS;
      const int base = (j - k) * R + k;
      static_for<0, R>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        buf[base + q * NS] = v[it][q];
      });
    }
  }
  wave_lds_order();
}

template <int R, int DIR, int N, int NS>
__device__ __forceinline__ void wstage(float2 *__restrict__ buf, const float2 *__restrict__ tw,
                                       int lane) {
  wstage_ld<R, DIR, N, NS>(buf, tw, lane, [&](int i) { return buf[i]; });
}

template <int DIR, int B, int T, int N, class TW, int S = 0>
__device__ __forceinline__ void cfft2(float2 *__restrict__ buf, const TW &tw, int tid) {
  if constexpr (S < CPlan<N>::stages()) {
    cstage2<CPlan<N>::radix(S), DIR, B, T, N, CPlan<N>::ns(S)>(buf, tw, tid);
    cfft2<DIR, B, T, N, TW, S + 1>(buf, tw, tid);
  }
}

template <int DIR, int B, int T, int N, int S = 0>
__device__ __forceinline__ void cfft(float2 *__restrict__ buf, const float2 *__restrict__ tw,
                                     int tid) {
  if constexpr (S < CPlan<N>::stages()) {
    cstage<CPlan<N>::radix(S), DIR, B, T, N, CPlan<N>::ns(S)>(buf, tw, tid);
    cfft<DIR, B, T, N, S + 1>(buf, tw, tid);
  }
}

}  // namespace cgh
