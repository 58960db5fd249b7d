// Kernels of the learned initialiser's U-Net (include/cgh_net.h): 3x3
// convolutions as implicit GEMMs on the matrix cores (BF16 inputs, FP32
// sums), their weight gradients, and the pooling, upsampling, ReLU and
// lattice glue around them.
//
// Matrix instructions (one wave, D = A B + D, D 32 x 32 FP32): in
// v_mfma_f32_32x32x8 bf16 (A 32 x 8, B 8 x 32) lane l supplies
// A[l % 32][4 (l / 32) + i] and B[4 (l / 32) + i][l % 32] (i < 4); in
// v_mfma_f32_32x32x16 bf16 (A 32 x 16, B 16 x 32) it supplies
// A[l % 32][8 (l / 32) + i] and B[8 (l / 32) + i][l % 32] (i < 8).  Both leave
// D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32] in accumulator v < 16.
#include <algorithm>
#include <cmath>

#include "cgh_internal.h"
#include "cgh_net.h"

namespace cgh {
namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);  // nearest, ties to even
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

bool al16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// eight consecutive channels (16 bytes) of the convolution input at (y, x),
// channel c0 (a multiple of 8) of [up(x1), x2]; zero outside the image and at
// c0 >= c1 + c2 (the upper half of a last, half-filled block of 16)
__device__ __forceinline__ v8s conv_in8(const uint16_t *__restrict__ x1, int c1, int up,
                                        const uint16_t *__restrict__ x2, int c2, int H, int W,
                                        int y, int x, int c0) {
  v8s r = {0, 0, 0, 0, 0, 0, 0, 0};
  if (y < 0 || y >= H || x < 0 || x >= W || c0 >= c1 + c2) return r;
  const uint16_t *src;
  if (c0 < c1) {
    src = up ? x1 + ((size_t)(y >> 1) * (W >> 1) + (x >> 1)) * c1 + c0
             : x1 + ((size_t)y * W + x) * c1 + c0;
  } else {
    src = x2 + ((size_t)y * W + x) * c2 + (c0 - c1);
  }
  return *reinterpret_cast<const v8s *>(src);
}

// ----------------------------------------------------------------------------
// Convolution: a workgroup of NWV waves takes 32 NWV consecutive pixels
// (row-major) p0 .. p0 + 32 NWV - 1 and 32 NB output channels.  For each
// block of 16 input channels it stages in LDS the three input row segments
// that the 3 x 3 taps of its pixels read (pixels p0 + (ky - 1) W - 1 ..
// p0 + (ky - 1) W + 32 NWV, ky < 3, zero outside the image) and the weights
// of its output channels for the 9 taps; wave w then takes its 32 pixels x
// 32 NB channels through the 9 taps from LDS.  A tap that leaves the image (a pixel in the first or last
// column or row) reads zero.  With one output block (NB = 1) each input
// block's global loads are issued before the workgroup waits for the previous
// block's products; with two or four, the loads of block k + 1 are issued
// before the products of block k.
// ----------------------------------------------------------------------------

// waves (of 32 pixels each) per convolution workgroup: 8 halves the weight
// traffic and the halo per pixel against 4 (16 was slower at every width)
constexpr int kConvWaves = 8;

// Workgroups are handed to the 8 XCDs in turn (block b to XCD b % 8).  This
// bijection on [0, nb) gives XCD x one contiguous run of pixel blocks, taken
// in order, so the three workgroups that read one input row (the blocks one
// image row above and below) run on the same XCD and share its L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

template <int NB, int NWV>
__global__ __launch_bounds__(64 * NWV) void k_conv3x3(
    const uint16_t *__restrict__ x1, int c1, int up, const uint16_t *__restrict__ x2, int c2,
    int H, int W, const uint16_t *__restrict__ w, const float *__restrict__ bias, int cout,
    int relu, float *__restrict__ out32, uint16_t *__restrict__ out16) {
  constexpr int CO = 32 * NB, NT = 64 * NWV, PX = 32 * NWV;
  constexpr int kSeg = PX + 2;  // pixels per staged row segment: one more on each side
  constexpr int NA = 3 * kSeg * 2, NW = 9 * CO * 2;  // 16-byte items: [ky][pixel][half], [t][co][half]
  constexpr int KA = (NA + NT - 1) / NT, KW = (NW + NT - 1) / NT;
  // the staged operands; after the products the same memory holds the
  // output tile [PX][32] (FP32) of one output block for the store
  static_assert((NA + NW) * 16 >= PX * 32 * 4, "output tile fits the staging memory");
  __shared__ v8s smem[NA + NW];
  v8s *const sa = smem, *const sw = smem + NA;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int P = H * W, cin = c1 + c2;
  const int pb = xcd_block(blockIdx.x, gridDim.x);
  const int p0 = pb * PX;
  const int i = wave * 32 + (lane & 31);  // this lane's A row: pixel p0 + i
  const int half = lane >> 5;             // its 8 channels of a block of 16
  const int p = p0 + i;
  const int co0 = blockIdx.y * CO;
  const int px = p - (p / W) * W;  // this lane's pixel column
  const int nk = (cin + 15) / 16;  // channel blocks (a last block of 8 is zero-filled)
  const v8s z = {0, 0, 0, 0, 0, 0, 0, 0};
  v16f acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[b][v] = 0.f;
  // The source of each staged item, worked out once: A item k is channel
  // ah[k] + 16 kb of pixel q2[k] (q1[k] in x1, which may be the half-size
  // image), or zero (q2[k] < 0); B item k is channel 8 (wo[k] & 1) + 16 kb of
  // weight row wo[k] >> 1 (an element offset), or zero (wo[k] < 0).
  int q2[KA], q1[KA], ah[KA], wo[KW];
#pragma unroll
  for (int k = 0; k < KA; ++k) {
    const int item = tid + NT * k;
    q2[k] = -1;
    q1[k] = 0;
    ah[k] = 0;
    if (KA * NT == NA || item < NA) {
      const int seg = item / (2 * kSeg), rem = item - seg * (2 * kSeg);
      const int q = p0 + (seg - 1) * W - 1 + (rem >> 1);
      ah[k] = 8 * (rem & 1);
      if (q >= 0 && q < P) {
        const int qy = q / W, qx = q - qy * W;
        q2[k] = q;
        q1[k] = up ? (qy >> 1) * (W >> 1) + (qx >> 1) : q;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < KW; ++k) {
    const int item = tid + NT * k;
    wo[k] = -1;
    if (KW * NT == NW || item < NW) {
      const int t = item / (2 * CO), rem = item - t * (2 * CO);
      const int co = co0 + (rem >> 1);
      if (co < cout) wo[k] = 2 * ((co * 9 + t) * cin) + (rem & 1);
    }
  }
  // block kb of 16 input channels: its staged A and B items, global -> registers
  v8s ra[KA], rw[KW];
  auto fetch = [&](int kb) {
#pragma unroll
    for (int k = 0; k < KA; ++k) {
      const int c0 = kb * 16 + ah[k];
      ra[k] = z;
      if (q2[k] >= 0 && c0 < cin) {
        const uint16_t *src = c0 < c1 ? x1 + (size_t)q1[k] * c1 + c0
                                      : x2 + (size_t)q2[k] * c2 + (c0 - c1);
        ra[k] = *reinterpret_cast<const v8s *>(src);
      }
    }
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      rw[k] = z;
      const int c0 = kb * 16 + 8 * (wo[k] & 1);
      if (wo[k] >= 0 && c0 < cin)
        rw[k] = *reinterpret_cast<const v8s *>(w + (size_t)(wo[k] >> 1) + c0);
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int k = 0; k < KA; ++k)
      if (KA * NT == NA || tid + NT * k < NA) sa[tid + NT * k] = ra[k];
#pragma unroll
    for (int k = 0; k < KW; ++k)
      if (KW * NT == NW || tid + NT * k < NW) sw[tid + NT * k] = rw[k];
  };
  // A tap above the first or below the last row reads a staged zero (its
  // linear pixel index is outside [0, P)) unless it also leaves the image at
  // the side; a tap that leaves at the side reads the neighbouring row's end
  // pixel in the staged segment, so it is masked here.  Outputs past P are
  // not stored.
  const bool in_l = px != 0, in_r = px != W - 1;
  auto products = [&]() {
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int ky = t / 3, kx = t - 3 * ky;
      const v8s sv = sa[(ky * kSeg + i + kx) * 2 + half];
      const v8s a = kx == 0 ? (in_l ? sv : z) : (kx == 2 ? (in_r ? sv : z) : sv);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const v8s bb = sw[(t * CO + 32 * b + (lane & 31)) * 2 + half];
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a),
                                                         __builtin_bit_cast(v8bf, bb), acc[b],
                                                         0, 0, 0);
      }
    }
  };
  if constexpr (NB == 1) {
    // each block's loads are issued before the workgroup waits for the
    // previous block's products
    for (int kb = 0; kb < nk; ++kb) {
      fetch(kb);
      if (kb > 0) __syncthreads();  // every wave is done with the previous block
      stage();
      __syncthreads();
      products();
    }
  } else {
    // the loads of block kb + 1 are issued before the products of block kb
    // (more registers: faster where 2 or 4 output blocks give the products
    // enough length to cover them, slower with one)
    fetch(0);
    stage();
    __syncthreads();
    for (int kb = 0; kb < nk; ++kb) {
      if (kb + 1 < nk) fetch(kb + 1);
      products();
      if (kb + 1 < nk) {
        __syncthreads();  // every wave is done with this block
        stage();
        __syncthreads();
      }
    }
  }
  // Store, one output block at a time: the accumulators (lane l holds output
  // channel l % 32 of 16 pixels) go through LDS as a [pixel][channel] FP32
  // tile, which each thread then reads and writes 16 bytes at a time.
  float *tile = reinterpret_cast<float *>(smem);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int cb = co0 + 32 * b;  // first output channel of the block
    {
      const int col = lane & 31;
      const float bv = (bias && cb + col < cout) ? bias[cb + col] : 0.f;
      __syncthreads();  // every wave is done with the staged operands (or the previous tile)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = wave * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        tile[row * 32 + col] = acc[b][v] + bv;
      }
      __syncthreads();
    }
    if (out32) {
      // 8 chunks of 4 channels per pixel
      for (int c = tid; c < PX * 8; c += NT) {
        const int row = c >> 3, part = c & 7, q = p0 + row, co = cb + 4 * part;
        if (q < P && co < cout) {
          // cout is a multiple of 8, so the 4 channels are all below cout
          *reinterpret_cast<float4 *>(out32 + (size_t)q * cout + co) =
              *reinterpret_cast<const float4 *>(tile + row * 32 + 4 * part);
        }
      }
    }
    if (out16) {
      // 4 chunks of 8 channels per pixel (cout is a multiple of 8)
      for (int c = tid; c < PX * 4; c += NT) {
        const int row = c >> 2, part = c & 3, q = p0 + row, co = cb + 8 * part;
        if (q < P && co < cout) {
          const float4 u0 = *reinterpret_cast<const float4 *>(tile + row * 32 + 8 * part);
          const float4 u1 = *reinterpret_cast<const float4 *>(tile + row * 32 + 8 * part + 4);
          const float f[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
          v8s o;
#pragma unroll
          for (int e = 0; e < 8; ++e) o[e] = (short)to_bf16(relu ? fmaxf(f[e], 0.f) : f[e]);
          *reinterpret_cast<v8s *>(out16 + (size_t)q * cout + co) = o;
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------
// Weight gradient: gw[co][t][ci] (tap t = 3 ky + kx) = sum_p gy[p][co]
// in[p + k(t) - 1][ci], a GEMM whose reduction runs over pixels.  Both operands
// are first copied channel-major, so that a lane's eight consecutive pixels of
// one channel are one aligned 16-byte load (Wr = W rounded up to 16):
//   gyT[co][y][x]      = gy[y][x][co]                (x < Wr; zero for x >= W)
//   ink[kx][ci][yy][x] = in[yy - 1][x + kx - 1][ci]  (yy < H + 2; zero outside)
// Tap (ky, kx) of output pixel (y, x) then reads ink[kx][ci][y + ky][x] with no
// border test.  One wave takes 32 output channels x 32 input channels, all nine
// taps, over a range of 16-pixel row chunks (v_mfma_f32_32x32x16 bf16, K = the
// chunk's pixels), and writes FP32 partials for its range; the bias gradient
// rides along in the waves of the first input-channel block.
// ----------------------------------------------------------------------------

// gyT: a workgroup transposes one row y, 64 columns and 32 channels through LDS
__global__ __launch_bounds__(256) void k_wg_gyT(const uint16_t *__restrict__ gy, int H, int W,
                                                int Wr, int cout, uint16_t *__restrict__ gyT) {
  __shared__ uint16_t tile[64][33];
  const int tid = threadIdx.x;
  const int y = blockIdx.y, x0 = blockIdx.x * 64, co0 = blockIdx.z * 32;
  {
    const int px = tid >> 2, g = tid & 3, x = x0 + px, co = co0 + 8 * g;
    v8s v = {0, 0, 0, 0, 0, 0, 0, 0};
    if (x < W && co < cout) v = *reinterpret_cast<const v8s *>(gy + ((size_t)y * W + x) * cout + co);
#pragma unroll
    for (int i = 0; i < 8; ++i) tile[px][8 * g + i] = (uint16_t)v[i];
  }
  __syncthreads();
  {
    const int co = tid >> 3, seg = tid & 7, x = x0 + 8 * seg;
    if (co0 + co < cout && x < Wr) {
      v8s v;
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = (short)tile[8 * seg + i][co];
      *reinterpret_cast<v8s *>(gyT + ((size_t)(co0 + co) * H + y) * Wr + x) = v;
    }
  }
}

// ink: a workgroup builds row yy (< H + 2) of the three shifted copies for 64
// columns and 32 channels from source columns x0 - 1 .. x0 + 64 staged in LDS
__global__ __launch_bounds__(256) void k_wg_ink(const uint16_t *__restrict__ x1, int c1, int up,
                                                const uint16_t *__restrict__ x2, int c2, int H,
                                                int W, int Wr, uint16_t *__restrict__ ink) {
  __shared__ uint16_t tile[66][33];
  const int tid = threadIdx.x;
  const int yy = blockIdx.y, x0 = blockIdx.x * 64, ci0 = blockIdx.z * 32;
  const int cin = c1 + c2;
  for (int item = tid; item < 66 * 4; item += 256) {
    const int col = item >> 2, g = item & 3;
    // conv_in8 is zero outside the image and past the last channel
    const v8s v = conv_in8(x1, c1, up, x2, c2, H, W, yy - 1, x0 - 1 + col, ci0 + 8 * g);
#pragma unroll
    for (int i = 0; i < 8; ++i) tile[col][8 * g + i] = (uint16_t)v[i];
  }
  __syncthreads();
  for (int item = tid; item < 3 * 256; item += 256) {
    const int kx = item >> 8, r = item & 255, ci = r >> 3, seg = r & 7, x = x0 + 8 * seg;
    if (ci0 + ci < cin && x < Wr) {
      v8s v;
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = (short)tile[8 * seg + i + kx][ci];  // column x + i + kx - 1
      *reinterpret_cast<v8s *>(ink + (((size_t)kx * cin + ci0 + ci) * (H + 2) + yy) * Wr + x) = v;
    }
  }
}

__global__ __launch_bounds__(64) void k_conv3x3_wgrad(const uint16_t *__restrict__ gyT,
                                                      const uint16_t *__restrict__ ink, int H,
                                                      int Wr, int cin, int cout, int cps,
                                                      int nchunks, float *__restrict__ part,
                                                      float *__restrict__ part_b) {
  const int lane = threadIdx.x, half = lane >> 5;
  const int cib = blockIdx.x, cob = blockIdx.y, s = blockIdx.z;
  const int N = 9 * cin, cw = Wr / 16;
  const int co = cob * 32 + (lane & 31), ci = cib * 32 + (lane & 31);
  const bool cov = co < cout, civ = ci < cin;
  const uint16_t *arow = gyT + (size_t)(cov ? co : 0) * H * Wr;
  const uint16_t *brow = ink + (size_t)(civ ? ci : 0) * (H + 2) * Wr;
  const size_t kstride = (size_t)cin * (H + 2) * Wr;  // between the kx copies
  const v8s z = {0, 0, 0, 0, 0, 0, 0, 0};
  v16f acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[t][v] = 0.f;
  float bsum = 0.f;
  const int cbeg = s * cps, cend = min(nchunks, cbeg + cps);
  for (int c = cbeg; c < cend; ++c) {
    const int y = c / cw, x = (c - y * cw) * 16 + 8 * half;
    const v8s a = cov ? *reinterpret_cast<const v8s *>(arow + (size_t)y * Wr + x) : z;
    v8s b[9];
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int kx = 0; kx < 3; ++kx)
        b[3 * ky + kx] =
            civ ? *reinterpret_cast<const v8s *>(brow + kx * kstride + (size_t)(y + ky) * Wr + x)
                : z;
    if (cib == 0) {
#pragma unroll
      for (int i = 0; i < 8; ++i) bsum += from_bf16((uint16_t)a[i]);
    }
#pragma unroll
    for (int t = 0; t < 9; ++t)
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a),
                                                       __builtin_bit_cast(v8bf, b[t]), acc[t], 0,
                                                       0, 0);
  }
  // D[row = co][col = ci] of tap t
  float *dst = part + (size_t)s * cout * N;
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = cob * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
      if (civ && r < cout) dst[(size_t)r * N + t * cin + ci] = acc[t][v];
    }
  if (cib == 0) {
    // lanes l and l + 32 hold the two halves of the pixels of channel co
    bsum += __shfl_down(bsum, 32, 64);
    if (lane < 32 && cov) part_b[(size_t)s * cout + co] = bsum;
  }
}

// fixed-order sum over the splits: a workgroup takes 16 outputs with 16 lanes
// each; lane g of an output adds splits g, g + 16, ... in order, then one lane
// adds the 16 lane sums in order.  Outputs i < len are the weight gradients;
// the workgroups with i < cout also sum the bias partials the same way.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *__restrict__ part,
                                                      const float *__restrict__ part_b,
                                                      int splits, int64_t len, int cout,
                                                      float *__restrict__ gw,
                                                      float *__restrict__ gb) {
  __shared__ float red[16][17];
  const int o = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int64_t i = (int64_t)blockIdx.x * 16 + o;
  float s = 0.f;
  if (i < len)
    for (int k = g; k < splits; k += 16) s += part[(size_t)k * len + i];
  red[g][o] = s;
  __syncthreads();
  if (g == 0 && i < len) {
    float t = 0.f;
    for (int q = 0; q < 16; ++q) t += red[q][o];
    gw[i] = t;
  }
  if (gb == nullptr || (int64_t)blockIdx.x * 16 >= cout) return;  // uniform per workgroup
  __syncthreads();
  s = 0.f;
  if (i < cout)
    for (int k = g; k < splits; k += 16) s += part_b[(size_t)k * cout + i];
  red[g][o] = s;
  __syncthreads();
  if (g == 0 && i < cout) {
    float t = 0.f;
    for (int q = 0; q < 16; ++q) t += red[q][o];
    gb[i] = t;
  }
}

__global__ void k_flip(const uint16_t *__restrict__ w, int cout, int cin,
                       uint16_t *__restrict__ wt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // over wt: [cin][9][cout]
  if (i >= cout * 9 * cin) return;
  const int co = i % cout, t = (i / cout) % 9, ci = i / (9 * cout);
  wt[i] = w[((size_t)co * 9 + (8 - t)) * cin + ci];  // (ky, kx) -> (2 - ky, 2 - kx)
}

__global__ void k_cast(const float *__restrict__ x, int64_t n, uint16_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = to_bf16(x[i]);
}

__global__ void k_relu_grad(const float *__restrict__ g, const uint16_t *__restrict__ a,
                            int64_t n, uint16_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = to_bf16((a == nullptr || from_bf16(a[i]) > 0.f) ? g[i] : 0.f);
}

__global__ void k_pool2(const uint16_t *__restrict__ x, int H, int W, int C,
                        uint16_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int Ho = H / 2, Wo = W / 2;
  if (i >= (int64_t)Ho * Wo * C) return;
  const int c = (int)(i % C);
  const int64_t q = i / C;
  const int y = (int)(q / Wo), xo = (int)(q - (int64_t)y * Wo);
  const uint16_t *s = x + ((size_t)(2 * y) * W + 2 * xo) * C + c;
  const float v = (from_bf16(s[0]) + from_bf16(s[C])) +
                  (from_bf16(s[(size_t)W * C]) + from_bf16(s[(size_t)W * C + C]));
  out[i] = to_bf16(0.25f * v);
}

__global__ void k_up_adjoint(const float *__restrict__ g, int H, int W, int stride, int C,
                             float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int Ho = H / 2, Wo = W / 2;
  if (i >= (int64_t)Ho * Wo * C) return;
  const int c = (int)(i % C);
  const int64_t q = i / C;
  const int y = (int)(q / Wo), x = (int)(q - (int64_t)y * Wo);
  const float *s = g + ((size_t)(2 * y) * W + 2 * x) * stride + c;
  out[i] = (s[0] + s[stride]) + (s[(size_t)W * stride] + s[(size_t)W * stride + stride]);
}

__global__ void k_grad_combine(const float *__restrict__ gp, const float *__restrict__ gs,
                               int stride, int off, int H, int W, int C,
                               float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)H * W * C) return;
  const int c = (int)(i % C);
  const int64_t q = i / C;
  const int y = (int)(q / W), x = (int)(q - (int64_t)y * W);
  float v = 0.f;
  if (gp) v = 0.25f * gp[((size_t)(y >> 1) * (W >> 1) + (x >> 1)) * C + c];
  if (gs) v += gs[(size_t)q * stride + off + c];
  out[i] = v;
}

// lattice point k = i gx + j: centre in FP64, its pixel
__device__ __forceinline__ void lattice_point(int k, int H, int W, int gy, int gx, double &cy,
                                              double &cx, int &iy, int &ix) {
  const int i = k / gx, j = k - i * gx;
  cy = (i + 0.5) * (double)H / gy;
  cx = (j + 0.5) * (double)W / gx;
  iy = (int)floor(cy);
  ix = (int)floor(cx);
}

constexpr double kLogScale0 = 0.69314718055994530942;  // ln 2
constexpr double kAmp0 = 0.5, kOpacity0 = -0.5;

__global__ void k_lattice_gather(const float *__restrict__ net, int H, int W, int gy, int gx,
                                 int C, float *__restrict__ params) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = gy * gx;
  if (k >= n) return;
  double cy, cx;
  int iy, ix;
  lattice_point(k, H, W, gy, gx, cy, cx, iy, ix);
  const float *o = net + ((size_t)iy * W + ix) * 8 * C;
  const double mx = fmin(fmax(cx + (double)o[0], 1e-3), W - 1e-3);
  const double my = fmin(fmax(cy + (double)o[1], 1e-3), H - 1e-3);
  // flat layout: mean_pre [n][2], log_scale [n][2], rotation [n], amplitude [n][C],
  // phase [n][C], opacity_pre [n]; colour c from output block c
  params[2 * k] = (float)atanh(2.0 * mx / W - 1.0);
  params[2 * k + 1] = (float)atanh(2.0 * my / H - 1.0);
  params[2 * (size_t)n + 2 * k] = (float)((double)o[2] + kLogScale0);
  params[2 * (size_t)n + 2 * k + 1] = (float)((double)o[3] + kLogScale0);
  params[4 * (size_t)n + k] = o[4];
  for (int c = 0; c < C; ++c) {
    params[5 * (size_t)n + (size_t)k * C + c] = (float)((double)o[8 * c + 5] + kAmp0);
    params[(size_t)(5 + C) * n + (size_t)k * C + c] = o[8 * c + 6];
  }
  params[(size_t)(5 + 2 * C) * n + k] = (float)((double)o[7] + kOpacity0);
}

__global__ void k_fill0(float *__restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.f;
}

__global__ void k_lattice_scatter(const float *__restrict__ net, const float *__restrict__ g,
                                  int H, int W, int gy, int gx, int C,
                                  float *__restrict__ gnet) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = gy * gx;
  if (k >= n) return;
  double cy, cx;
  int iy, ix;
  lattice_point(k, H, W, gy, gx, cy, cx, iy, ix);
  const float *o = net + ((size_t)iy * W + ix) * 8 * C;
  float *d = gnet + ((size_t)iy * W + ix) * 8 * C;
  const double mx = cx + (double)o[0], my = cy + (double)o[1];
  const double ux = 2.0 * mx / W - 1.0, uy = 2.0 * my / H - 1.0;
  // d atanh(2m / S - 1) / dm = (2 / S) / (1 - u^2); zero where the clip is active
  d[0] = (mx > 1e-3 && mx < W - 1e-3) ? (float)((double)g[2 * k] * (2.0 / W) / (1.0 - ux * ux)) : 0.f;
  d[1] = (my > 1e-3 && my < H - 1e-3) ? (float)((double)g[2 * k + 1] * (2.0 / H) / (1.0 - uy * uy)) : 0.f;
  d[2] = g[2 * (size_t)n + 2 * k];
  d[3] = g[2 * (size_t)n + 2 * k + 1];
  d[4] = g[4 * (size_t)n + k];
  for (int c = 0; c < C; ++c) {
    d[8 * c + 5] = g[5 * (size_t)n + (size_t)k * C + c];
    d[8 * c + 6] = g[(size_t)(5 + C) * n + (size_t)k * C + c];
  }
  d[7] = g[(size_t)(5 + 2 * C) * n + k];
}

__global__ void k_sqrt_field(const float *__restrict__ t, int64_t n, float2 *__restrict__ f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = make_float2(sqrtf(fmaxf(t[i], 0.f)), 0.f);
}

// planar [C][n] inputs -> [n][8 C]: block c of pixel i from colour c
__global__ void k_features(const float *__restrict__ t, const float2 *__restrict__ b, int64_t n,
                           int C, uint16_t *__restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n * C) return;
  const int c = (int)(j / n);
  const int64_t i = j - (int64_t)c * n;
  const float v = t[j];
  const float2 u = b[j];
  uint16_t *o = out + (i * C + c) * 8;
  o[0] = to_bf16(v);
  o[1] = to_bf16(sqrtf(fmaxf(v, 0.f)));
  o[2] = to_bf16(u.x);
  o[3] = to_bf16(u.y);
  o[4] = to_bf16(sqrtf(u.x * u.x + u.y * u.y));
  o[5] = o[6] = o[7] = 0;
}

unsigned blocks_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }


// the split of the weight-gradient GEMM: about 512 waves over the 16-pixel
// row chunks of a Wr-wide image, and the byte offsets of its workspace parts
struct WgPlan {
  int Wr, nchunks, cps, splits;
  size_t part, part_b, gyT, ink, bytes;
};
size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }
WgPlan wgrad_plan(int H, int W, int cin, int cout) {
  WgPlan p;
  p.Wr = (W + 15) & ~15;
  p.nchunks = H * (p.Wr / 16);
  const int pairs = ((cin + 31) / 32) * ((cout + 31) / 32);
  const int want = std::max(1, std::min(p.nchunks, (512 + pairs - 1) / pairs));
  p.cps = (p.nchunks + want - 1) / want;
  p.splits = (p.nchunks + p.cps - 1) / p.cps;
  const size_t len = (size_t)cout * 9 * cin;
  p.part = 0;
  p.part_b = round256(p.splits * len * sizeof(float));
  p.gyT = p.part_b + round256((size_t)p.splits * cout * sizeof(float));
  p.ink = p.gyT + round256((size_t)cout * H * p.Wr * sizeof(uint16_t));
  p.bytes = p.ink + round256((size_t)3 * cin * (H + 2) * p.Wr * sizeof(uint16_t));
  return p;
}

}  // namespace
}  // namespace cgh

using namespace cgh;

#define NET_CHECK(cond, ...) \
  do {                       \
    if (!(cond)) return report(CGH_ERR_INVALID_ARG, __VA_ARGS__); \
  } while (0)
#define NET_LAUNCHED(where)                                                           \
  do {                                                                                \
    const hipError_t e_ = hipGetLastError();                                          \
    if (e_ != hipSuccess) return report(CGH_ERR_DEVICE, "%s: %s", where, hipGetErrorString(e_)); \
  } while (0)

static cgh_status check_conv_shape(const cgh_bf16 *x1, int32_t c1, int32_t up,
                                   const cgh_bf16 *x2, int32_t c2, int32_t H, int32_t W) {
  NET_CHECK(x1 && c1 > 0 && c1 % 8 == 0, "x1 NULL or c1 = %d not a positive multiple of 8", c1);
  NET_CHECK((x2 == nullptr) == (c2 == 0) && c2 >= 0 && c2 % 8 == 0,
            "x2 / c2 = %d: both absent, or c2 a positive multiple of 8", c2);
  NET_CHECK(H >= 1 && W >= 1 && (int64_t)H * W < (1LL << 31), "bad size %d x %d", H, W);
  NET_CHECK(!up || (H % 2 == 0 && W % 2 == 0), "upsampled input needs even H, W");
  NET_CHECK(al16(x1) && al16(x2), "inputs must be 16-byte aligned");
  return CGH_OK;
}

extern "C" {

cgh_status cgh_net_conv3x3(const cgh_bf16 *x1, int32_t c1, int32_t up, const cgh_bf16 *x2,
                           int32_t c2, int32_t H, int32_t W, const cgh_bf16 *w,
                           const float *bias, int32_t cout, int32_t relu, float *out32,
                           cgh_bf16 *out16, void *stream) {
  const cgh_status st = check_conv_shape(x1, c1, up, x2, c2, H, W);
  if (st != CGH_OK) return st;
  NET_CHECK(w && cout > 0 && cout % 8 == 0, "w NULL or cout = %d not a multiple of 8", cout);
  NET_CHECK(out32 || out16, "no output");
  NET_CHECK(al16(w) && al16(out32) && al16(out16), "w, out32 and out16 must be 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const int nb = cout % 128 == 0 ? 4 : (cout % 64 == 0 ? 2 : 1);
  const dim3 grid(blocks_of((int64_t)H * W, 32 * kConvWaves), (cout + 32 * nb - 1) / (32 * nb));
#define NET_CONV(NB)                                                                         \
  hipLaunchKernelGGL((k_conv3x3<NB, kConvWaves>), grid, dim3(64 * kConvWaves), 0, s, x1, c1, up, \
                     x2, c2, H, W, w, bias, cout, relu, out32, out16)
  if (nb == 4) NET_CONV(4);
  else if (nb == 2) NET_CONV(2);
  else NET_CONV(1);
#undef NET_CONV
  NET_LAUNCHED("conv3x3");
  return CGH_OK;
}

cgh_status cgh_net_flip_weights(const cgh_bf16 *w, int32_t cout, int32_t cin, cgh_bf16 *w_t,
                                void *stream) {
  NET_CHECK(w && w_t && cout > 0 && cin > 0, "bad arguments");
  hipLaunchKernelGGL(k_flip, dim3(blocks_of((int64_t)cout * 9 * cin, 256)), dim3(256), 0,
                     (hipStream_t)stream, w, cout, cin, w_t);
  NET_LAUNCHED("flip_weights");
  return CGH_OK;
}

size_t cgh_net_wgrad_workspace(int32_t H, int32_t W, int32_t cin, int32_t cout) {
  if (H < 1 || W < 1 || cin < 1 || cout < 1) return 0;
  return wgrad_plan(H, W, cin, cout).bytes;
}

cgh_status cgh_net_conv3x3_wgrad(const cgh_bf16 *x1, int32_t c1, int32_t up, const cgh_bf16 *x2,
                                 int32_t c2, int32_t H, int32_t W, const cgh_bf16 *gy,
                                 int32_t cout, float *gw, float *gb, void *workspace,
                                 size_t workspace_bytes, void *stream) {
  const cgh_status st = check_conv_shape(x1, c1, up, x2, c2, H, W);
  if (st != CGH_OK) return st;
  NET_CHECK(gy && gw && cout > 0 && cout % 8 == 0, "gy/gw NULL or cout = %d not a multiple of 8",
            cout);
  const int cin = c1 + c2;
  const WgPlan pl = wgrad_plan(H, W, cin, cout);
  if (!workspace || workspace_bytes < pl.bytes)
    return report(CGH_ERR_WORKSPACE, "wgrad workspace has %zu bytes, needs %zu", workspace_bytes,
                  pl.bytes);
  NET_CHECK(al16(workspace) && al16(gy), "workspace and gy must be 16-byte aligned");
  const int64_t len = (int64_t)cout * 9 * cin;
  char *base = (char *)workspace;
  float *part = (float *)(base + pl.part), *part_b = (float *)(base + pl.part_b);
  uint16_t *gyT = (uint16_t *)(base + pl.gyT), *ink = (uint16_t *)(base + pl.ink);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_wg_gyT, dim3((pl.Wr + 63) / 64, H, (cout + 31) / 32), dim3(256), 0, s,
                     reinterpret_cast<const uint16_t *>(gy), H, W, pl.Wr, cout, gyT);
  hipLaunchKernelGGL(k_wg_ink, dim3((pl.Wr + 63) / 64, H + 2, (cin + 31) / 32), dim3(256), 0, s,
                     reinterpret_cast<const uint16_t *>(x1), c1, up,
                     reinterpret_cast<const uint16_t *>(x2), c2, H, W, pl.Wr, ink);
  NET_LAUNCHED("conv3x3_wgrad staging");
  hipLaunchKernelGGL(k_conv3x3_wgrad, dim3((cin + 31) / 32, (cout + 31) / 32, pl.splits), dim3(64),
                     0, s, gyT, ink, H, pl.Wr, cin, cout, pl.cps, pl.nchunks, part, part_b);
  NET_LAUNCHED("conv3x3_wgrad");
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks_of(std::max<int64_t>(len, cout), 16)),
                     dim3(256), 0, s, part, part_b, pl.splits, len, cout, gw, gb);
  NET_LAUNCHED("wgrad_reduce");
  return CGH_OK;
}

cgh_status cgh_net_cast_bf16(const float *x, int64_t count, cgh_bf16 *out, void *stream) {
  NET_CHECK(count >= 0 && (count == 0 || (x && out)), "bad arguments");
  if (count == 0) return CGH_OK;
  hipLaunchKernelGGL(k_cast, dim3(blocks_of(count, 256)), dim3(256), 0, (hipStream_t)stream, x,
                     count, out);
  NET_LAUNCHED("cast_bf16");
  return CGH_OK;
}

cgh_status cgh_net_relu_grad(const float *g, const cgh_bf16 *a, int64_t count, cgh_bf16 *out,
                             void *stream) {
  NET_CHECK(count >= 0 && (count == 0 || (g && out)), "bad arguments");
  if (count == 0) return CGH_OK;
  hipLaunchKernelGGL(k_relu_grad, dim3(blocks_of(count, 256)), dim3(256), 0,
                     (hipStream_t)stream, g, a, count, out);
  NET_LAUNCHED("relu_grad");
  return CGH_OK;
}

cgh_status cgh_net_pool2(const cgh_bf16 *x, int32_t H, int32_t W, int32_t C, cgh_bf16 *out,
                         void *stream) {
  NET_CHECK(x && out && H >= 2 && W >= 2 && H % 2 == 0 && W % 2 == 0 && C > 0, "bad arguments");
  hipLaunchKernelGGL(k_pool2, dim3(blocks_of((int64_t)(H / 2) * (W / 2) * C, 256)), dim3(256), 0,
                     (hipStream_t)stream, x, H, W, C, out);
  NET_LAUNCHED("pool2");
  return CGH_OK;
}

cgh_status cgh_net_up_adjoint(const float *g, int32_t H, int32_t W, int32_t stride, int32_t C,
                              float *out, void *stream) {
  NET_CHECK(g && out && H % 2 == 0 && W % 2 == 0 && H >= 2 && W >= 2 && C > 0 && stride >= C,
            "bad arguments");
  hipLaunchKernelGGL(k_up_adjoint, dim3(blocks_of((int64_t)(H / 2) * (W / 2) * C, 256)),
                     dim3(256), 0, (hipStream_t)stream, g, H, W, stride, C, out);
  NET_LAUNCHED("up_adjoint");
  return CGH_OK;
}

cgh_status cgh_net_grad_combine(const float *gp, const float *gs, int32_t stride, int32_t off,
                                int32_t H, int32_t W, int32_t C, float *out, void *stream) {
  NET_CHECK(out && H >= 1 && W >= 1 && C > 0, "bad arguments");
  NET_CHECK(!gp || (H % 2 == 0 && W % 2 == 0), "pooled gradient needs even H, W");
  NET_CHECK(!gs || (off >= 0 && off + C <= stride), "skip slice outside its rows");
  hipLaunchKernelGGL(k_grad_combine, dim3(blocks_of((int64_t)H * W * C, 256)), dim3(256), 0,
                     (hipStream_t)stream, gp, gs, stride, off, H, W, C, out);
  NET_LAUNCHED("grad_combine");
  return CGH_OK;
}

cgh_status cgh_net_lattice_gather(const float *net, int32_t H, int32_t W, int32_t gy,
                                  int32_t gx, int32_t C, float *params, void *stream) {
  NET_CHECK(net && params && gy >= 1 && gx >= 1 && gy <= H && gx <= W && C >= 1 &&
                C <= CGH_MAX_CHANNELS, "bad arguments");
  hipLaunchKernelGGL(k_lattice_gather, dim3(blocks_of((int64_t)gy * gx, 256)), dim3(256), 0,
                     (hipStream_t)stream, net, H, W, gy, gx, C, params);
  NET_LAUNCHED("lattice_gather");
  return CGH_OK;
}

cgh_status cgh_net_lattice_scatter(const float *net, const float *grads, int32_t H, int32_t W,
                                   int32_t gy, int32_t gx, int32_t C, float *g_net,
                                   void *stream) {
  NET_CHECK(net && grads && g_net && gy >= 1 && gx >= 1 && gy <= H && gx <= W && C >= 1 &&
                C <= CGH_MAX_CHANNELS, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_fill0, dim3(blocks_of((int64_t)H * W * 8 * C, 256)), dim3(256), 0, s,
                     g_net, (int64_t)H * W * 8 * C);
  hipLaunchKernelGGL(k_lattice_scatter, dim3(blocks_of((int64_t)gy * gx, 256)), dim3(256), 0, s,
                     net, grads, H, W, gy, gx, C, g_net);
  NET_LAUNCHED("lattice_scatter");
  return CGH_OK;
}

cgh_status cgh_net_sqrt_field(const float *target, int64_t count, cgh_c64 *field,
                              void *stream) {
  NET_CHECK(target && field && count > 0, "bad arguments");
  hipLaunchKernelGGL(k_sqrt_field, dim3(blocks_of(count, 256)), dim3(256), 0,
                     (hipStream_t)stream, target, count, reinterpret_cast<float2 *>(field));
  NET_LAUNCHED("sqrt_field");
  return CGH_OK;
}

cgh_status cgh_net_features(const float *target, const cgh_c64 *back, int64_t count, int32_t C,
                            cgh_bf16 *out, void *stream) {
  NET_CHECK(target && back && out && count > 0 && C >= 1 && C <= CGH_MAX_CHANNELS,
            "bad arguments");
  hipLaunchKernelGGL(k_features, dim3(blocks_of(count * C, 256)), dim3(256), 0,
                     (hipStream_t)stream, target, reinterpret_cast<const float2 *>(back), count, C,
                     out);
  NET_LAUNCHED("features");
  return CGH_OK;
}

}  // extern "C"
