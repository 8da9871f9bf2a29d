// Closing the quadrant ring on the gfx950 matrix cores (paper §4, Fig. 2b:
// the four quadrant tensors form a ring that is then fully contracted).
//
// C = 2^-(ea+eb) A^T B with A stored [k][m] and B stored [k][n] (both
// contiguous along the free index, exactly as the quadrant sweeps leave them),
// optionally fused with the closing dot: instead of storing C the epilogue
// multiplies every entry with W[m][n] and sums in float64.
//
// Tiling: 128 x 128 output tile per 256-thread workgroup, four waves of 64 x 64.
// Each k-slice of 16 is staged in LDS k-major ([k][m], [k][n]); a lane reads
// 4 consecutive m (and n) with one 16-byte LDS load and feeds element mm of
// its A vector and nn of its B vector to the MFMA for tile (mm, nn), so a
// wave's 4x4 register tiles come from two LDS reads per k.  Output tile
// (mm, nn) row i / column j is m = 4i + mm, n = 4j + nn inside the wave's
// 64 x 64 block.  Workgroups are renumbered so that consecutive tiles of one
// tile-row land on the same XCD (the dispatcher deals workgroups to the 8 XCDs
// round-robin), sharing A panels in that XCD's L2.
//
// Split BF16x3 (ring_mfma_bf16x3): the staging pass converts each scaled
// float to bf16 high/low parts and transposes into [m][k] / [n][k] so a lane
// reads its 8 consecutive k with one 16-byte load; each 16x16x32 MFMA tile
// accumulates hi*hi + hi*lo + lo*hi.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <type_traits>

#include "kernels.hpp"

namespace tn {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kT = 128;      // output tile edge
constexpr int kBK = 16;      // k-slice staged per step
constexpr int kThreads = 256;
constexpr int kXcd = 8;

__device__ inline int32_t shift_of(const int32_t* slot) {
  if (!slot) return 0;
  const int32_t e = *slot;
  return (e == kExpZero || e == kExpBad) ? 0 : e;
}

// Tile index -> (tile row, tile col) with XCD-aware renumbering.
__device__ inline void tile_of(uint32_t& tm, uint32_t& tn, uint32_t ntm, uint32_t ntn) {
  const uint32_t total = ntm * ntn;
  const uint32_t id = blockIdx.x;
  const uint32_t per = (total + kXcd - 1) / kXcd;
  uint32_t t = (id % kXcd) * per + id / kXcd;
  if (total % kXcd != 0) t = id;   // keep it a bijection when tiles do not split evenly
  tm = t / ntn;
  tn = t - tm * ntn;
}

__device__ inline double block_sum(double v) {
  __shared__ double red[kThreads / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kThreads / 64; ++w) s += red[w];
  return s;
}

// ------------------------------------------------------------ f32 / f64
template <typename T>
__global__ __launch_bounds__(kThreads) void ring_mfma(
    const T* __restrict__ A, const T* __restrict__ B, int64_t M, int64_t N, int64_t Kd,
    const int32_t* sa, const int32_t* sb, T* __restrict__ C, const T* __restrict__ W,
    double* __restrict__ partials) {
  constexpr bool F64 = std::is_same<T, double>::value;
  using V4 = typename std::conditional<F64, f64x4, f32x4>::type;
  constexpr int kVec = 16 / sizeof(T);                 // elements per 16-byte chunk
  constexpr int kChunks = kBK * kT / kVec;             // 16-byte chunks per operand tile
  constexpr int kPer = kChunks / kThreads;             // per thread
  __shared__ __attribute__((aligned(32))) T As[kBK][kT];
  __shared__ __attribute__((aligned(32))) T Bs[kBK][kT];

  const uint32_t ntm = static_cast<uint32_t>((M + kT - 1) / kT);
  const uint32_t ntn = static_cast<uint32_t>((N + kT - 1) / kT);
  uint32_t tm, tn;
  tile_of(tm, tn, ntm, ntn);
  const int64_t m0 = static_cast<int64_t>(tm) * kT, n0 = static_cast<int64_t>(tn) * kT;
  const int ea = shift_of(sa), eb = shift_of(sb);
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;

  // staging: chunk q -> (row kk, column cc)
  using C16 = typename std::conditional<F64, f64x2, f32x4>::type;
  C16 ra[kPer], rb[kPer];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int q = threadIdx.x + i * kThreads;
      const int kk = q / (kT / kVec), cc = (q % (kT / kVec)) * kVec;
      const int64_t kg = k0 + kk;
      C16 va = {}, vb = {};
      if (kg < Kd && m0 + cc < M) va = *reinterpret_cast<const C16*>(A + kg * M + m0 + cc);
      if (kg < Kd && n0 + cc < N) vb = *reinterpret_cast<const C16*>(B + kg * N + n0 + cc);
      ra[i] = va;
      rb[i] = vb;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int q = threadIdx.x + i * kThreads;
      const int kk = q / (kT / kVec), cc = (q % (kT / kVec)) * kVec;
      C16 va = ra[i], vb = rb[i];
#pragma unroll
      for (int e = 0; e < kVec; ++e) {
        va[e] = ldexp(va[e], -ea);
        vb[e] = ldexp(vb[e], -eb);
      }
      *reinterpret_cast<C16*>(&As[kk][cc]) = va;
      *reinterpret_cast<C16*>(&Bs[kk][cc]) = vb;
    }
  };

  V4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = V4{0, 0, 0, 0};

  fetch(0);
  for (int64_t k0 = 0; k0 < Kd; k0 += kBK) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + kBK < Kd) fetch(k0 + kBK);
#pragma unroll
    for (int kb = 0; kb < kBK; kb += 4) {
      const V4 a4 = *reinterpret_cast<const V4*>(&As[kb + g][wm + 4 * c]);
      const V4 b4 = *reinterpret_cast<const V4*>(&Bs[kb + g][wn + 4 * c]);
#pragma unroll
      for (int mm = 0; mm < 4; ++mm)
#pragma unroll
        for (int nn = 0; nn < 4; ++nn) {
          if constexpr (F64)
            acc[mm][nn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a4[mm], b4[nn], acc[mm][nn], 0, 0, 0);
          else
            acc[mm][nn] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[mm], b4[nn], acc[mm][nn], 0, 0, 0);
        }
    }
  }

  // epilogue: lane (c, g) register r of tile (mm, nn) holds
  //   m = wm + 4*i + mm with i = 4g + r (f32) or g + 4r (f64),  n = wn + 4c + nn
  double part = 0.0;
  const int64_t nb = n0 + wn + 4 * c;
#pragma unroll
  for (int mm = 0; mm < 4; ++mm) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = F64 ? (g + 4 * r) : (4 * g + r);
      const int64_t m = m0 + wm + 4 * i + mm;
      if (m >= M || nb >= N) continue;
      const V4 v = {acc[mm][0][r], acc[mm][1][r], acc[mm][2][r], acc[mm][3][r]};
      if (W) {
        const V4 y = *reinterpret_cast<const V4*>(W + m * N + nb);
#pragma unroll
        for (int e = 0; e < 4; ++e) part += static_cast<double>(v[e]) * static_cast<double>(y[e]);
      } else {
        *reinterpret_cast<V4*>(C + m * N + nb) = v;
      }
    }
  }
  if (W) {
    const double s = block_sum(part);
    if (threadIdx.x == 0) partials[static_cast<int64_t>(tm) * ntn + tn] = s;
  }
}

// ------------------------------------------------------------- bf16 x 3
__device__ inline uint16_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ inline float bf16_float(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

constexpr int kBK16 = 32;    // k-slice for the bf16 path (one MFMA k)
constexpr int kLdk = kBK16 + 8;   // padded LDS row (bf16 entries)

__global__ __launch_bounds__(kThreads) void ring_mfma_bf16x3(
    const float* __restrict__ A, const float* __restrict__ B, int64_t M, int64_t N, int64_t Kd,
    const int32_t* sa, const int32_t* sb, float* __restrict__ C, const float* __restrict__ W,
    double* __restrict__ partials) {
  __shared__ __attribute__((aligned(16))) uint16_t Ah[kT][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t Al[kT][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[kT][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t Bl[kT][kLdk];

  const uint32_t ntm = static_cast<uint32_t>((M + kT - 1) / kT);
  const uint32_t ntn = static_cast<uint32_t>((N + kT - 1) / kT);
  uint32_t tm, tn;
  tile_of(tm, tn, ntm, ntn);
  const int64_t m0 = static_cast<int64_t>(tm) * kT, n0 = static_cast<int64_t>(tn) * kT;
  const int ea = shift_of(sa), eb = shift_of(sb);
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;

  // staging: thread (kq, mq) = (t % 8, t / 8) owns the 4k x 4m block
  // k = 4kq..4kq+3, m = 4mq..4mq+3 of the 32 x 128 slice: four 16-byte loads
  // (one per k row), a register transpose, then one 8-byte LDS write of four
  // consecutive k per m row and per split part.
  const int kq = threadIdx.x & 7, mq = threadIdx.x >> 3;
  f32x4 ra[4], rb[4];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t kg = k0 + 4 * kq + i;
      const int cc = 4 * mq;
      f32x4 va = {0.f, 0.f, 0.f, 0.f}, vb = {0.f, 0.f, 0.f, 0.f};
      if (kg < Kd && m0 + cc < M) va = *reinterpret_cast<const f32x4*>(A + kg * M + m0 + cc);
      if (kg < Kd && n0 + cc < N) vb = *reinterpret_cast<const f32x4*>(B + kg * N + n0 + cc);
      ra[i] = va;
      rb[i] = vb;
    }
  };
  typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
  auto stash = [&]() {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      u16x4 h_a, l_a, h_b, l_b;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float xa = ldexpf(ra[i][e], -ea), xb = ldexpf(rb[i][e], -eb);
        h_a[i] = bf16_bits(xa);
        l_a[i] = bf16_bits(xa - bf16_float(h_a[i]));
        h_b[i] = bf16_bits(xb);
        l_b[i] = bf16_bits(xb - bf16_float(h_b[i]));
      }
      const int row = 4 * mq + e, col = 4 * kq;
      *reinterpret_cast<u16x4*>(&Ah[row][col]) = h_a;
      *reinterpret_cast<u16x4*>(&Al[row][col]) = l_a;
      *reinterpret_cast<u16x4*>(&Bh[row][col]) = h_b;
      *reinterpret_cast<u16x4*>(&Bl[row][col]) = l_b;
    }
  };

  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  fetch(0);
  for (int64_t k0 = 0; k0 < Kd; k0 += kBK16) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + kBK16 < Kd) fetch(k0 + kBK16);
    // tile (mt, nt): rows wm + 16 mt + c, k = 8g .. 8g+7
    bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ah[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&Ah[wm + 16 * t + c][8 * g]));
      al[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&Al[wm + 16 * t + c][8 * g]));
      bh[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&Bh[wn + 16 * t + c][8 * g]));
      bl[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&Bl[wn + 16 * t + c][8 * g]));
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        f32x4 a = acc[mt][nt];
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mt], bh[nt], a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], bl[nt], a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], bh[nt], a, 0, 0, 0);
        acc[mt][nt] = a;
      }
  }

  // lane (c, g) register r of tile (mt, nt): m = wm + 16 mt + 4g + r, n = wn + 16 nt + c
  double part = 0.0;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm + 16 * mt + 4 * g + r, n = n0 + wn + 16 * nt + c;
        if (m >= M || n >= N) continue;
        if (W) part += static_cast<double>(acc[mt][nt][r]) * static_cast<double>(W[m * N + n]);
        else C[m * N + n] = acc[mt][nt][r];
      }
  if (W) {
    const double s = block_sum(part);
    if (threadIdx.x == 0) partials[static_cast<int64_t>(tm) * ntn + tn] = s;
  }
}

// ------------------------------------------------ f32, 256 x 256 tiles
// Same operand scheme as ring_mfma<float> on a 256 x 256 output tile: eight
// waves in a 2 (m) x 4 (n) grid, each 128 x 64 (two 16-byte A reads and one
// B read per k feed 32 MFMA tiles).  Twice the flops per staged byte of the
// 128 x 128 tile; the LDS k-slices are double-buffered so one barrier per
// slice separates staging from compute.
constexpr int kBT = 256;
constexpr int kBThreads = 512;

__global__ __launch_bounds__(kBThreads) void ring_mfma_f32_big(
    const float* __restrict__ A, const float* __restrict__ B, int64_t M, int64_t N, int64_t Kd,
    const int32_t* sa, const int32_t* sb, float* __restrict__ C, const float* __restrict__ W,
    double* __restrict__ partials) {
  __shared__ __attribute__((aligned(16))) float As[2][kBK][kBT];
  __shared__ __attribute__((aligned(16))) float Bs[2][kBK][kBT];
  const uint32_t ntm = static_cast<uint32_t>((M + kBT - 1) / kBT);
  const uint32_t ntn = static_cast<uint32_t>((N + kBT - 1) / kBT);
  uint32_t tm, tn;
  tile_of(tm, tn, ntm, ntn);
  const int64_t m0 = static_cast<int64_t>(tm) * kBT, n0 = static_cast<int64_t>(tn) * kBT;
  const int ea = shift_of(sa), eb = shift_of(sb);
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
  const int wm = (w >> 2) * 128, wn = (w & 3) * 64;
  constexpr int kPer = kBK * kBT / 4 / kBThreads;   // 16-byte chunks per thread per operand

  f32x4 ra[kPer], rb[kPer];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int q = threadIdx.x + i * kBThreads;
      const int kk = q / (kBT / 4), cc = (q % (kBT / 4)) * 4;
      const int64_t kg = k0 + kk;
      f32x4 va = {0.f, 0.f, 0.f, 0.f}, vb = {0.f, 0.f, 0.f, 0.f};
      if (kg < Kd && m0 + cc < M) va = *reinterpret_cast<const f32x4*>(A + kg * M + m0 + cc);
      if (kg < Kd && n0 + cc < N) vb = *reinterpret_cast<const f32x4*>(B + kg * N + n0 + cc);
      ra[i] = va;
      rb[i] = vb;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int q = threadIdx.x + i * kBThreads;
      const int kk = q / (kBT / 4), cc = (q % (kBT / 4)) * 4;
      f32x4 va = ra[i], vb = rb[i];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        va[e] = ldexpf(va[e], -ea);
        vb[e] = ldexpf(vb[e], -eb);
      }
      *reinterpret_cast<f32x4*>(&As[buf][kk][cc]) = va;
      *reinterpret_cast<f32x4*>(&Bs[buf][kk][cc]) = vb;
    }
  };

  f32x4 acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  fetch(0);
  stash(0);
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = 0; k0 < Kd; k0 += kBK) {
    const bool more = k0 + kBK < Kd;
    if (more) fetch(k0 + kBK);
#pragma unroll
    for (int kb = 0; kb < kBK; kb += 4) {
      const f32x4 a0 = *reinterpret_cast<const f32x4*>(&As[buf][kb + g][wm + 4 * c]);
      const f32x4 a1 = *reinterpret_cast<const f32x4*>(&As[buf][kb + g][wm + 64 + 4 * c]);
      const f32x4 b4 = *reinterpret_cast<const f32x4*>(&Bs[buf][kb + g][wn + 4 * c]);
#pragma unroll
      for (int mm = 0; mm < 4; ++mm)
#pragma unroll
        for (int nn = 0; nn < 4; ++nn) {
          acc[mm][nn] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[mm], b4[nn], acc[mm][nn], 0, 0, 0);
          acc[4 + mm][nn] =
              __builtin_amdgcn_mfma_f32_16x16x4f32(a1[mm], b4[nn], acc[4 + mm][nn], 0, 0, 0);
        }
    }
    if (more) stash(buf ^ 1);   // the other buffer: last read before the previous barrier
    __syncthreads();
    buf ^= 1;
  }

  // lane (c, g) register r of tile (h*4 + mm, nn): m = wm + 64h + 4(4g + r) + mm, n = wn + 4c + nn
  double part = 0.0;
  const int64_t nb = n0 + wn + 4 * c;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int mm = 0; mm < 4; ++mm)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm + 64 * h + 4 * (4 * g + r) + mm;
        if (m >= M || nb >= N) continue;
        const f32x4 v = {acc[4 * h + mm][0][r], acc[4 * h + mm][1][r], acc[4 * h + mm][2][r],
                         acc[4 * h + mm][3][r]};
        if (W) {
          const f32x4 y = *reinterpret_cast<const f32x4*>(W + m * N + nb);
#pragma unroll
          for (int e = 0; e < 4; ++e) part += static_cast<double>(v[e]) * static_cast<double>(y[e]);
        } else {
          *reinterpret_cast<f32x4*>(C + m * N + nb) = v;
        }
      }
  if (W) {
    __shared__ double red[kBThreads / 64];
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if (lane == 0) red[w] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int i = 0; i < kBThreads / 64; ++i) sum += red[i];
      partials[static_cast<int64_t>(tm) * ntn + tn] = sum;
    }
  }
}

// ------------------------------------------- split + transpose for BF16x3
// T [kd][md] float (k-major, as a quadrant sweep leaves it), scaled by 2^-e,
// becomes H, L [md][kp] bf16 (hi, lo parts; k-contiguous, rows padded to kp
// with zeros) so the GEMM below reads 8 consecutive k with one 16-byte load.
// 64 (k) x 64 (m) tile per 256-thread workgroup: thread (kq, mq) = (t/16, t%16)
// loads four 16-byte row pieces (k = 4kq..4kq+3, m = 4mq..4mq+3; 16 lanes cover
// a 256-byte row), transposes its 4x4 block in registers and writes 8 bytes
// (4 consecutive k) per m row into LDS; the tile leaves as 128-byte row pieces.
constexpr int kPT = 64;
constexpr int kPLd = kPT + 8;   // padded LDS row (bf16 entries)

__global__ __launch_bounds__(kThreads) void split_transpose(const float* __restrict__ T,
                                                            int64_t kd, int64_t md, int64_t kp,
                                                            const int32_t* slot,
                                                            uint16_t* __restrict__ H,
                                                            uint16_t* __restrict__ L) {
  __shared__ __attribute__((aligned(16))) uint16_t sh[kPT][kPLd];
  __shared__ __attribute__((aligned(16))) uint16_t sl[kPT][kPLd];
  const int64_t k0 = static_cast<int64_t>(blockIdx.x) * kPT;
  const int64_t m0 = static_cast<int64_t>(blockIdx.y) * kPT;
  const int e = shift_of(slot);
  const int kq = threadIdx.x >> 4, mq = threadIdx.x & 15;
  f32x4 v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t k = k0 + 4 * kq + i, m = m0 + 4 * mq;
    v[i] = (k < kd && m < md) ? *reinterpret_cast<const f32x4*>(T + k * md + m)
                              : f32x4{0.f, 0.f, 0.f, 0.f};
  }
  typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    u16x4 h, l;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float x = ldexpf(v[i][c], -e);
      h[i] = bf16_bits(x);
      l[i] = bf16_bits(x - bf16_float(h[i]));
    }
    *reinterpret_cast<u16x4*>(&sh[4 * mq + c][4 * kq]) = h;
    *reinterpret_cast<u16x4*>(&sl[4 * mq + c][4 * kq]) = l;
  }
  __syncthreads();
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const int q = threadIdx.x + pass * kThreads;   // 512 chunks of 8 k
    const int row = q >> 3, j = q & 7;
    const int64_t m = m0 + row, k = k0 + 8 * j;
    if (m < md && k < kp) {
      *reinterpret_cast<u16x8*>(H + m * kp + k) = *reinterpret_cast<const u16x8*>(&sh[row][8 * j]);
      *reinterpret_cast<u16x8*>(L + m * kp + k) = *reinterpret_cast<const u16x8*>(&sl[row][8 * j]);
    }
  }
}

// ---------------------------------------------- bf16x3 GEMM, k-contiguous
// C[m][n] = sum_k A[m][k] B[n][k] with A, B given as bf16 (hi, lo) pairs
// [rows][kp]; three MFMA products per tile (lo*hi + hi*lo + hi*hi, float32
// accumulation).  Each 32-wide k-slice of the four operand tiles (128 x 32
// bf16 each) is copied to LDS with 16-byte loads (four lanes per 64-byte row
// piece), no conversion; lane (c, g) then reads its 8 consecutive k of row
// wm + 16 t + c with one 16-byte LDS load.
__global__ __launch_bounds__(kThreads) void ring_bf16x3_nt(
    const uint16_t* __restrict__ Ah, const uint16_t* __restrict__ Al,
    const uint16_t* __restrict__ Bh, const uint16_t* __restrict__ Bl, int64_t M, int64_t N,
    int64_t kp, float* __restrict__ C, const float* __restrict__ W,
    double* __restrict__ partials) {
  __shared__ __attribute__((aligned(16))) uint16_t sAh[kT][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t sAl[kT][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t sBh[kT][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t sBl[kT][kLdk];
  const uint32_t ntm = static_cast<uint32_t>((M + kT - 1) / kT);
  const uint32_t ntn = static_cast<uint32_t>((N + kT - 1) / kT);
  uint32_t tm, tn;
  tile_of(tm, tn, ntm, ntn);
  const int64_t m0 = static_cast<int64_t>(tm) * kT, n0 = static_cast<int64_t>(tn) * kT;
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;

  // staging: 128 rows x 4 chunks of 16 bytes per operand tile, 2 per thread
  u16x8 rah[2], ral[2], rbh[2], rbl[2];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int q = threadIdx.x + i * kThreads;
      const int row = q >> 2, j = q & 3;
      const int64_t ma = m0 + row, nb = n0 + row, k = k0 + 8 * j;
      const u16x8 z = {0, 0, 0, 0, 0, 0, 0, 0};
      rah[i] = ma < M ? *reinterpret_cast<const u16x8*>(Ah + ma * kp + k) : z;
      ral[i] = ma < M ? *reinterpret_cast<const u16x8*>(Al + ma * kp + k) : z;
      rbh[i] = nb < N ? *reinterpret_cast<const u16x8*>(Bh + nb * kp + k) : z;
      rbl[i] = nb < N ? *reinterpret_cast<const u16x8*>(Bl + nb * kp + k) : z;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int q = threadIdx.x + i * kThreads;
      const int row = q >> 2, j = q & 3;
      *reinterpret_cast<u16x8*>(&sAh[row][8 * j]) = rah[i];
      *reinterpret_cast<u16x8*>(&sAl[row][8 * j]) = ral[i];
      *reinterpret_cast<u16x8*>(&sBh[row][8 * j]) = rbh[i];
      *reinterpret_cast<u16x8*>(&sBl[row][8 * j]) = rbl[i];
    }
  };

  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  fetch(0);
  for (int64_t k0 = 0; k0 < kp; k0 += kBK16) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + kBK16 < kp) fetch(k0 + kBK16);
    bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ah[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sAh[wm + 16 * t + c][8 * g]));
      al[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sAl[wm + 16 * t + c][8 * g]));
      bh[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sBh[wn + 16 * t + c][8 * g]));
      bl[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sBl[wn + 16 * t + c][8 * g]));
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        f32x4 a = acc[mt][nt];
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mt], bh[nt], a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], bl[nt], a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], bh[nt], a, 0, 0, 0);
        acc[mt][nt] = a;
      }
  }

  double part = 0.0;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm + 16 * mt + 4 * g + r, n = n0 + wn + 16 * nt + c;
        if (m >= M || n >= N) continue;
        if (W) part += static_cast<double>(acc[mt][nt][r]) * static_cast<double>(W[m * N + n]);
        else C[m * N + n] = acc[mt][nt][r];
      }
  if (W) {
    const double s = block_sum(part);
    if (threadIdx.x == 0) partials[static_cast<int64_t>(tm) * ntn + tn] = s;
  }
}

// ------------------------------------------- bf16x3 NT, 256 x 256 tiles
// ring_bf16x3_nt on a 256 x 256 tile: eight waves (2 x 4), each 128 x 64, so
// every staged k-slice feeds twice the MFMA work.  The four 256 x 32 operand
// slices (80 KiB of LDS) are single-buffered with a register prefetch of the
// next slice.
__global__ __launch_bounds__(kBThreads) void ring_bf16x3_nt_big(
    const uint16_t* __restrict__ Ah, const uint16_t* __restrict__ Al,
    const uint16_t* __restrict__ Bh, const uint16_t* __restrict__ Bl, int64_t M, int64_t N,
    int64_t kp, float* __restrict__ C, const float* __restrict__ W,
    double* __restrict__ partials) {
  __shared__ __attribute__((aligned(16))) uint16_t sAh[kBT][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t sAl[kBT][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t sBh[kBT][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t sBl[kBT][kLdk];
  const uint32_t ntm = static_cast<uint32_t>((M + kBT - 1) / kBT);
  const uint32_t ntn = static_cast<uint32_t>((N + kBT - 1) / kBT);
  uint32_t tm, tn;
  tile_of(tm, tn, ntm, ntn);
  const int64_t m0 = static_cast<int64_t>(tm) * kBT, n0 = static_cast<int64_t>(tn) * kBT;
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
  const int wm = (w >> 2) * 128, wn = (w & 3) * 64;

  // 256 rows x 4 chunks of 16 bytes per operand slice, 2 per thread
  u16x8 rah[2], ral[2], rbh[2], rbl[2];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int q = threadIdx.x + i * kBThreads;
      const int row = q >> 2, j = q & 3;
      const int64_t ma = m0 + row, nb = n0 + row, k = k0 + 8 * j;
      const u16x8 z = {0, 0, 0, 0, 0, 0, 0, 0};
      rah[i] = ma < M ? *reinterpret_cast<const u16x8*>(Ah + ma * kp + k) : z;
      ral[i] = ma < M ? *reinterpret_cast<const u16x8*>(Al + ma * kp + k) : z;
      rbh[i] = nb < N ? *reinterpret_cast<const u16x8*>(Bh + nb * kp + k) : z;
      rbl[i] = nb < N ? *reinterpret_cast<const u16x8*>(Bl + nb * kp + k) : z;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int q = threadIdx.x + i * kBThreads;
      const int row = q >> 2, j = q & 3;
      *reinterpret_cast<u16x8*>(&sAh[row][8 * j]) = rah[i];
      *reinterpret_cast<u16x8*>(&sAl[row][8 * j]) = ral[i];
      *reinterpret_cast<u16x8*>(&sBh[row][8 * j]) = rbh[i];
      *reinterpret_cast<u16x8*>(&sBl[row][8 * j]) = rbl[i];
    }
  };

  f32x4 acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  fetch(0);
  for (int64_t k0 = 0; k0 < kp; k0 += kBK16) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + kBK16 < kp) fetch(k0 + kBK16);
    bf16x8 bh[4], bl[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      bh[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sBh[wn + 16 * t + c][8 * g]));
      bl[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sBl[wn + 16 * t + c][8 * g]));
    }
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
      const bf16x8 ah =
          __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sAh[wm + 16 * mt + c][8 * g]));
      const bf16x8 al =
          __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sAl[wm + 16 * mt + c][8 * g]));
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        f32x4 a = acc[mt][nt];
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[nt], a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[nt], a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[nt], a, 0, 0, 0);
        acc[mt][nt] = a;
      }
    }
  }

  double part = 0.0;
#pragma unroll
  for (int mt = 0; mt < 8; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm + 16 * mt + 4 * g + r, n = n0 + wn + 16 * nt + c;
        if (m >= M || n >= N) continue;
        if (W) part += static_cast<double>(acc[mt][nt][r]) * static_cast<double>(W[m * N + n]);
        else C[m * N + n] = acc[mt][nt][r];
      }
  if (W) {
    __shared__ double red[kBThreads / 64];
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if (lane == 0) red[w] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int i = 0; i < kBThreads / 64; ++i) sum += red[i];
      partials[static_cast<int64_t>(tm) * ntn + tn] = sum;
    }
  }
}

}  // namespace

bool ring_mfma_supported(const RingArgs& a) {
  return a.m % 4 == 0 && a.n % 4 == 0 && a.m >= 1 && a.n >= 1 && a.k >= 1;
}

int64_t ring_mfma_partials(int64_t m, int64_t n) {
  return ((m + kT - 1) / kT) * ((n + kT - 1) / kT);
}

int64_t ring_mfma_partials_for(const RingArgs& a) {
  if (a.type != EL_F64 && a.arith != AR_BF16X3 && a.m >= kBT && a.n >= kBT)
    return ((a.m + kBT - 1) / kBT) * ((a.n + kBT - 1) / kBT);
  return ring_mfma_partials(a.m, a.n);
}

hipError_t launch_ring_mfma(const RingArgs& a, hipStream_t stream, const char** kname) {
  const int64_t tiles = ring_mfma_partials(a.m, a.n);
  if (tiles > INT_MAX) return hipErrorInvalidValue;
  const dim3 grid(static_cast<uint32_t>(tiles)), block(kThreads);
  if (a.type == EL_F64) {
    *kname = "ring_mfma_f64";
    hipLaunchKernelGGL((ring_mfma<double>), grid, block, 0, stream,
                       static_cast<const double*>(a.A), static_cast<const double*>(a.B), a.m, a.n,
                       a.k, a.sa, a.sb, static_cast<double*>(a.c_out),
                       static_cast<const double*>(a.dot_with), a.partials);
  } else if (a.arith == AR_BF16X3) {
    *kname = "ring_mfma_bf16x3";
    hipLaunchKernelGGL(ring_mfma_bf16x3, grid, block, 0, stream, static_cast<const float*>(a.A),
                       static_cast<const float*>(a.B), a.m, a.n, a.k, a.sa, a.sb,
                       static_cast<float*>(a.c_out), static_cast<const float*>(a.dot_with),
                       a.partials);
  } else if (a.m >= kBT && a.n >= kBT) {
    *kname = "ring_mfma_f32";
    const int64_t big = ((a.m + kBT - 1) / kBT) * ((a.n + kBT - 1) / kBT);
    hipLaunchKernelGGL(ring_mfma_f32_big, dim3(static_cast<uint32_t>(big)), dim3(kBThreads), 0,
                       stream, static_cast<const float*>(a.A), static_cast<const float*>(a.B), a.m,
                       a.n, a.k, a.sa, a.sb, static_cast<float*>(a.c_out),
                       static_cast<const float*>(a.dot_with), a.partials);
  } else {
    *kname = "ring_mfma_f32";
    hipLaunchKernelGGL((ring_mfma<float>), grid, block, 0, stream,
                       static_cast<const float*>(a.A), static_cast<const float*>(a.B), a.m, a.n,
                       a.k, a.sa, a.sb, static_cast<float*>(a.c_out),
                       static_cast<const float*>(a.dot_with), a.partials);
  }
  return hipGetLastError();
}

}  // namespace tn

namespace tn {

int64_t split_k_padded(int64_t k) { return (k + kBK16 - 1) / kBK16 * kBK16; }

hipError_t launch_split_transpose(const float* T, int64_t kd, int64_t md, const int32_t* slot,
                                  uint16_t* H, uint16_t* L, hipStream_t stream) {
  const int64_t kp = split_k_padded(kd);
  const int64_t gx = (kp + kPT - 1) / kPT, gy = (md + kPT - 1) / kPT;
  if (gx > INT_MAX || gy > 65535 || md % 4 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(split_transpose, dim3(static_cast<uint32_t>(gx), static_cast<uint32_t>(gy)),
                     dim3(kThreads), 0, stream, T, kd, md, kp, slot, H, L);
  return hipGetLastError();
}

int64_t ring_bf16x3_nt_partials(int64_t m, int64_t n) {
  if (m >= kBT && n >= kBT) return ((m + kBT - 1) / kBT) * ((n + kBT - 1) / kBT);
  return ring_mfma_partials(m, n);
}

hipError_t launch_ring_bf16x3_nt(const uint16_t* Ah, const uint16_t* Al, const uint16_t* Bh,
                                 const uint16_t* Bl, int64_t m, int64_t n, int64_t kp, float* c_out,
                                 const float* dot_with, double* partials, hipStream_t stream) {
  if (m >= kBT && n >= kBT) {
    const int64_t tiles = ring_bf16x3_nt_partials(m, n);
    if (tiles > INT_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(ring_bf16x3_nt_big, dim3(static_cast<uint32_t>(tiles)), dim3(kBThreads), 0,
                       stream, Ah, Al, Bh, Bl, m, n, kp, c_out, dot_with, partials);
    return hipGetLastError();
  }
  const int64_t tiles = ring_mfma_partials(m, n);
  if (tiles > INT_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(ring_bf16x3_nt, dim3(static_cast<uint32_t>(tiles)), dim3(kThreads), 0, stream,
                     Ah, Al, Bh, Bl, m, n, kp, c_out, dot_with, partials);
  return hipGetLastError();
}

}  // namespace tn
