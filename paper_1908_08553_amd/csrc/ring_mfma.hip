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

}  // namespace

bool ring_mfma_supported(const RingArgs& a) {
  return a.m % 4 == 0 && a.n % 4 == 0 && a.m >= 1 && a.n >= 1 && a.k >= 1;
}

int64_t ring_mfma_partials(int64_t m, int64_t n) {
  return ((m + kT - 1) / kT) * ((n + kT - 1) / kT);
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
