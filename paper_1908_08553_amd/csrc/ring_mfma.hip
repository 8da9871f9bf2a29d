// Closing the quadrant ring on the gfx950 matrix cores (paper §4, Fig. 2b:
// the four quadrant tensors form a ring that is then fully contracted).
//
// C = 2^-(ea+eb) A^T B with A stored [k][m] and B stored [k][n] (both
// contiguous along the free index, exactly as the quadrant sweeps leave them),
// optionally fused with the closing dot: instead of storing C the epilogue
// multiplies every entry with W[m][n] and sums in float64.
//
// Tiling: 128 x 128 output tile per 256-thread workgroup, four waves of 64 x 64.
// Each k-slice of 16 is staged in LDS k-major ([k][m], [k][n]), double
// buffered; a lane reads 4 consecutive m (and n) with 16-byte LDS loads and
// feeds element mm of its A vector and nn of its B vector to the MFMA for tile
// (mm, nn), so a wave's 4x4 register tiles come from two LDS reads per k.
// Output tile (mm, nn) row i / column j is m = 4i + mm, n = 4j + nn inside the
// wave's 64 x 64 block.  Workgroups are renumbered so that consecutive tiles
// of one tile-row land on the same XCD (the dispatcher deals workgroups to the
// 8 XCDs round-robin), sharing A panels in that XCD's L2.
//
// Split-K: when the output has too few tiles to give every CU two workgroups
// the k extent is cut into S ranges of whole k-slices (workgroup s * tiles + t
// takes range s of tile t).  A stored product then leaves S partial slices
// C_s at stride m*n; the fused-dot launch that consumes it as W sums the
// slices in float64 in a fixed order, and its own split ranges each write one
// partial sum, so results do not depend on scheduling.
//
// Split BF16x3: split_transpose converts each scaled float to bf16 high/low
// parts in [m][k] / [n][k] order so a lane reads its 8 consecutive k with one
// 16-byte load; each 16x16x32 MFMA tile accumulates hi*hi + hi*lo + lo*hi.
#include <hip/hip_runtime.h>

#include <algorithm>
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
constexpr int kMaxSplits = 8;
constexpr int64_t kFillGroups = 512;   // two workgroups per CU
int32_t g_ring_operand_scale = 0;      // TN_OPT_RING_OPERAND_SCALE

__device__ inline int32_t shift_of(const int32_t* slot) {
  if (!slot) return 0;
  const int32_t e = *slot;
  return (e == kExpZero || e == kExpBad) ? 0 : e;
}

// Tile index id -> (tile row, tile col).  Workgroup id runs on XCD id % 8, so
// t = (id % 8) * per + id / 8 gives every XCD a contiguous range of t; t is
// then read in groups of kGroupRows tile rows walked column by column, so the
// workgroups resident on one XCD at a time form a near-square block of tiles
// and share their A and B panels in that XCD's L2.
constexpr uint32_t kGroupRows = 8;
__device__ inline void tile_of(uint32_t& tm, uint32_t& tn, uint32_t ntm, uint32_t ntn,
                               uint32_t id) {
  const uint32_t total = ntm * ntn;
  const uint32_t per = (total + kXcd - 1) / kXcd;
  uint32_t t = (id % kXcd) * per + id / kXcd;
  if (total % kXcd != 0) t = id;   // keep it a bijection when tiles do not split evenly
  const uint32_t g = t / (kGroupRows * ntn), r = t - g * kGroupRows * ntn;
  const uint32_t rows = min(kGroupRows, ntm - g * kGroupRows);
  tn = r / rows;
  tm = g * kGroupRows + (r - tn * rows);
}

// k range [b, e) of split s out of S, in whole slices of bk.
struct KRange {
  int64_t b, e;
};
__device__ inline KRange k_range(int64_t kd, int32_t S, uint32_t s, int bk) {
  const int64_t per = ((kd + bk - 1) / bk + S - 1) / S * bk;
  const int64_t b0 = static_cast<int64_t>(s) * per;
  const int64_t b = b0 < kd ? b0 : kd;
  return {b, b + per < kd ? b + per : kd};
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

// Four consecutive entries of the W operand, summed over its slices in float64.
template <typename T>
__device__ inline void w_sum(const T* __restrict__ W, int64_t slice, int32_t w_slices, int64_t at,
                             double (&y)[4]) {
  using V4 = typename std::conditional<std::is_same<T, double>::value, f64x4, f32x4>::type;
  const V4 w0 = *reinterpret_cast<const V4*>(W + at);
#pragma unroll
  for (int e = 0; e < 4; ++e) y[e] = static_cast<double>(w0[e]);
  for (int32_t j = 1; j < w_slices; ++j) {
    const V4 wj = *reinterpret_cast<const V4*>(W + j * slice + at);
#pragma unroll
    for (int e = 0; e < 4; ++e) y[e] += static_cast<double>(wj[e]);
  }
}

template <typename X>
struct TypeTag {
  using type = X;
};

// 16 bytes per lane from global memory straight into LDS: one instruction
// fills 1 KiB at lds + 16 * lane.
typedef __attribute__((address_space(3))) void* LdsPtrR;
__device__ inline void ring_fill16(const void* g, void* lds) {
#if __HIP_DEVICE_COMPILE__
  __builtin_amdgcn_global_load_lds(g, (LdsPtrR)(lds), 16, 0, 0);
#else
  (void)g;
  (void)lds;
#endif
}

// ------------------------------------------------------------ f32 / f64
// The register budget (two waves per SIMD) keeps the 64 (f32) or 128 (f64)
// accumulator registers in VGPRs; with more live registers the compiler parks
// them in AGPRs and copies them out and back around every k-slice, which
// drains the matrix pipe each time.  Two workgroups per CU (LDS: 32 KiB f32,
// 64 KiB f64); one barrier per k-slice.
template <typename T>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void ring_mfma(
    const T* __restrict__ A, const T* __restrict__ B, int64_t M, int64_t N, int64_t Kd, int32_t S,
    const int32_t* sa, const int32_t* sb, T* __restrict__ C, const T* __restrict__ W,
    int32_t w_slices, double* __restrict__ partials, int32_t operand_scale) {
  constexpr bool F64 = std::is_same<T, double>::value;
  using V4 = typename std::conditional<F64, f64x4, f32x4>::type;
  using C16 = typename std::conditional<F64, f64x2, f32x4>::type;
  constexpr int kVec = 16 / sizeof(T);                 // elements per 16-byte chunk
  constexpr int kPer = kBK * kT / kVec / kThreads;     // 16-byte chunks per thread per operand
  // two buffers per operand, declared apart: the compiler tracks the
  // asynchronous fills of one against reads of the other only for distinct
  // LDS variables
  __shared__ __attribute__((aligned(32))) T As0[kBK][kT];
  __shared__ __attribute__((aligned(32))) T As1[kBK][kT];
  __shared__ __attribute__((aligned(32))) T Bs0[kBK][kT];
  __shared__ __attribute__((aligned(32))) T Bs1[kBK][kT];
  auto a_buf = [&](int b) -> T (*)[kT] { return b ? As1 : As0; };
  auto b_buf = [&](int b) -> T (*)[kT] { return b ? Bs1 : Bs0; };

  const uint32_t ntm = static_cast<uint32_t>((M + kT - 1) / kT);
  const uint32_t ntn = static_cast<uint32_t>((N + kT - 1) / kT);
  const uint32_t tiles = ntm * ntn;
  const uint32_t s = blockIdx.x / tiles;
  uint32_t tm, tn;
  tile_of(tm, tn, ntm, ntn, blockIdx.x - s * tiles);
  const KRange kr = k_range(Kd, S, s, kBK);
  const int64_t m0 = static_cast<int64_t>(tm) * kT, n0 = static_cast<int64_t>(tn) * kT;
  const int ea = shift_of(sa), eb = shift_of(sb);
  // FP64: the 2^-(ea+eb) factor is applied once to the results instead of to
  // every staged operand (double-precision vector work slows the FP64 matrix
  // pipe).  Powers of two scale exactly, so both orders give the same bits
  // while the unscaled sums stay normal: |ea + eb| <= 512 leaves them more
  // than 2^400 from either end of the double range.
  const bool late = F64 && !operand_scale && ea + eb <= 512 && ea + eb >= -512;
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;

  // staging: chunk q -> (row kk, column cc)
  C16 ra[kPer], rb[kPer];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int q = threadIdx.x + i * kThreads;
      const int kk = q / (kT / kVec), cc = (q % (kT / kVec)) * kVec;
      const int64_t kg = k0 + kk;
      C16 va = {}, vb = {};
      if (kg < kr.e && m0 + cc < M) va = *reinterpret_cast<const C16*>(A + kg * M + m0 + cc);
      if (kg < kr.e && n0 + cc < N) vb = *reinterpret_cast<const C16*>(B + kg * N + n0 + cc);
      ra[i] = va;
      rb[i] = vb;
    }
  };
  // PS: scale each staged operand (the k loop is compiled once per mode, so
  // the late-scaled loop carries no ldexp)
  auto stash = [&](int buf, auto ps) {
    constexpr bool PS = decltype(ps)::value;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int q = threadIdx.x + i * kThreads;
      const int kk = q / (kT / kVec), cc = (q % (kT / kVec)) * kVec;
      C16 va = ra[i], vb = rb[i];
      if constexpr (PS) {
#pragma unroll
        for (int e = 0; e < kVec; ++e) {
          va[e] = ldexp(va[e], -ea);
          vb[e] = ldexp(vb[e], -eb);
        }
      }
      *reinterpret_cast<C16*>(&a_buf(buf)[kk][cc]) = va;
      *reinterpret_cast<C16*>(&b_buf(buf)[kk][cc]) = vb;
    }
  };

  V4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = V4{0, 0, 0, 0};

  auto k_loop = [&](auto ps) {
    fetch(kr.b);
    stash(0, ps);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = kr.b; k0 < kr.e; k0 += kBK) {
      const bool more = k0 + kBK < kr.e;
      if (more) fetch(k0 + kBK);
#pragma unroll
      for (int kb = 0; kb < kBK; kb += 4) {
        const V4 a4 = *reinterpret_cast<const V4*>(&a_buf(buf)[kb + g][wm + 4 * c]);
        const V4 b4 = *reinterpret_cast<const V4*>(&b_buf(buf)[kb + g][wn + 4 * c]);
#pragma unroll
        for (int mm = 0; mm < 4; ++mm)
#pragma unroll
          for (int nn = 0; nn < 4; ++nn) {
            if constexpr (F64)
              acc[mm][nn] =
                  __builtin_amdgcn_mfma_f64_16x16x4f64(a4[mm], b4[nn], acc[mm][nn], 0, 0, 0);
            else
              acc[mm][nn] =
                  __builtin_amdgcn_mfma_f32_16x16x4f32(a4[mm], b4[nn], acc[mm][nn], 0, 0, 0);
          }
      }
      if (more) stash(buf ^ 1, ps);   // the other buffer: last read before the previous barrier
      __syncthreads();
      buf ^= 1;
    }
  };
  // FP64 with the scaling applied to the results: each k row of A and B (128
  // doubles, 1 KiB) goes from global memory straight into LDS with one
  // instruction, wave w filling rows w, w + 4, ...; rows past the k range
  // are zeroed, columns past M or N are filled from column M - 2 (N - 2) and
  // their products never stored.  The next slice is in flight while the
  // current one is multiplied; one wait and barrier per slice.
  auto k_loop_async = [&](auto f64_tag) {
    using D4 = typename decltype(f64_tag)::type;
    const int64_t cm = std::min<int64_t>(m0 + 2 * lane, M - 2);
    const int64_t cn = std::min<int64_t>(n0 + 2 * lane, N - 2);
    auto fill = [&](int64_t k0, T (*sa)[kT], T (*sb)[kT]) {
#pragma unroll
      for (int i = 0; i < kBK / 4; ++i) {
        const int r = w + 4 * i;
        const int64_t kg = k0 + r;
        if (kg < kr.e) {
          ring_fill16(A + kg * M + cm, &sa[r][0]);
          ring_fill16(B + kg * N + cn, &sb[r][0]);
        } else {
          *reinterpret_cast<C16*>(&sa[r][2 * lane]) = C16{};
          *reinterpret_cast<C16*>(&sb[r][2 * lane]) = C16{};
        }
      }
    };
    // one slice from (sa, sb) while the next one fills (na, nb)
    auto slice = [&](int64_t k0, T (*sa)[kT], T (*sb)[kT], T (*na)[kT], T (*nb)[kT]) {
      // this slice's fills are done in every wave, and every wave has
      // finished reading the other buffers
      __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (0 << 8) | (0 << 14));
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      // the slice's operands are read before the next fills are issued: an
      // LDS read behind an asynchronous fill waits for that fill
      D4 a4[kBK / 4], b4[kBK / 4];
#pragma unroll
      for (int t = 0; t < kBK / 4; ++t) {
        a4[t] = *reinterpret_cast<const D4*>(&sa[4 * t + g][wm + 4 * c]);
        b4[t] = *reinterpret_cast<const D4*>(&sb[4 * t + g][wn + 4 * c]);
      }
      if (k0 + kBK < kr.e) fill(k0 + kBK, na, nb);
#pragma unroll
      for (int t = 0; t < kBK / 4; ++t)
#pragma unroll
        for (int mm = 0; mm < 4; ++mm)
#pragma unroll
          for (int nn = 0; nn < 4; ++nn)
            acc[mm][nn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a4[t][mm], b4[t][nn],
                                                               acc[mm][nn], 0, 0, 0);
    };
    fill(kr.b, As0, Bs0);
    for (int64_t k0 = kr.b; k0 < kr.e; k0 += 2 * kBK) {
      slice(k0, As0, Bs0, As1, Bs1);
      if (k0 + kBK < kr.e) slice(k0 + kBK, As1, Bs1, As0, Bs0);
    }
  };
  if constexpr (F64) {
    if (late)
      k_loop_async(TypeTag<f64x4>{});
    else
      k_loop(std::true_type{});
  } else {
    k_loop(std::true_type{});
  }

  // epilogue: lane (c, g) register r of tile (mm, nn) holds
  //   m = wm + 4*i + mm with i = 4g + r (f32) or g + 4r (f64),  n = wn + 4c + nn
  double part = 0.0;
  const int64_t nb = n0 + wn + 4 * c;
  T* Cs = C ? C + static_cast<int64_t>(s) * M * N : nullptr;
#pragma unroll
  for (int mm = 0; mm < 4; ++mm) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = F64 ? (g + 4 * r) : (4 * g + r);
      const int64_t m = m0 + wm + 4 * i + mm;
      if (m >= M || nb >= N) continue;
      V4 v = {acc[mm][0][r], acc[mm][1][r], acc[mm][2][r], acc[mm][3][r]};
      if (late && !W) {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = ldexp(v[e], -(ea + eb));
      }
      if (W) {
        double y[4];
        w_sum(W, M * N, w_slices, m * N + nb, y);
#pragma unroll
        for (int e = 0; e < 4; ++e) part += static_cast<double>(v[e]) * y[e];
      } else {
        *reinterpret_cast<V4*>(Cs + m * N + nb) = v;
      }
    }
  }
  if (W) {
    if (late) part = ldexp(part, -(ea + eb));
    const double sum = block_sum(part);
    if (threadIdx.x == 0) partials[static_cast<int64_t>(s) * tiles + tm * ntn + tn] = sum;
  }
}

// ------------------------------------------------ f32, 256 x 256 tiles
// Same operand scheme on a 256 x 256 output tile: eight waves in a 2 (m) x 4
// (n) grid, each 128 x 64 (two 16-byte A reads and one B read per k feed 32
// MFMA tiles).  Twice the flops per staged byte of the 128 x 128 tile; the
// LDS k-slices are double-buffered so one barrier per slice separates staging
// from compute.  Used without split-K, when the output alone fills the chip.
constexpr int kBT = 256;
constexpr int kBThreads = 512;

__global__ __launch_bounds__(kBThreads) void ring_mfma_f32_big(
    const float* __restrict__ A, const float* __restrict__ B, int64_t M, int64_t N, int64_t Kd,
    const int32_t* sa, const int32_t* sb, float* __restrict__ C, const float* __restrict__ W,
    int32_t w_slices, double* __restrict__ partials) {
  __shared__ __attribute__((aligned(16))) float As[2][kBK][kBT];
  __shared__ __attribute__((aligned(16))) float Bs[2][kBK][kBT];
  const uint32_t ntm = static_cast<uint32_t>((M + kBT - 1) / kBT);
  const uint32_t ntn = static_cast<uint32_t>((N + kBT - 1) / kBT);
  uint32_t tm, tn;
  tile_of(tm, tn, ntm, ntn, blockIdx.x);
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
          double y[4];
          w_sum(W, M * N, w_slices, m * N + nb, y);
#pragma unroll
          for (int e = 0; e < 4; ++e) part += static_cast<double>(v[e]) * y[e];
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

// Fused-dot terms of one lane's results, added to part in row order: entry
// (m, n) of the product times the sum of the W slices there, for a lane
// holding rows m = mb + r (r < 4) of column n.
__device__ inline void dot_bf16_lane(double& part, const f32x4& v, const float* __restrict__ W,
                                     int64_t M, int64_t N, int32_t w_slices, int64_t mb,
                                     int64_t n) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t m = mb + r;
    if (m >= M || n >= N) continue;
    double y = static_cast<double>(W[m * N + n]);
    for (int32_t j = 1; j < w_slices; ++j) y += static_cast<double>(W[j * M * N + m * N + n]);
    part += static_cast<double>(v[r]) * y;
  }
}

// ---------------------------------------------- bf16x3 GEMM, k-contiguous
// C[m][n] = sum_k A[m][k] B[n][k] with A, B given as bf16 (hi, lo) pairs
// [rows][kp]; three MFMA products per tile (lo*hi + hi*lo + hi*hi, float32
// accumulation).  Each 32-wide k-slice of the four operand tiles (128 x 32
// bf16 each) is copied to LDS with 16-byte loads (four lanes per 64-byte row
// piece), no conversion; lane (c, g) then reads its 8 consecutive k of row
// wm + 16 t + c with one 16-byte LDS load.  Split-K as ring_mfma.
__global__ __launch_bounds__(kThreads) void ring_bf16x3_nt(
    const uint16_t* __restrict__ Ah, const uint16_t* __restrict__ Al,
    const uint16_t* __restrict__ Bh, const uint16_t* __restrict__ Bl, int64_t M, int64_t N,
    int64_t kp, int32_t S, float* __restrict__ C, const float* __restrict__ W, int32_t w_slices,
    double* __restrict__ partials) {
  __shared__ __attribute__((aligned(16))) uint16_t sAh[kT][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t sAl[kT][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t sBh[kT][kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t sBl[kT][kLdk];
  const uint32_t ntm = static_cast<uint32_t>((M + kT - 1) / kT);
  const uint32_t ntn = static_cast<uint32_t>((N + kT - 1) / kT);
  const uint32_t tiles = ntm * ntn;
  const uint32_t s = blockIdx.x / tiles;
  uint32_t tm, tn;
  tile_of(tm, tn, ntm, ntn, blockIdx.x - s * tiles);
  const KRange kr = k_range(kp, S, s, kBK16);
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

  if (kr.b < kr.e) fetch(kr.b);
  for (int64_t k0 = kr.b; k0 < kr.e; k0 += kBK16) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + kBK16 < kr.e) fetch(k0 + kBK16);
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

  // lane (c, g) register r of tile (mt, nt): m = wm + 16 mt + 4g + r, n = wn + 16 nt + c
  double part = 0.0;
  float* Cs = C ? C + static_cast<int64_t>(s) * M * N : nullptr;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int64_t mb = m0 + wm + 16 * mt + 4 * g, n = n0 + wn + 16 * nt + c;
      if (W) {
        dot_bf16_lane(part, acc[mt][nt], W, M, N, w_slices, mb, n);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (mb + r < M && n < N) Cs[(mb + r) * N + n] = acc[mt][nt][r];
      }
    }
  if (W) {
    const double sum = block_sum(part);
    if (threadIdx.x == 0) partials[static_cast<int64_t>(s) * tiles + tm * ntn + tn] = sum;
  }
}

// ------------------------------------------- bf16x3 NT, 256 x 256 tiles
// ring_bf16x3_nt on a 256 x 256 tile: sixteen waves (4 x 4), each 64 x 64
// (four waves per SIMD to hide LDS latency), so every staged k-slice feeds
// four times the MFMA work of a 128 x 128 tile.  The four 256 x 32 operand
// slices (64 KiB) are double-buffered in LDS and filled with global_load_lds
// (16 bytes per lane straight into LDS, 1 KiB = 16 rows per instruction, no
// registers): the next slice is in flight while the current one is
// multiplied, and one barrier per slice separates the two.  The 16-byte
// chunk j of row r sits at position j ^ ((r / 4) % 4) of its 64-byte row, so
// the 16 lanes of an MFMA-layout read (rows base + c, one chunk) cover all 64
// banks.  Rows past M or N are filled from row M - 1 (N - 1); their products
// are never stored.  Used without split-K, when the output alone fills the
// chip.

// LDS reads that wait for their own results inside the asm block: the
// compiler does not count them as LDS loads, so they do not wait for the
// asynchronous fills of the other buffer that are in flight meanwhile.
typedef __attribute__((address_space(3))) const void* LdsCPtr;
typedef uint32_t u32x4r __attribute__((ext_vector_type(4)));
// Two 16-byte reads at p + O0 and p + O1 (immediate offsets).
template <int O0, int O1>
__device__ inline void lds_read2(const void* p, u16x8& r0, u16x8& r1) {
#if __HIP_DEVICE_COMPILE__
  u32x4r a, b;
  asm volatile(
      "ds_read_b128 %0, %2 offset:%3\n\t"
      "ds_read_b128 %1, %2 offset:%4\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(a), "=&v"(b)
      : "v"((LdsCPtr)p), "i"(O0), "i"(O1)
      : "memory");
  r0 = __builtin_bit_cast(u16x8, a);
  r1 = __builtin_bit_cast(u16x8, b);
#else
  (void)p;
  r0 = r1 = u16x8{};
#endif
}

// Four 16-byte reads at p + O0 .. p + O3 (immediate offsets).
template <int O0, int O1, int O2, int O3>
__device__ inline void lds_read4(const void* p, u16x8 (&r)[4]) {
#if __HIP_DEVICE_COMPILE__
  u32x4r a, b, c, d;
  asm volatile(
      "ds_read_b128 %0, %4 offset:%5\n\t"
      "ds_read_b128 %1, %4 offset:%6\n\t"
      "ds_read_b128 %2, %4 offset:%7\n\t"
      "ds_read_b128 %3, %4 offset:%8\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(a), "=&v"(b), "=&v"(c), "=&v"(d)
      : "v"((LdsCPtr)p), "i"(O0), "i"(O1), "i"(O2), "i"(O3)
      : "memory");
  r[0] = __builtin_bit_cast(u16x8, a);
  r[1] = __builtin_bit_cast(u16x8, b);
  r[2] = __builtin_bit_cast(u16x8, c);
  r[3] = __builtin_bit_cast(u16x8, d);
#else
  (void)p;
  for (int i = 0; i < 4; ++i) r[i] = u16x8{};
#endif
}

constexpr int kB16Threads = 1024;   // 16 waves, 64 x 64 each
__global__ __launch_bounds__(kB16Threads) void ring_bf16x3_nt_big(
    const uint16_t* __restrict__ Ah, const uint16_t* __restrict__ Al,
    const uint16_t* __restrict__ Bh, const uint16_t* __restrict__ Bl, int64_t M, int64_t N,
    int64_t kp, float* __restrict__ C, const float* __restrict__ W, int32_t w_slices,
    double* __restrict__ partials) {
  constexpr int SL = kBT * kBK16;   // entries of one operand slice
  __shared__ __attribute__((aligned(16))) uint16_t sbuf[2][4][SL];
  const uint32_t ntm = static_cast<uint32_t>((M + kBT - 1) / kBT);
  const uint32_t ntn = static_cast<uint32_t>((N + kBT - 1) / kBT);
  uint32_t tm, tn;
  tile_of(tm, tn, ntm, ntn, blockIdx.x);
  const int64_t m0 = static_cast<int64_t>(tm) * kBT, n0 = static_cast<int64_t>(tn) * kBT;
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
  const int wm = (w >> 2) * 64, wn = (w & 3) * 64;

  // fills of one slice: 4 operands x 16 instructions, wave w issuing q = w + 16 i
  // (operand q / 16, rows 16 (q % 16) ..); lane L takes row + L / 4 and puts
  // its chunk at position L % 4, i.e. chunk (L % 4) ^ ((row / 4) % 4)
  const uint16_t* ops[4] = {Ah, Al, Bh, Bl};
  auto fill = [&](int64_t k0, int b) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = w + 16 * i, o = q >> 4, r = 16 * (q & 15) + (lane >> 2);
      const int64_t lim = o < 2 ? M : N;
      const int64_t row = std::min<int64_t>((o < 2 ? m0 : n0) + r, lim - 1);
      const int j = (lane & 3) ^ ((r >> 2) & 3);
      ring_fill16(ops[o] + row * kp + k0 + 8 * j, &sbuf[b][o][16 * (q & 15) * kBK16]);
    }
  };

  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // position of chunk g in rows base + c (base a multiple of 16)
  const int pos = 8 * (g ^ ((c >> 2) & 3));
  fill(0, 0);
  int b = 0;
  for (int64_t k0 = 0; k0 < kp; k0 += kBK16, b ^= 1) {
    // this slice's fills (the only memory operations in flight) are done in
    // every wave, and every wave has finished reading the other buffer
    __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8) | (0 << 14));
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (k0 + kBK16 < kp) fill(k0 + kBK16, b ^ 1);
    const uint16_t* sAh = sbuf[b][0];
    const uint16_t* sBh = sbuf[b][2];
    // operand rows 16 apart are 1 KiB apart, the low parts (sbuf[b][1],
    // sbuf[b][3]) one 16 KiB slice after the high parts: one base address per
    // operand, immediate offsets
    static_assert(16 * kBK16 * 2 == 1024 && SL * 2 == 16384, "operand offsets");
    const uint16_t* pa = sAh + (wm + c) * kBK16 + pos;
    const uint16_t* pb = sBh + (wn + c) * kBK16 + pos;
    u16x8 rh[4], rl[4];
    lds_read4<0, 1024, 2048, 3072>(pb, rh);
    lds_read4<16384, 17408, 18432, 19456>(pb, rl);
    bf16x8 bh[4], bl[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      bh[t] = __builtin_bit_cast(bf16x8, rh[t]);
      bl[t] = __builtin_bit_cast(bf16x8, rl[t]);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      u16x8 h, l;
      if (mt == 0) lds_read2<0, 16384>(pa, h, l);
      if (mt == 1) lds_read2<1024, 17408>(pa, h, l);
      if (mt == 2) lds_read2<2048, 18432>(pa, h, l);
      if (mt == 3) lds_read2<3072, 19456>(pa, h, l);
      const bf16x8 ah = __builtin_bit_cast(bf16x8, h);
      const bf16x8 al = __builtin_bit_cast(bf16x8, l);
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
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int64_t mb = m0 + wm + 16 * mt + 4 * g, n = n0 + wn + 16 * nt + c;
      if (W) {
        dot_bf16_lane(part, acc[mt][nt], W, M, N, w_slices, mb, n);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (mb + r < M && n < N) C[(mb + r) * N + n] = acc[mt][nt][r];
      }
    }
  if (W) {
    __shared__ double red[kB16Threads / 64];
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if (lane == 0) red[w] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int i = 0; i < kB16Threads / 64; ++i) sum += red[i];
      partials[static_cast<int64_t>(tm) * ntn + tn] = sum;
    }
  }
}

// Split count for `tiles` output tiles over `slices` k-slices: double S while
// the grid is short of two workgroups per CU and every split keeps at least
// eight k-slices.
int32_t pick_splits(int64_t tiles, int64_t slices) {
  int32_t s = 1;
  while (tiles * s < kFillGroups && slices >= 16 * s && 2 * s <= kMaxSplits) s *= 2;
  return s;
}

int64_t tiles_of(int64_t m, int64_t n, int64_t edge) {
  return ((m + edge - 1) / edge) * ((n + edge - 1) / edge);
}

// The 256 x 256 kernels run when their tiles alone cover every CU.
bool big_tiles(int64_t m, int64_t n) { return tiles_of(m, n, kBT) >= 256; }

// Clamp S to what the caller's buffers hold: C slices for a stored product,
// partial sums for a fused dot.
int32_t capped(int32_t s, int64_t tiles, bool dot, int32_t c_cap, int64_t p_cap) {
  const int64_t cap = dot ? p_cap / std::max<int64_t>(tiles, 1) : c_cap;
  while (s > 1 && s > cap) s /= 2;
  return s;
}

}  // namespace

void set_ring_operand_scale(int32_t on) { g_ring_operand_scale = on ? 1 : 0; }

bool ring_mfma_supported(const RingArgs& a) {
  return a.m % 4 == 0 && a.n % 4 == 0 && a.m >= 1 && a.n >= 1 && a.k >= 1;
}

int32_t ring_mfma_splits(const RingArgs& a) {
  if (a.type != EL_F64 && a.arith != AR_BF16X3 && big_tiles(a.m, a.n)) return 1;
  return pick_splits(tiles_of(a.m, a.n, kT), (a.k + kBK - 1) / kBK);
}

int64_t ring_mfma_partials_for(const RingArgs& a) {
  if (a.type != EL_F64 && a.arith != AR_BF16X3 && big_tiles(a.m, a.n))
    return tiles_of(a.m, a.n, kBT);
  return tiles_of(a.m, a.n, kT) * ring_mfma_splits(a);
}

hipError_t launch_ring_mfma(const RingArgs& a, hipStream_t stream, const char** kname,
                            int64_t* n_partials, int32_t* c_slices) {
  const bool dot = a.dot_with != nullptr;
  if (a.w_slices < 1 || (dot && a.partials == nullptr) || (!dot && a.c_out == nullptr))
    return hipErrorInvalidValue;
  if (a.type != EL_F64 && a.arith != AR_BF16X3 && big_tiles(a.m, a.n)) {
    const int64_t tiles = tiles_of(a.m, a.n, kBT);
    if (tiles > INT_MAX || (dot && tiles > a.partials_cap)) return hipErrorInvalidValue;
    *kname = "ring_mfma_f32";
    *n_partials = dot ? tiles : 0;
    *c_slices = 1;
    hipLaunchKernelGGL(ring_mfma_f32_big, dim3(static_cast<uint32_t>(tiles)), dim3(kBThreads), 0,
                       stream, static_cast<const float*>(a.A), static_cast<const float*>(a.B), a.m,
                       a.n, a.k, a.sa, a.sb, static_cast<float*>(a.c_out),
                       static_cast<const float*>(a.dot_with), a.w_slices, a.partials);
    return hipGetLastError();
  }
  const int64_t tiles = tiles_of(a.m, a.n, kT);
  const int32_t S = capped(ring_mfma_splits(a), tiles, dot, a.c_slices_cap, a.partials_cap);
  if (tiles * S > INT_MAX || (dot && tiles * S > a.partials_cap) || (!dot && S > a.c_slices_cap))
    return hipErrorInvalidValue;
  const dim3 grid(static_cast<uint32_t>(tiles * S)), block(kThreads);
  *n_partials = dot ? tiles * S : 0;
  *c_slices = dot ? 0 : S;
  if (a.type == EL_F64) {
    *kname = "ring_mfma_f64";
    hipLaunchKernelGGL((ring_mfma<double>), grid, block, 0, stream,
                       static_cast<const double*>(a.A), static_cast<const double*>(a.B), a.m, a.n,
                       a.k, S, a.sa, a.sb, static_cast<double*>(a.c_out),
                       static_cast<const double*>(a.dot_with), a.w_slices, a.partials,
                       g_ring_operand_scale);
  } else if (a.arith == AR_BF16X3) {
    return hipErrorInvalidValue;   // split BF16x3 rings go through launch_ring_bf16x3_nt
  } else {
    *kname = "ring_mfma_f32";
    hipLaunchKernelGGL((ring_mfma<float>), grid, block, 0, stream,
                       static_cast<const float*>(a.A), static_cast<const float*>(a.B), a.m, a.n,
                       a.k, S, a.sa, a.sb, static_cast<float*>(a.c_out),
                       static_cast<const float*>(a.dot_with), a.w_slices, a.partials, 1);
  }
  return hipGetLastError();
}

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

int32_t ring_bf16x3_nt_splits(int64_t m, int64_t n, int64_t kp) {
  if (big_tiles(m, n)) return 1;
  return pick_splits(tiles_of(m, n, kT), (kp + kBK16 - 1) / kBK16);
}

int64_t ring_bf16x3_nt_partials(int64_t m, int64_t n, int64_t kp) {
  if (big_tiles(m, n)) return tiles_of(m, n, kBT);
  return tiles_of(m, n, kT) * ring_bf16x3_nt_splits(m, n, kp);
}

hipError_t launch_ring_bf16x3_nt(const NtArgs& a, hipStream_t stream, int64_t* n_partials,
                                 int32_t* c_slices) {
  const bool dot = a.dot_with != nullptr;
  if (a.w_slices < 1 || (dot && a.partials == nullptr) || (!dot && a.c_out == nullptr) ||
      a.kp % kBK16 != 0)
    return hipErrorInvalidValue;
  if (big_tiles(a.m, a.n)) {
    const int64_t tiles = tiles_of(a.m, a.n, kBT);
    if (tiles > INT_MAX || (dot && tiles > a.partials_cap)) return hipErrorInvalidValue;
    *n_partials = dot ? tiles : 0;
    *c_slices = 1;
    hipLaunchKernelGGL(ring_bf16x3_nt_big, dim3(static_cast<uint32_t>(tiles)), dim3(kB16Threads), 0,
                       stream, a.Ah, a.Al, a.Bh, a.Bl, a.m, a.n, a.kp, a.c_out, a.dot_with,
                       a.w_slices, a.partials);
    return hipGetLastError();
  }
  const int64_t tiles = tiles_of(a.m, a.n, kT);
  const int32_t S =
      capped(ring_bf16x3_nt_splits(a.m, a.n, a.kp), tiles, dot, a.c_slices_cap, a.partials_cap);
  if (tiles * S > INT_MAX || (dot && tiles * S > a.partials_cap) || (!dot && S > a.c_slices_cap))
    return hipErrorInvalidValue;
  *n_partials = dot ? tiles * S : 0;
  *c_slices = dot ? 0 : S;
  hipLaunchKernelGGL(ring_bf16x3_nt, dim3(static_cast<uint32_t>(tiles * S)), dim3(kThreads), 0,
                     stream, a.Ah, a.Al, a.Bh, a.Bl, a.m, a.n, a.kp, S, a.c_out, a.dot_with,
                     a.w_slices, a.partials);
  return hipGetLastError();
}

}  // namespace tn
