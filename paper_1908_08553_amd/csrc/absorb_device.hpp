// Single-site absorption on the gfx950 matrix cores.
//
// out[p][n][q] = sum_k (2^-shift in[p][k][q]) * S[k][n] with K, N <= 16 (every
// step of a lattice with bond dimension <= 4).  Each wavefront multiplies
// 16-fibre blocks of the boundary by the 16x16 (zero-padded) site matrix with
// 16x16 MFMA tiles; a fibre is one (p, q) pair.  Two data paths, chosen by the
// contiguous extent `post`:
//
//  * wide   (post % 64 == 0): 64 consecutive q of one p per super-block, each
//    lane loading 4 consecutive q (see the comment above absorb_wide).
//  * narrow (post == 1): the boundary is a row-major (pre x K) matrix.  MFMA
//    rows are n, columns are 16 consecutive p; lane (c, g) loads the 16-byte
//    slice in[p0+c][4g..4g+3] and feeds its four entries to four successive
//    MFMAs, so lane group g covers k = 4g..4g+3 (the sum over k is split
//    between lane groups instead of instructions).  Stores are 16-byte slices
//    of out[p0+c][4g..4g+3].  Both directions read/write whole 1 KiB spans.
//
// Result layouts (measured on gfx950): the f32 and bf16 16x16 MFMAs leave
// D[4g+r][c] in register r of lane (c, g); the f64 MFMA leaves D[g+4r][c].  The
// narrow f64 path feeds its A-operand rows in the order sigma(i) = 4(i%4) + i/4
// (a 4x4 transpose, its own inverse) so every lane again holds four
// consecutive outputs; the wide path folds the layout into its store offsets.
//
// Arithmetic: F32 -> v_mfma_f32_16x16x4_f32; F64 -> v_mfma_f64_16x16x4_f64;
// BF16X3 -> v_mfma_f32_16x16x32_bf16 on the K-concatenation
// [x_hi s_hi | x_hi s_lo | x_lo s_hi | 0] (products of the bf16 high/low
// parts of both operands, float32 accumulation).
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <type_traits>

#include "kernels.hpp"

namespace tn {
namespace dev {


typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kBlocksPerWave = 8;

enum Mode { M_F32 = 0, M_F64 = 1, M_BF16X3 = 2 };

__device__ inline int32_t exp_of_d(double m) {
  if (!(m == m) || m > 1.7976931348623157e308) return kExpBad;
  if (m == 0.0) return kExpZero;
  int e;
  (void)frexp(m, &e);
  return e;
}

__device__ inline int32_t shift_of(const int32_t* slot) {
  if (!slot) return 0;
  const int32_t e = *slot;
  return (e == kExpZero || e == kExpBad) ? 0 : e;
}

__device__ inline __bf16 bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  const uint16_t b = static_cast<uint16_t>(u >> 16);
  return __builtin_bit_cast(__bf16, b);
}
__device__ inline float bf16_to_f(__bf16 b) {
  return __uint_as_float(static_cast<uint32_t>(__builtin_bit_cast(uint16_t, b)) << 16);
}

template <typename T, int NW = kWaves>
__device__ inline void reduce_and_publish(T mx, int bad, int32_t* max_slot, int32_t* flags) {
  __shared__ double sm[NW];
  __shared__ int sb[NW];
  double m = static_cast<double>(mx);
  for (int off = 32; off > 0; off >>= 1) {
    m = fmax(m, __shfl_xor(m, off));
    bad |= __shfl_xor(bad, off);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { sm[w] = m; sb[w] = bad; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < NW; ++k) { m = fmax(m, sm[k]); bad |= sb[k]; }
    m = fmax(m, sm[0]);
    bad |= sb[0];
    const int32_t e = bad ? kExpBad : exp_of_d(m);
    // the slot only grows during a launch: skip the atomic (all workgroups
    // of a launch would queue on one cache line) when it cannot raise it
    if (e != kExpZero && e > __hip_atomic_load(max_slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(max_slot, e);
    if (bad) atomicOr(flags, 1);
  }
}

template <typename T>
__device__ inline void track(T v, T& mx, int& bad) {
  bad |= !isfinite(v);
  mx = fmax(mx, fabs(v));
}

// ------------------------------------------------------------------ wide
// Super-block = 64 consecutive fibres j0..j0+63 of the flattened (p, q)
// index (post % 4 == 0, so each lane's four fibres share one p).  Lane (c, g)
// loads the vector in[p][k][q..q+3] of fibres j0+4c..j0+4c+3 for k = 4kk+g;
// for post >= 64 each load instruction reads four 256-byte (512-byte for f64)
// runs, for smaller post four runs of 4*post entries per slab.  MFMA m (m = 0..3) consumes element m of every lane's vector: its rows
// are the fibres 4c+m.  With the f32/bf16 result layout, register r of MFMA m
// in lane (c, g) is fibre 16g+4r+m of output column n = c, so the four MFMAs'
// r-th registers form one 16-byte store; with the f64 layout it is fibre
// 4g+16r+m.  All loads of a wave's super-blocks are issued before its MFMAs.
constexpr int kSuperPerWave = 2;

// Waves wave0, wave0 + nwaves, ... of the caller each take kSuperPerWave
// consecutive super-blocks; |out| maxima and non-finite flags accumulate in
// (mx, bad).
template <typename Tin, typename Tout, int MODE>
__device__ inline void wide_body(const Tin* __restrict__ in, Tout* __restrict__ out,
                                 const Tout* __restrict__ S, const uint16_t* __restrict__ shi,
                                 const uint16_t* __restrict__ slo, int64_t pre, int32_t K,
                                 int32_t N, int64_t post, int32_t shift, uint32_t wave0,
                                 uint32_t nwaves, Tout& mx, int& bad) {
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
  const uint32_t nfib = static_cast<uint32_t>(pre * post);
  const uint32_t upost = static_cast<uint32_t>(post);
  const uint32_t nsb = (nfib + 63) / 64;
  using VI = typename std::conditional<std::is_same<Tin, double>::value, f64x4, f32x4>::type;
  using VO = typename std::conditional<MODE == M_F64, f64x4, f32x4>::type;
  if constexpr (MODE == M_BF16X3) {
    // B operand (site): segments [s_hi | s_lo | s_hi | 0] over k' = 0..63
    const int kb = 8 * (g & 1);
    bf16x8 b0, b1;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = kb + t;
      const bool ok = k < K && c < N;
      const uint16_t hb = ok ? shi[k * N + c] : 0, lb = ok ? slo[k * N + c] : 0;
      b0[t] = __builtin_bit_cast(__bf16, g < 2 ? hb : lb);
      b1[t] = __builtin_bit_cast(__bf16, g < 2 ? hb : static_cast<uint16_t>(0));
    }
    for (uint32_t wave = wave0; wave * kSuperPerWave < nsb; wave += nwaves) {
    f32x4 x[kSuperPerWave][8];
#pragma unroll
    for (int sb = 0; sb < kSuperPerWave; ++sb) {
      const uint32_t f = (wave * kSuperPerWave + sb) * 64 + 4 * c;
      const bool ok = f < nfib;
      const uint32_t p = ok ? f / upost : 0, q = ok ? f - p * upost : 0;
      const float* src = in + static_cast<int64_t>(p) * K * post + q;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int k = kb + t;
        x[sb][t] = (ok && k < K) ? *reinterpret_cast<const f32x4*>(src + k * post)
                                 : f32x4{0.f, 0.f, 0.f, 0.f};
      }
    }
#pragma unroll
    for (int sb = 0; sb < kSuperPerWave; ++sb) {
      const uint32_t blk = wave * kSuperPerWave + sb;
      if (blk >= nsb) continue;
      const uint32_t j0 = blk * 64;
      f32x4 acc[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        bf16x8 a0, a1;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const float xs = ldexpf(x[sb][t][m], -shift);
          const __bf16 h = bf16_rne(xs);
          a0[t] = h;
          a1[t] = g < 2 ? bf16_rne(xs - bf16_to_f(h))
                        : __builtin_bit_cast(__bf16, static_cast<uint16_t>(0));
        }
        acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[m], 0, 0, 0);
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[m], 0, 0, 0);
      }
      if (c < N) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t fo = j0 + 16 * g + 4 * r;
          if (fo >= nfib) continue;
          const uint32_t p = fo / upost, q = fo - p * upost;
          const f32x4 v = {acc[0][r], acc[1][r], acc[2][r], acc[3][r]};
          *reinterpret_cast<f32x4*>(out + static_cast<int64_t>(p) * N * post +
                                    static_cast<int64_t>(c) * post + q) = v;
#pragma unroll
          for (int m = 0; m < 4; ++m) track(v[m], mx, bad);
        }
      }
    }
    }
  } else {
    Tout b[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 4 * kk + g;
      b[kk] = (k < K && c < N) ? S[k * N + c] : Tout(0);
    }
    const int kg = (K + 3) >> 2;
    for (uint32_t wave = wave0; wave * kSuperPerWave < nsb; wave += nwaves) {
    VI x[kSuperPerWave][4];
#pragma unroll
    for (int sb = 0; sb < kSuperPerWave; ++sb) {
      const uint32_t f = (wave * kSuperPerWave + sb) * 64 + 4 * c;
      const bool ok = f < nfib;
      const uint32_t p = ok ? f / upost : 0, q = ok ? f - p * upost : 0;
      const Tin* src = in + static_cast<int64_t>(p) * K * post + q;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int k = 4 * kk + g;
        x[sb][kk] = (ok && kk < kg && k < K) ? *reinterpret_cast<const VI*>(src + k * post)
                                             : VI{0, 0, 0, 0};
      }
    }
#pragma unroll
    for (int sb = 0; sb < kSuperPerWave; ++sb) {
      const uint32_t blk = wave * kSuperPerWave + sb;
      if (blk >= nsb) continue;
      const uint32_t j0 = blk * 64;
      VO acc[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        acc[m] = VO{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          if (kk < kg) {
            const Tout a = static_cast<Tout>(ldexp(static_cast<Tout>(x[sb][kk][m]), -shift));
            if constexpr (MODE == M_F64)
              acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[kk], acc[m], 0, 0, 0);
            else
              acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[kk], acc[m], 0, 0, 0);
          }
        }
      }
      if (c < N) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t fo = j0 + ((MODE == M_F64) ? (4 * g + 16 * r) : (16 * g + 4 * r));
          if (fo >= nfib) continue;
          const uint32_t p = fo / upost, q = fo - p * upost;
          const VO v = {acc[0][r], acc[1][r], acc[2][r], acc[3][r]};
          *reinterpret_cast<VO*>(out + static_cast<int64_t>(p) * N * post +
                                 static_cast<int64_t>(c) * post + q) = v;
#pragma unroll
          for (int m = 0; m < 4; ++m) track(v[m], mx, bad);
        }
      }
    }
    }
  }
}

// ---------------------------------------------------------------- narrow
template <typename Tin, typename Tout, int MODE>
__device__ inline void narrow_body(const Tin* __restrict__ in, Tout* __restrict__ out,
                                   const Tout* __restrict__ S, const uint16_t* __restrict__ shi,
                                   const uint16_t* __restrict__ slo, int64_t pre, int32_t K,
                                   int32_t N, int32_t shift, uint32_t wave0, uint32_t nwaves,
                                   Tout& mx, int& bad) {
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
  const int64_t nblk = (pre + 15) / 16;
  if constexpr (MODE == M_BF16X3) {
    const int kb = 8 * (g & 1);
    bf16x8 a0, a1;   // A operand: site^T segments [s_hi | s_lo | s_hi | 0]
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = kb + t;
      const bool ok = k < K && c < N;
      const uint16_t hb = ok ? shi[k * N + c] : 0, lb = ok ? slo[k * N + c] : 0;
      a0[t] = __builtin_bit_cast(__bf16, g < 2 ? hb : lb);
      a1[t] = __builtin_bit_cast(__bf16, g < 2 ? hb : static_cast<uint16_t>(0));
    }
    for (int64_t wave = wave0; wave * kBlocksPerWave < nblk; wave += nwaves) {
#pragma unroll
    for (int bi = 0; bi < kBlocksPerWave; ++bi) {
      const int64_t blk = wave * kBlocksPerWave + bi;
      if (blk >= nblk) break;
      const int64_t p = blk * 16 + c;
      float x[8];
      if (p < pre && kb < K) {
        const f32x4* src = reinterpret_cast<const f32x4*>(in + p * K + kb);
        const f32x4 u = src[0];
        const f32x4 v = (kb + 4 < K) ? src[1] : f32x4{0.f, 0.f, 0.f, 0.f};
        x[0] = u[0]; x[1] = u[1]; x[2] = u[2]; x[3] = u[3];
        x[4] = v[0]; x[5] = v[1]; x[6] = v[2]; x[7] = v[3];
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) x[t] = 0.f;
      }
      bf16x8 b0, b1;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const float xs = ldexpf(x[t], -shift);
        const __bf16 h = bf16_rne(xs);
        b0[t] = h;
        b1[t] = g < 2 ? bf16_rne(xs - bf16_to_f(h)) : __builtin_bit_cast(__bf16, static_cast<uint16_t>(0));
      }
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc, 0, 0, 0);
      if (p < pre && 4 * g < N) {
        *reinterpret_cast<f32x4*>(out + p * N + 4 * g) = acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) track(acc[r], mx, bad);
      }
    }
    }
  } else {
    using V4 = typename std::conditional<MODE == M_F64, f64x4, f32x4>::type;
    using I4 = typename std::conditional<std::is_same<Tin, double>::value, f64x4, f32x4>::type;
    Tout a[4];   // A operand: S^T[n = cs][k = 4g + kk]
    const int cs = (MODE == M_F64) ? (4 * (c & 3) + (c >> 2)) : c;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 4 * g + kk;
      a[kk] = (k < K && cs < N) ? S[k * N + cs] : Tout(0);
    }
    for (int64_t wave = wave0; wave * kBlocksPerWave < nblk; wave += nwaves) {
    I4 v[kBlocksPerWave];
#pragma unroll
    for (int bi = 0; bi < kBlocksPerWave; ++bi) {
      const int64_t p = (wave * kBlocksPerWave + bi) * 16 + c;
      v[bi] = (p < pre && 4 * g < K) ? *reinterpret_cast<const I4*>(in + p * K + 4 * g)
                                     : I4{0, 0, 0, 0};
    }
#pragma unroll
    for (int bi = 0; bi < kBlocksPerWave; ++bi) {
      const int64_t blk = wave * kBlocksPerWave + bi;
      if (blk >= nblk) continue;
      const int64_t p = blk * 16 + c;
      V4 acc = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const Tout b = static_cast<Tout>(ldexp(static_cast<Tout>(v[bi][kk]), -shift));
        if constexpr (MODE == M_F64)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], b, acc, 0, 0, 0);
        else
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kk], b, acc, 0, 0, 0);
      }
      if (p < pre && 4 * g < N) {
        *reinterpret_cast<V4*>(out + p * N + 4 * g) = acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) track(acc[r], mx, bad);
      }
    }
    }
  }
}

// ------------------------------------------------------- any shape (VALU)
// Threads thread0, thread0 + nthreads, ... each own one (p, q) fibre: K loads
// at stride post, N accumulators in chunks of 16, N stores at stride post.
// Used where the MFMA bodies do not apply (K or N > 16, post not a multiple
// of 4 and not 1, or K, N not multiples of 4 with post == 1).
template <typename Tin, typename Tc, bool SPLIT>
__device__ inline void generic_body(const Tin* __restrict__ in, Tc* __restrict__ out,
                                    const Tc* __restrict__ S, const uint16_t* __restrict__ shi,
                                    const uint16_t* __restrict__ slo, int64_t pre, int32_t K,
                                    int32_t N, int64_t post, int32_t shift, int64_t thread0,
                                    int64_t nthreads, Tc& mx, int& bad) {
  const int64_t nf = pre * post;
  for (int64_t f = thread0; f < nf; f += nthreads) {
    const int64_t p = f / post, q = f - p * post;
    const Tin* src = in + p * K * post + q;
    Tc* dst = out + p * N * post + q;
    for (int32_t n0 = 0; n0 < N; n0 += 16) {
      const int32_t nn = min(16, N - n0);
      Tc acc[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] = 0;
      for (int32_t k = 0; k < K; ++k) {
        const Tc x = static_cast<Tc>(ldexp(static_cast<Tc>(src[k * post]), -shift));
        if constexpr (SPLIT) {
          const float xh = bf16_to_f(bf16_rne(static_cast<float>(x)));
          const float xl = bf16_to_f(bf16_rne(static_cast<float>(x) - xh));
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            if (j < nn) {
              const float sh = __uint_as_float(static_cast<uint32_t>(shi[k * N + n0 + j]) << 16);
              const float sl = __uint_as_float(static_cast<uint32_t>(slo[k * N + n0 + j]) << 16);
              float a = acc[j];
              a = fmaf(xl, sh, a);
              a = fmaf(xh, sl, a);
              a = fmaf(xh, sh, a);
              acc[j] = a;
            }
          }
        } else {
#pragma unroll
          for (int j = 0; j < 16; ++j)
            if (j < nn) acc[j] = fma(x, S[k * N + n0 + j], acc[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        if (j < nn) {
          dst[(n0 + j) * post] = acc[j];
          track(acc[j], mx, bad);
        }
      }
    }
  }
}

// Z = m * 2^E assembled into a tn_result (sign, exponent sum, log|Z|).
__device__ inline tn_result assemble_result(double m, int64_t E, int bad) {
  tn_result r;
  if (!isfinite(m)) bad = 1;
  r.status = bad ? TN_ENONFINITE : TN_OK;
  if (bad || m == 0.0) {
    r.sign = 0;
    r.mantissa = 0.0;
    r.exp2_sum = 0;
    r.log_abs = bad ? __builtin_nan("") : -INFINITY;
    r.value = bad ? __builtin_nan("") : 0.0;
    return r;
  }
  int em;
  const double f = frexp(m, &em);
  r.sign = f > 0 ? 1 : -1;
  r.mantissa = f;
  r.exp2_sum = E + em;
  r.log_abs = static_cast<double>(r.exp2_sum) * 0.69314718055994530942 + log(fabs(f));
  const int64_t ex = r.exp2_sum;
  r.value = (ex > 2000) ? r.sign * INFINITY
                        : (ex < -2000 ? 0.0 * r.sign : ldexp(f, static_cast<int>(ex)));
  return r;
}

// Shape tests shared by the per-step launchers and the batched kernel.
__host__ __device__ inline bool wide_ok(int64_t pre, int64_t K, int64_t N, int64_t post) {
  return K >= 1 && N >= 1 && K <= 16 && N <= 16 && post % 4 == 0 &&
         pre * post < (int64_t(1) << 31);
}
__host__ __device__ inline bool narrow_ok(int64_t pre, int64_t K, int64_t N, int64_t post) {
  return K >= 1 && N >= 1 && K <= 16 && N <= 16 && post == 1 && K % 4 == 0 && N % 4 == 0;
}

}  // namespace dev
}  // namespace tn
