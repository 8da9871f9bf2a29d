// Single-site absorption kernels on the gfx950 matrix cores; the per-wave
// bodies live in absorb_device.hpp (shared with the batch kernel).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>

#include "absorb_device.hpp"
#include "kernels.hpp"

namespace tn {
namespace {

using namespace dev;

template <typename Tin, typename Tout, int MODE>
__global__ __launch_bounds__(kThreads) void absorb_wide(
    const Tin* __restrict__ in, Tout* __restrict__ out, const Tout* __restrict__ S,
    const uint16_t* __restrict__ shi, const uint16_t* __restrict__ slo, int64_t pre, int32_t K,
    int32_t N, int64_t post, const int32_t* scale_slot, int32_t* max_slot, int32_t* flags) {
  Tout mx = 0;
  int bad = 0;
  wide_body<Tin, Tout, MODE>(in, out, S, shi, slo, pre, K, N, post, shift_of(scale_slot),
                             blockIdx.x * kWaves + (threadIdx.x >> 6), gridDim.x * kWaves, mx,
                             bad);
  if (max_slot) reduce_and_publish(mx, bad, max_slot, flags);
}

template <typename Tin, typename Tout, int MODE>
__global__ __launch_bounds__(kThreads) void absorb_narrow(
    const Tin* __restrict__ in, Tout* __restrict__ out, const Tout* __restrict__ S,
    const uint16_t* __restrict__ shi, const uint16_t* __restrict__ slo, int64_t pre, int32_t K,
    int32_t N, const int32_t* scale_slot, int32_t* max_slot, int32_t* flags) {
  Tout mx = 0;
  int bad = 0;
  narrow_body<Tin, Tout, MODE>(in, out, S, shi, slo, pre, K, N, shift_of(scale_slot),
                               blockIdx.x * kWaves + (threadIdx.x >> 6), gridDim.x * kWaves, mx,
                               bad);
  if (max_slot) reduce_and_publish(mx, bad, max_slot, flags);
}

// ------------------------------------------------------------- grouped
// Up to four independent steps of the same kind in one launch (the quadrant
// sweeps: same step index of each quadrant).  Workgroups [first[u], first[u+1])
// belong to step u.
constexpr int kMaxGroup = 4;

struct GroupStep {
  const void* in;
  void* out;
  const void* S;
  const uint16_t* shi;
  const uint16_t* slo;
  int64_t pre, post;
  int32_t K, N;
  const int32_t* scale_slot;
  int32_t* max_slot;
};

struct Group {
  GroupStep s[kMaxGroup];
  uint32_t first[kMaxGroup + 1];
  int32_t n;
  int32_t* flags;
};

template <typename Tin, typename Tout, int MODE, bool WIDE>
__global__ __launch_bounds__(kThreads) void absorb_group(Group g) {
  int u = 0;
  while (u + 1 < g.n && blockIdx.x >= g.first[u + 1]) ++u;
  const GroupStep& st = g.s[u];
  const uint32_t nb = g.first[u + 1] - g.first[u];
  const uint32_t wave0 = (blockIdx.x - g.first[u]) * kWaves + (threadIdx.x >> 6);
  Tout mx = 0;
  int bad = 0;
  if constexpr (WIDE)
    wide_body<Tin, Tout, MODE>(static_cast<const Tin*>(st.in), static_cast<Tout*>(st.out),
                               static_cast<const Tout*>(st.S), st.shi, st.slo, st.pre, st.K,
                               st.N, st.post, shift_of(st.scale_slot), wave0, nb * kWaves, mx,
                               bad);
  else
    narrow_body<Tin, Tout, MODE>(static_cast<const Tin*>(st.in), static_cast<Tout*>(st.out),
                                 static_cast<const Tout*>(st.S), st.shi, st.slo, st.pre, st.K,
                                 st.N, shift_of(st.scale_slot), wave0, nb * kWaves, mx, bad);
  if (st.max_slot) reduce_and_publish(mx, bad, st.max_slot, g.flags);
}

template <typename Tin, typename Tout, int MODE>
hipError_t go_group(const AbsorbArgs* a, int32_t n, bool wide, const StagedArrays& st,
                    DevState* state, hipStream_t stream) {
  Group g;
  std::memset(&g, 0, sizeof(g));
  g.n = n;
  g.flags = &state->flags;
  uint32_t total = 0;
  for (int32_t u = 0; u < n; ++u) {
    const AbsorbArgs& x = a[u];
    GroupStep& s = g.s[u];
    s.in = x.in;
    s.out = x.out;
    s.S = (MODE == M_F64) ? static_cast<const void*>(st.s64 + x.s_off)
                          : static_cast<const void*>(st.s32 + x.s_off);
    s.shi = st.shi + x.s_off;
    s.slo = st.slo + x.s_off;
    s.pre = x.pre;
    s.post = x.post;
    s.K = static_cast<int32_t>(x.K);
    s.N = static_cast<int32_t>(x.N);
    s.scale_slot = x.scale_slot;
    s.max_slot = x.max_slot;
    const int64_t units = wide ? (x.pre * x.post + 63) / 64 : (x.pre + 15) / 16;
    const int64_t per_block = wide ? kWaves * kSuperPerWave : kWaves * kBlocksPerWave;
    const int64_t blocks = std::max<int64_t>(1, (units + per_block - 1) / per_block);
    g.first[u] = total;
    if (total + blocks > static_cast<int64_t>(INT_MAX)) return hipErrorInvalidValue;
    total += static_cast<uint32_t>(blocks);
  }
  g.first[n] = total;
  if (wide)
    hipLaunchKernelGGL((absorb_group<Tin, Tout, MODE, true>), dim3(total), dim3(kThreads), 0,
                       stream, g);
  else
    hipLaunchKernelGGL((absorb_group<Tin, Tout, MODE, false>), dim3(total), dim3(kThreads), 0,
                       stream, g);
  return hipGetLastError();
}

// --------------------------------------------------------- fused pairs
// Two consecutive bulk steps of one column, s1 then s2, in one pass over the
// boundary (D = 4: K = N = 16 for both; s2.pre = 4 s1.pre, s1.post =
// 4 s2.post = 4 P).  With the zipper order s1 contracts (v, h_r) into
// (h'_r, v'') and s2 contracts (v'', h_{r+1}), so for a fixed slab p and a
// run of 64 consecutive q (q < P) the 4 x 64 s1-fibres q1 = h P + q (h =
// h_{r+1}) hold everything s2 needs for its fibres (4p + h'_r, q).  Workgroup
// = 4 waves: wave h applies s1 to fibres h P + q0 .. + 63 and leaves its
// 16 x 64 results in LDS; after a barrier wave h' gathers (v'', h) for
// h'_r = h' from LDS and applies s2, storing 16 contiguous 256-byte rows.
// Boundary traffic of the pair drops from 4 passes to 2.
struct PairStep {
  const void* in;
  void* out;
  const void* S1;
  const void* S2;
  const uint16_t* h1;
  const uint16_t* l1;
  const uint16_t* h2;
  const uint16_t* l2;
  int64_t pre, post2;
  const int32_t* scale_slot;
  int32_t* max_slot;
};

struct PairGroup {
  PairStep s[kMaxGroup];
  uint32_t first[kMaxGroup + 1];
  int32_t n;
  int32_t* flags;
};

constexpr int kPairLd = 68;

template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void absorb_pair(PairGroup g) {
  constexpr bool F64 = MODE == M_F64;
  using V4 = typename std::conditional<F64, f64x4, f32x4>::type;
  // rows padded to 68 entries: the 16 rows a wave stores at one fibre offset
  // land on distinct LDS banks
  __shared__ __attribute__((aligned(32))) T buf[4][16][kPairLd];
  int u = 0;
  while (u + 1 < g.n && blockIdx.x >= g.first[u + 1]) ++u;
  const PairStep& st = g.s[u];
  const int64_t tiles_q = st.post2 / 64;
  const int64_t t = blockIdx.x - g.first[u];
  const int64_t p = t / tiles_q, q0 = (t - p * tiles_q) * 64;
  const int lane = threadIdx.x & 63, c = lane & 15, gg = lane >> 4, w = threadIdx.x >> 6;
  const int64_t P = st.post2, post1 = 4 * P;
  const int32_t shift = shift_of(st.scale_slot);
  const T* in = static_cast<const T*>(st.in);
  T* out = static_cast<T*>(st.out);

  // ---- s1 on fibres q1 = w P + q0 + 4c .. +3 (64 per wave)
  {
    const T* src = in + p * 16 * post1 + static_cast<int64_t>(w) * P + q0 + 4 * c;
    V4 acc[4];
    if constexpr (MODE == M_BF16X3) {
      const int kb = 8 * (gg & 1);
      bf16x8 b0, b1;
#pragma unroll
      for (int tt = 0; tt < 8; ++tt) {
        const uint16_t hb = st.h1[(kb + tt) * 16 + c], lb = st.l1[(kb + tt) * 16 + c];
        b0[tt] = __builtin_bit_cast(__bf16, gg < 2 ? hb : lb);
        b1[tt] = __builtin_bit_cast(__bf16, gg < 2 ? hb : static_cast<uint16_t>(0));
      }
      f32x4 x[8];
#pragma unroll
      for (int tt = 0; tt < 8; ++tt) x[tt] = *reinterpret_cast<const f32x4*>(src + (kb + tt) * post1);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        bf16x8 a0, a1;
#pragma unroll
        for (int tt = 0; tt < 8; ++tt) {
          const float xs = ldexpf(x[tt][m], -shift);
          const __bf16 h = bf16_rne(xs);
          a0[tt] = h;
          a1[tt] = gg < 2 ? bf16_rne(xs - bf16_to_f(h))
                          : __builtin_bit_cast(__bf16, static_cast<uint16_t>(0));
        }
        acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[m], 0, 0, 0);
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[m], 0, 0, 0);
      }
    } else {
      const T* S1 = static_cast<const T*>(st.S1);
      V4 x[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) x[kk] = *reinterpret_cast<const V4*>(src + (4 * kk + gg) * post1);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        acc[m] = V4{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const T a = static_cast<T>(ldexp(x[kk][m], -shift));
          const T b = S1[(4 * kk + gg) * 16 + c];
          if constexpr (F64)
            acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[m], 0, 0, 0);
          else
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[m], 0, 0, 0);
        }
      }
    }
    // register r of MFMA m in lane (c, gg): fibre (F64 ? 4gg + 16r : 16gg + 4r) + m, n1 = c
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int f = F64 ? (4 * gg + 16 * r) : (16 * gg + 4 * r);
      const V4 v = {acc[0][r], acc[1][r], acc[2][r], acc[3][r]};
      *reinterpret_cast<V4*>(&buf[w][c][f]) = v;
    }
  }
  __syncthreads();

  // ---- s2 for h'_r = w: A[fibre q][k2 = (v'', h)] = buf[h][4w + v''][q]
  T mx = 0;
  int bad = 0;
  {
    V4 acc[4];
    if constexpr (MODE == M_BF16X3) {
      const int kb = 8 * (gg & 1);
      bf16x8 b0, b1;
#pragma unroll
      for (int tt = 0; tt < 8; ++tt) {
        const uint16_t hb = st.h2[(kb + tt) * 16 + c], lb = st.l2[(kb + tt) * 16 + c];
        b0[tt] = __builtin_bit_cast(__bf16, gg < 2 ? hb : lb);
        b1[tt] = __builtin_bit_cast(__bf16, gg < 2 ? hb : static_cast<uint16_t>(0));
      }
      f32x4 x[8];
#pragma unroll
      for (int tt = 0; tt < 8; ++tt) {
        const int k2 = kb + tt;
        x[tt] = *reinterpret_cast<const f32x4*>(&buf[k2 & 3][4 * w + (k2 >> 2)][4 * c]);
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        bf16x8 a0, a1;
#pragma unroll
        for (int tt = 0; tt < 8; ++tt) {
          const float xs = x[tt][m];
          const __bf16 h = bf16_rne(xs);
          a0[tt] = h;
          a1[tt] = gg < 2 ? bf16_rne(xs - bf16_to_f(h))
                          : __builtin_bit_cast(__bf16, static_cast<uint16_t>(0));
        }
        acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[m], 0, 0, 0);
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[m], 0, 0, 0);
      }
    } else {
      const T* S2 = static_cast<const T*>(st.S2);
      V4 x[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)   // k2 = 4 kk + gg: v'' = kk, h = gg
        x[kk] = *reinterpret_cast<const V4*>(&buf[gg][4 * w + kk][4 * c]);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        acc[m] = V4{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const T b = S2[(4 * kk + gg) * 16 + c];
          if constexpr (F64)
            acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[kk][m], b, acc[m], 0, 0, 0);
          else
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[kk][m], b, acc[m], 0, 0, 0);
        }
      }
    }
    // results go back through the wave's own LDS rows (every wave has read
    // its s2 operands once the barrier passes) so that each 16 lanes store
    // one whole 64-fibre output row
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int f = F64 ? (4 * gg + 16 * r) : (16 * gg + 4 * r);
      const V4 v = {acc[0][r], acc[1][r], acc[2][r], acc[3][r]};
      *reinterpret_cast<V4*>(&buf[w][c][f]) = v;
#pragma unroll
      for (int m = 0; m < 4; ++m) track(v[m], mx, bad);
    }
    __syncthreads();
    T* dst = out + (4 * p + w) * 16 * P + q0 + 4 * c;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 4 * i + gg;
      *reinterpret_cast<V4*>(dst + static_cast<int64_t>(row) * P) =
          *reinterpret_cast<const V4*>(&buf[w][row][4 * c]);
    }
  }
  if (st.max_slot) reduce_and_publish(mx, bad, st.max_slot, g.flags);
}

template <typename T, int MODE>
hipError_t go_pair(const PairArgs* a, int32_t n, const StagedArrays& st, DevState* state,
                   hipStream_t stream) {
  PairGroup g;
  std::memset(&g, 0, sizeof(g));
  g.n = n;
  g.flags = &state->flags;
  uint32_t total = 0;
  for (int32_t u = 0; u < n; ++u) {
    const PairArgs& x = a[u];
    PairStep& s = g.s[u];
    s.in = x.in;
    s.out = x.out;
    s.S1 = (MODE == M_F64) ? static_cast<const void*>(st.s64 + x.s_off1)
                           : static_cast<const void*>(st.s32 + x.s_off1);
    s.S2 = (MODE == M_F64) ? static_cast<const void*>(st.s64 + x.s_off2)
                           : static_cast<const void*>(st.s32 + x.s_off2);
    s.h1 = st.shi + x.s_off1;
    s.l1 = st.slo + x.s_off1;
    s.h2 = st.shi + x.s_off2;
    s.l2 = st.slo + x.s_off2;
    s.pre = x.pre;
    s.post2 = x.post2;
    s.scale_slot = x.scale_slot;
    s.max_slot = x.max_slot;
    const int64_t blocks = x.pre * (x.post2 / 64);
    g.first[u] = total;
    if (total + blocks > static_cast<int64_t>(INT_MAX)) return hipErrorInvalidValue;
    total += static_cast<uint32_t>(blocks);
  }
  g.first[n] = total;
  hipLaunchKernelGGL((absorb_pair<T, MODE>), dim3(total), dim3(kThreads), 0, stream, g);
  return hipGetLastError();
}

template <typename Tin, typename Tout, int MODE>
hipError_t go_wide(const AbsorbArgs& a, const StagedArrays& st, DevState* state,
                   hipStream_t stream, const Tout* S) {
  const int64_t nsb = (a.pre * a.post + 63) / 64;
  const int64_t grid = (nsb + kWaves * kSuperPerWave - 1) / (kWaves * kSuperPerWave);
  if (grid > INT_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((absorb_wide<Tin, Tout, MODE>), dim3(static_cast<uint32_t>(grid)),
                     dim3(kThreads), 0, stream, static_cast<const Tin*>(a.in),
                     static_cast<Tout*>(a.out), S, st.shi + a.s_off, st.slo + a.s_off, a.pre,
                     static_cast<int32_t>(a.K), static_cast<int32_t>(a.N), a.post, a.scale_slot,
                     a.max_slot, &state->flags);
  return hipGetLastError();
}

template <typename Tin, typename Tout, int MODE>
hipError_t go_narrow(const AbsorbArgs& a, const StagedArrays& st, DevState* state,
                     hipStream_t stream, const Tout* S) {
  const int64_t nblk = (a.pre + 15) / 16;
  const int64_t grid = (nblk + kWaves * kBlocksPerWave - 1) / (kWaves * kBlocksPerWave);
  if (grid > INT_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((absorb_narrow<Tin, Tout, MODE>), dim3(static_cast<uint32_t>(grid)),
                     dim3(kThreads), 0, stream, static_cast<const Tin*>(a.in),
                     static_cast<Tout*>(a.out), S, st.shi + a.s_off, st.slo + a.s_off, a.pre,
                     static_cast<int32_t>(a.K), static_cast<int32_t>(a.N), a.scale_slot,
                     a.max_slot, &state->flags);
  return hipGetLastError();
}

}  // namespace

bool absorb_mfma_supported(const AbsorbArgs& a) {
  return wide_ok(a.pre, a.K, a.N, a.post) || narrow_ok(a.pre, a.K, a.N, a.post);
}

hipError_t launch_absorb_mfma(const AbsorbArgs& a, const StagedArrays& st, DevState* state,
                              hipStream_t stream, const char** kname) {
  const bool wide = wide_ok(a.pre, a.K, a.N, a.post);
  if (a.out_type == EL_F64) {
    const double* S = st.s64 + a.s_off;
    if (a.in_type == EL_F64) {
      *kname = wide ? "absorb_mfma_wide_f64" : "absorb_mfma_narrow_f64";
      return wide ? go_wide<double, double, M_F64>(a, st, state, stream, S)
                  : go_narrow<double, double, M_F64>(a, st, state, stream, S);
    }
    *kname = wide ? "absorb_mfma_wide_f32_to_f64" : "absorb_mfma_narrow_f32_to_f64";
    return wide ? go_wide<float, double, M_F64>(a, st, state, stream, S)
                : go_narrow<float, double, M_F64>(a, st, state, stream, S);
  }
  const float* S = st.s32 + a.s_off;
  if (a.arith == AR_BF16X3) {
    *kname = wide ? "absorb_mfma_wide_bf16x3" : "absorb_mfma_narrow_bf16x3";
    return wide ? go_wide<float, float, M_BF16X3>(a, st, state, stream, S)
                : go_narrow<float, float, M_BF16X3>(a, st, state, stream, S);
  }
  *kname = wide ? "absorb_mfma_wide_f32" : "absorb_mfma_narrow_f32";
  return wide ? go_wide<float, float, M_F32>(a, st, state, stream, S)
              : go_narrow<float, float, M_F32>(a, st, state, stream, S);
}

}  // namespace tn

namespace tn {

bool absorb_group_supported(const AbsorbArgs* a, int32_t n) {
  if (n < 2 || n > 4) return false;
  const bool wide = wide_ok(a[0].pre, a[0].K, a[0].N, a[0].post);
  const bool narrow = !wide && narrow_ok(a[0].pre, a[0].K, a[0].N, a[0].post);
  if (!wide && !narrow) return false;
  for (int32_t u = 0; u < n; ++u) {
    if (a[u].in_type != a[0].in_type || a[u].out_type != a[0].out_type ||
        a[u].arith != a[0].arith)
      return false;
    if (wide != wide_ok(a[u].pre, a[u].K, a[u].N, a[u].post)) return false;
    if (!wide && !narrow_ok(a[u].pre, a[u].K, a[u].N, a[u].post)) return false;
  }
  return true;
}

hipError_t launch_absorb_group(const AbsorbArgs* a, int32_t n, const StagedArrays& st,
                               DevState* state, hipStream_t stream, const char** kname) {
  const bool wide = wide_ok(a[0].pre, a[0].K, a[0].N, a[0].post);
  if (a[0].out_type == EL_F64) {
    if (a[0].in_type == EL_F64) {
      *kname = wide ? "absorb_group_wide_f64" : "absorb_group_narrow_f64";
      return go_group<double, double, M_F64>(a, n, wide, st, state, stream);
    }
    *kname = wide ? "absorb_group_wide_f32_to_f64" : "absorb_group_narrow_f32_to_f64";
    return go_group<float, double, M_F64>(a, n, wide, st, state, stream);
  }
  if (a[0].arith == AR_BF16X3) {
    *kname = wide ? "absorb_group_wide_bf16x3" : "absorb_group_narrow_bf16x3";
    return go_group<float, float, M_BF16X3>(a, n, wide, st, state, stream);
  }
  *kname = wide ? "absorb_group_wide_f32" : "absorb_group_narrow_f32";
  return go_group<float, float, M_F32>(a, n, wide, st, state, stream);
}

}  // namespace tn

namespace tn {

hipError_t launch_absorb_pairs(const PairArgs* a, int32_t n, const StagedArrays& st,
                               DevState* state, hipStream_t stream, const char** kname) {
  if (n < 1 || n > 4) return hipErrorInvalidValue;
  for (int32_t u = 0; u < n; ++u)
    if (a[u].type != a[0].type || a[u].arith != a[0].arith || a[u].post2 % 64 != 0)
      return hipErrorInvalidValue;
  if (a[0].type == EL_F64) {
    *kname = "absorb_pair_f64";
    return go_pair<double, M_F64>(a, n, st, state, stream);
  }
  if (a[0].arith == AR_BF16X3) {
    *kname = "absorb_pair_bf16x3";
    return go_pair<float, M_BF16X3>(a, n, st, state, stream);
  }
  *kname = "absorb_pair_f32";
  return go_pair<float, M_F32>(a, n, st, state, stream);
}

}  // namespace tn
