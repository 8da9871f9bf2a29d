// The two largest steps at either edge of a column sweep, fused into one pass.
//
// A sweep's first column grows the boundary from nothing: every row's site
// adds its right leg to the prefix and the suffix stays 1, so the last two
// rows (the largest steps of the column) are
//   s1: in[p][k]  (K = 4)      -> t[p][h][v] = sum_k in[p][k] S1[k][4h + v]
//   s2: t[(4p+h)][v] (K = 4)   -> out[(4p+h)][n] = sum_v t[..][v] S2[v][n]
// (N2 = 4: the bottom row has no down leg).  The last column closes the boundary:
// the prefix is 1 and every row absorbs the leading suffix leg, so its first
// two rows are
//   s1: in[k][h][q] (K = 4, N = 4) -> t[n1][h][q] = sum_k in[k][h][q] S1[k][n1]
//   s2: t[(n1, h)][q] (K = 16)     -> out[n2][q] = sum_{n1,h} t[n1][h][q] S2[4 n1 + h][n2]
// (paper §4: the sequential pairwise contraction; these are the two ends of
// each column pass, D = 4).  The intermediate t stays in registers, so the
// pair reads s1's input and writes s2's output once: in FP64 at 12x12 each
// pair moves 168 MB instead of 436 MB (first column: 106 -> 30 us, last
// column: 93 -> 29 us).
//
// The work is a handful of FMAs per 8-byte element, far below the FP64 vector
// rate: plain VALU code, coalesced 16-byte loads and stores, site matrices
// read through the scalar cache where the index is uniform.  Arithmetic in
// double when the pair's output is FP64 (float inputs are widened first),
// else in float; the input of s1 is scaled by 2^-shift, the |max| of s2's
// output feeds the rescale slot as in the single-step kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>

#include "absorb_device.hpp"
#include "kernels.hpp"

namespace tn {
namespace {

using namespace dev;

constexpr int kEdgeThreads = 256;   // four waves (reduce_and_publish's width)
// First-column items per thread (measured on the 12x12 FP64 / FP32 sweeps:
// 30 and 25 us; 4 FP32 items per thread took 53 us, one item per thread 62
// and 44 us; renumbering the blocks per XCD changed nothing).
template <typename Tc>
constexpr int head_iter() { return sizeof(Tc) == 8 ? 8 : 16; }

struct EdgeStep {
  const void* in;
  void* out;
  const void* S1;   // staged K x N site matrices in the compute type
  const void* S2;
  int64_t items;    // work items of this step pair
  int64_t q2;       // last column: suffix of s2
  const int32_t* scale_slot;
  int32_t* max_slot;
};

struct EdgeGroup {
  EdgeStep s[4];
  uint32_t first[5];
  int32_t n;
  int32_t* flags;
};

template <typename T, int W>
struct Vec {
  T v[W];
};

template <typename T, int W>
__device__ inline Vec<T, W> load_vec(const T* p) {
  Vec<T, W> r;
  if constexpr (sizeof(T) * W == 16) {
    const uint4 u = *reinterpret_cast<const uint4*>(p);
    __builtin_memcpy(&r, &u, 16);
  } else if constexpr (sizeof(T) * W == 32) {
    const uint4 u0 = *reinterpret_cast<const uint4*>(p);
    const uint4 u1 = *reinterpret_cast<const uint4*>(p + W / 2);
    __builtin_memcpy(&r, &u0, 16);
    __builtin_memcpy(reinterpret_cast<char*>(&r) + 16, &u1, 16);
  } else {
#pragma unroll
    for (int e = 0; e < W; ++e) r.v[e] = p[e];
  }
  return r;
}

template <typename T, int W>
__device__ inline void store_vec(T* p, const T (&x)[W]) {
  static_assert((sizeof(T) * W) % 16 == 0, "16-byte stores");
#pragma unroll
  for (int b = 0; b < static_cast<int>(sizeof(T) * W / 16); ++b) {
    uint4 u;
    __builtin_memcpy(&u, reinterpret_cast<const char*>(x) + 16 * b, 16);
    *reinterpret_cast<uint4*>(reinterpret_cast<char*>(p) + 16 * b) = u;
  }
}

// HEAD: first-column pair (rows 4p + h of s2's output, N2 entries each).
// Tail: last-column pair, item i covers QV consecutive q.
template <typename Tin, typename Tc, bool HEAD, int N2>
__global__ __launch_bounds__(kEdgeThreads) void absorb_edge(EdgeGroup g) {
  int u = 0;
  while (u + 1 < g.n && blockIdx.x >= g.first[u + 1]) ++u;
  const EdgeStep& st = g.s[u];
  const Tc* __restrict__ S1 = static_cast<const Tc*>(st.S1);
  const Tc* __restrict__ S2 = static_cast<const Tc*>(st.S2);
  const int64_t i = static_cast<int64_t>(blockIdx.x - g.first[u]) * kEdgeThreads + threadIdx.x;
  const int shift = shift_of(st.scale_slot);
  Tc mx = 0;
  int bad = 0;
  if (HEAD || i < st.items) {
    if constexpr (HEAD) {
      // Item j covers 16 bytes (HV outputs) of s2's output, consecutive items
      // consecutive pieces; a thread takes head_iter<Tc>() items kEdgeThreads apart,
      // which all have the same row position h = row % 4 and piece, so its 16
      // entries of S1 and 4 HV of S2 are loaded once.
      constexpr int HV = 16 / sizeof(Tc), PARTS = N2 / HV;
      const int64_t j0 = static_cast<int64_t>(blockIdx.x - g.first[u]) * kEdgeThreads *
                             head_iter<Tc>() + threadIdx.x;
      const int part = static_cast<int>(j0 % PARTS);
      const int h = static_cast<int>((j0 / PARTS) & 3);
      Tc s1[4][4], s2[4][HV];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int v = 0; v < 4; ++v) s1[k][v] = S1[k * 16 + 4 * h + v];
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int e = 0; e < HV; ++e) s2[v][e] = S2[v * N2 + part * HV + e];
      const Tin* in = static_cast<const Tin*>(st.in);
      Tc* out = static_cast<Tc*>(st.out);
      Vec<Tin, 4> x[head_iter<Tc>()];
#pragma unroll
      for (int it = 0; it < head_iter<Tc>(); ++it) {
        const int64_t j = j0 + it * kEdgeThreads;
        if (j < st.items) x[it] = load_vec<Tin, 4>(in + 4 * (j / (4 * PARTS)));
      }
#pragma unroll
      for (int it = 0; it < head_iter<Tc>(); ++it) {
        const int64_t j = j0 + it * kEdgeThreads;
        if (j >= st.items) break;
        Tc xs[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) xs[k] = ldexp(static_cast<Tc>(x[it].v[k]), -shift);
        Tc t[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          Tc a = 0;
#pragma unroll
          for (int k = 0; k < 4; ++k) a = fma(xs[k], s1[k][v], a);
          t[v] = a;
        }
        Tc o[HV];
#pragma unroll
        for (int e = 0; e < HV; ++e) {
          Tc a = 0;
#pragma unroll
          for (int v = 0; v < 4; ++v) a = fma(t[v], s2[v][e], a);
          o[e] = a;
          track(a, mx, bad);
        }
        store_vec<Tc, HV>(out + j * HV, o);
      }
    } else {
      constexpr int QV = 16 / sizeof(Tin);
      const int64_t Q2 = st.q2, q = i * QV;
      const Tin* in = static_cast<const Tin*>(st.in) + q;
      Vec<Tin, QV> x[4][4];   // [k][h]
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int h = 0; h < 4; ++h) x[k][h] = load_vec<Tin, QV>(in + (4 * k + h) * Q2);
      Tc o[N2][QV];
#pragma unroll
      for (int n = 0; n < N2; ++n)
#pragma unroll
        for (int e = 0; e < QV; ++e) o[n][e] = 0;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        Tc xs[4][QV];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int e = 0; e < QV; ++e) xs[k][e] = ldexp(static_cast<Tc>(x[k][h].v[e]), -shift);
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) {
          Tc t[QV];
#pragma unroll
          for (int e = 0; e < QV; ++e) {
            Tc a = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) a = fma(xs[k][e], S1[k * 4 + n1], a);
            t[e] = a;
          }
#pragma unroll
          for (int n = 0; n < N2; ++n) {
            const Tc s = S2[(4 * n1 + h) * N2 + n];
#pragma unroll
            for (int e = 0; e < QV; ++e) o[n][e] = fma(t[e], s, o[n][e]);
          }
        }
      }
      Tc* out = static_cast<Tc*>(st.out) + q;
#pragma unroll
      for (int n = 0; n < N2; ++n) {
#pragma unroll
        for (int e = 0; e < QV; ++e) track(o[n][e], mx, bad);
        store_vec<Tc, QV>(out + n * Q2, o[n]);
      }
    }
  }
  if (st.max_slot) reduce_and_publish(mx, bad, st.max_slot, g.flags);
}

template <typename Tin, typename Tc, bool HEAD, int N2>
hipError_t go_edge(const EdgeArgs* a, int32_t n, const StagedArrays& sa, DevState* state,
                   hipStream_t stream) {
  constexpr bool F64 = sizeof(Tc) == 8;
  EdgeGroup g;
  std::memset(&g, 0, sizeof(g));
  g.n = n;
  g.flags = &state->flags;
  uint32_t total = 0;
  for (int32_t u = 0; u < n; ++u) {
    const EdgeArgs& x = a[u];
    EdgeStep& s = g.s[u];
    s.in = x.in;
    s.out = x.out;
    s.S1 = F64 ? static_cast<const void*>(sa.s64 + x.s_off1)
               : static_cast<const void*>(sa.s32 + x.s_off1);
    s.S2 = F64 ? static_cast<const void*>(sa.s64 + x.s_off2)
               : static_cast<const void*>(sa.s32 + x.s_off2);
    constexpr int QV = 16 / sizeof(Tin);
    s.items = HEAD ? 4 * x.pre1 * (N2 * sizeof(Tc) / 16) : x.post2 / QV;
    s.q2 = x.post2;
    s.scale_slot = x.scale_slot;
    s.max_slot = x.max_slot;
    const int64_t per_block = HEAD ? kEdgeThreads * head_iter<Tc>() : kEdgeThreads;
    const int64_t blocks = std::max<int64_t>(1, (s.items + per_block - 1) / per_block);
    if (total + blocks > static_cast<int64_t>(INT_MAX)) return hipErrorInvalidValue;
    g.first[u] = total;
    total += static_cast<uint32_t>(blocks);
  }
  g.first[n] = total;
  hipLaunchKernelGGL((absorb_edge<Tin, Tc, HEAD, N2>), dim3(total), dim3(kEdgeThreads), 0, stream,
                     g);
  return hipGetLastError();
}

template <bool HEAD, int N2>
hipError_t go_edge_types(const EdgeArgs* a, int32_t n, const StagedArrays& sa, DevState* state,
                         hipStream_t stream, const char** kname) {
  const EdgeArgs& x = a[0];
  if (x.out_type == EL_F64) {
    *kname = "absorb_edge_f64";
    if (x.in_type == EL_F64) return go_edge<double, double, HEAD, N2>(a, n, sa, state, stream);
    return go_edge<float, double, HEAD, N2>(a, n, sa, state, stream);
  }
  *kname = "absorb_edge_f32";
  return go_edge<float, float, HEAD, N2>(a, n, sa, state, stream);
}

}  // namespace

bool edge_pair_supported(const EdgeArgs& a) {
  if (a.in_type == EL_F64 && a.out_type != EL_F64) return false;
  if (a.out_type != EL_F64 && a.arith == AR_BF16X3) return false;   // float VALU is not BF16x3
  if (a.head) return a.n2 == 4 && a.pre1 >= 1 && a.pre1 <= INT64_MAX / 64;
  return a.n2 == 4 && a.post2 >= 4 && a.post2 % 4 == 0 && a.post2 <= INT64_MAX / 16;
}

hipError_t launch_absorb_edges(const EdgeArgs* a, int32_t n, const StagedArrays& sa,
                               DevState* state, hipStream_t stream, const char** kname) {
  if (n < 1 || n > 4) return hipErrorInvalidValue;
  for (int32_t u = 0; u < n; ++u)
    if (!edge_pair_supported(a[u]) || a[u].head != a[0].head || a[u].n2 != a[0].n2 ||
        a[u].in_type != a[0].in_type || a[u].out_type != a[0].out_type)
      return hipErrorInvalidValue;
  if (a[0].head) return go_edge_types<true, 4>(a, n, sa, state, stream, kname);
  return go_edge_types<false, 4>(a, n, sa, state, stream, kname);
}

}  // namespace tn
