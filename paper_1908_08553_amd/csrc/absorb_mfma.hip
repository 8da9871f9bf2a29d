// Single-site absorption kernels on the gfx950 matrix cores; the per-wave
// bodies live in absorb_device.hpp (shared with the batched persistent kernel).
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
