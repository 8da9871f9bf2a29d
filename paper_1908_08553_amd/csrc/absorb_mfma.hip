// Single-site absorption kernels on the gfx950 matrix cores; the per-wave
// bodies live in absorb_device.hpp (shared with the batched persistent kernel).
#include <hip/hip_runtime.h>

#include <climits>

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
