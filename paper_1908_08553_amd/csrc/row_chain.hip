// The row scheme's chain (paper §4, Fig. 2a): after every row of the lattice
// has been contracted into one tensor, the chain of row tensors is contracted
// from the first row down.  Each link is a matrix-vector product between the
// chain vector v (the rows above, summed) and the next row tensor R over that
// row's up legs, in float64:
//   side 0: out[n] = sum_k (v[k] 2^-ev) (R[k][n] 2^-er)    (R as [K][N])
//   side 1: out[n] = sum_k (R[n][k] 2^-er) (v[k] 2^-ev)    (R as [N][K])
// with ev, er the exponents of the rescale slots that measured v and R.  The
// product reads K*N entries of R once, 2 flops each: HBM-bound.
//
// Two launches per link, both deterministic: the first splits k into fixed
// chunks and writes one partial sum per (chunk, n) -- side 0 with threads
// along n (coalesced over R's rows), side 1 with a block per n and threads
// along k (coalesced over R's row n) -- and the second adds the chunks of
// each n in order, writes out[n] and publishes the exponent of max |out| to
// the link's rescale slot (none on the last link, whose output is the
// scalar).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "absorb_device.hpp"
#include "kernels.hpp"

namespace tn {
namespace {

constexpr int kLinkBlock = 256;

template <typename TV, typename TR>
__global__ __launch_bounds__(kLinkBlock) void link_side0(const TV* __restrict__ v,
                                                         const TR* __restrict__ R, int64_t K,
                                                         int64_t N, int64_t chunk,
                                                         const int32_t* slot_v,
                                                         const int32_t* slot_r,
                                                         double* __restrict__ partials) {
  const int64_t n = static_cast<int64_t>(blockIdx.x) * kLinkBlock + threadIdx.x;
  if (n >= N) return;
  const double sv = ldexp(1.0, -dev::shift_of(slot_v));
  const double sr = ldexp(1.0, -dev::shift_of(slot_r));
  const int64_t k0 = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t k1 = k0 + chunk < K ? k0 + chunk : K;
  double s = 0.0;
  for (int64_t k = k0; k < k1; ++k)
    s += (static_cast<double>(v[k]) * sv) * (static_cast<double>(R[k * N + n]) * sr);
  partials[static_cast<int64_t>(blockIdx.y) * N + n] = s;
}

template <typename TV, typename TR>
__global__ __launch_bounds__(kLinkBlock) void link_side1(const TV* __restrict__ v,
                                                         const TR* __restrict__ R, int64_t K,
                                                         int64_t N, int64_t chunk,
                                                         const int32_t* slot_v,
                                                         const int32_t* slot_r,
                                                         double* __restrict__ partials) {
  __shared__ double red[kLinkBlock];
  const int64_t n = blockIdx.x;
  const double sv = ldexp(1.0, -dev::shift_of(slot_v));
  const double sr = ldexp(1.0, -dev::shift_of(slot_r));
  const int64_t k0 = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t k1 = k0 + chunk < K ? k0 + chunk : K;
  const TR* row = R + n * K;
  double s = 0.0;
  for (int64_t k = k0 + threadIdx.x; k < k1; k += kLinkBlock)
    s += (static_cast<double>(row[k]) * sr) * (static_cast<double>(v[k]) * sv);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = kLinkBlock / 2; st > 0; st >>= 1) {
    if (static_cast<int>(threadIdx.x) < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[static_cast<int64_t>(blockIdx.y) * N + n] = red[0];
}

__global__ __launch_bounds__(kLinkBlock) void link_reduce(const double* __restrict__ partials,
                                                          int64_t chunks, int64_t N,
                                                          double* __restrict__ out,
                                                          int32_t* max_slot, int32_t* flags) {
  const int64_t n = static_cast<int64_t>(blockIdx.x) * kLinkBlock + threadIdx.x;
  double mx = 0.0;
  int bad = 0;
  if (n < N) {
    double s = 0.0;
    for (int64_t c = 0; c < chunks; ++c) s += partials[c * N + n];
    out[n] = s;
    dev::track(s, mx, bad);
  }
  if (max_slot) {
    dev::reduce_and_publish<double, kLinkBlock / 64>(mx, bad, max_slot, flags);
  } else if (bad) {
    atomicOr(flags, 1);
  }
}

template <typename TV, typename TR>
void launch_link(const LinkArgs& a, int64_t chunks, int64_t chunk, hipStream_t stream) {
  const TV* v = static_cast<const TV*>(a.v);
  const TR* R = static_cast<const TR*>(a.R);
  if (a.side == 0) {
    dim3 g(static_cast<uint32_t>((a.N + kLinkBlock - 1) / kLinkBlock),
           static_cast<uint32_t>(chunks));
    hipLaunchKernelGGL((link_side0<TV, TR>), g, dim3(kLinkBlock), 0, stream, v, R, a.K, a.N,
                       chunk, a.slot_v, a.slot_R, a.partials);
  } else {
    dim3 g(static_cast<uint32_t>(a.N), static_cast<uint32_t>(chunks));
    hipLaunchKernelGGL((link_side1<TV, TR>), g, dim3(kLinkBlock), 0, stream, v, R, a.K, a.N,
                       chunk, a.slot_v, a.slot_R, a.partials);
  }
}

}  // namespace

int64_t link_chunks(int32_t side, int64_t K, int64_t N) {
  // enough blocks to cover the chip (about 1024), each summing at least 64
  // (side 0) or 256 (side 1) terms
  const int64_t lanes = side == 0 ? (N + kLinkBlock - 1) / kLinkBlock : N;
  const int64_t want = std::max<int64_t>(1, (1024 + lanes - 1) / lanes);
  const int64_t most = std::max<int64_t>(1, (K + (side == 0 ? 63 : 255)) / (side == 0 ? 64 : 256));
  return std::min(want, most);
}

hipError_t launch_row_link(const LinkArgs& a, hipStream_t stream) {
  if (a.K < 1 || a.N < 1 || a.N > INT32_MAX || (a.side != 0 && a.side != 1) || !a.v || !a.R ||
      !a.out || !a.partials || !a.flags)
    return hipErrorInvalidValue;
  const int64_t chunks = link_chunks(a.side, a.K, a.N);
  const int64_t chunk = (a.K + chunks - 1) / chunks;
  if (a.v_f64 && a.R_f64) launch_link<double, double>(a, chunks, chunk, stream);
  else if (a.v_f64) launch_link<double, float>(a, chunks, chunk, stream);
  else if (a.R_f64) launch_link<float, double>(a, chunks, chunk, stream);
  else launch_link<float, float>(a, chunks, chunk, stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(link_reduce, dim3(static_cast<uint32_t>((a.N + kLinkBlock - 1) / kLinkBlock)),
                     dim3(kLinkBlock), 0, stream, a.partials, chunks, a.N, a.out, a.max_slot,
                     a.flags);
  return hipGetLastError();
}

}  // namespace tn
