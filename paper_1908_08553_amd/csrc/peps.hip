// Norm and expectation-value networks of a real PEPS (paper §3: the norm
// sums A* A over all spin configurations and each local observable is
// <Psi|O|Psi> / <Psi|Psi>; §5: every such value is one full contraction of
// O|Psi> against <Psi| along all spin indices).
//
// Contracting a site's spin index between ket, operator and bra leaves a
// single-layer site with paired bonds (dimension chi^2, index a * chi + a'):
//     E[(a_1 a_1') .. (a_r a_r')] = sum_{s'} (sum_s O[s'][s] A[s][a]) A[s'][a']
// One launch builds up to kDlPerLaunch such sites (descriptors by value in
// the kernel arguments); workgroup (x, y) covers output entries of site y.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>

#include "kernels.hpp"

namespace tn {
namespace {

constexpr int kDlPerLaunch = 48;
constexpr int kDlThreads = 256;

struct DlArgs {
  DoubleLayerSite s[kDlPerLaunch];
  int32_t n;
};

__global__ __launch_bounds__(kDlThreads) void double_layer_kernel(DlArgs args) {
  const DoubleLayerSite& x = args.s[blockIdx.y];
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kDlThreads + threadIdx.x;
  if (e >= x.n_out) return;
  // C-order strides of A's bond legs
  int64_t astr[4];
  int64_t st = 1;
  for (int k = x.rank - 1; k >= 0; --k) {
    astr[k] = st;
    st *= x.dims[k];
  }
  // E's leg k is A's leg perm[k]; its paired index p_k = a * dim + a' (E's
  // legs C-order, last fastest)
  int64_t rest = e, ket = 0, bra = 0;
  for (int k = x.rank - 1; k >= 0; --k) {
    const int a = x.perm[k];
    const int64_t dk = x.dims[a];
    const int64_t p = rest % (dk * dk);
    rest /= dk * dk;
    ket += (p / dk) * astr[a];
    bra += (p % dk) * astr[a];
  }
  double acc = 0.0;
  for (int sp = 0; sp < x.d; ++sp) {
    double oa = 0.0;   // (O A)[s'][ket]
    if (x.op) {
      for (int s = 0; s < x.d; ++s) oa += x.op[sp * x.d + s] * x.A[s * x.n_in + ket];
    } else {
      oa = x.A[sp * x.n_in + ket];
    }
    acc += oa * x.A[sp * x.n_in + bra];
  }
  x.E[e] = acc;
}

}  // namespace

bool double_layer_ok(const DoubleLayerSite& s) {
  if (!s.A || !s.E || s.d < 1 || s.d > 64 || s.rank < 0 || s.rank > 4) return false;
  int32_t seen = 0;
  for (int k = 0; k < s.rank; ++k) {
    if (s.perm[k] < 0 || s.perm[k] >= s.rank || (seen >> s.perm[k]) & 1) return false;
    seen |= 1 << s.perm[k];
  }
  int64_t n = 1;
  for (int k = 0; k < s.rank; ++k) {
    if (s.dims[k] < 1 || s.dims[k] > 46340) return false;
    n *= static_cast<int64_t>(s.dims[k]);
    if (n > (int64_t{1} << 30)) return false;
  }
  if (n != s.n_in || n * n != s.n_out) return false;
  return (s.n_out + kDlThreads - 1) / kDlThreads <= INT_MAX;
}

hipError_t launch_double_layer(const DoubleLayerSite* sites, int32_t n, hipStream_t stream) {
  for (int32_t i = 0; i < n; ++i)
    if (!double_layer_ok(sites[i])) return hipErrorInvalidValue;
  for (int32_t i0 = 0; i0 < n; i0 += kDlPerLaunch) {
    DlArgs a;
    a.n = n - i0 < kDlPerLaunch ? n - i0 : kDlPerLaunch;
    int64_t blocks = 1;
    for (int32_t j = 0; j < a.n; ++j) {
      a.s[j] = sites[i0 + j];
      blocks = std::max<int64_t>(blocks, (a.s[j].n_out + kDlThreads - 1) / kDlThreads);
    }
    hipLaunchKernelGGL(double_layer_kernel, dim3(static_cast<uint32_t>(blocks), a.n),
                       dim3(kDlThreads), 0, stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace tn
