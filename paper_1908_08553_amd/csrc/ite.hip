// Imaginary-time evolution of a PEPS on the GPU (paper §5): the one-body
// gates contracted into every site's spin index, and the two-body gates,
// each contracted into a pair of neighbouring sites and split back by a
// singular value decomposition with truncation.
//
// State layout: every site tensor A[s][legs] (spin first, d = 2, then its
// bond legs in canonical order left, up, right, down, each of dimension chi)
// lives at its own offset of one float64 buffer.
//
// Pair update (one workgroup per pair; the pairs of one launch share no
// site).  With b the shared bond, rest_i / rest_j the other bond legs of the
// two sites in canonical order:
//   theta[(s_i, rest_i)][(s_j, rest_j)]
//     = sum_{a,c} G[(s_i s_j)][(a c)] sum_b A_i[a, rest_i, b] A_j[c, b, rest_j]
// is an m x n matrix (m = 2 chi^(r_i - 1), n = 2 chi^(r_j - 1), both <= 64),
// held in LDS and decomposed by one-sided Jacobi (Hestenes): plane rotations
// of column pairs, pairs scheduled round-robin so that every round rotates
// disjoint pairs in parallel (eight lanes per pair), sweeps repeated until
// one applies no rotation.  The columns then hold sigma_k u_k and the
// accumulated rotations v_k.  Singular values at or above eps times the
// largest are kept, at most chi; each kept pair gets the sign that makes the
// first entry of its left vector above 1e-6 of the vector's largest
// positive; the sites become A_i = U sqrt(sigma), A_j = sqrt(sigma) V^T, the
// dropped bond indices zero.  Every sum runs in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kernels.hpp"

namespace tn {
namespace {

constexpr int kIteThreads = 256;
constexpr int kPairLanes = 8;             // lanes per column pair
constexpr int kMaxDim = kIteMaxDim;       // 64
constexpr int kMaxSweeps = 60;

__global__ __launch_bounds__(kIteThreads) void ite_gate1_kernel(double* __restrict__ state,
                                                                const IteSiteDesc* __restrict__ sites,
                                                                double g00, double g01, double g10,
                                                                double g11) {
  const IteSiteDesc s = sites[blockIdx.y];
  double* A = state + s.off;
  for (int64_t x = static_cast<int64_t>(blockIdx.x) * kIteThreads + threadIdx.x; x < s.half;
       x += static_cast<int64_t>(gridDim.x) * kIteThreads) {
    const double a0 = A[x], a1 = A[s.half + x];
    A[x] = g00 * a0 + g01 * a1;
    A[s.half + x] = g10 * a0 + g11 * a1;
  }
}

__global__ __launch_bounds__(kIteThreads) void ite_scale_kernel(double* __restrict__ state,
                                                                int64_t n, double f) {
  for (int64_t x = static_cast<int64_t>(blockIdx.x) * kIteThreads + threadIdx.x; x < n;
       x += static_cast<int64_t>(gridDim.x) * kIteThreads)
    state[x] *= f;
}

// offset of A[s][.. b at bond axis `ax` ..] for flattened rest index `rest`
// of a site with `rank` bond legs of dimension chi (pw[k] = chi^k)
__device__ inline int64_t site_off(int s, int64_t rest, int b, int rank, int ax, const int64_t* pw) {
  const int64_t after = pw[rank - 1 - ax];        // entries of the legs after the shared one
  const int64_t hi = rest / after, lo = rest - hi * after;
  return s * pw[rank] + hi * pw[rank - ax] + b * after + lo;
}

__global__ __launch_bounds__(kIteThreads) void ite_pair_kernel(double* __restrict__ state,
                                                               const ItePairDesc* __restrict__ pairs,
                                                               IteGate2 gate, int32_t chi,
                                                               double eps,
                                                               int32_t* __restrict__ kept) {
  __shared__ double W[kMaxDim * kMaxDim];     // theta (or its transpose), row-major
  __shared__ double V[kMaxDim * kMaxDim];     // accumulated rotations
  __shared__ double Xi[kMaxDim * 4];
  __shared__ double Xj[4 * kMaxDim];
  __shared__ double sig[kMaxDim];
  __shared__ int order[kMaxDim];
  __shared__ int changed;
  __shared__ int nkeep;
  __shared__ int first[4];
  const ItePairDesc p = pairs[blockIdx.x];
  const int tid = threadIdx.x;
  int64_t pw[6];
  pw[0] = 1;
  for (int k = 1; k < 6; ++k) pw[k] = pw[k - 1] * chi;
  const int m = 2 * static_cast<int>(pw[p.ri - 1]);
  const int n = 2 * static_cast<int>(pw[p.rj - 1]);
  const int64_t mi = pw[p.ri - 1], nj = pw[p.rj - 1];   // rest entries of i, j
  double* Ai = state + p.off_i;
  double* Aj = state + p.off_j;
  // load A_i as Xi[(s, rest_i)][b] and A_j as Xj[b][(s, rest_j)]
  for (int e = tid; e < m * chi; e += kIteThreads) {
    const int row = e / chi, b = e - (e / chi) * chi;
    const int s = static_cast<int>(row / mi);
    Xi[e] = Ai[site_off(s, row - s * mi, b, p.ri, p.ai, pw)];
  }
  for (int e = tid; e < chi * n; e += kIteThreads) {
    const int b = e / n, col = e - (e / n) * n;
    const int s = static_cast<int>(col / nj);
    Xj[e] = Aj[site_off(s, col - s * nj, b, p.rj, p.aj, pw)];
  }
  __syncthreads();
  // theta; when m < n the transpose is decomposed (rows >= columns)
  const bool tr = m < n;
  const int R = tr ? n : m, Cc = tr ? m : n;
  for (int e = tid; e < m * n; e += kIteThreads) {
    const int row = e / n, col = e - (e / n) * n;
    const int si = static_cast<int>(row / mi), sj = static_cast<int>(col / nj);
    const int64_t ri = row - si * mi, rj = col - sj * nj;
    double t = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 2; ++c) {
        const double g = gate.g[(si * 2 + sj) * 4 + a * 2 + c];
        if (g == 0.0) continue;
        double pbc = 0.0;
        for (int b = 0; b < chi; ++b)
          pbc += Xi[(a * mi + ri) * chi + b] * Xj[b * n + c * nj + rj];
        t += g * pbc;
      }
    if (tr) W[col * Cc + row] = t;
    else W[row * Cc + col] = t;
  }
  for (int e = tid; e < Cc * Cc; e += kIteThreads) V[e] = (e / Cc == e % Cc) ? 1.0 : 0.0;
  __syncthreads();
  // one-sided Jacobi: round-robin pairs (circle method over Cc columns)
  const int grp = tid / kPairLanes, lane = tid % kPairLanes;
  const int npairs = Cc / 2;
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (tid == 0) changed = 0;
    __syncthreads();
    for (int round = 0; round < Cc - 1; ++round) {
      if (grp < npairs) {
        int a, b;
        if (grp == 0) {
          a = Cc - 1;
          b = round;
        } else {
          a = (round + grp) % (Cc - 1);
          b = (round - grp + Cc - 1) % (Cc - 1);
        }
        const int pcol = a < b ? a : b, qcol = a < b ? b : a;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = lane; i < R; i += kPairLanes) {
          const double wp = W[i * Cc + pcol], wq = W[i * Cc + qcol];
          al += wp * wp;
          be += wq * wq;
          ga += wp * wq;
        }
        for (int off = 1; off < kPairLanes; off <<= 1) {
          al += __shfl_xor(al, off);
          be += __shfl_xor(be, off);
          ga += __shfl_xor(ga, off);
        }
        if (ga != 0.0 && fabs(ga) > 1e-15 * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
          for (int i = lane; i < R; i += kPairLanes) {
            const double wp = W[i * Cc + pcol], wq = W[i * Cc + qcol];
            W[i * Cc + pcol] = c * wp - s * wq;
            W[i * Cc + qcol] = s * wp + c * wq;
          }
          for (int i = lane; i < Cc; i += kPairLanes) {
            const double vp = V[i * Cc + pcol], vq = V[i * Cc + qcol];
            V[i * Cc + pcol] = c * vp - s * vq;
            V[i * Cc + qcol] = s * vp + c * vq;
          }
          if (lane == 0) changed = 1;
        }
      }
      __syncthreads();
    }
    const int again = changed;
    __syncthreads();
    if (!again) break;
  }
  // singular values (column norms), in a fixed order per column
  for (int j = tid; j < Cc; j += kIteThreads) {
    double s2 = 0.0;
    for (int i = 0; i < R; ++i) s2 += W[i * Cc + j] * W[i * Cc + j];
    sig[j] = sqrt(s2);
  }
  __syncthreads();
  if (tid == 0) {
    // descending, stable (equal values keep column order)
    for (int j = 0; j < Cc; ++j) order[j] = j;
    for (int j = 1; j < Cc; ++j) {
      const int x = order[j];
      int k = j - 1;
      while (k >= 0 && sig[order[k]] < sig[x]) {
        order[k + 1] = order[k];
        --k;
      }
      order[k + 1] = x;
    }
    int keep = 0;
    const double top = sig[order[0]];
    while (keep < chi && keep < Cc && sig[order[keep]] > 0.0 && sig[order[keep]] >= eps * top)
      ++keep;
    nkeep = keep;
    // sign rule on the left vector of theta: column of W (m rows) when not
    // transposed, column of V (m rows) when transposed
    for (int k = 0; k < keep; ++k) {
      const int j = order[k];
      double big = 0.0;
      for (int i = 0; i < m; ++i) big = fmax(big, fabs(tr ? V[i * Cc + j] : W[i * Cc + j]));
      int f = 1;
      for (int i = 0; i < m; ++i) {
        const double x = tr ? V[i * Cc + j] : W[i * Cc + j];
        if (fabs(x) > 1e-6 * big) {
          f = x < 0.0 ? -1 : 1;
          break;
        }
      }
      first[k] = f;
    }
  }
  __syncthreads();
  const int keep = nkeep;
  // A_i[(s, rest_i), b] = u_b[row] sqrt(sigma_b) for b < keep, else 0
  for (int e = tid; e < m * chi; e += kIteThreads) {
    const int row = e / chi, b = e - (e / chi) * chi;
    double x = 0.0;
    if (b < keep) {
      const int j = order[b];
      const double sq = sqrt(sig[j]);
      // left vector entry: W[row][j] / sigma_j, or V[row][j] when transposed
      x = first[b] * (tr ? V[row * Cc + j] * sq : W[row * Cc + j] / sig[j] * sq);
    }
    const int s = static_cast<int>(row / mi);
    Ai[site_off(s, row - s * mi, b, p.ri, p.ai, pw)] = x;
  }
  // A_j[(s, b, rest_j)] = sqrt(sigma_b) v_b[col]
  for (int e = tid; e < chi * n; e += kIteThreads) {
    const int b = e / n, col = e - (e / n) * n;
    double x = 0.0;
    if (b < keep) {
      const int j = order[b];
      const double sq = sqrt(sig[j]);
      x = first[b] * (tr ? W[col * Cc + j] / sig[j] * sq : V[col * Cc + j] * sq);
    }
    const int s = static_cast<int>(col / nj);
    Aj[site_off(s, col - s * nj, b, p.rj, p.aj, pw)] = x;
  }
  if (tid == 0 && kept) kept[blockIdx.x] = keep;
}

}  // namespace

hipError_t launch_ite_gate1(double* state, const IteSiteDesc* sites, int32_t n_sites,
                            int64_t max_half, const double g[4], hipStream_t stream) {
  if (n_sites < 1 || n_sites > 65535 || max_half < 1) return hipErrorInvalidValue;
  const int64_t bx = std::min<int64_t>((max_half + kIteThreads - 1) / kIteThreads, 1024);
  hipLaunchKernelGGL(ite_gate1_kernel, dim3(static_cast<uint32_t>(bx), n_sites),
                     dim3(kIteThreads), 0, stream, state, sites, g[0], g[1], g[2], g[3]);
  return hipGetLastError();
}

hipError_t launch_ite_scale(double* state, int64_t n, double f, hipStream_t stream) {
  if (n < 1) return hipSuccess;
  const int64_t bx = std::min<int64_t>((n + kIteThreads - 1) / kIteThreads, 4096);
  hipLaunchKernelGGL(ite_scale_kernel, dim3(static_cast<uint32_t>(bx)), dim3(kIteThreads), 0,
                     stream, state, n, f);
  return hipGetLastError();
}

hipError_t launch_ite_pairs(double* state, const ItePairDesc* pairs, int32_t n_pairs,
                            const IteGate2& gate, int32_t chi, double eps, int32_t* kept,
                            hipStream_t stream) {
  if (n_pairs < 1) return hipSuccess;
  if (chi < 1 || chi > kIteMaxChi) return hipErrorInvalidValue;
  hipLaunchKernelGGL(ite_pair_kernel, dim3(static_cast<uint32_t>(n_pairs)), dim3(kIteThreads), 0,
                     stream, state, pairs, gate, chi, eps, kept);
  return hipGetLastError();
}

}  // namespace tn
