// Generic HIP kernels for gfx950: site staging, single-site absorption on the
// vector ALUs (any K, N, pre, post), the quadrant-ring product with a fused
// float64 dot, and the final assembly of sign / exponent / log|Z|.
//
// Each absorption step computes out[pre][N][post] = sum_k in[pre][k][post] *
// S[k][N]: the paper's pairwise contraction of the boundary with one site,
// done by folding both into matrices (paper §6: tensors folded into matrices
// and multiplied).  The boundary's leg order is chosen by the planner so the
// shared legs are always adjacent and the contiguous axis ("post") is never
// permuted, so reads and writes stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <cmath>

#include "absorb_device.hpp"
#include "kernels.hpp"

namespace tn {
namespace {

constexpr int kBlock = 256;

__device__ inline int32_t exp_of(double m) {
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

// bf16 round-to-nearest-even of a finite float, as its 16 high bits
__device__ inline uint16_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ inline float bf16_float(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

template <typename T>
__device__ inline T wave_max(T v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}
__device__ inline int wave_or(int v) {
  for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off);
  return v;
}

// block-wide max of |x| and "any non-finite"; result valid in thread 0
template <typename T>
__device__ inline void block_max_bad(T& m, int& bad) {
  __shared__ double sm[kBlock / 64];
  __shared__ int sb[kBlock / 64];
  m = wave_max(m);
  bad = wave_or(bad);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) { sm[w] = static_cast<double>(m); sb[w] = bad; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = sm[0];
    int bb = sb[0];
    for (int k = 1; k < static_cast<int>(blockDim.x >> 6); ++k) { mm = fmax(mm, sm[k]); bb |= sb[k]; }
    m = static_cast<T>(mm);
    bad = bb;
  }
}

// ---------------------------------------------------------------- staging
// SPB site tensors per workgroup, kBlock / SPB threads each: one workgroup
// per site for a single lattice (144 sites at 12 x 12 keep every CU busy),
// one wavefront per site for batches (tens of thousands of sites of at most a
// few hundred entries: one workgroup each left the GPU dispatching rather
// than copying).
constexpr int kStagePer = 4;          // entries per thread per round
constexpr int kStageWaveSites = 1024; // from this many sites on, one wavefront per site

template <int SPB>
__global__ __launch_bounds__(kBlock) void stage_kernel(const StageDesc* __restrict__ descs,
                                                       int32_t n_sites, StagedArrays st,
                                                       StageTargets tg) {
  constexpr int TPS = kBlock / SPB;
  static_assert(TPS == 64 || SPB == 1, "a site takes one wavefront or the workgroup");
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < tg.n_slots; i += blockDim.x) tg.slot_exp[i] = kExpZero;
    if (threadIdx.x == 0) {
      if (tg.flags) *tg.flags = 0;
      if (tg.counter) *tg.counter = 0;
    }
    if (tg.seed_rec) {
      __syncthreads();   // the slot initialisation above is complete
      if (threadIdx.x == 0) {
        tg.slot_exp[tg.seed_slot] = tg.seed_rec->e;
        *tg.e_bias = tg.seed_rec->bias;
      }
    }
  }
  const int t = threadIdx.x % TPS;
  const int32_t site = blockIdx.x * SPB + threadIdx.x / TPS;
  if (SPB > 1 && site >= n_sites) return;   // whole wavefronts
  const StageDesc& d = descs[site];   // read in place: its arrays are indexed by axis
  // kStagePer entries per thread per round, their loads issued together
  double m = 0.0;
  int bad = 0;
  for (int64_t q0 = 0; q0 < d.entries; q0 += TPS * kStagePer) {
    double x[kStagePer];
#pragma unroll
    for (int j = 0; j < kStagePer; ++j) {
      const int64_t q = q0 + TPS * j + t;
      x[j] = q < d.entries ? d.src[q] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kStagePer; ++j) {
      bad |= !isfinite(x[j]);
      m = fmax(m, fabs(x[j]));
    }
  }
  __shared__ int32_t sh_e;
  int32_t e;
  if constexpr (SPB == 1) {
    block_max_bad(m, bad);   // valid in thread 0
    if (threadIdx.x == 0) {
      const int32_t e0 = bad ? 0 : exp_of(m);
      sh_e = (e0 == kExpZero) ? 0 : e0;
      tg.site_exp[site] = sh_e;
      tg.site_bad[site] = bad;
    }
    __syncthreads();
    e = sh_e;
  } else {
    m = wave_max(m);
    bad = wave_or(bad);
    const int32_t e0 = bad ? 0 : exp_of(m);
    e = (e0 == kExpZero) ? 0 : e0;
    if (t == 0) {
      tg.site_exp[site] = e;
      tg.site_bad[site] = bad;
    }
  }
  for (int64_t q0 = 0; q0 < d.entries; q0 += TPS * kStagePer) {
    double x[kStagePer];
#pragma unroll
    for (int j = 0; j < kStagePer; ++j) {
      const int64_t q = q0 + TPS * j + t;
      int64_t rem = q, off = 0;
      for (int a = d.ndim - 1; a >= 0; --a) {
        const int64_t i = rem % d.dims[a];
        rem /= d.dims[a];
        off += i * d.cstride[a];
      }
      x[j] = q < d.entries ? d.src[off] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kStagePer; ++j) {
      const int64_t q = q0 + TPS * j + t;
      if (q >= d.entries) break;
      const double v = ldexp(x[j], -e);
      const float f = static_cast<float>(v);
      const uint16_t hi = bf16_bits(f);
      const uint16_t lo = bf16_bits(f - bf16_float(hi));
      st.s64[d.s_off + q] = v;
      st.s32[d.s_off + q] = f;
      st.shi[d.s_off + q] = hi;
      st.slo[d.s_off + q] = lo;
      if (d.init_dst) {
        if (d.init_double) static_cast<double*>(d.init_dst)[q] = v;
        else static_cast<float*>(d.init_dst)[q] = f;
      }
    }
  }
}

// -------------------------------------------------------------- absorption
// One thread per (pre, post) fiber; N processed in chunks of 16 accumulators.
template <typename Tin, typename Tc, bool SPLIT>
__global__ __launch_bounds__(kBlock) void absorb_generic(
    const Tin* __restrict__ in, Tc* __restrict__ out, const Tc* __restrict__ S,
    const uint16_t* __restrict__ shi, const uint16_t* __restrict__ slo, int64_t pre, int32_t K,
    int32_t N, int64_t post, const int32_t* scale_slot, int32_t* max_slot,
    int32_t* flags) {
  const int64_t f = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nf = pre * post;
  const int32_t shift = shift_of(scale_slot);
  Tc mx = 0;
  int bad = 0;
  if (f < nf) {
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
          const uint16_t xh_b = bf16_bits(static_cast<float>(x));
          const float xh = bf16_float(xh_b);
          const float xl = bf16_float(bf16_bits(static_cast<float>(x) - xh));
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            if (j < nn) {
              const float sh = bf16_float(shi[k * N + n0 + j]);
              const float sl = bf16_float(slo[k * N + n0 + j]);
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
          bad |= !isfinite(acc[j]);
          mx = fmax(mx, fabs(acc[j]));
        }
      }
    }
  }
  if (max_slot) {
    block_max_bad(mx, bad);
    if (threadIdx.x == 0) {
      const int32_t e = bad ? kExpBad : exp_of(static_cast<double>(mx));
      if (e != kExpZero) atomicMax(max_slot, e);
      if (bad) atomicOr(flags, 1);
    }
  }
}

// ------------------------------------------------------------------- ring
// 64x64 output tile per block, 256 threads, 4x4 outputs per thread.
constexpr int kRT = 64, kRK = 16;

template <typename T, bool SPLIT>
__global__ __launch_bounds__(kBlock) void ring_generic(
    const T* __restrict__ A, const T* __restrict__ B, int64_t m, int64_t n, int64_t k,
    const int32_t* sa, const int32_t* sb, T* __restrict__ C, const T* __restrict__ dotw,
    double* __restrict__ partials) {
  __shared__ T As[kRK][kRT];
  __shared__ T Bs[kRK][kRT];
  const int64_t m0 = static_cast<int64_t>(blockIdx.y) * kRT;
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * kRT;
  const int32_t ea = shift_of(sa), eb = shift_of(sb);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0;
  for (int64_t k0 = 0; k0 < k; k0 += kRK) {
    for (int e = threadIdx.x; e < kRK * kRT; e += blockDim.x) {
      const int kk = e / kRT, ii = e % kRT;
      const int64_t kg = k0 + kk;
      As[kk][ii] = (kg < k && m0 + ii < m) ? static_cast<T>(ldexp(A[kg * m + m0 + ii], -ea)) : T(0);
      Bs[kk][ii] = (kg < k && n0 + ii < n) ? static_cast<T>(ldexp(B[kg * n + n0 + ii], -eb)) : T(0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kRK; ++kk) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const T a = As[kk][ty * 4 + i];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const T b = Bs[kk][tx * 4 + j];
          if constexpr (SPLIT) {
            const float ah = bf16_float(bf16_bits(a)), al = bf16_float(bf16_bits(a - ah));
            const float bh = bf16_float(bf16_bits(b)), bl = bf16_float(bf16_bits(b - bh));
            float s = acc[i][j];
            s = fmaf(al, bh, s);
            s = fmaf(ah, bl, s);
            s = fmaf(ah, bh, s);
            acc[i][j] = s;
          } else {
            acc[i][j] = fma(a, b, acc[i][j]);
          }
        }
      }
    }
    __syncthreads();
  }
  double part = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t gi = m0 + ty * 4 + i;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t gj = n0 + tx * 4 + j;
      if (gi < m && gj < n) {
        if (dotw) part += static_cast<double>(acc[i][j]) * static_cast<double>(dotw[gi * n + gj]);
        else C[gi * n + gj] = acc[i][j];
      }
    }
  }
  if (dotw) {
    // fixed-order block reduction (deterministic)
    __shared__ double red[kBlock];
    red[threadIdx.x] = part;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
      if (static_cast<int>(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) partials[static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
  }
}

// --------------------------------------------------------------- finalize
// Block-wide totals, valid in thread 0: the fixed-order sum of `np` partials
// (strided per thread, then a tree), the exponent sum over the rescale slots
// and step exponents, and the non-finite flag.
__device__ void block_totals(const DevState* state, const double* partials, int64_t np,
                             double& sum, int64_t& E_out, int32_t& bad_out) {
  __shared__ double red[kBlock];
  __shared__ int64_t red_e[kBlock];
  __shared__ int32_t red_bad[kBlock];
  const int32_t* slot_exp = reinterpret_cast<const int32_t*>(state + 1);
  const int32_t* site_exp = slot_exp + state->n_slots;
  const int32_t* site_bad = site_exp + state->n_steps;
  double s = 0.0;
  if (partials) {
    for (int64_t i = threadIdx.x; i < np; i += blockDim.x) s += partials[i];
  }
  int64_t E = 0;
  int32_t bad = 0;
  for (int i = threadIdx.x; i < state->n_slots; i += blockDim.x) {
    const int32_t e = slot_exp[i];
    if (e == kExpBad) bad = 1;
    else if (e != kExpZero) E += e;
  }
  for (int i = threadIdx.x; i < state->n_steps; i += blockDim.x) {
    E += site_exp[i];
    bad |= site_bad[i];
  }
  red[threadIdx.x] = s;
  red_e[threadIdx.x] = E;
  red_bad[threadIdx.x] = bad;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (static_cast<int>(threadIdx.x) < st) {
      red[threadIdx.x] += red[threadIdx.x + st];
      red_e[threadIdx.x] += red_e[threadIdx.x + st];
      red_bad[threadIdx.x] |= red_bad[threadIdx.x + st];
    }
    __syncthreads();
  }
  sum = red[0];
  E_out = red_e[0];
  bad_out = red_bad[0];
}

__global__ __launch_bounds__(kBlock) void finalize_kernel(DevState* state, const double* scalar,
                                                          const double* partials, int64_t np,
                                                          const EnvRec* cap, tn_result* copy) {
  double sum;
  int64_t E;
  int32_t bad;
  block_totals(state, partials, np, sum, E, bad);
  if (threadIdx.x != 0) return;
  const double mval = partials ? sum : *scalar;
  E += state->e_bias;
  if (cap) {
    // the boundary the cap dot closed against, scaled by 2^-e in the dot
    const int32_t e = cap->e;
    if (e == kExpBad) bad = 1;
    E += cap->bias + ((e == kExpZero || e == kExpBad) ? 0 : e);
  }
  const tn_result r = dev::assemble_result(mval, E, bad | (state->flags & 1));
  state->result = r;
  if (copy) *copy = r;
}

// ------------------------------------------------------------ environments
constexpr int64_t kCapChunk = 1024;   // least entries per block of the cap dot
constexpr int64_t kCapBlocks = 2048;  // most blocks

__global__ __launch_bounds__(kBlock) void env_cap_kernel(const void* __restrict__ B,
                                                         const void* __restrict__ Rv, int64_t n,
                                                         int64_t chunk, int32_t f64,
                                                         const int32_t* slot_b, const EnvRec* rec,
                                                         double* __restrict__ partials) {
  __shared__ double red[kBlock];
  const int32_t er_raw = rec->e;
  const int32_t er = (er_raw == kExpZero || er_raw == kExpBad) ? 0 : er_raw;
  const double sb = ldexp(1.0, -shift_of(slot_b));
  const double sr = ldexp(1.0, -er);
  const int64_t lo = static_cast<int64_t>(blockIdx.x) * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  double s = 0.0;
  if (f64) {
    const double* b = static_cast<const double*>(B);
    const double* r = static_cast<const double*>(Rv);
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s += (b[i] * sb) * (r[i] * sr);
  } else {
    const float* b = static_cast<const float*>(B);
    const float* r = static_cast<const float*>(Rv);
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x)
      s += (static_cast<double>(b[i]) * sb) * (static_cast<double>(r[i]) * sr);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (static_cast<int>(threadIdx.x) < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void env_tap_kernel(DevState* state, const int32_t* slot_last,
                                                         EnvRec* rec) {
  double unused;
  int64_t E;
  int32_t bad;
  block_totals(state, nullptr, 0, unused, E, bad);
  if (threadIdx.x != 0) return;
  const int32_t e = slot_last ? *slot_last : kExpZero;
  EnvRec out;
  out.pad = 0;
  if (bad || (state->flags & 1) || e == kExpBad) {
    out.bias = 0;
    out.e = kExpBad;
  } else {
    out.e = e;
    out.bias = E + state->e_bias - (e == kExpZero ? 0 : e);
  }
  *rec = out;
}

// ------------------------------------------------------- site environments
constexpr int kSiteTMax = 128;                                // (p, q) positions per tile
constexpr int kSiteLds = 48 * 1024;                           // LDS bytes for the two tiles
constexpr int kSitePer = (kSiteEnvMaxXY + kBlock - 1) / kBlock;   // (x, y) pairs per thread

__device__ inline double env_scale(const EnvRec* rec) {
  if (!rec) return 1.0;
  const int32_t e = rec->e;
  return ldexp(1.0, (e == kExpZero || e == kExpBad) ? 0 : -e);
}

__device__ inline double load_any(const void* p, int64_t i, int32_t f64) {
  return f64 ? static_cast<const double*>(p)[i] : static_cast<double>(static_cast<const float*>(p)[i]);
}

// positions per tile: as many as fit the LDS budget with one pad entry per row
__host__ __device__ inline int site_tile(int rows) {
  int t = kSiteLds / (8 * rows) - 1;
  return t > kSiteTMax ? kSiteTMax : (t < 1 ? 1 : t);
}

__global__ __launch_bounds__(kBlock) void site_env_kernel(SiteEnvArgs a) {
  extern __shared__ double sm[];
  const int rows = a.X + a.Y;
  const int T = site_tile(rows), ld = T + 1;   // padded row stride: rows fall in distinct banks
  double* Ls = sm;                             // [X][ld]
  double* Rs = sm + a.X * ld;                  // [Y][ld]
  const int64_t n = a.P * a.Q;
  const int32_t nxy = a.X * a.Y;
  const double sl = env_scale(a.l_rec), sr = env_scale(a.r_rec);
  double acc[kSitePer];
  for (int i = 0; i < kSitePer; ++i) acc[i] = 0.0;
  for (int64_t t0 = static_cast<int64_t>(blockIdx.x) * T; t0 < n;
       t0 += static_cast<int64_t>(gridDim.x) * T) {
    for (int idx = threadIdx.x; idx < rows * T; idx += blockDim.x) {
      const int row = idx / T, t = idx % T;
      const int64_t j = t0 + t;
      double v = 0.0;
      if (j < n) {
        const int64_t p = j / a.Q, q = j % a.Q;
        if (row < a.X) {
          v = a.L ? load_any(a.L, (p * a.X + row) * a.Q + q, a.l_f64) * sl : 1.0;
        } else {
          const int y = row - a.X;
          v = a.Rv ? load_any(a.Rv, (p * a.Y + y) * a.Q + q, a.r_f64) * sr : 1.0;
        }
      }
      if (row < a.X) Ls[row * ld + t] = v;
      else Rs[(row - a.X) * ld + t] = v;
    }
    __syncthreads();
    for (int i = 0; i < kSitePer; ++i) {
      const int xy = threadIdx.x + i * kBlock;
      if (xy < nxy) {
        const int x = xy / a.Y, y = xy % a.Y;
        double s = 0.0;
        for (int t = 0; t < T; ++t) s += Ls[x * ld + t] * Rs[y * ld + t];
        acc[i] += s;
      }
    }
    __syncthreads();
  }
  for (int i = 0; i < kSitePer; ++i) {
    const int xy = threadIdx.x + i * kBlock;
    if (xy < nxy) a.partials[static_cast<int64_t>(blockIdx.x) * nxy + xy] = acc[i];
  }
}

struct SiteDots {
  SiteDot d[kSiteDotsMax];
  int32_t n;
};

__global__ __launch_bounds__(kBlock) void site_dots_kernel(SiteEnvArgs a, SiteDots ds) {
  extern __shared__ double env[];         // [X * Y]
  __shared__ double red[kBlock];
  __shared__ int red_bad[kBlock];
  const int32_t nxy = a.X * a.Y;
  for (int xy = threadIdx.x; xy < nxy; xy += blockDim.x) {
    double s = 0.0;
    for (int32_t b = 0; b < a.blocks; ++b) s += a.partials[static_cast<int64_t>(b) * nxy + xy];
    env[xy] = s;
  }
  __syncthreads();
  int64_t E = 0;
  int bad0 = 0;
  for (const EnvRec* rec : {a.l_rec, a.r_rec}) {
    if (!rec) continue;
    const int32_t e = rec->e;
    if (e == kExpBad) bad0 = 1;
    E += rec->bias + ((e == kExpZero || e == kExpBad) ? 0 : e);
  }
  for (int32_t k = 0; k < ds.n; ++k) {
    const SiteDot& d = ds.d[k];
    double s = 0.0;
    int bad = 0;
    for (int xy = threadIdx.x; xy < nxy; xy += blockDim.x) {
      int64_t rem = xy, off = 0;
      for (int ax = d.ndim - 1; ax >= 0; --ax) {
        const int64_t i = rem % d.dims[ax];
        rem /= d.dims[ax];
        off += i * d.cstride[ax];
      }
      const double o = d.site[off];
      bad |= !isfinite(o);
      s += env[xy] * o;
    }
    red[threadIdx.x] = s;
    red_bad[threadIdx.x] = bad;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
      if (static_cast<int>(threadIdx.x) < st) {
        red[threadIdx.x] += red[threadIdx.x + st];
        red_bad[threadIdx.x] |= red_bad[threadIdx.x + st];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) *d.out = dev::assemble_result(red[0], E, bad0 | red_bad[0]);
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_stage(const StageDesc* descs, int32_t n_steps, StagedArrays st, StageTargets t,
                        hipStream_t stream) {
  if (n_steps <= 0) return hipSuccess;
  if (n_steps < kStageWaveSites) {
    hipLaunchKernelGGL(stage_kernel<1>, dim3(n_steps), dim3(kBlock), 0, stream, descs, n_steps, st,
                       t);
  } else {
    constexpr int spb = kBlock / 64;
    hipLaunchKernelGGL(stage_kernel<spb>, dim3((n_steps + spb - 1) / spb), dim3(kBlock), 0, stream,
                       descs, n_steps, st, t);
  }
  return hipGetLastError();
}

namespace {
int32_t g_absorb_policy = 0;
int32_t g_fuse_steps = 2;
}

void set_absorb_policy(int32_t policy) { g_absorb_policy = policy; }
int32_t absorb_policy() { return g_absorb_policy; }
void set_fuse_steps(int32_t on) { g_fuse_steps = on; }
int32_t fuse_steps() { return g_fuse_steps; }

hipError_t launch_absorb(const AbsorbArgs& a, const StagedArrays& st, DevState* state,
                         hipStream_t stream, const char** kname) {
  if (g_absorb_policy == 0 && absorb_mfma_supported(a))
    return launch_absorb_mfma(a, st, state, stream, kname);
  const int64_t nf = a.pre * a.post;
  const int64_t blocks = (nf + kBlock - 1) / kBlock;
  if (blocks <= 0) return hipSuccess;
  if (blocks > INT_MAX || a.K > INT_MAX || a.N > INT_MAX) return hipErrorInvalidValue;
  int32_t* flags = &state->flags;
  const int32_t K = static_cast<int32_t>(a.K), N = static_cast<int32_t>(a.N);
  dim3 g(static_cast<uint32_t>(blocks)), b(kBlock);
  if (a.out_type == EL_F64) {
    *kname = a.in_type == EL_F64 ? "absorb_valu_f64" : "absorb_valu_f32_to_f64";
    if (a.in_type == EL_F64)
      hipLaunchKernelGGL((absorb_generic<double, double, false>), g, b, 0, stream,
                         static_cast<const double*>(a.in), static_cast<double*>(a.out),
                         st.s64 + a.s_off, st.shi + a.s_off, st.slo + a.s_off, a.pre, K, N,
                         a.post, a.scale_slot, a.max_slot, flags);
    else
      hipLaunchKernelGGL((absorb_generic<float, double, false>), g, b, 0, stream,
                         static_cast<const float*>(a.in), static_cast<double*>(a.out),
                         st.s64 + a.s_off, st.shi + a.s_off, st.slo + a.s_off, a.pre, K, N,
                         a.post, a.scale_slot, a.max_slot, flags);
  } else if (a.arith == AR_BF16X3) {
    *kname = "absorb_valu_bf16x3";
    hipLaunchKernelGGL((absorb_generic<float, float, true>), g, b, 0, stream,
                       static_cast<const float*>(a.in), static_cast<float*>(a.out),
                       st.s32 + a.s_off, st.shi + a.s_off, st.slo + a.s_off, a.pre, K, N, a.post,
                       a.scale_slot, a.max_slot, flags);
  } else {
    *kname = "absorb_valu_f32";
    hipLaunchKernelGGL((absorb_generic<float, float, false>), g, b, 0, stream,
                       static_cast<const float*>(a.in), static_cast<float*>(a.out),
                       st.s32 + a.s_off, st.shi + a.s_off, st.slo + a.s_off, a.pre, K, N, a.post,
                       a.scale_slot, a.max_slot, flags);
  }
  return hipGetLastError();
}

int64_t ring_partials(int64_t m, int64_t n) {
  // the vector-ALU kernel's 64 x 64 tiles give the larger count
  return ((m + kRT - 1) / kRT) * ((n + kRT - 1) / kRT);
}

hipError_t launch_ring(const RingArgs& a, hipStream_t stream, const char** kname,
                       int64_t* n_partials, int32_t* c_slices) {
  // split BF16x3 rings on the matrix cores take launch_ring_bf16x3_nt
  if (g_absorb_policy == 0 && ring_mfma_supported(a) && a.arith != AR_BF16X3)
    return launch_ring_mfma(a, stream, kname, n_partials, c_slices);
  // one 64 x 64 tile per workgroup, no split-K
  const bool dot = a.dot_with != nullptr;
  *n_partials = dot ? ring_partials(a.m, a.n) : 0;
  *c_slices = dot ? 0 : 1;
  const int64_t gx = (a.n + kRT - 1) / kRT, gy = (a.m + kRT - 1) / kRT;
  if (gx > INT_MAX || gy > 65535 || a.w_slices != 1 || (dot && *n_partials > a.partials_cap) ||
      (!dot && a.c_slices_cap < 1))
    return hipErrorInvalidValue;
  dim3 g(static_cast<uint32_t>(gx), static_cast<uint32_t>(gy)), b(kBlock);
  *kname = a.type == EL_F64 ? "ring_valu_f64" : (a.arith == AR_BF16X3 ? "ring_valu_bf16x3" : "ring_valu_f32");
  if (a.type == EL_F64) {
    hipLaunchKernelGGL((ring_generic<double, false>), g, b, 0, stream,
                       static_cast<const double*>(a.A), static_cast<const double*>(a.B), a.m, a.n,
                       a.k, a.sa, a.sb, static_cast<double*>(a.c_out),
                       static_cast<const double*>(a.dot_with), a.partials);
  } else if (a.arith == AR_BF16X3) {
    hipLaunchKernelGGL((ring_generic<float, true>), g, b, 0, stream,
                       static_cast<const float*>(a.A), static_cast<const float*>(a.B), a.m, a.n,
                       a.k, a.sa, a.sb, static_cast<float*>(a.c_out),
                       static_cast<const float*>(a.dot_with), a.partials);
  } else {
    hipLaunchKernelGGL((ring_generic<float, false>), g, b, 0, stream,
                       static_cast<const float*>(a.A), static_cast<const float*>(a.B), a.m, a.n,
                       a.k, a.sa, a.sb, static_cast<float*>(a.c_out),
                       static_cast<const float*>(a.dot_with), a.partials);
  }
  return hipGetLastError();
}

hipError_t launch_finalize(DevState* state, const double* scalar, tn_result* copy,
                           const double* partials, int64_t n_partials, hipStream_t stream,
                           const EnvRec* cap) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kBlock), 0, stream, state, scalar, partials,
                     n_partials, cap, copy);
  return hipGetLastError();
}

int64_t env_cap_blocks(int64_t n) {
  const int64_t chunk = std::max<int64_t>(kCapChunk, (n + kCapBlocks - 1) / kCapBlocks);
  return std::max<int64_t>((n + chunk - 1) / chunk, 1);
}

hipError_t launch_env_cap(const void* B, const void* Rv, int64_t n, int32_t f64,
                          const int32_t* slot_b, const EnvRec* rec, double* partials,
                          hipStream_t stream) {
  const int64_t chunk = std::max<int64_t>(kCapChunk, (n + kCapBlocks - 1) / kCapBlocks);
  const int64_t blocks = env_cap_blocks(n);
  hipLaunchKernelGGL(env_cap_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(kBlock), 0, stream,
                     B, Rv, n, chunk, f64, slot_b, rec, partials);
  return hipGetLastError();
}

int32_t site_env_blocks(int64_t P, int64_t Q, int32_t X, int32_t Y) {
  const int64_t T = site_tile(X + Y);
  const int64_t tiles = (P * Q + T - 1) / T;
  return static_cast<int32_t>(std::max<int64_t>(1, std::min<int64_t>(tiles, 256)));
}

hipError_t launch_site_env(const SiteEnvArgs& a, hipStream_t stream) {
  if (a.X < 1 || a.Y < 1 || a.X * a.Y > kSiteEnvMaxXY || a.P < 1 || a.Q < 1 ||
      a.blocks != site_env_blocks(a.P, a.Q, a.X, a.Y))
    return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * static_cast<size_t>(a.X + a.Y) * (site_tile(a.X + a.Y) + 1);
  hipLaunchKernelGGL(site_env_kernel, dim3(static_cast<uint32_t>(a.blocks)), dim3(kBlock), lds,
                     stream, a);
  return hipGetLastError();
}

hipError_t launch_site_dots(const SiteEnvArgs& a, const SiteDot* dots, int32_t n,
                            hipStream_t stream) {
  if (n < 1 || n > kSiteDotsMax || a.X * a.Y > kSiteEnvMaxXY) return hipErrorInvalidValue;
  SiteDots ds;
  std::memset(&ds, 0, sizeof(ds));
  for (int32_t i = 0; i < n; ++i) {
    int64_t entries = 1;
    for (int32_t ax = 0; ax < dots[i].ndim; ++ax) entries *= dots[i].dims[ax];
    if (dots[i].ndim < 0 || dots[i].ndim > 4 || entries != static_cast<int64_t>(a.X) * a.Y)
      return hipErrorInvalidValue;
    ds.d[i] = dots[i];
  }
  ds.n = n;
  const size_t lds = sizeof(double) * static_cast<size_t>(a.X) * a.Y;
  hipLaunchKernelGGL(site_dots_kernel, dim3(1), dim3(kBlock), lds, stream, a, ds);
  return hipGetLastError();
}

hipError_t launch_env_tap(DevState* state, const int32_t* slot_last, EnvRec* rec,
                          hipStream_t stream) {
  hipLaunchKernelGGL(env_tap_kernel, dim3(1), dim3(kBlock), 0, stream, state, slot_last, rec);
  return hipGetLastError();
}

}  // namespace tn
