// Column chunks held in registers: k consecutive rows (2 <= k <= 4) of one
// column of a sweep applied to 16 boundary columns by one wavefront, the
// intermediate results never leaving its registers (paper §4: the pairwise,
// sequential contraction; only the memory schedule changes).
//
// Slice.  As in the LDS chunk kernel the chunk's input, for one spectator
// fibre s = (p, q), is the run of rows
//     row = kidx0 * M1 + m,   m = (h_1, ..., h_{k-1}) in base 4, M1 = 4^(k-1)
// (kidx0 = (v, h_0), the first step's K index; h_0 only at the top edge).  A
// wavefront takes 16 fibres as the 16 MFMA columns: 16 consecutive q of one p
// when the suffix is a multiple of 16 (each row a 64- or 128-byte run), or 16
// consecutive p when the suffix is 1 (each fibre's rows contiguous).
//
// Registers.  After step j the wavefront holds Y_j[t][r] in lane group g
// (lane = 16 g + column): 4^(k-1) tiles t of 16 x 16, where the base-4 digits
// of t are (h'_0, ..., h'_{j-1}, h_{j+1}, ..., h_{k-1}) (outputs so far, then
// horizontal legs still to absorb), g = v'_j (the vertical leg just produced)
// and r = h'_j.  Step j + 1 contracts (v'_j, h_{j+1}) = (g, kk) for kk = 0..3:
// the four tiles that differ only in the digit h_{j+1} hold, in register a,
// exactly the B operand of the product for h'_j = a, and the product's output
// replaces them in place.  This layout is made by the row order of the A
// operand (the site matrix): MFMA row i holds output n = 4 h' + v' with
// (lane group, register) of row i equal to (v', h').  The f32 and bf16 16x16
// MFMAs leave row i in (i / 4, i % 4), so A row i is n = 4 (i % 4) + i / 4;
// the f64 MFMA leaves row i in (i % 4, i / 4), so A row i is n = i.  No lane
// exchanges, no LDS, no barriers.
//
// K slots.  Lane group g supplies the K indices kidx = 4 g + kk (kk = 0..3)
// of every step (kidx0 = g at the top edge, one MFMA); bf16x3 concatenates
// [x_hi s_hi | x_hi s_lo] and [x_lo s_hi | 0] over those four indices in two
// 16x16x32 MFMAs.
//
// Last step: 16 outputs (n = MFMA row) stored as 64-/128-byte row runs, or at
// the bottom edge 4 outputs n' in the four registers of lane group 0 (f32: A
// rows 0..3; f64: rows 0, 4, 8, 12), stored as one 16- or 32-byte vector per
// fibre.
//
// Occupancy: 4^(k-1) * 4 accumulator values per lane (256 for a 4-row f32
// chunk, one wavefront per SIMD; 64 values for 3 rows).  Workgroups are one
// wavefront, so the phases (loads + first step, inner steps, stores) of the
// wavefronts on one CU drift apart and overlap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <type_traits>

#include "absorb_device.hpp"
#include "chunk_group.hpp"
#include "kernels.hpp"

namespace tn {
namespace {

using namespace dev;
using chunk::GroupRef;
using chunk::UnitRef;

// Output n of MFMA row i, or -1 for a zero row.  NK: 0 = step feeding the
// next one in registers; 1 = last step with 16 outputs; 2 = last step with 4.
template <int MODE, int NK>
__device__ inline int n_of_row(int i) {
  if constexpr (NK == 0) return MODE == M_F64 ? i : 4 * (i & 3) + (i >> 2);
  if constexpr (NK == 1) return i;
  if constexpr (MODE == M_F64) return (i & 3) ? -1 : (i >> 2);
  return i < 4 ? i : -1;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// bf16 high and low parts of x0, x1 (round to nearest even, as one packed
// conversion each): hi = [hi(x0) | hi(x1) << 16], lo likewise of x - hi.
__device__ inline void split_bf16(float x0, float x1, uint32_t& hi, uint32_t& lo) {
  hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{x0, x1}, bf16x2));
  const float h0 = __uint_as_float(hi << 16), h1 = __uint_as_float(hi & 0xffff0000u);
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{x0 - h0, x1 - h1}, bf16x2));
}

// A operands of one step for lane (c, g).  f32/f64: a[kk] = S[4g + kk][n(c)];
// bf16x3 against B = [hi(x) | lo(x)] over kidx = 4g .. 4g + 3: a0 = [hi(S) |
// hi(S)], a1 = [lo(S) | 0] (the three products hi hi, hi lo, lo hi).  ONE (one
// K index per lane group, kidx = g + 4 kq): a[0] = S[kidx][n(c)]; bf16x3 a0 =
// [hi, hi, lo, 0 ...] against B = [hi(x), lo(x), hi(x), 0 ...].
template <typename T, int MODE>
struct ROps {
  T a[4];
  bf16x8 a0, a1;
};

// The loads of reg_ops apart from its arithmetic: raw values as loaded (f32 /
// f64 entries; bf16x3 bit patterns of the hi and lo parts; lanes of zero rows
// load row 0 and are zeroed when built), so a kernel can issue them early and
// use them after a wait of its own.
template <typename T, int MODE>
struct RawOps {
  T a[4];
  uint32_t h[4], l[4];
  bool live;
};

template <typename T, int MODE, bool ONE, int NK>
__device__ inline RawOps<T, MODE> reg_ops_load(const void* Sv, const uint16_t* H,
                                               const uint16_t* L, int c, int g, int kq = 0) {
  constexpr int N = NK == 2 ? 4 : 16;
  const int n = n_of_row<MODE, NK>(c), nn = n >= 0 ? n : 0;
  RawOps<T, MODE> r;
  r.live = n >= 0;
  if constexpr (MODE == M_BF16X3) {
#pragma unroll
    for (int i = 0; i < (ONE ? 1 : 4); ++i) {
      const int k = ONE ? g + 4 * kq : 4 * g + i;
      r.h[i] = H[k * N + nn];
      r.l[i] = L[k * N + nn];
    }
  } else {
    const T* S = static_cast<const T*>(Sv);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      r.a[kk] = (!ONE || kk == 0) ? S[(ONE ? g + 4 * kq : 4 * g + kk) * N + nn] : T(0);
  }
  return r;
}

template <typename T, int MODE, bool ONE>
__device__ inline ROps<T, MODE> reg_ops_build(const RawOps<T, MODE>& r) {
  ROps<T, MODE> o;
  if constexpr (MODE == M_BF16X3) {
    const __bf16 z = __builtin_bit_cast(__bf16, static_cast<uint16_t>(0));
    auto bf = [&](uint32_t v) { return r.live ? __builtin_bit_cast(__bf16, static_cast<uint16_t>(v)) : z; };
    if constexpr (ONE) {
      o.a0 = bf16x8{bf(r.h[0]), bf(r.h[0]), bf(r.l[0]), z, z, z, z, z};
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        o.a0[i] = bf(r.h[i]);
        o.a0[4 + i] = bf(r.h[i]);
        o.a1[i] = bf(r.l[i]);
        o.a1[4 + i] = z;
      }
    }
  } else {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) o.a[kk] = r.live ? r.a[kk] : T(0);
  }
  return o;
}

// The values pass through an empty asm block: nothing that uses them can be
// scheduled before this point.
template <typename T, int MODE, bool ONE>
__device__ inline void launder(RawOps<T, MODE>& r) {
  if constexpr (MODE == M_BF16X3) {
#pragma unroll
    for (int i = 0; i < (ONE ? 1 : 4); ++i) asm volatile("" : "+v"(r.h[i]), "+v"(r.l[i]));
  } else {
#pragma unroll
    for (int kk = 0; kk < (ONE ? 1 : 4); ++kk) asm volatile("" : "+v"(r.a[kk]));
  }
}

template <typename T, int MODE, bool ONE, int NK>
__device__ inline ROps<T, MODE> reg_ops(const void* Sv, const uint16_t* H, const uint16_t* L,
                                        int c, int g, int kq = 0) {
  return reg_ops_build<T, MODE, ONE>(reg_ops_load<T, MODE, ONE, NK>(Sv, H, L, c, g, kq));
}

template <int MODE>
using RV4 = typename std::conditional<MODE == M_F64, f64x4, f32x4>::type;

// The ONE form accumulating into acc: acc += A x over the lane groups' K
// indices.
template <typename T, int MODE>
__device__ inline RV4<MODE> reg_mma_one(const ROps<T, MODE>& o, T x, RV4<MODE> acc) {
  if constexpr (MODE == M_BF16X3) {
    uint32_t h, l;
    split_bf16(x, x, h, l);
    // [hi, lo, hi, 0 ...]: word 0 = hi | lo << 16, word 1 = hi
    const u32x4 w0 = {(h & 0xffffu) | (l << 16), h & 0xffffu, 0u, 0u};
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.a0, __builtin_bit_cast(bf16x8, w0), acc,
                                                   0, 0, 0);
  } else if constexpr (MODE == M_F64) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(o.a[0], x, acc, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(o.a[0], x, acc, 0, 0, 0);
  }
}

// Two ONE-form products (tiles with entries x0, x1) sharing the bf16 splits.
template <typename T, int MODE>
__device__ inline void reg_mma_one2(const ROps<T, MODE>& o, T x0, T x1, RV4<MODE>& acc0,
                                    RV4<MODE>& acc1) {
  if constexpr (MODE == M_BF16X3) {
    uint32_t h, l;
    split_bf16(x0, x1, h, l);
    const u32x4 w0 = {(h & 0xffffu) | (l << 16), h & 0xffffu, 0u, 0u};
    const u32x4 w1 = {(h >> 16) | (l & 0xffff0000u), h >> 16, 0u, 0u};
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.a0, __builtin_bit_cast(bf16x8, w0), acc0,
                                                   0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.a0, __builtin_bit_cast(bf16x8, w1), acc1,
                                                   0, 0, 0);
  } else {
    acc0 = reg_mma_one<T, MODE>(o, x0, acc0);
    acc1 = reg_mma_one<T, MODE>(o, x1, acc1);
  }
}

// NG independent 16x16 products; xs[q][kk] is slot (g, kk) of product q.
template <typename T, int MODE, bool TOPF, int NG>
__device__ inline void reg_mma(const ROps<T, MODE>& o, const T (&xs)[NG][4],
                               RV4<MODE> (&acc)[NG]) {
  if constexpr (MODE == M_BF16X3) {
    // operands built per product, right before its MFMAs (short live ranges),
    // two entries per conversion
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      if constexpr (TOPF) {
        if (q % 2 == 0) {
          acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
          acc[q + 1] = f32x4{0.f, 0.f, 0.f, 0.f};
          reg_mma_one2<T, MODE>(o, xs[q][0], xs[q + 1][0], acc[q], acc[q + 1]);
        }
      } else {
        uint32_t h01, l01, h23, l23;
        split_bf16(xs[q][0], xs[q][1], h01, l01);
        split_bf16(xs[q][2], xs[q][3], h23, l23);
        const bf16x8 b = __builtin_bit_cast(bf16x8, u32x4{h01, h23, l01, l23});
        acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.a0, b, f32x4{0.f, 0.f, 0.f, 0.f}, 0,
                                                          0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.a1, b, acc[q], 0, 0, 0);
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < NG; ++q) acc[q] = RV4<MODE>{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < (TOPF ? 1 : 4); ++kk)
#pragma unroll
      for (int q = 0; q < NG; ++q) {
        if constexpr (MODE == M_F64)
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(o.a[kk], xs[q][kk], acc[q], 0, 0, 0);
        else
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.a[kk], xs[q][kk], acc[q], 0, 0, 0);
      }
  }
}

// Step J >= 1 in place: tiles t = (P, kk, R) -> (P, a, R), the digit h_J at
// stride S = 4^(k-1-J).
template <typename T, int MODE, int K, int J>
__device__ inline void reg_step(RV4<MODE> (&y)[1 << (2 * (K - 1))], const ROps<T, MODE>& o) {
  constexpr int S = 1 << (2 * (K - 1 - J)), NP = 1 << (2 * (J - 1));
#pragma unroll
  for (int P = 0; P < NP; ++P)
#pragma unroll
    for (int R = 0; R < S; ++R) {
      T xs[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) xs[a][kk] = y[P * 4 * S + kk * S + R][a];
      RV4<MODE> acc[4];
      reg_mma<T, MODE, false, 4>(o, xs, acc);
#pragma unroll
      for (int a = 0; a < 4; ++a) y[P * 4 * S + a * S + R] = acc[a];
    }
}

template <typename T, int MODE, int K, int J, bool P1>
__device__ inline void reg_steps_from(RV4<MODE> (&y)[1 << (2 * (K - 1))], UnitRef d, int c, int g) {
  if constexpr (J < K) {
    constexpr int NK = J + 1 < K ? 0 : (P1 ? 2 : 1);
    const ROps<T, MODE> o = reg_ops<T, MODE, false, NK>(d.S[J], d.hi[J], d.lo[J], c, g);
    reg_step<T, MODE, K, J>(y, o);
    reg_steps_from<T, MODE, K, J + 1, P1>(y, d, c, g);
  }
}

template <typename T>
__device__ inline void publish_wave(T mx, int bad, int32_t* max_slot, int32_t* flags) {
  double m = static_cast<double>(mx);
  for (int off = 32; off > 0; off >>= 1) {
    m = fmax(m, __shfl_xor(m, off));
    bad |= __shfl_xor(bad, off);
  }
  if ((threadIdx.x & 63) == 0) {
    const int32_t e = bad ? kExpBad : exp_of_d(m);
    // the slot only grows during a launch: skip the atomic when it cannot
    // raise it
    if (e != kExpZero && e > __hip_atomic_load(max_slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(max_slot, e);
    if (bad) atomicOr(flags, 1);
  }
}

// Tile forms (HBM streams at 3.0-3.5 TB/s when the row runs one wavefront
// instruction touches are 64 bytes long and at 4.7-5.0 TB/s when they are 128
// bytes, whatever the instruction width or the occupancy: copy kernels of
// both shapes on MI355X):
//   FORM_DIRECT (8-byte entries, or a suffix of 16): 16 consecutive q of one
//     p per one-wavefront workgroup; the registers are loaded and stored
//     directly (row runs of 16 entries), step 0 with the K slots kidx0 =
//     4 g + kk of all four MFMAs at once.
//   FORM_PAIR (4-byte entries, suffix a multiple of 32): 32 consecutive q per
//     two-wavefront workgroup, wavefront w taking q0 + 16 w + c; the slice
//     goes through an LDS stage shared by the two, a quarter at a time, with
//     128-byte row runs.
//   FORM_BOTTOM (suffix 1): 16 consecutive p whose slices are one contiguous
//     block, through an LDS stage private to the wavefront.
// A quarter is QR = 4^k rows: step 0's K indices kidx0 = 4 kk + g (g = 0..3)
// of quarter kk, or the whole slice at the top edge (kidx0 = g).  Staged
// forms take step 0 one quarter at a time (one K index per lane group,
// accumulating) while the next two quarters' loads are in flight.
enum { FORM_DIRECT = 0, FORM_PAIR = 1, FORM_BOTTOM = 2 };

template <int K>
constexpr int quarter_rows() { return 4 << (2 * (K - 1)); }
// FORM_BOTTOM stage: fibre i, row j at i * pitch + j.
template <typename T, int K>
constexpr int bottom_pitch() { return quarter_rows<K>() + static_cast<int>(16 / sizeof(T)); }
template <typename T, int K, int FORM>
constexpr int stage_entries() {
  return FORM == FORM_PAIR ? 2 * (32 * quarter_rows<K>() + 64)
                           : FORM == FORM_BOTTOM ? 2 * 16 * bottom_pitch<T, K>() : 1;
}

// Uniform 64-bit base plus a 32-bit per-lane byte offset: one VGPR of
// address per lane for all of a wavefront's accesses.
template <typename V>
__device__ inline V ld_at(const void* ubase, uint32_t off) {
  return *reinterpret_cast<const V*>(static_cast<const char*>(ubase) + static_cast<uint64_t>(off));
}
template <typename V>
__device__ inline void st_at(void* ubase, uint32_t off, V v) {
  *reinterpret_cast<V*>(static_cast<char*>(ubase) + static_cast<uint64_t>(off)) = v;
}

// FORM_DIRECT.
template <typename T, int MODE, int K, bool TOP>
__device__ inline void tile_direct(UnitRef d, int64_t tile, T& mx, int& bad) {
  using V4 = RV4<MODE>;
  constexpr int M1 = 1 << (2 * (K - 1)), KK0 = TOP ? 1 : 4;
  constexpr int RIN = KK0 * quarter_rows<K>(), ROUT = 16 * M1;
  constexpr int ES = sizeof(T);
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
  const int32_t shift = shift_of(d.scale_slot);
  const int64_t post = d.post, tq = post / 16, p = tile / tq, q0 = (tile - p * tq) * 16;
  const int64_t rowb = post * ES;
  // rows kidx0 M1 + t, kidx0 = (TOP ? g : 4 g) + kk
  const char* src = static_cast<const char*>(d.in) + (p * RIN * post + q0) * ES;
  const uint32_t lin = static_cast<uint32_t>((TOP ? g : 4 * g) * M1 * rowb + c * ES);
  T x[M1][4];
#pragma unroll
  for (int kk = 0; kk < KK0; ++kk)
#pragma unroll
    for (int t = 0; t < M1; ++t) x[t][kk] = ld_at<T>(src + (kk * M1 + t) * rowb, lin);
  if (shift) {
#pragma unroll
    for (int t = 0; t < M1; ++t)
#pragma unroll
      for (int kk = 0; kk < KK0; ++kk) x[t][kk] = static_cast<T>(ldexp(x[t][kk], -shift));
  }
  V4 y[M1];
  {
    const ROps<T, MODE> o = reg_ops<T, MODE, TOP, 0>(d.S[0], d.hi[0], d.lo[0], c, g);
#pragma unroll
    for (int t = 0; t < M1; t += 4) {
      T xs[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) xs[q][kk] = kk < KK0 ? x[t + q][kk] : T(0);
      V4 acc[4];
      reg_mma<T, MODE, TOP, 4>(o, xs, acc);
#pragma unroll
      for (int q = 0; q < 4; ++q) y[t + q] = acc[q];
    }
  }
  reg_steps_from<T, MODE, K, 1, false>(y, d, c, g);
  // register r of lane (c, g): output n = 4g + r (f32, bf16) or g + 4r (f64)
  char* dst = static_cast<char*>(d.out) + (p * ROUT * post + q0) * ES;
  const uint32_t lout = static_cast<uint32_t>((MODE == M_F64 ? g : 4 * g) * rowb + c * ES);
#pragma unroll
  for (int t = 0; t < M1; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const T v = static_cast<T>(y[t][r]);
      st_at<T>(dst + (t * 16 + (MODE == M_F64 ? 4 * r : r)) * rowb, lout, v);
      track(v, mx, bad);
    }
}

// Step 0 of the staged forms, one quarter: y[t] += S_0^T x over lane group g's
// K index of the quarter (operands o of that quarter).
template <typename T, int MODE, int K>
__device__ inline void step0_quarter(const ROps<T, MODE>& o, RV4<MODE> (&y)[1 << (2 * (K - 1))],
                                     T (&x)[1 << (2 * (K - 1))], int32_t shift) {
  constexpr int M1 = 1 << (2 * (K - 1));
  if (shift) {
#pragma unroll
    for (int t = 0; t < M1; ++t) x[t] = static_cast<T>(ldexp(x[t], -shift));
  }
#pragma unroll
  for (int t = 0; t < M1; t += 2) reg_mma_one2<T, MODE>(o, x[t], x[t + 1], y[t], y[t + 1]);
}

// Asynchronous fills of the stage: global_load_lds with 16 bytes per lane
// writes lane L's 16 bytes to LDS at (uniform base) + 16 L, without passing
// through registers, so two quarters can be in flight while a third is
// multiplied.  The compiler does not see these writes: the waits below are
// explicit (s_waitcnt on the number of fills issued after the ones needed;
// fills complete in issue order), followed by a compiler memory barrier.  The
// workgroup barrier is the bare s_barrier: the fence of __syncthreads would
// also wait for the fills still in flight.
typedef __attribute__((address_space(3))) void* LdsPtr;
__device__ inline void lds_fill16(const void* g, void* lds) {
#if __HIP_DEVICE_COMPILE__
  __builtin_amdgcn_global_load_lds(g, (LdsPtr)(lds), 16, 0, 0);
#else
  (void)g;
  (void)lds;
#endif
}
// s_waitcnt immediates: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8;
// the fields not waited on hold their maxima.
template <int N>
__device__ inline void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | (((N >> 4) & 3) << 14));
  asm volatile("" ::: "memory");
}
__device__ inline void wait_lds() {
  __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14));
  asm volatile("" ::: "memory");
}
__device__ inline void wg_barrier() {
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// FORM_PAIR (4-byte entries).  Two input buffers of rows of 32 fibres: row j
// at j * 32 + s + 16 (j / SB), SB = max(M1, 8) (the quarter's K blocks
// shifted apart so the lane groups of an MFMA-layout read fall on different
// banks; a fill covers 8 rows); output row j at (j / 4) * 144 + (j % 4) * 32
// + s (rows 4 apart, one register of the four lane groups, 16 banks apart).
template <typename T, int MODE, int K, bool TOP>
__device__ inline void tile_pair(UnitRef d, int64_t tile, T& mx, int& bad, T* stage) {
  using V4 = RV4<MODE>;
  static_assert(sizeof(T) == 4, "4-byte entries");
  constexpr int M1 = 1 << (2 * (K - 1)), KK0 = TOP ? 1 : 4, QR = quarter_rows<K>();
  constexpr int RIN = KK0 * QR, ROUT = 16 * M1, NIT = QR / 16;
  constexpr int SB = M1 >= 8 ? M1 : 8, IB = 32 * QR + 64;
  constexpr int LPW = QR / 16;   // 1 KiB fills per wavefront and quarter (8 rows each)
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, c = lane & 15, g = lane >> 4;
  const int32_t shift = shift_of(d.scale_slot);
  const int64_t post = d.post, tq = post / 32, run = tile / 2, p = run / tq;
  const int64_t q0 = (run - p * tq) * 32, rowb = post * 4;
  const char* src = static_cast<const char*>(d.in) + (p * RIN * post + q0) * 4;
  // step 0's operands for every quarter, complete before the first fill (a
  // later wait for them would also wait for the fills issued before them)
  ROps<T, MODE> o0[KK0];
#pragma unroll
  for (int kk = 0; kk < KK0; ++kk) o0[kk] = reg_ops<T, MODE, true, 0>(d.S[0], d.hi[0], d.lo[0], c, g, kk);
  wait_vm<0>();
  // fill i of wavefront w: rows j0 = 8 (2i + w) .. j0 + 7; lane L takes row
  // j0 + L / 8, fibres 4 (L % 8) .. + 3
  const uint32_t lfill = static_cast<uint32_t>((lane >> 3) * rowb + 16 * (lane & 7));
  auto fill_q = [&](int kk, T* buf) {
#pragma unroll
    for (int i = 0; i < LPW; ++i) {
      const int j0 = 8 * (2 * i + w);
      lds_fill16(src + (kk * QR + j0) * rowb + lfill, buf + j0 * 32 + 16 * (j0 / SB));
    }
  };
  V4 y[M1];
#pragma unroll
  for (int t = 0; t < M1; ++t) y[t] = V4{0, 0, 0, 0};
  fill_q(0, stage);
  if (KK0 > 1) fill_q(1, stage + IB);
#pragma unroll
  for (int kk = 0; kk < KK0; ++kk) {
    T* buf = stage + (kk & 1) * IB;
    if (kk + 1 < KK0) wait_vm<LPW>();
    else wait_vm<0>();
    wg_barrier();
    T x[M1];
#pragma unroll
    for (int t = 0; t < M1; ++t) {
      const int j = g * M1 + t;
      x[t] = buf[j * 32 + 16 * w + c + 16 * (j / SB)];
    }
    wait_lds();
    wg_barrier();
    if (kk + 2 < KK0) fill_q(kk + 2, buf);
    step0_quarter<T, MODE, K>(o0[kk], y, x, shift);
  }
  reg_steps_from<T, MODE, K, 1, false>(y, d, c, g);
  // output rows t * 16 + n, a quarter (M1 / 4 tiles, QR rows) at a time;
  // register r of lane (c, g) is n = 4g + r
  char* dst = static_cast<char*>(d.out) + (p * ROUT * post + q0) * 4;
  const int jr = tid >> 3, s4 = 4 * (tid & 7);
  const uint32_t lio = static_cast<uint32_t>(jr * rowb + s4 * 4);
  constexpr int TQ = M1 / 4;
#pragma unroll
  for (int qo = 0; qo < 4; ++qo) {
#pragma unroll
    for (int tt = 0; tt < TQ; ++tt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = tt * 16 + 4 * g + r;
        stage[(j >> 2) * 144 + (j & 3) * 32 + 16 * w + c] = y[qo * TQ + tt][r];
      }
    wait_lds();
    wg_barrier();
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int j = 16 * it + jr;
      const V4 v = *reinterpret_cast<const V4*>(stage + (j >> 2) * 144 + (j & 3) * 32 + s4);
      st_at<V4>(dst + (qo * QR + 16 * it) * rowb, lio, v);
#pragma unroll
      for (int r = 0; r < 4; ++r) track(static_cast<T>(v[r]), mx, bad);
    }
    wait_lds();
    wg_barrier();
  }
}

// FORM_BOTTOM.  Two input buffers, fibre i's rows at i * pitch + j (each
// fibre's quarter filled by its own fills, or by the first QR ES / 16 lanes
// of one when it is under 1 KiB); the outputs (4 rows per tile t, in the four
// registers of lane group 0) through the first buffer.
template <typename T, int MODE, int K, bool TOP>
__device__ inline void tile_bottom(UnitRef d, int64_t tile, T& mx, int& bad, T* stage) {
  using V4 = RV4<MODE>;
  constexpr int M1 = 1 << (2 * (K - 1)), KK0 = TOP ? 1 : 4, QR = quarter_rows<K>();
  constexpr int RIN = KK0 * QR, ROUT = 4 * M1, NIT = QR / 16, ES = sizeof(T);
  constexpr int PT = bottom_pitch<T, K>(), VQ = QR / 4, BB = 16 * PT;
  constexpr int FB = QR * ES;                             // bytes of one fibre's quarter
  constexpr int PIECES = FB >= 1024 ? FB / 1024 : 1;      // fills per fibre
  constexpr int LANES = FB >= 1024 ? 64 : FB / 16;        // active lanes of a fill
  constexpr int LPW = 16 * PIECES;                        // fills per quarter
  static_assert(ROUT == QR, "the output fits the staging rows");
  static_assert(LPW < 64, "vmcnt range");
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
  const int32_t shift = shift_of(d.scale_slot);
  const char* src = static_cast<const char*>(d.in) + tile * 16 * RIN * ES;
  ROps<T, MODE> o0[KK0];
#pragma unroll
  for (int kk = 0; kk < KK0; ++kk) o0[kk] = reg_ops<T, MODE, true, 0>(d.S[0], d.hi[0], d.lo[0], c, g, kk);
  wait_vm<0>();
  auto fill_q = [&](int kk, T* buf) {
#pragma unroll
    for (int i = 0; i < 16; ++i)
#pragma unroll
      for (int pc = 0; pc < PIECES; ++pc)
        if (lane < LANES)
          lds_fill16(src + (i * RIN + kk * QR) * ES + pc * 1024 + 16 * lane,
                     buf + i * PT + pc * (1024 / ES));
  };
  V4 y[M1];
#pragma unroll
  for (int t = 0; t < M1; ++t) y[t] = V4{0, 0, 0, 0};
  fill_q(0, stage);
  if (KK0 > 1) fill_q(1, stage + BB);
#pragma unroll
  for (int kk = 0; kk < KK0; ++kk) {
    T* buf = stage + (kk & 1) * BB;
    if (kk + 1 < KK0) wait_vm<LPW>();
    else wait_vm<0>();
    T x[M1];
#pragma unroll
    for (int t4 = 0; t4 < M1 / 4; ++t4) {
      const V4 v = *reinterpret_cast<const V4*>(buf + c * PT + g * M1 + 4 * t4);
#pragma unroll
      for (int e = 0; e < 4; ++e) x[4 * t4 + e] = v[e];
    }
    wait_lds();
    if (kk + 2 < KK0) fill_q(kk + 2, buf);
    step0_quarter<T, MODE, K>(o0[kk], y, x, shift);
  }
  reg_steps_from<T, MODE, K, 1, true>(y, d, c, g);
  if (g == 0) {
#pragma unroll
    for (int t = 0; t < M1; ++t) *reinterpret_cast<V4*>(stage + c * PT + 4 * t) = y[t];
  }
  wait_lds();
  T* dst = static_cast<T*>(d.out) + tile * 16 * ROUT;
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int v = it * 64 + lane, i = v / VQ, j = 4 * (v - i * VQ);
    const V4 val = *reinterpret_cast<const V4*>(stage + i * PT + j);
    *reinterpret_cast<V4*>(dst + i * ROUT + j) = val;
#pragma unroll
    for (int r = 0; r < 4; ++r) track(static_cast<T>(val[r]), mx, bad);
  }
}

// FORM_BOTTOM streamed over tiles, for the longest chunks (4 rows of 4-byte
// entries, 3 rows of 8-byte ones): their accumulators leave one or two
// wavefronts per SIMD, so in the one-tile form a wavefront's loads wait for
// its own matrix work and the reverse.  Here a wavefront takes tiles b,
// b + G, b + 2G, ... of one unit (G wavefronts, as many as fit on the CUs).
// Once step 0 has read the last quarter of a tile's slice, the first two
// quarters of its next tile are filled into the two stage buffers; they
// arrive during the register-only steps 1..k-1 and the stores.  Step 0's
// operands and the scale are loaded once; those of steps 1..k-1 are loaded
// while the last quarter is in flight and first used after the wait for it
// (the compiler's own wait for a register load issued among stage fills
// waits for every fill).  The outputs leave through a third, small buffer, a
// quarter of each fibre at a time.  Waits: at quarter 0 at most LPW
// operations may be outstanding (the fills of quarter 1, then the previous
// tile's stores), at quarter 1 LPW + NST after a previous tile (its stores
// and the fills of quarter 2), else as in the one-tile form.
template <typename T, int K>
constexpr int stream_out_pitch() { return (1 << (2 * (K - 1))) + static_cast<int>(16 / sizeof(T)); }

// Eight 16-byte LDS reads at p + 16 i into v[i] (as lds_read16 below).
typedef __attribute__((address_space(3))) const void* LdsCPtr;
__device__ inline void lds_read8(const void* p, f32x4 (&v)[8]) {
#if __HIP_DEVICE_COMPILE__
  asm volatile(
      "ds_read_b128 %0, %8\n\t"
      "ds_read_b128 %1, %8 offset:16\n\t"
      "ds_read_b128 %2, %8 offset:32\n\t"
      "ds_read_b128 %3, %8 offset:48\n\t"
      "ds_read_b128 %4, %8 offset:64\n\t"
      "ds_read_b128 %5, %8 offset:80\n\t"
      "ds_read_b128 %6, %8 offset:96\n\t"
      "ds_read_b128 %7, %8 offset:112\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4]), "=&v"(v[5]),
        "=&v"(v[6]), "=&v"(v[7])
      : "v"((LdsCPtr)p)
      : "memory");
#else
  (void)p;
  for (int i = 0; i < 8; ++i) v[i] = f32x4{};
#endif
}

// Sixteen 16-byte LDS reads at p + 16 i into v[i], in one asm block that waits
// for its own results.  The compiler does not count it as an LDS load, so it
// adds no wait for the stage fills in flight (it cannot tell which buffer a
// fill targets and would wait for all of them).
__device__ inline void lds_read16(const void* p, f32x4 (&v)[16]) {
#if __HIP_DEVICE_COMPILE__
  asm volatile(
      "ds_read_b128 %0, %16\n\t"
      "ds_read_b128 %1, %16 offset:16\n\t"
      "ds_read_b128 %2, %16 offset:32\n\t"
      "ds_read_b128 %3, %16 offset:48\n\t"
      "ds_read_b128 %4, %16 offset:64\n\t"
      "ds_read_b128 %5, %16 offset:80\n\t"
      "ds_read_b128 %6, %16 offset:96\n\t"
      "ds_read_b128 %7, %16 offset:112\n\t"
      "ds_read_b128 %8, %16 offset:128\n\t"
      "ds_read_b128 %9, %16 offset:144\n\t"
      "ds_read_b128 %10, %16 offset:160\n\t"
      "ds_read_b128 %11, %16 offset:176\n\t"
      "ds_read_b128 %12, %16 offset:192\n\t"
      "ds_read_b128 %13, %16 offset:208\n\t"
      "ds_read_b128 %14, %16 offset:224\n\t"
      "ds_read_b128 %15, %16 offset:240\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4]), "=&v"(v[5]),
        "=&v"(v[6]), "=&v"(v[7]), "=&v"(v[8]), "=&v"(v[9]), "=&v"(v[10]), "=&v"(v[11]),
        "=&v"(v[12]), "=&v"(v[13]), "=&v"(v[14]), "=&v"(v[15])
      : "v"((LdsCPtr)p)
      : "memory");
#else
  (void)p;
  for (int i = 0; i < 16; ++i) v[i] = f32x4{};
#endif
}

template <typename T, int MODE, int K>
__global__ __launch_bounds__(64) void absorb_chunk_reg_stream(chunk::Group arg) {
  (void)arg;   // read in place below
  static_assert((sizeof(T) == 4 && K == 4) || (sizeof(T) == 8 && K == 3),
                "4-row chunks of 4-byte entries or 3-row chunks of 8-byte ones");
  using V4 = RV4<MODE>;
  constexpr int M1 = 1 << (2 * (K - 1)), QR = quarter_rows<K>();
  constexpr int RIN = 4 * QR, ROUT = 4 * M1, ES = sizeof(T);
  constexpr int PT = bottom_pitch<T, K>(), BB = 16 * PT, OPT = stream_out_pitch<T, K>();
  constexpr int FB = QR * ES;                 // bytes of one fibre's quarter
  constexpr int LANES = FB >= 1024 ? 64 : FB / 16;   // active lanes of a fill
  constexpr int LPW = 16;                     // fills per quarter (one per fibre)
  constexpr int NR = M1 * ES / 16;            // 16-byte LDS reads per lane and quarter
  constexpr int TQ = M1 / 4;                  // tiles t per output quarter
  constexpr int NIT = M1 / 16;                // stores per lane and output quarter
  constexpr int NST = 4 * NIT;                // stores per tile
  static_assert(FB <= 1024 && (NR == 16 || NR == 8) && LPW + NST < 64, "shapes");
  __shared__ __attribute__((aligned(16))) T stage[2 * BB];
  __shared__ __attribute__((aligned(16))) T ostage[16 * OPT];
  const GroupRef g = (GroupRef)__builtin_amdgcn_kernarg_segment_ptr();
  UnitRef d = g->u[0];
  const uint32_t ntiles = g->first[chunk::kGroup], G = gridDim.x;
  uint32_t t = blockIdx.x;
  if (t >= ntiles) return;
  const int lane = threadIdx.x & 63, c = lane & 15, gl = lane >> 4;
  auto fill_q = [&](const char* src, int kk, T* buf) {
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (lane < LANES) lds_fill16(src + (i * RIN + kk * QR) * ES + 16 * lane, buf + i * PT);
  };
  auto src_of = [&](uint32_t tt) {
    return static_cast<const char*>(d.in) + static_cast<int64_t>(tt) * 16 * RIN * ES;
  };
  ROps<T, MODE> o0[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) o0[kk] = reg_ops<T, MODE, true, 0>(d.S[0], d.hi[0], d.lo[0], c, gl, kk);
  const int32_t shift = shift_of(d.scale_slot);
  wait_vm<0>();
  const char* src = src_of(t);
  fill_q(src, 0, stage);
  fill_q(src, 1, stage + BB);
  T mx = 0;
  int bad = 0;
  for (bool first = true;; first = false) {
    const uint32_t next = t + G;
    const bool more = next < ntiles;
    V4 y[M1];
#pragma unroll
    for (int q = 0; q < M1; ++q) y[q] = V4{0, 0, 0, 0};
    RawOps<T, MODE> r1, r2, r3;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      T* buf = stage + (kk & 1) * BB;
      if (kk == 0) wait_vm<LPW>();
      else if (kk == 1) {
        if (first) wait_vm<LPW>();
        else wait_vm<LPW + NST>();
      } else if (kk == 2) wait_vm<LPW>();
      else wait_vm<0>();
      T x[M1];
      {
        f32x4 v[NR];
        if constexpr (NR == 16) lds_read16(buf + c * PT + gl * M1, v);
        else lds_read8(buf + c * PT + gl * M1, v);
        constexpr int PER = 16 / ES;   // entries per 16-byte read
#pragma unroll
        for (int i = 0; i < NR; ++i) {
          typedef T TV __attribute__((ext_vector_type(PER)));
          const TV tv = __builtin_bit_cast(TV, v[i]);
#pragma unroll
          for (int e = 0; e < PER; ++e) x[PER * i + e] = tv[e];
        }
      }
      if (kk < 2) fill_q(src, kk + 2, buf);
      if (kk == 2) {
        r1 = reg_ops_load<T, MODE, false, 0>(d.S[1], d.hi[1], d.lo[1], c, gl);
        if constexpr (K == 4) {
          r2 = reg_ops_load<T, MODE, false, 0>(d.S[2], d.hi[2], d.lo[2], c, gl);
          r3 = reg_ops_load<T, MODE, false, 2>(d.S[3], d.hi[3], d.lo[3], c, gl);
        } else {
          r2 = reg_ops_load<T, MODE, false, 2>(d.S[2], d.hi[2], d.lo[2], c, gl);
        }
      }
      if (kk == 3) {
        launder<T, MODE, false>(r1);
        launder<T, MODE, false>(r2);
        if constexpr (K == 4) launder<T, MODE, false>(r3);
        // issued on every path (after the last tile they re-read its first
        // two quarters, from L2) so that no compiler wait depends on the path
        if (more) src = src_of(next);
        fill_q(src, 0, stage);
        fill_q(src, 1, stage + BB);
      }
      step0_quarter<T, MODE, K>(o0[kk], y, x, shift);
    }
    reg_step<T, MODE, K, 1>(y, reg_ops_build<T, MODE, false>(r1));
    reg_step<T, MODE, K, 2>(y, reg_ops_build<T, MODE, false>(r2));
    if constexpr (K == 4) reg_step<T, MODE, K, 3>(y, reg_ops_build<T, MODE, false>(r3));
    // outputs: fibre i's row j = 4 t + r at i * ROUT + j; output quarter qo
    // holds t in [qo TQ, (qo + 1) TQ), M1 entries of each fibre
    T* dst = static_cast<T*>(d.out) + static_cast<int64_t>(t) * 16 * ROUT;
#pragma unroll
    for (int qo = 0; qo < 4; ++qo) {
      if (gl == 0) {
#pragma unroll
        for (int tt = 0; tt < TQ; ++tt) *reinterpret_cast<V4*>(ostage + c * OPT + 4 * tt) = y[qo * TQ + tt];
      }
      wait_lds();
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int v = it * 64 + lane, i = v / TQ, j = 4 * (v - i * TQ);
        const V4 val = *reinterpret_cast<const V4*>(ostage + i * OPT + j);
        *reinterpret_cast<V4*>(dst + i * ROUT + qo * M1 + j) = val;
#pragma unroll
        for (int r = 0; r < 4; ++r) track(static_cast<T>(val[r]), mx, bad);
      }
      wait_lds();
    }
    if (!more) break;
    t = next;
  }
  wait_vm<0>();   // no fill may land in LDS after the workgroup ends
  if (d.max_slot) publish_wave(mx, bad, d.max_slot, g->flags);
}

template <typename T, int MODE, int K, bool TOP, int FORM>
__global__ __launch_bounds__(FORM == FORM_PAIR ? 128 : 64) void absorb_chunk_reg(chunk::Group arg) {
  (void)arg;   // read in place below
  constexpr int NWG = FORM == FORM_PAIR ? 2 : 1;   // tiles (wavefronts) per workgroup
  __shared__ __attribute__((aligned(16))) T stage[stage_entries<T, K, FORM>()];
  const GroupRef g = (GroupRef)__builtin_amdgcn_kernarg_segment_ptr();
  // consecutive workgroups' tiles on one XCD (workgroup b runs on XCD b % 8)
  const uint32_t nb = gridDim.x;
  const uint32_t b = (nb % 8 == 0) ? (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8 : blockIdx.x;
  const uint32_t t = b * NWG;   // first tile of the workgroup; units hold whole workgroups
  if (t >= g->first[chunk::kGroup]) return;
  const int ui = chunk::unit_index(g, t);
  UnitRef d = g->u[ui];
  const int64_t tile = t - g->first[ui];
  T mx = 0;
  int bad = 0;
  if constexpr (FORM == FORM_DIRECT) tile_direct<T, MODE, K, TOP>(d, tile, mx, bad);
  else if constexpr (FORM == FORM_PAIR) tile_pair<T, MODE, K, TOP>(d, tile, mx, bad, stage);
  else tile_bottom<T, MODE, K, TOP>(d, tile, mx, bad, stage);
  if (d.max_slot) publish_wave(mx, bad, d.max_slot, g->flags);
}

int form_of(const ChunkArgs& a) {
  if (a.post == 1) return FORM_BOTTOM;
  return (a.type != EL_F64 && a.post % 32 == 0) ? FORM_PAIR : FORM_DIRECT;
}

int32_t g_chunk_stream = 1;   // TN_OPT_CHUNK_STREAM: 0 off, 1 as many as fit, n >= 2 at most n

// Compute units of the current device (cached per device).
uint32_t cu_count() {
  static std::atomic<int32_t> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 256;
  if (dev < 64) {
    const int32_t v = cache[dev].load(std::memory_order_relaxed);
    if (v > 0) return static_cast<uint32_t>(v);
  }
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
    n = 256;
  if (dev < 64) cache[dev].store(n, std::memory_order_relaxed);
  return static_cast<uint32_t>(n);
}

template <typename T, int MODE, int K, bool TOP>
hipError_t go_reg(const chunk::Group& grp, int form, hipStream_t stream, bool* streamed) {
  const uint32_t tiles = grp.first[chunk::kGroup];
  if (tiles == 0) return hipSuccess;
  if constexpr (!TOP && ((K == 4 && sizeof(T) == 4) || (K == 3 && sizeof(T) == 8))) {
    if (form == FORM_BOTTOM && g_chunk_stream && grp.n == 1) {
      *streamed = true;
      // one-wavefront workgroups, as many per CU as the registers allow (one
      // per SIMD with 4-byte entries, two with 8-byte ones), each over
      // tiles / G tiles; or at most the number the option names
      constexpr uint32_t kPerCU = sizeof(T) == 4 ? 4 : 8;
      const uint32_t cap = g_chunk_stream == 1 ? kPerCU * cu_count() : static_cast<uint32_t>(g_chunk_stream);
      const uint32_t grid = std::min(tiles, cap);
      hipLaunchKernelGGL((absorb_chunk_reg_stream<T, MODE, K>), dim3(grid), dim3(64), 0, stream,
                         grp);
      return hipGetLastError();
    }
  }
  if (form == FORM_BOTTOM) {
    hipLaunchKernelGGL((absorb_chunk_reg<T, MODE, K, TOP, FORM_BOTTOM>), dim3(tiles), dim3(64),
                       0, stream, grp);
  } else if (form == FORM_PAIR) {
    if constexpr (sizeof(T) == 4) {
      hipLaunchKernelGGL((absorb_chunk_reg<T, MODE, K, TOP, FORM_PAIR>), dim3(tiles / 2),
                         dim3(128), 0, stream, grp);
    } else {
      return hipErrorInvalidValue;
    }
  } else {
    hipLaunchKernelGGL((absorb_chunk_reg<T, MODE, K, TOP, FORM_DIRECT>), dim3(tiles), dim3(64),
                       0, stream, grp);
  }
  return hipGetLastError();
}

template <typename T, int MODE>
hipError_t go_reg_k(const chunk::Group& grp, int k, bool top, int form, hipStream_t stream,
                    bool* streamed) {
  if (k == 2) return top ? go_reg<T, MODE, 2, true>(grp, form, stream, streamed)
                         : go_reg<T, MODE, 2, false>(grp, form, stream, streamed);
  if (k == 3) return top ? go_reg<T, MODE, 3, true>(grp, form, stream, streamed)
                         : go_reg<T, MODE, 3, false>(grp, form, stream, streamed);
  if constexpr (MODE != M_F64) {
    if (k == 4) return top ? go_reg<T, MODE, 4, true>(grp, form, stream, streamed)
                           : go_reg<T, MODE, 4, false>(grp, form, stream, streamed);
  }
  return hipErrorInvalidValue;
}

}  // namespace

void set_chunk_stream(int32_t v) { g_chunk_stream = v; }

int32_t chunk_reg_max_steps(int32_t type) { return type == EL_F64 ? 3 : 4; }

bool chunk_reg_shape_ok(int32_t type, int64_t pre, int64_t post, int32_t k, int32_t k1,
                        int32_t nl) {
  if (k < 2 || k > chunk_reg_max_steps(type) || (k1 != 4 && k1 != 16)) return false;
  if (pre < 1 || post < 1 || pre > INT_MAX / post) return false;
  if (post == 1) return nl == 4 && pre % 16 == 0;
  // per-lane byte offsets within a slice are 32-bit
  const int64_t es = type == EL_F64 ? 8 : 4;
  const int64_t span = static_cast<int64_t>(16) << (2 * (k - 1));   // rows of a slice, N = 16
  if (span * post * es >= (int64_t(1) << 31)) return false;
  return nl == 16 && post % 16 == 0;
}

hipError_t launch_absorb_chunks_reg(const ChunkArgs* a, int32_t n, const StagedArrays& st,
                                    DevState* state, hipStream_t stream, const char** kname) {
  if (n < 1 || n > chunk::kGroup) return hipErrorInvalidValue;
  const bool f64 = a[0].type == EL_F64, bf = !f64 && a[0].arith == AR_BF16X3;
  *kname = f64 ? "absorb_chunk_reg_f64" : bf ? "absorb_chunk_reg_bf16x3" : "absorb_chunk_reg_f32";
  bool done[chunk::kGroup] = {false, false, false, false};
  bool streamed = false;
  // one launch per (rows, top edge, tile form) among the units
  for (int32_t u = 0; u < n; ++u) {
    if (done[u]) continue;
    if (a[u].type != a[0].type || a[u].arith != a[0].arith ||
        !chunk_reg_shape_ok(a[u].type, a[u].pre, a[u].post, a[u].k, a[u].k1, a[u].nl))
      return hipErrorInvalidValue;
    const bool top = a[u].k1 == 4;
    const int form = form_of(a[u]);
    ChunkArgs sel[chunk::kGroup];
    int32_t ns = 0;
    for (int32_t v = u; v < n; ++v)
      if (!done[v] && a[v].k == a[u].k && (a[v].k1 == 4) == top && form_of(a[v]) == form &&
          a[v].type == a[u].type && a[v].arith == a[u].arith &&
          chunk_reg_shape_ok(a[v].type, a[v].pre, a[v].post, a[v].k, a[v].k1, a[v].nl)) {
        sel[ns++] = a[v];
        done[v] = true;
      }
    chunk::Group grp;
    if (!chunk::fill_group(grp, sel, ns, st, &state->flags, f64)) return hipErrorInvalidValue;
    const hipError_t e = f64  ? go_reg_k<double, M_F64>(grp, a[u].k, top, form, stream, &streamed)
                         : bf ? go_reg_k<float, M_BF16X3>(grp, a[u].k, top, form, stream, &streamed)
                              : go_reg_k<float, M_F32>(grp, a[u].k, top, form, stream, &streamed);
    if (e != hipSuccess) return e;
  }
  if (streamed)
    *kname = f64 ? "absorb_chunk_reg_stream_f64"
                 : bf ? "absorb_chunk_reg_stream_bf16x3" : "absorb_chunk_reg_stream_f32";
  return hipSuccess;
}

}  // namespace tn
