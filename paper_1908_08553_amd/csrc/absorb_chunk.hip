// Column-chunk absorption: k consecutive rows (2 <= k <= 4) of one column of a
// sweep applied to a slice of the boundary held in LDS, so the boundary makes
// one HBM round trip per chunk instead of one per step (paper §4: the
// pairwise, sequential contraction; only the memory schedule changes).
//
// Slice.  Before the chunk the boundary is [p][K1 legs][h_{i+1} .. h_{i+k-1}]
// [q] (p = prefix of the first step, q = suffix of the last one).  A workgroup
// takes SP "spectator" fibres s = (p, q), SP * sizeof(T) = 128 bytes: SP
// consecutive q of one p when the suffix has at least SP entries, else SP /
// post consecutive p with all their q.  For those spectators the chunk only
// touches the rows
//     row = (prefix * 16 + kidx) * M + m
// (prefix = new h' legs so far, kidx = (v, h) = the step's K index, m = the
// h legs still to absorb, M = 4^(rows left after this one)): the natural
// linear order of the slice.  Step j reads, for each (prefix, m), the 16 rows
// kidx = 0..15 and writes its 16 outputs n = (h', v') to the same 16 rows, so
// the slice is updated in place: one LDS buffer of 16 * 4^(k-1) rows x SP.
//
// Products.  D[n][s] = sum_k S[k][n] X[k][s] on 16x16 MFMA tiles: A = the
// (zero-padded) site matrix transposed, B = 16 spectators of the 16 rows.
// Edge rows: a first step with K = 4 (top edge) reads only kidx < 4 and its
// site matrix is padded with zero rows; a last step with N = 4 (bottom edge)
// writes n = 4 n' (zero columns elsewhere) and only those rows are stored.
// The padded matrices of the chunk's steps are staged in LDS once per unit.
//
// Schedule: see Cfg.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>

#include "absorb_device.hpp"
#include "chunk_group.hpp"
#include "kernels.hpp"

namespace tn {
namespace {

using namespace dev;

constexpr int kChunkGroup = chunk::kGroup;
typedef chunk::Group ChunkGroup;
using chunk::GroupRef;
using chunk::UnitRef;

// Launch shape: SP spectators per tile, at most KM rows per chunk, NW waves
// per workgroup; one workgroup per tile, two or more resident per CU (float:
// 64 KiB slices of 64-byte row runs; tiles spread over the XCDs in contiguous
// runs so both halves of a 128-byte line go through one L2).
template <typename T>
struct Cfg;
template <>
struct Cfg<float> {
  static constexpr int SP = 16, KM = 4, NW = 8;
};
template <>
struct Cfg<double> {
  static constexpr int SP = 16, KM = 3, NW = 8;
};

// XOR of the base-4 digits of x (x < 2^16), two bits.
__host__ __device__ constexpr int dx4(int x) {
  x ^= x >> 8;
  x ^= x >> 4;
  x ^= x >> 2;
  return x & 3;
}

// LDS placement.  Slice row r, spectator s = 16 h + c; with the swizzle digit
// d = (r & 3) ^ dx4(r >> 2) = 2 d1 + d0,
//     word = (r & ~3) * SP + (G(d) ^ 16 h) + c,
// G(d) = 16 d (SP = 16) or 80 d0 + 32 d1 (SP = 32).  Word bit 4 (the 16-bank
// half of a 32-bank cycle) carries d0, bits 4-5 (the 16-bank quarter of 64
// banks) carry (d0, d1): MFMA operand reads and result writes, whose four
// lane groups address rows that differ in one base-4 digit (the low bit of
// that digit between the two groups of a half-wave), never share a bank.  G
// is XOR-linear in d.
template <int SP>
__host__ __device__ constexpr int gsw(int d) {
  return SP == 16 ? (d << 4) : (((d & 1) ? 80 : 0) | ((d & 2) << 4));
}
template <int SP>
__device__ inline int word_of(int row, int s) {
  const int d = (row & 3) ^ dx4(row >> 2);
  return (row & ~3) * SP + (gsw<SP>(d) ^ (s & 16)) + (s & 15);
}

// In the step loops a row is base + koff with base (tile) and koff = kidx *
// 4^(jsh/2) (kidx = K or N index < 16) in disjoint base-4 digits, so
//     word = TB + H(kidx) + (LX ^ G(X(kidx)))
// with TB = (base & ~3) * SP + c and LX = G(dx of base) ^ 16 h per tile,
// H(kidx) = (jsh ? kidx : kidx & ~3) << (jsh + log2 SP) and X(kidx) =
// (kidx & 3) ^ (kidx >> 2).  The lane-dependent parts of kidx go into
// per-lane bases, the rest into uniform terms and XOR immediates.
template <int SP>
__device__ inline void tile_of(int grp, int h, int jsh, int c, int& tb, int& lx) {
  const int base = ((grp >> jsh) << (jsh + 4)) + (grp & ((1 << jsh) - 1));
  tb = (base & ~3) * SP + c;
  lx = gsw<SP>((base & 3) ^ dx4(base >> 2)) ^ (h << 4);
}

template <typename T>
__device__ inline T scale(T x, int32_t shift) {
  return shift ? static_cast<T>(ldexp(x, -shift)) : x;
}

// Site operands of one step, from the padded matrices staged in LDS.
//   f32/f64: lane (c, g) holds A[c][g] = S[4kk + g][c] for kk = 0..3
//   bf16x3:  lane (c, g) holds S[2t + (g & 1)][c], t = 0..7 (high parts for
//            g < 2 and low parts for g >= 2 in the first product; high parts
//            and zeros in the second)
template <typename T, int MODE>
struct SiteOps {
  T a[4];
  bf16x8 a0, a1;
};

template <typename T, int MODE>
__device__ inline SiteOps<T, MODE> site_ops(const T* sS, const uint16_t* sH, const uint16_t* sL,
                                            int c, int gg) {
  SiteOps<T, MODE> o;
  if constexpr (MODE == M_BF16X3) {
    const uint16_t zero = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = (2 * t + (gg & 1)) * 16 + c;
      const uint16_t hb = sH[e], lb = sL[e];
      o.a0[t] = __builtin_bit_cast(__bf16, gg < 2 ? hb : lb);
      o.a1[t] = __builtin_bit_cast(__bf16, gg < 2 ? hb : zero);
    }
  } else {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) o.a[kk] = sS[(4 * kk + gg) * 16 + c];
  }
  return o;
}

// Slice row of the first (kidx = 0) row of group `grp` at base-4 shift JSH:
// the group index is (prefix, m); the K/N index sits between them.  A bit
// permutation of grp.
__host__ __device__ constexpr int base_of(int grp, int jsh) {
  return ((grp >> jsh) << (jsh + 4)) + (grp & ((1 << jsh) - 1));
}

// Step J of a K-row chunk on every 16-spectator tile of the slice.  Wave w
// takes tiles w + i NW (i = 0, 1, ...): group g0 + i GS (g0 = w / HS, GS =
// NW / HS, a power of two > g0) and half h = w % HS.  Group indices g0 and
// i GS occupy disjoint bits, base_of permutes bits, and both the row offset
// and the swizzle digit are XOR-linear over disjoint bits, so tile i differs
// from tile 0 by compile-time constants: a row offset T_i (in the immediate
// offset of the LDS instruction) and an XOR term L_i.  Lane (c, g):
//   reads f32/f64: kidx = 4kk + g;  bf16: kidx = 2t + (g & 1)
//   writes f32/bf16: kidx = 4g + r;  f64: kidx = g + 4r
// The word offset of (row base + kidx * 4^(JSH/2), spectator 16h + c) is
//     TB + H(kidx) + (LX ^ G(X(kidx)))
// (see tile_of) with H(kidx) = (JSH ? kidx : kidx & ~3) << (JSH + log2 SP)
// split into per-lane terms and constants.
// TOP: first step of a top-edge chunk (only kidx < 4 carries data).
template <typename T, int MODE, int SP, int NW, int K, int J, bool TOP, int NBM>
__device__ inline void step_kj(T* lds, const SiteOps<T, MODE>& o, int c, int gg, int w) {
  using V4 = typename std::conditional<MODE == M_F64, f64x4, f32x4>::type;
  constexpr int JSH = 2 * (K - 1 - J), LS = SP == 16 ? 4 : 5, HS = SP / 16, JB = JSH + LS;
  constexpr int NTILE = (1 << (2 * (K - 1))) * HS;   // tiles of the step
  constexpr int GS = NW / HS;
  constexpr int NTW = NTILE >= NW ? NTILE / NW : 1;  // tiles per wave
  static_assert(NTILE < NW || NTILE % NW == 0, "tiles spread evenly over the waves");
  if (NTILE < NW && w >= NTILE) return;
  const int g0 = w / HS, h = w % HS;
  const int base0 = base_of(g0, JSH);
  const int tb = (base0 & ~3) * SP + c;
  const int lx = gsw<SP>((base0 & 3) ^ dx4(base0 >> 2)) ^ (h << 4);
  // per-lane parts of H and of the XOR term
  const int rb = tb + ((MODE == M_BF16X3) ? (JSH ? (gg & 1) << JB : 0) : (JSH ? gg << JB : 0));
  const int wb = tb + ((MODE == M_F64) ? (JSH ? gg << JB : 0) : (JSH ? gg << (JB + 2) : gg << (LS + 2)));
  const int lr = lx ^ ((MODE == M_BF16X3) ? gsw<SP>(gg & 1) : gsw<SP>(gg));
  const int lw = lx ^ gsw<SP>(gg);
  constexpr int NB = NTW < NBM ? NTW : NBM;   // tiles in flight
  static_assert(NTW % NB == 0, "whole batches");
#pragma unroll
  for (int bb = 0; bb < NTW; bb += NB) {
    V4 acc[NB];
    if constexpr (MODE == M_BF16X3) {
      const __bf16 zero = __builtin_bit_cast(__bf16, static_cast<uint16_t>(0));
      bf16x8 b0[NB], b1[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int bi = base_of((bb + i) * GS, JSH);
        const int ti = bi * SP, li = gsw<SP>(dx4(bi >> 2));
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          if (TOP && t >= 2) {
            b0[i][t] = zero;
            b1[i][t] = zero;
            continue;
          }
          const int ht = JSH ? ((2 * t) << JB) : ((t >> 1) << (LS + 2));
          const float x = lds[rb + ti + ht + (lr ^ (li ^ gsw<SP>((2 * (t & 1)) ^ (t >> 1))))];
          const __bf16 hi = static_cast<__bf16>(x);
          b0[i][t] = hi;
          b1[i][t] = gg < 2 ? static_cast<__bf16>(x - static_cast<float>(hi)) : zero;
        }
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.a0, b0[i], acc[i], 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < NB; ++i)
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.a1, b1[i], acc[i], 0, 0, 0);
    } else {
      constexpr int KK = TOP ? 1 : 4;
      T b[NB][KK];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int bi = base_of((bb + i) * GS, JSH);
        const int ti = bi * SP, li = gsw<SP>(dx4(bi >> 2));
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
          const int ht = JSH ? (kk << (JB + 2)) : (kk << (LS + 2));
          b[i][kk] = lds[rb + ti + ht + (lr ^ (li ^ gsw<SP>(kk)))];
        }
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) acc[i] = V4{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < KK; ++kk)
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          if constexpr (MODE == M_F64)
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(o.a[kk], b[i][kk], acc[i], 0, 0, 0);
          else
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.a[kk], b[i][kk], acc[i], 0, 0, 0);
        }
    }
    // register r of lane (c, g) holds D[n][c], n = 4g + r (f32 and bf16
    // results) or n = g + 4r (f64)
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int bi = base_of((bb + i) * GS, JSH);
      const int ti = bi * SP, li = gsw<SP>(dx4(bi >> 2));
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ht = (MODE == M_F64) ? (JSH ? (r << (JB + 2)) : (r << (LS + 2))) : (JSH ? (r << JB) : 0);
        lds[wb + ti + ht + (lw ^ (li ^ gsw<SP>(r)))] = acc[i][r];
      }
    }
  }
}

// All K steps of a K-row chunk (barrier after each).
template <typename T, int MODE, int SP, int NW, int K, int NBM>
__device__ inline void chunk_steps(T* lds, const T* sS, const uint16_t* sH, const uint16_t* sL,
                                   bool top, int c, int gg, int w) {
  {
    const SiteOps<T, MODE> o = site_ops<T, MODE>(sS, sH, sL, c, gg);
    if (top) step_kj<T, MODE, SP, NW, K, 0, true, NBM>(lds, o, c, gg, w);
    else step_kj<T, MODE, SP, NW, K, 0, false, NBM>(lds, o, c, gg, w);
    __syncthreads();
  }
  {
    const SiteOps<T, MODE> o = site_ops<T, MODE>(sS + 256, sH + 256, sL + 256, c, gg);
    step_kj<T, MODE, SP, NW, K, 1, false, NBM>(lds, o, c, gg, w);
    __syncthreads();
  }
  if constexpr (K >= 3) {
    const SiteOps<T, MODE> o = site_ops<T, MODE>(sS + 512, sH + 512, sL + 512, c, gg);
    step_kj<T, MODE, SP, NW, K, 2, false, NBM>(lds, o, c, gg, w);
    __syncthreads();
  }
  if constexpr (K >= 4) {
    const SiteOps<T, MODE> o = site_ops<T, MODE>(sS + 768, sH + 768, sL + 768, c, gg);
    step_kj<T, MODE, SP, NW, K, 3, false, NBM>(lds, o, c, gg, w);
    __syncthreads();
  }
}

// Geometry of one tile (SP spectators of one unit).
struct Tile {
  int64_t p0, q0;
  int ui;
  int rows_in, rows_out, qn;
  int qrun;   // no padding bytes: they would become a private array
  int pad;
};

template <int SP>
__device__ inline Tile tile_at(GroupRef g, uint32_t t) {
  Tile x;
  const int ui = chunk::unit_index(g, t);
  UnitRef d = g->u[ui];
  const int64_t tile = t - g->first[ui];
  x.ui = ui;
  const int M1 = 1 << (2 * (d.k - 1));
  x.rows_in = d.k1 * M1;
  x.rows_out = d.nl * M1;
  x.qrun = d.post >= SP ? 1 : 0;
  x.qn = x.qrun ? SP : static_cast<int>(d.post);
  if (x.qrun) {
    const int64_t tq = d.post / SP;
    x.p0 = tile / tq;
    x.q0 = (tile - x.p0 * tq) * SP;
  } else {
    x.p0 = tile * (SP / x.qn);
    x.q0 = 0;
  }
  x.pad = 0;
  return x;
}

// Global <-> LDS traffic of a slice of `rows` rows.  Vector (4 entries)
// index f = it * NTH + tid.
//  * Row runs (q-run, or whole suffixes of 4..SP/2 entries): f -> (row, 4
//    spectators s..s+3), 4 consecutive entries in global memory and in LDS.
//    Rows are visited in the order 0, 2, 1, 3 within each group of four, so
//    the two rows of a 16-lane LDS cycle sit in different bank halves.
//  * Whole suffixes of 1 entry (the tile is SP consecutive p): f -> (4 rows,
//    4 spectators); four 4-row loads transposed in registers into four rows
//    of 4 spectators.
// Iteration it adds a multiple of 4 rows that shares no bits with the
// thread's own row, so its LDS word is the thread's word plus a compile-time
// offset, with a compile-time XOR of the swizzle (word_of is XOR-linear over
// disjoint bits); see run_lds / blk_lds.
__host__ __device__ constexpr int swap01(int r) { return (r & ~3) | ((r & 1) << 1) | ((r >> 1) & 1); }

template <int SP, int NTH>
struct RunPos {
  static constexpr int PR = SP / 4, RS = NTH / PR;   // vectors per row; rows per iteration
  static_assert(RS % 4 == 0, "iterations move whole row quads");
  int row0, s0, bw, x0;   // first row and spectator; LDS word = bw + (x0 ^ X(it)) + it RS SP
  __device__ explicit RunPos(int tid) {
    row0 = swap01(tid / PR);
    s0 = 4 * (tid % PR);
    const int d = (row0 & 3) ^ dx4(row0 >> 2);
    bw = (row0 & ~3) * SP + (s0 & 15);
    x0 = gsw<SP>(d) ^ (s0 & 16);
  }
  __device__ int lds(int it) const { return bw + it * RS * SP + (x0 ^ gsw<SP>(dx4((it * RS) >> 2))); }
};

template <int SP, int NTH>
struct BlkPos {
  static constexpr int PB = SP / 4, RB = 4 * (NTH / PB);   // blocks per row quad; rows per iteration
  int row4, s0, bw, x0;   // LDS word of row row4 + it RB + u: bw + it RB SP + (x0 ^ G(u) ^ X(it))
  __device__ explicit BlkPos(int tid) {
    row4 = 4 * swap01(tid / PB);
    s0 = 4 * (tid % PB);
    bw = row4 * SP + (s0 & 15);
    x0 = gsw<SP>(dx4(row4 >> 2)) ^ (s0 & 16);
  }
  __device__ int lds(int it, int u, int lsh) const {
    // the store of a bottom-edge chunk reads rows (row4 + it RB + u) << 2
    if (lsh == 0) return bw + it * RB * SP + ((x0 ^ gsw<SP>(u)) ^ gsw<SP>(dx4((it * RB) >> 2)));
    return word_of<SP>((row4 + it * RB + u) << lsh, s0);
  }
};

// Global element offset (from the tile's base) of (row, spectator s) on the
// row-run path.
__device__ inline int64_t run_off(const Tile& x, int64_t post, int rows, int row, int s) {
  if (x.qrun) return static_cast<int64_t>(row) * post + s;
  const int pl = s / x.qn, q = s - pl * x.qn;   // whole suffixes: [p_local][row][q]
  return (static_cast<int64_t>(pl) * rows + row) * x.qn + q;
}

template <int IT>
struct Regs {
  static constexpr int N = IT < 4 ? 4 : IT;
  static constexpr int NB = (IT + 3) / 4;   // 4x4 blocks per thread
};

// Issue the global loads of a tile's input slice into v (no wait).
template <typename T, typename V4, int SP, int NTH, int IT>
__device__ inline void slice_load(UnitRef d, const Tile& x, V4* v) {
  const int tid = threadIdx.x;
  const T* src = static_cast<const T*>(d.in) + x.p0 * x.rows_in * d.post + x.q0;
  if (x.qn >= 4) {
    using P = RunPos<SP, NTH>;
    const P ps(tid);
    const int total = x.rows_in * SP / 4;
    const T* g0 = src + run_off(x, d.post, x.rows_in, ps.row0, ps.s0);
    const int64_t step = static_cast<int64_t>(P::RS) * (x.qrun ? d.post : x.qn);
#pragma unroll
    for (int it = 0; it < Regs<IT>::N; ++it)   // slots past IT are never in range
      if (it * NTH + tid < total) v[it] = *reinterpret_cast<const V4*>(g0 + it * step);
  } else {
    using P = BlkPos<SP, NTH>;
    const P ps(tid);
    const int total = x.rows_in * SP / 16;
    const T* g0 = src + static_cast<int64_t>(ps.s0) * x.rows_in + ps.row4;
#pragma unroll
    for (int it = 0; it < Regs<IT>::NB; ++it)
      if (it * NTH + tid < total) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          v[4 * it + i] = *reinterpret_cast<const V4*>(g0 + static_cast<int64_t>(i) * x.rows_in +
                                                       it * P::RB);
      }
  }
}

// Scale the loaded slice by 2^-shift and write it to its LDS rows.
template <typename T, typename V4, int SP, int NTH, int IT>
__device__ inline void slice_to_lds(UnitRef d, const Tile& x, V4* v, T* lds) {
  const int tid = threadIdx.x;
  const int32_t shift = shift_of(d.scale_slot);
  if (x.qn >= 4) {
    const RunPos<SP, NTH> ps(tid);
    const int total = x.rows_in * SP / 4;
#pragma unroll
    for (int it = 0; it < Regs<IT>::N; ++it)
      if (it * NTH + tid < total) {
        V4 y = v[it];
#pragma unroll
        for (int i = 0; i < 4; ++i) y[i] = scale(y[i], shift);
        *reinterpret_cast<V4*>(&lds[ps.lds(it)]) = y;
      }
  } else {
    const BlkPos<SP, NTH> ps(tid);
    const int total = x.rows_in * SP / 16;
#pragma unroll
    for (int it = 0; it < Regs<IT>::NB; ++it)
      if (it * NTH + tid < total) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          V4 y;
#pragma unroll
          for (int i = 0; i < 4; ++i) y[i] = scale(v[4 * it + i][u], shift);
          *reinterpret_cast<V4*>(&lds[ps.lds(it, u, 0)]) = y;
        }
      }
  }
}

// Stage the chunk's padded site matrices (and their bf16 parts) in LDS.
template <typename T, int MODE, int NTH>
__device__ inline void stage_sites(UnitRef d, T* sS, uint16_t* sH, uint16_t* sL) {
  for (int e = threadIdx.x; e < d.k * 256; e += NTH) {
    const int j = e >> 8, k = (e >> 4) & 15, n = e & 15;
    const bool top = j == 0 && d.k1 == 4, bottom = j == d.k - 1 && d.nl == 4;
    const bool zero = (top && k >= 4) || (bottom && (n & 3));
    const int src = bottom ? k * 4 + (n >> 2) : k * 16 + n;
    if constexpr (MODE == M_BF16X3) {
      sH[e] = zero ? uint16_t(0) : d.hi[j][src];
      sL[e] = zero ? uint16_t(0) : d.lo[j][src];
    } else {
      sS[e] = zero ? T(0) : static_cast<const T*>(d.S[j])[src];
    }
  }
}

// The chunk's k steps on the slice in LDS, in place (ends with a barrier).
template <typename T, int MODE, int SP, int NW, int KM, int NBM>
__device__ inline void slice_steps(UnitRef d, T* lds, const T* sS, const uint16_t* sH,
                                   const uint16_t* sL) {
  const int lane = threadIdx.x & 63, c = lane & 15, gg = lane >> 4, w = threadIdx.x >> 6;
  const bool top = d.k1 == 4;
  if (d.k == 2) {
    chunk_steps<T, MODE, SP, NW, 2, NBM>(lds, sS, sH, sL, top, c, gg, w);
  } else if (d.k == 3 || KM < 4) {
    chunk_steps<T, MODE, SP, NW, 3, NBM>(lds, sS, sH, sL, top, c, gg, w);
  } else {
    if constexpr (KM >= 4) chunk_steps<T, MODE, SP, NW, 4, NBM>(lds, sS, sH, sL, top, c, gg, w);
  }
}

// Store the rows of the last step's real outputs; track max |x| and
// non-finite values.
template <typename T, typename V4, int SP, int NTH, int IT>
__device__ inline void slice_store(UnitRef d, const Tile& x, const T* lds, T& mx, int& bad) {
  const int tid = threadIdx.x;
  const int lsh = d.nl == 4 ? 2 : 0;
  T* dst = static_cast<T*>(d.out) + x.p0 * x.rows_out * d.post + x.q0;
  if (x.qn >= 4) {
    using P = RunPos<SP, NTH>;
    const P ps(tid);
    const int total = x.rows_out * SP / 4;
    T* g0 = dst + run_off(x, d.post, x.rows_out, ps.row0, ps.s0);
    const int64_t step = static_cast<int64_t>(P::RS) * (x.qrun ? d.post : x.qn);
#pragma unroll
    for (int it = 0; it < Regs<IT>::N; ++it)
      if (it * NTH + tid < total) {
        const int wd = lsh ? word_of<SP>((ps.row0 + it * P::RS) << lsh, ps.s0) : ps.lds(it);
        const V4 v = *reinterpret_cast<const V4*>(&lds[wd]);
        *reinterpret_cast<V4*>(g0 + it * step) = v;
#pragma unroll
        for (int i = 0; i < 4; ++i) track(v[i], mx, bad);
      }
  } else {
    using P = BlkPos<SP, NTH>;
    const P ps(tid);
    const int total = x.rows_out * SP / 16;
    T* g0 = dst + static_cast<int64_t>(ps.s0) * x.rows_out + ps.row4;
#pragma unroll
    for (int it = 0; it < Regs<IT>::NB; ++it)
      if (it * NTH + tid < total) {
        V4 r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = *reinterpret_cast<const V4*>(&lds[ps.lds(it, u, lsh)]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const V4 v = {r[0][i], r[1][i], r[2][i], r[3][i]};
          *reinterpret_cast<V4*>(g0 + static_cast<int64_t>(i) * x.rows_out + it * P::RB) = v;
#pragma unroll
          for (int q = 0; q < 4; ++q) track(v[q], mx, bad);
        }
      }
  }
}

template <typename T, int MODE>
__global__ __launch_bounds__((64 * Cfg<T>::NW)) __attribute__((amdgpu_waves_per_eu(4))) void
absorb_chunk(ChunkGroup arg) {
  (void)arg;   // read in place below
  using C = Cfg<T>;
  using V4 = typename std::conditional<MODE == M_F64, f64x4, f32x4>::type;
  constexpr int SP = C::SP, NW = C::NW, NTH = 64 * NW, KM = C::KM;
  constexpr int RMAX = 16 << (2 * (KM - 1));
  constexpr int IT = RMAX * SP / (NTH * 4);
  __shared__ __attribute__((aligned(32))) T lds[RMAX * SP];
  __shared__ __attribute__((aligned(16))) T sS[MODE == M_BF16X3 ? 1 : KM * 256];
  __shared__ __attribute__((aligned(16))) uint16_t sH[MODE == M_BF16X3 ? KM * 256 : 1];
  __shared__ __attribute__((aligned(16))) uint16_t sL[MODE == M_BF16X3 ? KM * 256 : 1];
  const GroupRef g = (GroupRef)__builtin_amdgcn_kernarg_segment_ptr();
  V4 v[Regs<IT>::N];

  // one tile; consecutive tiles on one XCD (workgroup b runs on XCD b % 8)
  const uint32_t nb = gridDim.x;
  const uint32_t t = (nb % 8 == 0) ? (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8 : blockIdx.x;
  const Tile x = tile_at<SP>(g, t);
  UnitRef d = g->u[x.ui];
  slice_load<T, V4, SP, NTH, IT>(d, x, v);   // in flight while the sites are staged
  stage_sites<T, MODE, NTH>(d, sS, sH, sL);
  slice_to_lds<T, V4, SP, NTH, IT>(d, x, v, lds);
  __syncthreads();
  slice_steps<T, MODE, SP, NW, KM, 8>(d, lds, sS, sH, sL);
  T mx = 0;
  int bad = 0;
  slice_store<T, V4, SP, NTH, IT>(d, x, lds, mx, bad);
  if (d.max_slot) reduce_and_publish<T, NW>(mx, bad, d.max_slot, g->flags);
}

template <typename T, int MODE>
hipError_t go_chunk(const ChunkArgs* a, int32_t n, const StagedArrays& st, DevState* state,
                    hipStream_t stream) {
  for (int32_t u = 0; u < n; ++u)
    if (a[u].k < 2 || a[u].k > Cfg<T>::KM) return hipErrorInvalidValue;
  ChunkGroup g;
  if (!chunk::fill_group(g, a, n, st, &state->flags, MODE == M_F64)) return hipErrorInvalidValue;
  const uint32_t grid = g.first[kChunkGroup];
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((absorb_chunk<T, MODE>), dim3(grid), dim3(64 * Cfg<T>::NW), 0, stream, g);
  return hipGetLastError();
}

hipError_t go_chunk_lds(const ChunkArgs* a, int32_t n, const StagedArrays& st, DevState* state,
                        hipStream_t stream, const char** kname) {
  if (a[0].type == EL_F64) {
    *kname = "absorb_chunk_f64";
    return go_chunk<double, M_F64>(a, n, st, state, stream);
  }
  if (a[0].arith == AR_BF16X3) {
    *kname = "absorb_chunk_bf16x3";
    return go_chunk<float, M_BF16X3>(a, n, st, state, stream);
  }
  *kname = "absorb_chunk_f32";
  return go_chunk<float, M_F32>(a, n, st, state, stream);
}

// Kernel of the column chunks: 0 = registers where the shape allows (rows of
// up to 4 in FP32/BF16x3, 3 in FP64), 1 = LDS slices only, 2 = registers with
// at most 3 rows in every precision.
int32_t g_chunk_sched = 0;

}  // namespace

int32_t chunk_max_steps(int32_t type) {
  if (g_chunk_sched == 2) return 3;
  return type == EL_F64 ? Cfg<double>::KM : Cfg<float>::KM;
}

void set_chunk_schedule(int32_t s) { g_chunk_sched = s; }

bool chunk_shape_ok(int32_t type, int64_t pre, int64_t post, int32_t k, int32_t k1, int32_t nl) {
  const int64_t sp = type == EL_F64 ? Cfg<double>::SP : Cfg<float>::SP;
  if (k < 2 || k > chunk_max_steps(type) || (k1 != 4 && k1 != 16) || (nl != 4 && nl != 16))
    return false;
  if (pre < 1 || post < 1) return false;
  if (post >= sp) {
    if (post % sp) return false;
  } else {
    // whole suffixes per tile: SP / post consecutive p; a suffix of 2 has no
    // kernel path (not a shape of D = 4 networks)
    if (sp % post || pre % (sp / post) || post == 2) return false;
  }
  return pre <= INT_MAX / post;
}

hipError_t launch_absorb_chunks(const ChunkArgs* a, int32_t n, const StagedArrays& st,
                                DevState* state, hipStream_t stream, const char** kname) {
  if (n < 1 || n > kChunkGroup) return hipErrorInvalidValue;
  ChunkArgs reg[kChunkGroup], lds[kChunkGroup];
  int32_t nr = 0, nl = 0;
  for (int32_t u = 0; u < n; ++u) {
    if (a[u].type != a[0].type || a[u].arith != a[0].arith) return hipErrorInvalidValue;
    if (!chunk_shape_ok(a[u].type, a[u].pre, a[u].post, a[u].k, a[u].k1, a[u].nl))
      return hipErrorInvalidValue;
    if (g_chunk_sched != 1 &&
        chunk_reg_shape_ok(a[u].type, a[u].pre, a[u].post, a[u].k, a[u].k1, a[u].nl))
      reg[nr++] = a[u];
    else
      lds[nl++] = a[u];
  }
  if (nr > 0) {
    const hipError_t e = launch_absorb_chunks_reg(reg, nr, st, state, stream, kname);
    if (e != hipSuccess) return e;
  }
  if (nl > 0) return go_chunk_lds(lds, nl, st, state, stream, kname);
  return hipSuccess;
}

}  // namespace tn
