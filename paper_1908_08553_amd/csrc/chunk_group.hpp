// Launch argument of the column-chunk kernels: up to four units (one column
// chunk of each of up to four sweeps) whose 16-fibre tiles form one grid.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace tn {
namespace chunk {

constexpr int kGroup = 4;

struct Unit {
  const void* in;
  void* out;
  const void* S[kChunkMax];
  const uint16_t* hi[kChunkMax];
  const uint16_t* lo[kChunkMax];
  int64_t pre, post;     // prefix of the first step, suffix of the last
  int32_t k, k1, nl;     // steps; K of the first step (4 or 16); N of the last (4 or 16)
  int32_t pad;
  const int32_t* scale_slot;
  int32_t* max_slot;
};

struct Group {
  Unit u[kGroup];
  uint32_t first[kGroup + 1];   // unused entries hold the total tile count
  int32_t n;
  int32_t* flags;
};

// The launch's Group is read in place from the kernel-argument segment
// (constant address space, uniform: scalar loads), so dynamic unit and step
// indices need no private copy of it.
#define TN_KARG __attribute__((address_space(4)))
typedef const TN_KARG Group* GroupRef;
typedef const TN_KARG Unit& UnitRef;

// Unit of group tile t.
__device__ inline int unit_index(GroupRef g, uint32_t t) {
  return static_cast<int>(t >= g->first[1]) + static_cast<int>(t >= g->first[2]) +
         static_cast<int>(t >= g->first[3]);
}

// Fill a Group from the host-side chunk arguments (site operands from the
// staged arrays); tiles = pre * post / 16 per unit.  False when the tile count
// does not fit the 32-bit grid.
inline bool fill_group(Group& g, const ChunkArgs* a, int32_t n, const StagedArrays& st,
                       int32_t* flags, bool f64) {
  g = Group{};
  g.n = n;
  g.flags = flags;
  uint64_t total = 0;
  for (int32_t u = 0; u < n; ++u) {
    const ChunkArgs& x = a[u];
    Unit& c = g.u[u];
    c.in = x.in;
    c.out = x.out;
    for (int j = 0; j < x.k; ++j) {
      c.S[j] = f64 ? static_cast<const void*>(st.s64 + x.s_off[j])
                   : static_cast<const void*>(st.s32 + x.s_off[j]);
      c.hi[j] = st.shi + x.s_off[j];
      c.lo[j] = st.slo + x.s_off[j];
    }
    c.pre = x.pre;
    c.post = x.post;
    c.k = x.k;
    c.k1 = x.k1;
    c.nl = x.nl;
    c.scale_slot = x.scale_slot;
    c.max_slot = x.max_slot;
    g.first[u] = static_cast<uint32_t>(total);
    total += static_cast<uint64_t>(x.pre * x.post / 16);
    if (total > 0x7fffffffull) return false;
  }
  for (int32_t u = n; u <= kGroup; ++u) g.first[u] = static_cast<uint32_t>(total);
  return true;
}

}  // namespace chunk
}  // namespace tn
