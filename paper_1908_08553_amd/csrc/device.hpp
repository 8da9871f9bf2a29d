// Structures shared by the host executor and the HIP kernels.
#pragma once

#include <cstdint>

#include "tn.h"

namespace tn {

// Exponent-slot sentinels: INT32_MIN = "all entries zero" (no shift),
// INT32_MAX = "a non-finite entry was seen".
constexpr int32_t kExpZero = INT32_MIN;
constexpr int32_t kExpBad = INT32_MAX;

// One block of the staging kernel folds one site for one step:
// staged[q] = 2^-e * site[canonical offset of staged index q], where e is the
// exponent of the site's largest magnitude (exact power-of-two
// pre-normalisation; e is added back in the final exponent sum).
struct StageDesc {
  const double* src;        // canonical float64 site tensor (device)
  void* init_dst;           // INIT step: unit boundary buffer, else nullptr
  int64_t entries;
  int64_t s_off;            // offset (entries) into the staged arrays
  int64_t cstride[4];       // canonical stride of each staged axis
  int32_t dims[4];          // staged-order dims
  int32_t ndim;
  int32_t init_double;      // INIT boundary element type: 1 = double, 0 = float
};

// Device-side bookkeeping at the start of the workspace.
struct DevState {
  tn_result result;
  int32_t flags;            // bit 0: non-finite seen
  int32_t n_slots;
  int32_t n_steps;
  int32_t pad;
  int64_t e_bias;           // exponent carried in by a supplied boundary (cut plans)
  // followed by: int32 slot_exp[n_slots], int32 site_exp[n_steps], int32 site_bad[n_steps]
};

// A boundary kept between launches (cached environment) and its scale: the
// exact boundary is buffer * 2^-e * 2^(bias + e), with e the exponent of its
// largest magnitude as the rescale slots hold it (kExpZero: no shift and no
// exponent, kExpBad: a non-finite value was seen on the way).
struct EnvRec {
  int64_t bias;
  int32_t e;
  int32_t pad;
};

}  // namespace tn
