// Contraction planner for the planar square lattice (host only, integers only).
//
// Paper §4: a planar network is contracted by pairwise, sequential
// contractions; each intermediate has a "dimension" (entry count) and the
// largest one, the bottleneck, fixes memory and operation count.  Two orders
// are described -- along rows from one edge to the other, and quadrants
// contracted from the edges to the middle, leaving a ring of four tensors --
// and the heuristic keeps the order with the smallest bottleneck.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "tn.h"

namespace tn {

enum : int32_t { LEG_LEFT = 0, LEG_UP = 1, LEG_RIGHT = 2, LEG_DOWN = 3 };
enum : int32_t { FRAME_ID = 0, FRAME_T = 1, FRAME_MH = 2, FRAME_MHV = 3, FRAME_MV = 4 };
enum : int32_t { STEP_INIT = 0, STEP_ABSORB = 1, STEP_SEED = 2 };

// One pairwise step: out[pre][N][post] = sum_k in[pre][k][post] * S[k][n], where
// S is the site tensor folded to (K legs, N legs) by the axis permutation perm.
// An INIT step copies the folded site into the unit's boundary (pre=K=post=1).
// A SEED step (first step of a cut plan) stands for a boundary supplied from
// outside: out = N = its entries, no site, its rescale slot holds the
// supplied boundary's exponent.
struct Step {
  int32_t unit = 0, r = 0, c = 0, kind = STEP_INIT;
  int64_t pre = 1, K = 1, N = 1, post = 1, out = 1, flops = 0;
  int32_t nperm = 0;
  int32_t perm[4] = {0, 0, 0, 0};
  int32_t rescale = -1;    // exponent slot measured after this step
  int32_t scale_in = -1;   // slot whose exponent scales this step's input
  int32_t col = 0;         // local column within the unit's sweep
  int32_t last_col = 0;    // 1 when the step is in the unit's last column
  int64_t site_entries = 1;
};

struct Unit {
  int32_t frame = FRAME_ID;
  int32_t rows = 0, cols = 0;   // local (swept) extent
  int64_t result = 1;           // entries of the unit's final tensor
  int32_t first_step = 0, n_steps = 0;
  int32_t final_slot = -1;      // rescale slot of the last step (-1: none)
};

// Closing the quadrant ring: X = A^T B with A = unit xa as [kx][m], B = unit
// xb as [kx][n]; Yt = C^T E with C = unit ya as [ky][m], E = unit yb as
// [ky][n]; Z = sum over (i,j) of X[i][j] * Yt[i][j].
struct Ring {
  int32_t xa = 0, xb = 1, ya = 3, yb = 2;
  int64_t m = 1, n = 1, kx = 1, ky = 1, flops = 0;
};

// One link of the row scheme's chain (paper §4, Fig. 2a): the chain vector v
// (the first row's tensor, then each link's output) meets the next row's
// tensor R over the row's up legs: v <- v R with R as [K][N] (side 0) or
// v <- R v with R as [N][K] (side 1).  K = up legs, N = down legs (1 for the
// last row, whose link yields the scalar).
struct Link {
  int32_t unit = 0, side = 0;
  int64_t K = 1, N = 1, flops = 0;
  int32_t rescale = -1;     // exponent slot measured after the link (-1: last)
  int32_t scale_v = -1;     // slot whose exponent scales v on load
};

struct Plan {
  int32_t rows = 0, cols = 0;
  std::vector<int32_t> hdim, vdim;
  int32_t requested = TN_ORDER_COLSWEEP, order = TN_ORDER_COLSWEEP;
  int32_t transpose = 0, qh = 0, qw = 0;
  std::vector<Unit> units;
  std::vector<Step> steps;
  bool has_ring = false;
  Ring ring;
  std::vector<Link> chain;         // ROWS: links in order (empty otherwise)
  int32_t slots = 0;
  int64_t peak = 0, flops = 0, moved = 0;
  // intermediate storage the order keeps at once, in entries: two buffers of
  // each unit's largest intermediate, plus the stored ring product or two
  // chain vectors of the largest link output
  int64_t buffers = 0;
  int64_t total_site_entries = 0;
  // Cut plans: local columns [cut_c0, cut_c1) of a full-lattice column sweep,
  // left to right (cut_mirror 0) or right to left (1).  They start with a SEED
  // step when cut_c0 > 0 and end in the boundary after column cut_c1 - 1 when
  // cut_c1 < cols (the column-sweep scalar otherwise).
  bool is_cut = false;
  bool cut_open_end = false;       // ends in a boundary (else in the sweep's scalar)
  int32_t cut_mirror = 0, cut_c0 = 0, cut_c1 = 0;
  int64_t cut_k0 = 0, cut_k1 = 0;  // sweep steps [cut_k0, cut_k1)
  std::vector<int32_t> cut_legs;   // bond ids of the ending boundary, slowest first
};

// Builds a plan.  Returns TN_OK, TN_EINVAL, TN_EOVERFLOW or, when the plan
// (for HEURISTIC / SWEEP_AUTO: every candidate) keeps more than `budget`
// entries of intermediate storage, TN_ENOMEM (budget <= 0: no limit).
tn_status build_plan(const tn_grid& grid, int32_t order, int32_t quad_h,
                     int32_t quad_w, Plan& out, std::string& err, int64_t budget = 0);

// Cut plans of the column sweep (see Plan::is_cut): same steps, site folds and
// rescale points as the full sweep over sweep steps [k0, k1) (step k absorbs
// local site (k mod rows, k / rows)), or over local columns [c0, c1).
// TN_EINVAL unless 0 <= k0 < k1 <= rows*cols (0 <= c0 < c1 <= cols).
tn_status build_sweep_cut(const tn_grid& grid, int32_t mirror, int64_t k0, int64_t k1, Plan& out,
                          std::string& err);
tn_status build_cut_plan(const tn_grid& grid, int32_t mirror, int32_t c0, int32_t c1, Plan& out,
                         std::string& err);

// One reverse step in column c (cached environments inside a column): the
// boundary of all sites after (r, c) in the left-to-right sweep order (the
// right environment at column c+1 with rows r+1..rows-1 of column c absorbed
// from the bottom), in the sweep's own leg order, absorbs site (r, c) by its
// right and down legs and puts its up and left legs in their place; the
// result is the boundary of all sites after (r-1, c), in the leg order the
// sweep has after absorbing (r-1, c).  A SEED step supplies the input, except
// at the bottom-right site, which starts the boundary (INIT).  1 <= r < rows.
tn_status build_rev_step(const tn_grid& grid, int32_t r, int32_t c, Plan& out, std::string& err);

// Bond ids of the boundary after every step of the full left-to-right column
// sweep (legs[k] after step k, slowest first): the leg order every cut plan,
// environment and reverse step of the sweep must share.
tn_status sweep_legs(const tn_grid& grid, std::vector<std::vector<int32_t>>& legs,
                     std::string& err);

// Canonical text: identical bytes for identical plans.
std::string plan_text(const Plan& p);

}  // namespace tn
