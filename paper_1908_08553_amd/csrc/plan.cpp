// Contraction planner: column sweep, quadrant ring and the minimal-bottleneck
// heuristic (paper §4, Fig. 2).  See plan.hpp for the step model.
//
// Readings where the paper is silent or garbled:
//  * Dimension rule: the printed d(B) = d(A1) d(A2) / d(x) counts the shared
//    legs once; both operands carry them, so the planner tracks legs and the
//    result is d(A1) d(A2) / d(x)^2.
//  * The row scheme runs sequentially as a sweep: the boundary absorbs one
//    site at a time, columns left to right, rows top to bottom, in a frame.
//    The absorbed site's shared legs (local up, local left) are replaced in
//    place by its new legs (local right, then local down).
//  * Quadrant split rows [0,h) / [h,R), columns [0,w) / [w,C), default
//    h = ceil(R/2), w = ceil(C/2).  Each quadrant is swept from its outer
//    lattice corner; legs that leave a quadrant stay on its tensor.
//  * Heuristic key: (bottleneck entries, total flops, candidate index) over
//    sweep, transposed sweep, then quadrant splits (h, w) in lexicographic
//    order.
//  * Exact power-of-two rescale points after every local column except the
//    last column of a sweep order (which ends in the scalar).
#include "plan.hpp"

#include <algorithm>
#include <cstdio>
#include <stdexcept>
#include <sstream>

namespace tn {
namespace {

struct Overflow {};

inline int64_t mul(int64_t a, int64_t b) {
  int64_t r;
  if (__builtin_mul_overflow(a, b, &r)) throw Overflow{};
  return r;
}
inline int64_t add(int64_t a, int64_t b) {
  int64_t r;
  if (__builtin_add_overflow(a, b, &r)) throw Overflow{};
  return r;
}

// local legs L, U, R, Dn of each frame, as canonical legs
const int32_t kFrameLegs[5][4] = {
    {LEG_LEFT, LEG_UP, LEG_RIGHT, LEG_DOWN},   // ID
    {LEG_UP, LEG_LEFT, LEG_DOWN, LEG_RIGHT},   // T   (transpose)
    {LEG_RIGHT, LEG_UP, LEG_LEFT, LEG_DOWN},   // MH  (mirror left-right)
    {LEG_RIGHT, LEG_DOWN, LEG_LEFT, LEG_UP},   // MHV (mirror both)
    {LEG_LEFT, LEG_DOWN, LEG_RIGHT, LEG_UP},   // MV  (mirror top-bottom)
};
const char* kFrameName[5] = {"ID", "T", "MH", "MHV", "MV"};
const char* kOrderName[6] = {"COLSWEEP", "QUADRANT", "HEURISTIC", "SWEEP_AUTO", "ROWS",
                             "ROWS_T"};

struct Lattice {
  int32_t R, C;
  const std::vector<int32_t>* h;
  const std::vector<int32_t>* v;
  int32_t nh() const { return R * (C - 1); }
  // bond ids: h(r,c) -> r*(C-1)+c ; v(r,c) -> nh + r*C + c
  int32_t hid(int32_t r, int32_t c) const { return r * (C - 1) + c; }
  int32_t vid(int32_t r, int32_t c) const { return nh() + r * C + c; }
  int64_t dim(int32_t b) const { return b < nh() ? (*h)[b] : (*v)[b - nh()]; }
  bool has(int32_t r, int32_t c, int32_t leg) const {
    switch (leg) {
      case LEG_LEFT: return c > 0;
      case LEG_UP: return r > 0;
      case LEG_RIGHT: return c < C - 1;
      default: return r < R - 1;
    }
  }
  int32_t bond(int32_t r, int32_t c, int32_t leg) const {
    switch (leg) {
      case LEG_LEFT: return hid(r, c - 1);
      case LEG_UP: return vid(r - 1, c);
      case LEG_RIGHT: return hid(r, c);
      default: return vid(r, c);
    }
  }
  // canonical axis index of `leg` at (r,c): count of present legs before it
  int32_t axis(int32_t r, int32_t c, int32_t leg) const {
    int32_t a = 0;
    for (int32_t l = 0; l < leg; ++l) a += has(r, c, l) ? 1 : 0;
    return a;
  }
  void site_of(int32_t frame, int32_t i, int32_t j, int32_t& r, int32_t& c) const {
    switch (frame) {
      case FRAME_ID: r = i; c = j; break;
      case FRAME_T: r = j; c = i; break;
      case FRAME_MH: r = i; c = C - 1 - j; break;
      case FRAME_MHV: r = R - 1 - i; c = C - 1 - j; break;
      default: r = R - 1 - i; c = j; break;
    }
  }
};

// Sweep local rows [0,nh) x cols [0,nw) of `frame`; appends steps, returns the
// final boundary legs.
std::vector<int32_t> sweep(const Lattice& L, int32_t unit, int32_t frame, int32_t nh,
                           int32_t nw, bool rescale_last, int32_t& slot,
                           std::vector<Step>& steps,
                           std::vector<std::vector<int32_t>>* legs_after = nullptr) {
  std::vector<int32_t> bnd;
  const int32_t* fl = kFrameLegs[frame];
  for (int32_t j = 0; j < nw; ++j) {
    for (int32_t i = 0; i < nh; ++i) {
      int32_t r, c;
      L.site_of(frame, i, j, r, c);
      Step s;
      s.unit = unit; s.r = r; s.c = c; s.col = j; s.last_col = (j == nw - 1);
      s.site_entries = 1;
      for (int32_t leg = 0; leg < 4; ++leg)
        if (L.has(r, c, leg)) s.site_entries = mul(s.site_entries, L.dim(L.bond(r, c, leg)));
      // shared legs sit at local L / U, new legs at local R then Dn
      std::vector<int32_t> shared_legs, new_legs;
      for (int32_t loc : {0, 1})
        if (L.has(r, c, fl[loc])) shared_legs.push_back(fl[loc]);
      for (int32_t loc : {2, 3})
        if (L.has(r, c, fl[loc])) new_legs.push_back(fl[loc]);
      if (i == 0 && j == 0) {
        s.kind = STEP_INIT;
        int64_t n = 1;
        for (int32_t leg : new_legs) {
          s.perm[s.nperm++] = L.axis(r, c, leg);
          n = mul(n, L.dim(L.bond(r, c, leg)));
          bnd.push_back(L.bond(r, c, leg));
        }
        s.pre = s.K = s.post = 1;
        s.N = n;
        s.out = n;
        s.flops = 0;
        steps.push_back(s);
        if (nh == 1 && (j < nw - 1 || rescale_last)) steps.back().rescale = slot++;
        if (legs_after) legs_after->push_back(bnd);
        continue;
      }
      // locate the shared bonds in the boundary; they must be adjacent
      size_t k0 = bnd.size();
      for (int32_t leg : shared_legs) {
        auto it = std::find(bnd.begin(), bnd.end(), L.bond(r, c, leg));
        k0 = std::min(k0, static_cast<size_t>(it - bnd.begin()));
      }
      const size_t nk = shared_legs.size();
      int64_t pre = 1, post = 1, K = 1, N = 1;
      for (size_t a = 0; a < k0; ++a) pre = mul(pre, L.dim(bnd[a]));
      for (size_t a = k0 + nk; a < bnd.size(); ++a) post = mul(post, L.dim(bnd[a]));
      for (size_t a = k0; a < k0 + nk; ++a) {
        const int32_t b = bnd[a];
        int32_t leg = -1;
        for (int32_t l : shared_legs)
          if (L.bond(r, c, l) == b) leg = l;
        if (leg < 0) throw std::runtime_error("shared legs are not adjacent");
        s.perm[s.nperm++] = L.axis(r, c, leg);
        K = mul(K, L.dim(b));
      }
      std::vector<int32_t> nb(bnd.begin(), bnd.begin() + k0);
      for (int32_t leg : new_legs) {
        s.perm[s.nperm++] = L.axis(r, c, leg);
        N = mul(N, L.dim(L.bond(r, c, leg)));
        nb.push_back(L.bond(r, c, leg));
      }
      nb.insert(nb.end(), bnd.begin() + k0 + nk, bnd.end());
      bnd.swap(nb);
      s.kind = STEP_ABSORB;
      s.pre = pre; s.K = K; s.N = N; s.post = post;
      s.out = mul(mul(pre, N), post);
      s.flops = mul(mul(s.out, K), 2);
      steps.push_back(s);
      if (i == nh - 1 && (j < nw - 1 || rescale_last)) steps.back().rescale = slot++;
      if (legs_after) legs_after->push_back(bnd);
    }
  }
  return bnd;
}

void finish(Plan& p) {
  p.peak = 0; p.flops = 0; p.moved = 0; p.total_site_entries = 0;
  for (size_t k = 0; k < p.steps.size(); ++k) {
    Step& s = p.steps[k];
    p.peak = std::max(p.peak, s.out);
    p.flops = add(p.flops, s.flops);
    p.total_site_entries = add(p.total_site_entries, s.site_entries);
    if (s.kind == STEP_ABSORB) {
      p.moved = add(p.moved, add(mul(mul(s.pre, s.K), s.post), s.out));
      const Step& prev = p.steps[k - 1];
      if (prev.unit == s.unit && prev.rescale >= 0) s.scale_in = prev.rescale;
    }
  }
  for (size_t u = 0; u < p.units.size(); ++u) {
    Unit& U = p.units[u];
    U.final_slot = p.steps[U.first_step + U.n_steps - 1].rescale;
  }
  if (p.has_ring) {
    const int64_t mn = mul(p.ring.m, p.ring.n);
    p.peak = std::max(p.peak, mn);
    p.flops = add(p.flops, p.ring.flops);
    for (const Unit& U : p.units) p.moved = add(p.moved, U.result);
    p.moved = add(p.moved, mul(mn, 2));
  }
  int32_t vslot = p.units.empty() ? -1 : p.units[0].final_slot;
  int64_t big_link = 0;
  for (Link& lk : p.chain) {
    p.peak = std::max(p.peak, lk.N);
    p.flops = add(p.flops, lk.flops);
    p.moved = add(p.moved, add(mul(lk.K, lk.N), add(lk.K, lk.N)));
    lk.scale_v = vslot;
    vslot = lk.rescale;
    big_link = std::max(big_link, lk.N);
  }
  // intermediate storage: two buffers of every unit's largest intermediate,
  // the stored ring product, two chain vectors
  p.buffers = 0;
  for (const Unit& U : p.units) {
    int64_t big = 1;
    for (int32_t k = U.first_step; k < U.first_step + U.n_steps; ++k)
      big = std::max(big, p.steps[k].out);
    p.buffers = add(p.buffers, mul(big, 2));
  }
  if (p.has_ring) p.buffers = add(p.buffers, mul(p.ring.m, p.ring.n));
  if (!p.chain.empty()) p.buffers = add(p.buffers, mul(big_link, 2));
}

void plan_colsweep(const Lattice& L, int32_t transpose, int32_t requested, Plan& p) {
  p.requested = requested;
  p.order = TN_ORDER_COLSWEEP;
  p.transpose = transpose;
  p.qh = p.qw = 0;
  p.has_ring = false;
  p.units.clear();
  p.steps.clear();
  const int32_t frame = transpose ? FRAME_T : FRAME_ID;
  const int32_t nh = transpose ? L.C : L.R, nw = transpose ? L.R : L.C;
  int32_t slot = 0;
  sweep(L, 0, frame, nh, nw, false, slot, p.steps);
  Unit U;
  U.frame = frame; U.rows = nh; U.cols = nw; U.result = 1;
  U.first_step = 0; U.n_steps = static_cast<int32_t>(p.steps.size());
  p.units.push_back(U);
  p.slots = slot;
  finish(p);
}

void plan_quadrant(const Lattice& L, int32_t h, int32_t w, int32_t requested, Plan& p) {
  p.requested = requested;
  p.order = TN_ORDER_QUADRANT;
  p.transpose = 0;
  p.qh = h; p.qw = w;
  p.units.clear();
  p.steps.clear();
  const int32_t R = L.R, C = L.C;
  const int32_t frames[4] = {FRAME_ID, FRAME_MH, FRAME_MHV, FRAME_MV};
  const int32_t nhs[4] = {h, h, R - h, R - h};
  const int32_t nws[4] = {w, C - w, C - w, w};
  int32_t slot = 0;
  for (int32_t u = 0; u < 4; ++u) {
    Unit U;
    U.frame = frames[u]; U.rows = nhs[u]; U.cols = nws[u];
    U.first_step = static_cast<int32_t>(p.steps.size());
    std::vector<int32_t> legs = sweep(L, u, frames[u], nhs[u], nws[u], true, slot, p.steps);
    U.n_steps = static_cast<int32_t>(p.steps.size()) - U.first_step;
    U.result = 1;
    for (int32_t b : legs) U.result = mul(U.result, L.dim(b));
    p.units.push_back(U);
  }
  Ring& g = p.ring;
  g.xa = 0; g.xb = 1; g.ya = 3; g.yb = 2;
  g.kx = 1; g.ky = 1; g.m = 1; g.n = 1;
  for (int32_t r = 0; r < h; ++r) g.kx = mul(g.kx, L.dim(L.hid(r, w - 1)));
  for (int32_t r = h; r < R; ++r) g.ky = mul(g.ky, L.dim(L.hid(r, w - 1)));
  for (int32_t c = 0; c < w; ++c) g.m = mul(g.m, L.dim(L.vid(h - 1, c)));
  for (int32_t c = w; c < C; ++c) g.n = mul(g.n, L.dim(L.vid(h - 1, c)));
  const int64_t mn = mul(g.m, g.n);
  g.flops = add(add(mul(mul(mn, g.kx), 2), mul(mul(mn, g.ky), 2)), mul(mn, 2));
  p.has_ring = true;
  p.slots = slot;
  finish(p);
}

// Row i of `frame` contracted left to right into one tensor (paper §4, the
// row scheme).  Each site joins by its local left leg; its other legs go in
// place of the joined one, ordered up, right, down (up_first) or down,
// right, up, so the row tensor ends as [up legs left->right][down legs
// right->left] or [down legs left->right][up legs right->left].  Rescale
// after every step (the last one only with rescale_last).
std::vector<int32_t> row_unit(const Lattice& L, int32_t unit, int32_t frame, int32_t i,
                              int32_t nw, bool up_first, bool rescale_last, int32_t& slot,
                              std::vector<Step>& steps) {
  const int32_t* fl = kFrameLegs[frame];
  const int32_t order_a[3] = {1, 2, 3}, order_b[3] = {3, 2, 1};
  const int32_t* order = up_first ? order_a : order_b;
  std::vector<int32_t> bnd;
  for (int32_t j = 0; j < nw; ++j) {
    int32_t r, c;
    L.site_of(frame, i, j, r, c);
    Step s;
    s.unit = unit; s.r = r; s.c = c; s.col = j; s.last_col = (j == nw - 1);
    s.site_entries = 1;
    for (int32_t leg = 0; leg < 4; ++leg)
      if (L.has(r, c, leg)) s.site_entries = mul(s.site_entries, L.dim(L.bond(r, c, leg)));
    std::vector<int32_t> new_legs;
    for (int32_t k = 0; k < 3; ++k)
      if (L.has(r, c, fl[order[k]])) new_legs.push_back(fl[order[k]]);
    int64_t N = 1;
    for (int32_t leg : new_legs) N = mul(N, L.dim(L.bond(r, c, leg)));
    if (j == 0) {
      s.kind = STEP_INIT;
      for (int32_t leg : new_legs) {
        s.perm[s.nperm++] = L.axis(r, c, leg);
        bnd.push_back(L.bond(r, c, leg));
      }
      s.pre = s.K = s.post = 1;
      s.N = s.out = N;
      s.flops = 0;
    } else {
      const int32_t jl = fl[0];
      const int32_t joined = L.bond(r, c, jl);
      const size_t k = static_cast<size_t>(std::find(bnd.begin(), bnd.end(), joined) - bnd.begin());
      if (k == bnd.size()) throw std::runtime_error("row leg missing");
      int64_t pre = 1, post = 1;
      for (size_t a = 0; a < k; ++a) pre = mul(pre, L.dim(bnd[a]));
      for (size_t a = k + 1; a < bnd.size(); ++a) post = mul(post, L.dim(bnd[a]));
      s.perm[s.nperm++] = L.axis(r, c, jl);
      std::vector<int32_t> nb(bnd.begin(), bnd.begin() + k);
      for (int32_t leg : new_legs) {
        s.perm[s.nperm++] = L.axis(r, c, leg);
        nb.push_back(L.bond(r, c, leg));
      }
      nb.insert(nb.end(), bnd.begin() + k + 1, bnd.end());
      bnd.swap(nb);
      s.kind = STEP_ABSORB;
      s.pre = pre; s.K = L.dim(joined); s.N = N; s.post = post;
      s.out = mul(mul(pre, N), post);
      s.flops = mul(mul(s.out, s.K), 2);
    }
    steps.push_back(s);
    if (j < nw - 1 || rescale_last) steps.back().rescale = slot++;
  }
  return bnd;
}

// The row scheme (paper §4, Fig. 2a): one unit per row (per column when
// transposed), then the chain of row tensors closed from the first row on.
// Even rows keep their up legs first and odd rows their down legs first, so
// a link's summed legs have the same order on the chain vector and the row.
void plan_rows(const Lattice& L, int32_t transpose, int32_t requested, Plan& p) {
  p.requested = requested;
  p.order = TN_ORDER_ROWS;
  p.transpose = transpose;
  p.qh = p.qw = 0;
  p.has_ring = false;
  p.units.clear();
  p.steps.clear();
  p.chain.clear();
  const int32_t frame = transpose ? FRAME_T : FRAME_ID;
  const int32_t nh = transpose ? L.C : L.R, nw = transpose ? L.R : L.C;
  const int32_t* fl = kFrameLegs[frame];
  int32_t slot = 0;
  std::vector<std::vector<int32_t>> legs(nh);
  for (int32_t i = 0; i < nh; ++i) {
    Unit U;
    U.frame = frame; U.rows = 1; U.cols = nw;
    U.first_step = static_cast<int32_t>(p.steps.size());
    legs[i] = row_unit(L, i, frame, i, nw, i % 2 == 0, nh > 1, slot, p.steps);
    U.n_steps = static_cast<int32_t>(p.steps.size()) - U.first_step;
    U.result = 1;
    for (int32_t b : legs[i]) U.result = mul(U.result, L.dim(b));
    p.units.push_back(U);
  }
  std::vector<int32_t> v = nh > 1 ? legs[0] : std::vector<int32_t>{};
  for (int32_t i = 1; i < nh; ++i) {
    std::vector<int32_t> ups, downs;
    for (int32_t j = 0; j < nw; ++j) {
      int32_t r, c;
      L.site_of(frame, i, j, r, c);
      ups.push_back(L.bond(r, c, fl[1]));
      if (i < nh - 1) downs.push_back(L.bond(r, c, fl[3]));
    }
    const std::vector<int32_t>& lg = legs[i];
    std::vector<int32_t> up_part, down_part;
    Link lk;
    lk.unit = i;
    if (i % 2 == 0) {
      lk.side = 0;
      up_part.assign(lg.begin(), lg.begin() + nw);
      down_part.assign(lg.begin() + nw, lg.end());
      std::reverse(downs.begin(), downs.end());
    } else {
      lk.side = 1;
      down_part.assign(lg.begin(), lg.begin() + downs.size());
      up_part.assign(lg.begin() + downs.size(), lg.end());
      std::reverse(ups.begin(), ups.end());
    }
    if (up_part != ups || down_part != downs || up_part != v)
      throw std::runtime_error("row chain legs out of order");
    for (int32_t b : up_part) lk.K = mul(lk.K, L.dim(b));
    for (int32_t b : down_part) lk.N = mul(lk.N, L.dim(b));
    lk.flops = mul(mul(lk.K, lk.N), 2);
    if (i < nh - 1) lk.rescale = slot++;
    p.chain.push_back(lk);
    v = down_part;
  }
  p.slots = slot;
  finish(p);
}

}  // namespace

tn_status build_plan(const tn_grid& grid, int32_t order, int32_t quad_h, int32_t quad_w,
                     Plan& out, std::string& err, int64_t budget) {
  const int32_t R = grid.rows, C = grid.cols;
  if (R < 1 || C < 1) { err = "rows and cols must be >= 1"; return TN_EINVAL; }
  if (static_cast<int64_t>(R) * C > (1 << 20)) { err = "lattice too large"; return TN_EINVAL; }
  Plan p;
  p.rows = R; p.cols = C;
  p.hdim.resize(static_cast<size_t>(R) * (C - 1));
  p.vdim.resize(static_cast<size_t>(R - 1) * C);
  for (size_t k = 0; k < p.hdim.size(); ++k) p.hdim[k] = grid.hdim ? grid.hdim[k] : grid.D;
  for (size_t k = 0; k < p.vdim.size(); ++k) p.vdim[k] = grid.vdim ? grid.vdim[k] : grid.D;
  if ((!grid.hdim || !grid.vdim) && grid.D < 1 && (!p.hdim.empty() || !p.vdim.empty())) {
    err = "D must be >= 1"; return TN_EINVAL;
  }
  for (int32_t d : p.hdim) if (d < 1) { err = "bond dimension < 1"; return TN_EINVAL; }
  for (int32_t d : p.vdim) if (d < 1) { err = "bond dimension < 1"; return TN_EINVAL; }
  Lattice L{R, C, &p.hdim, &p.vdim};
  auto fits = [&](const Plan& q) { return budget <= 0 || q.buffers <= budget; };
  bool too_large = false;
  try {
    if (order == TN_ORDER_COLSWEEP) {
      plan_colsweep(L, 0, TN_ORDER_COLSWEEP, p);
      too_large = !fits(p);
    } else if (order == TN_ORDER_QUADRANT) {
      if (R < 2 || C < 2) { err = "QUADRANT needs >= 2 rows and >= 2 columns"; return TN_EINVAL; }
      const int32_t h = quad_h ? quad_h : (R + 1) / 2;
      const int32_t w = quad_w ? quad_w : (C + 1) / 2;
      if (h < 1 || h > R - 1 || w < 1 || w > C - 1) { err = "quadrant split out of range"; return TN_EINVAL; }
      plan_quadrant(L, h, w, TN_ORDER_QUADRANT, p);
      too_large = !fits(p);
    } else if (order == TN_ORDER_ROWS || order == TN_ORDER_ROWS_T) {
      plan_rows(L, order == TN_ORDER_ROWS_T ? 1 : 0, order, p);
      too_large = !fits(p);
    } else if (order == TN_ORDER_SWEEP_AUTO || order == TN_ORDER_HEURISTIC) {
      // candidates in enumeration order: sweep, transposed sweep, then (for
      // HEURISTIC) every quadrant split (h, w) lexicographically, the row
      // scheme and the transposed row scheme; the smallest bottleneck, then
      // the fewest flops, then the earliest candidate among those that fit
      bool have = false, built = false;
      Plan best;
      auto consider = [&](Plan& cand) {
        built = true;
        if (!fits(cand)) return;
        if (!have || cand.peak < best.peak || (cand.peak == best.peak && cand.flops < best.flops)) {
          best = cand;
          have = true;
        }
      };
      for (int32_t t = 0; t < 2; ++t) {
        Plan cand = p;
        try { plan_colsweep(L, t, order, cand); consider(cand); } catch (Overflow&) {}
      }
      if (order == TN_ORDER_HEURISTIC) {
        if (R >= 2 && C >= 2) {
          for (int32_t h = 1; h < R; ++h)
            for (int32_t w = 1; w < C; ++w) {
              Plan cand = p;
              try { plan_quadrant(L, h, w, TN_ORDER_HEURISTIC, cand); consider(cand); } catch (Overflow&) {}
            }
        }
        for (int32_t t = 0; t < 2; ++t) {
          Plan cand = p;
          try { plan_rows(L, t, TN_ORDER_HEURISTIC, cand); consider(cand); } catch (Overflow&) {}
        }
      }
      if (!built) throw Overflow{};
      if (have) p = best;
      too_large = !have;
    } else {
      err = "unknown order";
      return TN_EINVAL;
    }
  } catch (Overflow&) {
    err = "plan integers overflow int64";
    return TN_EOVERFLOW;
  }
  if (too_large) {
    err = "no plan keeps at most " + std::to_string(budget) + " entries of intermediate storage";
    return TN_ENOMEM;
  }
  out = std::move(p);
  return TN_OK;
}

tn_status build_sweep_cut(const tn_grid& grid, int32_t mirror, int64_t k0, int64_t k1, Plan& out,
                          std::string& err) {
  Plan p;
  const tn_status st = build_plan(grid, TN_ORDER_COLSWEEP, 0, 0, p, err);
  if (st != TN_OK) return st;
  const int32_t R = p.rows, C = p.cols;
  const int64_t total = static_cast<int64_t>(R) * C;
  if (k0 < 0 || k1 > total || k0 >= k1) { err = "cut steps out of range"; return TN_EINVAL; }
  Lattice L{R, C, &p.hdim, &p.vdim};
  const int32_t frame = mirror ? FRAME_MH : FRAME_ID;
  std::vector<Step> all;
  std::vector<std::vector<int32_t>> legs;
  int32_t slot = 0;
  try {
    sweep(L, 0, frame, R, C, false, slot, all, &legs);
  } catch (Overflow&) {
    err = "plan integers overflow int64";
    return TN_EOVERFLOW;
  }
  p.steps.clear();
  if (k0 > 0) {
    const Step& last = all[k0 - 1];
    Step s;
    s.unit = 0; s.r = last.r; s.c = last.c; s.kind = STEP_SEED;
    s.pre = s.K = s.post = 1;
    s.N = s.out = last.out;
    s.col = last.col; s.last_col = last.last_col;
    s.site_entries = 0;
    s.rescale = 0;
    p.steps.push_back(s);
  }
  // rescale slots renumbered in order of appearance, after the seed's slot 0
  int32_t next = k0 > 0 ? 1 : 0, prev_old = -1;
  for (int64_t k = k0; k < k1; ++k) {
    Step s = all[k];
    s.scale_in = -1;
    if (s.rescale >= 0) {
      if (s.rescale != prev_old) { prev_old = s.rescale; ++next; }
      s.rescale = next - 1;
    }
    p.steps.push_back(s);
  }
  p.slots = 0;
  for (const Step& s : p.steps) p.slots = std::max(p.slots, s.rescale + 1);
  p.units.clear();
  Unit U;
  U.frame = frame; U.rows = R; U.cols = static_cast<int32_t>((k1 - k0 + R - 1) / R);
  U.result = p.steps.back().out;
  U.first_step = 0; U.n_steps = static_cast<int32_t>(p.steps.size());
  p.units.push_back(U);
  p.is_cut = true;
  p.cut_mirror = mirror ? 1 : 0;
  p.cut_k0 = k0;
  p.cut_k1 = k1;
  p.cut_c0 = static_cast<int32_t>(k0 / R);
  p.cut_c1 = static_cast<int32_t>((k1 + R - 1) / R);
  p.cut_open_end = k1 < total;
  p.cut_legs = legs[k1 - 1];
  try {
    finish(p);
  } catch (Overflow&) {
    err = "plan integers overflow int64";
    return TN_EOVERFLOW;
  }
  out = std::move(p);
  return TN_OK;
}

tn_status sweep_legs(const tn_grid& grid, std::vector<std::vector<int32_t>>& legs,
                     std::string& err) {
  Plan p;
  const tn_status st = build_plan(grid, TN_ORDER_COLSWEEP, 0, 0, p, err);
  if (st != TN_OK) return st;
  Lattice L{p.rows, p.cols, &p.hdim, &p.vdim};
  std::vector<Step> all;
  int32_t slot = 0;
  legs.clear();
  try {
    sweep(L, 0, FRAME_ID, p.rows, p.cols, false, slot, all, &legs);
  } catch (Overflow&) {
    err = "plan integers overflow int64";
    return TN_EOVERFLOW;
  }
  return TN_OK;
}

tn_status build_cut_plan(const tn_grid& grid, int32_t mirror, int32_t c0, int32_t c1, Plan& out,
                         std::string& err) {
  if (grid.rows < 1 || c0 < 0 || c1 < c0) { err = "cut columns out of range"; return TN_EINVAL; }
  return build_sweep_cut(grid, mirror, static_cast<int64_t>(c0) * grid.rows,
                         static_cast<int64_t>(c1) * grid.rows, out, err);
}

static std::vector<int32_t> rev_input_legs(const Plan& g, int32_t r, int32_t c) {
  const int32_t R = g.rows, C = g.cols;
  Lattice L{R, C, &g.hdim, &g.vdim};
  std::vector<int32_t> b;
  if (r == R - 1) {
    if (c < C - 1)
      for (int32_t i = 0; i < R; ++i) b.push_back(L.hid(i, c));
    return b;
  }
  for (int32_t i = 0; i <= r; ++i)
    if (c < C - 1) b.push_back(L.hid(i, c));
  b.push_back(L.vid(r, c));
  for (int32_t i = r + 1; i < R; ++i)
    if (c > 0) b.push_back(L.hid(i, c - 1));
  return b;
}

tn_status build_rev_step(const tn_grid& grid, int32_t r, int32_t c, Plan& out, std::string& err) {
  Plan p;
  const tn_status st = build_plan(grid, TN_ORDER_COLSWEEP, 0, 0, p, err);
  if (st != TN_OK) return st;
  const int32_t R = p.rows, C = p.cols;
  if (r < 1 || r >= R || c < 0 || c >= C) { err = "reverse step out of range"; return TN_EINVAL; }
  Lattice L{R, C, &p.hdim, &p.vdim};
  try {
    std::vector<int32_t> bnd = rev_input_legs(p, r, c);
    std::vector<int32_t> k_legs, n_legs;
    for (int32_t leg : {LEG_RIGHT, LEG_DOWN})
      if (L.has(r, c, leg)) k_legs.push_back(leg);
    for (int32_t leg : {LEG_UP, LEG_LEFT})
      if (L.has(r, c, leg)) n_legs.push_back(leg);
    p.steps.clear();
    Step s;
    s.unit = 0; s.r = r; s.c = c; s.col = c; s.last_col = (c == C - 1);
    s.site_entries = 1;
    for (int32_t leg = 0; leg < 4; ++leg)
      if (L.has(r, c, leg)) s.site_entries = mul(s.site_entries, L.dim(L.bond(r, c, leg)));
    if (!bnd.empty()) {
      Step seed;
      seed.unit = 0; seed.r = r; seed.c = c; seed.kind = STEP_SEED;
      seed.pre = seed.K = seed.post = 1;
      int64_t n = 1;
      for (int32_t b : bnd) n = mul(n, L.dim(b));
      seed.N = seed.out = n;
      seed.col = c; seed.last_col = s.last_col;
      seed.site_entries = 0;
      seed.rescale = 0;
      p.steps.push_back(seed);
    }
    if (k_legs.empty()) {
      s.kind = STEP_INIT;
      int64_t n = 1;
      for (int32_t leg : n_legs) {
        s.perm[s.nperm++] = L.axis(r, c, leg);
        n = mul(n, L.dim(L.bond(r, c, leg)));
        bnd.push_back(L.bond(r, c, leg));
      }
      s.pre = s.K = s.post = 1;
      s.N = s.out = n;
      s.flops = 0;
    } else {
      // the contracted legs (right, then down) sit side by side in the boundary
      const auto it = std::find(bnd.begin(), bnd.end(), L.bond(r, c, k_legs[0]));
      const size_t k0 = static_cast<size_t>(it - bnd.begin());
      if (it == bnd.end() || k0 + k_legs.size() > bnd.size())
        throw std::runtime_error("reverse step legs not found");
      for (size_t a = 0; a < k_legs.size(); ++a)
        if (bnd[k0 + a] != L.bond(r, c, k_legs[a])) throw std::runtime_error("reverse step legs not adjacent");
      int64_t pre = 1, post = 1, K = 1, N = 1;
      for (size_t a = 0; a < k0; ++a) pre = mul(pre, L.dim(bnd[a]));
      for (size_t a = k0 + k_legs.size(); a < bnd.size(); ++a) post = mul(post, L.dim(bnd[a]));
      for (int32_t leg : k_legs) {
        s.perm[s.nperm++] = L.axis(r, c, leg);
        K = mul(K, L.dim(L.bond(r, c, leg)));
      }
      std::vector<int32_t> nb(bnd.begin(), bnd.begin() + k0);
      for (int32_t leg : n_legs) {
        s.perm[s.nperm++] = L.axis(r, c, leg);
        N = mul(N, L.dim(L.bond(r, c, leg)));
        nb.push_back(L.bond(r, c, leg));
      }
      nb.insert(nb.end(), bnd.begin() + k0 + k_legs.size(), bnd.end());
      bnd.swap(nb);
      s.kind = STEP_ABSORB;
      s.pre = pre; s.K = K; s.N = N; s.post = post;
      s.out = mul(mul(pre, N), post);
      s.flops = mul(mul(s.out, K), 2);
    }
    p.steps.push_back(s);
    p.cut_legs = bnd;
  } catch (Overflow&) {
    err = "plan integers overflow int64";
    return TN_EOVERFLOW;
  } catch (const std::runtime_error& e) {
    err = e.what();
    return TN_EINVAL;
  }
  p.slots = p.steps.size() > 1 ? 1 : 0;
  p.units.clear();
  Unit U;
  U.frame = FRAME_ID; U.rows = 1; U.cols = 1; U.result = p.steps.back().out;
  U.first_step = 0; U.n_steps = static_cast<int32_t>(p.steps.size());
  p.units.push_back(U);
  p.is_cut = true;
  p.cut_mirror = 2;
  p.cut_open_end = true;
  try {
    finish(p);
  } catch (Overflow&) {
    err = "plan integers overflow int64";
    return TN_EOVERFLOW;
  }
  out = std::move(p);
  return TN_OK;
}

namespace {
void ints(std::ostringstream& os, const std::vector<int32_t>& v) {
  if (v.empty()) { os << "-"; return; }
  for (size_t k = 0; k < v.size(); ++k) os << (k ? "," : "") << v[k];
}
}  // namespace

std::string plan_text(const Plan& p) {
  std::ostringstream os;
  os << "tnplan v1 rows=" << p.rows << " cols=" << p.cols
     << " requested=" << kOrderName[p.requested] << " order=" << kOrderName[p.order]
     << " transpose=" << p.transpose << " quad=" << p.qh << "," << p.qw << "\n";
  os << "hdim "; ints(os, p.hdim); os << "\n";
  os << "vdim "; ints(os, p.vdim); os << "\n";
  for (size_t u = 0; u < p.units.size(); ++u) {
    const Unit& U = p.units[u];
    os << "unit " << u << " frame=" << kFrameName[U.frame] << " rows=" << U.rows
       << " cols=" << U.cols << " result=" << U.result << "\n";
  }
  for (size_t k = 0; k < p.steps.size(); ++k) {
    const Step& s = p.steps[k];
    os << "step " << k << " unit=" << s.unit << " site=" << s.r << "," << s.c
       << " kind=" << (s.kind == STEP_INIT ? "INIT" : (s.kind == STEP_SEED ? "SEED" : "ABSORB"))
       << " pre=" << s.pre
       << " K=" << s.K << " N=" << s.N << " post=" << s.post << " perm=";
    if (s.nperm == 0) os << "-";
    for (int32_t a = 0; a < s.nperm; ++a) os << (a ? "." : "") << s.perm[a];
    os << " out=" << s.out << " flops=" << s.flops << " rescale=";
    if (s.rescale >= 0) os << s.rescale; else os << "-";
    os << "\n";
  }
  if (p.has_ring) {
    const Ring& g = p.ring;
    os << "ring xa=" << g.xa << " xb=" << g.xb << " ya=" << g.ya << " yb=" << g.yb
       << " m=" << g.m << " n=" << g.n << " kx=" << g.kx << " ky=" << g.ky
       << " flops=" << g.flops << "\n";
  }
  for (size_t k = 0; k < p.chain.size(); ++k) {
    const Link& lk = p.chain[k];
    os << "link " << k << " unit=" << lk.unit << " side=" << lk.side << " K=" << lk.K
       << " N=" << lk.N << " flops=" << lk.flops << " rescale=";
    if (lk.rescale >= 0) os << lk.rescale; else os << "-";
    os << "\n";
  }
  os << "totals steps=" << p.steps.size() << " slots=" << p.slots << " peak=" << p.peak
     << " flops=" << p.flops << " moved=" << p.moved << "\n";
  return os.str();
}

}  // namespace tn
