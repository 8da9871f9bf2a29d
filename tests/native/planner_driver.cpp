// Drives the C++ planner over every lattice shape 1..12 x 1..12, bond
// dimensions 1..5 (uniform and mixed), every order and every quadrant split,
// checking the plan's bookkeeping on the way, and every column-sweep cut plan
// of those shapes.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitized.py (host code only).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "plan.hpp"

namespace {

int fails = 0;

void check(bool ok, const char* what, int r, int c, int D, int order) {
  if (!ok) {
    std::fprintf(stderr, "FAIL %s: %dx%d D=%d order=%d\n", what, r, c, D, order);
    ++fails;
  }
}

void run(int r, int c, int D, const int32_t* h, const int32_t* v, int order, int qh, int qw,
         long& plans) {
  tn_grid g{r, c, D, h, v};
  tn::Plan p;
  std::string err;
  const tn_status s = tn::build_plan(g, order, qh, qw, p, err);
  if (s != TN_OK) {
    // QUADRANT needs two rows and two columns; splits must be inside the lattice
    const bool quad_ok = r >= 2 && c >= 2 && qh >= 0 && qh < r && qw >= 0 && qw < c;
    // the row scheme's D^(2L) row tensors may not fit int64
    const bool rows_big = (order == TN_ORDER_ROWS || order == TN_ORDER_ROWS_T) && s == TN_EOVERFLOW;
    check((order == TN_ORDER_QUADRANT && !quad_ok) || rows_big, "unexpected planning error", r, c,
          D, order);
    return;
  }
  ++plans;
  check(!p.steps.empty() && p.peak >= 1 && p.flops >= 0, "empty plan", r, c, D, order);
  int64_t f = 0;
  for (const tn::Step& st : p.steps) {
    check(st.pre >= 1 && st.K >= 1 && st.N >= 1 && st.post >= 1, "step dims", r, c, D, order);
    check(st.out == st.pre * st.N * st.post, "step out", r, c, D, order);
    check(st.out <= p.peak, "peak", r, c, D, order);
    f += st.flops;
  }
  int64_t fl = 0;
  for (const tn::Link& lk : p.chain) fl += lk.flops;
  check(f + (p.has_ring ? p.ring.flops : 0) + fl == p.flops, "flop total", r, c, D, order);
  // the row chain: each link sums the previous output (the first row's
  // tensor first) against a row tensor of K x N entries; the last one ends
  // in the scalar; every slot scales exactly the tensor measured into it
  if (!p.chain.empty()) {
    int64_t k = p.units[0].result;
    int32_t vslot = p.units[0].final_slot;
    for (size_t i = 0; i < p.chain.size(); ++i) {
      const tn::Link& lk = p.chain[i];
      const bool last = i + 1 == p.chain.size();
      check(lk.K == k && p.units[lk.unit].result == lk.K * lk.N && lk.scale_v == vslot &&
                (last ? (lk.N == 1 && lk.rescale < 0) : lk.rescale >= 0) &&
                lk.unit == static_cast<int32_t>(i + 1),
            "row chain", r, c, D, order);
      k = lk.N;
      vslot = lk.rescale;
    }
  }
  // under a budget just below this plan's storage an explicit order is
  // refused, and the heuristic returns a plan within the budget or nothing
  if (p.buffers > 1 && order != TN_ORDER_SWEEP_AUTO) {
    tn::Plan q;
    const tn_status sb = tn::build_plan(g, order, qh, qw, q, err, p.buffers - 1);
    if (order == TN_ORDER_HEURISTIC)
      check(sb == TN_ENOMEM || (sb == TN_OK && q.buffers <= p.buffers - 1 && q.peak >= p.peak),
            "budgeted heuristic", r, c, D, order);
    else
      check(sb == TN_ENOMEM, "budget refused", r, c, D, order);
  }
  const std::string t = tn::plan_text(p);
  check(t.rfind("tnplan v1", 0) == 0, "plan text", r, c, D, order);
}

// Cut plans of the column sweep (cached environments): the same steps as the
// full sweep over their columns, a SEED step exactly when they start inside
// the lattice, rescale slots renumbered from the seed, and left and right
// cuts at the same column ending in the same bonds in the same order.
void run_cuts(int r, int c, int D, const int32_t* h, const int32_t* v, long& plans) {
  tn_grid g{r, c, D, h, v};
  tn::Plan full;
  std::string err;
  if (tn::build_plan(g, TN_ORDER_COLSWEEP, 0, 0, full, err) != TN_OK) return;
  for (int mirror = 0; mirror < 2; ++mirror)
    for (int c0 = 0; c0 < c; ++c0)
      for (int c1 = c0 + 1; c1 <= c; ++c1) {
        tn::Plan p;
        if (tn::build_cut_plan(g, mirror, c0, c1, p, err) != TN_OK) {
          check(false, "cut plan error", r, c, D, 100 + mirror);
          continue;
        }
        ++plans;
        // entries of the boundary after `cols` local columns: its h bonds
        auto bnd = [&](int cols) {
          int64_t e = 1;
          const int bc = mirror ? c - 1 - cols : cols - 1;
          for (int rr = 0; rr < r; ++rr) e *= h ? h[rr * (c - 1) + bc] : D;
          return e;
        };
        const int seed = c0 > 0 ? 1 : 0;
        check(static_cast<int>(p.steps.size()) == seed + (c1 - c0) * r, "cut step count", r, c, D, 100);
        check(p.is_cut && p.cut_c0 == c0 && p.cut_c1 == c1, "cut fields", r, c, D, 100);
        if (seed) {
          check(p.steps[0].kind == tn::STEP_SEED && p.steps[0].rescale == 0 &&
                    p.steps[0].out == bnd(c0) &&
                    (mirror || p.steps[0].out == full.steps[static_cast<size_t>(c0) * r - 1].out),
                "seed step", r, c, D, 100 + mirror);
        }
        const int off = c0 > 0 ? c0 - 1 : 0;
        for (size_t k = seed; k < p.steps.size(); ++k) {
          const tn::Step& s = p.steps[k];
          const int j = c0 + static_cast<int>(k - seed) / r;        // local column
          const int i = static_cast<int>(k - seed) % r;             // local row
          const int cc = mirror ? c - 1 - j : j;
          check(s.r == i && s.c == cc, "cut step site", r, c, D, 100 + mirror);
          const bool resc = (i == r - 1) && j < c - 1;
          check((s.rescale >= 0) == resc && (!resc || s.rescale == j - off), "cut rescale", r, c,
                D, 100 + mirror);
          if (k > 0 && s.kind == tn::STEP_ABSORB)
            check(s.scale_in == p.steps[k - 1].rescale, "cut scale_in", r, c, D, 100 + mirror);
          if (!mirror) {
            const tn::Step& f = full.steps[static_cast<size_t>(c0) * r + (k - seed)];
            bool same = f.kind == s.kind && f.pre == s.pre && f.K == s.K && f.N == s.N &&
                        f.post == s.post && f.nperm == s.nperm;
            for (int a = 0; a < f.nperm; ++a) same = same && f.perm[a] == s.perm[a];
            check(same, "cut step differs from the full sweep", r, c, D, 100);
          }
        }
        if (c1 < c) check(p.steps.back().out == bnd(c1), "cut boundary entries", r, c, D, 100 + mirror);
        else check(p.steps.back().out == 1, "cut scalar end", r, c, D, 100 + mirror);
      }
  // step-granular cuts: the full sweep's steps from any step k0, to the next
  // step, the end of a column or the end of the sweep
  const int64_t total = static_cast<int64_t>(r) * c;
  for (int64_t k0 = 0; k0 < total; ++k0) {
    for (int64_t k1 : {k0 + 1, std::min<int64_t>(total, k0 + r), total}) {
      tn::Plan p;
      if (tn::build_sweep_cut(g, 0, k0, k1, p, err) != TN_OK) {
        check(false, "step cut error", r, c, D, 103);
        continue;
      }
      ++plans;
      const int seed = k0 > 0 ? 1 : 0;
      bool same = static_cast<int64_t>(p.steps.size()) == seed + (k1 - k0) &&
                  p.cut_open_end == (k1 < total);
      if (seed) same = same && p.steps[0].kind == tn::STEP_SEED && p.steps[0].out == full.steps[k0 - 1].out;
      for (int64_t k = k0; same && k < k1; ++k) {
        const tn::Step& f = full.steps[k];
        const tn::Step& q = p.steps[seed + (k - k0)];
        same = f.kind == q.kind && f.pre == q.pre && f.K == q.K && f.N == q.N && f.post == q.post &&
               (f.rescale >= 0) == (q.rescale >= 0) && q.last_col == f.last_col;
        if (k > k0 || seed) same = same && (q.kind != tn::STEP_ABSORB || q.scale_in ==
                                            p.steps[seed + (k - k0) - 1].rescale);
      }
      check(same, "step cut differs from the full sweep", r, c, D, 103);
    }
  }
  // reverse steps inside a column: each ends in the bonds the sweep has after
  // the site above, and chains from the right environment (or the corner)
  for (int cc = 0; cc < c; ++cc) {
    std::vector<int32_t> prev;
    if (cc < c - 1) {
      tn::Plan e;
      if (tn::build_cut_plan(g, 1, 0, c - 1 - cc, e, err) == TN_OK) prev = e.cut_legs;
      else check(false, "right environment error", r, c, D, 104);
    }
    for (int rr = r - 1; rr >= 1; --rr) {
      tn::Plan q, f;
      if (tn::build_rev_step(g, rr, cc, q, err) != TN_OK ||
          tn::build_sweep_cut(g, 0, 0, static_cast<int64_t>(cc) * r + rr, f, err) != TN_OK) {
        check(false, "reverse step error", r, c, D, 104);
        break;
      }
      ++plans;
      const bool starts = rr == r - 1 && cc == c - 1;
      bool ok = q.cut_legs == f.cut_legs && q.cut_open_end;
      ok = ok && (starts ? (q.steps.size() == 1 && q.steps[0].kind == tn::STEP_INIT)
                         : (q.steps.size() == 2 && q.steps[0].kind == tn::STEP_SEED &&
                            q.steps[1].kind == tn::STEP_ABSORB && q.steps[1].scale_in == 0));
      if (!starts) {
        int64_t n = 1;
        for (int32_t b : prev) {
          const int nh = r * (c - 1);
          n *= b < nh ? (h ? h[b] : D) : (v ? v[b - nh] : D);
        }
        ok = ok && q.steps[0].out == n;
      }
      check(ok, "reverse step legs", r, c, D, 104);
      prev = q.cut_legs;
    }
  }
  // the full sweep's boundary legs after every step: every forward cut ends
  // in them, every right environment and reverse step (the boundary of all
  // sites after a step, as site environments and caps read it) too
  {
    std::vector<std::vector<int32_t>> legs;
    if (tn::sweep_legs(g, legs, err) != TN_OK || legs.size() != static_cast<size_t>(total)) {
      check(false, "sweep legs", r, c, D, 105);
    } else {
      for (int64_t k = 0; k + 1 < total; ++k) {
        tn::Plan f;
        if (tn::build_sweep_cut(g, 0, 0, k + 1, f, err) != TN_OK || f.cut_legs != legs[k])
          check(false, "forward cut legs", r, c, D, 105);
        const int rr = static_cast<int>((k + 1) % r), cc = static_cast<int>((k + 1) / r);
        tn::Plan q;
        if (rr == 0) {   // after a whole column: the right environment at that cut
          if (cc < c && (tn::build_cut_plan(g, 1, 0, c - cc, q, err) != TN_OK || q.cut_legs != legs[k]))
            check(false, "right environment legs", r, c, D, 105);
        } else if (tn::build_rev_step(g, rr, cc, q, err) != TN_OK || q.cut_legs != legs[k]) {
          // the reverse step at (rr, cc) ends in the boundary after (rr - 1, cc)
          check(false, "reverse step legs vs sweep", r, c, D, 105);
        }
      }
    }
  }
  // a left cut ending at column cut q meets the right cut ending there
  for (int q = 1; q < c; ++q) {
    tn::Plan a, b;
    if (tn::build_cut_plan(g, 0, q - 1, q, a, err) != TN_OK ||
        tn::build_cut_plan(g, 1, c - 1 - q, c - q, b, err) != TN_OK) {
      check(false, "cut pair error", r, c, D, 102);
      continue;
    }
    check(a.cut_legs == b.cut_legs && static_cast<int>(a.cut_legs.size()) == r, "cut legs differ",
          r, c, D, 102);
  }
}

}  // namespace

int main() {
  long plans = 0;
  for (int r = 1; r <= 12; ++r)
    for (int c = 1; c <= 12; ++c) {
      std::vector<int32_t> h(static_cast<size_t>(r) * (c > 1 ? c - 1 : 0));
      std::vector<int32_t> v(static_cast<size_t>(r > 1 ? r - 1 : 0) * c);
      for (size_t i = 0; i < h.size(); ++i) h[i] = 1 + static_cast<int32_t>((i * 7 + 3) % 4);
      for (size_t i = 0; i < v.size(); ++i) v[i] = 1 + static_cast<int32_t>((i * 5 + 1) % 4);
      for (int D = 1; D <= 5; ++D)
        for (int order = 0; order < 6; ++order) {
          run(r, c, D, nullptr, nullptr, order, 0, 0, plans);
          if (order == TN_ORDER_QUADRANT)
            for (int qh = 1; qh < r; ++qh)
              for (int qw = 1; qw < c; ++qw) run(r, c, D, nullptr, nullptr, order, qh, qw, plans);
        }
      for (int order = 0; order < 6; ++order)
        run(r, c, 1, h.empty() ? nullptr : h.data(), v.empty() ? nullptr : v.data(), order, 0, 0,
            plans);
      for (int D = 1; D <= 3; ++D) run_cuts(r, c, D, nullptr, nullptr, plans);
      run_cuts(r, c, 1, h.empty() ? nullptr : h.data(), v.empty() ? nullptr : v.data(), plans);
    }
  // invalid grids are rejected, not crashed on
  std::string err;
  tn::Plan p;
  tn_grid bad{0, 3, 2, nullptr, nullptr};
  if (tn::build_plan(bad, TN_ORDER_COLSWEEP, 0, 0, p, err) == TN_OK) ++fails;
  tn_grid bad2{3, 3, 0, nullptr, nullptr};
  if (tn::build_plan(bad2, TN_ORDER_COLSWEEP, 0, 0, p, err) == TN_OK) ++fails;
  std::printf("plans %ld fails %d\n", plans, fails);
  return fails ? 1 : 0;
}
