// Drives the C++ planner over every lattice shape 1..12 x 1..12, bond
// dimensions 1..5 (uniform and mixed), every order and every quadrant split,
// checking the plan's bookkeeping on the way.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitized.py (host code only).
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
    check(order == TN_ORDER_QUADRANT && !quad_ok, "unexpected planning error", r, c, D, order);
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
  check(f + (p.has_ring ? p.ring.flops : 0) == p.flops, "flop total", r, c, D, order);
  const std::string t = tn::plan_text(p);
  check(t.rfind("tnplan v1", 0) == 0, "plan text", r, c, D, order);
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
        for (int order = 0; order < 4; ++order) {
          run(r, c, D, nullptr, nullptr, order, 0, 0, plans);
          if (order == TN_ORDER_QUADRANT)
            for (int qh = 1; qh < r; ++qh)
              for (int qw = 1; qw < c; ++qw) run(r, c, D, nullptr, nullptr, order, qh, qw, plans);
        }
      for (int order = 0; order < 4; ++order)
        run(r, c, 1, h.empty() ? nullptr : h.data(), v.empty() ? nullptr : v.data(), order, 0, 0,
            plans);
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
