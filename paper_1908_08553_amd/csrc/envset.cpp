// Cached column environments for families of networks that share all but a
// few sites.
//
// Paper §5: every local observable <O> is a full contraction of O|Psi>
// against <Psi|, and those networks differ from the norm network only at the
// sites the operator touches.  The column sweep of §4 passes a boundary from
// column to column, so the boundary of the norm network after columns
// 0..c-1 (left environment L_c) is also the boundary of every network whose
// changed sites lie in columns >= c, and the sweep from the right edge gives
// the right environments R_c.  A network whose changed sites span columns
// [c0, c1) is then L_c0, the absorption of columns c0..c1-1 with its own
// sites, and a dot with R_c1: the same pairwise contractions as the full
// sweep up to column c1-1, then one boundary contraction instead of the
// remaining columns.  With c1 = cols it is the full sweep's own arithmetic.
//
// Inside a column the same holds row by row: the norm network's boundary just
// before sweep step k is the seed of every network whose first changed site
// is step k, and the boundary of all sites after step k, built from the right
// environment by reverse steps that keep the sweep's leg order, closes every
// network whose last changed site is step k.  A single site then costs one
// absorption step and a dot.
//
// Everything is issued without waiting, except the final result copy: the
// left and right environment sweeps (one cut plan per column, each in its own
// workspace region, which keeps its ending boundary for the rest of the run)
// on the caller's stream and a side stream; then the forward and reverse
// chains inside every column, dealt over S streams; then the base network and
// every network, dealt round-robin over the S streams (each with its own
// region), all joined back into the caller's stream.
#include "envset.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <utility>
#include <vector>

#include "device.hpp"
#include "exec.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace tn {

struct EnvSetImpl {
  int32_t R = 0, C = 0, prec = 0, n = 0;
  std::vector<Plan> left, right;            // cut [j, j+1), left to right / right to left
  // Inside columns (rows_on): fwd[k] = sweep step k alone, for rows 0..R-2 of
  // each column (its boundary is the one before step k+1); rev[k] = the
  // reverse step at site k, for rows 1..R-1 (its boundary is all sites after
  // step k-1).  Indexed by sweep step k = c * R + r; unused entries empty.
  bool rows_on = false;
  std::vector<Plan> fwd, rev;
  std::vector<Plan> cuts;                   // distinct network plans
  std::vector<int32_t> net_plan;            // n + 1 entries (0: base network; -1: site path)
  // Single-site networks through site environments (with rows_on): per site,
  // the shapes around its sweep step and the networks (index, substitution)
  // that replace it.
  struct SiteWork {
    int64_t k;
    SiteEnvArgs args;                       // pointers and partials filled per run
    SiteDot fold;                           // site pointer and output filled per run
    std::vector<std::pair<int32_t, int32_t>> nets;
  };
  std::vector<SiteWork> sites_work;
  size_t site_partials_off = 0, site_partials_bytes = 0;
  std::vector<int32_t> sub_first, sub_count, sub_site;
  std::vector<size_t> left_off, right_off, fwd_off, rev_off;
  int32_t S = 1;                            // streams the networks are spread over
  size_t shared_off = 0, shared_bytes = 0, recs_off = 0, partials_off = 0, partials_bytes = 0,
         results_off = 0;
  size_t total = 0;
  char* ws = nullptr;
  std::vector<std::unique_ptr<HostKeep>> keeps;
  std::vector<const double*> sites;         // scratch site table of one network
  std::vector<hipStream_t> side;            // S - 1 streams beside the caller's
  std::vector<hipEvent_t> ev;               // start, then S per barrier (two) and S for the join

  ~EnvSetImpl() {
    for (hipStream_t st : side) (void)hipStreamDestroy(st);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  // exponent records: 2 (C-1) column environments, then R C forward and R C
  // reverse ones indexed by sweep step
  size_t n_recs() const { return static_cast<size_t>(2 * (C - 1) + 2 * R * C); }
};

int32_t g_env_streams = 4;
void set_env_streams(int32_t n) { g_env_streams = n; }
int32_t g_env_rows = 32;
void set_env_rows(int32_t gib) { g_env_rows = gib; }
int32_t g_env_sites = 1;
void set_env_sites(int32_t on) { g_env_sites = on ? 1 : 0; }

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

tn_status layout(EnvSetImpl& es, const tn_grid& grid, int32_t n, const int32_t* n_subst,
                 const int32_t* subst_site, std::string& err) {
  Plan full;
  tn_status s = build_plan(grid, TN_ORDER_COLSWEEP, 0, 0, full, err);
  if (s != TN_OK) return s;
  const int32_t R = full.rows, C = full.cols;
  const int64_t total_steps = static_cast<int64_t>(R) * C;
  es.R = R; es.C = C; es.n = n;
  if (n < 0) { err = "negative network count"; return TN_EINVAL; }
  if (n > 0 && !n_subst) { err = "null substitution counts"; return TN_EINVAL; }
  es.sub_first.assign(n, 0);
  es.sub_count.assign(n, 0);
  int64_t total_sub = 0;
  for (int32_t k = 0; k < n; ++k) {
    if (n_subst[k] < 0 || n_subst[k] > R * C) { err = "bad substitution count"; return TN_EINVAL; }
    es.sub_first[k] = static_cast<int32_t>(total_sub);
    es.sub_count[k] = n_subst[k];
    total_sub += n_subst[k];
  }
  if (total_sub > 0 && !subst_site) { err = "null substitution sites"; return TN_EINVAL; }
  es.sub_site.assign(subst_site, subst_site + total_sub);

  for (int32_t j = 0; j + 1 < C; ++j) {
    for (int32_t m = 0; m < 2; ++m) {
      Plan p;
      s = build_cut_plan(grid, m, j, j + 1, p, err);
      if (s != TN_OK) return s;
      (m ? es.right : es.left).push_back(std::move(p));
    }
  }
  // environments inside columns, if their regions fit the budget
  es.rows_on = false;
  es.fwd.clear();
  es.rev.clear();
  if (g_env_rows && R > 1) {
    es.fwd.resize(static_cast<size_t>(total_steps));
    es.rev.resize(static_cast<size_t>(total_steps));
    size_t bytes = 0;
    for (int32_t c = 0; c < C; ++c)
      for (int32_t r = 0; r < R; ++r) {
        const int64_t k = static_cast<int64_t>(c) * R + r;
        if (r < R - 1) {
          s = build_sweep_cut(grid, 0, k, k + 1, es.fwd[k], err);
          if (s != TN_OK) return s;
          bytes += align_up(make_layout(es.fwd[k], es.prec).total);
        }
        if (r >= 1) {
          s = build_rev_step(grid, r, c, es.rev[k], err);
          if (s != TN_OK) return s;
          bytes += align_up(make_layout(es.rev[k], es.prec).total);
        }
      }
    es.rows_on = bytes <= (static_cast<size_t>(g_env_rows) << 30);
    if (!es.rows_on) { es.fwd.clear(); es.rev.clear(); }
  }

  std::map<std::pair<int64_t, int64_t>, int32_t> index;
  auto plan_for = [&](int64_t k0, int64_t k1, int32_t* out) -> tn_status {
    const auto key = std::make_pair(k0, k1);
    auto it = index.find(key);
    if (it != index.end()) { *out = it->second; return TN_OK; }
    Plan p;
    const tn_status st = build_sweep_cut(grid, 0, k0, k1, p, err);
    if (st != TN_OK) return st;
    es.cuts.push_back(std::move(p));
    *out = index[key] = static_cast<int32_t>(es.cuts.size() - 1);
    return TN_OK;
  };
  es.net_plan.assign(n + 1, 0);
  // the base network: the last column from the left environment (the full
  // sweep's own arithmetic)
  s = plan_for(total_steps - R, total_steps, &es.net_plan[0]);
  if (s != TN_OK) return s;
  es.sites_work.clear();
  std::map<int64_t, size_t> site_index;
  for (int32_t k = 0; k < n; ++k) {
    if (es.rows_on && g_env_sites && es.sub_count[k] == 1) {
      const int32_t site = es.sub_site[es.sub_first[k]];
      if (site < 0 || site >= R * C) { err = "substituted site out of range"; return TN_EINVAL; }
      const int64_t step = static_cast<int64_t>(site % C) * R + site / C;
      const Step& st = full.steps[step];
      // measured: a site environment beats absorbing and closing each
      // single-site network while the boundary around the step stays within
      // about 2^20 entries (8 x 8 at chi = 2), not at 4^11 (10 x 10)
      if (st.K * st.N <= kSiteEnvMaxXY && st.pre * std::max(st.K, st.N) * st.post <= (1 << 20)) {
        auto it = site_index.find(step);
        if (it == site_index.end()) {
          EnvSetImpl::SiteWork w;
          w.k = step;
          std::memset(&w.args, 0, sizeof(w.args));
          w.args.P = st.pre; w.args.Q = st.post;
          w.args.X = static_cast<int32_t>(st.K); w.args.Y = static_cast<int32_t>(st.N);
          w.args.l_f64 = (es.prec == TN_PREC_F64 || (step > 0 && full.steps[step - 1].last_col)) ? 1 : 0;
          w.args.r_f64 = (es.prec == TN_PREC_F64 || st.last_col) ? 1 : 0;
          w.args.blocks = site_env_blocks(st.pre, st.post, w.args.X, w.args.Y);
          // the site folded as the step folds it: canonical dims and strides
          std::memset(&w.fold, 0, sizeof(w.fold));
          int32_t cdims[4];
          int64_t cstr[4];
          int32_t nd = 0;
          const int32_t r = st.r, c = st.c;
          if (c > 0) cdims[nd++] = full.hdim[static_cast<size_t>(r) * (C - 1) + c - 1];
          if (r > 0) cdims[nd++] = full.vdim[static_cast<size_t>(r - 1) * C + c];
          if (c < C - 1) cdims[nd++] = full.hdim[static_cast<size_t>(r) * (C - 1) + c];
          if (r < R - 1) cdims[nd++] = full.vdim[static_cast<size_t>(r) * C + c];
          int64_t stride = 1;
          for (int32_t a = nd - 1; a >= 0; --a) { cstr[a] = stride; stride *= cdims[a]; }
          w.fold.ndim = st.nperm;
          for (int32_t a = 0; a < st.nperm; ++a) {
            w.fold.dims[a] = cdims[st.perm[a]];
            w.fold.cstride[a] = cstr[st.perm[a]];
          }
          it = site_index.emplace(step, es.sites_work.size()).first;
          es.sites_work.push_back(w);
        }
        es.sites_work[it->second].nets.push_back({k, es.sub_first[k]});
        es.net_plan[k + 1] = -1;
        continue;
      }
    }
    int64_t k0 = total_steps - R, k1 = total_steps - 1;   // no substitution: the base network
    if (es.sub_count[k] > 0) {
      k0 = total_steps; k1 = -1;
      std::vector<int32_t> seen;
      for (int32_t i = 0; i < es.sub_count[k]; ++i) {
        const int32_t site = es.sub_site[es.sub_first[k] + i];
        if (site < 0 || site >= R * C) { err = "substituted site out of range"; return TN_EINVAL; }
        if (std::find(seen.begin(), seen.end(), site) != seen.end()) {
          err = "a site is substituted twice in one network";
          return TN_EINVAL;
        }
        seen.push_back(site);
        const int64_t step = static_cast<int64_t>(site % C) * R + site / C;   // sweep order
        k0 = std::min(k0, step);
        k1 = std::max(k1, step);
      }
      if (!es.rows_on) {   // whole columns between column environments
        k0 = k0 / R * R;
        k1 = k1 / R * R + R - 1;
      }
    }
    s = plan_for(k0, k1 + 1, &es.net_plan[k + 1]);
    if (s != TN_OK) return s;
  }

  // a network's seed and cap, and a site environment's two boundaries, are
  // the environments at its cuts: the same bonds in the same order as the
  // full sweep's boundary there (a planner invariant, checked once here, bond
  // by bond)
  std::vector<std::vector<int32_t>> legs;
  s = sweep_legs(grid, legs, err);
  if (s != TN_OK) return s;
  auto seed_env = [&](int64_t k) -> const Plan& {   // boundary before step k
    return (k % R == 0) ? es.left[k / R - 1] : es.fwd[k - 1];
  };
  auto cap_env = [&](int64_t k) -> const Plan& {    // all sites after step k
    return (k % R == R - 1) ? es.right[C - 2 - k / R] : es.rev[k + 1];
  };
  for (const Plan& p : es.cuts) {
    if (p.cut_k0 > 0) {
      const int64_t k = p.cut_k0;
      const Plan& l = seed_env(k);
      if (l.cut_legs != legs[k - 1] || l.steps.back().out != p.steps[0].out) {
        err = "seed does not match its environment";
        return TN_EINVAL;
      }
    }
    if (p.cut_open_end) {
      const int64_t k = p.cut_k1 - 1;
      const Plan& r = cap_env(k);
      if (p.cut_legs != r.cut_legs || p.cut_legs != legs[k]) {
        err = "cap does not match its environment";
        return TN_EINVAL;
      }
    }
  }
  for (const auto& w : es.sites_work) {
    if (w.k > 0 && seed_env(w.k).cut_legs != legs[w.k - 1]) {
      err = "site environment: boundary before the step out of leg order";
      return TN_EINVAL;
    }
    if (w.k < total_steps - 1 && cap_env(w.k).cut_legs != legs[w.k]) {
      err = "site environment: boundary after the step out of leg order";
      return TN_EINVAL;
    }
  }
  es.S = g_env_streams;
  size_t off = 0;
  auto place = [&](const std::vector<Plan>& plans, std::vector<size_t>& offs) {
    offs.assign(plans.size(), 0);
    for (size_t i = 0; i < plans.size(); ++i) {
      if (plans[i].steps.empty()) continue;
      offs[i] = off;
      off += align_up(make_layout(plans[i], es.prec).total);
    }
  };
  place(es.left, es.left_off);
  place(es.right, es.right_off);
  place(es.fwd, es.fwd_off);
  place(es.rev, es.rev_off);
  es.shared_off = off;
  es.shared_bytes = 0;
  int64_t parts = 1;
  for (const Plan& p : es.cuts) {
    es.shared_bytes = std::max(es.shared_bytes, align_up(make_layout(p, es.prec).total));
    if (p.cut_open_end) parts = std::max(parts, env_cap_blocks(p.steps.back().out));
  }
  off += es.shared_bytes * es.S;
  es.site_partials_bytes = 0;
  for (const auto& w : es.sites_work)
    es.site_partials_bytes = std::max(es.site_partials_bytes,
                                      align_up(sizeof(double) * static_cast<size_t>(w.args.blocks) *
                                               w.args.X * w.args.Y));
  es.site_partials_off = off;
  off += es.site_partials_bytes * es.S;
  es.recs_off = off;
  off = align_up(off + sizeof(EnvRec) * std::max<size_t>(es.n_recs(), 1));
  es.partials_off = off;
  es.partials_bytes = align_up(sizeof(double) * static_cast<size_t>(parts));
  off += es.partials_bytes * es.S;
  es.results_off = off;
  off = align_up(off + sizeof(tn_result) * static_cast<size_t>(n + 1));
  es.total = off;
  return TN_OK;
}

}  // namespace

tn_status envset_workspace(const tn_grid& grid, int32_t prec, int32_t n, const int32_t* n_subst,
                           const int32_t* subst_site, size_t* bytes, std::string& err) {
  EnvSetImpl es;
  es.prec = prec;
  const tn_status s = layout(es, grid, n, n_subst, subst_site, err);
  if (s != TN_OK) return s;
  *bytes = es.total;
  return TN_OK;
}

tn_status envset_create(const tn_grid& grid, int32_t prec, int32_t n, const int32_t* n_subst,
                        const int32_t* subst_site, void* ws, size_t ws_bytes, EnvSetImpl** out,
                        std::string& err) {
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) {
    err = "workspace must be 256-byte aligned";
    return TN_EINVAL;
  }
  auto es = std::make_unique<EnvSetImpl>();
  es->prec = prec;
  const tn_status s = layout(*es, grid, n, n_subst, subst_site, err);
  if (s != TN_OK) return s;
  if (ws_bytes < es->total) {
    err = "environment workspace too small: need " + std::to_string(es->total) + " bytes";
    return TN_ENOMEM;
  }
  es->ws = static_cast<char*>(ws);
  for (int32_t i = 0; i + 1 < es->S; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      err = "hipStreamCreateWithFlags failed";
      return TN_EDEVICE;
    }
    es->side.push_back(st);
  }
  for (int32_t i = 0; es->S > 1 && i < 1 + 3 * es->S; ++i) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      err = "hipEventCreateWithFlags failed";
      return TN_EDEVICE;
    }
    es->ev.push_back(e);
  }
  size_t calls = es->left.size() + es->right.size() + static_cast<size_t>(n) + 1;
  for (const Plan& p : es->fwd) calls += p.steps.empty() ? 0 : 1;
  for (const Plan& p : es->rev) calls += p.steps.empty() ? 0 : 1;
  for (size_t i = 0; i < calls; ++i) es->keeps.push_back(std::make_unique<HostKeep>());
  es->keeps.push_back(std::make_unique<HostKeep>());   // result records
  es->sites.resize(static_cast<size_t>(es->R) * es->C);
  *out = es.release();
  return TN_OK;
}

tn_status envset_run(EnvSetImpl* es, const double* const* base, const double* const* subst,
                     hipStream_t stream, tn_result* outs, std::string& err) {
  const int32_t R = es->R, C = es->C, n = es->n;
  for (int32_t s = 0; s < R * C; ++s)
    if (!base[s]) { err = "null site pointer"; return TN_EINVAL; }
  const size_t total_sub = es->sub_site.size();
  for (size_t i = 0; i < total_sub; ++i)
    if (!subst || !subst[i]) { err = "null substituted site pointer"; return TN_EINVAL; }

  char* ws = es->ws;
  EnvRec* recs = reinterpret_cast<EnvRec*>(ws + es->recs_off);
  tn_result* results = reinterpret_cast<tn_result*>(ws + es->results_off);
  const int32_t S = es->S;
  const int64_t total_steps = static_cast<int64_t>(R) * C;
  std::vector<hipStream_t> streams{stream};
  for (hipStream_t st : es->side) streams.push_back(st);
  std::vector<std::unique_ptr<LaunchTimer>> timers;
  for (hipStream_t st : streams) timers.push_back(std::make_unique<LaunchTimer>(st));
  // one stream needs no events: stream order alone serialises the work
  const bool multi = S > 1;
  size_t call = 0;
  const int32_t ne = C - 1;
  EnvRec* lrec = recs;                              // column environments
  EnvRec* rrec = recs + ne;
  EnvRec* frec = recs + 2 * ne;                     // inside columns, by sweep step
  EnvRec* vrec = frec + total_steps;
  std::vector<const void*> ltap(ne, nullptr), rtap(ne, nullptr);
  std::vector<const void*> ftap(es->rows_on ? total_steps : 0, nullptr);
  std::vector<const void*> vtap(es->rows_on ? total_steps : 0, nullptr);
  hipError_t e = hipSuccess;
  tn_status status = TN_OK;

  // every stream waits for what every stream has issued so far
  auto barrier = [&](int32_t first_event) -> tn_status {
    if (!multi) return TN_OK;
    for (int32_t i = 0; i < S && e == hipSuccess; ++i) e = hipEventRecord(es->ev[first_event + i], streams[i]);
    for (int32_t i = 0; i < S && e == hipSuccess; ++i)
      for (int32_t j = 0; j < S && e == hipSuccess; ++j)
        if (i != j) e = hipStreamWaitEvent(streams[i], es->ev[first_event + j], 0);
    if (e != hipSuccess) { err = hipGetErrorString(e); return TN_EDEVICE; }
    return TN_OK;
  };
  auto run_env = [&](const Plan& p, size_t off, int32_t si, const void* seed, const EnvRec* seed_rec,
                     const void** tap, EnvRec* tap_rec) -> tn_status {
    CutIO io;
    io.seed = seed;
    io.seed_rec = seed_rec;
    io.tap = tap;
    io.tap_rec = tap_rec;
    return enqueue(p, base, true, es->prec, ws + off, make_layout(p, es->prec).total, streams[si],
                   *es->keeps[call++], *timers[si], err, nullptr, nullptr, &io);
  };
  // the boundary before sweep step k (seed) and after it (cap)
  auto seed_of = [&](int64_t k, const void** ptr, const EnvRec** rec) {
    if (k % R == 0) { *ptr = ltap[k / R - 1]; *rec = lrec + k / R - 1; }
    else { *ptr = ftap[k - 1]; *rec = frec + k - 1; }
  };
  auto cap_of = [&](int64_t k, const void** ptr, const EnvRec** rec) {
    if (k % R == R - 1) {
      const int64_t j = C - 2 - k / R;
      *ptr = rtap[j]; *rec = rrec + j;
    } else {
      *ptr = vtap[k + 1]; *rec = vrec + k + 1;
    }
  };

  auto issue = [&]() -> tn_status {
    if (multi) e = hipEventRecord(es->ev[0], stream);
    for (int32_t i = 1; i < S && e == hipSuccess; ++i) e = hipStreamWaitEvent(streams[i], es->ev[0], 0);
    if (e != hipSuccess) { err = hipGetErrorString(e); return TN_EDEVICE; }
    // column environments: left on the caller's stream, right on a side stream
    for (int32_t side = 0; side < 2; ++side) {
      const int32_t si = (side && S > 1) ? 1 : 0;
      for (int32_t j = 0; j < ne; ++j) {
        const tn_status st = side
            ? run_env(es->right[j], es->right_off[j], si, j > 0 ? rtap[j - 1] : nullptr,
                      j > 0 ? rrec + j - 1 : nullptr, &rtap[j], rrec + j)
            : run_env(es->left[j], es->left_off[j], si, j > 0 ? ltap[j - 1] : nullptr,
                      j > 0 ? lrec + j - 1 : nullptr, &ltap[j], lrec + j);
        if (st != TN_OK) return st;
      }
    }
    tn_status st = barrier(1);
    if (st != TN_OK) return st;
    // inside columns: per column a forward chain down from the left
    // environment and a reverse chain up from the right one, dealt over the
    // streams
    if (es->rows_on) {
      for (int32_t c = 0; c < C; ++c) {
        const int32_t sf = (2 * c) % S, sr = (2 * c + 1) % S;
        for (int32_t r = 0; r + 1 < R; ++r) {
          const int64_t k = static_cast<int64_t>(c) * R + r;
          const void* sp = nullptr;
          const EnvRec* sq = nullptr;
          if (k > 0) seed_of(k, &sp, &sq);
          st = run_env(es->fwd[k], es->fwd_off[k], sf, sp, sq, &ftap[k], frec + k);
          if (st != TN_OK) return st;
        }
        for (int32_t r = R - 1; r >= 1; --r) {
          const int64_t k = static_cast<int64_t>(c) * R + r;
          const void* sp = nullptr;
          const EnvRec* sq = nullptr;
          if (!(c == C - 1 && r == R - 1)) cap_of(k, &sp, &sq);
          st = run_env(es->rev[k], es->rev_off[k], sr, sp, sq, &vtap[k], vrec + k);
          if (st != TN_OK) return st;
        }
      }
      st = barrier(1 + S);
      if (st != TN_OK) return st;
    }
    // single-site networks: one site environment per site, dotted with each
    // replacing site
    for (size_t w = 0; w < es->sites_work.size(); ++w) {
      const int32_t si = static_cast<int32_t>(w % S);
      EnvSetImpl::SiteWork& sw = es->sites_work[w];
      SiteEnvArgs a = sw.args;
      a.L = nullptr; a.l_rec = nullptr; a.Rv = nullptr; a.r_rec = nullptr;
      if (sw.k > 0) seed_of(sw.k, &a.L, &a.l_rec);
      if (sw.k < total_steps - 1) cap_of(sw.k, &a.Rv, &a.r_rec);
      a.partials = reinterpret_cast<double*>(ws + es->site_partials_off + es->site_partials_bytes * si);
      timers[si]->before();
      e = launch_site_env(a, streams[si]);
      timers[si]->after("site_env",
                        8.0 * static_cast<double>(a.P * a.Q) * (a.X + a.Y), 2.0 * static_cast<double>(a.P * a.Q) * a.X * a.Y);
      if (e != hipSuccess) { err = std::string("site environment: ") + hipGetErrorString(e); return TN_EDEVICE; }
      for (size_t i0 = 0; i0 < sw.nets.size(); i0 += kSiteDotsMax) {
        SiteDot dots[kSiteDotsMax];
        const int32_t nd = static_cast<int32_t>(std::min<size_t>(kSiteDotsMax, sw.nets.size() - i0));
        for (int32_t i = 0; i < nd; ++i) {
          dots[i] = sw.fold;
          dots[i].site = subst[sw.nets[i0 + i].second];
          dots[i].out = results + sw.nets[i0 + i].first + 1;
        }
        timers[si]->before();
        e = launch_site_dots(a, dots, nd, streams[si]);
        timers[si]->after("site_dots", 0.0, 0.0);
        if (e != hipSuccess) { err = std::string("site dots: ") + hipGetErrorString(e); return TN_EDEVICE; }
      }
    }
    for (int32_t k = 0; k <= n; ++k) {
      const int32_t si = k % S;
      if (es->net_plan[k] < 0) continue;
      const Plan& p = es->cuts[es->net_plan[k]];
      for (int32_t t = 0; t < R * C; ++t) es->sites[t] = base[t];
      if (k > 0) {
        const int32_t f = es->sub_first[k - 1];
        for (int32_t i = 0; i < es->sub_count[k - 1]; ++i) es->sites[es->sub_site[f + i]] = subst[f + i];
      }
      CutIO io;
      if (p.cut_k0 > 0) seed_of(p.cut_k0, &io.seed, &io.seed_rec);
      if (p.cut_open_end) {
        cap_of(p.cut_k1 - 1, &io.cap, &io.cap_rec);
        io.partials = reinterpret_cast<double*>(ws + es->partials_off + es->partials_bytes * si);
      }
      io.result = results + k;
      st = enqueue(p, es->sites.data(), true, es->prec,
                   ws + es->shared_off + es->shared_bytes * si, es->shared_bytes, streams[si],
                   *es->keeps[call++], *timers[si], err, nullptr, nullptr, &io);
      if (st != TN_OK) return st;
    }
    return TN_OK;
  };
  status = issue();
  // join every side stream back into the caller's stream, also after an error
  for (int32_t i = 1; i < S; ++i) {
    hipError_t e2 = hipEventRecord(es->ev[1 + 2 * S + i], streams[i]);
    if (e2 == hipSuccess) e2 = hipStreamWaitEvent(stream, es->ev[1 + 2 * S + i], 0);
    if (e2 != hipSuccess && status == TN_OK) { err = hipGetErrorString(e2); status = TN_EDEVICE; }
  }
  if (status != TN_OK) {
    (void)hipStreamSynchronize(stream);
    return status;
  }
  HostKeep& rk = *es->keeps[call];
  tn_result* staged = reinterpret_cast<tn_result*>(rk.block(sizeof(tn_result) * (n + 1), &e));
  if (!staged) { err = std::string("hipHostMalloc: ") + hipGetErrorString(e); return TN_ENOMEM; }
  e = hipMemcpyAsync(staged, results, sizeof(tn_result) * (n + 1), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) { err = hipGetErrorString(e); return TN_EDEVICE; }
  for (auto& t : timers) t->flush();
  std::memcpy(outs, staged, sizeof(tn_result) * (n + 1));
  for (int32_t k = 0; k <= n; ++k)
    if (outs[k].status != TN_OK) {
      err = "non-finite value in network " + std::to_string(k);
      return TN_ENONFINITE;
    }
  return TN_OK;
}

void envset_destroy(EnvSetImpl* es) { delete es; }

}  // namespace tn
