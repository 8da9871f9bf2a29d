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
// Everything is issued without waiting, except the final result copy: the
// left and right environment sweeps (one cut plan per column, each in its own
// workspace region, which keeps its ending boundary for the rest of the run)
// on the caller's stream and a side stream, then the base network and every
// network, dealt round-robin over S streams (each with its own region), all
// joined back into the caller's stream.
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
  std::vector<Plan> cuts;                   // distinct network plans (left to right)
  std::vector<int32_t> net_plan;            // n + 1 entries (0: base network)
  std::vector<int32_t> sub_first, sub_count, sub_site;
  std::vector<size_t> left_off, right_off;
  int32_t S = 1;                            // streams the networks are spread over
  size_t shared_off = 0, shared_bytes = 0, recs_off = 0, partials_off = 0, partials_bytes = 0,
         results_off = 0;
  size_t total = 0;
  char* ws = nullptr;
  std::vector<std::unique_ptr<HostKeep>> keeps;
  std::vector<const double*> sites;         // scratch site table of one network
  std::vector<hipStream_t> side;            // S - 1 streams beside the caller's
  std::vector<hipEvent_t> ev;               // start, left done, right done, S stream ends

  ~EnvSetImpl() {
    for (hipStream_t st : side) (void)hipStreamDestroy(st);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

int32_t g_env_streams = 4;
void set_env_streams(int32_t n) { g_env_streams = n; }

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

tn_status layout(EnvSetImpl& es, const tn_grid& grid, int32_t n, const int32_t* n_subst,
                 const int32_t* subst_site, std::string& err) {
  Plan full;
  tn_status s = build_plan(grid, TN_ORDER_COLSWEEP, 0, 0, full, err);
  if (s != TN_OK) return s;
  const int32_t R = full.rows, C = full.cols;
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
  std::map<std::pair<int32_t, int32_t>, int32_t> index;
  auto plan_for = [&](int32_t c0, int32_t c1, int32_t* out) -> tn_status {
    const auto key = std::make_pair(c0, c1);
    auto it = index.find(key);
    if (it != index.end()) { *out = it->second; return TN_OK; }
    Plan p;
    const tn_status st = build_cut_plan(grid, 0, c0, c1, p, err);
    if (st != TN_OK) return st;
    es.cuts.push_back(std::move(p));
    *out = index[key] = static_cast<int32_t>(es.cuts.size() - 1);
    return TN_OK;
  };
  es.net_plan.assign(n + 1, 0);
  s = plan_for(C - 1, C, &es.net_plan[0]);
  if (s != TN_OK) return s;
  for (int32_t k = 0; k < n; ++k) {
    int32_t c0 = C - 1, c1 = C;
    if (es.sub_count[k] > 0) {
      c0 = C; c1 = 0;
      std::vector<int32_t> seen;
      for (int32_t i = 0; i < es.sub_count[k]; ++i) {
        const int32_t site = es.sub_site[es.sub_first[k] + i];
        if (site < 0 || site >= R * C) { err = "substituted site out of range"; return TN_EINVAL; }
        if (std::find(seen.begin(), seen.end(), site) != seen.end()) {
          err = "a site is substituted twice in one network";
          return TN_EINVAL;
        }
        seen.push_back(site);
        c0 = std::min(c0, site % C);
        c1 = std::max(c1, site % C + 1);
      }
    }
    s = plan_for(c0, c1, &es.net_plan[k + 1]);
    if (s != TN_OK) return s;
  }

  // a network's seed and cap are the environments at its column cuts: same
  // bonds in the same order (a planner invariant, checked once here)
  for (const Plan& p : es.cuts) {
    if (p.cut_c0 > 0) {
      const Plan& l = es.left[p.cut_c0 - 1];
      if (l.steps.back().out != p.steps[0].out) { err = "seed does not match its environment"; return TN_EINVAL; }
    }
    if (p.cut_c1 < C && p.cut_legs != es.right[C - 1 - p.cut_c1].cut_legs) {
      err = "cap does not match its environment";
      return TN_EINVAL;
    }
  }
  es.S = g_env_streams;
  size_t off = 0;
  for (const Plan& p : es.left) { es.left_off.push_back(off); off += align_up(make_layout(p, es.prec).total); }
  for (const Plan& p : es.right) { es.right_off.push_back(off); off += align_up(make_layout(p, es.prec).total); }
  es.shared_off = off;
  es.shared_bytes = 0;
  int64_t parts = 1;
  for (const Plan& p : es.cuts) {
    es.shared_bytes = std::max(es.shared_bytes, align_up(make_layout(p, es.prec).total));
    if (p.cut_c1 < C) parts = std::max(parts, env_cap_blocks(p.steps.back().out));
  }
  off += es.shared_bytes * es.S;
  es.recs_off = off;
  off = align_up(off + sizeof(EnvRec) * static_cast<size_t>(std::max(2 * (C - 1), 1)));
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
  for (int32_t i = 0; es->S > 1 && i < 3 + es->S; ++i) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      err = "hipEventCreateWithFlags failed";
      return TN_EDEVICE;
    }
    es->ev.push_back(e);
  }
  const size_t calls = es->left.size() + es->right.size() + static_cast<size_t>(n) + 1;
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
  std::vector<hipStream_t> streams{stream};
  for (hipStream_t st : es->side) streams.push_back(st);
  std::vector<std::unique_ptr<LaunchTimer>> timers;
  for (hipStream_t st : streams) timers.push_back(std::make_unique<LaunchTimer>(st));
  // one stream needs no events: stream order alone serialises the work
  const bool multi = S > 1;
  hipEvent_t ev_start = multi ? es->ev[0] : nullptr, ev_left = multi ? es->ev[1] : nullptr,
             ev_right = multi ? es->ev[2] : nullptr;
  size_t call = 0;
  const int32_t ne = C - 1;
  std::vector<const void*> ltap(ne, nullptr), rtap(ne, nullptr);
  hipError_t e = hipSuccess;
  tn_status status = TN_OK;

  // Left environments on the caller's stream, right ones on the first side
  // stream (one column per call); the networks wait for both and are dealt
  // round-robin over the streams, each stream with its own region.
  auto issue = [&]() -> tn_status {
    if (multi) e = hipEventRecord(ev_start, stream);
    for (int32_t i = 1; i < S && e == hipSuccess; ++i) e = hipStreamWaitEvent(streams[i], ev_start, 0);
    if (e != hipSuccess) { err = hipGetErrorString(e); return TN_EDEVICE; }
    for (int32_t side = 0; side < 2; ++side) {
      const std::vector<Plan>& plans = side ? es->right : es->left;
      const std::vector<size_t>& offs = side ? es->right_off : es->left_off;
      std::vector<const void*>& taps = side ? rtap : ltap;
      const int32_t si = (side && S > 1) ? 1 : 0;
      for (int32_t j = 0; j < ne; ++j) {
        CutIO io;
        if (j > 0) { io.seed = taps[j - 1]; io.seed_rec = recs + side * ne + j - 1; }
        io.tap = &taps[j];
        io.tap_rec = recs + side * ne + j;
        const Plan& p = plans[j];
        const tn_status st = enqueue(p, base, true, es->prec, ws + offs[j],
                                     make_layout(p, es->prec).total, streams[si],
                                     *es->keeps[call++], *timers[si], err, nullptr, nullptr, &io);
        if (st != TN_OK) return st;
      }
      if (multi) e = hipEventRecord(side ? ev_right : ev_left, streams[si]);
      if (e != hipSuccess) { err = hipGetErrorString(e); return TN_EDEVICE; }
    }
    for (int32_t i = 0; multi && i < S && e == hipSuccess; ++i) {
      e = hipStreamWaitEvent(streams[i], ev_left, 0);
      if (e == hipSuccess) e = hipStreamWaitEvent(streams[i], ev_right, 0);
    }
    if (e != hipSuccess) { err = hipGetErrorString(e); return TN_EDEVICE; }
    for (int32_t k = 0; k <= n; ++k) {
      const int32_t si = k % S;
      const Plan& p = es->cuts[es->net_plan[k]];
      for (int32_t t = 0; t < R * C; ++t) es->sites[t] = base[t];
      if (k > 0) {
        const int32_t f = es->sub_first[k - 1];
        for (int32_t i = 0; i < es->sub_count[k - 1]; ++i) es->sites[es->sub_site[f + i]] = subst[f + i];
      }
      CutIO io;
      if (p.cut_c0 > 0) { io.seed = ltap[p.cut_c0 - 1]; io.seed_rec = recs + p.cut_c0 - 1; }
      if (p.cut_c1 < C) {
        const int32_t j = C - 1 - p.cut_c1;
        io.cap = rtap[j];
        io.cap_rec = recs + ne + j;
        io.partials = reinterpret_cast<double*>(ws + es->partials_off + es->partials_bytes * si);
      }
      io.result = results + k;
      const tn_status st = enqueue(p, es->sites.data(), true, es->prec,
                                   ws + es->shared_off + es->shared_bytes * si, es->shared_bytes,
                                   streams[si], *es->keeps[call++], *timers[si], err, nullptr,
                                   nullptr, &io);
      if (st != TN_OK) return st;
    }
    return TN_OK;
  };
  status = issue();
  // join every side stream back into the caller's stream, also after an error
  for (int32_t i = 1; i < S; ++i) {
    hipError_t e2 = hipEventRecord(es->ev[3 + i], streams[i]);
    if (e2 == hipSuccess) e2 = hipStreamWaitEvent(stream, es->ev[3 + i], 0);
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
