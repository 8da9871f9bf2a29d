// Imaginary-time evolution driver (paper §5) for the transverse-field Ising
// model of §3, H = -J sum_<ij> S^z_i S^z_j - Gamma sum_i S^x_i with S = sigma
// (S^z takes the values +1 and -1).
//
// One step is the second-order Trotter-Suzuki product
// U^Gamma(dtau/2) U^J(dtau) U^Gamma(dtau/2): the one-body gate
// exp(Gamma t sigma^x) in every site's spin index (ite.hip), the state
// normalised, the pair gate exp(J dtau s_i s_j) on every nearest-neighbour
// pair, split back by an SVD with truncation (ite.hip; pairs in four classes
// of disjoint bonds: horizontal with even left column, odd, vertical with
// even upper row, odd), normalised, the one-body gate again, normalised.
// Normalising contracts the norm network <Psi|Psi> (double-layer sites, the
// library's contraction in float64) and scales every site by the same factor
// so the norm becomes 1.  The energy <H> comes from the expectation-value
// networks of §5 (norm, S^x and S^z at every site, S^z S^z on every bond),
// all contracted by one batched launch.
#include "ite.hpp"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "batch.hpp"
#include "exec.hpp"
#include "kernels.hpp"

namespace tn {

namespace {

size_t al(size_t x) { return (x + 255) & ~size_t{255}; }

struct Setup {
  int32_t rows = 0, cols = 0, chi = 0, n = 0;
  std::vector<int32_t> rank;
  std::vector<int64_t> off, half, eoff;
  int64_t state_entries = 0, e_entries = 0, max_half = 1;
  std::vector<std::vector<ItePairDesc>> classes;
  Plan norm_plan, net_plan;
  int32_t n_nets = 0;
  // byte offsets in the workspace
  size_t state = 0, e[3] = {0, 0, 0}, ops = 0, sites = 0, cls = 0, norm_ws = 0, batch_ws = 0,
         total = 0, norm_bytes = 0, batch_bytes = 0;
  std::vector<size_t> cls_off;
};

// bond legs present at (r, c): left, up, right, down
void legs_of(int32_t rows, int32_t cols, int32_t r, int32_t c, bool present[4]) {
  present[0] = c > 0;
  present[1] = r > 0;
  present[2] = c < cols - 1;
  present[3] = r < rows - 1;
}

int32_t axis_of(const bool present[4], int32_t leg) {
  int32_t a = 0;
  for (int32_t l = 0; l < leg; ++l) a += present[l] ? 1 : 0;
  return a;
}

tn_status make_setup(const tn_ite_config& cfg, Setup& S, std::string& err) {
  if (cfg.rows < 1 || cfg.cols < 1 || static_cast<int64_t>(cfg.rows) * cfg.cols > 4096) {
    err = "rows and cols must be >= 1 (at most 4096 sites)";
    return TN_EINVAL;
  }
  if (cfg.chi_max < 1 || cfg.chi_max > kIteMaxChi) {
    err = "chi_max must be 1.." + std::to_string(kIteMaxChi);
    return TN_EINVAL;
  }
  if (cfg.reserved != 0 || !std::isfinite(cfg.J) || !std::isfinite(cfg.gamma) ||
      !(cfg.eps >= 0.0) || !std::isfinite(cfg.eps)) {
    err = "bad couplings, cutoff or reserved field";
    return TN_EINVAL;
  }
  S.rows = cfg.rows; S.cols = cfg.cols; S.chi = cfg.chi_max;
  S.n = cfg.rows * cfg.cols;
  const int64_t chi = cfg.chi_max;
  for (int32_t r = 0; r < S.rows; ++r)
    for (int32_t c = 0; c < S.cols; ++c) {
      bool pr[4];
      legs_of(S.rows, S.cols, r, c, pr);
      const int32_t rk = pr[0] + pr[1] + pr[2] + pr[3];
      int64_t h = 1, e = 1;
      for (int32_t k = 0; k < rk; ++k) { h *= chi; e *= chi * chi; }
      S.rank.push_back(rk);
      S.off.push_back(S.state_entries);
      S.half.push_back(h);
      S.eoff.push_back(S.e_entries);
      S.state_entries += 2 * h;
      S.e_entries += e;
      S.max_half = std::max(S.max_half, h);
    }
  // pair classes: horizontal (even, odd left column), vertical (even, odd upper row)
  auto pair = [&](int32_t i, int32_t j, bool horizontal) {
    bool pi[4], pj[4];
    legs_of(S.rows, S.cols, i / S.cols, i % S.cols, pi);
    legs_of(S.rows, S.cols, j / S.cols, j % S.cols, pj);
    ItePairDesc d;
    d.off_i = S.off[i]; d.off_j = S.off[j];
    d.ri = S.rank[i]; d.rj = S.rank[j];
    d.ai = axis_of(pi, horizontal ? 2 : 3);
    d.aj = axis_of(pj, horizontal ? 0 : 1);
    return d;
  };
  for (int par = 0; par < 2; ++par) {
    std::vector<ItePairDesc> v;
    for (int32_t r = 0; r < S.rows; ++r)
      for (int32_t c = par; c + 1 < S.cols; c += 2) v.push_back(pair(r * S.cols + c, r * S.cols + c + 1, true));
    if (!v.empty()) S.classes.push_back(v);
  }
  for (int par = 0; par < 2; ++par) {
    std::vector<ItePairDesc> v;
    for (int32_t r = par; r + 1 < S.rows; r += 2)
      for (int32_t c = 0; c < S.cols; ++c) v.push_back(pair(r * S.cols + c, (r + 1) * S.cols + c, false));
    if (!v.empty()) S.classes.push_back(v);
  }
  // the double-layer networks: bond dimension chi^2 everywhere
  tn_grid g{S.rows, S.cols, static_cast<int32_t>(chi * chi), nullptr, nullptr};
  tn_status st = build_plan(g, TN_ORDER_HEURISTIC, 0, 0, S.norm_plan, err);
  if (st != TN_OK) return st;
  st = build_plan(g, TN_ORDER_SWEEP_AUTO, 0, 0, S.net_plan, err);
  if (st != TN_OK) return st;
  const int64_t bonds = static_cast<int64_t>(S.rows) * (S.cols - 1) +
                        static_cast<int64_t>(S.rows - 1) * S.cols;
  S.n_nets = static_cast<int32_t>(1 + 2 * S.n + bonds);
  std::vector<const Plan*> plans(static_cast<size_t>(S.n_nets), &S.net_plan);
  st = batch_workspace(plans.data(), S.n_nets, TN_PREC_F64, &S.batch_bytes, err);
  if (st != TN_OK) return st;
  S.norm_bytes = make_layout(S.norm_plan, TN_PREC_F64).total;
  size_t o = 0;
  S.state = o; o = al(o + 8 * static_cast<size_t>(S.state_entries));
  for (int k = 0; k < 3; ++k) { S.e[k] = o; o = al(o + 8 * static_cast<size_t>(S.e_entries)); }
  S.ops = o; o = al(o + 8 * 8);
  S.sites = o; o = al(o + sizeof(IteSiteDesc) * static_cast<size_t>(S.n));
  for (const auto& v : S.classes) { S.cls_off.push_back(o); o = al(o + sizeof(ItePairDesc) * v.size()); }
  S.cls = S.cls_off.empty() ? o : S.cls_off[0];
  S.norm_ws = o; o = al(o + S.norm_bytes);
  S.batch_ws = o; o = al(o + S.batch_bytes);
  S.total = o;
  return TN_OK;
}

}  // namespace

struct IteImpl {
  Setup S;
  tn_ite_config cfg{};
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  BatchImpl* batch = nullptr;
  std::vector<std::vector<const double*>> net_sites;
  std::vector<const double* const*> net_ptrs;

  double* state() const { return reinterpret_cast<double*>(ws + S.state); }
  double* E(int k) const { return reinterpret_cast<double*>(ws + S.e[k]); }
};

namespace {

#define ITE_HIP(call)                                       \
  do {                                                      \
    const hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) {                                 \
      err = std::string(#call) + ": " + hipGetErrorString(e_); \
      return TN_EDEVICE;                                    \
    }                                                       \
  } while (0)

// double-layer sites of the listed operators (0 = identity, 1 = S^x, 2 = S^z)
tn_status build_layers(IteImpl& t, int32_t kinds, std::string& err) {
  const Setup& S = t.S;
  std::vector<DoubleLayerSite> v;
  const double* ops = reinterpret_cast<const double*>(t.ws + S.ops);
  for (int32_t k = 0; k < kinds; ++k)
    for (int32_t i = 0; i < S.n; ++i) {
      DoubleLayerSite d{};
      d.A = t.state() + S.off[i];
      d.op = k == 0 ? nullptr : ops + 4 * (k - 1);
      d.E = t.E(k) + S.eoff[i];
      d.n_in = S.half[i];
      d.n_out = S.half[i] * S.half[i];
      d.d = 2;
      d.rank = S.rank[i];
      for (int32_t a = 0; a < 4; ++a) {
        d.dims[a] = a < S.rank[i] ? S.chi : 1;
        d.perm[a] = a;
      }
      v.push_back(d);
    }
  ITE_HIP(launch_double_layer(v.data(), static_cast<int32_t>(v.size()), t.stream));
  return TN_OK;
}

tn_status normalize(IteImpl& t, std::string& err) {
  const Setup& S = t.S;
  tn_status st = build_layers(t, 1, err);
  if (st != TN_OK) return st;
  std::vector<const double*> sites(static_cast<size_t>(S.n));
  for (int32_t i = 0; i < S.n; ++i) sites[i] = t.E(0) + S.eoff[i];
  tn_result r{};
  st = contract(S.norm_plan, sites.data(), true, TN_PREC_F64, t.ws + S.norm_ws, S.norm_bytes,
                t.stream, &r, err);
  if (st != TN_OK) return st;
  if (r.sign <= 0) {
    err = "the state's norm is zero";
    return TN_ENONFINITE;
  }
  const double f = std::exp(-r.log_abs / (2.0 * S.n));
  if (!std::isfinite(f)) {
    err = "normalisation factor out of range";
    return TN_ENONFINITE;
  }
  ITE_HIP(launch_ite_scale(t.state(), S.state_entries, f, t.stream));
  return TN_OK;
}

tn_status gate1(IteImpl& t, double time, std::string& err) {
  const double c = std::cosh(t.cfg.gamma * time), s = std::sinh(t.cfg.gamma * time);
  const double g[4] = {c, s, s, c};
  ITE_HIP(launch_ite_gate1(t.state(), reinterpret_cast<const IteSiteDesc*>(t.ws + t.S.sites),
                           t.S.n, t.S.max_half, g, t.stream));
  return TN_OK;
}

}  // namespace

tn_status ite_workspace(const tn_ite_config& cfg, size_t* bytes, std::string& err) {
  Setup S;
  const tn_status st = make_setup(cfg, S, err);
  if (st == TN_OK) *bytes = S.total;
  return st;
}

tn_status ite_create(const tn_ite_config& cfg, void* ws, size_t ws_bytes, hipStream_t stream,
                     IteImpl** out, std::string& err) {
  auto* t = new IteImpl;
  tn_status st = make_setup(cfg, t->S, err);
  if (st != TN_OK) { delete t; return st; }
  const Setup& S = t->S;
  if (ws_bytes < S.total) {
    err = "workspace too small: need " + std::to_string(S.total) + " bytes";
    delete t;
    return TN_ENOMEM;
  }
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) {
    err = "workspace must be 256-byte aligned";
    delete t;
    return TN_EINVAL;
  }
  t->cfg = cfg;
  t->stream = stream;
  t->ws = static_cast<char*>(ws);
  auto fail = [&](tn_status s) { ite_destroy(t); return s; };
  // tables and operators (pageable copies, complete when the call returns)
  std::vector<IteSiteDesc> sd(static_cast<size_t>(S.n));
  for (int32_t i = 0; i < S.n; ++i) sd[i] = IteSiteDesc{S.off[i], S.half[i]};
  const double ops[8] = {0.0, 1.0, 1.0, 0.0, 1.0, 0.0, 0.0, -1.0};   // sigma^x, sigma^z
  hipError_t e = hipMemcpyAsync(t->ws + S.sites, sd.data(), sizeof(IteSiteDesc) * sd.size(),
                                hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(t->ws + S.ops, ops, sizeof(ops), hipMemcpyHostToDevice, stream);
  for (size_t c = 0; e == hipSuccess && c < S.classes.size(); ++c)
    e = hipMemcpyAsync(t->ws + S.cls_off[c], S.classes[c].data(),
                       sizeof(ItePairDesc) * S.classes[c].size(), hipMemcpyHostToDevice, stream);
  // the product state (|up> + |down>) / sqrt(2) at every site, bond index 0
  std::vector<double> st0(static_cast<size_t>(S.state_entries), 0.0);
  for (int32_t i = 0; i < S.n; ++i) {
    st0[S.off[i]] = 1.0 / std::sqrt(2.0);
    st0[S.off[i] + S.half[i]] = 1.0 / std::sqrt(2.0);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(t->state(), st0.data(), sizeof(double) * st0.size(), hipMemcpyHostToDevice,
                       stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    err = std::string("ITE set-up copies: ") + hipGetErrorString(e);
    return fail(TN_EDEVICE);
  }
  std::vector<const Plan*> plans(static_cast<size_t>(S.n_nets), &S.net_plan);
  st = batch_create(plans.data(), S.n_nets, TN_PREC_F64, 512, t->ws + S.batch_ws, S.batch_bytes,
                    &t->batch, err);
  if (st != TN_OK) return fail(st);
  // site tables of the networks: norm, S^x at k, S^z at k, S^z S^z on each bond
  auto net = [&](int32_t kx, int32_t z1, int32_t z2) {
    std::vector<const double*> v(static_cast<size_t>(S.n));
    for (int32_t i = 0; i < S.n; ++i) {
      const int32_t kind = i == kx ? 1 : ((i == z1 || i == z2) ? 2 : 0);
      v[i] = t->E(kind) + S.eoff[i];
    }
    t->net_sites.push_back(v);
  };
  net(-1, -1, -1);
  for (int32_t k = 0; k < S.n; ++k) net(k, -1, -1);
  for (int32_t k = 0; k < S.n; ++k) net(-1, k, -1);
  for (int32_t r = 0; r < S.rows; ++r)
    for (int32_t c = 0; c + 1 < S.cols; ++c) net(-1, r * S.cols + c, r * S.cols + c + 1);
  for (int32_t r = 0; r + 1 < S.rows; ++r)
    for (int32_t c = 0; c < S.cols; ++c) net(-1, r * S.cols + c, (r + 1) * S.cols + c);
  for (const auto& v : t->net_sites) t->net_ptrs.push_back(v.data());
  *out = t;
  return TN_OK;
}

tn_status ite_step(IteImpl* t, double dtau, int32_t n_steps, std::string& err) {
  if (!(dtau > 0.0) || !std::isfinite(dtau) || n_steps < 0) {
    err = "dtau must be positive and finite, n_steps >= 0";
    return TN_EINVAL;
  }
  const Setup& S = t->S;
  IteGate2 g2{};
  const double jt = t->cfg.J * dtau;
  for (int a = 0; a < 4; ++a) {
    const double si = (a >> 1) ? -1.0 : 1.0, sj = (a & 1) ? -1.0 : 1.0;
    g2.g[a * 4 + a] = std::exp(jt * si * sj);
  }
  for (int32_t step = 0; step < n_steps; ++step) {
    tn_status st = gate1(*t, dtau / 2, err);
    if (st == TN_OK) st = normalize(*t, err);
    if (st != TN_OK) return st;
    for (size_t c = 0; c < S.classes.size(); ++c) {
      const hipError_t e = launch_ite_pairs(
          t->state(), reinterpret_cast<const ItePairDesc*>(t->ws + S.cls_off[c]),
          static_cast<int32_t>(S.classes[c].size()), g2, S.chi, t->cfg.eps, nullptr, t->stream);
      if (e != hipSuccess) {
        err = std::string("pair gates: ") + hipGetErrorString(e);
        return TN_EDEVICE;
      }
    }
    st = normalize(*t, err);
    if (st == TN_OK) st = gate1(*t, dtau / 2, err);
    if (st == TN_OK) st = normalize(*t, err);
    if (st != TN_OK) return st;
  }
  return TN_OK;
}

tn_status ite_energy(IteImpl* t, double* energy, double* mx, double* mz, double* czz,
                     std::string& err) {
  const Setup& S = t->S;
  tn_status st = build_layers(*t, 3, err);
  if (st != TN_OK) return st;
  std::vector<tn_result> res(static_cast<size_t>(S.n_nets));
  st = batch_run(t->batch, t->net_ptrs.data(), t->stream, res.data(), err);
  if (st != TN_OK) return st;
  st = tn_observables(res.data(), S.rows, S.cols, mx, mz, czz);
  if (st != TN_OK) {
    err = tn_last_error();
    return st;
  }
  double zz = 0.0, x = 0.0;
  int64_t b = 0;
  for (int32_t r = 0; r < S.rows; ++r)
    for (int32_t c = 0; c + 1 < S.cols; ++c, ++b) {
      const int32_t i = r * S.cols + c;
      zz += czz[b] + mz[i] * mz[i + 1];
    }
  for (int32_t r = 0; r + 1 < S.rows; ++r)
    for (int32_t c = 0; c < S.cols; ++c, ++b) {
      const int32_t i = r * S.cols + c;
      zz += czz[b] + mz[i] * mz[i + S.cols];
    }
  for (int32_t i = 0; i < S.n; ++i) x += mx[i];
  *energy = -t->cfg.J * zz - t->cfg.gamma * x;
  return TN_OK;
}

void ite_sites(const IteImpl* t, double** sites) {
  for (int32_t i = 0; i < t->S.n; ++i) sites[i] = t->state() + t->S.off[i];
}

int32_t ite_bonds(const IteImpl* t) {
  return t->S.rows * (t->S.cols - 1) + (t->S.rows - 1) * t->S.cols;
}

void ite_destroy(IteImpl* t) {
  if (!t) return;
  if (t->batch) batch_destroy(t->batch);
  delete t;
}

}  // namespace tn
