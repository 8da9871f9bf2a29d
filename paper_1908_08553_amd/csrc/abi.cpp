// extern "C" entry points declared in include/tn.h.  Every entry point
// catches everything: no exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "batch.hpp"
#include "envset.hpp"
#include "ite.hpp"
#include "exec.hpp"
#include "server.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "tn.h"

struct tn_plan {
  tn::Plan p;
};

struct tn_batch {
  tn::BatchImpl* impl;
};

struct tn_server {
  tn::ServerImpl* impl;
};

struct tn_envset {
  tn::EnvSetImpl* impl;
};

struct tn_ite {
  tn::IteImpl* impl;
};

namespace {

thread_local std::string g_err;
int32_t g_batch_threads = 512;

tn_status fail(tn_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

}  // namespace

extern "C" {

const char* tn_last_error(void) { return g_err.c_str(); }

tn_status tn_plan_grid(const tn_grid* grid, int32_t order, int32_t quad_h, int32_t quad_w,
                       tn_plan** out) {
  return tn_plan_grid_budget(grid, order, quad_h, quad_w, 0, out);
}

tn_status tn_plan_grid_budget(const tn_grid* grid, int32_t order, int32_t quad_h,
                              int32_t quad_w, int64_t max_buffer_entries, tn_plan** out) {
  try {
    if (!grid || !out) return fail(TN_EINVAL, "null argument");
    *out = nullptr;
    auto* h = new (std::nothrow) tn_plan;
    if (!h) return fail(TN_ENOMEM, "out of host memory");
    std::string err;
    const tn_status s = tn::build_plan(*grid, order, quad_h, quad_w, h->p, err,
                                       max_buffer_entries);
    if (s != TN_OK) {
      delete h;
      return fail(s, err);
    }
    *out = h;
    g_err.clear();
    return TN_OK;
  } catch (const std::exception& e) {
    return fail(TN_EINVAL, e.what());
  } catch (...) {
    return fail(TN_EINVAL, "unknown error");
  }
}

tn_status tn_plan_stats(const tn_plan* plan, tn_plan_info* out) {
  try {
    if (!plan || !out) return fail(TN_EINVAL, "null argument");
    const tn::Plan& p = plan->p;
    std::memset(out, 0, sizeof(*out));
    out->order = p.order;
    out->transpose = p.transpose;
    out->quad_h = p.qh;
    out->quad_w = p.qw;
    out->n_steps = static_cast<int32_t>(p.steps.size());
    out->n_units = static_cast<int32_t>(p.units.size());
    out->n_slots = p.slots;
    out->n_links = static_cast<int32_t>(p.chain.size());
    out->buffer_entries = p.buffers;
    out->peak_entries = p.peak;
    out->flops = p.flops;
    out->moved_entries = p.moved;
    for (int32_t prec = 0; prec < 3; ++prec) {
      const tn::Layout L = tn::make_layout(p, prec);
      out->workspace_bytes[prec] = static_cast<int64_t>(L.total);
      out->hbm_bytes[prec] = tn::algorithmic_bytes(p, prec);
      out->ring_slices[prec] = p.has_ring ? L.yt_slices : 0;
    }
    return TN_OK;
  } catch (...) {
    return fail(TN_EINVAL, "tn_plan_stats failed");
  }
}

tn_status tn_plan_text(const tn_plan* plan, char* buf, size_t* len) {
  try {
    if (!plan || !len) return fail(TN_EINVAL, "null argument");
    const std::string t = tn::plan_text(plan->p);
    const size_t need = t.size() + 1;
    if (!buf || *len < need) {
      *len = need;
      return fail(TN_ENOMEM, "text buffer too small");
    }
    std::memcpy(buf, t.c_str(), need);
    *len = need;
    return TN_OK;
  } catch (...) {
    return fail(TN_EINVAL, "tn_plan_text failed");
  }
}

void tn_plan_free(tn_plan* plan) { delete plan; }

tn_status tn_contract_grid(const tn_plan* plan, const double* const* sites,
                           int32_t sites_on_device, int32_t precision, void* workspace,
                           size_t ws_bytes, void* hip_stream, tn_result* out) {
  try {
    if (!plan || !sites || !workspace || !out) return fail(TN_EINVAL, "null argument");
    if (precision < TN_PREC_F64 || precision > TN_PREC_BF16X3)
      return fail(TN_EINVAL, "unknown precision");
    const tn::Plan& p = plan->p;
    for (int32_t s = 0; s < p.rows * p.cols; ++s)
      if (!sites[s]) return fail(TN_EINVAL, "null site pointer");
    std::memset(out, 0, sizeof(*out));
    std::string err;
    const tn_status s = tn::contract(p, sites, sites_on_device != 0, precision, workspace,
                                     ws_bytes, static_cast<hipStream_t>(hip_stream), out, err);
    if (s != TN_OK) return fail(s, err);
    g_err.clear();
    return TN_OK;
  } catch (const std::exception& e) {
    return fail(TN_EDEVICE, e.what());
  } catch (...) {
    return fail(TN_EDEVICE, "unknown error");
  }
}

namespace {
// Host image of the workspace head for tn_contract_grid_static: ordinary
// (pageable) memory of fixed size, so the call allocates nothing; one call at
// a time in the process uses it.
constexpr size_t kStaticHeadBytes = static_cast<size_t>(1) << 20;
std::mutex g_static_mu;
alignas(256) char g_static_head[kStaticHeadBytes];
}  // namespace

tn_status tn_contract_grid_static(const tn_plan* plan, const double* const* sites,
                                  int32_t sites_on_device, int32_t precision, void* hip_stream,
                                  tn_result* out) {
  try {
    if (!plan || !sites || !out) return fail(TN_EINVAL, "null argument");
    if (precision < TN_PREC_F64 || precision > TN_PREC_BF16X3)
      return fail(TN_EINVAL, "unknown precision");
    const tn::Plan& p = plan->p;
    for (int32_t s = 0; s < p.rows * p.cols; ++s)
      if (!sites[s]) return fail(TN_EINVAL, "null site pointer");
    std::memset(out, 0, sizeof(*out));
    const tn::Layout L = tn::make_layout(p, precision);
    if (L.total > TN_STATIC_SCRATCH_BYTES)
      return fail(TN_ENOMEM, "plan needs " + std::to_string(L.total) +
                                 " bytes of workspace; the static workspace holds " +
                                 std::to_string(static_cast<size_t>(TN_STATIC_SCRATCH_BYTES)));
    std::string err;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    tn_status s = tn::static_scratch(&ws, &ws_bytes, err);
    if (s != TN_OK) return fail(s, err);
    std::lock_guard<std::mutex> lk(g_static_mu);
    tn::HostKeep keep;
    keep.adopt(g_static_head, kStaticHeadBytes);
    s = tn::contract_with(p, sites, sites_on_device != 0, precision, ws, ws_bytes,
                          static_cast<hipStream_t>(hip_stream), keep, false, out, err);
    if (s != TN_OK) return fail(s, err);
    g_err.clear();
    return TN_OK;
  } catch (const std::exception& e) {
    return fail(TN_EDEVICE, e.what());
  } catch (...) {
    return fail(TN_EDEVICE, "unknown error");
  }
}

namespace {
tn_status collect(const tn_plan* const* plans, int32_t n, std::vector<const tn::Plan*>& v) {
  if (!plans || n < 1) return fail(TN_EINVAL, "empty or null plan list");
  v.resize(n);
  for (int32_t i = 0; i < n; ++i) {
    if (!plans[i]) return fail(TN_EINVAL, "null plan");
    v[i] = &plans[i]->p;
  }
  return TN_OK;
}
}  // namespace

tn_status tn_batch_workspace(const tn_plan* const* plans, int32_t n, int32_t precision,
                             size_t* bytes) {
  try {
    if (!bytes) return fail(TN_EINVAL, "null argument");
    if (precision < TN_PREC_F64 || precision > TN_PREC_BF16X3) return fail(TN_EINVAL, "unknown precision");
    std::vector<const tn::Plan*> v;
    if (collect(plans, n, v) != TN_OK) return TN_EINVAL;
    std::string err;
    const tn_status s = tn::batch_workspace(v.data(), n, precision, bytes, err);
    return s == TN_OK ? s : fail(s, err);
  } catch (...) {
    return fail(TN_EINVAL, "tn_batch_workspace failed");
  }
}

tn_status tn_batch_create(const tn_plan* const* plans, int32_t n, int32_t precision,
                          const tn_batch_config* cfg, void* workspace, size_t ws_bytes,
                          tn_batch** out) {
  try {
    if (!out || !workspace) return fail(TN_EINVAL, "null argument");
    *out = nullptr;
    if (precision < TN_PREC_F64 || precision > TN_PREC_BF16X3) return fail(TN_EINVAL, "unknown precision");
    std::vector<const tn::Plan*> v;
    if (collect(plans, n, v) != TN_OK) return TN_EINVAL;
    if (cfg && (cfg->split < 0 || cfg->split > n))
      return fail(TN_EINVAL, "tn_batch_config.split must be 0..n");
    const int32_t threads = (cfg && cfg->threads) ? cfg->threads : g_batch_threads;
    const int32_t split = cfg ? cfg->split : 0;
    std::string err;
    tn::BatchImpl* impl = nullptr;
    const tn_status s = tn::batch_create(v.data(), n, precision, threads, workspace, ws_bytes,
                                         &impl, err, split);
    if (s != TN_OK) return fail(s, err);
    *out = new tn_batch{impl};
    return TN_OK;
  } catch (const std::exception& e) {
    return fail(TN_EDEVICE, e.what());
  } catch (...) {
    return fail(TN_EDEVICE, "tn_batch_create failed");
  }
}

tn_status tn_batch_run(tn_batch* batch, const double* const* const* sites, void* hip_stream,
                       tn_result* outs) {
  try {
    if (!batch || !sites || !outs) return fail(TN_EINVAL, "null argument");
    std::string err;
    const tn_status s = tn::batch_run(batch->impl, sites, static_cast<hipStream_t>(hip_stream),
                                      outs, err);
    return s == TN_OK ? s : fail(s, err);
  } catch (...) {
    return fail(TN_EDEVICE, "tn_batch_run failed");
  }
}

tn_status tn_batch_destroy(tn_batch* batch) {
  if (!batch) return TN_OK;
  tn::batch_destroy(batch->impl);
  delete batch;
  return TN_OK;
}

tn_status tn_contract_batch(const tn_plan* const* plans, const double* const* const* sites,
                            int32_t n, int32_t precision, void* workspace, size_t ws_bytes,
                            void* hip_stream, tn_result* outs) {
  tn_batch* b = nullptr;
  tn_status s = tn_batch_create(plans, n, precision, nullptr, workspace, ws_bytes, &b);
  if (s != TN_OK) return s;
  s = tn_batch_run(b, sites, hip_stream, outs);
  const std::string keep = g_err;
  tn_batch_destroy(b);
  g_err = keep;
  return s;
}

tn_status tn_envset_workspace(const tn_grid* grid, int32_t precision, int32_t n,
                              const int32_t* n_subst, const int32_t* subst_site, size_t* bytes) {
  try {
    if (!grid || !bytes) return fail(TN_EINVAL, "null argument");
    if (precision < TN_PREC_F64 || precision > TN_PREC_BF16X3) return fail(TN_EINVAL, "unknown precision");
    std::string err;
    const tn_status s = tn::envset_workspace(*grid, precision, n, n_subst, subst_site, bytes, err);
    return s == TN_OK ? s : fail(s, err);
  } catch (...) {
    return fail(TN_EINVAL, "tn_envset_workspace failed");
  }
}

tn_status tn_envset_create(const tn_grid* grid, int32_t precision, int32_t n,
                           const int32_t* n_subst, const int32_t* subst_site, void* workspace,
                           size_t ws_bytes, tn_envset** out) {
  try {
    if (!grid || !out || !workspace) return fail(TN_EINVAL, "null argument");
    *out = nullptr;
    if (precision < TN_PREC_F64 || precision > TN_PREC_BF16X3) return fail(TN_EINVAL, "unknown precision");
    std::string err;
    tn::EnvSetImpl* impl = nullptr;
    const tn_status s = tn::envset_create(*grid, precision, n, n_subst, subst_site, workspace,
                                          ws_bytes, &impl, err);
    if (s != TN_OK) return fail(s, err);
    *out = new tn_envset{impl};
    return TN_OK;
  } catch (const std::exception& e) {
    return fail(TN_EINVAL, e.what());
  } catch (...) {
    return fail(TN_EINVAL, "tn_envset_create failed");
  }
}

tn_status tn_envset_run(tn_envset* set, const double* const* base, const double* const* subst,
                        void* hip_stream, tn_result* outs) {
  try {
    if (!set || !base || !outs) return fail(TN_EINVAL, "null argument");
    std::string err;
    const tn_status s = tn::envset_run(set->impl, base, subst,
                                       static_cast<hipStream_t>(hip_stream), outs, err);
    return s == TN_OK ? s : fail(s, err);
  } catch (...) {
    return fail(TN_EDEVICE, "tn_envset_run failed");
  }
}

tn_status tn_envset_destroy(tn_envset* set) {
  if (!set) return TN_OK;
  tn::envset_destroy(set->impl);
  delete set;
  return TN_OK;
}

tn_status tn_server_create(void* arena, size_t arena_bytes, int32_t max_slots,
                           int32_t queue_depth, tn_server** out) {
  try {
    if (!out) return fail(TN_EINVAL, "null argument");
    *out = nullptr;
    std::string err;
    tn::ServerImpl* impl = nullptr;
    const tn_status s = tn::server_create(arena, arena_bytes, max_slots, queue_depth, &impl, err);
    if (s != TN_OK) return fail(s, err);
    *out = new tn_server{impl};
    return TN_OK;
  } catch (...) {
    return fail(TN_EDEVICE, "tn_server_create failed");
  }
}

tn_status tn_submit(tn_server* server, const tn_grid* grid, int32_t order, int32_t precision,
                    const double* const* host_sites, uint64_t* ticket) {
  try {
    if (!server || !grid) return fail(TN_EINVAL, "null argument");
    std::string err;
    const tn_status s = tn::server_submit(server->impl, *grid, order, precision, host_sites,
                                          ticket, err);
    return s == TN_OK ? s : fail(s, err);
  } catch (...) {
    return fail(TN_EINVAL, "tn_submit failed");
  }
}

tn_status tn_poll_ex(tn_server* server, uint64_t ticket, tn_result* out, int64_t* times_ns) {
  try {
    if (!server) return fail(TN_EINVAL, "null argument");
    std::string err;
    const tn_status s = tn::server_poll(server->impl, ticket, out, times_ns, err);
    return (s == TN_OK || s == TN_PENDING) ? s : fail(s, err);
  } catch (...) {
    return fail(TN_EINVAL, "tn_poll failed");
  }
}

tn_status tn_poll(tn_server* server, uint64_t ticket, tn_result* out) {
  return tn_poll_ex(server, ticket, out, nullptr);
}

tn_status tn_server_stats(tn_server* server, tn_server_info* out) {
  if (!server || !out) return fail(TN_EINVAL, "null argument");
  tn::server_info(server->impl, out);
  return TN_OK;
}

tn_status tn_server_destroy(tn_server* server) {
  if (!server) return TN_OK;
  try {
    tn::server_destroy(server->impl);
  } catch (...) {
  }
  delete server;
  return TN_OK;
}

tn_status tn_set_option(int32_t option, int64_t value) {
  if (option == TN_OPT_BATCH_THREADS) {
    if (value != 256 && value != 512 && value != 1024)
      return fail(TN_EINVAL, "TN_OPT_BATCH_THREADS must be 256, 512 or 1024");
    g_batch_threads = static_cast<int32_t>(value);
    return TN_OK;
  }
  if (option == TN_OPT_KERNEL_IMPL) {
    if (value < 0 || value > 1) return fail(TN_EINVAL, "TN_OPT_KERNEL_IMPL must be 0 or 1");
    tn::set_absorb_policy(static_cast<int32_t>(value));
    return TN_OK;
  }
  if (option == TN_OPT_ENV_SITES) {
    if (value < 0 || value > 1) return fail(TN_EINVAL, "TN_OPT_ENV_SITES must be 0 or 1");
    tn::set_env_sites(static_cast<int32_t>(value));
    return TN_OK;
  }
  if (option == TN_OPT_ENV_ROWS) {
    if (value < 0 || value > 1024) return fail(TN_EINVAL, "TN_OPT_ENV_ROWS must be 0..1024 (GiB)");
    tn::set_env_rows(static_cast<int32_t>(value));
    return TN_OK;
  }
  if (option == TN_OPT_ENV_STREAMS) {
    if (value < 1 || value > 4) return fail(TN_EINVAL, "TN_OPT_ENV_STREAMS must be 1..4");
    tn::set_env_streams(static_cast<int32_t>(value));
    return TN_OK;
  }
  if (option == TN_OPT_CHAIN_STEPS) {
    if (value < 0 || value > 1) return fail(TN_EINVAL, "TN_OPT_CHAIN_STEPS must be 0 or 1");
    tn::set_chain_steps(static_cast<int32_t>(value));
    return TN_OK;
  }
  if (option == TN_OPT_QUADRANT_STREAMS) {
    if (value < 0 || value > 1) return fail(TN_EINVAL, "TN_OPT_QUADRANT_STREAMS must be 0 or 1");
    tn::set_quadrant_streams(static_cast<int32_t>(value));
    return TN_OK;
  }
  if (option == TN_OPT_CHUNK_SCHEDULE) {
    if (value < 0 || value > 2) return fail(TN_EINVAL, "TN_OPT_CHUNK_SCHEDULE must be 0, 1 or 2");
    tn::set_chunk_schedule(static_cast<int32_t>(value));
    return TN_OK;
  }
  if (option == TN_OPT_RING_OPERAND_SCALE) {
    if (value < 0 || value > 1) return fail(TN_EINVAL, "TN_OPT_RING_OPERAND_SCALE must be 0 or 1");
    tn::set_ring_operand_scale(static_cast<int32_t>(value));
    return TN_OK;
  }
  if (option == TN_OPT_CHUNK_STREAM) {
    if (value < 0 || value > 65536) return fail(TN_EINVAL, "TN_OPT_CHUNK_STREAM must be 0..65536");
    tn::set_chunk_stream(static_cast<int32_t>(value));
    return TN_OK;
  }
  if (option == TN_OPT_FUSE_STEPS) {
    if (value < 0 || value > 2) return fail(TN_EINVAL, "TN_OPT_FUSE_STEPS must be 0, 1 or 2");
    tn::set_fuse_steps(static_cast<int32_t>(value));
    return TN_OK;
  }
  return fail(TN_EINVAL, "unknown option");
}

tn_status tn_profile_enable(int32_t on) {
  try {
    tn::profile_enable(on != 0);
    return TN_OK;
  } catch (...) {
    return fail(TN_EINVAL, "tn_profile_enable failed");
  }
}

tn_status tn_profile_read(tn_kernel_stat* out, int32_t cap, int32_t* n) {
  try {
    if (!n || (cap > 0 && !out)) return fail(TN_EINVAL, "null argument");
    *n = tn::profile_read(out, cap);
    return TN_OK;
  } catch (...) {
    return fail(TN_EINVAL, "tn_profile_read failed");
  }
}

tn_status tn_double_layer(const tn_double_layer_site* sites, int32_t n, void* hip_stream) {
  try {
    if (n < 0 || (n > 0 && !sites)) return fail(TN_EINVAL, "null argument");
    std::vector<tn::DoubleLayerSite> v(static_cast<size_t>(n));
    for (int32_t i = 0; i < n; ++i) {
      const tn_double_layer_site& x = sites[i];
      tn::DoubleLayerSite& y = v[static_cast<size_t>(i)];
      y.A = x.A;
      y.op = x.op;
      y.E = x.E;
      y.d = x.d;
      y.rank = x.rank;
      int64_t m = 1;
      for (int k = 0; k < 4; ++k) {
        y.dims[k] = k < x.rank ? x.dims[k] : 1;
        if (k < x.rank && (x.dims[k] < 1 || m > (int64_t{1} << 30)))
          return fail(TN_EINVAL, "bad double-layer site dimensions");
        if (k < x.rank) m *= x.dims[k];
      }
      y.n_in = m;
      y.n_out = m * m;
      bool given = false;
      for (int k = 0; k < 4; ++k) given = given || x.perm[k] != 0;
      for (int k = 0; k < 4; ++k) y.perm[k] = given ? x.perm[k] : k;
      if (x.rank < 0 || x.rank > 4 || !tn::double_layer_ok(y))
        return fail(TN_EINVAL, "bad double-layer site " + std::to_string(i));
    }
    if (n == 0) return TN_OK;
    const hipError_t e =
        tn::launch_double_layer(v.data(), n, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(TN_EDEVICE, hipGetErrorString(e));
    return TN_OK;
  } catch (...) {
    return fail(TN_EINVAL, "tn_double_layer failed");
  }
}

tn_status tn_ite_workspace(const tn_ite_config* cfg, size_t* bytes) {
  try {
    if (!cfg || !bytes) return fail(TN_EINVAL, "null argument");
    std::string err;
    const tn_status s = tn::ite_workspace(*cfg, bytes, err);
    return s == TN_OK ? s : fail(s, err);
  } catch (...) {
    return fail(TN_EINVAL, "tn_ite_workspace failed");
  }
}

tn_status tn_ite_create(const tn_ite_config* cfg, void* workspace, size_t ws_bytes,
                        void* hip_stream, tn_ite** out) {
  try {
    if (!cfg || !workspace || !out) return fail(TN_EINVAL, "null argument");
    *out = nullptr;
    std::string err;
    tn::IteImpl* impl = nullptr;
    const tn_status s = tn::ite_create(*cfg, workspace, ws_bytes,
                                       static_cast<hipStream_t>(hip_stream), &impl, err);
    if (s != TN_OK) return fail(s, err);
    *out = new tn_ite{impl};
    return TN_OK;
  } catch (const std::exception& e) {
    return fail(TN_EDEVICE, e.what());
  } catch (...) {
    return fail(TN_EDEVICE, "tn_ite_create failed");
  }
}

tn_status tn_ite_step(tn_ite* ite, double dtau, int32_t n_steps) {
  try {
    if (!ite) return fail(TN_EINVAL, "null argument");
    std::string err;
    const tn_status s = tn::ite_step(ite->impl, dtau, n_steps, err);
    return s == TN_OK ? s : fail(s, err);
  } catch (const std::exception& e) {
    return fail(TN_EDEVICE, e.what());
  } catch (...) {
    return fail(TN_EDEVICE, "tn_ite_step failed");
  }
}

tn_status tn_ite_energy(tn_ite* ite, double* energy, double* mx, double* mz, double* czz) {
  try {
    if (!ite || !energy || !mx || !mz || !czz) return fail(TN_EINVAL, "null argument");
    std::string err;
    const tn_status s = tn::ite_energy(ite->impl, energy, mx, mz, czz, err);
    return s == TN_OK ? s : fail(s, err);
  } catch (const std::exception& e) {
    return fail(TN_EDEVICE, e.what());
  } catch (...) {
    return fail(TN_EDEVICE, "tn_ite_energy failed");
  }
}

tn_status tn_ite_sites(tn_ite* ite, double** sites) {
  if (!ite || !sites) return fail(TN_EINVAL, "null argument");
  tn::ite_sites(ite->impl, sites);
  return TN_OK;
}

tn_status tn_ite_destroy(tn_ite* ite) {
  if (!ite) return TN_OK;
  tn::ite_destroy(ite->impl);
  delete ite;
  return TN_OK;
}

tn_status tn_observables(const tn_result* results, int32_t rows, int32_t cols, double* mx,
                         double* mz, double* czz) {
  try {
    if (!results || !mx || !mz || !czz || rows < 1 || cols < 1)
      return fail(TN_EINVAL, "null argument or empty lattice");
    const int64_t n = static_cast<int64_t>(rows) * cols;
    const int64_t pairs = static_cast<int64_t>(rows) * (cols - 1) + static_cast<int64_t>(rows - 1) * cols;
    const int64_t total = 1 + 2 * n + pairs;
    for (int64_t i = 0; i < total; ++i)
      if (results[i].status != TN_OK) return fail(TN_ENONFINITE, "non-finite network result");
    const tn_result& norm = results[0];
    if (norm.sign == 0) return fail(TN_EINVAL, "zero norm");
    // <O> = Z_O / Z: mantissas in [0.5, 1) carry the sign, exponents are exact
    auto ratio = [&](const tn_result& r) {
      if (r.sign == 0) return 0.0;
      return std::ldexp(r.mantissa / norm.mantissa, static_cast<int>(r.exp2_sum - norm.exp2_sum));
    };
    for (int64_t k = 0; k < n; ++k) {
      mx[k] = ratio(results[1 + k]);
      mz[k] = ratio(results[1 + n + k]);
    }
    int64_t b = 0;
    for (int32_t r = 0; r < rows; ++r)
      for (int32_t c = 0; c + 1 < cols; ++c, ++b) {
        const int64_t i = static_cast<int64_t>(r) * cols + c;
        czz[b] = ratio(results[1 + 2 * n + b]) - mz[i] * mz[i + 1];
      }
    for (int32_t r = 0; r + 1 < rows; ++r)
      for (int32_t c = 0; c < cols; ++c, ++b) {
        const int64_t i = static_cast<int64_t>(r) * cols + c;
        czz[b] = ratio(results[1 + 2 * n + b]) - mz[i] * mz[i + cols];
      }
    return TN_OK;
  } catch (...) {
    return fail(TN_EINVAL, "tn_observables failed");
  }
}

}  // extern "C"
