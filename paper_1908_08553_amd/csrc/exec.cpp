// Executor for one lattice contraction on one GPU.
//
// Sequence on the caller's stream: (host sites -> workspace copy), one
// staging launch (fold every site into its step's K x N matrix with an exact
// power-of-two pre-normalisation), one absorption launch per pairwise step
// (paper §4: pairwise, sequential contraction), the ring closure for the
// quadrant order, and a finalize launch that assembles sign, exponent and
// log|Z|; the 64-byte result is then copied back and the stream synchronised.
#include "exec.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>

namespace tn {
namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

inline int32_t elem_bytes(int32_t t) { return t == EL_F64 ? 8 : 4; }

// A colsweep's last column runs in float64 whatever the precision: it shrinks
// the boundary to the scalar (the "final reduction").
int32_t step_out_type(const Plan& p, const Step& s, int32_t prec) {
  if (prec == TN_PREC_F64) return EL_F64;
  if (p.order == TN_ORDER_COLSWEEP && s.last_col) return EL_F64;
  // a one-row row scheme is that row's sweep: its last step is the scalar
  if (p.order == TN_ORDER_ROWS && p.units.size() == 1 && s.last_col) return EL_F64;
  return EL_F32;
}

const char* hip_msg(hipError_t e) { return hipGetErrorString(e); }

// Steps s1, s2 are consecutive rows of one column of one sweep whose four
// legs between them all have dimension 4 (K = N = 16 for both, the leg s2
// adds to the prefix and the one s1 keeps in the suffix of dimension 4), no
// rescale between them, and a suffix of whole 64-entry runs: the shape
// absorb_pair fuses.
bool pair_ok(const Step& s1, const Step& s2) {
  if (s1.kind != STEP_ABSORB || s2.kind != STEP_ABSORB) return false;
  if (s1.unit != s2.unit || s1.col != s2.col || s1.rescale >= 0 || s2.scale_in >= 0) return false;
  if (s1.K != 16 || s1.N != 16 || s2.K != 16 || s2.N != 16) return false;
  if (s2.pre != 4 * s1.pre || s1.post != 4 * s2.post || s2.post % 64 != 0) return false;
  return s1.pre * (s2.post / 64) <= static_cast<int64_t>(INT32_MAX);
}

// Steps k0 .. k0+len-1 are consecutive rows of one column of one sweep that
// absorb_chunk can run on one slice: first K in {4, 16}, inner K = N = 16 with
// every leg between consecutive rows of dimension 4 (each row adds a
// dimension-4 leg to the prefix and takes one from the suffix), last N in
// {4, 16}, rescale only after the last row, one element type throughout.
bool chunk_ok(const Plan& p, const Layout& L, int32_t k0, int32_t len) {
  if (k0 < 1 || k0 + len > static_cast<int32_t>(p.steps.size())) return false;
  const Step& a = p.steps[k0];
  for (int32_t j = 0; j < len; ++j) {
    const Step& s = p.steps[k0 + j];
    if (s.kind != STEP_ABSORB || s.unit != a.unit || s.col != a.col) return false;
    if (j + 1 < len && s.rescale >= 0) return false;
    if (j > 0 && s.scale_in >= 0) return false;
    if (j == 0 ? (s.K != 4 && s.K != 16) : s.K != 16) return false;
    if (j + 1 == len ? (s.N != 4 && s.N != 16) : s.N != 16) return false;
    if (L.out_type[k0 + j] != L.out_type[k0 - 1]) return false;
    if (j + 1 < len) {
      const Step& nx = p.steps[k0 + j + 1];
      if (nx.pre != 4 * s.pre || s.post != 4 * nx.post) return false;
    }
  }
  const Step& z = p.steps[k0 + len - 1];
  return chunk_shape_ok(L.out_type[k0], a.pre, z.post, len, static_cast<int32_t>(a.K),
                        static_cast<int32_t>(z.N));
}

// Steps k, k+1 that absorb_edge fuses: 1 = the last two rows of a column with
// suffix 1 (a sweep's first column), 2 = the first two rows of a column with
// prefix 1 (its last column); D = 4 legs, no rescale between them, and large
// enough for the saved pass to matter (smaller pairs stay in chained launches).
int32_t edge_kind(const Plan& p, int32_t k, int32_t end) {
  if (k + 1 >= end) return 0;
  const Step& s1 = p.steps[k];
  const Step& s2 = p.steps[k + 1];
  if (s1.kind != STEP_ABSORB || s2.kind != STEP_ABSORB) return 0;
  if (s1.unit != s2.unit || s1.col != s2.col || s1.rescale >= 0 || s2.scale_in >= 0) return 0;
  if (s1.pre * s1.K * s1.post + s2.out < (int64_t{1} << 18)) return 0;
  if (s1.post == 1 && s2.post == 1 && s1.K == 4 && s1.N == 16 && s2.K == 4 && s2.N == 4 &&
      s2.pre == 4 * s1.pre && (k + 2 >= end || p.steps[k + 2].col != s2.col))
    return 1;
  if (s1.pre == 1 && s2.pre == 1 && s1.K == 4 && s1.N == 4 && s2.K == 16 && s2.N == 4 &&
      s1.post == 4 * s2.post && s2.post % 4 == 0)
    return 2;
  return 0;
}

struct KStat { int64_t launches = 0; double ms = 0, bytes = 0, flops = 0; };
std::mutex g_prof_mu;
bool g_prof_on = false;
std::map<std::string, KStat> g_prof;

}  // namespace

void profile_enable(bool on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.clear();
  g_prof_on = on;
}

bool profile_on() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  return g_prof_on;
}

int32_t profile_read(tn_kernel_stat* out, int32_t cap) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  int32_t k = 0;
  for (const auto& kv : g_prof) {
    if (out && k < cap) {
      tn_kernel_stat& o = out[k];
      std::memset(&o, 0, sizeof(o));
      std::strncpy(o.name, kv.first.c_str(), sizeof(o.name) - 1);
      o.launches = kv.second.launches;
      o.total_ms = kv.second.ms;
      o.bytes = kv.second.bytes;
      o.flops = kv.second.flops;
    }
    ++k;
  }
  return k;
}

LaunchTimer::LaunchTimer(hipStream_t s, bool allow) : stream_(s), on_(allow && profile_on()) {}

LaunchTimer::~LaunchTimer() {
  for (Rec& r : recs_) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  if (pending_) (void)hipEventDestroy(pending_);
}

void LaunchTimer::before() {
  if (!on_) return;
  if (hipEventCreate(&pending_) != hipSuccess) { pending_ = nullptr; return; }
  (void)hipEventRecord(pending_, stream_);
}

void LaunchTimer::after(const char* name, double bytes, double flops) {
  if (!on_ || !pending_) return;
  Rec r{pending_, nullptr, name, bytes, flops};
  pending_ = nullptr;
  if (hipEventCreate(&r.b) != hipSuccess) { (void)hipEventDestroy(r.a); return; }
  (void)hipEventRecord(r.b, stream_);
  recs_.push_back(r);
}

void LaunchTimer::flush() {
  if (!on_) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (Rec& r : recs_) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
    KStat& k = g_prof[r.name];
    k.launches += 1;
    k.ms += ms;
    k.bytes += r.bytes;
    k.flops += r.flops;
  }
}

Layout make_layout(const Plan& p, int32_t prec) {
  Layout L;
  const size_t nsteps = p.steps.size();
  L.state = 0;
  L.state_bytes = align_up(sizeof(DevState) + sizeof(int32_t) * (p.slots + 2 * nsteps));
  size_t off = L.state_bytes;
  L.descs = off;
  off = align_up(off + sizeof(StageDesc) * nsteps);
  L.raw = off;
  off = align_up(off + sizeof(double) * static_cast<size_t>(p.total_site_entries));
  L.s_off.resize(nsteps);
  L.out_type.resize(nsteps);
  int64_t staged = 0;
  for (size_t k = 0; k < nsteps; ++k) {
    L.s_off[k] = staged;
    staged += p.steps[k].site_entries;
    L.out_type[k] = step_out_type(p, p.steps[k], prec);
  }
  const size_t ns = static_cast<size_t>(std::max<int64_t>(staged, 1));
  L.s64 = off; off = align_up(off + 8 * ns);
  L.s32 = off; off = align_up(off + 4 * ns);
  L.shi = off; off = align_up(off + 2 * ns);
  L.slo = off; off = align_up(off + 2 * ns);
  L.buf.assign(p.units.size(), {0, 0});
  L.buf_bytes.assign(p.units.size(), 0);
  for (size_t u = 0; u < p.units.size(); ++u) {
    const Unit& U = p.units[u];
    size_t mx = 0;
    for (int32_t k = U.first_step; k < U.first_step + U.n_steps; ++k)
      mx = std::max(mx, static_cast<size_t>(p.steps[k].out) * elem_bytes(L.out_type[k]));
    L.buf_bytes[u] = align_up(mx);
    L.buf[u][0] = off; off += L.buf_bytes[u];
    // a seeded single absorption reads the seed in place and writes only the
    // second buffer: one buffer serves both
    const bool one_out = p.is_cut && p.steps.size() == 2 && p.steps[0].kind == STEP_SEED;
    L.buf[u][1] = one_out ? L.buf[u][0] : off;
    if (!one_out) off += L.buf_bytes[u];
  }
  if (p.has_ring) {
    const int32_t t = prec == TN_PREC_F64 ? EL_F64 : EL_F32;
    const Ring& g = p.ring;
    L.split_ring = prec == TN_PREC_BF16X3 && g.m % 4 == 0 && g.n % 4 == 0;
    // Room for every kernel choice of either ring product, whatever the
    // kernel policy is when the plan runs: split-K slices of X and partial
    // sums of the fused dot follow from the shapes alone.
    RingArgs rx{};
    rx.type = t;
    rx.arith = prec == TN_PREC_F64 ? AR_F64 : AR_F32;
    rx.m = g.m; rx.n = g.n; rx.k = g.kx;
    RingArgs ry = rx;
    ry.k = g.ky;
    int32_t slices = 1;
    int64_t parts = ring_partials(g.m, g.n);
    if (ring_mfma_supported(rx)) {
      slices = std::max(slices, ring_mfma_splits(rx));
      parts = std::max(parts, ring_mfma_partials_for(ry));
    }
    if (L.split_ring) {
      slices = std::max(slices, ring_bf16x3_nt_splits(g.m, g.n, split_k_padded(g.kx)));
      parts = std::max(parts, ring_bf16x3_nt_partials(g.m, g.n, split_k_padded(g.ky)));
    }
    L.yt = off;
    L.yt_slices = slices;
    L.yt_bytes = align_up(static_cast<size_t>(slices) * static_cast<size_t>(g.m * g.n) *
                          elem_bytes(t));
    off += L.yt_bytes;
    L.n_partials = parts;
    L.partials = off;
    off = align_up(off + sizeof(double) * static_cast<size_t>(L.n_partials));
    if (L.split_ring) {
      // unit u as [k][rows]: rows = m for TL/BL, n for TR/BR; k = kx (top) / ky (bottom)
      const int64_t rows[4] = {g.m, g.n, g.n, g.m};
      const int64_t kk[4] = {g.kx, g.kx, g.ky, g.ky};
      for (int u = 0; u < 4; ++u) {
        const size_t bytes = align_up(static_cast<size_t>(rows[u] * split_k_padded(kk[u])) * 2);
        L.split[u][0] = off; off += bytes;
        L.split[u][1] = off; off += bytes;
      }
    }
  }
  if (!p.chain.empty()) {
    int64_t vmax = 1, parts = 1;
    for (const Link& lk : p.chain) {
      vmax = std::max(vmax, lk.N);
      parts = std::max(parts, link_chunks(lk.side, lk.K, lk.N) * lk.N);
    }
    L.vbuf_bytes = align_up(sizeof(double) * static_cast<size_t>(vmax));
    L.vbuf[0] = off; off += L.vbuf_bytes;
    L.vbuf[1] = off; off += L.vbuf_bytes;
    L.n_link_partials = parts;
    L.link_partials = off;
    off = align_up(off + sizeof(double) * static_cast<size_t>(parts));
  }
  L.total = off;
  return L;
}

int64_t algorithmic_bytes(const Plan& p, int32_t prec) {
  const Layout L = make_layout(p, prec);
  int64_t bytes = 0;
  for (size_t k = 0; k < p.steps.size(); ++k) {
    const Step& s = p.steps[k];
    const int64_t eo = elem_bytes(L.out_type[k]);
    if (s.kind == STEP_INIT) { bytes += s.out * eo; continue; }
    if (s.kind == STEP_SEED) { bytes += 2 * s.out * eo; continue; }
    const int64_t ei = elem_bytes(L.out_type[k - 1]);
    bytes += s.pre * s.K * s.post * ei + s.out * eo;
  }
  if (p.has_ring) {
    const int64_t e = prec == TN_PREC_F64 ? 8 : 4;
    for (const Unit& U : p.units) bytes += U.result * e;
    bytes += 2 * p.ring.m * p.ring.n * e;
  }
  for (size_t i = 0; i < p.chain.size(); ++i) {
    const Link& lk = p.chain[i];
    const Unit& U = p.units[lk.unit];
    const int64_t er = elem_bytes(L.out_type[U.first_step + U.n_steps - 1]);
    const Unit& U0 = p.units[0];
    const int64_t ev = i == 0 ? elem_bytes(L.out_type[U0.first_step + U0.n_steps - 1]) : 8;
    bytes += lk.K * lk.N * er + lk.K * ev + lk.N * 8;
  }
  return bytes;
}

void fill_stage_descs(const Plan& p, const Layout& L, int64_t s_base,
                      const double* const* dsite, char* const* init_dst, StageDesc* descs) {
  const int32_t R = p.rows, C = p.cols;
  auto hd = [&](int32_t r, int32_t c) { return p.hdim[static_cast<size_t>(r) * (C - 1) + c]; };
  auto vd = [&](int32_t r, int32_t c) { return p.vdim[static_cast<size_t>(r) * C + c]; };
  for (size_t k = 0; k < p.steps.size(); ++k) {
    const Step& s = p.steps[k];
    StageDesc& d = descs[k];
    std::memset(&d, 0, sizeof(d));
    d.src = dsite[s.r * C + s.c];
    d.entries = s.site_entries;
    d.s_off = s_base + L.s_off[k];
    d.ndim = s.nperm;
    // canonical dims / strides of the site
    int32_t cdims[4];
    int64_t cstr[4];
    int32_t nd = 0;
    if (s.c > 0) cdims[nd++] = hd(s.r, s.c - 1);
    if (s.r > 0) cdims[nd++] = vd(s.r - 1, s.c);
    if (s.c < C - 1) cdims[nd++] = hd(s.r, s.c);
    if (s.r < R - 1) cdims[nd++] = vd(s.r, s.c);
    int64_t st = 1;
    for (int32_t a = nd - 1; a >= 0; --a) { cstr[a] = st; st *= cdims[a]; }
    for (int32_t a = 0; a < s.nperm; ++a) {
      d.dims[a] = cdims[s.perm[a]];
      d.cstride[a] = cstr[s.perm[a]];
    }
    if (s.kind == STEP_INIT) {
      d.init_dst = init_dst[s.unit];
      d.init_double = L.out_type[k] == EL_F64;
    }
  }
}

int32_t g_quadrant_streams = 0;
int32_t g_chain_steps = 1;
void set_chain_steps(int32_t on) { g_chain_steps = on ? 1 : 0; }
void set_quadrant_streams(int32_t on) { g_quadrant_streams = on ? 1 : 0; }

HostKeep::~HostKeep() {
  if (p_ && !fixed_) (void)hipHostFree(p_);
}

char* HostKeep::block(size_t bytes, hipError_t* e) {
  *e = hipSuccess;
  if (bytes <= cap_) return p_;
  if (fixed_) {
    *e = hipErrorOutOfMemory;
    return nullptr;
  }
  if (p_) (void)hipHostFree(p_);
  p_ = nullptr;
  cap_ = 0;
  const size_t want = std::max<size_t>(align_up(bytes), 64 * 1024);
  void* q = nullptr;
  *e = hipHostMalloc(&q, want, hipHostMallocDefault);
  if (*e != hipSuccess) return nullptr;
  p_ = static_cast<char*>(q);
  cap_ = want;
  return p_;
}

size_t head_bytes(const Plan& p, const Layout& L) {
  return align_up(L.descs + sizeof(StageDesc) * p.steps.size());
}

tn_status enqueue(const Plan& p, const double* const* sites, bool on_device, int32_t prec,
                  void* ws, size_t ws_bytes, hipStream_t stream, HostKeep& keep,
                  LaunchTimer& timer, std::string& err, const SideStream* side,
                  LaunchTimer* side_timer, const CutIO* io) {
  const Layout L = make_layout(p, prec);
  const bool seeded = !p.steps.empty() && p.steps[0].kind == STEP_SEED;
  const bool open_end = p.is_cut && p.cut_open_end;
  if (seeded && (!io || !io->seed || !io->seed_rec)) {
    err = "cut plan needs a seed boundary";
    return TN_EINVAL;
  }
  if (open_end && (!io || !((io->cap && io->cap_rec && io->partials) || (io->tap && io->tap_rec)))) {
    err = "cut plan needs a cap boundary or a tap record";
    return TN_EINVAL;
  }
  if (ws_bytes < L.total) {
    err = "workspace too small: need " + std::to_string(L.total) + " bytes";
    return TN_ENOMEM;
  }
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) {
    err = "workspace must be 256-byte aligned";
    return TN_EINVAL;
  }
  char* base = static_cast<char*>(ws);
  const int32_t nsites = p.rows * p.cols;
  hipError_t e;
#define TN_HIP(call)                                          \
  do {                                                        \
    e = (call);                                               \
    if (e != hipSuccess) {                                    \
      err = std::string(#call) + ": " + hip_msg(e);           \
      return TN_EDEVICE;                                      \
    }                                                         \
  } while (0)

  // site pointers on the device
  std::vector<const double*> dsite(nsites);
  if (on_device) {
    for (int32_t s = 0; s < nsites; ++s) dsite[s] = sites[s];
  } else {
    size_t off = L.raw;
    for (int32_t s = 0; s < nsites; ++s) {
      const Step* st = nullptr;
      for (const Step& x : p.steps)
        if (x.r * p.cols + x.c == s) { st = &x; break; }
      const size_t bytes = sizeof(double) * static_cast<size_t>(st->site_entries);
      TN_HIP(hipMemcpyAsync(base + off, sites[s], bytes, hipMemcpyHostToDevice, stream));
      dsite[s] = reinterpret_cast<const double*>(base + off);
      off += bytes;
    }
  }

  // head image: state header (zeroed counters), exponent slots (written by the
  // staging launch) and staging descriptors, uploaded in one copy
  const size_t nsteps = p.steps.size();
  const size_t head = head_bytes(p, L);
  char* img = keep.block(head + sizeof(tn_result), &e);
  if (!img) {
    err = "host image of the workspace head (" + std::to_string(head + sizeof(tn_result)) +
          " bytes): " + hip_msg(e);
    return TN_ENOMEM;
  }
  std::memset(img, 0, L.descs);
  DevState* hs = reinterpret_cast<DevState*>(img + L.state);
  hs->n_slots = p.slots;
  hs->n_steps = static_cast<int32_t>(nsteps);
  std::vector<char*> init_dst(p.units.size());
  for (size_t u = 0; u < p.units.size(); ++u) init_dst[u] = base + L.buf[u][0];
  fill_stage_descs(p, L, 0, dsite.data(), init_dst.data(),
                   reinterpret_cast<StageDesc*>(img + L.descs));
  TN_HIP(hipMemcpyAsync(base + L.state, img + L.state, head - L.state, hipMemcpyHostToDevice,
                        stream));

  DevState* state = reinterpret_cast<DevState*>(base + L.state);
  int32_t* slot_exp = reinterpret_cast<int32_t*>(state + 1);
  StagedArrays sa{reinterpret_cast<double*>(base + L.s64), reinterpret_cast<float*>(base + L.s32),
                  reinterpret_cast<uint16_t*>(base + L.shi),
                  reinterpret_cast<uint16_t*>(base + L.slo)};
  timer.before();
  StageTargets tg;
  tg.slot_exp = slot_exp;
  tg.n_slots = p.slots;
  tg.site_exp = slot_exp + p.slots;
  tg.site_bad = tg.site_exp + nsteps;
  tg.flags = &state->flags;
  tg.counter = nullptr;
  if (seeded) {
    tg.seed_rec = io->seed_rec;
    tg.seed_slot = p.steps[0].rescale;
    tg.e_bias = &state->e_bias;
  }
  TN_HIP(launch_stage(reinterpret_cast<const StageDesc*>(base + L.descs),
                      static_cast<int32_t>(nsteps), sa, tg, stream));
  timer.after("stage", 8.0 * 2 * static_cast<double>(p.total_site_entries), 0.0);

  const int32_t arith = prec == TN_PREC_F64 ? AR_F64 : (prec == TN_PREC_F32 ? AR_F32 : AR_BF16X3);
  // Steps of different units are independent: walk step index t across the
  // units and launch same-kind steps of several units together.
  const size_t nu = p.units.size();
  std::vector<int32_t> final_buf(nu, 0), cur(nu, 0);
  // a seeded cut plan's first absorption reads the supplied boundary in place
  const void* first_in = seeded ? io->seed : nullptr;
  auto args_of = [&](size_t u, int32_t k) {
    const Step& s = p.steps[k];
    AbsorbArgs a;
    a.in = base + L.buf[u][cur[u]];
    a.out = base + L.buf[u][1 - cur[u]];
    a.in_type = L.out_type[k - 1];
    a.out_type = L.out_type[k];
    a.arith = arith;
    a.pre = s.pre; a.K = s.K; a.N = s.N; a.post = s.post;
    a.s_off = L.s_off[k];
    a.scale_slot = s.scale_in >= 0 ? slot_exp + s.scale_in : nullptr;
    a.max_slot = s.rescale >= 0 ? slot_exp + s.rescale : nullptr;
    return a;
  };
  auto step_bytes = [&](const AbsorbArgs& a, const Step& s) {
    const double sb = a.out_type == EL_F64 ? 8.0 : (prec == TN_PREC_F64 ? 8.0 : 4.0);
    return static_cast<double>(s.pre * s.K * s.post) * elem_bytes(a.in_type) +
           static_cast<double>(s.out) * elem_bytes(a.out_type) +
           static_cast<double>(s.K * s.N) * sb;
  };
  // Per unit, the absorption steps in order, each either alone or fused with
  // the next one (first step index of each action; pair flag).
  // Per unit, the absorption steps in order: alone, fused with the next one
  // (pair), or the first of a column chunk of `len` steps.
  enum { ACT_ONE = 0, ACT_PAIR = 1, ACT_CHUNK = 2, ACT_CHAIN = 3, ACT_EDGE = 4 };
  // the fused edge pair starting at step k of unit u (kind from edge_kind)
  auto edge_args = [&](size_t u, int32_t k, int32_t kind) {
    const Step& s1 = p.steps[k];
    const Step& s2 = p.steps[k + 1];
    const AbsorbArgs a = args_of(u, k);
    EdgeArgs e;
    e.in = a.in;
    e.out = a.out;
    e.in_type = L.out_type[k - 1];
    e.out_type = L.out_type[k + 1];
    e.arith = arith;
    e.head = kind == 1;
    e.n2 = static_cast<int32_t>(s2.N);
    e.pre1 = s1.pre;
    e.post2 = s2.post;
    e.s_off1 = L.s_off[k];
    e.s_off2 = L.s_off[k + 1];
    e.scale_slot = a.scale_slot;
    e.max_slot = s2.rescale >= 0 ? slot_exp + s2.rescale : nullptr;
    return e;
  };
  struct Action { int32_t k, kind, len, sub = 0; };   // sub: edge_kind of an ACT_EDGE
  std::vector<std::vector<Action>> acts(nu);
  size_t max_acts = 0;
  const int32_t fuse = absorb_policy() == 0 ? fuse_steps() : 0;
  for (size_t u = 0; u < nu; ++u) {
    const Unit& U = p.units[u];
    const int32_t end = U.first_step + U.n_steps;
    for (int32_t k = U.first_step + 1; k < end;) {
      Action a{k, ACT_ONE, 1};
      const bool pair = k + 1 < end && pair_ok(p.steps[k], p.steps[k + 1]) &&
                        L.out_type[k - 1] == L.out_type[k] && L.out_type[k] == L.out_type[k + 1];
      const int32_t ek = fuse == 2 ? edge_kind(p, k, end) : 0;
      if (ek && L.out_type[k] == L.out_type[k + 1] && edge_pair_supported(edge_args(u, k, ek))) {
        a = {k, ACT_EDGE, 2, ek};
      } else if (fuse == 2) {
        // the rest of the column in as few chunks as the longest chunk
        // allows, their lengths as equal as possible (6 rows: 3 + 3, not
        // 4 + 2; 12 rows: 4 + 4 + 4); two rows go to the pair kernel where it
        // applies (a 2-row slice is too small to amortise a chunk workgroup)
        int32_t ce = k;
        while (ce < end && p.steps[ce].kind == STEP_ABSORB && p.steps[ce].col == p.steps[k].col)
          ++ce;
        const int32_t kmax = chunk_max_steps(L.out_type[k - 1]);
        const int32_t passes = (ce - k + kmax - 1) / kmax;
        const int32_t even = passes > 0 ? (ce - k + passes - 1) / passes : kmax;
        for (int32_t len = std::min(std::max(even, 2), end - k); len >= 2; --len)
          if (chunk_ok(p, L, k, len)) { a = {k, ACT_CHUNK, len}; break; }
        if (a.kind == ACT_CHUNK && a.len == 2 && pair) a = {k, ACT_PAIR, 2};
      } else if (fuse == 1 && pair) {
        a = {k, ACT_PAIR, 2};
      }
      acts[u].push_back(a);
      k += a.len;
    }
    if (fuse == 2 && g_chain_steps) {
      // runs of small single steps: one workgroup, one launch
      auto small = [&](const Action& a) {
        const Step& st = p.steps[a.k];
        return a.kind == ACT_ONE && st.kind == STEP_ABSORB && st.out <= kChainEntries &&
               st.pre * st.K * st.post <= kChainEntries;
      };
      std::vector<Action> merged;
      for (size_t i = 0; i < acts[u].size();) {
        size_t j = i;
        while (j < acts[u].size() && small(acts[u][j]) && j - i < static_cast<size_t>(kChainMax)) ++j;
        if (j - i >= 2) {
          merged.push_back({acts[u][i].k, ACT_CHAIN, static_cast<int32_t>(j - i)});
          i = j;
        } else {
          merged.push_back(acts[u][i]);
          ++i;
        }
      }
      acts[u].swap(merged);
    }
    max_acts = std::max(max_acts, acts[u].size());
  }
  // Launch action t of the units in `units` on stream `st` (same-kind steps of
  // several units go out together).
#define TN_HIP_L(call)                                        \
  do {                                                        \
    const hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) {                                   \
      err = std::string(#call) + ": " + hip_msg(e_);          \
      return TN_EDEVICE;                                      \
    }                                                         \
  } while (0)
  auto launch_actions = [&](const std::vector<size_t>& units, size_t t, hipStream_t st,
                            LaunchTimer& tm) -> tn_status {
    AbsorbArgs group[4];
    const Step* gsteps[4];
    PairArgs pairs[4];
    ChunkArgs chunks[4];
    ChainUnit chains[4];
    EdgeArgs edges[4];
    double pair_bytes = 0.0, pair_flops = 0.0, chunk_bytes = 0.0, chunk_flops = 0.0;
    double chain_bytes = 0.0, chain_flops = 0.0, edge_bytes[4], edge_flops[4];
    int32_t n = 0, np = 0, nc = 0, nch = 0, ne = 0;
    for (size_t u : units) {
      if (t >= acts[u].size()) continue;
      const Action& ac = acts[u][t];
      AbsorbArgs a = args_of(u, ac.k);
      const void* in0 = (u == 0 && t == 0) ? first_in : nullptr;
      if (in0) a.in = in0;
      if (ac.kind == ACT_CHAIN) {
        ChainUnit& x = chains[nch++];
        x.buf[0] = base + L.buf[u][0];
        x.buf[1] = base + L.buf[u][1];
        x.in0 = in0;
        x.cur = cur[u];
        x.n = ac.len;
        for (int32_t j = 0; j < ac.len; ++j) {
          const int32_t k = ac.k + j;
          const Step& sj = p.steps[k];
          ChainStep& c = x.s[j];
          c.pre = sj.pre; c.post = sj.post; c.s_off = L.s_off[k];
          c.K = static_cast<int32_t>(sj.K); c.N = static_cast<int32_t>(sj.N);
          c.in_f64 = L.out_type[k - 1] == EL_F64;
          c.out_f64 = L.out_type[k] == EL_F64;
          c.rescale_slot = sj.rescale;
          c.scale_slot = sj.scale_in;
          chain_bytes += step_bytes(args_of(u, k), sj);
          chain_flops += static_cast<double>(sj.flops);
        }
        // every step of the chain swaps the buffers; the common swap below is one
        if ((ac.len & 1) == 0) cur[u] = 1 - cur[u];
      } else if (ac.kind == ACT_CHUNK) {
        const Step& s1 = p.steps[ac.k];
        const Step& sl = p.steps[ac.k + ac.len - 1];
        ChunkArgs& x = chunks[nc++];
        x.in = a.in;
        x.out = a.out;
        x.type = a.in_type;
        x.arith = arith;
        x.pre = s1.pre;
        x.post = sl.post;
        x.k = ac.len;
        x.k1 = static_cast<int32_t>(s1.K);
        x.nl = static_cast<int32_t>(sl.N);
        for (int32_t j = 0; j < kChunkMax; ++j) x.s_off[j] = j < ac.len ? L.s_off[ac.k + j] : 0;
        x.scale_slot = a.scale_slot;
        x.max_slot = sl.rescale >= 0 ? slot_exp + sl.rescale : nullptr;
        const double eb = elem_bytes(a.in_type);
        chunk_bytes += static_cast<double>(s1.pre * s1.K * s1.post) * eb +
                       static_cast<double>(sl.out) * eb;
        for (int32_t j = 0; j < ac.len; ++j) {
          const Step& sj = p.steps[ac.k + j];
          chunk_bytes += static_cast<double>(sj.K * sj.N) * eb;
          chunk_flops += static_cast<double>(sj.flops);
        }
      } else if (ac.kind == ACT_EDGE) {
        const Step& s1 = p.steps[ac.k];
        const Step& s2 = p.steps[ac.k + 1];
        EdgeArgs e = edge_args(u, ac.k, ac.sub);
        e.in = a.in;
        edge_bytes[ne] = static_cast<double>(s1.pre * s1.K * s1.post) * elem_bytes(e.in_type) +
                         static_cast<double>(s2.out) * elem_bytes(e.out_type);
        edge_flops[ne] = static_cast<double>(s1.flops + s2.flops);
        edges[ne++] = e;
      } else if (ac.kind == ACT_PAIR) {
        const Step& s1 = p.steps[ac.k];
        const Step& s2 = p.steps[ac.k + 1];
        PairArgs& x = pairs[np++];
        x.in = a.in;
        x.out = a.out;
        x.type = a.in_type;
        x.arith = arith;
        x.pre = s1.pre;
        x.post2 = s2.post;
        x.s_off1 = L.s_off[ac.k];
        x.s_off2 = L.s_off[ac.k + 1];
        x.scale_slot = a.scale_slot;
        x.max_slot = s2.rescale >= 0 ? slot_exp + s2.rescale : nullptr;
        const double eb = elem_bytes(a.in_type);
        pair_bytes += static_cast<double>(s1.pre * s1.K * s1.post) * eb +
                      static_cast<double>(s2.out) * eb + 2.0 * 256.0 * eb;
        pair_flops += static_cast<double>(s1.flops + s2.flops);
      } else {
        group[n] = a;
        gsteps[n] = &p.steps[ac.k];
        ++n;
      }
      cur[u] = 1 - cur[u];
    }
    if (nc > 0) {
      const char* cname = "";
      tm.before();
      TN_HIP_L(launch_absorb_chunks(chunks, nc, sa, state, st, &cname));
      tm.after(cname, chunk_bytes, chunk_flops);
    }
    const char* kname = "";
    if (ne > 0) {
      bool same = true;
      for (int32_t i = 1; i < ne; ++i)
        same = same && edges[i].head == edges[0].head && edges[i].n2 == edges[0].n2 &&
               edges[i].in_type == edges[0].in_type && edges[i].out_type == edges[0].out_type;
      if (same) {
        double b = 0.0, f = 0.0;
        for (int32_t i = 0; i < ne; ++i) { b += edge_bytes[i]; f += edge_flops[i]; }
        tm.before();
        TN_HIP_L(launch_absorb_edges(edges, ne, sa, state, st, &kname));
        tm.after(kname, b, f);
      } else {
        for (int32_t i = 0; i < ne; ++i) {
          tm.before();
          TN_HIP_L(launch_absorb_edges(&edges[i], 1, sa, state, st, &kname));
          tm.after(kname, edge_bytes[i], edge_flops[i]);
        }
      }
    }
    if (np > 0) {
      tm.before();
      TN_HIP_L(launch_absorb_pairs(pairs, np, sa, state, st, &kname));
      tm.after(kname, pair_bytes, pair_flops);
    }
    if (nch > 0) {
      tm.before();
      TN_HIP_L(launch_chain(chains, nch, sa, slot_exp, &state->flags, arith, st, &kname));
      tm.after(kname, chain_bytes, chain_flops);
    }
    if (n > 1 && absorb_policy() == 0 && absorb_group_supported(group, n)) {
      double bytes = 0.0, flops = 0.0;
      for (int32_t i = 0; i < n; ++i) {
        bytes += step_bytes(group[i], *gsteps[i]);
        flops += static_cast<double>(gsteps[i]->flops);
      }
      tm.before();
      TN_HIP_L(launch_absorb_group(group, n, sa, state, st, &kname));
      tm.after(kname, bytes, flops);
    } else {
      for (int32_t i = 0; i < n; ++i) {
        tm.before();
        TN_HIP_L(launch_absorb(group[i], sa, state, st, &kname));
        tm.after(kname, step_bytes(group[i], *gsteps[i]), static_cast<double>(gsteps[i]->flops));
      }
    }
    return TN_OK;
  };
#undef TN_HIP_L
  // Quadrant plans with a side stream: the bottom units (ya, yb) run on the
  // side stream, concurrently with the top units and the first ring product.
  const bool split_streams = p.has_ring && nu == 4 && side != nullptr && side_timer != nullptr;
  std::vector<size_t> main_units, side_units;
  if (split_streams) {
    main_units = {static_cast<size_t>(p.ring.xa), static_cast<size_t>(p.ring.xb)};
    side_units = {static_cast<size_t>(p.ring.ya), static_cast<size_t>(p.ring.yb)};
    TN_HIP(hipEventRecord(side->fork, stream));
    TN_HIP(hipStreamWaitEvent(side->stream, side->fork, 0));
  } else {
    for (size_t u = 0; u < nu; ++u) main_units.push_back(u);
  }
  for (size_t t = 0; t < max_acts; ++t) {
    // at most four units' actions go out together (the launchers' group size)
    for (size_t g0 = 0; g0 < main_units.size(); g0 += 4) {
      const std::vector<size_t> grp(main_units.begin() + g0,
                                    main_units.begin() + std::min(main_units.size(), g0 + 4));
      tn_status st = launch_actions(grp, t, stream, timer);
      if (st != TN_OK) return st;
    }
    if (split_streams) {
      tn_status st = launch_actions(side_units, t, side->stream, *side_timer);
      if (st != TN_OK) return st;
    }
  }
  // a rescale on the INIT step of a one-row unit needs no measurement: its
  // slot stays "zero" and scales by 2^0
  for (size_t u = 0; u < nu; ++u) final_buf[u] = cur[u];

  tn_result* copy = io ? io->result : nullptr;
  if (open_end) {
    const size_t kl = p.steps.size() - 1;
    const Step& sl = p.steps[kl];
    const char* fin = base + L.buf[0][final_buf[0]];
    // inside a column there is no rescale point: no shift, no exponent
    const int32_t* slot_last = sl.rescale >= 0 ? slot_exp + sl.rescale : nullptr;
    if (io->cap) {
      const int32_t f64 = L.out_type[kl] == EL_F64;
      timer.before();
      TN_HIP(launch_env_cap(fin, io->cap, sl.out, f64, slot_last, io->cap_rec, io->partials,
                            stream));
      timer.after("env_cap", 2.0 * static_cast<double>(sl.out) * (f64 ? 8.0 : 4.0),
                  2.0 * static_cast<double>(sl.out));
      timer.before();
      TN_HIP(launch_finalize(state, nullptr, copy, io->partials, env_cap_blocks(sl.out), stream,
                             io->cap_rec));
      timer.after("finalize", 0.0, 0.0);
    } else {
      *io->tap = fin;
      timer.before();
      TN_HIP(launch_env_tap(state, slot_last, io->tap_rec, stream));
      timer.after("env_tap", 0.0, 0.0);
    }
  } else if (!p.chain.empty()) {
    // the row chain: v = first row's tensor, then one matrix-vector product
    // per row in float64, each rescaled exactly but the last (the scalar)
    auto unit_out = [&](int32_t u, int32_t* type) {
      const Unit& U = p.units[u];
      *type = L.out_type[U.first_step + U.n_steps - 1];
      return static_cast<const void*>(base + L.buf[u][final_buf[u]]);
    };
    const double* vout = nullptr;
    for (size_t i = 0; i < p.chain.size(); ++i) {
      const Link& lk = p.chain[i];
      LinkArgs a;
      int32_t vt = EL_F64, rt = EL_F64;
      a.v = i == 0 ? unit_out(0, &vt) : static_cast<const void*>(vout);
      a.v_f64 = vt == EL_F64;
      a.R = unit_out(lk.unit, &rt);
      a.R_f64 = rt == EL_F64;
      a.K = lk.K; a.N = lk.N; a.side = lk.side;
      a.slot_v = lk.scale_v >= 0 ? slot_exp + lk.scale_v : nullptr;
      const int32_t rs = p.units[lk.unit].final_slot;
      a.slot_R = rs >= 0 ? slot_exp + rs : nullptr;
      a.out = reinterpret_cast<double*>(base + L.vbuf[i & 1]);
      a.max_slot = lk.rescale >= 0 ? slot_exp + lk.rescale : nullptr;
      a.flags = &state->flags;
      a.partials = reinterpret_cast<double*>(base + L.link_partials);
      timer.before();
      TN_HIP(launch_row_link(a, stream));
      timer.after(a.v_f64 && a.R_f64 ? "row_link_f64" : "row_link_f32_to_f64",
                  static_cast<double>(lk.K * lk.N) * (a.R_f64 ? 8.0 : 4.0) +
                      static_cast<double>(lk.K) * (a.v_f64 ? 8.0 : 4.0) +
                      8.0 * static_cast<double>(lk.N),
                  static_cast<double>(lk.flops));
      vout = a.out;
    }
    timer.before();
    TN_HIP(launch_finalize(state, vout, copy, nullptr, 0, stream));
    timer.after("finalize", 0.0, 0.0);
  } else if (!p.has_ring) {
    const double* scalar = reinterpret_cast<const double*>(base + L.buf[0][final_buf[0]]);
    timer.before();
    TN_HIP(launch_finalize(state, scalar, copy, nullptr, 0, stream));
    timer.after("finalize", 0.0, 0.0);
  } else {
    const Ring& g = p.ring;
    const int32_t t = prec == TN_PREC_F64 ? EL_F64 : EL_F32;
    auto unit_ptr = [&](int32_t u) { return base + L.buf[u][final_buf[u]]; };
    auto unit_slot = [&](int32_t u) -> const int32_t* {
      const int32_t s = p.units[u].final_slot;
      return s >= 0 ? slot_exp + s : nullptr;
    };
    int64_t n_part = 0;
    const char* kname = "";
    const double es = (t == EL_F64) ? 8.0 : 4.0;
    double* partials = reinterpret_cast<double*>(base + L.partials);
    // X = TL^T TR (units xa, xb) first, stored; then Yt = BL^T BR (units ya,
    // yb) with the float64 dot sum X o Yt fused into its epilogue.  With a
    // side stream the bottom units were swept there: join before Yt.
    hipStream_t ys = split_streams ? side->stream : stream;
    LaunchTimer& ytm = split_streams ? *side_timer : timer;
    auto join = [&]() -> hipError_t {
      if (!split_streams) return hipSuccess;
      hipError_t e2 = hipEventRecord(side->join, side->stream);
      if (e2 == hipSuccess) e2 = hipStreamWaitEvent(stream, side->join, 0);
      return e2;
    };
    if (L.split_ring && absorb_policy() == 0) {
      // BF16x3: split + transpose each quadrant tensor once, then NT GEMMs
      const int64_t rows[4] = {g.m, g.n, g.n, g.m};
      const int64_t kk[4] = {g.kx, g.kx, g.ky, g.ky};
      uint16_t* hs[4];
      uint16_t* ls[4];
      for (int u = 0; u < 4; ++u) {
        hs[u] = reinterpret_cast<uint16_t*>(base + L.split[u][0]);
        ls[u] = reinterpret_cast<uint16_t*>(base + L.split[u][1]);
      }
      auto split = [&](int32_t u, hipStream_t st, LaunchTimer& tm) -> hipError_t {
        tm.before();
        const hipError_t e2 = launch_split_transpose(reinterpret_cast<const float*>(unit_ptr(u)),
                                                     kk[u], rows[u], unit_slot(u), hs[u], ls[u], st);
        tm.after("split_transpose",
                 4.0 * static_cast<double>(kk[u] * rows[u]) +
                     4.0 * static_cast<double>(rows[u] * split_k_padded(kk[u])),
                 0.0);
        return e2;
      };
      TN_HIP(split(g.xa, stream, timer));
      TN_HIP(split(g.xb, stream, timer));
      TN_HIP(split(g.ya, ys, ytm));
      TN_HIP(split(g.yb, ys, ytm));
      NtArgs x{};
      x.Ah = hs[g.xa]; x.Al = ls[g.xa]; x.Bh = hs[g.xb]; x.Bl = ls[g.xb];
      x.m = g.m; x.n = g.n; x.kp = split_k_padded(g.kx);
      x.c_out = reinterpret_cast<float*>(base + L.yt); x.dot_with = nullptr;
      x.c_slices_cap = L.yt_slices;
      int32_t x_slices = 0;
      int64_t unused = 0;
      timer.before();
      TN_HIP(launch_ring_bf16x3_nt(x, stream, &unused, &x_slices));
      timer.after("ring_mfma_bf16x3",
                  es * static_cast<double>(g.kx * (g.m + g.n) + x_slices * g.m * g.n),
                  2.0 * static_cast<double>(g.m * g.n * g.kx));
      TN_HIP(join());
      NtArgs y{};
      y.Ah = hs[g.ya]; y.Al = ls[g.ya]; y.Bh = hs[g.yb]; y.Bl = ls[g.yb];
      y.m = g.m; y.n = g.n; y.kp = split_k_padded(g.ky);
      y.c_out = nullptr; y.dot_with = reinterpret_cast<const float*>(base + L.yt);
      y.w_slices = x_slices;
      y.partials = partials; y.partials_cap = L.n_partials;
      int32_t none = 0;
      timer.before();
      TN_HIP(launch_ring_bf16x3_nt(y, stream, &n_part, &none));
      timer.after("ring_mfma_bf16x3",
                  es * static_cast<double>(g.ky * (g.m + g.n) + x_slices * g.m * g.n),
                  2.0 * static_cast<double>(g.m * g.n * g.ky) + 2.0 * static_cast<double>(g.m * g.n));
    } else {
      RingArgs x;
      x.A = unit_ptr(g.xa); x.B = unit_ptr(g.xb);
      x.type = t; x.arith = arith;
      x.m = g.m; x.n = g.n; x.k = g.kx;
      x.sa = unit_slot(g.xa); x.sb = unit_slot(g.xb);
      x.c_out = base + L.yt; x.dot_with = nullptr; x.partials = nullptr;
      x.c_slices_cap = L.yt_slices;
      int32_t x_slices = 0;
      int64_t unused = 0;
      timer.before();
      TN_HIP(launch_ring(x, stream, &kname, &unused, &x_slices));
      timer.after(kname, es * static_cast<double>(g.kx * (g.m + g.n) + x_slices * g.m * g.n),
                  2.0 * static_cast<double>(g.m * g.n * g.kx));
      TN_HIP(join());
      RingArgs y = x;
      y.A = unit_ptr(g.ya); y.B = unit_ptr(g.yb);
      y.k = g.ky;
      y.sa = unit_slot(g.ya); y.sb = unit_slot(g.yb);
      y.c_out = nullptr; y.dot_with = base + L.yt;
      y.w_slices = x_slices;
      y.partials = partials; y.partials_cap = L.n_partials;
      int32_t none = 0;
      timer.before();
      TN_HIP(launch_ring(y, stream, &kname, &n_part, &none));
      timer.after(kname, es * static_cast<double>(g.ky * (g.m + g.n) + x_slices * g.m * g.n),
                  2.0 * static_cast<double>(g.m * g.n * g.ky) + 2.0 * static_cast<double>(g.m * g.n));
    }
    timer.before();
    TN_HIP(launch_finalize(state, nullptr, copy, partials, n_part, stream));
    timer.after("finalize", 0.0, 0.0);
  }
#undef TN_HIP
  return TN_OK;
}

// Copies the result record back once the stream has drained and folds the
// launch timings in.
tn_status finish(const Plan& p, int32_t prec, void* ws, hipStream_t stream, HostKeep& keep,
                 LaunchTimer& timer, LaunchTimer* side_timer, tn_result* out, std::string& err);

tn_status contract(const Plan& p, const double* const* sites, bool on_device, int32_t prec,
                   void* ws, size_t ws_bytes, hipStream_t stream, tn_result* out,
                   std::string& err) {
  // each call waits for its stream before returning, so one pinned image per
  // thread is free again at the next call; it is kept until the process ends
  // (never freed from a thread-exit destructor that may run after the HIP
  // runtime has shut down)
  thread_local HostKeep* const keep_ptr = new HostKeep;
  HostKeep& keep = *keep_ptr;
  // one side stream per thread and device, kept like the pinned image; only
  // with the quadrant-streams option (each stream takes one of the process's
  // few hardware queues)
  thread_local int side_dev = -1;
  thread_local SideStream side;
  thread_local bool side_ok = false;
  int dev = 0;
  if (g_quadrant_streams && hipGetDevice(&dev) == hipSuccess && dev != side_dev) {
    side = SideStream{};
    side_ok = hipStreamCreateWithFlags(&side.stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&side.fork, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&side.join, hipEventDisableTiming) == hipSuccess;
    side_dev = dev;
  }
  const bool use_side = g_quadrant_streams && side_ok;
  LaunchTimer timer(stream);
  LaunchTimer side_timer(use_side ? side.stream : stream, use_side);
  const tn_status s = enqueue(p, sites, on_device, prec, ws, ws_bytes, stream, keep, timer, err,
                              use_side ? &side : nullptr, use_side ? &side_timer : nullptr);
  if (s != TN_OK) return s;
  return finish(p, prec, ws, stream, keep, timer, &side_timer, out, err);
}

tn_status contract_with(const Plan& p, const double* const* sites, bool on_device, int32_t prec,
                        void* ws, size_t ws_bytes, hipStream_t stream, HostKeep& keep,
                        bool timed, tn_result* out, std::string& err) {
  LaunchTimer timer(stream, timed);
  const tn_status s = enqueue(p, sites, on_device, prec, ws, ws_bytes, stream, keep, timer, err);
  if (s != TN_OK) return s;
  return finish(p, prec, ws, stream, keep, timer, nullptr, out, err);
}

tn_status finish(const Plan& p, int32_t prec, void* ws, hipStream_t stream, HostKeep& keep,
                 LaunchTimer& timer, LaunchTimer* side_timer, tn_result* out, std::string& err) {
  const Layout L = make_layout(p, prec);
  const DevState* state = reinterpret_cast<const DevState*>(static_cast<char*>(ws) + L.state);
  tn_result* staged = reinterpret_cast<tn_result*>(keep.data() + head_bytes(p, L));
  hipError_t e = hipMemcpyAsync(staged, &state->result, sizeof(tn_result), hipMemcpyDeviceToHost,
                                stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    err = std::string("result copy: ") + hip_msg(e);
    return TN_EDEVICE;
  }
  *out = *staged;
  timer.flush();
  if (side_timer) side_timer->flush();
  if (out->status != TN_OK) {
    err = "non-finite value in the inputs or an intermediate";
    return out->status;
  }
  return TN_OK;
}

}  // namespace tn
