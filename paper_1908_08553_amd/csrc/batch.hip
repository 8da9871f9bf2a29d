// Many independent lattices in one captured launch graph.
//
// The paper evaluates physical quantities by contracting many planar
// networks (§5: one contraction per local observable, L^2 + 2L(L-1) per
// evaluation), so independent contractions are the natural unit of batching.
//
// Two paths run side by side in the graph, on two captured streams:
//  * lock-step: the `split` costliest lattices advance one sweep step per
//    launch, every step spread over as many workgroups as its size calls
//    for (the same step bodies, each 64-fibre super-block or 16-row block
//    computed whole by one wave, so results do not depend on the split);
//    rescale exponents go through per-lattice slots (atomicMax), and a last
//    launch assembles the results;
//  * one workgroup per lattice for the rest, described below.
// Without the split the costliest lattice, swept by one compute unit, sets
// the batch's time.
//
// Workgroup b of the one-workgroup kernel sweeps lattice order[b]
// column by column with all of its waves, the order putting the costliest
// lattices first so the dispatcher (which starts workgroups in index order as
// compute units free up) schedules largest-first; the lattice's two boundary
// buffers are its own, so no data crosses workgroups and the only
// synchronisation is the workgroup barrier between steps.  There is
// deliberately no device-side work counter: a claim loop whose body ends and
// begins with single-lane regions (store the result, claim the next lattice)
// lets the compiler merge them across the back-edge into an inner loop that
// only lane 0 can leave, which livelocks the workgroup.  Per-column rescaling is a workgroup reduction, the exponent sum is
// kept in registers and the result record is assembled by the workgroup that
// finished the lattice.  Staging + the batch kernels are captured once in a
// hipGraph and replayed; only the site pointers change between runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "absorb_device.hpp"
#include "batch.hpp"
#include "exec.hpp"

namespace tn {
namespace {

using namespace dev;

constexpr int kMaxWaves = 16;

struct BStep {
  int64_t pre, post, s_off;
  int32_t K, N;
  int32_t in_f64, out_f64;
  int32_t rescale;    // measure the max exponent after this step
  int32_t scale_in;   // scale the input by the last measured exponent
  int32_t rslot;      // lock-step: the lattice's slot measured after it (-1: none)
  int32_t sslot;      // lock-step: the slot that scales its input (-1: none)
};

struct BLattice {
  int64_t buf0, buf1;        // byte offsets of the two boundary buffers
  int32_t first_step, n_steps;
  int32_t first_site_step;   // index of its first step in the staging tables
  int32_t slot0, n_slots;    // lock-step: its rescale slots in the slot table
  int32_t pad;
};

// Lock-step launch t: item i covers workgroups [wg0, wg0 + nwg) of lattice
// `lat`'s step t (items sorted by wg0).
struct LsItem {
  int32_t lat, wg0, nwg, pad;
};

// One step by the waves wave, wave + nw, ... (and, for the vector-ALU body,
// threads tid0, tid0 + nth, ...) of the caller.
__device__ inline void run_step(const BStep& s, const void* in, void* out, int32_t shift,
                                int32_t arith, const StagedArrays& st, uint32_t wave,
                                uint32_t nw, double& mx, int& bad, int64_t tid0 = -1,
                                int64_t nth = 0) {
  const uint16_t* shi = st.shi + s.s_off;
  const uint16_t* slo = st.slo + s.s_off;
  if (tid0 < 0) {
    tid0 = threadIdx.x;
    nth = blockDim.x;
  }
  if (s.out_f64) {
    double m = 0.0;
    const double* S = st.s64 + s.s_off;
    double* o = static_cast<double*>(out);
    if (s.in_f64) {
      const double* i = static_cast<const double*>(in);
      if (wide_ok(s.pre, s.K, s.N, s.post))
        wide_body<double, double, M_F64>(i, o, S, shi, slo, s.pre, s.K, s.N, s.post, shift, wave, nw, m, bad);
      else if (narrow_ok(s.pre, s.K, s.N, s.post))
        narrow_body<double, double, M_F64>(i, o, S, shi, slo, s.pre, s.K, s.N, shift, wave, nw, m, bad);
      else
        generic_body<double, double, false>(i, o, S, shi, slo, s.pre, s.K, s.N, s.post, shift, tid0, nth, m, bad);
    } else {
      const float* i = static_cast<const float*>(in);
      if (wide_ok(s.pre, s.K, s.N, s.post))
        wide_body<float, double, M_F64>(i, o, S, shi, slo, s.pre, s.K, s.N, s.post, shift, wave, nw, m, bad);
      else if (narrow_ok(s.pre, s.K, s.N, s.post))
        narrow_body<float, double, M_F64>(i, o, S, shi, slo, s.pre, s.K, s.N, shift, wave, nw, m, bad);
      else
        generic_body<float, double, false>(i, o, S, shi, slo, s.pre, s.K, s.N, s.post, shift, tid0, nth, m, bad);
    }
    mx = fmax(mx, m);
    return;
  }
  float m = 0.f;
  const float* S = st.s32 + s.s_off;
  const float* i = static_cast<const float*>(in);
  float* o = static_cast<float*>(out);
  if (arith == AR_BF16X3) {
    if (wide_ok(s.pre, s.K, s.N, s.post))
      wide_body<float, float, M_BF16X3>(i, o, S, shi, slo, s.pre, s.K, s.N, s.post, shift, wave, nw, m, bad);
    else if (narrow_ok(s.pre, s.K, s.N, s.post))
      narrow_body<float, float, M_BF16X3>(i, o, S, shi, slo, s.pre, s.K, s.N, shift, wave, nw, m, bad);
    else
      generic_body<float, float, true>(i, o, S, shi, slo, s.pre, s.K, s.N, s.post, shift, tid0, nth, m, bad);
  } else {
    if (wide_ok(s.pre, s.K, s.N, s.post))
      wide_body<float, float, M_F32>(i, o, S, shi, slo, s.pre, s.K, s.N, s.post, shift, wave, nw, m, bad);
    else if (narrow_ok(s.pre, s.K, s.N, s.post))
      narrow_body<float, float, M_F32>(i, o, S, shi, slo, s.pre, s.K, s.N, shift, wave, nw, m, bad);
    else
      generic_body<float, float, false>(i, o, S, shi, slo, s.pre, s.K, s.N, s.post, shift, tid0, nth, m, bad);
  }
  mx = fmax(mx, static_cast<double>(m));
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void batch_kernel(
    const BLattice* __restrict__ lats, const int32_t* __restrict__ order, int32_t n,
    const BStep* __restrict__ steps, char* __restrict__ ws, StagedArrays st,
    const int32_t* __restrict__ site_exp, const int32_t* __restrict__ site_bad,
    tn_result* __restrict__ results, int32_t arith) {
  __shared__ double s_max[kMaxWaves];
  __shared__ int s_bad[kMaxWaves];
  const uint32_t wave = threadIdx.x >> 6, nw = THREADS / 64;
  if (static_cast<int32_t>(blockIdx.x) < n) {
    const int32_t idx = order[blockIdx.x];
    const BLattice L = lats[idx];
    int64_t E = 0;
    int bad = 0;
    int32_t shift = 0;
    int cur = 0;
    for (int32_t k = L.first_step + 1; k < L.first_step + L.n_steps; ++k) {
      const BStep s = steps[k];
      const void* in = ws + (cur ? L.buf1 : L.buf0);
      void* out = ws + (cur ? L.buf0 : L.buf1);
      double mx = 0.0;
      int b = 0;
      run_step(s, in, out, s.scale_in ? shift : 0, arith, st, wave, nw, mx, b);
      if (s.rescale) {
        for (int off = 32; off > 0; off >>= 1) {
          mx = fmax(mx, __shfl_xor(mx, off));
          b |= __shfl_xor(b, off);
        }
        if ((threadIdx.x & 63) == 0) { s_max[wave] = mx; s_bad[wave] = b; }
        __syncthreads();
        double m = 0.0;
        int bb = 0;
        for (uint32_t w = 0; w < nw; ++w) { m = fmax(m, s_max[w]); bb |= s_bad[w]; }
        const int32_t e = bb ? kExpBad : exp_of_d(m);
        if (e == kExpBad) { bad = 1; shift = 0; }
        else if (e == kExpZero) shift = 0;
        else { shift = e; E += e; }
      }
      __syncthreads();   // the step's output is complete before anyone reads it
      cur ^= 1;
    }
    if (threadIdx.x == 0) {
      const double m = *reinterpret_cast<const double*>(ws + (cur ? L.buf1 : L.buf0));
      for (int32_t k = 0; k < L.n_steps; ++k) {
        E += site_exp[L.first_site_step + k];
        bad |= site_bad[L.first_site_step + k];
      }
      results[idx] = assemble_result(m, E, bad);
    }
  }
}

// ------------------------------------------------------------------ lock-step
constexpr int kLsThreads = 512;
constexpr int32_t kLsMaxWg = 256;    // most workgroups one lattice step takes

__global__ __launch_bounds__(kLsThreads) void lockstep_reset(int32_t* slots, int32_t n_slots,
                                                             int32_t* flags, int32_t n_lat) {
  for (int32_t i = blockIdx.x * kLsThreads + threadIdx.x; i < n_slots; i += gridDim.x * kLsThreads)
    slots[i] = kExpZero;
  for (int32_t i = blockIdx.x * kLsThreads + threadIdx.x; i < n_lat; i += gridDim.x * kLsThreads)
    flags[i] = 0;
}

__global__ __launch_bounds__(kLsThreads) void lockstep_kernel(
    const LsItem* __restrict__ items, int32_t n_items, int32_t t,
    const BLattice* __restrict__ lats, const BStep* __restrict__ steps, char* __restrict__ ws,
    StagedArrays st, int32_t* __restrict__ slots, int32_t* __restrict__ flags, int32_t arith) {
  const int32_t b = blockIdx.x;
  int32_t lo = 0, hi = n_items - 1;   // last item with wg0 <= b
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (items[mid].wg0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const LsItem it = items[lo];
  const BLattice L = lats[it.lat];
  const BStep s = steps[L.first_step + t];
  const bool odd = ((t - 1) & 1) != 0;
  const void* in = ws + (odd ? L.buf1 : L.buf0);
  void* out = ws + (odd ? L.buf0 : L.buf1);
  const int32_t shift = s.sslot >= 0 ? shift_of(slots + L.slot0 + s.sslot) : 0;
  constexpr uint32_t nw = kLsThreads / 64;
  const uint32_t local = static_cast<uint32_t>(b - it.wg0);
  double mx = 0.0;
  int bad = 0;
  run_step(s, in, out, shift, arith, st, local * nw + (threadIdx.x >> 6),
           static_cast<uint32_t>(it.nwg) * nw, mx, bad,
           static_cast<int64_t>(local) * kLsThreads + threadIdx.x,
           static_cast<int64_t>(it.nwg) * kLsThreads);
  if (s.rslot >= 0)
    reduce_and_publish<double, kLsThreads / 64>(mx, bad, slots + L.slot0 + s.rslot,
                                                flags + it.lat);
}

__global__ __launch_bounds__(kLsThreads) void lockstep_finalize(
    const int32_t* __restrict__ big, int32_t n_big, const BLattice* __restrict__ lats,
    const char* __restrict__ ws, const int32_t* __restrict__ slots,
    const int32_t* __restrict__ flags, const int32_t* __restrict__ site_exp,
    const int32_t* __restrict__ site_bad, tn_result* __restrict__ results) {
  const int32_t j = blockIdx.x * kLsThreads + threadIdx.x;
  if (j >= n_big) return;
  const int32_t i = big[j];
  const BLattice L = lats[i];
  // the last step (n_steps - 1 absorptions after the first) wrote buffer
  // 1 when it was odd-numbered
  const bool in1 = ((L.n_steps - 1) & 1) != 0;
  const double m = *reinterpret_cast<const double*>(ws + (in1 ? L.buf1 : L.buf0));
  int64_t E = 0;
  int bad = flags[i];
  for (int32_t k = 0; k < L.n_slots; ++k) {
    const int32_t e = slots[L.slot0 + k];
    if (e == kExpBad) bad = 1;
    else if (e != kExpZero) E += e;
  }
  for (int32_t k = 0; k < L.n_steps; ++k) {
    E += site_exp[L.first_site_step + k];
    bad |= site_bad[L.first_site_step + k];
  }
  results[i] = assemble_result(m, E, bad);
}

// Workgroups step s takes in the lock-step path: its waves' share of
// super-blocks (wide body), row blocks (narrow body) or fibres (vector-ALU
// body), at most kLsMaxWg.
int32_t lockstep_wgs(const BStep& s) {
  constexpr int64_t nw = kLsThreads / 64;
  int64_t waves;
  if (wide_ok(s.pre, s.K, s.N, s.post)) {
    const int64_t nsb = (s.pre * s.post + 63) / 64;
    waves = (nsb + kSuperPerWave - 1) / kSuperPerWave;
  } else if (narrow_ok(s.pre, s.K, s.N, s.post)) {
    const int64_t nblk = (s.pre + 15) / 16;
    waves = (nblk + kBlocksPerWave - 1) / kBlocksPerWave;
  } else {
    waves = (s.pre * s.post + 63) / 64;
  }
  return static_cast<int32_t>(std::max<int64_t>(1, std::min<int64_t>(kLsMaxWg, (waves + nw - 1) / nw)));
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// ------------------------------------------------------------------ chains
// Small consecutive steps of up to four sweep units, one workgroup per unit:
// the steps' single-launch arithmetic (run_step) with a workgroup barrier
// between steps instead of a kernel boundary.  A rescale slot the chain
// measures is kept in registers for the steps after it; other slots were
// written by earlier launches.
constexpr int kChainUnits = 4;
constexpr int kChainThreads = 512;

struct ChainLaunch {
  ChainUnit u[kChainUnits];
  StagedArrays st;
  int32_t* slot_exp;
  int32_t* flags;
  int32_t arith;
};

__global__ __launch_bounds__(kChainThreads) void chain_kernel(ChainLaunch a) {
  __shared__ double s_max[kChainThreads / 64];
  __shared__ int s_bad[kChainThreads / 64];
  const uint32_t wave = threadIdx.x >> 6, nw = kChainThreads / 64;
  const ChainUnit& c = a.u[blockIdx.x];
  int cur = c.cur;
  int32_t known_slot = -1, known_shift = 0;
  for (int32_t j = 0; j < c.n; ++j) {
    const ChainStep& x = c.s[j];
    int32_t shift = 0;
    if (x.scale_slot >= 0) {
      if (x.scale_slot == known_slot) {
        shift = known_shift;
      } else {
        const int32_t e = a.slot_exp[x.scale_slot];
        shift = (e == kExpZero || e == kExpBad) ? 0 : e;
      }
    }
    BStep s;
    s.pre = x.pre;
    s.post = x.post;
    s.s_off = x.s_off;
    s.K = x.K;
    s.N = x.N;
    s.in_f64 = x.in_f64;
    s.out_f64 = x.out_f64;
    s.rescale = x.rescale_slot >= 0;
    s.scale_in = x.scale_slot >= 0;
    double mx = 0.0;
    int b = 0;
    const void* in = (j == 0 && c.in0) ? c.in0 : c.buf[cur];
    run_step(s, in, c.buf[cur ^ 1], shift, a.arith, a.st, wave, nw, mx, b);
    if (x.rescale_slot >= 0) {
      for (int off = 32; off > 0; off >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, off));
        b |= __shfl_xor(b, off);
      }
      if ((threadIdx.x & 63) == 0) { s_max[wave] = mx; s_bad[wave] = b; }
      __syncthreads();
      double m = 0.0;
      int bb = 0;
      for (uint32_t w = 0; w < nw; ++w) { m = fmax(m, s_max[w]); bb |= s_bad[w]; }
      const int32_t e = bb ? kExpBad : exp_of_d(m);
      if (threadIdx.x == 0) {
        if (e != kExpZero) a.slot_exp[x.rescale_slot] = e;
        if (bb) atomicOr(a.flags, 1);
      }
      known_slot = x.rescale_slot;
      known_shift = (e == kExpZero || e == kExpBad) ? 0 : e;
    }
    __syncthreads();   // the step's output is complete before anyone reads it
    cur ^= 1;
  }
}

}  // namespace

hipError_t launch_chain(const ChainUnit* units, int32_t n, const StagedArrays& st,
                        int32_t* slot_exp, int32_t* flags, int32_t arith, hipStream_t stream,
                        const char** kname) {
  if (n < 1 || n > kChainUnits) return hipErrorInvalidValue;
  ChainLaunch a;
  std::memset(&a, 0, sizeof(a));
  for (int32_t i = 0; i < n; ++i) {
    if (units[i].n < 1 || units[i].n > kChainMax) return hipErrorInvalidValue;
    a.u[i] = units[i];
  }
  a.st = st;
  a.slot_exp = slot_exp;
  a.flags = flags;
  a.arith = arith;
  const bool f64 = units[0].s[0].out_f64 && units[0].s[0].in_f64;
  *kname = f64 ? "absorb_chain_f64" : (arith == AR_BF16X3 ? "absorb_chain_bf16x3" : "absorb_chain_f32");
  hipLaunchKernelGGL(chain_kernel, dim3(static_cast<uint32_t>(n)), dim3(kChainThreads), 0, stream,
                     a);
  return hipGetLastError();
}

struct BatchImpl {
  std::vector<Plan> plan_copies;        // the batch owns copies of its plans
  std::vector<const Plan*> plans;
  std::vector<Layout> layouts;
  int32_t prec = 0;
  int32_t threads = 512, grid = 1, split = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t off_results = 0, off_lats = 0, off_order = 0, off_steps = 0,
         off_descs = 0, off_site_exp = 0, off_site_bad = 0, off_s64 = 0, off_s32 = 0,
         off_shi = 0, off_slo = 0, off_bufs = 0, off_slots = 0, off_lflags = 0,
         off_items = 0, total = 0;
  int32_t n_steps = 0, n_slots = 0;
  int64_t n_staged = 0;
  std::vector<int64_t> s_base;          // staged offset base per lattice
  std::vector<int32_t> step_base;       // first global step per lattice
  std::vector<std::vector<char*>> init_dst;
  std::vector<StageDesc> descs;
  // the site pointers the device descriptors were last built from (the
  // descriptor table in the reserved workspace only changes with them)
  std::vector<const double*> desc_sites;
  bool descs_valid = false;
  tn_result* host_res = nullptr;        // pinned landing buffer of the results
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

tn_status layout_batch(BatchImpl& b, std::string& err) {
  const int32_t n = static_cast<int32_t>(b.plans.size());
  b.layouts.clear();
  b.s_base.assign(n, 0);
  b.step_base.assign(n, 0);
  int64_t staged = 0;
  int32_t steps = 0;
  for (int32_t i = 0; i < n; ++i) {
    const Plan& p = *b.plans[i];
    if (p.order != TN_ORDER_COLSWEEP || p.is_cut) {
      err = "batched contraction needs column-sweep plans";
      return TN_EINVAL;
    }
    b.layouts.push_back(make_layout(p, b.prec));
    b.s_base[i] = staged;
    b.step_base[i] = steps;
    staged += p.total_site_entries;
    steps += static_cast<int32_t>(p.steps.size());
  }
  b.n_steps = steps;
  b.n_staged = std::max<int64_t>(staged, 1);
  b.n_slots = 0;
  for (int32_t i = 0; i < n; ++i) b.n_slots += b.plans[i]->slots;
  size_t off = 0;
  b.off_results = off; off = align_up(off + sizeof(tn_result) * n);
  b.off_lats = off; off = align_up(off + sizeof(BLattice) * n);
  b.off_order = off; off = align_up(off + sizeof(int32_t) * n);
  b.off_steps = off; off = align_up(off + sizeof(BStep) * steps);
  b.off_descs = off; off = align_up(off + sizeof(StageDesc) * steps);
  b.off_site_exp = off; off = align_up(off + sizeof(int32_t) * steps);
  b.off_site_bad = off; off = align_up(off + sizeof(int32_t) * steps);
  b.off_s64 = off; off = align_up(off + 8 * b.n_staged);
  b.off_s32 = off; off = align_up(off + 4 * b.n_staged);
  b.off_shi = off; off = align_up(off + 2 * b.n_staged);
  b.off_slo = off; off = align_up(off + 2 * b.n_staged);
  // lock-step tables, sized for any split: slots of every lattice, a flag
  // per lattice, at most one item per lattice and step
  b.off_slots = off; off = align_up(off + sizeof(int32_t) * std::max(b.n_slots, 1));
  b.off_lflags = off; off = align_up(off + sizeof(int32_t) * n);
  b.off_items = off; off = align_up(off + sizeof(LsItem) * steps);
  b.off_bufs = off;
  for (int32_t i = 0; i < n; ++i) off += 2 * b.layouts[i].buf_bytes[0];
  b.total = off;
  return TN_OK;
}

}  // namespace

tn_status batch_workspace(const Plan* const* plans, int32_t n, int32_t prec, size_t* bytes,
                          std::string& err) {
  BatchImpl b;
  b.plans.assign(plans, plans + n);
  b.prec = prec;
  const tn_status s = layout_batch(b, err);
  if (s != TN_OK) return s;
  *bytes = b.total;
  return TN_OK;
}

tn_status batch_create(const Plan* const* plans, int32_t n, int32_t prec, int32_t threads,
                       void* ws, size_t ws_bytes, BatchImpl** out, std::string& err,
                       int32_t split) {
  if (n < 1) { err = "empty batch"; return TN_EINVAL; }
  if (split < 0 || split > n) { err = "split must be 0..n"; return TN_EINVAL; }
  if (threads != 256 && threads != 512 && threads != 1024) {
    err = "threads must be 256, 512 or 1024";
    return TN_EINVAL;
  }
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) { err = "workspace must be 256-byte aligned"; return TN_EINVAL; }
  auto* b = new BatchImpl;
  b->plan_copies.reserve(n);
  for (int32_t i = 0; i < n; ++i) b->plan_copies.push_back(*plans[i]);
  for (int32_t i = 0; i < n; ++i) b->plans.push_back(&b->plan_copies[i]);
  b->prec = prec;
  b->threads = threads;
  b->split = split;
  tn_status s = layout_batch(*b, err);
  if (s != TN_OK) { delete b; return s; }
  if (ws_bytes < b->total) {
    err = "batch workspace too small: need " + std::to_string(b->total) + " bytes";
    delete b;
    return TN_ENOMEM;
  }
  b->ws = static_cast<char*>(ws);
  b->ws_bytes = ws_bytes;
  if (hipHostMalloc(reinterpret_cast<void**>(&b->host_res), sizeof(tn_result) * n) !=
      hipSuccess) {
    err = "pinned result buffer";
    b->host_res = nullptr;
    delete b;
    return TN_ENOMEM;
  }

  // tables
  std::vector<BLattice> lats(n);
  std::vector<BStep> steps(b->n_steps);
  std::vector<double> cost(n);
  b->init_dst.assign(n, std::vector<char*>(1, nullptr));
  b->descs.assign(b->n_steps, StageDesc{});
  size_t buf_off = b->off_bufs;
  for (int32_t i = 0; i < n; ++i) {
    const Plan& p = *b->plans[i];
    const Layout& L = b->layouts[i];
    BLattice& bl = lats[i];
    bl.buf0 = static_cast<int64_t>(buf_off);
    bl.buf1 = static_cast<int64_t>(buf_off + L.buf_bytes[0]);
    buf_off += 2 * L.buf_bytes[0];
    bl.first_step = b->step_base[i];
    bl.n_steps = static_cast<int32_t>(p.steps.size());
    bl.first_site_step = b->step_base[i];
    bl.slot0 = 0;
    bl.n_slots = p.slots;
    bl.pad = 0;
    b->init_dst[i][0] = b->ws + bl.buf0;
    cost[i] = static_cast<double>(p.flops) + 4.0 * static_cast<double>(p.moved);
    for (size_t k = 0; k < p.steps.size(); ++k) {
      const Step& ps = p.steps[k];
      BStep& bs = steps[b->step_base[i] + k];
      bs.pre = ps.pre; bs.post = ps.post; bs.K = static_cast<int32_t>(ps.K);
      bs.N = static_cast<int32_t>(ps.N);
      bs.s_off = b->s_base[i] + L.s_off[k];
      bs.out_f64 = L.out_type[k] == EL_F64;
      bs.in_f64 = k > 0 ? (L.out_type[k - 1] == EL_F64) : 0;
      bs.rescale = ps.rescale >= 0 && ps.kind == STEP_ABSORB;
      bs.scale_in = ps.scale_in >= 0;
      bs.rslot = (ps.rescale >= 0 && ps.kind == STEP_ABSORB) ? ps.rescale : -1;
      bs.sslot = ps.scale_in;
    }
  }
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return cost[a] > cost[c]; });

  // lock-step set: the `split` costliest lattices; their slots, and the items
  // of every step launch t = 1 .. tmax - 1
  int32_t slot_total = 0, tmax = 0;
  for (int32_t j = 0; j < split; ++j) {
    BLattice& bl = lats[order[j]];
    bl.slot0 = slot_total;
    slot_total += bl.n_slots;
    tmax = std::max(tmax, bl.n_steps);
  }
  std::vector<LsItem> items;
  std::vector<std::pair<size_t, int32_t>> launches;   // (first item, grid) per t
  for (int32_t t = 1; t < tmax; ++t) {
    const size_t first = items.size();
    int32_t wg = 0;
    for (int32_t j = 0; j < split; ++j) {
      const int32_t i = order[j];
      if (t >= lats[i].n_steps) continue;
      const int32_t nwg = lockstep_wgs(steps[lats[i].first_step + t]);
      items.push_back(LsItem{i, wg, nwg, 0});
      wg += nwg;
    }
    launches.push_back({first, wg});
  }

  hipError_t e = hipSuccess;
  b->grid = n - split;   // one workgroup per remaining lattice, largest first

#define TN_HIPB(call)                                        \
  do {                                                       \
    e = (call);                                              \
    if (e != hipSuccess) {                                   \
      err = std::string(#call) + ": " + hipGetErrorString(e); \
      batch_destroy(b);                                      \
      return TN_EDEVICE;                                     \
    }                                                        \
  } while (0)

  TN_HIPB(hipMemcpy(b->ws + b->off_lats, lats.data(), sizeof(BLattice) * n, hipMemcpyHostToDevice));
  TN_HIPB(hipMemcpy(b->ws + b->off_order, order.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
  TN_HIPB(hipMemcpy(b->ws + b->off_steps, steps.data(), sizeof(BStep) * steps.size(),
                    hipMemcpyHostToDevice));
  if (!items.empty())
    TN_HIPB(hipMemcpy(b->ws + b->off_items, items.data(), sizeof(LsItem) * items.size(),
                      hipMemcpyHostToDevice));

  // capture staging, then the lock-step launches on a second stream beside
  // the one-workgroup kernel, once
  hipStream_t cs, cs2;
  hipEvent_t fork, join;
  TN_HIPB(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  if ((e = hipStreamCreateWithFlags(&cs2, hipStreamNonBlocking)) != hipSuccess) {
    (void)hipStreamDestroy(cs);
    TN_HIPB(e);
  }
  if ((e = hipEventCreateWithFlags(&fork, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&join, hipEventDisableTiming)) != hipSuccess) {
    (void)hipStreamDestroy(cs);
    (void)hipStreamDestroy(cs2);
    TN_HIPB(e);
  }
  StagedArrays st{reinterpret_cast<double*>(b->ws + b->off_s64),
                  reinterpret_cast<float*>(b->ws + b->off_s32),
                  reinterpret_cast<uint16_t*>(b->ws + b->off_shi),
                  reinterpret_cast<uint16_t*>(b->ws + b->off_slo)};
  StageTargets tg;
  tg.site_exp = reinterpret_cast<int32_t*>(b->ws + b->off_site_exp);
  tg.site_bad = reinterpret_cast<int32_t*>(b->ws + b->off_site_bad);
  tg.slot_exp = nullptr;
  tg.n_slots = 0;
  tg.flags = nullptr;
  tg.counter = nullptr;
  const int32_t arith = prec == TN_PREC_F64 ? AR_F64 : (prec == TN_PREC_F32 ? AR_F32 : AR_BF16X3);
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    e = launch_stage(reinterpret_cast<const StageDesc*>(b->ws + b->off_descs), b->n_steps, st, tg, cs);
    const BLattice* a_l = reinterpret_cast<const BLattice*>(b->ws + b->off_lats);
    const int32_t* a_o = reinterpret_cast<const int32_t*>(b->ws + b->off_order);
    const BStep* a_s = reinterpret_cast<const BStep*>(b->ws + b->off_steps);
    tn_result* a_r = reinterpret_cast<tn_result*>(b->ws + b->off_results);
    int32_t* a_slots = reinterpret_cast<int32_t*>(b->ws + b->off_slots);
    int32_t* a_flags = reinterpret_cast<int32_t*>(b->ws + b->off_lflags);
    const LsItem* a_items = reinterpret_cast<const LsItem*>(b->ws + b->off_items);
    if (e == hipSuccess && split > 0) {
      e = hipEventRecord(fork, cs);
      if (e == hipSuccess) e = hipStreamWaitEvent(cs2, fork, 0);
      if (e == hipSuccess) {
        const int32_t rb = static_cast<int32_t>(std::max<int64_t>(
            1, std::min<int64_t>(64, (std::max(slot_total, split) + kLsThreads - 1) / kLsThreads)));
        hipLaunchKernelGGL(lockstep_reset, dim3(rb), dim3(kLsThreads), 0, cs2, a_slots,
                           slot_total, a_flags, n);
        e = hipGetLastError();
      }
      for (size_t t = 0; e == hipSuccess && t < launches.size(); ++t) {
        const size_t f0 = launches[t].first;
        const size_t f1 = t + 1 < launches.size() ? launches[t + 1].first : items.size();
        hipLaunchKernelGGL(lockstep_kernel, dim3(static_cast<uint32_t>(launches[t].second)),
                           dim3(kLsThreads), 0, cs2, a_items + f0, static_cast<int32_t>(f1 - f0),
                           static_cast<int32_t>(t + 1), a_l, a_s, b->ws, st, a_slots, a_flags,
                           arith);
        e = hipGetLastError();
      }
      if (e == hipSuccess) {
        hipLaunchKernelGGL(lockstep_finalize, dim3((split + kLsThreads - 1) / kLsThreads),
                           dim3(kLsThreads), 0, cs2, a_o, split, a_l, b->ws, a_slots, a_flags,
                           tg.site_exp, tg.site_bad, a_r);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = hipEventRecord(join, cs2);
    }
    if (e == hipSuccess && b->grid > 0) {
      const dim3 grid(b->grid);
      const int32_t* rest = a_o + split;
      const int32_t nr = n - split;
      if (b->threads == 256)
        hipLaunchKernelGGL(batch_kernel<256>, grid, dim3(256), 0, cs, a_l, rest, nr, a_s, b->ws,
                           st, tg.site_exp, tg.site_bad, a_r, arith);
      else if (b->threads == 512)
        hipLaunchKernelGGL(batch_kernel<512>, grid, dim3(512), 0, cs, a_l, rest, nr, a_s, b->ws,
                           st, tg.site_exp, tg.site_bad, a_r, arith);
      else
        hipLaunchKernelGGL(batch_kernel<1024>, grid, dim3(1024), 0, cs, a_l, rest, nr, a_s, b->ws,
                           st, tg.site_exp, tg.site_bad, a_r, arith);
      e = hipGetLastError();
    }
    if (e == hipSuccess && split > 0) e = hipStreamWaitEvent(cs, join, 0);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess) e = e2;
    b->graph = g;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  (void)hipStreamDestroy(cs2);
  (void)hipEventDestroy(fork);
  (void)hipEventDestroy(join);
  if (e != hipSuccess) {
    err = std::string("graph capture: ") + hipGetErrorString(e);
    batch_destroy(b);
    return TN_EDEVICE;
  }
#undef TN_HIPB
  *out = b;
  return TN_OK;
}

tn_status batch_run(BatchImpl* b, const double* const* const* sites, hipStream_t stream,
                    tn_result* outs, std::string& err) {
  const int32_t n = static_cast<int32_t>(b->plans.size());
  // the staging descriptors depend only on the site pointers: rebuild and
  // upload them when a lattice's pointers changed since the last run
  bool dirty = !b->descs_valid;
  if (b->desc_sites.empty()) {
    size_t total = 0;
    for (int32_t i = 0; i < n; ++i) total += b->plans[i]->rows * b->plans[i]->cols;
    b->desc_sites.assign(total, nullptr);
  }
  for (int32_t i = 0; i < n; ++i) {
    if (!sites[i]) { err = "null site array"; return TN_EINVAL; }
    const Plan& p = *b->plans[i];
    for (int32_t s = 0; s < p.rows * p.cols; ++s)
      if (!sites[i][s]) { err = "null site pointer"; return TN_EINVAL; }
  }
  size_t o = 0;
  for (int32_t i = 0; i < n; ++i) {
    const Plan& p = *b->plans[i];
    const int32_t ns = p.rows * p.cols;
    bool same = b->descs_valid;
    for (int32_t s = 0; same && s < ns; ++s) same = b->desc_sites[o + s] == sites[i][s];
    if (!same) {
      fill_stage_descs(p, b->layouts[i], b->s_base[i], sites[i], b->init_dst[i].data(),
                       b->descs.data() + b->step_base[i]);
      std::copy(sites[i], sites[i] + ns, b->desc_sites.begin() + o);
      dirty = true;
    }
    o += ns;
  }
  hipError_t e = hipSuccess;
  if (dirty) {
    b->descs_valid = false;
    e = hipMemcpyAsync(b->ws + b->off_descs, b->descs.data(), sizeof(StageDesc) * b->descs.size(),
                       hipMemcpyHostToDevice, stream);
  }
  if (e == hipSuccess) e = hipGraphLaunch(b->exec, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->host_res, b->ws + b->off_results, sizeof(tn_result) * n,
                       hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) { err = hipGetErrorString(e); return TN_EDEVICE; }
  b->descs_valid = true;
  std::memcpy(outs, b->host_res, sizeof(tn_result) * n);
  for (int32_t i = 0; i < n; ++i)
    if (outs[i].status != TN_OK) {
      err = "non-finite value in lattice " + std::to_string(i);
      return TN_ENONFINITE;
    }
  return TN_OK;
}

void batch_destroy(BatchImpl* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->host_res) (void)hipHostFree(b->host_res);
  delete b;
}

int32_t batch_grid(const BatchImpl* b) { return b->grid; }

}  // namespace tn
