// Executor: turns a plan plus device pointers into kernel launches.
#pragma once

#include <hip/hip_runtime_api.h>

#include <array>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "device.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace tn {

// Byte offsets of every region of the caller's workspace for one
// (plan, precision) pair.  All offsets are 256-byte aligned.
struct Layout {
  size_t state = 0, state_bytes = 0;
  size_t descs = 0;
  size_t raw = 0;                    // host sites are copied here
  size_t s64 = 0, s32 = 0, shi = 0, slo = 0;
  std::vector<std::array<size_t, 2>> buf;   // unit boundary ping-pong buffers
  std::vector<size_t> buf_bytes;
  size_t vbuf[2] = {};               // row chain: float64 chain vectors
  size_t vbuf_bytes = 0;
  size_t link_partials = 0;          // row chain: per-link partial sums
  int64_t n_link_partials = 0;
  size_t yt = 0, yt_bytes = 0;       // ring: the stored product X (split-K slices)
  int32_t yt_slices = 1;
  size_t partials = 0;
  int64_t n_partials = 0;
  bool split_ring = false;           // BF16x3 ring from pre-split operands
  size_t split[4][2] = {};           // unit tensor -> (hi, lo) [rows][kp] bf16
  size_t total = 0;
  std::vector<int64_t> s_off;        // staged offset of each step
  std::vector<int32_t> out_type;     // ElemType of each step's output
};

Layout make_layout(const Plan& p, int32_t prec);

// Algorithmic HBM bytes of one contraction (boundary in + out per step, sites,
// ring operands) for the element sizes `prec` uses.
int64_t algorithmic_bytes(const Plan& p, int32_t prec);

// Launch timing for roofline accounting (see tn_profile_enable in tn.h).
void profile_enable(bool on);
int32_t profile_read(tn_kernel_stat* out, int32_t cap);
bool profile_on();

// Records HIP events around launches on one stream and folds the elapsed
// times into the process-wide totals once the stream has been synchronised.
class LaunchTimer {
 public:
  explicit LaunchTimer(hipStream_t s, bool allow = true);
  ~LaunchTimer();
  void before();
  void after(const char* name, double bytes, double flops);
  void flush();   // call after the stream is synchronised
 private:
  struct Rec { hipEvent_t a, b; const char* name; double bytes, flops; };
  hipStream_t stream_;
  bool on_;
  std::vector<Rec> recs_;
  hipEvent_t pending_ = nullptr;
};

// Staging descriptors for every step of p: site pointers from dsite (indexed by
// lattice site), staged offsets s_base + L.s_off[k], INIT steps written to
// init_dst[unit] in the element type of that step.
void fill_stage_descs(const Plan& p, const Layout& L, int64_t s_base,
                      const double* const* dsite, char* const* init_dst, StageDesc* descs);

// Pinned host image of the workspace head (DevState, exponent slots, stage
// descriptors) that an enqueue uploads in one asynchronous copy, plus room
// for the result record copied back.  Grown with hipHostMalloc and reused;
// the stream work that reads it must finish before the next enqueue through
// the same HostKeep (one per calling thread, one per server slot).
class HostKeep {
 public:
  HostKeep() = default;
  ~HostKeep();
  HostKeep(const HostKeep&) = delete;
  HostKeep& operator=(const HostKeep&) = delete;
  // At least `bytes` of pinned memory (contents unspecified), or nullptr with
  // *e set when the allocation fails.  After adopt(), never allocates: the
  // adopted buffer or nullptr (*e = hipErrorOutOfMemory) when it is too small.
  char* block(size_t bytes, hipError_t* e);
  char* data() const { return p_; }
  // Use `cap` bytes of caller-owned host memory (pageable; not freed here)
  // instead of pinned blocks.
  void adopt(char* p, size_t cap) { p_ = p; cap_ = cap; fixed_ = true; }
 private:
  char* p_ = nullptr;
  size_t cap_ = 0;
  bool fixed_ = false;
};

// Bytes of the uploaded head image and offset of the result record in it.
size_t head_bytes(const Plan& p, const Layout& L);

// A second stream and two events: the bottom quadrant units of a quadrant
// plan are swept on `stream` concurrently with the top units and the first
// ring product (fork after staging, join before the second ring product).
struct SideStream {
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

// 1: tn_contract_grid sweeps the bottom quadrant units on a second stream of
// the calling thread (see SideStream); 0 (default): one stream.
void set_quadrant_streams(int32_t on);
// Runs of small consecutive single steps of a unit as one chain launch
// (default on; only with the default step fusion).
void set_chain_steps(int32_t on);
extern int32_t g_chain_steps;
constexpr int64_t kChainEntries = 16384;   // largest step input / output of a chain
extern int32_t g_quadrant_streams;

// Ends of a cut plan (Plan::is_cut): the boundary its SEED step starts from,
// and either the boundary its last column is closed against (cap: the
// mirrored sweep's boundary at the same column cut, same leg order) or the
// record of the boundary it ends in (tap).  All pointers are device memory
// except `tap`, which receives the address of the ending boundary (inside
// the plan's workspace).  `partials` holds env_cap_blocks(entries) doubles.
// With `result` the result record is also written there.
struct CutIO {
  const void* seed = nullptr;
  const EnvRec* seed_rec = nullptr;
  const void* cap = nullptr;
  const EnvRec* cap_rec = nullptr;
  EnvRec* tap_rec = nullptr;
  const void** tap = nullptr;
  double* partials = nullptr;
  tn_result* result = nullptr;
};

// Issue every copy and launch of one contraction on `stream` without waiting;
// the result record lands in the workspace's DevState (offset Layout.state).
// With `side` (and `side_timer` for its launches) quadrant plans also use
// side->stream; all work is joined back into `stream` before it ends.
tn_status enqueue(const Plan& p, const double* const* sites, bool on_device, int32_t prec,
                  void* ws, size_t ws_bytes, hipStream_t stream, HostKeep& keep,
                  LaunchTimer& timer, std::string& err, const SideStream* side = nullptr,
                  LaunchTimer* side_timer = nullptr, const CutIO* io = nullptr);

tn_status contract(const Plan& p, const double* const* sites, bool on_device, int32_t prec,
                   void* ws, size_t ws_bytes, hipStream_t stream, tn_result* out,
                   std::string& err);

// As contract(), with the head image and result record in `keep` and on
// `stream` alone (no side stream); with timed = false no profiling events
// are created.  Creates no stream, event, pinned block or device memory when
// `keep` was adopted and timed is false.
tn_status contract_with(const Plan& p, const double* const* sites, bool on_device, int32_t prec,
                        void* ws, size_t ws_bytes, hipStream_t stream, HostKeep& keep,
                        bool timed, tn_result* out, std::string& err);

// The allocation-free workspace (defined beside its device array): the
// current device's copy of the library's static scratch array and its size.
// Looked up once per device; TN_EDEVICE when the lookup fails.
tn_status static_scratch(void** ptr, size_t* bytes, std::string& err);

}  // namespace tn
