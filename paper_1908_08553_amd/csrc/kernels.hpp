// Host-side launchers for the HIP kernels (defined in kernels.hip).
// Every launcher checks nothing itself: the executor validates shapes and
// buffer sizes against the plan before calling.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "device.hpp"

namespace tn {

enum ElemType : int32_t { EL_F32 = 0, EL_F64 = 1 };
enum Arith : int32_t { AR_F64 = 0, AR_F32 = 1, AR_BF16X3 = 2 };

struct StagedArrays {
  double* s64;
  float* s32;
  uint16_t* shi;   // bf16 bits of the high part
  uint16_t* slo;   // bf16 bits of the low part
};

// Where the staging launch writes its bookkeeping.  Block 0 also resets the
// rescale slots to "zero", clears *flags and *counter (each nullable).
struct StageTargets {
  int32_t* site_exp;    // [n_steps] exponent divided out of each staged site
  int32_t* site_bad;    // [n_steps] 1 if the site held a non-finite entry
  int32_t* slot_exp;    // [n_slots] or nullptr
  int32_t n_slots;
  int32_t* flags;       // nullable
  int32_t* counter;     // nullable (work counter of the batched kernel)
  // A cut plan's supplied boundary: slot_exp[seed_slot] = seed_rec->e and
  // *e_bias = seed_rec->bias (seed_rec nullable).
  const EnvRec* seed_rec = nullptr;
  int32_t seed_slot = 0;
  int64_t* e_bias = nullptr;
};

hipError_t launch_stage(const StageDesc* descs, int32_t n_steps, StagedArrays st,
                        StageTargets t, hipStream_t stream);

// out[pre][N][post] = sum_k (2^-shift * in[pre][k][post]) * S[k][n]
struct AbsorbArgs {
  const void* in;
  void* out;
  int32_t in_type, out_type;   // ElemType
  int32_t arith;               // Arith: F64 needs out F64; F32/BF16X3 compute in float
                               // unless out_type is F64 (then double)
  int64_t pre, K, N, post;
  int64_t s_off;               // staged offset of S (K x N)
  const int32_t* scale_slot;   // nullable
  int32_t* max_slot;           // nullable
};

// MFMA absorption (absorb_mfma.hip): K, N <= 16 and post % 16 == 0 or post == 1.
bool absorb_mfma_supported(const AbsorbArgs& a);
hipError_t launch_absorb_mfma(const AbsorbArgs& a, const StagedArrays& st, DevState* state,
                              hipStream_t stream, const char** kname);

// Several independent steps of one kind (same element types, all wide or all
// narrow) in a single launch; n in 2..4.
bool absorb_group_supported(const AbsorbArgs* a, int32_t n);
hipError_t launch_absorb_group(const AbsorbArgs* a, int32_t n, const StagedArrays& st,
                               DevState* state, hipStream_t stream, const char** kname);

// Split BF16x3 ring: T [kd][md] float scaled by 2^-slot -> H, L [md][kp] bf16
// hi/lo parts, kp = split_k_padded(kd) (zero padded); md % 4 == 0.
int64_t split_k_padded(int64_t k);
hipError_t launch_split_transpose(const float* T, int64_t kd, int64_t md, const int32_t* slot,
                                  uint16_t* H, uint16_t* L, hipStream_t stream);
// C = A B^T from split operands (A [m][kp], B [n][kp], kp a multiple of 32);
// split-K slices, caps and the fused dot as RingArgs / launch_ring.
struct NtArgs {
  const uint16_t* Ah;
  const uint16_t* Al;
  const uint16_t* Bh;
  const uint16_t* Bl;
  int64_t m, n, kp;
  float* c_out;
  const float* dot_with;
  int32_t w_slices = 1;
  int32_t c_slices_cap = 1;
  double* partials = nullptr;
  int64_t partials_cap = 0;
};
int32_t ring_bf16x3_nt_splits(int64_t m, int64_t n, int64_t kp);
int64_t ring_bf16x3_nt_partials(int64_t m, int64_t n, int64_t kp);
hipError_t launch_ring_bf16x3_nt(const NtArgs& a, hipStream_t stream, int64_t* n_partials,
                                 int32_t* c_slices);

// Two consecutive D = 4 bulk steps of one column fused into one pass (see
// absorb_pair in absorb_mfma.hip): s1 = (pre, 16, 16, 4*post2), s2 = (4*pre,
// 16, 16, post2), post2 % 64 == 0, same element type in and out.
struct PairArgs {
  const void* in;
  void* out;
  int32_t type;                // ElemType of in and out
  int32_t arith;
  int64_t pre, post2;
  int64_t s_off1, s_off2;
  const int32_t* scale_slot;   // scales s1's input (nullable)
  int32_t* max_slot;           // measured after s2 (nullable)
};
hipError_t launch_absorb_pairs(const PairArgs* a, int32_t n, const StagedArrays& st,
                               DevState* state, hipStream_t stream, const char** kname);

// Two consecutive steps at an edge of a column sweep, fused (absorb_edge.hip):
//   head (first column, suffix 1): s1 = (pre1, 4, 16, 1), s2 = (4 pre1, 4, 4, 1);
//   tail (last column, prefix 1): s1 = (1, 4, 4, 4 post2), s2 = (1, 16, 4, post2)
//   with 4 | post2 (n2 = 4 in both).
// Input of s1 in in_type, output of s2 (and the intermediate) in out_type;
// arithmetic in double when out_type is F64, else float (not BF16x3).
struct EdgeArgs {
  const void* in;
  void* out;
  int32_t in_type, out_type;   // ElemType
  int32_t arith;
  bool head;
  int32_t n2;
  int64_t pre1, post2;
  int64_t s_off1, s_off2;
  const int32_t* scale_slot;   // scales s1's input (nullable)
  int32_t* max_slot;           // measured after s2 (nullable)
};
bool edge_pair_supported(const EdgeArgs& a);
hipError_t launch_absorb_edges(const EdgeArgs* a, int32_t n, const StagedArrays& st,
                               DevState* state, hipStream_t stream, const char** kname);

// Up to kChunkMax consecutive rows of one column (see absorb_chunk.hip): the
// first step has K = 4 or 16, inner steps K = N = 16 with D = 4 legs between
// them, the last N = 4 or 16; the boundary slice stays in LDS for the chunk.
constexpr int kChunkMax = 4;
struct ChunkArgs {
  const void* in;
  void* out;
  int32_t type;                // ElemType of in and out
  int32_t arith;
  int64_t pre, post;           // prefix of the first step, suffix of the last
  int32_t k, k1, nl;           // steps; K of the first; N of the last
  int64_t s_off[kChunkMax];
  const int32_t* scale_slot;   // scales the first step's input (nullable)
  int32_t* max_slot;           // measured after the last step (nullable)
};
int32_t chunk_max_steps(int32_t type);
// 0 = register chunks where the shape allows, else LDS slices; 1 = LDS slices
// only; 2 = register chunks of at most 3 rows (absorb_chunk_reg.hip)
void set_chunk_schedule(int32_t s);
bool chunk_shape_ok(int32_t type, int64_t pre, int64_t post, int32_t k, int32_t k1, int32_t nl);
hipError_t launch_absorb_chunks(const ChunkArgs* a, int32_t n, const StagedArrays& st,
                                DevState* state, hipStream_t stream, const char** kname);
// The register-resident chunk kernel: suffix a multiple of 16 with N = 16 at
// the last step, or suffix 1 with N = 4 (bottom edge) and 16 | prefix.
int32_t chunk_reg_max_steps(int32_t type);
bool chunk_reg_shape_ok(int32_t type, int64_t pre, int64_t post, int32_t k, int32_t k1,
                        int32_t nl);
hipError_t launch_absorb_chunks_reg(const ChunkArgs* a, int32_t n, const StagedArrays& st,
                                    DevState* state, hipStream_t stream, const char** kname);

// Kernel policy: 0 = matrix-core kernels where the shape allows, 1 = vector-ALU
// kernels only (absorption and ring products).
void set_absorb_policy(int32_t policy);
int32_t absorb_policy();
// 2 = column chunks (absorb_chunk), 1 = step pairs (absorb_pair), 0 = one
// launch per step.
void set_fuse_steps(int32_t on);
int32_t fuse_steps();

// *kname receives the name of the kernel variant launched.
hipError_t launch_absorb(const AbsorbArgs& a, const StagedArrays& st, DevState* state,
                         hipStream_t stream, const char** kname);

// Ring: C = 2^-(sa+sb) * A^T B with A [k][m], B [k][n].  If dot_with != nullptr
// the tile results are multiplied elementwise with W = sum of the w_slices
// slices of dot_with (each [m][n], stride m*n) and summed in float64 into
// partials (at most partials_cap); otherwise C is stored to c_out as up to
// c_slices_cap split-K slices [m][n] whose sum is the product.
struct RingArgs {
  const void* A;
  const void* B;
  int32_t type;                // ElemType of A, B, c_out, dot_with
  int32_t arith;
  int64_t m, n, k;
  const int32_t* sa;
  const int32_t* sb;
  void* c_out;
  const void* dot_with;
  double* partials;
  int32_t w_slices = 1;
  int32_t c_slices_cap = 1;
  int64_t partials_cap = 0;
};

// Partials the vector-ALU ring writes (64 x 64 tiles).
int64_t ring_partials(int64_t m, int64_t n);
// *n_partials receives the number of partials this launch writes (fused dot),
// *c_slices the number of slices it stored (stored product).
hipError_t launch_ring(const RingArgs& a, hipStream_t stream, const char** kname,
                       int64_t* n_partials, int32_t* c_slices);

// MFMA ring products (ring_mfma.hip): m % 4 == 0 and n % 4 == 0.  The split
// count and partial count follow from the shape alone (before the caps).
bool ring_mfma_supported(const RingArgs& a);
int32_t ring_mfma_splits(const RingArgs& a);
int64_t ring_mfma_partials_for(const RingArgs& a);
// 1: FP64 ring products scale every staged operand (else automatic)
void set_ring_operand_scale(int32_t on);
void set_chunk_stream(int32_t v);
hipError_t launch_ring_mfma(const RingArgs& a, hipStream_t stream, const char** kname,
                            int64_t* n_partials, int32_t* c_slices);

// A run of consecutive small single steps of one sweep unit in one workgroup
// (batch.hip): step j reads buf[cur ^ (j & 1)] and writes the other buffer,
// with the same per-step arithmetic as one launch per step.  Slots are
// indices into slot_exp (-1: none); a step with rescale_slot writes that
// slot's exponent (it starts at the "zero" sentinel and has no other writer).
constexpr int kChainMax = 14;
struct ChainStep {
  int64_t pre, post, s_off;
  int32_t K, N;
  int32_t in_f64, out_f64;
  int32_t rescale_slot, scale_slot;
};
struct ChainUnit {
  void* buf[2];
  const void* in0;      // input of the first step instead of buf[cur] (nullable)
  int32_t cur, n;
  ChainStep s[kChainMax];
};
hipError_t launch_chain(const ChainUnit* units, int32_t n, const StagedArrays& st,
                        int32_t* slot_exp, int32_t* flags, int32_t arith, hipStream_t stream,
                        const char** kname);

// Double-layer site of a real PEPS tensor (peps.hip): A [d][dims...] and
// E [dims_0^2]..[dims_{rank-1}^2] on the device, op [d][d] or null
// (identity); n_in = prod dims, n_out = n_in^2.
struct DoubleLayerSite {
  const double* A;
  const double* op;
  double* E;
  int64_t n_in, n_out;
  int32_t d, rank;
  int32_t dims[4];
  int32_t perm[4];   // E's bond leg k is A's bond leg perm[k] (a permutation)
};
bool double_layer_ok(const DoubleLayerSite& s);
hipError_t launch_double_layer(const DoubleLayerSite* sites, int32_t n, hipStream_t stream);

// One link of the row scheme's chain (row_chain.hip): out = v R (side 0, R as
// [K][N]) or R v (side 1, R as [N][K]), float64, v and R scaled by 2^-e of
// their slots on load; the exponent of max |out| goes to max_slot (null on
// the last link).  `partials` holds link_chunks(side, K, N) * N doubles.
struct LinkArgs {
  const void* v = nullptr;
  const void* R = nullptr;
  int32_t v_f64 = 1, R_f64 = 1;
  int64_t K = 1, N = 1;
  int32_t side = 0;
  const int32_t* slot_v = nullptr;
  const int32_t* slot_R = nullptr;
  double* out = nullptr;
  int32_t* max_slot = nullptr;
  int32_t* flags = nullptr;
  double* partials = nullptr;
};
int64_t link_chunks(int32_t side, int64_t K, int64_t N);
hipError_t launch_row_link(const LinkArgs& a, hipStream_t stream);

// Imaginary-time evolution kernels (ite.hip).  Site k of the state is
// A[2][chi^rank] at `off` entries into the state buffer (half = chi^rank).
constexpr int32_t kIteMaxChi = 3;
constexpr int32_t kIteMaxDim = 64;
struct IteSiteDesc {
  int64_t off, half;
};
// A pair gate's sites: offsets, bond-leg counts and the index of the shared
// bond among each site's bond legs (canonical order).
struct ItePairDesc {
  int64_t off_i, off_j;
  int32_t ri, rj, ai, aj;
};
struct IteGate2 {
  double g[16];    // G[(s_i s_j)][(a c)], row-major
};
hipError_t launch_ite_gate1(double* state, const IteSiteDesc* sites, int32_t n_sites,
                            int64_t max_half, const double g[4], hipStream_t stream);
hipError_t launch_ite_scale(double* state, int64_t n, double f, hipStream_t stream);
hipError_t launch_ite_pairs(double* state, const ItePairDesc* pairs, int32_t n_pairs,
                            const IteGate2& gate, int32_t chi, double eps, int32_t* kept,
                            hipStream_t stream);

// Writes state->result from the final scalar (or the sum of `n_partials`
// partials), the site exponents, the rescale slots and state->e_bias, plus
// the exponent of `cap` (the boundary a cap dot closed against; nullable);
// with `copy` the record is also written there.
hipError_t launch_finalize(DevState* state, const double* scalar, tn_result* copy,
                           const double* partials, int64_t n_partials, hipStream_t stream,
                           const EnvRec* cap = nullptr);

// Cut plans (cached environments).  Cap: partial sums of
// sum_i (B[i] 2^-eb)(Rv[i] 2^-er) with eb = *slot_b and er = rec->e, one per
// block of env_cap_blocks(n) blocks; launch_finalize(..., cap = rec) sums
// them in a fixed order.
int64_t env_cap_blocks(int64_t n);
hipError_t launch_env_cap(const void* B, const void* Rv, int64_t n, int32_t f64,
                          const int32_t* slot_b, const EnvRec* rec, double* partials,
                          hipStream_t stream);
// Site environment (cached environments): with L the boundary before sweep
// step k, as [P][X][Q] (X: the legs step k contracts), and Rv the boundary of
// all sites after step k, as [P][Y][Q] (Y: the legs step k writes), both in the
// sweep's leg order, Env[x][y] = sum_{p,q} (L 2^-el)(Rv 2^-er) is the network
// with site k removed.  A null L or Rv is the scalar 1 (nothing before the
// first or after the last step).  launch_site_env writes `blocks` partial
// matrices (fixed split of the P*Q range); launch_site_dots sums them in a
// fixed order and dots Env with each listed site tensor, folded to [X][Y] by
// the step's axis order, writing sign, exponent and log|Z| per site.
constexpr int32_t kSiteEnvMaxXY = 6561;   // X * Y up to 81 * 81
constexpr int32_t kSiteDotsMax = 8;
struct SiteEnvArgs {
  const void* L;
  const void* Rv;
  int32_t l_f64, r_f64;
  int64_t P, Q;
  int32_t X, Y;
  const EnvRec* l_rec;   // nullable: exponent 0
  const EnvRec* r_rec;
  double* partials;      // [blocks][X * Y]
  int32_t blocks;
};
struct SiteDot {
  const double* site;    // canonical float64 site tensor (device)
  int64_t cstride[4];    // canonical stride of each folded axis
  int32_t dims[4];       // folded-order dims (X legs, then Y legs)
  int32_t ndim;
  tn_result* out;        // device
};
int32_t site_env_blocks(int64_t P, int64_t Q, int32_t X, int32_t Y);
hipError_t launch_site_env(const SiteEnvArgs& a, hipStream_t stream);
hipError_t launch_site_dots(const SiteEnvArgs& a, const SiteDot* dots, int32_t n,
                            hipStream_t stream);

// Tap: the record of the boundary a cut plan ends in, whose largest-magnitude
// exponent is *slot_last (null inside a column: no shift), from the exponent
// sums of finalize (one block).
hipError_t launch_env_tap(DevState* state, const int32_t* slot_last, EnvRec* rec,
                          hipStream_t stream);

}  // namespace tn
