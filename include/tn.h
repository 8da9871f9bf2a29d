/*
 * tn.h -- C ABI of the MI355X exact planar-lattice contraction library.
 *
 * The problem (paper §4): an Lh x Lw planar square lattice of tensors with no
 * external indices -- corner tensors of order 2, edge tensors of order 3,
 * bulk tensors of order 4 -- is summed over all internal indices to one
 * scalar by a sequence of pairwise contractions.  The order of contraction
 * changes memory and cost, not the result (§4, "the order of the
 * contraction matters"; the method is exact).
 *
 * Conventions used by every call:
 *   - Sites are listed row-major, site (0,0) at the top-left.
 *   - Bond h(r,c) joins (r,c)-(r,c+1); bond v(r,c) joins (r,c)-(r+1,c).
 *   - A site tensor's legs are ordered (left, up, right, down) with absent
 *     legs omitted; entries are float64, C-order (last leg fastest).
 *   - Results are exact up to rounding: Z = mantissa * 2^exp2_sum with
 *     |mantissa| in [0.5, 1), sign in {-1, 0, +1}, log_abs = ln|Z|.
 *
 * Every call returns a tn_status; no C++ exception, abort or exit crosses
 * the ABI.  tn_last_error() returns a message for the calling thread's last
 * failure.  Device memory is always supplied by the caller (pointer +
 * bytes); the library allocates none on the contraction path.  Streams are
 * the caller's hipStream_t passed as void*.
 */
#ifndef TN_H_
#define TN_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tn_status;
#define TN_OK          0
#define TN_PENDING     1    /* tn_poll: the request has not finished yet          */
#define TN_EINVAL     -1    /* bad shape, dimension, pointer or enum               */
#define TN_ENOMEM     -2    /* workspace / arena / text buffer too small           */
#define TN_EBUSY      -3    /* server queue full                                   */
#define TN_EDEVICE    -4    /* a HIP runtime call failed                           */
#define TN_ENOTFOUND  -5    /* unknown or already retired ticket                   */
#define TN_ENONFINITE -6    /* NaN/Inf in the inputs or in an intermediate          */
#define TN_EOVERFLOW  -7    /* a plan integer (size, flops) exceeds int64          */

/* Contraction orders (paper §4 and Fig. 2).
 *   COLSWEEP : one boundary tensor absorbs the lattice column by column, top to
 *              bottom -- the sequential form of the paper's row contraction
 *              (boundary of chi^L entries between columns).
 *   QUADRANT : the four quadrants are swept from their outer corners towards the
 *              middle; the ring of four tensors is then closed by two matrix
 *              products and an elementwise dot.
 *   HEURISTIC: the candidate (sweep, transposed sweep, every quadrant split)
 *              with the smallest bottleneck tensor; ties broken by total flops,
 *              then by enumeration order (§4, last paragraph).
 *   SWEEP_AUTO: the column sweep in the orientation with the smaller bottleneck
 *              (boundary along the shorter side); ties: fewer flops, then
 *              untransposed.  Planned order is COLSWEEP.                      */
#define TN_ORDER_COLSWEEP   0
#define TN_ORDER_QUADRANT   1
#define TN_ORDER_HEURISTIC  2
#define TN_ORDER_SWEEP_AUTO 3
/*   ROWS     : the paper's row scheme (§4, Fig. 2a): every row is contracted
 *              left to right into one tensor with all its vertical legs open
 *              (chi^(2L) entries in the bulk), and the resulting chain of row
 *              tensors is contracted from the top row down by matrix-vector
 *              products, in float64 (the chain is the final reduction).
 *   ROWS_T   : the same over columns (planned order ROWS, transpose = 1).
 *   HEURISTIC also enumerates ROWS and ROWS_T, after the quadrant splits.   */
#define TN_ORDER_ROWS       4
#define TN_ORDER_ROWS_T     5

/* Arithmetic of the contraction.
 *   F64    : every step in float64.
 *   F32    : boundary and sites in float32, float32 products and sums; the
 *            last column of a sweep and the ring's final dot in float64.
 *   BF16X3 : float32 storage; every product formed from bf16 hi/lo splits of
 *            both operands as hi*hi + hi*lo + lo*hi on MFMA with float32
 *            accumulation; last column and final dot in float64.
 * Rescaling is exact in all three: after every column the boundary is scaled
 * by 2^-e, e = exponent of its largest magnitude, and e is summed in int64. */
#define TN_PREC_F64    0
#define TN_PREC_F32    1
#define TN_PREC_BF16X3 2

typedef struct {
  int32_t rows;            /* Lh >= 1                                            */
  int32_t cols;            /* Lw >= 1                                            */
  int32_t D;               /* uniform bond dimension (>= 1), used when hdim/vdim */
                           /* are NULL                                           */
  const int32_t* hdim;     /* NULL or rows*(cols-1) dims of h(r,c), row-major    */
  const int32_t* vdim;     /* NULL or (rows-1)*cols dims of v(r,c), row-major    */
} tn_grid;

typedef struct {
  int32_t sign;            /* -1, 0 or +1                                        */
  int32_t status;          /* TN_OK or TN_ENONFINITE                             */
  double  log_abs;         /* ln|Z|; -inf when Z == 0                            */
  double  value;           /* Z as a double (may be +-inf when |Z| > DBL_MAX)    */
  double  mantissa;        /* Z = mantissa * 2^exp2_sum, |mantissa| in [0.5,1)   */
  int64_t exp2_sum;
} tn_result;

typedef struct {
  int32_t order;           /* order actually planned (COLSWEEP or QUADRANT)      */
  int32_t transpose;       /* COLSWEEP: 1 if the sweep runs along rows           */
  int32_t quad_h, quad_w;  /* QUADRANT split (rows [0,h), cols [0,w))            */
  int32_t n_steps;         /* INIT + ABSORB steps over all units                 */
  int32_t n_units;         /* 1 (sweep) or 4 (quadrant)                          */
  int32_t n_slots;         /* rescale points                                     */
  int32_t n_links;         /* ROWS: links of the row chain (0 otherwise)         */
  int64_t peak_entries;    /* bottleneck: largest intermediate, in entries       */
  int64_t flops;           /* algorithmic: sum of 2 * d(out) * d(shared)         */
  int64_t moved_entries;   /* algorithmic boundary traffic: sum of d(in)+d(out)  */
  int64_t workspace_bytes[3]; /* per precision (TN_PREC_*): bytes tn_contract_grid needs */
  int64_t hbm_bytes[3];       /* per precision: algorithmic HBM bytes of one contraction */
  int32_t ring_slices[3];     /* per precision: split-K slices the workspace holds for the
                                 stored ring product (1 = unsplit, 0 = no ring)          */
  int32_t reserved2;
  int64_t buffer_entries;  /* intermediate storage kept at once: two buffers of   */
                           /* each unit's largest intermediate, plus the stored   */
                           /* ring product or two row-chain vectors (entries)     */
} tn_plan_info;

typedef struct tn_plan tn_plan;
typedef struct tn_server tn_server;

/* Message describing the calling thread's last error ("" if none).  The
 * pointer stays valid until the thread's next library call.                */
const char* tn_last_error(void);

/* Plan the contraction of `grid` in `order` (TN_ORDER_*).  quad_h / quad_w
 * select the QUADRANT split (0 = ceil(rows/2) / ceil(cols/2)); ignored for the
 * other orders.  Host only, integer only, deterministic.  The plan is
 * immutable and may be shared between threads; free it with tn_plan_free.
 * Errors: TN_EINVAL (rows/cols/D < 1, a dim < 1, QUADRANT on a lattice with
 * fewer than 2 rows or columns, split out of range), TN_EOVERFLOW.         */
tn_status tn_plan_grid(const tn_grid* grid, int32_t order, int32_t quad_h,
                       int32_t quad_w, tn_plan** out);

/* As tn_plan_grid, with a memory-feasibility check (§4: the order decides
 * the intermediate sizes and with them whether the contraction fits; §6:
 * the row scheme runs out of memory first).  max_buffer_entries bounds the
 * plan's buffer_entries (<= 0: no bound).  An explicit order whose plan
 * exceeds it returns TN_ENOMEM; HEURISTIC and SWEEP_AUTO drop the candidates
 * that exceed it and return TN_ENOMEM only when none is left.             */
tn_status tn_plan_grid_budget(const tn_grid* grid, int32_t order, int32_t quad_h,
                              int32_t quad_w, int64_t max_buffer_entries, tn_plan** out);

/* Sizes and costs of a plan (§4: element counts of every pairwise step and
 * the bottleneck).                                                          */
tn_status tn_plan_stats(const tn_plan* plan, tn_plan_info* out);

/* Canonical text of a plan, used for bit-exact comparison.  On entry *len is
 * the capacity of buf; on return it is the size needed including the NUL.
 * Returns TN_ENOMEM (nothing written) if the capacity is too small.          */
tn_status tn_plan_text(const tn_plan* plan, char* buf, size_t* len);

void tn_plan_free(tn_plan* plan);

/* Contract one lattice to its scalar on the GPU (paper §4: the sum over all
 * internal indices, by pairwise contractions along `plan`).
 *   sites           : rows*cols pointers (a host array) to the float64 site
 *                     tensors in canonical leg order; each points to device
 *                     memory if sites_on_device != 0, else to host memory
 *                     (copied in on `stream`).  Borrowed for the call only.
 *   precision       : TN_PREC_*.
 *   workspace       : device memory of at least tn_plan_info.workspace_bytes
 *                     [precision] bytes, 256-byte aligned, owned by the caller;
 *                     its contents on entry are ignored.
 *   hip_stream      : hipStream_t (NULL = the null stream).
 * Blocks until *out is written.  Errors: TN_EINVAL, TN_ENOMEM (workspace
 * too small), TN_EDEVICE, TN_ENONFINITE (also stored in out->status).      */
tn_status tn_contract_grid(const tn_plan* plan, const double* const* sites,
                           int32_t sites_on_device, int32_t precision,
                           void* workspace, size_t ws_bytes, void* hip_stream,
                           tn_result* out);

/* Allocation-free form of tn_contract_grid, for callers that cannot allocate
 * memory: code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, arithmetic and kernels as
 * tn_contract_grid, except the workspace: the call contracts in the
 * library's own static device array of TN_STATIC_SCRATCH_BYTES bytes, one
 * copy per GPU (held from the first call on that device until the process
 * ends), and builds the workspace head in a fixed host buffer of 1 MiB.  It
 * calls no hipMalloc, hipHostMalloc, hipFree or other allocating routine,
 * creates no stream or event, and runs every launch on hip_stream (the
 * quadrant side-stream option and profiling do not apply).  The array keeps
 * the last call's contents; nothing in it needs to start at zero, since each
 * call uploads its own counters and slots.  Calls are serialised within the
 * process (a lock held until the result is written); calls from different
 * processes use different copies.  Blocks until *out is written.
 * Errors: as tn_contract_grid, and TN_ENOMEM when the plan's workspace_bytes
 * [precision] exceed TN_STATIC_SCRATCH_BYTES or its workspace head exceeds
 * the host buffer (plans with more than about 8000 steps).                */
#define TN_STATIC_SCRATCH_BYTES (160ull << 20)
tn_status tn_contract_grid_static(const tn_plan* plan, const double* const* sites,
                                  int32_t sites_on_device, int32_t precision, void* hip_stream,
                                  tn_result* out);

/* ------------------------------------------------------------ batching
 * Many independent lattices contracted by one replayed launch graph (the
 * paper's observable evaluations need one full contraction per local
 * quantity, §5).  Every plan must be a column-sweep plan (TN_ORDER_COLSWEEP,
 * transposed or not).  The batch copies the plans; the caller may free them
 * after create.
 *
 * The graph stages every site, then runs two paths side by side: the `split`
 * costliest lattices advance in lock-step, one launch per sweep step, each
 * step spread over as many workgroups as its size calls for; every other
 * lattice is swept by one workgroup with all its waves, costliest first (one
 * launch).  Both paths compute every output block with the same per-wave
 * arithmetic, so results are bitwise independent of `threads` and `split`.
 * Staging and both paths are captured once into a hipGraph at create time and
 * replayed by every tn_batch_run.                                          */
typedef struct tn_batch tn_batch;

typedef struct {
  int32_t threads;         /* workgroup size of the one-workgroup path: 256,   */
                           /* 512 or 1024 (0 = default)                        */
  int32_t split;           /* costliest lattices run in lock-step, 0..n        */
} tn_batch_config;

/* Workspace bytes a batch of these plans needs in `precision`.              */
tn_status tn_batch_workspace(const tn_plan* const* plans, int32_t n, int32_t precision,
                             size_t* bytes);

/* Build device tables in `workspace` (>= tn_batch_workspace bytes, 256-byte
 * aligned, owned by the caller and reserved for this batch until destroy)
 * and capture the launch graph.  cfg may be NULL (defaults).  Uses the
 * current HIP device.  Errors: TN_EINVAL (non-sweep plan, bad config),
 * TN_ENOMEM (workspace), TN_EDEVICE.                                        */
tn_status tn_batch_create(const tn_plan* const* plans, int32_t n, int32_t precision,
                          const tn_batch_config* cfg, void* workspace, size_t ws_bytes,
                          tn_batch** out);

/* Contract every lattice: sites[i] is an array of rows*cols DEVICE pointers
 * to lattice i's float64 sites (canonical legs), borrowed for the call.
 * Writes outs[0..n-1]; blocks until done.  Returns TN_ENONFINITE if any
 * lattice hit a non-finite value (its outs[i].status says so; the others are
 * valid).                                                                  */
tn_status tn_batch_run(tn_batch* batch, const double* const* const* sites, void* hip_stream,
                       tn_result* outs);

tn_status tn_batch_destroy(tn_batch* batch);

/* One-shot form: create with the process-wide default configuration
 * (TN_OPT_BATCH_THREADS), run once, destroy.                               */
tn_status tn_contract_batch(const tn_plan* const* plans, const double* const* const* sites,
                            int32_t n, int32_t precision, void* workspace, size_t ws_bytes,
                            void* hip_stream, tn_result* outs);

/* ------------------------------------------------------------ PEPS observables
 * Paper §3: a state's amplitudes A({s}) are a planar network of rank-5 site
 * tensors (four bonds and the spin index; edges and corners have fewer
 * bonds); its norm is the sum over all spin configurations of A* A, and
 * m^x_k = <S^x_k>, m^z_k = <S^z_k>, c_ij = <S^z_i S^z_j> - <S^z_i><S^z_j>,
 * each <O> = <Psi|O|Psi> / <Psi|Psi>.  §5: each of these is one contraction
 * of O|Psi> against <Psi| along every spin index, L^2 (m^x) and 2L(L-1)
 * (c_ij, nearest neighbours) networks on an L x L lattice.  Tensors are real.
 *
 * tn_double_layer builds, for each site j, the single-layer tensor of that
 * contraction:
 *   E[(a_1 a_1')..(a_r a_r')] = sum_{s,s'} A[s][a_1..a_r] O[s'][s] A[s'][a_1'..a_r']
 * with the paired bond index a_k * dims[k] + a_k' (ket-major), so a lattice
 * of such sites is a planar network with bond dimensions dims^2 that
 * tn_contract_grid / the batch calls contract.  All pointers are device
 * memory the caller owns; the work is enqueued on hip_stream (asynchronous:
 * synchronise the stream before reading E).  Errors: TN_EINVAL (NULL A or E,
 * d outside 1..64, rank outside 0..4, a dimension < 1, more than 2^30
 * entries in A), TN_EDEVICE.                                                */
typedef struct {
  const double* A;   /* [d][dims[0]]..[dims[rank-1]], C-order                  */
  const double* op;  /* [d][d] operator O[s'][s], or NULL for the identity     */
  double* E;         /* [dims[perm[0]]^2]..[dims[perm[rank-1]]^2], C-order      */
  int32_t d;         /* spin dimension                                         */
  int32_t rank;      /* bond legs in canonical order (left, up, right, down)   */
  int32_t dims[4];   /* bond dimensions of A, the first `rank` are used        */
  int32_t perm[4];   /* E's bond leg k is A's bond leg perm[k] (the first     */
                     /* `rank` entries, a permutation); all zero: E's legs in */
                     /* A's order.  Used to lay a site out for the transposed */
                     /* lattice (left <-> up, right <-> down).                */
} tn_double_layer_site;

tn_status tn_double_layer(const tn_double_layer_site* sites, int32_t n, void* hip_stream);

/* Observables of a rows x cols state from the results of its networks, in
 * this order: the norm (no operator), S^x at each site (row-major), S^z at
 * each site, S^z S^z on each nearest-neighbour pair (horizontal pairs row by
 * row, then vertical pairs row by row): 1 + 2 rows cols + rows (cols - 1) +
 * (rows - 1) cols results.  Writes mx[rows cols], mz[rows cols] and
 * czz[pairs] (host arrays) from exact ratios of the results' mantissas and
 * exponents.  Errors: TN_EINVAL (NULL, rows or cols < 1, zero norm),
 * TN_ENONFINITE (a result with a non-finite status).                        */
tn_status tn_observables(const tn_result* results, int32_t rows, int32_t cols, double* mx,
                         double* mz, double* czz);

/* ------------------------------------------------------------ cached environments
 * Families of networks that equal one base network except at a few sites
 * (§5: the observable networks equal the norm network except where the
 * operator acts), contracted with the column sweep of §4 and its boundaries
 * kept: the boundary after columns 0..c-1 of the base network (left
 * environment) and the one after columns cols-1..c (right environment, the
 * same sweep run from the right edge) are computed once per run.  A network
 * whose substituted sites lie in columns [c0, c1) then costs the absorption
 * of those columns, started from the left environment at c0, and one dot
 * with the right environment at c1 (none when c1 = cols: that network is the
 * full sweep's own arithmetic), instead of a full contraction; with the
 * environments inside columns (TN_OPT_ENV_ROWS) only the sweep steps from
 * its first to its last substituted site are absorbed.  Every value
 * is the exact contraction of its network up to rounding, with the exact
 * power-of-two rescaling of the sweep.
 *
 * Network k substitutes subst_site[o_k .. o_k + n_subst[k]) (row-major site
 * indices r * cols + c, distinct within a network; o_k = n_subst[0] + ... +
 * n_subst[k-1]); n_subst[k] = 0 is the base network itself.  The set copies
 * the grid and the lists.  Precision as tn_contract_grid (the last column of
 * every sweep and every environment dot accumulate in float64).             */
typedef struct tn_envset tn_envset;

/* Workspace bytes for this family in `precision`: the 2 (cols - 1) column
 * environments, one region the networks take in turn, and small tables.
 * Errors: TN_EINVAL (bad grid, counts, a site index outside the lattice or
 * repeated in one network), TN_EOVERFLOW.                                   */
tn_status tn_envset_workspace(const tn_grid* grid, int32_t precision, int32_t n,
                              const int32_t* n_subst, const int32_t* subst_site, size_t* bytes);

/* Build the plans; `workspace` (>= tn_envset_workspace bytes, 256-byte
 * aligned, device memory owned by the caller) is reserved for this set until
 * destroy.  Errors: as tn_envset_workspace, TN_ENOMEM (workspace too small). */
tn_status tn_envset_create(const tn_grid* grid, int32_t precision, int32_t n,
                           const int32_t* n_subst, const int32_t* subst_site, void* workspace,
                           size_t ws_bytes, tn_envset** out);

/* Contract the base network and every network of the set.  base: rows*cols
 * DEVICE pointers to the base sites (float64, canonical legs); subst: one
 * DEVICE pointer per entry of subst_site, the replacing site (same shape as
 * the site it replaces).  All borrowed for the call.  outs[0] is the base
 * network, outs[1 + k] network k.  Issued on hip_stream and on the set's own
 * streams (TN_OPT_ENV_STREAMS), which are joined back into hip_stream;
 * blocks until the results are copied back.  One run at a time per set (a
 * run reuses the set's host tables and workspace regions).  Errors:
 * TN_EINVAL (NULL pointer), TN_EDEVICE, TN_ENONFINITE (a network met a
 * non-finite value: its outs[] status says so, the other results are
 * valid).                                                                   */
tn_status tn_envset_run(tn_envset* set, const double* const* base, const double* const* subst,
                        void* hip_stream, tn_result* outs);

tn_status tn_envset_destroy(tn_envset* set);

/* ------------------------------------------------------------ imaginary time
 * Ground state of the transverse-field Ising model (§3)
 *   H = -J sum_<ij> S^z_i S^z_j - gamma sum_i S^x_i,  S = Pauli matrices
 * (S^z takes the values +1 and -1; the critical point lies near gamma = 3J)
 * by imaginary-time evolution of a PEPS (§5): from the uniform superposition
 * of product states (bond dimension 1), each step applies the second-order
 * Trotter-Suzuki product U^gamma(dtau/2) U^J(dtau) U^gamma(dtau/2):
 *   - the one-body gate exp(gamma t sigma^x) contracted into every site's
 *     spin index;
 *   - the two-body gate exp(J dtau s_i s_j) on every nearest-neighbour pair:
 *     the two sites contracted over their shared bond and the gate over their
 *     spins, the result folded into a matrix (each site's open indices) and
 *     split by a singular value decomposition (one-sided Jacobi on the GPU)
 *     into U sqrt(lambda) and sqrt(lambda) V^T, keeping the singular values
 *     at or above eps times the largest, at most chi_max of them (the rest of
 *     every bond, up to chi_max, holds zeros).  Pairs go in four classes of
 *     disjoint bonds: horizontal bonds with the left site in an even column,
 *     in an odd column, vertical bonds with the upper site in an even row, in
 *     an odd row;
 *   - the state normalised to <Psi|Psi> = 1 after each of the three operator
 *     sets (the norm network contracted in float64 by this library, every
 *     site scaled by the same factor).
 * The energy <H> and the local m^x, m^z, c_ij come from the expectation-value
 * networks of §5, contracted in one batched launch.  Each pair's singular
 * pair is signed so that the first entry of the left vector above 1e-6 of
 * its largest magnitude is positive.  All device memory is the caller's
 * workspace; every call runs on the stream given at create and blocks until
 * its work is done.                                                         */
typedef struct tn_ite tn_ite;

typedef struct {
  int32_t rows, cols;      /* lattice (>= 1 each, at most 4096 sites)           */
  int32_t chi_max;         /* largest bond dimension kept, 1..3                */
  int32_t reserved;        /* must be 0                                        */
  double  J, gamma;        /* couplings of H                                   */
  double  eps;             /* relative singular-value cutoff (>= 0; the paper's */
                           /* timing runs use 0.01)                            */
} tn_ite_config;

/* Workspace bytes (device memory) an evolution of this configuration needs.
 * Errors: TN_EINVAL (bad configuration), TN_EOVERFLOW.                      */
tn_status tn_ite_workspace(const tn_ite_config* cfg, size_t* bytes);

/* Set up the evolution in `workspace` (>= tn_ite_workspace bytes, 256-byte
 * aligned, owned by the caller, reserved until destroy) on hip_stream, with
 * the state set to the uniform product state.  Uses the current device.     */
tn_status tn_ite_create(const tn_ite_config* cfg, void* workspace, size_t ws_bytes,
                        void* hip_stream, tn_ite** out);

/* n_steps Trotter steps of imaginary time dtau each (dtau > 0).  Errors:
 * TN_EINVAL, TN_EDEVICE, TN_ENONFINITE (the norm became zero or non-finite). */
tn_status tn_ite_step(tn_ite* ite, double dtau, int32_t n_steps);

/* <H> / <Psi|Psi> of the current state, with m^x and m^z per site (row-major,
 * rows*cols each) and c_ij per nearest-neighbour bond (horizontal bonds row
 * by row, then vertical), the same layout as tn_observables.  Host arrays. */
tn_status tn_ite_energy(tn_ite* ite, double* energy, double* mx, double* mz, double* czz);

/* Device pointers to the current site tensors, rows*cols of them, row-major:
 * site k is A[2][chi_max]...[chi_max] (spin index first, then its bond legs
 * in canonical order), float64, C-order.  They stay valid until destroy; a
 * caller may write a state into them between calls.                       */
tn_status tn_ite_sites(tn_ite* ite, double** sites);

tn_status tn_ite_destroy(tn_ite* ite);

/* ------------------------------------------------------------ serving
 * A request loop that admits contractions of different sizes and precisions
 * as they arrive.  A scheduler thread admits queued requests first-come-
 * first-served as soon as a slot (a HIP stream of the server's own) and a
 * contiguous region of the arena large enough for the request's whole
 * workspace are free; the request's contraction is then enqueued on its
 * stream and its boundary tensors stay in the arena until the result is
 * written.  Kernels of different requests interleave on the device, so small
 * requests complete while large ones are still running.  The arena is device
 * memory owned by the caller, 256-byte aligned, reserved for the server until
 * tn_server_destroy; the library allocates no device memory for requests.  */
typedef struct {
  int64_t submitted, completed;   /* since create                              */
  int64_t queued, active;         /* waiting for admission / on the device     */
  int64_t arena_bytes, arena_in_use, peak_arena_in_use;
  int64_t peak_active;            /* most requests on the device at once       */
} tn_server_info;

/* max_slots: requests on the device at once (1..64); queue_depth: requests
 * waiting for admission before tn_submit returns TN_EBUSY.  Uses the current
 * HIP device.  Each slot is a HIP stream; the runtime maps streams onto a
 * limited number of hardware queues per process (GPU_MAX_HW_QUEUES, 4 by
 * default), and streams sharing a queue run their kernels in order, so slots
 * beyond the free hardware queues add admission capacity but no overlap.   */
tn_status tn_server_create(void* arena, size_t arena_bytes, int32_t max_slots,
                           int32_t queue_depth, tn_server** out);

/* Queue one contraction of `grid` in `order` and `precision`.  host_sites are
 * rows*cols HOST pointers to canonical float64 sites; they are copied before
 * tn_submit returns.  Errors: TN_EINVAL, TN_EOVERFLOW, TN_ENOMEM (footprint
 * larger than the whole arena), TN_EBUSY (queue full).                     */
tn_status tn_submit(tn_server* server, const tn_grid* grid, int32_t order, int32_t precision,
                    const double* const* host_sites, uint64_t* ticket);

/* TN_PENDING while queued or running; on completion writes *out, retires the
 * ticket and returns TN_OK (or the request's error: TN_ENONFINITE,
 * TN_EDEVICE).  TN_ENOTFOUND for unknown or retired tickets.               */
tn_status tn_poll(tn_server* server, uint64_t ticket, tn_result* out);

/* As tn_poll; also returns steady-clock times in ns: times_ns[0] submit,
 * [1] admission, [2] completion seen by the scheduler.                     */
tn_status tn_poll_ex(tn_server* server, uint64_t ticket, tn_result* out, int64_t* times_ns);

tn_status tn_server_stats(tn_server* server, tn_server_info* out);

/* Finishes every queued and running request, then releases the server's
 * streams and thread.  Unpolled results are dropped.                       */
tn_status tn_server_destroy(tn_server* server);

/* Library-wide options (process-wide; not for concurrent change during a
 * contraction).
 *   TN_OPT_KERNEL_IMPL : 0 = matrix-core (MFMA) kernels for absorption steps
 *                        and ring products wherever the shape allows,
 *                        vector-ALU kernels elsewhere;
 *                        1 = vector-ALU kernels only (reference path).
 *   TN_OPT_BATCH_THREADS : batch workgroup size used when a tn_batch_config is
 *                        NULL or zero (and by tn_contract_batch).
 *   TN_OPT_FUSE_STEPS  : how consecutive absorptions of one column share a
 *                        pass over the boundary (only with
 *                        TN_OPT_KERNEL_IMPL = 0):
 *                        2 (default) = chunks of up to 4 rows (3 in FP64)
 *                        with D = 4 legs between them, the slice held on chip;
 *                        1 = pairs of bulk rows (same products in the same
 *                        order as single steps: bitwise-identical results);
 *                        0 = one launch per step.
 *   TN_OPT_CHUNK_SCHEDULE : kernel of the column chunks: 0 (default) = the
 *                        chunk's intermediate results held in each
 *                        wavefront's registers (suffix 1 or a multiple of
 *                        16; other suffixes as with 1); 1 = the slice held in
 *                        LDS by a workgroup and every step passing through
 *                        LDS; 2 = as 0 with chunks of at most 3 rows in every
 *                        precision.  All give results within the stated
 *                        tolerances (sums may differ in the last bits).     */
#define TN_OPT_KERNEL_IMPL 0
#define TN_OPT_BATCH_THREADS 1
#define TN_OPT_FUSE_STEPS 2
#define TN_OPT_CHUNK_SCHEDULE 3
/*   TN_OPT_QUADRANT_STREAMS : 1 = tn_contract_grid sweeps the two bottom
 *                        quadrants on a second stream it creates for the
 *                        calling thread, concurrently with the top quadrants
 *                        and the first ring product (measured at 12x12,
 *                        D=4: FP64 -0.3 %, split BF16x3 -3 %, FP32 +0.5 %
 *                        time; the sweeps and the GEMM share the CUs); the
 *                        stream takes one of the process's hardware queues
 *                        (GPU_MAX_HW_QUEUES, 4 by default) for good.
 *                        0 (default) = one stream.                          */
#define TN_OPT_QUADRANT_STREAMS 4
/*   TN_OPT_CHAIN_STEPS : 1 (default) = with TN_OPT_FUSE_STEPS = 2, runs of
 *                        2..14 consecutive single steps of a unit whose
 *                        input and output have at most 16384 entries each
 *                        (the edge columns, small lattices) run as one
 *                        launch, one workgroup per unit, with the same
 *                        per-step arithmetic as one launch per step
 *                        (bitwise-identical results); 0 = one launch each. */
#define TN_OPT_CHAIN_STEPS 5
/*   TN_OPT_ENV_STREAMS : streams a tn_envset uses, 1..4 (default 4), read
 *                        when its workspace is sized and when it is created:
 *                        with 2 or more the right environments are swept on a
 *                        second stream concurrently with the left ones, and
 *                        the networks are dealt round-robin over all of them,
 *                        each stream with its own region of the workspace;
 *                        the set creates the extra streams (each takes one
 *                        of the process's hardware queues while the set
 *                        lives) and joins them into the caller's stream.   */
#define TN_OPT_ENV_STREAMS 6
/*   TN_OPT_ENV_ROWS    : the most GiB (0..1024, default 32) that
 *                        environments inside columns may add to a tn_envset's
 *                        workspace.  Within that budget the set also keeps the
 *                        norm network's boundary before every sweep step and
 *                        the boundary of all sites after every step (built
 *                        from the right environment by reverse steps in the
 *                        sweep's leg order), so a network whose changed sites
 *                        are sweep steps k0..k1 absorbs only those steps;
 *                        beyond it (or with 0) whole columns between column
 *                        environments.  Read when the workspace is sized and
 *                        when the set is created.                          */
#define TN_OPT_ENV_ROWS 7
/*   TN_OPT_ENV_SITES   : 1 (default) = with environments inside columns, a
 *                        network that replaces one site whose step boundary
 *                        has at most 2^20 entries is the site environment
 *                        (the boundary before the site's sweep step and the
 *                        boundary of all sites after it, contracted over
 *                        their common legs into a matrix over the site's
 *                        legs, once per site) dotted with the replacing
 *                        tensor; otherwise (and with 0) the site is absorbed
 *                        and closed against the boundary after it.  Read
 *                        when the set is created.                           */
#define TN_OPT_ENV_SITES 8
/*   TN_OPT_RING_OPERAND_SCALE : 1 = the FP64 ring products scale every staged
 *                        operand by its power of two (the path they take by
 *                        themselves when the two exponents sum beyond
 *                        +-512); 0 (default) = automatic: within that range
 *                        the factor is applied once to the results.  Both
 *                        give the same bits (power-of-two scaling is exact
 *                        while nothing leaves the normal range).           */
#define TN_OPT_RING_OPERAND_SCALE 9
/*   TN_OPT_CHUNK_STREAM : 1 (default) = the register chunks that end a
 *                        column (suffix 1) with the most rows (4 in FP32 and
 *                        BF16x3, 3 in FP64) run streamed: each wavefront
 *                        (as many as fit on the CUs) takes several tiles and
 *                        fills the first half of its next tile's slice while
 *                        the current tile's register-only steps and stores
 *                        run; n = 2..65536: streamed with at most
 *                        n wavefronts (more tiles each); 0 = one tile per
 *                        wavefront.  All give the same bits (the same
 *                        products in the same order).                      */
#define TN_OPT_CHUNK_STREAM 10
tn_status tn_set_option(int32_t option, int64_t value);

/* ------------------------------------------------------------ profiling
 * Kernel timing for roofline accounting.  While enabled, every kernel launch
 * the library issues is bracketed by HIP events on the stream it is launched
 * on; after each contraction the elapsed times are added to per-kernel
 * totals together with the kernel's algorithmic bytes and flops (boundary in
 * + out + site for an absorption step; operands + result for a ring
 * product).  Process-wide, guarded by a mutex; costs two event records per
 * launch, so leave it off outside measurements.                            */
typedef struct {
  char    name[48];        /* kernel variant, e.g. "absorb_mfma_f32"          */
  int64_t launches;
  double  total_ms;        /* sum of event-measured durations                 */
  double  bytes;           /* sum of algorithmic HBM bytes                    */
  double  flops;           /* sum of algorithmic flops                        */
} tn_kernel_stat;

/* Start (clear and enable) or stop recording.                               */
tn_status tn_profile_enable(int32_t on);
/* Copy up to `cap` per-kernel totals into `out`; *n receives the number of
 * kernels recorded (may exceed cap).                                        */
tn_status tn_profile_read(tn_kernel_stat* out, int32_t cap, int32_t* n);

#ifdef __cplusplus
}
#endif
#endif /* TN_H_ */
