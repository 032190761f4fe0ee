/*
 * tn.h -- sliced tensor-network contraction of random quantum circuits on one
 * MI355X (gfx950).  C ABI: plain integers, doubles and pointers; no C++ or
 * torch types cross it.  Every function returns a tn_status (0 = OK, < 0 =
 * error) and never aborts; tn_last_error_message() gives the detail of the
 * last failure on the calling thread.
 *
 * The problem statement follows the paper (arXiv 2310.03978):
 *   - a network of tensors with labelled indices; each pairwise step is the
 *     einsum C_gamma = sum_delta A_alpha B_beta of Sec. 2.4, where delta are
 *     the labels shared by A and B that no other live tensor and no output
 *     carries; shared labels that are still needed are carried as batch labels;
 *   - the contraction path of Sec. 3.1: n-1 pairs of tensor slots, the result
 *     of step (i, j) takes slot i and slot j dies;
 *   - slicing (Sec. 3.2): fixing the sliced labels splits the contraction into
 *     independent sub-tasks whose results are summed (Sec. 5, final sum of the
 *     per-device result tensors);
 *   - open output labels: the correlated amplitudes of the open qubits of the
 *     subspace form of the final state (Appendix A.1).
 *
 * Every extent must be a power of two (1 allowed): quantum-circuit bonds have
 * extent 2 and merged bonds 2^b.  Other extents give TN_E_UNSUPPORTED.
 *
 * Threading: a plan is not thread-safe.  Different plans may run on different
 * streams concurrently.
 */
#ifndef TN_H
#define TN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tn_plan_s* tn_plan;
typedef struct tn_group_s* tn_group;

typedef enum {
  TN_OK = 0,
  TN_E_ARG = -1,          /* null pointer, bad count, bad option value */
  TN_E_LABEL = -2,        /* negative label, extent mismatch, repeated label in one tensor, open label on no tensor */
  TN_E_PATH = -3,         /* wrong path length, dead/duplicate/out-of-range slot */
  TN_E_SLICE = -4,        /* sliced label open, repeated, or on no tensor; slice range out of bounds */
  TN_E_CAP = -5,          /* an intermediate exceeds options.mem_cap_elems */
  TN_E_NOMEM = -6,        /* device or host allocation failed, or workspace too small */
  TN_E_DEVICE = -7,       /* HIP error (launch failure, fault surfaced at a synchronising call) */
  TN_E_STATE = -8,        /* call not valid in this state (e.g. contraction on a host-only plan) */
  TN_E_UNSUPPORTED = -9,  /* extent that is not a power of two, too many bits for the kernels */
  TN_E_NUMERIC = -10      /* Inf or NaN reached a slice result */
} tn_status;

/* Arithmetic of the pairwise products (Sec. 4.2 of the paper).
 *  TN_PREC_C64    complex64 operands, FP32 MFMA products, FP32 accumulate.
 *  TN_PREC_F16X3  each operand scaled by a power of two, split into
 *                 hi = fp16(x), lo = fp16(x - hi); C ~ hi*hi + hi*lo + lo*hi
 *                 on FP16 MFMA with FP32 accumulate (lo*lo dropped).
 *  TN_PREC_BF16X3 the same split with bf16.
 * Intermediates are stored as complex64 in HBM in every mode; in the split
 * modes each (tensor, slice) also carries an int32 power-of-two exponent and
 * the cross-slice sum applies it in FP64. */
typedef enum { TN_PREC_C64 = 0, TN_PREC_F16X3 = 1, TN_PREC_BF16X3 = 2 } tn_precision;

/* Options.  Zero-initialise, set struct_size = sizeof(tn_options), then the
 * fields you need.  A NULL options pointer means all defaults. */
typedef struct {
  int32_t struct_size;     /* sizeof(tn_options) */
  int32_t precision;       /* tn_precision; default TN_PREC_C64 */
  int64_t mem_cap_elems;   /* largest allowed intermediate (elements per slice); 0 = no cap */
  void* stream;            /* hipStream_t for every launch of this plan; NULL = default stream */
  int32_t slice_batch;     /* slices contracted together per chunk (power of two); 0 = auto:
                              8, raised to 16 or 32 (never beyond the slice count) while the
                              chunk's per-slice intermediates fit in 32 GiB.  Tiles and K splits
                              are chosen for full chunks: a caller that contracts fewer slices
                              per call gets underfilled launches and should pass a smaller value */
  int32_t host_only;       /* 1 = plan on the host only: describe/steps work, contraction
                              calls return TN_E_STATE and no device memory is touched */
  int32_t split_policy;    /* 0 = split products on steps that are MFMA-bound, FP32 elsewhere;
                              1 = split products on every MFMA step;
                              2 = split products on every step, small ones included, except steps
                                  that read an intermediate of fewer than 4 elements (small
                                  networks and tests that must exercise the split kernels) */
  int32_t record_steps;    /* 1 = time every step's main kernel launch with HIP events on the
                              plan's stream (read with tn_plan_step_times) */
  int32_t tuning;          /* 0 = tile shapes from the shape heuristic (m and n extents);
                              1 = autotune: time every MFMA step with each tile shape at plan
                                  creation and keep the fastest (cached per step signature for the
                                  life of the process, and in tuning_cache when given);
                              2 = learned model: every MFMA step takes the tile with the least
                                  time predicted by cost_model (tn_plan_tune_with_model), which
                                  then must be non-NULL; works on host-only plans too */
  int32_t deterministic;   /* 0 or 1.  Every reduction of this library (K splits, cross-slice
                              sums, gradient sums) runs in a fixed order, so results are bitwise
                              reproducible run to run with either value; other values: TN_E_ARG */
  void* workspace;         /* caller-owned device memory for every device buffer of the plan (e.g.
                              a torch uint8 tensor), or NULL: the library allocates.  It must hold
                              the workspace_bytes a host-only plan of the same network reports, must
                              outlive the plan and is not freed by it.  Too small: TN_E_NOMEM. */
  int64_t workspace_bytes; /* size of workspace */
  /* Fields below are read only when struct_size covers them (zero otherwise). */
  const char* tuning_cache;          /* tuning = 1: path of a text file of measured tile choices
                                        ("signature tile" lines).  Read before tuning, when it
                                        exists; the choices of this plan are merged into it after
                                        tuning.  Unreadable lines are ignored; a file that cannot
                                        be written gives TN_E_ARG.  NULL = in-process cache only. */
  struct tn_costmodel_s* cost_model; /* tuning = 2: the model that picks the tiles (borrowed for
                                        the duration of tn_plan_create only) */
} tn_options;

/* Plan summary.  Operation counts follow Sec. 2.4: flops = 8*B*M*N*K per step
 * (8 real operations per complex multiply-add), bytes = 8*(|A|+|B|+|C|)
 * (complex64 storage). */
typedef struct {
  int64_t n_slices;            /* product of the sliced labels' extents (1 if none) */
  int64_t n_amplitudes;        /* product of the open labels' extents */
  int32_t n_steps;             /* pairwise steps (n_tensors - 1, or 1 for a single tensor) */
  int32_t n_slice_steps;       /* steps that depend on the slice (run once per slice) */
  double flops_per_slice;      /* sum over slice-dependent steps */
  double flops_invariant;      /* steps independent of the slice: run once per contract call */
  double bytes_per_slice;
  double bytes_invariant;
  int64_t max_intermediate;    /* elements of the largest step result (per slice) */
  int64_t workspace_bytes;     /* device bytes held by the plan; host-only plans: the bytes a
                                  caller-owned workspace (tn_options.workspace) must hold */
  int32_t slice_batch;         /* slices per chunk actually used */
  int32_t precision;
} tn_plan_info;

/* Per-step record (tests, cost-model harvesting). */
typedef struct {
  int32_t slot_a, slot_b;      /* path pair */
  int32_t per_slice;           /* 1 = depends on the slice */
  int32_t kernel;              /* 0 = small VALU kernel, 1 = FP32 MFMA, 2 = split FP16 MFMA, 3 = split BF16 MFMA */
  int64_t batch, m, n, k;      /* complex GEMM extents (k includes labels summed on one operand only) */
  int32_t split_k;             /* K partitions (1 = none) */
  int32_t tile_m, tile_n;      /* output tile in complex elements */
  int32_t a_contig, b_contig;  /* log2 of the contiguous run (elements) of A and B along the tile */
  double flops, bytes;
  int32_t tile;                /* tile id (0..3, see TN_N_TILE_SHAPES) of an MFMA step; -1 for the small kernel */
  int32_t lds_copy;            /* split operands copied global -> LDS without registers (both operands
                                  stored split, k pairs contiguous, tile id 256x128): 1 = 256 x 128 tiles,
                                  three stages; 2 = 512 x 64 tiles for steps with exactly 64 columns, two
                                  stages; 3 = 512 x 32 tiles for steps with exactly 32 columns, two
                                  stages; 0 = not */
  int32_t terms;               /* split steps: 3 = hi*hi + hi*lo + lo*hi (default), 1 = hi*hi only
                                  (tn_plan_set_step_terms); 0 for the other kernels */
  int32_t merged_bits;         /* sparse-state plans: bits of the merged open bond of a sparse einsum
                                  (its lowest batch bits, indexed through tables); -1 otherwise */
  int32_t values_first;        /* sparse einsums on MFMA kernels: 1 = blocks of consecutive merged
                                  values run together (runs of consecutive values share A's slice,
                                  which the resident blocks then read once through L2); 0 = the
                                  tiles of one value together */
} tn_step_info;

/* Build a plan.
 *  n_tensors        number of leaves (>= 1)
 *  ranks[t]         rank of leaf t (0 allowed: a scalar)
 *  labels[t][r]     label id (>= 0) of axis r of leaf t; a label may not repeat within a leaf
 *  extents[t][r]    extent of that axis; every occurrence of a label must agree
 *  data[t]          host complex128, interleaved (re, im), row-major in labels[t] order
 *                   (axis 0 slowest); prod(extents[t]) complex values; COPIED, the caller may
 *                   free it on return.  Ignored (may be NULL) for host-only plans.
 *  n_open, open_labels   output labels; amplitude index is row-major over them, the first
 *                   open label most significant.  An open label must appear on some leaf.
 *  n_steps, path    2*n_steps slot ids; step s contracts slots (path[2s], path[2s+1]); the
 *                   result goes to slot path[2s] and slot path[2s+1] dies (Sec. 3.1).
 *                   n_steps must be n_tensors - 1.
 *  n_sliced, sliced_labels   labels fixed per slice; slice id is the mixed-radix number of
 *                   their values with the first sliced label most significant (Sec. 3.2).
 *                   A sliced label may not be open.
 *  opts             may be NULL.
 * A label that appears on one leaf only and is not open is summed.
 * On success *out owns device memory (leaves, intermediates, FP64 accumulator) until
 * tn_plan_destroy.  On failure *out is NULL. */
tn_status tn_plan_create(tn_plan* out, int32_t n_tensors, const int32_t* ranks,
                         const int32_t* const* labels, const int64_t* const* extents,
                         const double* const* data, int32_t n_open, const int32_t* open_labels,
                         int32_t n_steps, const int32_t* path, int32_t n_sliced,
                         const int32_t* sliced_labels, const tn_options* opts);

/* Build a sparse-state plan (Sec. 3.3): the amplitudes of n_bitstrings sampled
 * bitstrings from one contraction.  Arguments as tn_plan_create, plus
 *  bitstrings       host uint8 [n_bitstrings][n_open], row-major, values 0 or 1: bitstring
 *                   i gives open label j the value bitstrings[i * n_open + j].  COPIED.
 * Every open label must have extent 2 and sit on exactly one leaf; n_open <= 64.
 * When two tensors that both hold open labels meet, their open bonds merge into one
 * bond whose values are the distinct restrictions of the bitstrings to the qubits they
 * hold (the sparse einsum), computed as one batched product whose operand offsets come
 * from per-step tables.  The plan's amplitude vector (tn_plan_info.n_amplitudes,
 * tn_amplitudes, tn_slice_partials) then holds one entry per value of the root's merged
 * bond; tn_plan_sparse_index gives each bitstring's entry.  TN_E_UNSUPPORTED for open
 * labels that break these rules, TN_E_ARG for bad bitstrings. */
tn_status tn_plan_create_sparse(tn_plan* out, int32_t n_tensors, const int32_t* ranks,
                                const int32_t* const* labels, const int64_t* const* extents,
                                const double* const* data, int32_t n_open, const int32_t* open_labels,
                                int32_t n_steps, const int32_t* path, int32_t n_sliced,
                                const int32_t* sliced_labels, int64_t n_bitstrings,
                                const uint8_t* bitstrings, const tn_options* opts);

/* For a sparse-state plan: index[i] = the entry of the plan's amplitude vector that holds
 * bitstring i's amplitude (host array of n_bitstrings, which must match the plan).
 * TN_E_STATE for a plan built without bitstrings. */
tn_status tn_plan_sparse_index(tn_plan plan, int64_t* index, int64_t n_bitstrings);

/* Free a plan; legal on NULL and on partly built plans.  Synchronises the plan's stream. */
void tn_plan_destroy(tn_plan plan);

tn_status tn_plan_describe(tn_plan plan, tn_plan_info* out);

/* Copy min(cap, n_steps) step records into steps[] (host memory). */
tn_status tn_plan_steps(tn_plan plan, tn_step_info* steps, int32_t cap);

/* Per-step kernel times recorded since the last call (options.record_steps = 1):
 * synchronises the stream, then writes for step i < cap the summed duration in
 * milliseconds of its main kernel launches (ms_total[i], may be NULL) and their
 * number (launches[i], may be NULL), and clears the record.  A step split along K
 * is timed from its main launch to the end of its reduction launch.  TN_E_STATE if
 * recording is off. */
tn_status tn_plan_step_times(tn_plan plan, double* ms_total, int64_t* launches, int32_t cap);

/* Per-step precision (Sec. 4.3, Table 3: the extended-precision product replaced by a
 * single low-precision one on the steps that cost most).  terms = 3 runs split step
 * `step` as hi*hi + hi*lo + lo*hi (the default), terms = 1 as hi*hi only: a third of the
 * MFMA work, with the operands' rounding to 16-bit (relative 2^-11 for fp16, 2^-8 for
 * bf16) no longer compensated.  Takes effect from the next contraction.  TN_E_ARG for a
 * step that does not run a split kernel or terms other than 1 and 3. */
tn_status tn_plan_set_step_terms(tn_plan plan, int32_t step, int32_t terms);

/* Split-precision steps ranked costliest first, into order[0 .. min(cap, *n_split)) (step
 * indices; *n_split, may be NULL, receives their number).  by_time = 1 ranks by the time
 * the steps take on one chunk of slices, measured with events on the plan's stream (Sec.
 * 4.3 sorts contractions by actual computation time; device plans only, the accumulator
 * is untouched); by_time = 0 by flops per contraction (slice-dependent steps counted once
 * per slice).  Steps of equal cost keep their order. */
tn_status tn_plan_rank_split_steps(tn_plan plan, int32_t by_time, int32_t* order, int32_t cap, int32_t* n_split);

/* Per-step precision chosen under an error budget (Sec. 4.3, Table 3 and the equation for
 * epsilon_L2^2).  The split steps are ranked by measured time (as tn_plan_rank_split_steps
 * with by_time = 1).  The per-slice amplitudes of slice_ids[0 .. n_ids) are computed with
 * three products on every step (the reference), then with one product (hi * hi) on the
 * top k steps for growing k (1, 2, 3, 4, 6, 9, ..., every split step), each time with
 * epsilon_L2^2 = |L2^2 - L2^2'| / L2^2 over all those amplitudes.  The largest k reached
 * before the first k whose epsilon_L2^2 exceeds `budget` is kept: the plan leaves this call
 * with one product on its top k steps and three elsewhere (*k_chosen = k, 0 if even k = 1
 * exceeds the budget; *eps_l2sq = its epsilon_L2^2; either may be NULL).  The accumulator
 * is untouched.  TN_E_STATE for host-only plans and plans without split steps. */
tn_status tn_plan_choose_single_products(tn_plan plan, double budget, const int64_t* slice_ids, int64_t n_ids,
                                         int32_t* k_chosen, double* eps_l2sq);

/* Contract slices [first_slice, first_slice + n_slices) and ADD their amplitudes into the
 * plan's FP64 accumulator, summing in increasing slice id (Sec. 3.2, Sec. 5: sub-task
 * results are summed).  Asynchronous on opts.stream; slice-independent steps are computed
 * once per call.  Re-running a range adds it again: the caller owns range bookkeeping.
 * TN_E_SLICE if the range leaves [0, n_slices). */
tn_status tn_contract_slices(tn_plan plan, int64_t first_slice, int64_t n_slices);

/* Amplitudes of individual slices (not accumulated): out[i*2*n_amp + 2*o + {0,1}] for
 * slice_ids[i], in true scale, complex128 interleaved.  Synchronous.  Leaves the
 * accumulator untouched. */
tn_status tn_slice_partials(tn_plan plan, const int64_t* slice_ids, int64_t n, double* out);

/* Synchronise the stream and copy the accumulator (n_amp complex128, interleaved) to out.
 * n_amp must equal n_amplitudes.  *slices_accumulated (may be NULL) receives the number
 * of slices added since the last reset.  TN_E_NUMERIC if Inf/NaN reached a slice result,
 * TN_E_DEVICE if a kernel failed. */
tn_status tn_amplitudes(tn_plan plan, double* out, int64_t n_amp, int64_t* slices_accumulated);

/* Verification statistics of the accumulated amplitudes (Sec. 2.2 LXEB; Sec. 4.3 LXEB
 * through the squared norm; Sec. 5.1 Porter-Thomas histogram), computed on the GPU in FP64.
 * The samples are the plan's bitstrings for a sparse-state plan (a repeated bitstring counts
 * each time), else every amplitude of the accumulator; sample i has p_i = |a_i|^2 (the
 * accumulator is taken as is: the caller divides by nothing and contracts every slice
 * first).  With D = 2^n_qubits and m samples:
 *   sum_p = sum p_i, sum_p2 = sum p_i^2 (fixed-order sums), mean_dp = D sum_p / m,
 *   mean_dp2 = D^2 sum_p2 / m, lxeb = mean_dp - 1 (F_l of the sampled LXEB equation).
 * hist (n_bins int64 on the host, may be NULL when n_bins = 0) counts x = log(D p_i) in
 * n_bins equal bins over [x_lo, x_hi); samples below x_lo (p = 0 included) go to the first
 * bin, samples at or above x_hi to the last.  Synchronises the plan's stream; allocates and
 * frees about 8 m + 16 m / 256 + 8 n_bins bytes of device memory.  TN_E_NUMERIC if Inf/NaN
 * reached a slice result. */
typedef struct {
  int64_t samples;
  double sum_p, sum_p2;
  double mean_dp, mean_dp2;
  double lxeb;
} tn_xeb_stats;
tn_status tn_plan_xeb(tn_plan plan, int32_t n_qubits, int32_t n_bins, double x_lo, double x_hi,
                      tn_xeb_stats* stats, int64_t* hist);

/* Restore an accumulator (checkpoint resume): acc is n_amp complex128 on the host. */
tn_status tn_accumulator_set(tn_plan plan, const double* acc, int64_t n_amp,
                             int64_t slices_accumulated);

/* Zero the accumulator and the slice count. */
tn_status tn_reset(tn_plan plan);

/* Batching form: many independent contractions -- slice ranges of one network and
 * many small, uneven sub-networks -- submitted as ONE replay of a captured hipGraph
 * (Sec. 4.1 batched execution; slices and sub-networks are independent sub-tasks,
 * Sec. 3.2).  The group captures, once per set of ranges, every plan's kernel chain
 * (its slice-independent steps, then per chunk of slices its slice-dependent steps
 * and the FP64 cross-slice sum) into one graph whose parallel branches each run
 * the chains of a subset of the plans.  Plans go to branches by
 * longest-processing-time-first on their flop counts, so branches carry similar
 * work; branches run concurrently on the device.  Within a branch the chains
 * advance in rounds: round r is the r-th launch of each of the branch's plans.
 * The element-wise launches of a round (small steps, split-K sums, FP64 slice
 * sums, fills) go out as ONE batched launch whose blocks look their task up in a
 * table; the round's MFMA launches follow one by one.  Every block runs the code
 * the plan runs on its own, with the plan's own tiles, so a group adds exactly
 * what tn_contract_slices on each plan adds (bit for bit).  The task tables live
 * in device memory the group allocates with each captured graph (about 300 bytes
 * per batched task and 4 bytes per block).
 *
 * tn_group_create: plans[0..n) must be device plans of one precision; they stay
 *   owned by the caller and must outlive the group, and must not be used for
 *   contraction concurrently with it.  opts may be NULL; opts->stream orders the
 *   group after and before the caller's stream; opts->slice_batch, when > 0, is the
 *   number of graph branches (default min(n, 8)).
 * tn_group_contract: for every plan i, contracts slices [first[i], first[i] +
 *   count[i]) and ADDS them into plan i's accumulator, like tn_contract_slices.
 *   Asynchronous; read results with tn_amplitudes on each plan.  The graph is
 *   captured on the first call with a given set of ranges and replayed (one
 *   hipGraphLaunch) on later calls with the same ranges.
 *   A graph branch holds at most 8192 kernel nodes (a plan's launches, a batched launch
 *   counting once): larger ranges give TN_E_UNSUPPORTED before anything is captured, and the
 *   caller splits them over several calls.
 * tn_group_prepare: captures (or finds in the group's cache) the graph of those ranges
 *   without launching it, so that a later tn_group_contract with the same ranges is a
 *   replay only (for callers that keep capture out of a timed or latency-bound region).
 *   Adds nothing to any accumulator; errors as tn_group_contract.
 * tn_group_describe: kernel nodes (a batched launch counts once) and branches of
 *   the graph of the last call. */
tn_status tn_group_create(tn_group* out, const tn_plan* plans, int32_t n_plans, const tn_options* opts);
tn_status tn_group_contract(tn_group group, const int64_t* first, const int64_t* count);
tn_status tn_group_prepare(tn_group group, const int64_t* first, const int64_t* count);
tn_status tn_group_describe(tn_group group, int64_t* n_kernels, int32_t* n_branches);
void tn_group_destroy(tn_group group);

/* ---- Learned step-time cost model ----
 * The paper orders contraction candidates by their measured time on the device
 * (Sec. 4.1) and scores trees with a cost that weighs compute and memory
 * traffic (Sec. 3.2).  Here a small MLP learns the time of one kernel launch of
 * a step from that step's shape, layout and kernel configuration, trained on
 * the library's own timings; it picks tile shapes without timing every
 * candidate, and can score whole plans (e.g. candidate slicings, planned on the
 * host only).
 *
 * Features (TN_COST_FEATURES floats per (step, tile)), in this order:
 *   0 batch bits (own + slice-local chunk bits)   1 m bits   2 n bits   3 k bits
 *   4 log2 flops per launch   5 log2 operand+result bytes per launch   6 (4) - (5)
 *   7 tile-grid m bits   8 tile-grid n bits   9 log2 K splits   10 log2 blocks per launch
 *   11 slice-dependent step   12..15 kernel one-hot (small, FP32 MFMA, split FP16, split BF16)
 *   16..19 tile one-hot (256x128, 128x128, 128x64, 64x64; all 0 for the small kernel)
 *   20 contiguous run bits of A's tile   21 of B's tile   22 of C's tile
 *   23..25 split storage of A, B, C   26 min(0, m bits - tile m bits)
 *   27 min(0, n bits - tile n bits)   28 log2 K stages (16 complex each) per split
 * The target is ln(microseconds per launch). */
#define TN_COST_FEATURES 29
#define TN_N_TILE_SHAPES 4 /* tile ids 0..3: 256x128, 128x128, 128x64, 64x64 complex */

typedef struct tn_costmodel_s* tn_costmodel;

/* Features of step `step` run with tile id `tile` (-1 = the step's current tile) into
 * out[0..TN_COST_FEATURES); cap must be >= TN_COST_FEATURES.  Works on host-only plans.
 * The tile id is ignored for steps on the small kernel.  TN_E_ARG on a bad step or tile. */
tn_status tn_plan_step_features(tn_plan plan, int32_t step, int32_t tile, float* out, int32_t cap);

/* Run MFMA step `step` with tile id `tile` from now on (the K split follows the tile).
 * TN_E_ARG for a step on the small kernel or a bad tile id.  Device plans: may grow the
 * split-K scratch buffer; ordered on the plan's stream. */
tn_status tn_plan_set_tile(tn_plan plan, int32_t step, int32_t tile);

/* Choose every MFMA step's tile as the argmin of the model's predicted time over the
 * tile ids and apply it (tn_plan_set_tile).  predicted_us (may be NULL; cap entries)
 * receives the predicted microseconds per launch of every step with its chosen tile.
 * The model must have TN_COST_FEATURES inputs.  Works on host-only plans. */
tn_status tn_plan_tune_with_model(tn_plan plan, tn_costmodel model, float* predicted_us, int32_t cap);

/* Predicted microseconds per launch of canonical pairwise steps, for scoring contraction
 * trees by predicted time instead of flop and byte counts (the hardware-weighted score of
 * Sec. 3.2, learned).  shapes[4 i .. 4 i + 3] = (batch, m, n, k) bit counts of step i, each
 * 0..30, batch at most 16: extents 2^batch x 2^m x 2^n x 2^k complex, laid out as a plan
 * lays out intermediates for their consumer (k innermost in both operands, operands and
 * result stored split when the step runs a split kernel), in `precision` (tn_precision).
 * The kernel and K split follow the planner's rules for such a step; us[i] receives the
 * model's time for the tile it predicts fastest.  The model must have TN_COST_FEATURES
 * inputs.  Synchronous (one forward pass over all candidates on the GPU).
 * TN_E_UNSUPPORTED for bit counts out of range. */
tn_status tn_costmodel_predict_shapes(tn_costmodel model, int32_t precision, const int32_t* shapes, int64_t n,
                                      float* us);

/* MLP with n_features inputs (1..32), two hidden layers of 64 ReLU units and one output,
 * FP32, trained with MSE loss and Adam (beta1 0.9, beta2 0.999, eps 1e-8) by the library's
 * HIP kernels (forward, per-sample deltas, per-weight gradient sums in sample order, Adam).
 * Parameters are one flat FP32 array: W1 [64 x F] row-major, b1 [64], W2 [64 x 64], b2 [64],
 * w3 [64], b3.  Inputs are standardised as (x - mean) / std before the first layer.
 * create: He-uniform weights from a counter-based generator (splitmix64) seeded by `seed`,
 *   zero biases, mean 0, std 1.  All calls are synchronous and use the null stream. */
tn_status tn_costmodel_create(tn_costmodel* out, int32_t n_features, uint64_t seed);
void tn_costmodel_destroy(tn_costmodel model);
tn_status tn_costmodel_describe(tn_costmodel model, int32_t* n_features, int32_t* hidden,
                                int64_t* n_params);
/* mean, std: n_features host floats each; std must be > 0. */
tn_status tn_costmodel_set_normalization(tn_costmodel model, const float* mean, const float* std);
/* n must equal n_params.  set_params also clears the Adam moments and step count. */
tn_status tn_costmodel_get_params(tn_costmodel model, float* out, int64_t n);
tn_status tn_costmodel_set_params(tn_costmodel model, const float* params, int64_t n);
/* y[i] = model(X[i]) for n rows of X (host, row-major [n x n_features]). */
tn_status tn_costmodel_predict(tn_costmodel model, const float* X, int64_t n, float* y);
/* Gradient of the mean squared error over n samples (host X [n x F], t [n]) into grad
 * (n_params floats, may be NULL) and the loss into *loss (may be NULL); parameters unchanged. */
tn_status tn_costmodel_gradient(tn_costmodel model, const float* X, const float* t, int64_t n,
                                float* grad, float* loss);
/* One Adam update of the parameters with the given gradient (n_params host floats). */
tn_status tn_costmodel_adam_step(tn_costmodel model, const float* grad, int64_t n, float lr);
/* Minibatch training: `epochs` passes over the n samples in an order shuffled per epoch,
 * one Adam step per batch of `batch` consecutive samples of that order (the last batch of an
 * epoch may be smaller; its loss is the mean over its own samples).  The order starts as
 * 0..n-1 and is shuffled in place before every epoch e = 0, 1, ... by Fisher-Yates
 * (Durstenfeld's form): for i = n-1 down to 1, swap entries i and
 * j = splitmix64(seed XOR splitmix64(e * 2^32 + i)) mod (i + 1), with splitmix64 the
 * generator of Steele, Lea and Flood (2014) applied to its argument as the state (state +
 * 0x9e3779b97f4a7c15, then its two xor-shift-multiply rounds and the final xor-shift).
 * *final_loss (may be NULL) receives the MSE over all n samples after training. */
tn_status tn_costmodel_train(tn_costmodel model, const float* X, const float* t, int64_t n,
                             int32_t epochs, int32_t batch, float lr, uint64_t seed,
                             float* final_loss);

/* Diagnostic entry points on caller-owned device memory (complex64 interleaved),
 * asynchronous on `stream` (hipStream_t or NULL).  They run the same kernels as plan
 * steps and exist for kernel-level tests and microbenchmarks.
 *
 * tn_gemm: C[b][m][n] = sum_k A[b][m][k] * B[b][k][n], all row-major contiguous; batch, m,
 * n, k powers of two (>= 1).  precision as tn_precision; the split modes scale each operand
 * by one power of two (from its largest |re|, |im|) and write C in true scale.
 * Synchronous: returns after the stream has finished the product. */
tn_status tn_gemm(int32_t precision, int64_t batch, int64_t m, int64_t n, int64_t k,
                  const void* A, const void* B, void* C, void* stream);

/* tn_gemm_noalloc: tn_gemm for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * kernels and results as tn_gemm (bit for bit), but the product's scratch (its layout
 * descriptor, the max / exponent slots of the split modes and the K-split partials) lives
 * in a fixed device array of TN_GEMM_NOALLOC_SCRATCH_BYTES that the library's code object
 * holds on every GPU it runs on until the process ends; the call makes no hipMalloc,
 * hipFree or other allocating device call.  The array of the current device is used (the
 * stream must belong to it); its device address is looked up once per device on the first
 * call there.  The slots are cleared by a fill kernel on every call and the partials are
 * overwritten, so nothing carries over between calls, but every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other threads, other streams) race and must
 * be serialised by the caller.  Synchronous like tn_gemm.  A product whose scratch exceeds
 * the array (large outputs with a K split) gives TN_E_NOMEM and launches nothing. */
#define TN_GEMM_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
tn_status tn_gemm_noalloc(int32_t precision, int64_t batch, int64_t m, int64_t n, int64_t k,
                          const void* A, const void* B, void* C, void* stream);

/* tn_permute: out = in with axes permuted: out axis r is in axis perm[r]; dims are the
 * input extents (powers of two), row-major.  rank <= 32. */
tn_status tn_permute(int32_t rank, const int64_t* dims, const int32_t* perm, const void* in,
                     void* out, void* stream);

const char* tn_status_string(tn_status status);
const char* tn_last_error_message(void);

#ifdef __cplusplus
}
#endif

#endif /* TN_H */
