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
  int32_t slice_batch;     /* slices contracted together per chunk (power of two); 0 = auto */
  int32_t host_only;       /* 1 = plan on the host only: describe/steps work, contraction
                              calls return TN_E_STATE and no device memory is touched */
  int32_t split_policy;    /* 0 = split products on steps that are MFMA-bound, FP32 elsewhere;
                              1 = split products on every MFMA step */
  int32_t record_steps;    /* 1 = time every step's main kernel launch with HIP events on the
                              plan's stream (read with tn_plan_step_times) */
  int32_t tuning;          /* 0 = tile shapes from the shape heuristic; 1 = autotune: time every
                              MFMA step with each tile shape at plan creation and keep the
                              fastest (cached per step signature for the life of the process) */
  int32_t reserved[5];
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
  int64_t workspace_bytes;     /* device bytes held by the plan */
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

/* Free a plan; legal on NULL and on partly built plans.  Synchronises the plan's stream. */
void tn_plan_destroy(tn_plan plan);

tn_status tn_plan_describe(tn_plan plan, tn_plan_info* out);

/* Copy min(cap, n_steps) step records into steps[] (host memory). */
tn_status tn_plan_steps(tn_plan plan, tn_step_info* steps, int32_t cap);

/* Per-step kernel times recorded since the last call (options.record_steps = 1):
 * synchronises the stream, then writes for step i < cap the summed duration in
 * milliseconds of its main kernel launches (ms_total[i], may be NULL) and their
 * number (launches[i], may be NULL), and clears the record.  Split-K reduction
 * launches are not included.  TN_E_STATE if recording is off. */
tn_status tn_plan_step_times(tn_plan plan, double* ms_total, int64_t* launches, int32_t cap);

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

/* Restore an accumulator (checkpoint resume): acc is n_amp complex128 on the host. */
tn_status tn_accumulator_set(tn_plan plan, const double* acc, int64_t n_amp,
                             int64_t slices_accumulated);

/* Zero the accumulator and the slice count. */
tn_status tn_reset(tn_plan plan);

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
