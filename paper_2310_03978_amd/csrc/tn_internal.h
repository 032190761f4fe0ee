// Internal structures shared by the host planner and the gfx950 kernels.
//
// Every extent is a power of two, so every tensor index is a bit string and
// every layout is a permutation of bits: the storage offset of an element is
// the sum, over its set index bits, of that bit's stride (a power of two, or
// 0 when an operand does not carry the bit).  A pairwise step (the einsum of
// Sec. 2.4) becomes a batched complex GEMM over four bit groups:
//   batch bits  -- carried by A, B and C (labels still needed elsewhere), plus
//                  the slice-local bits of a chunk of slices (Sec. 3.2),
//   m bits      -- A and C only,   n bits -- B and C only,
//   k bits      -- summed: A and B, or only one of them (stride 0 in the other).
// The planner lays every intermediate out the way its consumer reads it
// (consumer-driven index order, Sec. 4.1), so an operand of a step is stored
// [batch][free][k] with its k bits innermost.
#pragma once

#include <stdint.h>

#define TN_MAXB 24   // batch bits incl. slice-local bits
#define TN_MAXR 40   // m or n bits
#define TN_MAXK 40   // k bits
#define TN_MAXE 16   // local bits of one operand tile

// Small tile enumeration: the local bits of one operand tile, sorted by storage
// stride so that consecutive threads touch consecutive addresses.
struct TileEnum {
  int32_t n;                    // number of local bits
  int32_t pad_;
  int64_t stride[TN_MAXE];      // storage stride of the j-th local bit
  int32_t row[TN_MAXE];         // increment of the tile row index (m or n) for that bit
  int32_t col[TN_MAXE];         // increment of the tile column index (k, or n for C)
};

struct GettDesc {
  int32_t nbb;                  // batch bits present in the descriptor (own + max slice-local)
  int32_t own_bb;               // own batch bits (slice-local bits follow them)
  int32_t mb, nb, kb;           // m, n, k bit counts
  int32_t c_nbits;              // storage bits of C without slice-local bits
  int64_t c_elems;              // elements of one slice of C
  int64_t a_b[TN_MAXB], a_m[TN_MAXR], a_k[TN_MAXK];
  int64_t b_b[TN_MAXB], b_k[TN_MAXK], b_n[TN_MAXR];
  int64_t c_b[TN_MAXB], c_m[TN_MAXR], c_n[TN_MAXR];
  // K-stage advance of the MFMA kernels: a stage covers the 4 lowest k bits
  // (16 complex), and going from stage s to s + 1 changes the operand offsets
  // by a_kd[t] / b_kd[t], t = trailing one bits of s:
  //   kd[t] = k_stride[4 + t] - sum_{j < t} k_stride[4 + j].
  int64_t a_kd[TN_MAXK], b_kd[TN_MAXK];
  // k_linear = 1 when the k bits above the stage have strides kstep << j in both
  // operands: the offset of stage s is then s * kstep and no table is read
  int64_t a_kstep, b_kstep;
  int32_t k_linear;
  int32_t pad_k;
  // role of each storage position of C, LSB first (own layout then slice-local bits):
  // (role << 8) | index, role 0 = batch, 1 = m, 2 = n
  int32_t c_pos[TN_MAXR + TN_MAXB];
  // tile enumerations for the MFMA kernels (filled for the step's tile shape)
  TileEnum ea, eb, ec;
};

// Per-launch arguments (by value).
struct GettArgs {
  const float* A;               // complex64 interleaved
  const float* B;
  float* C;
  float* scratch;               // split-K partials [split][batch][m][n] (complex64)
  const uint32_t* maxA; const uint32_t* maxB; uint32_t* maxC;   // |.|max bits per (tensor, slice)
  const int32_t* expA; const int32_t* expB; int32_t* expC;       // power-of-two exponents
  int32_t a_ps, b_ps, c_ps;     // 1: index max/exp by slice-local index, 0: slot 0
  int32_t scale_mode;           // 0: no scaling/exponents; 1: scale operands to target_exp
  int32_t target_exp;           // floor(log2 max) after scaling (14 for fp16 products)
  int32_t chunk_bits;           // active slice-local bits in this launch
  int32_t splits;               // K partitions
  int32_t k_split_bits;         // log2(K per split)
  int32_t tiles_m_bits, tiles_n_bits;
  int32_t write_scratch;        // 1: this launch writes split partials to scratch
  int32_t fa, fb, fc;           // storage format of A, B, C: TN_FMT_C64 or TN_FMT_SPLIT
  int32_t split_bf16;           // split storage uses bf16 halves (else fp16)
  int32_t dma;                  // split kernels: operands copied global -> LDS directly (k_gett_dma)
  int32_t terms;                // split kernels: 3 = hi.hi + hi.lo + lo.hi, 1 = hi.hi only
  // sparse einsum: the lowest tab_bits batch bits index per-step tables of element
  // offsets added to A's and B's batch offsets (null when the step has none)
  const int64_t* tab_a;
  const int64_t* tab_b;
  int32_t tab_bits;
  // 1: the table bits are the lowest bits of the MFMA kernels' block index, so blocks of
  // consecutive merged values (which share A's slice) run together; 0: tiles of one value
  int32_t values_first;
  int32_t dot;                  // small steps: one block per output element, K split over the block
};

// Storage formats of an intermediate.  TN_FMT_SPLIT keeps, per complex element,
// the word (hi_re, hi_im) and the word (lo_re, lo_im) of 16-bit halves with
// hi = rn(x), lo = rn(x - hi) of the scaled value: 8 bytes, like complex64.
// The words are blocked by 4 elements: for the group of elements 4g .. 4g + 3 the
// four hi words come first, then the four lo words (word 8g + j holds hi of element
// 4g + j, word 8g + 4 + j its lo), so four consecutive k of one operand row are one
// 16-byte hi quad and one 16-byte lo quad.  Split tensors have a multiple of 4
// elements.
#define TN_FMT_C64 0
#define TN_FMT_SPLIT 1

struct ReduceArgs {
  const float* root;            // [slice][amp] complex64
  const int32_t* exp;           // per slice exponent or null
  double* acc;                  // [amp] complex128 accumulator
  double* out;                  // partials output or null
  int32_t* flag;                // set to 1 on Inf/NaN
  int64_t n_amp;
  int32_t n_slices;             // slices in this chunk
};

// Detail text for tn_last_error_message() on the calling thread (defined with the planner).
void tn_set_error_detail(const char* msg);

// Exception barrier of the C entry points: no C++ exception crosses the ABI.  Called
// inside a catch handler, tn_api_exception_status() records the detail and returns
// TN_E_NOMEM for a failed or impossible host allocation, TN_E_STATE otherwise.
int tn_api_exception_status() noexcept;
#define TN_TRY try {
#define TN_CATCH \
  }              \
  catch (...) { return (tn_status)tn_api_exception_status(); }
#define TN_TRY_VOID try {
#define TN_CATCH_VOID \
  }                   \
  catch (...) {}

