// Launch interface of the gfx950 kernels (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tn_internal.h"

enum {
  TN_K_SMALL = 0,
  TN_K_MFMA_F32 = 1,
  TN_K_MFMA_F16X3 = 2,
  TN_K_MFMA_BF16X3 = 3,
  TN_K_SPLITK_REDUCE = 4,
  TN_K_SLICE_REDUCE = 5,
  TN_K_FILL = 6
};

// MFMA tile shapes (complex outputs per block, waves)
enum {
  TN_TILE_256x128 = 0,   // 4 x 2 waves
  TN_TILE_128x128 = 1,   // 2 x 2 waves
  TN_TILE_128x64 = 2,    // 2 x 1 waves
  TN_TILE_64x64 = 3,     // 1 wave
  TN_N_TILES = 4
};

#define PERM_LOCAL_MAX 12

// Permutation of one bit-indexed tensor: the block owns the local bits
// (enumerated by ein in input-stride order and by eout in output-stride order,
// row = LDS position increment, combined by XOR); block index bits select the
// high bits.  pairs = 1: 16-byte accesses of two elements along the lowest input
// and output bits (needs 16-byte aligned buffers, the local bit of input stride 1
// at LDS position 1, and every other row even).
struct PermDesc {
  int32_t nh;
  int32_t pad_;
  int64_t h_in[64];
  int64_t h_out[64];
  TileEnum ein, eout;
  // per iteration of a thread (the enumeration bits above the pair bit, if any, and
  // the 8 thread bits): offsets and LDS rows in input and output order
  int32_t iters;
  int32_t pad2_;
  int64_t it_in_off[1 << (PERM_LOCAL_MAX - 8)], it_out_off[1 << (PERM_LOCAL_MAX - 8)];
  int32_t it_in_row[1 << (PERM_LOCAL_MAX - 8)], it_out_row[1 << (PERM_LOCAL_MAX - 8)];
};

hipError_t tn_launch_gett(int kind, int tile, const GettDesc* d, const GettArgs& g, int64_t blocks, hipStream_t s);
hipError_t tn_launch_permute(const PermDesc* p, int pairs, int64_t blocks, const void* in, void* out,
                             hipStream_t s);
// One element-wise launch (a small step, a split-K sum, an FP64 slice sum or a fill)
// inside a batched launch: its blocks are first_block .. first_block + blocks - 1 of
// the batched grid, and block_task maps each block of the grid to its task.
struct BatchTask {
  int32_t kind;                 // TN_K_SMALL (not the dot form), TN_K_SPLITK_REDUCE, TN_K_SLICE_REDUCE, TN_K_FILL
  int32_t pad_;
  int64_t first_block;
  const GettDesc* desc;
  GettArgs g;
  ReduceArgs r;
  uint32_t* fill_ptr;
  int64_t fill_n;
};

hipError_t tn_launch_batch(const BatchTask* tasks, const int32_t* block_task, int64_t blocks, hipStream_t s);
hipError_t tn_launch_slice_reduce(const ReduceArgs& r, hipStream_t s);
hipError_t tn_launch_absmax(const void* x, int64_t n, uint32_t* dst, hipStream_t s);
// part: 2 * ceil(m / 256) doubles; hist: nbins zeroed counters; out: 2 doubles (sum p, sum p^2)
hipError_t tn_launch_xeb(const double* acc, const int64_t* idx, int64_t m, double log_d, int32_t nbins, double x_lo,
                         double x_hi, double* part, unsigned long long* hist, double* out, hipStream_t s);
hipError_t tn_launch_fill_u32(void* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t tn_launch_scale_pow2(void* x, int64_t n, const int32_t* e, hipStream_t s);
void tn_tile_shape(int tile, int* bm, int* bn, int* threads);
hipError_t tn_prepare_kernels();
