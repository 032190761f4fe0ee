// gfx950 kernels for sliced tensor-network contraction.
//
//  k_gett_small       one thread per output element, FP32 VALU; tiny steps.
//  k_gett_mfma<P,WM,WN>  tiled complex GEMM over bit-strided operands (the GETT
//                     form of the einsum of Sec. 2.4).  P = 0: complex64 on FP32
//                     MFMA (v_mfma_f32_32x32x2_f32).  P = 1 / 2: the extended-
//                     precision split of Sec. 4.2 with fp16 / bf16 operands on
//                     v_mfma_f32_32x32x16_{f16,bf16}: operands are split into
//                     hi = rn(x), lo = rn(x - hi) and C += hi*hi + hi*lo + lo*hi in
//                     FP32 (lo*lo dropped).  WM x WN waves, 64 x 64 complex outputs
//                     per wave, K step 16 complex, double-buffered LDS with the next
//                     stage prefetched into registers during the MFMA phase.
//  k_gett_dma<P,L>    the split kernels' 256x128 tile id for steps whose operands are
//                     both stored split with k pairs contiguous: operands are copied
//                     global -> LDS by the DMA path (no registers, no LDS stores),
//                     one barrier per stage; L = 0: 256 x 128 tiles, three stages;
//                     L = 1 / 2: 512 x 64 / 512 x 32 tiles for 64- / 32-column steps,
//                     two stages.
//  k_gett_dot         batched dot products: one block per output element.
//  k_splitk_reduce    sums K partitions in fixed order, writes C in its layout.
//  k_permute<V>       LDS-staged index permutation, coalesced on both sides.
//  k_slice_reduce     FP64 cross-slice sum in increasing slice order.
//  k_batch            element-wise launches of many plans as one kernel (groups).
//  k_xeb_blocks / k_xeb_final  LXEB sums and the Porter-Thomas histogram of the
//                     FP64 amplitudes (verification, Sec. 2.2 and Sec. 5.1).
//
// The complex product is a real GEMM on stacked blocks: A is read as the real
// matrix [Ar Ai] (M x 2K, the interleaved complex storage itself), B is expanded
// per element into the 2x2 block [[Br, Bi], [-Bi, Br]] (2K x 2N, built in
// registers from the stored (re, im) word), and the real product is C = [Cr Ci]
// interleaved (M x 2N): 8 real flops per complex multiply-add, the same count as
// the complex product.
//
// Scaling (Sec. 4.2 dynamic scaling): an operand stored as complex64 is scaled by
// 2^s so that its largest |re|, |im| lands in [2^target, 2^(target+1)); an operand
// stored split is already in range and is used as stored.  A result written split
// is scaled by 2^t with t chosen from the bound |C| <= 2 K max|A| max|B|, so it
// fits fp16 without a second pass.  Every (tensor, slice) carries an exponent:
// true value = stored value * 2^e, e_C = e_A + e_B - s_A - s_B - t.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <type_traits>

#include "tn_internal.h"
#include "tn_kernels.h"

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ int64_t bits_offset(uint64_t v, const int64_t* __restrict__ stride, int nbits) {
  int64_t off = 0;
  for (int i = 0; i < nbits; ++i)
    if ((v >> i) & 1) off += stride[i];
  return off;
}

// frexp exponent of a positive finite float given by its bits: x in [2^(e-1), 2^e)
__device__ __forceinline__ int fexp_bits(uint32_t bits) {
  int e;
  frexpf(__uint_as_float(bits), &e);
  return e;
}

__device__ __forceinline__ bool usable_max(uint32_t bits) { return bits != 0u && bits < 0x7f800000u; }

// Power-of-two shift that brings the tensor maximum to [2^target, 2^(target+1)).
__device__ __forceinline__ int scale_shift(uint32_t maxbits, int target) {
  if (!usable_max(maxbits)) return 0;
  return target - (fexp_bits(maxbits) - 1);
}

__device__ __forceinline__ uint32_t abs_bits(float2 v) {
  const uint32_t a = __float_as_uint(v.x) & 0x7fffffffu;
  const uint32_t b = __float_as_uint(v.y) & 0x7fffffffu;
  return a > b ? a : b;
}

__device__ __forceinline__ uint32_t wave_umax(uint32_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Block-wide max of non-negative float bit patterns, one atomic per block.
// Must be reached by every thread of the block.
__device__ void block_umax_atomic(uint32_t v, uint32_t* dst, uint32_t* red) {
  v = wave_umax(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) m = red[i] > m ? red[i] : m;
    if (dst) atomicMax(dst, m);
  }
}

__device__ __forceinline__ uint32_t pack16(uint16_t lo, uint16_t hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }

// Split a scaled complex value into the hi word and the lo word of 16-bit pairs.
__device__ __forceinline__ uint2 split_pair(float re, float im, bool bf) {
  if (!bf) {
    const _Float16 hr = (_Float16)re, hm = (_Float16)im;
    const _Float16 lr = (_Float16)(re - (float)hr), lm = (_Float16)(im - (float)hm);
    return make_uint2(pack16(__builtin_bit_cast(uint16_t, hr), __builtin_bit_cast(uint16_t, hm)),
                      pack16(__builtin_bit_cast(uint16_t, lr), __builtin_bit_cast(uint16_t, lm)));
  }
  const __bf16 hr = (__bf16)re, hm = (__bf16)im;
  const __bf16 lr = (__bf16)(re - (float)hr), lm = (__bf16)(im - (float)hm);
  return make_uint2(pack16(__builtin_bit_cast(uint16_t, hr), __builtin_bit_cast(uint16_t, hm)),
                    pack16(__builtin_bit_cast(uint16_t, lr), __builtin_bit_cast(uint16_t, lm)));
}

__device__ __forceinline__ float half_bits_to_float(uint32_t h16, bool bf) {
  if (bf) return __uint_as_float(h16 << 16);
  return (float)__builtin_bit_cast(_Float16, (uint16_t)h16);
}

// hi + lo of a split element as float2 (for maxima of split-written tensors)
__device__ __forceinline__ float2 split_value(uint2 w, bool bf) {
  return make_float2(half_bits_to_float(w.x & 0xffffu, bf) + half_bits_to_float(w.y & 0xffffu, bf),
                     half_bits_to_float(w.x >> 16, bf) + half_bits_to_float(w.y >> 16, bf));
}

template <int P>
__device__ __forceinline__ floatx16 mfma16(const u32x4& a, const u32x4& b, const floatx16& c) {
  if constexpr (P == 1) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(halfx8, a), __builtin_bit_cast(halfx8, b), c,
                                                  0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
  }
}

// Per-step scale shifts (uniform within a block).
struct Scales {
  int sa, sb, t;
  float fa, fb, ft;
};

__device__ __forceinline__ Scales step_scales(const GettDesc* __restrict__ d, const GettArgs& g, int sl) {
  Scales r{0, 0, 0, 1.f, 1.f, 1.f};
  if (!g.scale_mode) return r;
  const uint32_t ma = g.maxA[g.a_ps ? sl : 0];
  const uint32_t mb = g.maxB[g.b_ps ? sl : 0];
  r.sa = g.fa == TN_FMT_SPLIT ? 0 : scale_shift(ma, g.target_exp);
  r.sb = g.fb == TN_FMT_SPLIT ? 0 : scale_shift(mb, g.target_exp);
  if (g.fc == TN_FMT_SPLIT && usable_max(ma) && usable_max(mb)) {
    // |C| < 2 K 2^(ea + sa) 2^(eb + sb); write it below 2^15
    r.t = 15 - (1 + d->kb + fexp_bits(ma) + r.sa + fexp_bits(mb) + r.sb);
  }
  r.fa = ldexpf(1.f, r.sa);
  r.fb = ldexpf(1.f, r.sb);
  r.ft = ldexpf(1.f, r.t);
  return r;
}

__device__ __forceinline__ void write_exp(const GettArgs& g, int sl, const Scales& sc) {
  g.expC[g.c_ps ? sl : 0] = g.expA[g.a_ps ? sl : 0] + g.expB[g.b_ps ? sl : 0] - sc.sa - sc.sb - sc.t;
}

// Word index of the hi word of element `off` in the blocked split format (the lo
// word is 4 words further).
__device__ __forceinline__ int64_t split_hi_word(int64_t off) { return 2 * (off & ~int64_t(3)) + (off & 3); }

// Store one result element in C's format; returns the bits of its max(|re|, |im|).
__device__ __forceinline__ uint32_t store_c(float* C, int64_t off, float2 v, const GettArgs& g, float ft) {
  v.x *= ft;
  v.y *= ft;
  if (g.fc == TN_FMT_SPLIT) {
    const uint2 w = split_pair(v.x, v.y, g.split_bf16 != 0);
    uint32_t* Cw = reinterpret_cast<uint32_t*>(C) + split_hi_word(off);
    Cw[0] = w.x;
    Cw[4] = w.y;
    return abs_bits(split_value(w, g.split_bf16 != 0));
  }
  reinterpret_cast<float2*>(C)[off] = v;
  return abs_bits(v);
}

struct ThreadEnum {
  int64_t off;
  int row, col;
};

template <int TB>
__device__ __forceinline__ ThreadEnum thread_part(const TileEnum& en, int t) {
  ThreadEnum r{0, 0, 0};
  const int lo = en.n < TB ? en.n : TB;
  for (int j = 0; j < lo; ++j) {
    if ((t >> j) & 1) {
      r.off += en.stride[j];
      r.row += en.row[j];
      r.col += en.col[j];
    }
  }
  return r;
}

template <int TB>
__device__ __forceinline__ ThreadEnum iter_part(const TileEnum& en, int it) {
  ThreadEnum r{0, 0, 0};
  for (int j = TB; j < en.n; ++j) {
    if ((it >> (j - TB)) & 1) {
      r.off += en.stride[j];
      r.row += en.row[j];
      r.col += en.col[j];
    }
  }
  return r;
}

}  // namespace

// ---------------------------------------------------------------------------
// Small steps: one thread per element of C, enumerated in C's storage order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int block_bits() { return blockDim.x == 512 ? 9 : blockDim.x == 256 ? 8 : 7; }

__device__ void gett_small_block(const GettDesc* __restrict__ d, const GettArgs& g, int64_t block, uint32_t* red) {
  const int nbb = d->own_bb + g.chunk_bits;
  const int cbits = d->c_nbits + g.chunk_bits;
  const int64_t total = (int64_t)1 << cbits;
  const int64_t e = block * blockDim.x + threadIdx.x;
  uint32_t mx = 0;
  int sl = 0;
  if (e < total) {
    uint64_t bidx = 0, m = 0, n = 0;
    for (int p = 0; p < cbits; ++p) {
      if ((e >> p) & 1) {
        const int code = d->c_pos[p];
        const int role = code >> 8, idx = code & 255;
        if (role == 0) bidx |= 1ull << idx;
        else if (role == 1) m |= 1ull << idx;
        else n |= 1ull << idx;
      }
    }
    sl = (int)(bidx >> d->own_bb);
    const Scales sc = step_scales(d, g, sl);
    int64_t oa = bits_offset(bidx, d->a_b, nbb) + bits_offset(m, d->a_m, d->mb);
    int64_t ob = bits_offset(bidx, d->b_b, nbb) + bits_offset(n, d->b_n, d->nb);
    if (g.tab_bits) {   // sparse einsum: the merged bond's value selects the operands' slices
      const uint64_t f = bidx & ((1ull << g.tab_bits) - 1);
      oa += g.tab_a[f];
      ob += g.tab_b[f];
    }
    const float2* A = reinterpret_cast<const float2*>(g.A);
    const float2* B = reinterpret_cast<const float2*>(g.B);
    float cr = 0.f, ci = 0.f;
    const int64_t K = (int64_t)1 << d->kb;
    // K in groups of 8: the group's 16 loads are issued before its products, so a
    // thread waits for memory once per group rather than once per k (the products
    // still run in increasing k)
    constexpr int KU = 8;
    const int lb = d->kb < 3 ? d->kb : 3;
    int64_t lo_a[KU], lo_b[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      lo_a[u] = bits_offset((uint64_t)u, d->a_k, lb);
      lo_b[u] = bits_offset((uint64_t)u, d->b_k, lb);
    }
    for (int64_t k0 = 0; k0 < K; k0 += KU) {
      const int64_t ga = oa + bits_offset((uint64_t)k0, d->a_k, d->kb);
      const int64_t gb = ob + bits_offset((uint64_t)k0, d->b_k, d->kb);
      float2 av[KU], bv[KU];
#pragma unroll
      for (int u = 0; u < KU; ++u)
        if (u < K) {
          av[u] = A[ga + lo_a[u]];
          bv[u] = B[gb + lo_b[u]];
        }
#pragma unroll
      for (int u = 0; u < KU; ++u)
        if (u < K) {
          const float ar = av[u].x * sc.fa, ai = av[u].y * sc.fa, br = bv[u].x * sc.fb, bi = bv[u].y * sc.fb;
          cr = fmaf(ar, br, cr);
          cr = fmaf(-ai, bi, cr);
          ci = fmaf(ar, bi, ci);
          ci = fmaf(ai, br, ci);
        }
    }
    mx = store_c(g.C, e, make_float2(cr, ci), g, sc.ft);
    const uint64_t own_mask = (1ull << d->own_bb) - 1;
    if (g.scale_mode && m == 0 && n == 0 && (bidx & own_mask) == 0) write_exp(g, sl, sc);
  }
  if (g.maxC) {
    if (d->c_nbits >= block_bits()) {
      // the whole block lies in one slice
      block_umax_atomic(mx, g.maxC + (g.c_ps ? (int)((block * blockDim.x) >> d->c_nbits) : 0), red);
    } else if (e < total) {
      atomicMax(g.maxC + (g.c_ps ? sl : 0), mx);
    }
  }
}

__global__ __launch_bounds__(256) void k_gett_small(const GettDesc* __restrict__ d, GettArgs g) {
  __shared__ uint32_t red[8];
  gett_small_block(d, g, blockIdx.x, red);
}

// Steps with (almost) no free output extent and a long K (batched dot products, such as
// the last sparse einsum of a sparse state): one block per output element, the block's
// threads split K (k = 256 j + t) and add their partial sums in a fixed tree.
__global__ __launch_bounds__(256) void k_gett_dot(const GettDesc* __restrict__ d, GettArgs g) {
  __shared__ float2 part[256];
  __shared__ int64_t hd_a[TN_MAXK], hd_b[TN_MAXK];
  const int t = threadIdx.x;
  const int nbb = d->own_bb + g.chunk_bits;
  const int cbits = d->c_nbits + g.chunk_bits;
  const int64_t e = blockIdx.x;
  uint64_t bidx = 0, m = 0, n = 0;
  for (int p = 0; p < cbits; ++p) {
    if ((e >> p) & 1) {
      const int code = d->c_pos[p];
      const int role = code >> 8, idx = code & 255;
      if (role == 0) bidx |= 1ull << idx;
      else if (role == 1) m |= 1ull << idx;
      else n |= 1ull << idx;
    }
  }
  const int sl = (int)(bidx >> d->own_bb);
  const Scales sc = step_scales(d, g, sl);
  int64_t oa = bits_offset(bidx, d->a_b, nbb) + bits_offset(m, d->a_m, d->mb);
  int64_t ob = bits_offset(bidx, d->b_b, nbb) + bits_offset(n, d->b_n, d->nb);
  if (g.tab_bits) {
    const uint64_t f = bidx & ((1ull << g.tab_bits) - 1);
    oa += g.tab_a[f];
    ob += g.tab_b[f];
  }
  // k bits 0..7 from the thread, bits 8.. from the iteration j (offsets advanced with
  // per-bit deltas: going from j to j + 1 sets bit ctz(~j) and clears the bits below it)
  const int lob = d->kb < 8 ? d->kb : 8, hib = d->kb - lob;
  if (t < hib) {
    int64_t sa = 0, sb = 0;
    for (int i = 0; i < t; ++i) {
      sa += d->a_k[lob + i];
      sb += d->b_k[lob + i];
    }
    hd_a[t] = d->a_k[lob + t] - sa;
    hd_b[t] = d->b_k[lob + t] - sb;
  }
  __syncthreads();
  float cr = 0.f, ci = 0.f;
  if (t < (1 << lob)) {
    const float2* A = reinterpret_cast<const float2*>(g.A);
    const float2* B = reinterpret_cast<const float2*>(g.B);
    int64_t ka = oa + bits_offset((uint64_t)t, d->a_k, lob);
    int64_t kb = ob + bits_offset((uint64_t)t, d->b_k, lob);
    const int64_t nj = (int64_t)1 << hib;
    for (int64_t j = 0; j < nj; ++j) {
      const float2 a = A[ka];
      const float2 b = B[kb];
      const float ar = a.x * sc.fa, ai = a.y * sc.fa, br = b.x * sc.fb, bi = b.y * sc.fb;
      cr = fmaf(ar, br, cr);
      cr = fmaf(-ai, bi, cr);
      ci = fmaf(ar, bi, ci);
      ci = fmaf(ai, br, ci);
      if (j + 1 < nj) {
        const int tz = __builtin_ctzll(~(uint64_t)j);
        ka += hd_a[tz];
        kb += hd_b[tz];
      }
    }
  }
  part[t] = make_float2(cr, ci);
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) part[t] = make_float2(part[t].x + part[t + w].x, part[t].y + part[t + w].y);
    __syncthreads();
  }
  if (t == 0) {
    const uint32_t mx = store_c(g.C, e, part[0], g, sc.ft);
    const uint64_t own_mask = (1ull << d->own_bb) - 1;
    if (g.scale_mode && m == 0 && n == 0 && (bidx & own_mask) == 0) write_exp(g, sl, sc);
    if (g.maxC) atomicMax(g.maxC + (g.c_ps ? sl : 0), mx);
  }
}

// ---------------------------------------------------------------------------
// Tiled MFMA kernel.
// ---------------------------------------------------------------------------
namespace {
constexpr int KB = 16;        // complex k per LDS stage
constexpr int LDK = KB;       // split: words per LDS row ([row][k] tiles, 4-word chunks XOR-swizzled)

// Word index of (row, k) in a swizzled [row][16] tile: the 16-byte chunk k/4 is
// XORed with (row / 4) % 4, so 16 consecutive rows read at one chunk hit 16
// distinct bank groups.
__device__ __forceinline__ int swz(int row, int k) { return row * LDK + ((((k >> 2) ^ (row >> 2)) & 3) << 2) + (k & 3); }

template <int P, int WM, int WN>
struct Tile {
  static constexpr int NT = 64 * WM * WN;
  static constexpr int TB = NT == 512 ? 9 : NT == 256 ? 8 : NT == 128 ? 7 : 6;
  static constexpr int BM = 64 * WM, BN = 64 * WN;
  static constexpr int IA = BM * KB / NT, IB = BN * KB / NT;
  static constexpr int LDA0 = 2 * BM + 2, LDB0 = 2 * BN + 2;   // c64: floats per k row
  // split: A hi/lo [BM][16]; B hi/lo expanded to real columns [2 BN][16]
  static constexpr int BUF = P == 0 ? KB * LDA0 + KB * LDB0 : 2 * BM * LDK + 4 * BN * LDK;  // words
  static constexpr int LDC = 2 * BN + 8;                        // epilogue floats per row (64 rows)
  static constexpr int SMEM = 4 * (2 * BUF > 64 * LDC ? 2 * BUF : 64 * LDC);
  // Waves per SIMD that the LDS (160 KiB per CU) lets resident: where it allows fewer
  // than two, the register budget of two waves would only cause spills, so the
  // launch bound asks for one (the wave may then use the whole register file).
  static constexpr int LDS_WAVES = (160 * 1024 / (SMEM + 64)) * WM * WN;
  static constexpr int MIN_WAVES = LDS_WAVES >= 8 ? 2 : 1;
};
}  // namespace

// Coordinates of one output tile: block -> (tile_m, tile_n, batch, K split), with
// tiles in groups of 4 (m) x 8 (n) so that blocks resident together share A and B
// panels in L2.
struct TileCtx {
  uint64_t tile_m, tile_n, bidx;
  int split, nbb, lm, ln, lk, sl;
  int64_t a_tab, b_tab;   // sparse-einsum table offsets of the tile's batch (0 without tables)
  Scales sc;
};

template <int WM, int WN>
__device__ __forceinline__ TileCtx tile_ctx(const GettDesc* __restrict__ d, const GettArgs& g, uint64_t bid) {
  TileCtx c;
  c.nbb = d->own_bb + g.chunk_bits;
  const int tmb = g.tiles_m_bits, tnb = g.tiles_n_bits;
  uint64_t tix;
  if (g.values_first) {
    // block index = value | tile << tab_bits | (batch bits above the values) | split
    const int tb = g.tab_bits;
    const uint64_t f = bid & ((1ull << tb) - 1);
    bid >>= tb;
    tix = bid & ((1ull << (tmb + tnb)) - 1);
    bid = ((bid >> (tmb + tnb)) << tb) | f;
  } else {
    tix = bid & ((1ull << (tmb + tnb)) - 1);
    bid >>= tmb + tnb;
  }
  const int gm = tmb < 2 ? tmb : 2, gn = tnb < 3 ? tnb : 3;
  c.tile_m = (tix & ((1ull << gm) - 1)) | (((tix >> (gm + gn)) & ((1ull << (tmb - gm)) - 1)) << gm);
  c.tile_n = ((tix >> gm) & ((1ull << gn) - 1)) | ((tix >> (gm + gn + tmb - gm)) << gn);
  c.bidx = bid & ((1ull << c.nbb) - 1);
  c.split = (int)(bid >> c.nbb);
  constexpr int LMAX = WM == 8 ? 9 : WM == 4 ? 8 : WM == 2 ? 7 : 6;
  constexpr int NMAX = WN == 4 ? 8 : WN == 2 ? 7 : 6;
  c.lm = d->mb < LMAX ? d->mb : LMAX;
  c.ln = d->nb < NMAX ? d->nb : NMAX;
  c.lk = d->kb < 4 ? d->kb : 4;
  c.sl = (int)(c.bidx >> d->own_bb);
  c.sc = step_scales(d, g, c.sl);
  c.a_tab = c.b_tab = 0;
  if (g.tab_bits) {
    const uint64_t f = c.bidx & ((1ull << g.tab_bits) - 1);
    c.a_tab = g.tab_a[f];
    c.b_tab = g.tab_b[f];
  }
  return c;
}

// PAIRED: accumulator blocks 0, 1 hold the real parts and blocks 2, 3 the imaginary
// parts of the wave's complex columns 0-31 and 32-63 (else real columns 2n, 2n + 1 sit
// in adjacent lanes of one block).
template <int P, int WM, int WN, bool PAIRED = false, int NBLK = 4>
__device__ __forceinline__ void store_tile(const GettDesc* __restrict__ d, const GettArgs& g, const TileCtx& cx,
                           floatx16 (&acc)[2][4], uint32_t* smem, uint32_t* red);

// One output tile of an MFMA step; `bid` is the step's block index.
template <int P, int WM, int WN>
__device__ void gett_mfma_tile(const GettDesc* __restrict__ d, const GettArgs& g, uint64_t bid, uint32_t* smem,
                               uint32_t* red) {
  using T = Tile<P, WM, WN>;
  constexpr int NT = T::NT, TB = T::TB, BM = T::BM, BN = T::BN, IA = T::IA, IB = T::IB;
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wm = w / WN, wn = w % WN;
  const TileCtx cx = tile_ctx<WM, WN>(d, g, bid);
  const int nbb = cx.nbb, lm = cx.lm, ln = cx.ln, lk = cx.lk, split = cx.split;
  const uint64_t tile_m = cx.tile_m, tile_n = cx.tile_n, bidx = cx.bidx;
  const Scales& sc = cx.sc;
  constexpr bool bf = P == 2;

  const int64_t a_base = bits_offset(bidx, d->a_b, nbb) + bits_offset(tile_m << lm, d->a_m, d->mb) + cx.a_tab;
  const int64_t b_base = bits_offset(bidx, d->b_b, nbb) + bits_offset(tile_n << ln, d->b_n, d->nb) + cx.b_tab;
  const uint2* A = reinterpret_cast<const uint2*>(g.A);
  const uint2* B = reinterpret_cast<const uint2*>(g.B);

  const int ea_elems = 1 << d->ea.n, eb_elems = 1 << d->eb.n;
  const ThreadEnum ta = thread_part<TB>(d->ea, t);
  const ThreadEnum tb = thread_part<TB>(d->eb, t);
  // Per-thread element offsets and LDS positions.  Elements beyond a small
  // operand tile load from offset 0 (always valid) and are not stored, so the
  // loads are unconditional and stay in flight together.
  // tile-local offsets stay below the operand's element count, which the planner
  // keeps below 2^31 for MFMA steps
  int32_t ia_off[IA], ib_off[IB];
  int ia_pos[IA], ib_pos[IB];
  uint32_t a_valid = 0, b_valid = 0;
#pragma unroll
  for (int i = 0; i < IA; ++i) {
    const ThreadEnum ip = iter_part<TB>(d->ea, i);
    const bool ok = t + NT * i < ea_elems;
    a_valid |= ok ? 1u << i : 0u;
    ia_off[i] = ok ? (int32_t)(ta.off + ip.off) : 0;
    const int r = ta.row + ip.row, c = ta.col + ip.col;   // r = m_loc, c = k_loc
    ia_pos[i] = P == 0 ? c * T::LDA0 + 2 * r : swz(r, c);
  }
#pragma unroll
  for (int i = 0; i < IB; ++i) {
    const ThreadEnum ip = iter_part<TB>(d->eb, i);
    const bool ok = t + NT * i < eb_elems;
    b_valid |= ok ? 1u << i : 0u;
    ib_off[i] = ok ? (int32_t)(tb.off + ip.off) : 0;
    const int r = tb.row + ip.row, c = tb.col + ip.col;   // r = n_loc, c = k_loc
    // split: real columns 2r and 2r + 1 are adjacent LDS rows with the same swizzle
    // (rows 2r and 2r + 1 share row / 4), so column 2r + 1 sits LDK words further
    ib_pos[i] = P == 0 ? c * T::LDB0 + 2 * r : swz(2 * r, c);
  }

  floatx16 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  const int64_t n_iters = (int64_t)1 << (g.k_split_bits - lk);
  const int64_t k_first = (int64_t)split << g.k_split_bits;

  if (lk < 4) {  // short K: columns beyond K stay zero in both buffers
    for (int i = t; i < 2 * T::BUF; i += NT) smem[i] = 0u;
    __syncthreads();
  }

  uint2 ra[IA], rb[IB];
  // operand offsets of the current K stage, advanced with the per-stage deltas
  int64_t ak = a_base + bits_offset(k_first, d->a_k, d->kb);
  int64_t bk = b_base + bits_offset(k_first, d->b_k, d->kb);
  const bool k_linear = d->k_linear != 0;
  const int64_t a_kstep = d->a_kstep, b_kstep = d->b_kstep;
  // split-stored operands: hi and lo words of an element sit 4 words apart
  const bool a_split = g.fa == TN_FMT_SPLIT, b_split = g.fb == TN_FMT_SPLIT;
  const uint32_t* Aw = reinterpret_cast<const uint32_t*>(g.A);
  const uint32_t* Bw = reinterpret_cast<const uint32_t*>(g.B);
  auto load_stage = [&]() {
    if (a_split) {
#pragma unroll
      for (int i = 0; i < IA; ++i) {
        const uint32_t* q = Aw + split_hi_word(ak + ia_off[i]);
        ra[i] = make_uint2(q[0], q[4]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < IA; ++i) ra[i] = A[ak + ia_off[i]];
    }
    if (b_split) {
#pragma unroll
      for (int i = 0; i < IB; ++i) {
        const uint32_t* q = Bw + split_hi_word(bk + ib_off[i]);
        rb[i] = make_uint2(q[0], q[4]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < IB; ++i) rb[i] = B[bk + ib_off[i]];
    }
  };
  auto store_stage = [&](uint32_t* buf) {
    if constexpr (P == 0) {
      float* As = reinterpret_cast<float*>(buf);
      float* Bs = As + KB * T::LDA0;
#pragma unroll
      for (int i = 0; i < IA; ++i)
        if ((a_valid >> i) & 1) {
          const float2 v = __builtin_bit_cast(float2, ra[i]);
          *reinterpret_cast<float2*>(As + ia_pos[i]) = make_float2(v.x * sc.fa, v.y * sc.fa);
        }
#pragma unroll
      for (int i = 0; i < IB; ++i)
        if ((b_valid >> i) & 1) {
          const float2 v = __builtin_bit_cast(float2, rb[i]);
          *reinterpret_cast<float2*>(Bs + ib_pos[i]) = make_float2(v.x * sc.fb, v.y * sc.fb);
        }
    } else {
      uint32_t* Ah = buf;
      uint32_t* Al = Ah + BM * LDK;
      uint32_t* Bh = Al + BM * LDK;
      uint32_t* Bl = Bh + 2 * BN * LDK;
      // operands stored split are used as loaded; complex64 operands are scaled and split
      // here (one uniform branch per operand and stage)
      if (g.fa == TN_FMT_SPLIT) {
#pragma unroll
        for (int i = 0; i < IA; ++i)
          if ((a_valid >> i) & 1) {
            Ah[ia_pos[i]] = ra[i].x;
            Al[ia_pos[i]] = ra[i].y;
          }
      } else {
#pragma unroll
        for (int i = 0; i < IA; ++i)
          if ((a_valid >> i) & 1) {
            const float2 v = __builtin_bit_cast(float2, ra[i]);
            const uint2 wv = split_pair(v.x * sc.fa, v.y * sc.fa, bf);
            Ah[ia_pos[i]] = wv.x;
            Al[ia_pos[i]] = wv.y;
          }
      }
      // B as real columns: column 2n holds (Br, -Bi), column 2n+1 (the next LDS row) (Bi, Br)
      auto put_b = [&](int i, uint2 wv) {
        Bh[ib_pos[i]] = wv.x ^ 0x80000000u;
        Bh[ib_pos[i] + LDK] = __builtin_amdgcn_alignbit(wv.x, wv.x, 16);
        Bl[ib_pos[i]] = wv.y ^ 0x80000000u;
        Bl[ib_pos[i] + LDK] = __builtin_amdgcn_alignbit(wv.y, wv.y, 16);
      };
      if (g.fb == TN_FMT_SPLIT) {
#pragma unroll
        for (int i = 0; i < IB; ++i)
          if ((b_valid >> i) & 1) put_b(i, rb[i]);
      } else {
#pragma unroll
        for (int i = 0; i < IB; ++i)
          if ((b_valid >> i) & 1) {
            const float2 v = __builtin_bit_cast(float2, rb[i]);
            put_b(i, split_pair(v.x * sc.fb, v.y * sc.fb, bf));
          }
      }
    }
  };

  const int c_half = lane >> 5, dd = lane & 1;
  const bool use_im = (c_half ^ dd) != 0;
  const float sgn = (c_half == 1 && dd == 0) ? -1.f : 1.f;

  // One K step of 8 complex (split) from the LDS stage `cur`.
  auto mfma_ks = [&](const uint32_t* cur, int ks) {
    const uint32_t* Ah = cur;
    const uint32_t* Al = Ah + BM * LDK;
    const uint32_t* Bh = Al + BM * LDK;
    const uint32_t* Bl = Bh + 2 * BN * LDK;
    const int kw = ks * 8 + (lane >> 5) * 4;
    u32x4 ah[2], al[2], bh[4], bl[4];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
      const int r = wm * 64 + mi * 32 + (lane & 31);
      ah[mi] = *reinterpret_cast<const u32x4*>(Ah + swz(r, kw));
      al[mi] = *reinterpret_cast<const u32x4*>(Al + swz(r, kw));
    }
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
      const int r = wn * 128 + ni * 32 + (lane & 31);   // real column
      bh[ni] = *reinterpret_cast<const u32x4*>(Bh + swz(r, kw));
      bl[ni] = *reinterpret_cast<const u32x4*>(Bl + swz(r, kw));
    }
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = mfma16<P>(ah[mi], bh[ni], acc[mi][ni]);
    if (g.terms == 1) return;   // hi x hi only
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = mfma16<P>(ah[mi], bl[ni], acc[mi][ni]);
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = mfma16<P>(al[mi], bh[ni], acc[mi][ni]);
  };
  // One complex k (FP32 MFMA) from the LDS stage `cur`.
  auto mfma_kk = [&](const uint32_t* cur, int kk) {
    const float* As = reinterpret_cast<const float*>(cur);
    const float* Bs = As + KB * T::LDA0;
    float a[2], b[4];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) a[mi] = As[kk * T::LDA0 + 2 * (wm * 64 + mi * 32 + (lane & 31)) + c_half];
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
      const float2 bv = *reinterpret_cast<const float2*>(Bs + kk * T::LDB0 + 2 * (wn * 64 + ni * 16 + ((lane & 31) >> 1)));
      b[ni] = sgn * (use_im ? bv.y : bv.x);
    }
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 4; ++ni)
        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
  };

  // Pipeline: stage k+1 is requested into registers, stage k is multiplied
  // from LDS, then stage k+1 is written to the other LDS buffer.  One barrier
  // per stage.
  load_stage();
  store_stage(smem);
  __syncthreads();

  for (int64_t kit = 0; kit < n_iters; ++kit) {
    const uint32_t* cur = smem + (kit & 1) * T::BUF;
    uint32_t* nxt = smem + ((kit + 1) & 1) * T::BUF;
    const bool more = kit + 1 < n_iters;
    if (more) {
      if (k_linear) {
        ak += a_kstep;
        bk += b_kstep;
      } else {
        const int t = __builtin_ctzll(~(uint64_t)kit);
        ak += d->a_kd[t];
        bk += d->b_kd[t];
      }
      load_stage();
    }
    if constexpr (P == 0) {
#pragma unroll 1
      for (int kk = 0; kk < (1 << lk); ++kk) mfma_kk(cur, kk);
    } else {
      // K < 16: one step of 8, columns beyond K are zero
      const int ks_n = lk == 4 ? 2 : 1;
#pragma unroll 1
      for (int ks = 0; ks < ks_n; ++ks) mfma_ks(cur, ks);
    }
    if (more) store_stage(nxt);
    __syncthreads();
  }

  store_tile<P, WM, WN>(d, g, cx, acc, smem, red);
}

// Epilogue: accumulators -> LDS (64 rows per pass) -> C in its layout and format
// (or split-K partials to scratch), plus the tile's contribution to C's maximum.
template <int P, int WM, int WN, bool PAIRED, int NBLK>
__device__ __forceinline__ void store_tile(const GettDesc* __restrict__ d, const GettArgs& g, const TileCtx& cx,
                           floatx16 (&acc)[2][4], uint32_t* smem, uint32_t* red) {
  using T = Tile<P, WM, WN>;
  constexpr int NT = T::NT, TB = T::TB;
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wm = w / WN, wn = w % WN;
  const int nbb = cx.nbb, lm = cx.lm, ln = cx.ln, split = cx.split, sl = cx.sl;
  const uint64_t tile_m = cx.tile_m, tile_n = cx.tile_n, bidx = cx.bidx;
  const Scales& sc = cx.sc;
  float* Cs = reinterpret_cast<float*>(smem);
  const int64_t N_loc = (int64_t)1 << ln;
  const int64_t Mtot = (int64_t)1 << d->mb, Ntot = (int64_t)1 << d->nb;
  const int npass = lm > 6 ? 1 << (lm - 6) : 1;
  const int nc = d->ec.n;
  const int ec_elems = 1 << nc;
  const ThreadEnum tc = thread_part<TB>(d->ec, t);
  const int it_c = ec_elems > NT ? ec_elems >> TB : 1;
  // the pass bits (local m bits >= 6) are the top bits of the C enumeration
  const bool pass_major = (nc - (lm > 6 ? lm - 6 : 0)) >= TB;
  const int it_per_pass = pass_major ? it_c / npass : it_c;
  int64_t c_base = 0, s_base = 0;
  if (g.write_scratch) {
    s_base = ((((int64_t)split << nbb) + (int64_t)bidx) * Mtot + ((int64_t)tile_m << lm)) * Ntot +
             ((int64_t)tile_n << ln);
  } else {
    c_base = bits_offset(bidx, d->c_b, nbb) + bits_offset(tile_m << lm, d->c_m, d->mb) +
             bits_offset(tile_n << ln, d->c_n, d->nb);
  }
  uint32_t mx = 0;
  for (int pass = 0; pass < npass; ++pass) {
    if (wm == pass) {
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < NBLK; ++ni)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int row = mi * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
            // PAIRED: blocks ni < NBLK / 2 hold real parts, the others imaginary parts
            const int col = wn * 128 + (PAIRED ? 2 * ((ni % (NBLK / 2)) * 32 + (lane & 31)) + ni / (NBLK / 2)
                                               : ni * 32 + (lane & 31));
            Cs[row * T::LDC + col] = acc[mi][ni][v];
          }
    }
    __syncthreads();
    if (g.write_scratch) {
      float2* S = reinterpret_cast<float2*>(g.scratch);
      const int64_t M_loc = (int64_t)1 << lm;
      const int64_t rows = M_loc - pass * 64 < 64 ? M_loc - pass * 64 : 64;
      for (int64_t e = t; e < rows * N_loc; e += NT) {
        const int r = (int)(e >> ln), c = (int)(e & (N_loc - 1));
        S[s_base + (int64_t)(pass * 64 + r) * Ntot + c] = *reinterpret_cast<const float2*>(Cs + r * T::LDC + 2 * c);
      }
    } else {
      const int it0 = pass_major ? pass * it_per_pass : 0;
      for (int it = it0; it < it0 + it_per_pass; ++it) {
        if (t < ec_elems) {
          const ThreadEnum ip = iter_part<TB>(d->ec, it);
          const int r = tc.row + ip.row, c = tc.col + ip.col;
          if ((r >> 6) == pass) {
            const float2 v = *reinterpret_cast<const float2*>(Cs + (r & 63) * T::LDC + 2 * c);
            const uint32_t b = store_c(g.C, c_base + tc.off + ip.off, v, g, sc.ft);
            mx = b > mx ? b : mx;
          }
        }
      }
    }
    __syncthreads();
  }
  if (!g.write_scratch) {
    if (g.scale_mode && tile_m == 0 && tile_n == 0 && t == 0 && (bidx & ((1ull << d->own_bb) - 1)) == 0)
      write_exp(g, sl, sc);
    if (g.maxC) block_umax_atomic(mx, g.maxC + (g.c_ps ? sl : 0), red);
  }
}

// ---------------------------------------------------------------------------
// Split-precision tile with operands copied global -> LDS by the DMA path
// (global_load_lds_dwordx4), three LDS stages deep.  For steps whose operands
// are both stored split and contiguous along k bit 0 (two consecutive k are one
// 16-byte pair), tile 256 x 128 complex, 8 waves.  No operand data passes
// through registers on its way to LDS, so the copy of stage k + 2 is in flight
// while stage k is multiplied, with one barrier per stage.
//
// LDS stage: A rows [256][16 k], then B columns [128][16 k]; one 128-byte row
// holds eight 16-byte slots of two elements (hi word, lo word each), XOR-swizzled
// per row (dma_swz) so that the lanes of one LDS read phase hit distinct banks.  A DMA instruction of a wave fills 1 KiB of
// LDS (8 rows) in lane order; each lane fetches the pair that belongs in its slot.
// Fragments: lane (r, half) of A takes k = 4 * half .. 4 * half + 3 of row r as
// hi and lo words; lane (n, half) of B the same k of complex column n, as (Br, -Bi)
// for the blocks of real parts of the output and as (Bi, Br) for the blocks of
// imaginary parts (one VALU operation per word either way), the products the staged
// kernel forms in LDS.
// ---------------------------------------------------------------------------
namespace {
// Tile layouts of the LDS-copy kernel: L = 0 is 256 x 128 complex (4 x 2 waves, three
// stages), L = 1 is 512 x 64 (8 x 1 waves, two stages) for steps with 64 columns, L = 2
// is 512 x 32 (8 x 1 waves of 64 x 32, two stages) for steps with 32 columns.
template <int L>
struct DmaShape {
  static constexpr int WM = L ? 8 : 4, WN = L ? 1 : 2;
  static constexpr int NB = L == 2 ? 1 : 2;                  // 32-column blocks per wave
  static constexpr int ROWS = 64 * WM, COLS = 32 * NB * WN;  // A rows and B columns of a tile
  static constexpr int MBITS = L ? 9 : 8, NBITS = L == 0 ? 7 : L == 1 ? 6 : 5;
  static constexpr int A_BYTES = ROWS * 128, STAGE = (ROWS + COLS) * 128;
  static constexpr int STAGES = L ? 2 : 3;
  // copies per wave per stage (one copy fills 8 rows); with 32 columns only waves 0-3 copy B
  static constexpr int CA = ROWS / 64, CB = (COLS / 8 + 7) / 8;
  static constexpr int NCOPY = CA + CB;
};
constexpr int DMA_SMEM = 3 * DmaShape<0>::STAGE;              // 144 KiB (the epilogue reuses it)
static_assert(2 * DmaShape<1>::STAGE <= DMA_SMEM && 2 * DmaShape<2>::STAGE <= DMA_SMEM,
              "every layout fits the same LDS");
static_assert(DMA_SMEM >= 4 * 64 * (2 * 128 + 8), "epilogue staging must fit");

// s_waitcnt with only the vector-memory counter constrained (gfx9 encoding:
// vmcnt bits 3:0 and 15:14, expcnt 6:4 = 7, lgkmcnt 11:8 = 15).
// 16-byte slot of pair s in row r is s ^ dma_swz(r): 8 consecutive rows hit 8 distinct
// slots, and 16 consecutive rows 16 distinct (row parity, slot) bank groups
__device__ __forceinline__ int dma_swz(int r) { return (r & 7) ^ ((r >> 3) & 1); }

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  __builtin_amdgcn_s_waitcnt((N & 0xf) | (0x7 << 4) | (0xf << 8) | ((N >> 4) << 14));
}

// s_waitcnt with only the LDS / scalar-memory counter constrained, to zero
__device__ __forceinline__ void wait_lgkmcnt0() { __builtin_amdgcn_s_waitcnt(0xf | (0x7 << 4) | (0x3 << 14)); }
}  // namespace

template <int P, int L>
__device__ void gett_dma_tile(const GettDesc* __restrict__ d, const GettArgs& g, uint64_t bid, uint32_t* smem,
                              uint32_t* red) {
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  using S = DmaShape<L>;
  const int wm = w / S::WN, wn = w % S::WN;
  const TileCtx cx = tile_ctx<S::WM, S::WN>(d, g, bid);
  const int nbb = cx.nbb;

  const int64_t a_base =
      bits_offset(cx.bidx, d->a_b, nbb) + bits_offset(cx.tile_m << S::MBITS, d->a_m, d->mb) + cx.a_tab;
  const int64_t b_base =
      bits_offset(cx.bidx, d->b_b, nbb) + bits_offset(cx.tile_n << S::NBITS, d->b_n, d->nb) + cx.b_tab;
  char* lds = reinterpret_cast<char*>(smem);

  // The quad each lane copies: DMA instruction i of wave w fills rows (8 i + w) * 8 + lane / 8
  // (A: i < CA, 64 CA rows; B: i < CB, 64 CB columns).  Logical slot s of a row holds the hi
  // (s even) or lo (s odd) quad of k = 4 (s / 2) .. 4 (s / 2) + 3; the lane in physical
  // slot p = lane % 8 copies logical slot p ^ dma_swz(row).  a_word / b_word: word offset
  // of that quad from the stage's element offset (doubled: two words per element).
  const int prow = lane >> 3, pslot = lane & 7;
  int32_t a_word[S::CA], b_word[S::CB];
#pragma unroll
  for (int i = 0; i < S::CA; ++i) {
    const int r = (8 * i + w) * 8 + prow;
    const int sl = pslot ^ dma_swz(r);
    a_word[i] = (int32_t)(2 * (bits_offset((uint64_t)r, d->a_m, S::MBITS) +
                               bits_offset((uint64_t)(4 * (sl >> 1)), d->a_k, 4)) +
                          4 * (sl & 1));
  }
#pragma unroll
  for (int i = 0; i < S::CB; ++i) {
    const int c = ((8 * i + w) * 8 + prow) & (S::COLS - 1);   // (wraps only for copies not issued)
    const int sl = pslot ^ dma_swz(c);
    b_word[i] = (int32_t)(2 * (bits_offset((uint64_t)c, d->b_n, S::NBITS) +
                               bits_offset((uint64_t)(4 * (sl >> 1)), d->b_k, 4)) +
                          4 * (sl & 1));
  }
  const uint32_t* Aw = reinterpret_cast<const uint32_t*>(g.A);
  const uint32_t* Bw = reinterpret_cast<const uint32_t*>(g.B);

  const int n_iters = 1 << (g.k_split_bits - 4);   // the host keeps k_split_bits - 4 <= 30
  const int64_t k_first = (int64_t)cx.split << g.k_split_bits;
  int64_t ak = a_base + bits_offset(k_first, d->a_k, d->kb);
  int64_t bk = b_base + bits_offset(k_first, d->b_k, d->kb);
  const bool k_linear = d->k_linear != 0;
  const int64_t a_kstep = d->a_kstep, b_kstep = d->b_kstep;
  int next_it = 0;   // stage whose copy is issued next
  // Copy stage next_it into LDS buffer `buf`.  Every loop iteration issues exactly one stage,
  // so the copy count in flight is the same on every iteration; stages past the last one
  // re-copy the last stage's (in-bounds) data into a buffer no wave reads again.
  auto issue = [&](int buf) {
    char* st = lds + buf * S::STAGE;
#pragma unroll
    for (int i = 0; i < S::CA; ++i)
      __builtin_amdgcn_global_load_lds(Aw + 2 * ak + a_word[i], st + (8 * i + w) * 1024, 16, 0, 0);
#pragma unroll
    for (int i = 0; i < S::CB; ++i)
      if (S::COLS >= 64 * S::CB || (8 * i + w) * 8 < S::COLS)   // every wave copies when the columns fill CB rounds
        __builtin_amdgcn_global_load_lds(Bw + 2 * bk + b_word[i], st + S::A_BYTES + (8 * i + w) * 1024, 16, 0, 0);
    if (next_it + 1 < n_iters) {
      if (k_linear) {
        ak += a_kstep;
        bk += b_kstep;
      } else {
        const int tz = __builtin_ctz(~(uint32_t)next_it);
        ak += d->a_kd[tz];
        bk += d->b_kd[tz];
      }
    }
    ++next_it;
  };

  floatx16 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  // accumulator blocks 0, 1: real parts of complex columns wn * 64 + [0, 32) and
  // [32, 64); blocks 2, 3: their imaginary parts
  const int half = lane >> 5;

  auto read_frags = [&](const char* st, int ks, u32x4 (&xa)[2][2], u32x4 (&xb)[2][2]) {
    const int s0 = ks * 4 + half * 2;      // hi slot of this lane's 4 k (lo slot: s0 + 1)
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
      const int r = wm * 64 + mi * 32 + (lane & 31);
      xa[mi][0] = *reinterpret_cast<const u32x4*>(st + r * 128 + ((s0 ^ dma_swz(r)) << 4));
      xa[mi][1] = *reinterpret_cast<const u32x4*>(st + r * 128 + (((s0 + 1) ^ dma_swz(r)) << 4));
    }
#pragma unroll
    for (int nb = 0; nb < S::NB; ++nb) {
      const int n = wn * 64 + nb * 32 + (lane & 31);
      const char* bp = st + S::A_BYTES + n * 128;
      xb[nb][0] = *reinterpret_cast<const u32x4*>(bp + ((s0 ^ dma_swz(n)) << 4));
      xb[nb][1] = *reinterpret_cast<const u32x4*>(bp + (((s0 + 1) ^ dma_swz(n)) << 4));
    }
  };
  // block ni < NB: (Br, -Bi) of column block ni; ni >= NB: (Bi, Br) of block ni - NB
  auto expand = [&](const u32x4 (&x)[2][2], int ni, int hl) {
    const u32x4& v = x[ni % S::NB][hl];
    if (ni < S::NB) return u32x4{v.x ^ 0x80000000u, v.y ^ 0x80000000u, v.z ^ 0x80000000u, v.w ^ 0x80000000u};
    return u32x4{__builtin_amdgcn_alignbit(v.x, v.x, 16), __builtin_amdgcn_alignbit(v.y, v.y, 16),
                 __builtin_amdgcn_alignbit(v.z, v.z, 16), __builtin_amdgcn_alignbit(v.w, v.w, 16)};
  };
  // Software pipeline over half-stages (8 complex k): the fragments of the next
  // half-stage are read from LDS while the products of the current one run, so
  // the MFMA pipe does not wait for LDS latency after each barrier.  The barrier
  // sits between the two halves of a stage: by then this wave's reads of the
  // stage are complete (the buffer may be refilled with stage it + STAGES) and the
  // next stage's copies have landed (its first half may be read).  The loop body has
  // no data-dependent branch: the same copies, waits and LDS reads on every iteration
  // (the last one reads fragments it does not use), so the wait for a half-stage's
  // fragments never covers the reads issued for the next one.
  auto pipeline = [&](auto terms_c) {
    constexpr int TERMS = decltype(terms_c)::value;
    // hi x hi, hi x lo, lo x hi (slot 2q: hi quad, slot 2q + 1: lo quad), column-major
    // over the wave tile (dependent products on one accumulator stay 8 MFMAs apart)
    auto products = [&](const u32x4 (&xa)[2][2], const u32x4 (&xb)[2][2]) {
#pragma unroll
      for (int ni = 0; ni < 2 * S::NB; ++ni) {
        const u32x4 bh = expand(xb, ni, 0);
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) acc[mi][ni] = mfma16<P>(xa[mi][0], bh, acc[mi][ni]);
      }
      if constexpr (TERMS == 3) {
#pragma unroll
        for (int ni = 0; ni < 2 * S::NB; ++ni) {
          const u32x4 bl = expand(xb, ni, 1);
#pragma unroll
          for (int mi = 0; mi < 2; ++mi) acc[mi][ni] = mfma16<P>(xa[mi][0], bl, acc[mi][ni]);
        }
#pragma unroll
        for (int ni = 0; ni < 2 * S::NB; ++ni) {
          const u32x4 bh = expand(xb, ni, 0);
#pragma unroll
          for (int mi = 0; mi < 2; ++mi) acc[mi][ni] = mfma16<P>(xa[mi][1], bh, acc[mi][ni]);
        }
      }
    };
    // stages 0 .. STAGES - 2 in flight, wait for stage 0, then the last buffer's stage
#pragma unroll
    for (int st0 = 0; st0 + 1 < S::STAGES; ++st0) issue(st0);
    wait_vmcnt<(S::STAGES - 2) * S::NCOPY>();
    asm volatile("s_barrier" ::: "memory");
    issue(S::STAGES - 1);
    u32x4 fa[2][2], fb[2][2], ga[2][2], gb[2][2];
    read_frags(lds, 0, fa, fb);
    int cur = 0;   // buffer of stage it
    // (scheduling barriers keep each LDS read ahead of the products it overlaps: left
    // alone, the compiler sinks the reads next to their first use)
    for (int it = 0; it < n_iters; ++it) {
      const int nxt = cur + 1 == S::STAGES ? 0 : cur + 1;
      // this half-stage's fragments (read during the previous products) have landed; waiting
      // here, before the next reads go out, keeps the wait from covering those reads
      wait_lgkmcnt0();
      read_frags(lds + cur * S::STAGE, 1, ga, gb);   // in flight during the first half's products
      __builtin_amdgcn_sched_barrier(0);
      products(fa, fb);
      __builtin_amdgcn_sched_barrier(0);
      // stage it + 1 landed (the STAGES - 2 younger stages may fly); this wave's reads of
      // stage it are done, so after the barrier its buffer takes stage it + STAGES
      wait_vmcnt<(S::STAGES - 2) * S::NCOPY>();
      wait_lgkmcnt0();
      __builtin_amdgcn_s_barrier();   // no fence: it would wait for the copies in flight
      issue(cur);
      read_frags(lds + nxt * S::STAGE, 0, fa, fb);
      __builtin_amdgcn_sched_barrier(0);
      products(ga, gb);
      __builtin_amdgcn_sched_barrier(0);
      cur = nxt;
    }
  };
  if (g.terms == 1) pipeline(std::integral_constant<int, 1>{});
  else pipeline(std::integral_constant<int, 3>{});
  wait_vmcnt<0>();   // the trailing copies land before the epilogue reuses the buffers
  __syncthreads();
  store_tile<P, S::WM, S::WN, true, 2 * S::NB>(d, g, cx, acc, smem, red);
}

template <int P, int L>
__global__ __launch_bounds__(512, 2) void k_gett_dma(const GettDesc* __restrict__ d, GettArgs g) {
  extern __shared__ __align__(16) uint32_t smem[];
  __shared__ uint32_t red[16];
  uint64_t bid = blockIdx.x;
  if ((gridDim.x & 7u) == 0) bid = (bid & 7) * (gridDim.x >> 3) + (bid >> 3);
  gett_dma_tile<P, L>(d, g, bid, smem, red);
}

template <int P, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN, (Tile<P, WM, WN>::MIN_WAVES)) void k_gett_mfma(const GettDesc* __restrict__ d, GettArgs g) {
  extern __shared__ __align__(16) uint32_t smem[];
  __shared__ uint32_t red[16];
  // Blocks are dealt to the 8 XCDs round-robin; renumber so that each XCD owns
  // a contiguous range of tiles (and so shares panels in its own L2).
  uint64_t bid = blockIdx.x;
  if ((gridDim.x & 7u) == 0) bid = (bid & 7) * (gridDim.x >> 3) + (bid >> 3);
  gett_mfma_tile<P, WM, WN>(d, g, bid, smem, red);
}

// ---------------------------------------------------------------------------
// Split-K reduction: C[e] = sum_s partial[s][b][m][n] in increasing s.
// ---------------------------------------------------------------------------
__device__ void splitk_reduce_block(const GettDesc* __restrict__ d, const GettArgs& g, int64_t block, uint32_t* red) {
  const int nbb = d->own_bb + g.chunk_bits;
  const int cbits = d->c_nbits + g.chunk_bits;
  const int64_t total = (int64_t)1 << cbits;
  const int64_t e = block * blockDim.x + threadIdx.x;
  uint32_t mx = 0;
  int sl = 0;
  if (e < total) {
    uint64_t bidx = 0, m = 0, n = 0;
    for (int p = 0; p < cbits; ++p) {
      if ((e >> p) & 1) {
        const int code = d->c_pos[p];
        const int role = code >> 8, idx = code & 255;
        if (role == 0) bidx |= 1ull << idx;
        else if (role == 1) m |= 1ull << idx;
        else n |= 1ull << idx;
      }
    }
    sl = (int)(bidx >> d->own_bb);
    const Scales sc = step_scales(d, g, sl);
    const int64_t MN = (int64_t)1 << (d->mb + d->nb);
    const int64_t per_split = MN << nbb;
    const int64_t off = ((int64_t)bidx * MN) + ((int64_t)m << d->nb) + (int64_t)n;
    const float2* S = reinterpret_cast<const float2*>(g.scratch);
    float cr = 0.f, ci = 0.f;
    for (int s = 0; s < g.splits; ++s) {
      const float2 v = S[off + s * per_split];
      cr += v.x;
      ci += v.y;
    }
    mx = store_c(g.C, e, make_float2(cr, ci), g, sc.ft);
    const uint64_t own_mask = (1ull << d->own_bb) - 1;
    if (g.scale_mode && m == 0 && n == 0 && (bidx & own_mask) == 0) write_exp(g, sl, sc);
  }
  if (g.maxC) {
    if (d->c_nbits >= block_bits()) {
      block_umax_atomic(mx, g.maxC + (g.c_ps ? (int)((block * blockDim.x) >> d->c_nbits) : 0), red);
    } else if (e < total) {
      atomicMax(g.maxC + (g.c_ps ? sl : 0), mx);
    }
  }
}

__global__ __launch_bounds__(256) void k_splitk_reduce(const GettDesc* __restrict__ d, GettArgs g) {
  __shared__ uint32_t red[8];
  splitk_reduce_block(d, g, blockIdx.x, red);
}

// ---------------------------------------------------------------------------
// Permutation: the block owns the local bits (low input bits U low output bits);
// loads follow input order, stores follow output order, staged through LDS.
// The row field of a local bit is its LDS position increment, combined by XOR
// (the planner folds a bank swizzle into them).  With V = 2 every access moves
// two elements along the lowest input (load) or output (store) bit: 16 bytes.
// ---------------------------------------------------------------------------
struct PermPart {
  int64_t off;
  int row;
};

// bits first .. first + count - 1 of an enumeration, selected by the bits of v
__device__ __forceinline__ PermPart perm_part(const TileEnum& en, int first, int count, int v) {
  PermPart r{0, 0};
  const int last = en.n < first + count ? en.n : first + count;
  for (int j = first; j < last; ++j)
    if ((v >> (j - first)) & 1) {
      r.off += en.stride[j];
      r.row ^= en.row[j];
    }
  return r;
}

template <int V>
__global__ __launch_bounds__(256) void k_permute(const PermDesc* __restrict__ p, const float2* __restrict__ in,
                                                 float2* __restrict__ out) {
  using vec = typename std::conditional<V == 2, float4, float2>::type;
  constexpr int VB = V == 2 ? 1 : 0;                              // enumeration bits inside one access
  constexpr int MAXIT = (1 << (PERM_LOCAL_MAX - VB)) >> 8;
  __shared__ float4 tile4[1 << (PERM_LOCAL_MAX - 1)];
  float2* tile = reinterpret_cast<float2*>(tile4);
  const int t = threadIdx.x;
  const uint64_t bid = blockIdx.x;
  int64_t ib = 0, ob = 0;
  for (int j = 0; j < p->nh; ++j)
    if ((bid >> j) & 1) {
      ib += p->h_in[j];
      ob += p->h_out[j];
    }
  const PermPart ti = perm_part(p->ein, VB, 8, t);
  const PermPart to = perm_part(p->eout, VB, 8, t);
  const float2* src = in + ib + ti.off;
  float2* dst = out + ob + to.off;
  const int pair = p->eout.row[0];   // LDS offset of the second element of an output pair
  auto gather = [&](int r) -> vec {
    if constexpr (V == 2) {
      if (pair == 1) return tile4[r >> 1];
      const float2 x0 = tile[r], x1 = tile[r ^ pair];
      return make_float4(x0.x, x0.y, x1.x, x1.y);
    } else {
      return tile[r];
    }
  };
  if (p->iters == MAXIT) {
    // full tile, every thread busy: all loads of the thread in flight together
    vec v[MAXIT];
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) v[it] = *reinterpret_cast<const vec*>(src + p->it_in_off[it]);
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) *reinterpret_cast<vec*>(tile + (ti.row ^ p->it_in_row[it])) = v[it];
    __syncthreads();
    if (V == 1 || pair == 1) {
#pragma unroll
      for (int it = 0; it < MAXIT; ++it)
        *reinterpret_cast<vec*>(dst + p->it_out_off[it]) =
            *reinterpret_cast<const vec*>(tile + (to.row ^ p->it_out_row[it]));
    } else {
#pragma unroll
      for (int it = 0; it < MAXIT; ++it) v[it] = gather(to.row ^ p->it_out_row[it]);
#pragma unroll
      for (int it = 0; it < MAXIT; ++it) *reinterpret_cast<vec*>(dst + p->it_out_off[it]) = v[it];
    }
  } else {
    const bool active = t < (1 << (p->ein.n - VB));
    for (int it = 0; it < p->iters; ++it)
      if (active) *reinterpret_cast<vec*>(tile + (ti.row ^ p->it_in_row[it])) =
                      *reinterpret_cast<const vec*>(src + p->it_in_off[it]);
    __syncthreads();
    for (int it = 0; it < p->iters; ++it)
      if (active) *reinterpret_cast<vec*>(dst + p->it_out_off[it]) = gather(to.row ^ p->it_out_row[it]);
  }
}

// ---------------------------------------------------------------------------
// FP64 cross-slice sum (or per-slice partials) with the slice exponents.
// ---------------------------------------------------------------------------
__device__ void slice_reduce_block(const ReduceArgs& r, int64_t block) {
  const int64_t o = block * blockDim.x + threadIdx.x;
  if (o >= r.n_amp) return;
  const float2* root = reinterpret_cast<const float2*>(r.root);
  bool bad = false;
  if (r.out) {
    for (int s = 0; s < r.n_slices; ++s) {
      const float2 v = root[(int64_t)s * r.n_amp + o];
      const int e = r.exp ? r.exp[s] : 0;
      const double re = ldexp((double)v.x, e), im = ldexp((double)v.y, e);
      bad |= !isfinite(re) || !isfinite(im);
      r.out[2 * ((int64_t)s * r.n_amp + o)] = re;
      r.out[2 * ((int64_t)s * r.n_amp + o) + 1] = im;
    }
  } else {
    double re = r.acc[2 * o], im = r.acc[2 * o + 1];
    for (int s = 0; s < r.n_slices; ++s) {
      const float2 v = root[(int64_t)s * r.n_amp + o];
      const int e = r.exp ? r.exp[s] : 0;
      const double vr = ldexp((double)v.x, e), vi = ldexp((double)v.y, e);
      bad |= !isfinite(vr) || !isfinite(vi);
      re += vr;
      im += vi;
    }
    r.acc[2 * o] = re;
    r.acc[2 * o + 1] = im;
  }
  if (bad) atomicOr(r.flag, 1);
}

__global__ __launch_bounds__(256) void k_slice_reduce(ReduceArgs r) { slice_reduce_block(r, blockIdx.x); }

// ---------------------------------------------------------------------------
// Verification statistics (LXEB, Porter-Thomas histogram) of the FP64 amplitudes:
// sample i has probability p_i = |acc[idx ? idx[i] : i]|^2; each block sums p and p^2
// of its samples in a fixed tree order into part[block][0..1] and counts x = log(D p)
// into histogram bins (integer atomics: the counts do not depend on order);
// k_xeb_final adds the block sums in block order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_xeb_blocks(const double* __restrict__ acc, const int64_t* __restrict__ idx,
                                                    int64_t m, double log_d, int32_t nbins, double x_lo,
                                                    double inv_width, double* __restrict__ part,
                                                    unsigned long long* __restrict__ hist) {
  __shared__ double s1[256], s2[256];
  const int t = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * 256 + t;
  double p = 0.0;
  if (i < m) {
    const int64_t j = idx ? idx[i] : i;
    const double re = acc[2 * j], im = acc[2 * j + 1];
    p = re * re + im * im;
    if (nbins > 0) {
      const double x = p > 0.0 ? log(p) + log_d : -INFINITY;
      const double fb = (x - x_lo) * inv_width;
      int64_t b;
      if (!(fb < (double)nbins)) b = nbins - 1;   // above the range (and NaN)
      else if (!(fb >= 0.0)) b = 0;               // below the range (and p = 0)
      else b = (int64_t)fb;
      atomicAdd(hist + b, 1ull);
    }
  }
  s1[t] = p;
  s2[t] = p * p;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      s1[t] += s1[t + w];
      s2[t] += s2[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[2 * blockIdx.x] = s1[0];
    part[2 * blockIdx.x + 1] = s2[0];
  }
}

__global__ void k_xeb_final(const double* __restrict__ part, int64_t blocks, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int64_t k = 0; k < blocks; ++k) {
    a += part[2 * k];
    b += part[2 * k + 1];
  }
  out[0] = a;
  out[1] = b;
}

// max(|re|, |im|) over a buffer, as float bits
__global__ __launch_bounds__(256) void k_absmax(const float2* __restrict__ x, int64_t n, uint32_t* dst) {
  __shared__ uint32_t red[8];
  uint32_t mx = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t b = abs_bits(x[i]);
    mx = b > mx ? b : mx;
  }
  block_umax_atomic(mx, dst, red);
}

// x *= 2^e[0] (turns a scaled product back into true values)
__global__ void k_scale_pow2(float2* __restrict__ x, int64_t n, const int32_t* __restrict__ e) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const float2 v = x[i];
    x[i] = make_float2(ldexpf(v.x, e[0]), ldexpf(v.y, e[0]));
  }
}

__device__ __forceinline__ void fill_block(uint32_t* p, uint32_t v, int64_t n, int64_t block) {
  const int64_t i = block * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) { fill_block(p, v, n, blockIdx.x); }

// ---------------------------------------------------------------------------
// Batched element-wise launches: each block looks up its task (one launch of one
// plan) and runs that launch's block, so the element-wise launches of many
// independent plans go out as one kernel.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_batch(const BatchTask* __restrict__ tasks,
                                               const int32_t* __restrict__ block_task) {
  __shared__ uint32_t red[8];
  const BatchTask& tk = tasks[block_task[blockIdx.x]];
  const int64_t b = (int64_t)blockIdx.x - tk.first_block;
  switch (tk.kind) {
    case TN_K_SMALL: gett_small_block(tk.desc, tk.g, b, red); break;
    case TN_K_SPLITK_REDUCE: splitk_reduce_block(tk.desc, tk.g, b, red); break;
    case TN_K_SLICE_REDUCE: slice_reduce_block(tk.r, b); break;
    default: fill_block(tk.fill_ptr, 0, tk.fill_n, b); break;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
namespace {
template <int P, int WM, int WN>
hipError_t launch_mfma(const GettDesc* d, const GettArgs& g, int64_t blocks, hipStream_t s) {
  using T = Tile<P, WM, WN>;
  hipError_t e = tn_prepare_kernels();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_gett_mfma<P, WM, WN>), dim3((unsigned)blocks), dim3(T::NT), T::SMEM, s, d, g);
  return hipGetLastError();
}

template <int P>
hipError_t launch_dma(const GettDesc* d, const GettArgs& g, int64_t blocks, hipStream_t s) {
  hipError_t e = tn_prepare_kernels();
  if (e != hipSuccess) return e;
  if (g.dma == 3)
    hipLaunchKernelGGL((k_gett_dma<P, 2>), dim3((unsigned)blocks), dim3(512), DMA_SMEM, s, d, g);
  else if (g.dma == 2)
    hipLaunchKernelGGL((k_gett_dma<P, 1>), dim3((unsigned)blocks), dim3(512), DMA_SMEM, s, d, g);
  else
    hipLaunchKernelGGL((k_gett_dma<P, 0>), dim3((unsigned)blocks), dim3(512), DMA_SMEM, s, d, g);
  return hipGetLastError();
}

template <int P>
hipError_t launch_mfma_tile(int tile, const GettDesc* d, const GettArgs& g, int64_t blocks, hipStream_t s) {
  if constexpr (P != 0)
    if (g.dma && tile == TN_TILE_256x128) return launch_dma<P>(d, g, blocks, s);
  switch (tile) {
    case TN_TILE_256x128: return launch_mfma<P, 4, 2>(d, g, blocks, s);
    case TN_TILE_128x128: return launch_mfma<P, 2, 2>(d, g, blocks, s);
    case TN_TILE_128x64: return launch_mfma<P, 2, 1>(d, g, blocks, s);
    case TN_TILE_64x64: return launch_mfma<P, 1, 1>(d, g, blocks, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

hipError_t tn_launch_gett(int kind, int tile, const GettDesc* d, const GettArgs& g, int64_t blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  switch (kind) {
    case TN_K_SMALL:
      if (g.dot)
        hipLaunchKernelGGL(k_gett_dot, dim3((unsigned)blocks), dim3(256), 0, s, d, g);
      else
        hipLaunchKernelGGL(k_gett_small, dim3((unsigned)blocks), dim3(256), 0, s, d, g);
      return hipGetLastError();
    case TN_K_MFMA_F32: return launch_mfma_tile<0>(tile, d, g, blocks, s);
    case TN_K_MFMA_F16X3: return launch_mfma_tile<1>(tile, d, g, blocks, s);
    case TN_K_MFMA_BF16X3: return launch_mfma_tile<2>(tile, d, g, blocks, s);
    case TN_K_SPLITK_REDUCE:
      hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)blocks), dim3(256), 0, s, d, g);
      return hipGetLastError();
    default: return hipErrorInvalidValue;
  }
}

hipError_t tn_launch_permute(const PermDesc* p, int pairs, int64_t blocks, const void* in, void* out,
                             hipStream_t s) {
  if (pairs)
    hipLaunchKernelGGL(k_permute<2>, dim3((unsigned)blocks), dim3(256), 0, s, p, reinterpret_cast<const float2*>(in),
                       reinterpret_cast<float2*>(out));
  else
    hipLaunchKernelGGL(k_permute<1>, dim3((unsigned)blocks), dim3(256), 0, s, p, reinterpret_cast<const float2*>(in),
                       reinterpret_cast<float2*>(out));
  return hipGetLastError();
}

hipError_t tn_launch_batch(const BatchTask* tasks, const int32_t* block_task, int64_t blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch, dim3((unsigned)blocks), dim3(256), 0, s, tasks, block_task);
  return hipGetLastError();
}

hipError_t tn_launch_slice_reduce(const ReduceArgs& r, hipStream_t s) {
  const int64_t blocks = (r.n_amp + 255) / 256;
  hipLaunchKernelGGL(k_slice_reduce, dim3((unsigned)blocks), dim3(256), 0, s, r);
  return hipGetLastError();
}

hipError_t tn_launch_xeb(const double* acc, const int64_t* idx, int64_t m, double log_d, int32_t nbins, double x_lo,
                         double x_hi, double* part, unsigned long long* hist, double* out, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int64_t blocks = (m + 255) / 256;
  const double inv_width = nbins > 0 ? nbins / (x_hi - x_lo) : 0.0;
  hipLaunchKernelGGL(k_xeb_blocks, dim3((unsigned)blocks), dim3(256), 0, s, acc, idx, m, log_d, nbins, x_lo,
                     inv_width, part, hist);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_xeb_final, dim3(1), dim3(64), 0, s, part, blocks, out);
  return hipGetLastError();
}

hipError_t tn_launch_absmax(const void* x, int64_t n, uint32_t* dst, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_absmax, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<const float2*>(x), n, dst);
  return hipGetLastError();
}

hipError_t tn_launch_fill_u32(void* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<uint32_t*>(p), v, n);
  return hipGetLastError();
}

hipError_t tn_launch_scale_pow2(void* x, int64_t n, const int32_t* e, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_scale_pow2, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<float2*>(x), n, e);
  return hipGetLastError();
}

// Set the dynamic-LDS limit of every MFMA kernel instance (before any launch
// is captured into a graph: attributes are not stream operations).
hipError_t tn_prepare_kernels() {
  static bool done = false;
  if (done) return hipSuccess;
  hipError_t e = hipSuccess;
  auto set = [&](const void* f, int bytes) {
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  };
#define TN_SET_ATTR(P, WM, WN) set(reinterpret_cast<const void*>(&k_gett_mfma<P, WM, WN>), Tile<P, WM, WN>::SMEM)
  TN_SET_ATTR(0, 4, 2); TN_SET_ATTR(0, 2, 2); TN_SET_ATTR(0, 2, 1); TN_SET_ATTR(0, 1, 1);
  TN_SET_ATTR(1, 4, 2); TN_SET_ATTR(1, 2, 2); TN_SET_ATTR(1, 2, 1); TN_SET_ATTR(1, 1, 1);
  TN_SET_ATTR(2, 4, 2); TN_SET_ATTR(2, 2, 2); TN_SET_ATTR(2, 2, 1); TN_SET_ATTR(2, 1, 1);
#undef TN_SET_ATTR
  set(reinterpret_cast<const void*>(&k_gett_dma<1, 0>), DMA_SMEM);
  set(reinterpret_cast<const void*>(&k_gett_dma<2, 0>), DMA_SMEM);
  set(reinterpret_cast<const void*>(&k_gett_dma<1, 1>), DMA_SMEM);
  set(reinterpret_cast<const void*>(&k_gett_dma<2, 1>), DMA_SMEM);
  set(reinterpret_cast<const void*>(&k_gett_dma<1, 2>), DMA_SMEM);
  set(reinterpret_cast<const void*>(&k_gett_dma<2, 2>), DMA_SMEM);
  if (e == hipSuccess) done = true;
  return e;
}

void tn_tile_shape(int tile, int* bm, int* bn, int* threads) {
  int wm = 2, wn = 2;
  switch (tile) {
    case TN_TILE_256x128: wm = 4; wn = 2; break;
    case TN_TILE_128x128: wm = 2; wn = 2; break;
    case TN_TILE_128x64: wm = 2; wn = 1; break;
    case TN_TILE_64x64: wm = 1; wn = 1; break;
  }
  *bm = 64 * wm;
  *bn = 64 * wn;
  *threads = 64 * wm * wn;
}
