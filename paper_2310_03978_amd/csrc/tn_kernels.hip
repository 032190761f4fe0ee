// gfx950 kernels for sliced tensor-network contraction.
//
//  k_gett_small      one thread per output element, FP32 VALU; tiny steps.
//  k_gett_mfma<P>    tiled complex GEMM over bit-strided operands (GETT form of
//                    the einsum of Sec. 2.4).  P = 0: complex64 on FP32 MFMA
//                    (v_mfma_f32_32x32x2_f32).  P = 1 / 2: the extended-precision
//                    split of Sec. 4.2 with fp16 / bf16 operands on
//                    v_mfma_f32_32x32x16_{f16,bf16}: each operand is scaled by a
//                    power of two, split into hi = rn(x), lo = rn(x - hi), and
//                    C += hi*hi + hi*lo + lo*hi in FP32 (lo*lo dropped).
//  k_splitk_reduce   sums K partitions in fixed order, writes C in its layout.
//  k_permute         LDS-staged index permutation, coalesced on both sides.
//  k_slice_reduce    FP64 cross-slice sum in increasing slice order.
//
// The complex product is a real GEMM on stacked blocks: A is read as the real
// matrix [Ar Ai] (M x 2K, the interleaved complex storage itself), B is expanded
// per element into the 2x2 block [[Br, Bi], [-Bi, Br]] (2K x 2N), and the real
// product is C = [Cr Ci] interleaved (M x 2N): 8 real flops per complex
// multiply-add, the same count as the complex product.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "tn_internal.h"
#include "tn_kernels.h"

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ int64_t bits_offset(uint64_t v, const int64_t* __restrict__ stride,
                                               int nbits) {
  int64_t off = 0;
  for (int i = 0; i < nbits; ++i)
    if ((v >> i) & 1) off += stride[i];
  return off;
}

// Power-of-two shift that brings the tensor maximum to [2^target, 2^(target+1)).
__device__ __forceinline__ int scale_shift(uint32_t maxbits, int target) {
  float mx = __uint_as_float(maxbits);
  if (!(mx > 0.f) || maxbits >= 0x7f800000u) return 0;
  int e;
  frexpf(mx, &e);
  return target - (e - 1);
}

__device__ __forceinline__ uint32_t abs_bits(float2 v) {
  uint32_t a = __float_as_uint(v.x) & 0x7fffffffu;
  uint32_t b = __float_as_uint(v.y) & 0x7fffffffu;
  return a > b ? a : b;
}

__device__ __forceinline__ uint32_t wave_umax(uint32_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    uint32_t o = __shfl_xor(v, off, 64);
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

__device__ __forceinline__ uint32_t pack_h2(_Float16 lo, _Float16 hi) {
  return (uint32_t)__builtin_bit_cast(uint16_t, lo) | ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
}
__device__ __forceinline__ uint32_t pack_b2(__bf16 lo, __bf16 hi) {
  return (uint32_t)__builtin_bit_cast(uint16_t, lo) | ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
}

// Split a (scaled) complex value into hi and lo words of packed (re, im) pairs.
template <int P>
__device__ __forceinline__ void split2(float re, float im, uint32_t& hi, uint32_t& lo,
                                       uint32_t& hi_neg_im, uint32_t& hi_swap,
                                       uint32_t& lo_neg_im, uint32_t& lo_swap) {
  if constexpr (P == 1) {
    _Float16 hr = (_Float16)re, hm = (_Float16)im;
    _Float16 lr = (_Float16)(re - (float)hr), lm = (_Float16)(im - (float)hm);
    hi = pack_h2(hr, hm);
    lo = pack_h2(lr, lm);
    hi_neg_im = pack_h2(hr, -hm);
    hi_swap = pack_h2(hm, hr);
    lo_neg_im = pack_h2(lr, -lm);
    lo_swap = pack_h2(lm, lr);
  } else {
    __bf16 hr = (__bf16)re, hm = (__bf16)im;
    __bf16 lr = (__bf16)(re - (float)hr), lm = (__bf16)(im - (float)hm);
    hi = pack_b2(hr, hm);
    lo = pack_b2(lr, lm);
    hi_neg_im = pack_b2(hr, -hm);
    hi_swap = pack_b2(hm, hr);
    lo_neg_im = pack_b2(lr, -lm);
    lo_swap = pack_b2(lm, lr);
  }
}

template <int P>
__device__ __forceinline__ floatx16 mfma16(const u32x4& a, const u32x4& b, const floatx16& c) {
  if constexpr (P == 1) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(halfx8, a),
                                                  __builtin_bit_cast(halfx8, b), c, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Small steps: one thread per element of C, enumerated in C's storage order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gett_small(const GettDesc* __restrict__ d, GettArgs g) {
  __shared__ uint32_t red[8];
  const int nbb = d->own_bb + g.chunk_bits;
  const int cbits = d->c_nbits + g.chunk_bits;
  const int64_t total = (int64_t)1 << cbits;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
    float sa = 1.f, sb = 1.f;
    int sha = 0, shb = 0;
    if (g.scale_mode) {
      sha = scale_shift(g.maxA[g.a_ps ? sl : 0], g.target_exp);
      shb = scale_shift(g.maxB[g.b_ps ? sl : 0], g.target_exp);
      sa = ldexpf(1.f, sha);
      sb = ldexpf(1.f, shb);
    }
    const int64_t oa = bits_offset(bidx, d->a_b, nbb) + bits_offset(m, d->a_m, d->mb);
    const int64_t ob = bits_offset(bidx, d->b_b, nbb) + bits_offset(n, d->b_n, d->nb);
    const float2* A = reinterpret_cast<const float2*>(g.A);
    const float2* B = reinterpret_cast<const float2*>(g.B);
    float cr = 0.f, ci = 0.f;
    const int64_t K = (int64_t)1 << d->kb;
    for (int64_t k = 0; k < K; ++k) {
      const float2 a = A[oa + bits_offset(k, d->a_k, d->kb)];
      const float2 b = B[ob + bits_offset(k, d->b_k, d->kb)];
      const float ar = a.x * sa, ai = a.y * sa, br = b.x * sb, bi = b.y * sb;
      cr = fmaf(ar, br, cr);
      cr = fmaf(-ai, bi, cr);
      ci = fmaf(ar, bi, ci);
      ci = fmaf(ai, br, ci);
    }
    reinterpret_cast<float2*>(g.C)[e] = make_float2(cr, ci);
    mx = abs_bits(make_float2(cr, ci));
    const uint64_t own_mask = (1ull << d->own_bb) - 1;
    if (g.scale_mode && m == 0 && n == 0 && (bidx & own_mask) == 0) {
      g.expC[g.c_ps ? sl : 0] = g.expA[g.a_ps ? sl : 0] + g.expB[g.b_ps ? sl : 0] - sha - shb;
    }
  }
  if (g.maxC) {
    if (d->c_nbits >= 8) {
      // the whole block lies in one slice
      block_umax_atomic(mx, g.maxC + (g.c_ps ? (int)(((int64_t)blockIdx.x * blockDim.x) >> d->c_nbits) : 0), red);
    } else if (e < total) {
      atomicMax(g.maxC + (g.c_ps ? sl : 0), mx);
    }
  }
}

// ---------------------------------------------------------------------------
// Tiled MFMA kernel.  Tile: 128 x 64 complex outputs, K step 16 complex.
// 256 threads = 4 waves in a 2 x 2 grid, each wave 64 x 32 complex
// (64 x 64 real: 2 x 2 blocks of 32 x 32 MFMA outputs).
// ---------------------------------------------------------------------------
namespace {
constexpr int BM = 128, BN = 64, BK = 16;
constexpr int LDA_F = 2 * BM + 2;      // c64: A tile [BK][BM] float2, row stride in floats
constexpr int LDB_F = 2 * BN + 2;      // c64: B tile [BK][BN] float2
constexpr int LDW = BK + 4;            // split: words per row of the [row][k] tiles
constexpr int LDC_F = 2 * BN + 8;      // epilogue C tile [BM][BN] float2
constexpr int SMEM_C64 = (BK * LDA_F + BK * LDB_F) * 4;
constexpr int SMEM_X3 = (2 * BM * LDW + 2 * (2 * BN) * LDW) * 4;
constexpr int SMEM_C = 64 * LDC_F * 4;
constexpr int SMEM_BYTES = (SMEM_C > SMEM_C64 ? (SMEM_C > SMEM_X3 ? SMEM_C : SMEM_X3)
                                              : (SMEM_C64 > SMEM_X3 ? SMEM_C64 : SMEM_X3));

struct ThreadEnum {
  int64_t off;
  int row, col;
};

__device__ __forceinline__ ThreadEnum thread_part(const TileEnum& en, int t) {
  ThreadEnum r{0, 0, 0};
  const int lo = en.n < 8 ? en.n : 8;
  for (int j = 0; j < lo; ++j) {
    if ((t >> j) & 1) {
      r.off += en.stride[j];
      r.row += en.row[j];
      r.col += en.col[j];
    }
  }
  return r;
}

__device__ __forceinline__ ThreadEnum iter_part(const TileEnum& en, int it) {
  ThreadEnum r{0, 0, 0};
  for (int j = 8; j < en.n; ++j) {
    if ((it >> (j - 8)) & 1) {
      r.off += en.stride[j];
      r.row += en.row[j];
      r.col += en.col[j];
    }
  }
  return r;
}
}  // namespace

template <int P>
__global__ __launch_bounds__(256, 2) void k_gett_mfma(const GettDesc* __restrict__ d, GettArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t red[8];
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int nbb = d->own_bb + g.chunk_bits;

  // block -> (tile_m, tile_n, batch, split)
  uint64_t bid = blockIdx.x;
  const uint64_t tile_m = bid & ((1ull << g.tiles_m_bits) - 1);
  bid >>= g.tiles_m_bits;
  const uint64_t tile_n = bid & ((1ull << g.tiles_n_bits) - 1);
  bid >>= g.tiles_n_bits;
  const uint64_t bidx = bid & ((1ull << nbb) - 1);
  const int split = (int)(bid >> nbb);

  const int lm = d->mb < 7 ? d->mb : 7;
  const int ln = d->nb < 6 ? d->nb : 6;
  const int lk = d->kb < 4 ? d->kb : 4;
  const int sl = (int)(bidx >> d->own_bb);

  int sha = 0, shb = 0;
  float sa = 1.f, sb = 1.f;
  if (g.scale_mode) {
    sha = scale_shift(g.maxA[g.a_ps ? sl : 0], g.target_exp);
    shb = scale_shift(g.maxB[g.b_ps ? sl : 0], g.target_exp);
    sa = ldexpf(1.f, sha);
    sb = ldexpf(1.f, shb);
  }

  const int64_t a_base = bits_offset(bidx, d->a_b, nbb) + bits_offset(tile_m << lm, d->a_m, d->mb);
  const int64_t b_base = bits_offset(bidx, d->b_b, nbb) + bits_offset(tile_n << ln, d->b_n, d->nb);
  const float2* A = reinterpret_cast<const float2*>(g.A);
  const float2* B = reinterpret_cast<const float2*>(g.B);

  const int na = d->ea.n, nbn = d->eb.n;
  const int ea_elems = 1 << na, eb_elems = 1 << nbn;
  const ThreadEnum ta = thread_part(d->ea, t);
  const ThreadEnum tb = thread_part(d->eb, t);
  const int it_a = ea_elems > 256 ? ea_elems >> 8 : 1;
  const int it_b = eb_elems > 256 ? eb_elems >> 8 : 1;

  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  const int64_t k_iters = (int64_t)1 << (g.k_split_bits - lk);
  const int64_t k_first = (int64_t)split << g.k_split_bits;

  float* As = reinterpret_cast<float*>(smem);
  float* Bs = As + BK * LDA_F;
  uint32_t* Ahi = reinterpret_cast<uint32_t*>(smem);
  uint32_t* Alo = Ahi + BM * LDW;
  uint32_t* Bhi = Alo + BM * LDW;
  uint32_t* Blo = Bhi + 2 * BN * LDW;

  if constexpr (P != 0) {
    // zero k columns beyond K (only when K < BK)
    if (lk < 4) {
      for (int i = t; i < 2 * BM * LDW + 4 * BN * LDW; i += 256) Ahi[i] = 0u;
      __syncthreads();
    }
  }

  for (int64_t kit = 0; kit < k_iters; ++kit) {
    const int64_t k0 = k_first + (kit << lk);
    const int64_t ak = bits_offset(k0, d->a_k, d->kb);
    const int64_t bk = bits_offset(k0, d->b_k, d->kb);
    // ---- global -> LDS ----
    for (int it = 0; it < it_a; ++it) {
      if (t < ea_elems) {
        const ThreadEnum ip = iter_part(d->ea, it);
        const float2 v = A[a_base + ak + ta.off + ip.off];
        const int r = ta.row + ip.row, c = ta.col + ip.col;   // r = m_loc, c = k_loc
        if constexpr (P == 0) {
          *reinterpret_cast<float2*>(As + c * LDA_F + 2 * r) = make_float2(v.x * sa, v.y * sa);
        } else {
          uint32_t hi, lo, h1, h2, l1, l2;
          split2<P>(v.x * sa, v.y * sa, hi, lo, h1, h2, l1, l2);
          Ahi[r * LDW + c] = hi;
          Alo[r * LDW + c] = lo;
        }
      }
    }
    for (int it = 0; it < it_b; ++it) {
      if (t < eb_elems) {
        const ThreadEnum ip = iter_part(d->eb, it);
        const float2 v = B[b_base + bk + tb.off + ip.off];
        const int r = tb.row + ip.row, c = tb.col + ip.col;   // r = n_loc, c = k_loc
        if constexpr (P == 0) {
          *reinterpret_cast<float2*>(Bs + c * LDB_F + 2 * r) = make_float2(v.x * sb, v.y * sb);
        } else {
          uint32_t hi, lo, h1, h2, l1, l2;
          split2<P>(v.x * sb, v.y * sb, hi, lo, h1, h2, l1, l2);
          Bhi[(2 * r) * LDW + c] = h1;       // real column 2n:   (Br, -Bi)
          Bhi[(2 * r + 1) * LDW + c] = h2;   // real column 2n+1: (Bi,  Br)
          Blo[(2 * r) * LDW + c] = l1;
          Blo[(2 * r + 1) * LDW + c] = l2;
        }
      }
    }
    __syncthreads();
    // ---- MFMA ----
    if constexpr (P == 0) {
      const int kk_n = 1 << lk;
      const int c = lane >> 5, dd = lane & 1;
      const bool use_im = (c ^ dd) != 0;
      const float sgn = (c == 1 && dd == 0) ? -1.f : 1.f;
      for (int kk = 0; kk < kk_n; ++kk) {
        float a[2], b[2];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) a[mi] = As[kk * LDA_F + 2 * (wm * 64 + mi * 32 + (lane & 31)) + c];
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
          const float2 bv = *reinterpret_cast<const float2*>(Bs + kk * LDB_F + 2 * (wn * 32 + ni * 16 + ((lane & 31) >> 1)));
          b[ni] = sgn * (use_im ? bv.y : bv.x);
        }
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
          for (int ni = 0; ni < 2; ++ni)
            acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 8) {
        u32x4 ah[2], al[2], bh[2], bl[2];
        const int kw = kk + (lane >> 5) * 4;
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
          const int r = wm * 64 + mi * 32 + (lane & 31);
          ah[mi] = *reinterpret_cast<const u32x4*>(Ahi + r * LDW + kw);
          al[mi] = *reinterpret_cast<const u32x4*>(Alo + r * LDW + kw);
        }
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
          const int r = wn * 64 + ni * 32 + (lane & 31);
          bh[ni] = *reinterpret_cast<const u32x4*>(Bhi + r * LDW + kw);
          bl[ni] = *reinterpret_cast<const u32x4*>(Blo + r * LDW + kw);
        }
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
          for (int ni = 0; ni < 2; ++ni) {
            acc[mi][ni] = mfma16<P>(ah[mi], bh[ni], acc[mi][ni]);
            acc[mi][ni] = mfma16<P>(ah[mi], bl[ni], acc[mi][ni]);
            acc[mi][ni] = mfma16<P>(al[mi], bh[ni], acc[mi][ni]);
          }
      }
    }
    __syncthreads();
  }

  // ---- epilogue: accumulators -> LDS (64 rows per pass) -> global ----
  float* Cs = reinterpret_cast<float*>(smem);
  const int64_t M_loc = (int64_t)1 << lm, N_loc = (int64_t)1 << ln;
  const int64_t Mtot = (int64_t)1 << d->mb, Ntot = (int64_t)1 << d->nb;
  const int64_t s_base = ((((int64_t)split << nbb) + (int64_t)bidx) * Mtot + ((int64_t)tile_m << lm)) * Ntot +
                         ((int64_t)tile_n << ln);
  const int64_t c_base = bits_offset(bidx, d->c_b, nbb) + bits_offset(tile_m << lm, d->c_m, d->mb) +
                         bits_offset(tile_n << ln, d->c_n, d->nb);
  const int nc = d->ec.n;
  const int ec_elems = 1 << nc;
  const ThreadEnum tc = thread_part(d->ec, t);
  const int it_c = ec_elems > 256 ? ec_elems >> 8 : 1;
  uint32_t mx = 0;
  for (int pass = 0; pass < 2; ++pass) {
    if (wm == pass) {
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int row = mi * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
            const int col = wn * 64 + ni * 32 + (lane & 31);
            Cs[row * LDC_F + col] = acc[mi][ni][v];
          }
    }
    __syncthreads();
    if (g.write_scratch) {
      // partials [split][batch][M][N] row-major
      float2* S = reinterpret_cast<float2*>(g.scratch);
      for (int64_t e = t; e < M_loc * N_loc; e += 256) {
        const int r = (int)(e >> ln), c = (int)(e & (N_loc - 1));
        if ((r >> 6) != pass) continue;
        S[s_base + (int64_t)r * Ntot + c] = *reinterpret_cast<const float2*>(Cs + (r & 63) * LDC_F + 2 * c);
      }
    } else {
      float2* C = reinterpret_cast<float2*>(g.C);
      for (int it = 0; it < it_c; ++it) {
        if (t < ec_elems) {
          const ThreadEnum ip = iter_part(d->ec, it);
          const int r = tc.row + ip.row, c = tc.col + ip.col;
          if ((r >> 6) == pass) {
            const float2 v = *reinterpret_cast<const float2*>(Cs + (r & 63) * LDC_F + 2 * c);
            C[c_base + tc.off + ip.off] = v;
            const uint32_t b = abs_bits(v);
            mx = b > mx ? b : mx;
          }
        }
      }
    }
    __syncthreads();
  }
  if (!g.write_scratch) {
    if (g.scale_mode && tile_m == 0 && tile_n == 0 && t == 0 &&
        (bidx & ((1ull << d->own_bb) - 1)) == 0) {
      g.expC[g.c_ps ? sl : 0] = g.expA[g.a_ps ? sl : 0] + g.expB[g.b_ps ? sl : 0] - sha - shb;
    }
    if (g.maxC) block_umax_atomic(mx, g.maxC + (g.c_ps ? sl : 0), red);
  }
}

// ---------------------------------------------------------------------------
// Split-K reduction: C[e] = sum_s partial[s][b][m][n] in increasing s.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_splitk_reduce(const GettDesc* __restrict__ d, GettArgs g) {
  __shared__ uint32_t red[8];
  const int nbb = d->own_bb + g.chunk_bits;
  const int cbits = d->c_nbits + g.chunk_bits;
  const int64_t total = (int64_t)1 << cbits;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
    reinterpret_cast<float2*>(g.C)[e] = make_float2(cr, ci);
    mx = abs_bits(make_float2(cr, ci));
    const uint64_t own_mask = (1ull << d->own_bb) - 1;
    if (g.scale_mode && m == 0 && n == 0 && (bidx & own_mask) == 0) {
      const int sha = scale_shift(g.maxA[g.a_ps ? sl : 0], g.target_exp);
      const int shb = scale_shift(g.maxB[g.b_ps ? sl : 0], g.target_exp);
      g.expC[g.c_ps ? sl : 0] = g.expA[g.a_ps ? sl : 0] + g.expB[g.b_ps ? sl : 0] - sha - shb;
    }
  }
  if (g.maxC) {
    if (d->c_nbits >= 8) {
      block_umax_atomic(mx, g.maxC + (g.c_ps ? (int)(((int64_t)blockIdx.x * blockDim.x) >> d->c_nbits) : 0), red);
    } else if (e < total) {
      atomicMax(g.maxC + (g.c_ps ? sl : 0), mx);
    }
  }
}

// ---------------------------------------------------------------------------
// Permutation: the block owns the local bits (low input bits U low output bits);
// loads follow input order, stores follow output order, staged through LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_permute(const PermDesc* __restrict__ p, const float2* __restrict__ in,
                                                 float2* __restrict__ out) {
  __shared__ float2 tile[1 << PERM_LOCAL_MAX];
  const int t = threadIdx.x;
  uint64_t bid = blockIdx.x;
  int64_t ib = 0, ob = 0;
  for (int j = 0; j < p->nh; ++j)
    if ((bid >> j) & 1) {
      ib += p->h_in[j];
      ob += p->h_out[j];
    }
  const int n = p->ein.n;
  const int elems = 1 << n;
  const ThreadEnum ti = thread_part(p->ein, t);
  const ThreadEnum to = thread_part(p->eout, t);
  const int iters = elems > 256 ? elems >> 8 : 1;
  for (int it = 0; it < iters; ++it) {
    if (t < elems) {
      const ThreadEnum ip = iter_part(p->ein, it);
      tile[ti.row + ip.row] = in[ib + ti.off + ip.off];
    }
  }
  __syncthreads();
  for (int it = 0; it < iters; ++it) {
    if (t < elems) {
      const ThreadEnum ip = iter_part(p->eout, it);
      out[ob + to.off + ip.off] = tile[to.row + ip.row];
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 cross-slice sum (or per-slice partials) with the slice exponents.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_slice_reduce(ReduceArgs r) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t tn_launch_gett(int kind, const GettDesc* d, const GettArgs& g, int64_t blocks,
                          hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  switch (kind) {
    case TN_K_SMALL:
      hipLaunchKernelGGL(k_gett_small, dim3((unsigned)blocks), dim3(256), 0, s, d, g);
      break;
    case TN_K_MFMA_F32:
      hipLaunchKernelGGL(k_gett_mfma<0>, dim3((unsigned)blocks), dim3(256), SMEM_BYTES, s, d, g);
      break;
    case TN_K_MFMA_F16X3:
      hipLaunchKernelGGL(k_gett_mfma<1>, dim3((unsigned)blocks), dim3(256), SMEM_BYTES, s, d, g);
      break;
    case TN_K_MFMA_BF16X3:
      hipLaunchKernelGGL(k_gett_mfma<2>, dim3((unsigned)blocks), dim3(256), SMEM_BYTES, s, d, g);
      break;
    case TN_K_SPLITK_REDUCE:
      hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)blocks), dim3(256), 0, s, d, g);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t tn_launch_permute(const PermDesc* p, int64_t blocks, const void* in, void* out, hipStream_t s) {
  hipLaunchKernelGGL(k_permute, dim3((unsigned)blocks), dim3(256), 0, s, p,
                     reinterpret_cast<const float2*>(in), reinterpret_cast<float2*>(out));
  return hipGetLastError();
}

hipError_t tn_launch_slice_reduce(const ReduceArgs& r, hipStream_t s) {
  const int64_t blocks = (r.n_amp + 255) / 256;
  hipLaunchKernelGGL(k_slice_reduce, dim3((unsigned)blocks), dim3(256), 0, s, r);
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

int tn_mfma_tile_m() { return BM; }
int tn_mfma_tile_n() { return BN; }
int tn_mfma_tile_k() { return BK; }
