// Host planner and C ABI for sliced tensor-network contraction (see include/tn.h).
//
// Planning (once per network):
//   1. validate labels, extents, open and sliced labels and the path (Sec. 3.1);
//   2. expand every label into bits (all extents are powers of two);
//   3. replay the path: for each pairwise step classify labels into batch /
//      m / n / k (the einsum of Sec. 2.4; a label only one operand carries and
//      nobody needs later is summed too), and mark steps that depend on the
//      slice (Sec. 3.2);
//   4. choose layouts from the root down: the root is stored in output order,
//      and every other tensor is stored the way its consumer reads it,
//      [k][free][batch] from the least significant bit up, with free bits in the
//      order the consumer's result needs them (consumer-driven index order,
//      Sec. 4.1 "reorder indices" applied to every step);
//   5. pick a kernel, tile and K split per step, build the bit-stride
//      descriptors, and place intermediates in two arenas by liveness;
//   6. upload leaves and permute them on the device into their planned layouts.
// Execution: slice-independent steps run once per call; slice-dependent steps
// run per chunk of slices, with the slice-local index as extra batch bits;
// every chunk ends with the FP64 cross-slice sum (Sec. 5: result tensors summed).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <set>
#include <string>
#include <vector>

#include "../../include/tn.h"
#include "tn_internal.h"
#include "tn_kernels.h"

namespace {

thread_local std::string g_err;

tn_status fail(tn_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

}  // namespace

void tn_set_error_detail(const char* msg) { g_err = msg ? msg : ""; }

int tn_api_exception_status() noexcept {
  int status = TN_E_STATE;
  const char* what = "internal error";
  try {
    throw;
  } catch (const std::bad_alloc&) {
    status = TN_E_NOMEM;
    what = "host memory allocation failed";
  } catch (const std::length_error&) {
    status = TN_E_NOMEM;
    what = "requested host buffer is larger than the host can address";
  } catch (...) {
  }
  try {
    g_err = what;
  } catch (...) {
    g_err.clear();
  }
  return status;
}

namespace {

int ilog2_exact(int64_t v) {
  if (v < 1) return -1;
  int b = 0;
  while ((int64_t(1) << b) < v) ++b;
  return (int64_t(1) << b) == v ? b : -1;
}

struct Label {
  int64_t ext = 0;
  int nb = 0;       // bits
  int bit0 = 0;     // first bit id
  bool open = false;
  int slice_pos = -1;
  int user = 0;
  int qubit = -1;   // sparse-state plans: column of the bitstrings this open label measures
  bool merged = false;  // sparse-state plans: a merged open bond (made by the planner)
};

struct Tensor {
  std::vector<int> labels;   // dense label ids (non-sliced), in no particular order
  std::vector<int> bits;     // storage order, LSB first (non-sliced bits)
  std::vector<int> sbits;    // leaves: sliced bits stored above `bits` (LSB first)
  bool per_slice = false;
  bool leaf = false;
  bool layout_set = false;
  int64_t elems = 1;         // 2^bits.size()
  int fmt = TN_FMT_C64;      // storage format, chosen for the consumer
  int arena = 0;             // 0 leaves, 1 invariant, 2 per-slice
  int64_t offset = 0;        // elements
  std::vector<int> user_layout;  // leaves: bits of the caller's row-major data, LSB first
  // sparse-state plans (Sec. 3.3): measured qubits whose open bonds this tensor holds
  // (bit i = bitstring column i), either as their own labels (raw) or as one merged bond
  // `merged` whose value v stands for keys[v], a distinct restriction of the bitstrings
  uint64_t sq = 0;
  int merged = -1;
  std::vector<uint64_t> keys;
  std::vector<std::pair<uint64_t, int64_t>> key_value;   // (key, value) sorted by key, for lookups
};

struct Step {
  int slot_a = 0, slot_b = 0;
  int ta = 0, tb = 0, tc = 0;
  std::vector<int> lb, lm, ln, lk;   // label classes
  std::vector<int> bb, mb, nb, kb;   // bit lists in GEMM order, LSB first
  bool per_slice = false;
  int kernel = TN_K_SMALL;
  int tile = TN_TILE_128x128;
  int splits = 1;
  int k_split_bits = 0;
  int tiles_m_bits = 0, tiles_n_bits = 0;
  int a_contig = 0, b_contig = 0;
  int dma = 0;                       // split tile fed by global -> LDS copies: 1 = 256x128, 2 = 512x64, 3 = 512x32
  int terms = 3;                     // split steps: products per complex multiply-add term (3 or 1)
  bool dot = false;                  // small steps with <= 4 outputs per batch and long K: block per output
  double flops = 0, bytes = 0;
  int64_t scratch_elems = 0;         // split-K partials (elements)
  // sparse einsum (Sec. 3.3): the result's merged bond `tab_label` is the step's lowest
  // batch bits; operand offsets for its value f come from tables (element offsets)
  int tab_label = -1;
  std::vector<int> ia_labels, ib_labels;   // open-bond labels of A and B the tables index
  std::vector<int64_t> tab_a, tab_b;
  int64_t tab_a_max = 0, tab_b_max = 0;
  int values_first = 0;   // MFMA block order: merged values fastest (see build_tables)
  int64_t* d_tab_a = nullptr;
  int64_t* d_tab_b = nullptr;
  GettDesc desc;
};

// First-fit interval allocator (units: elements), records the peak.
struct Arena {
  std::map<int64_t, int64_t> free_;  // offset -> size
  int64_t top = 0, peak = 0;
  static int64_t align(int64_t n) { return (n + 63) & ~int64_t(63); }
  int64_t alloc(int64_t n) {
    n = align(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        int64_t off = it->first, sz = it->second;
        free_.erase(it);
        if (sz > n) free_[off + n] = sz - n;
        return off;
      }
    }
    int64_t off = top;
    top += n;
    peak = std::max(peak, top);
    return off;
  }
  void release(int64_t off, int64_t n) {
    n = align(n);
    free_[off] = n;
    // coalesce
    auto it = free_.find(off);
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
        it = prev;
      }
    }
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it->first + it->second == top) {
      top = it->first;
      free_.erase(it);
    }
  }
};

}  // namespace

struct tn_plan_s {
  tn_options opts{};
  bool host_only = false;
  int64_t epoch = 0;         // bumped whenever a step is re-tiled (graphs captured before are stale)
  hipStream_t stream = nullptr;
  int precision = TN_PREC_C64;

  std::vector<Label> labels;
  int n_bits = 0;
  std::vector<int> slice_bits;        // global slice id bit j -> bit id
  int n_slice_bits = 0;
  int64_t n_slices = 1;
  int64_t n_amp = 1;
  int n_leaves = 0;
  // sparse-state plans: bitstring keys (bit i = column i) and, per bitstring, the index of
  // its amplitude in the root's merged open bond
  bool sparse = false;
  std::vector<uint64_t> bkeys;
  std::vector<int64_t> amp_index;

  std::vector<Tensor> tensors;
  std::vector<Step> steps;
  std::vector<int> inv_order, ps_order;   // step indices
  int root = -1;

  int S = 1, s_bits = 0;                  // slice chunk size
  int64_t leaf_elems = 0, inv_elems = 0, ps_elems = 0;  // arena sizes (ps: for S slices)
  int64_t max_intermediate = 0;
  double flops_ps = 0, flops_inv = 0, bytes_ps = 0, bytes_inv = 0;

  // device
  float* d_leaves = nullptr;
  float* d_inv = nullptr;
  float* d_ps = nullptr;
  GettDesc* d_desc = nullptr;
  uint32_t* d_max_inv = nullptr;   // [n_tensors]
  uint32_t* d_max_ps = nullptr;    // [n_tensors][S]
  int32_t* d_exp_inv = nullptr;
  int32_t* d_exp_ps = nullptr;
  double* d_acc = nullptr;
  double* d_part = nullptr;        // [S][n_amp] complex128 partials
  int32_t* d_flag = nullptr;
  float* d_scratch = nullptr;      // split-K partials, shared by all steps (one stream)
  int64_t* d_tabs = nullptr;       // sparse-einsum tables of every step (element offsets)
  int64_t tab_elems = 0;
  int64_t scratch_elems = 0;
  // caller-owned workspace (options.workspace): every device buffer is carved from it
  bool own_memory = true;
  char* ws = nullptr;
  size_t ws_size = 0, ws_used = 0;
  int64_t ws_need = 0;             // bytes a workspace must hold (computed for every plan)
  int64_t slices_acc = 0;
  size_t device_bytes = 0;

  // step timing (options.record_steps)
  struct Timing {
    int step;
    hipEvent_t start, stop;
  };
  std::vector<Timing> pending;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> event_pool;
  std::vector<double> step_ms;
  std::vector<int64_t> step_launches;

  ~tn_plan_s() {
    if (stream) hipStreamSynchronize(stream);
    else if (!host_only) hipDeviceSynchronize();
    void* ptrs[] = {d_leaves, d_inv, d_ps, d_desc, d_max_inv, d_max_ps, d_exp_inv, d_exp_ps, d_acc, d_part, d_flag,
                    d_scratch, d_tabs};
    if (own_memory)
      for (void* p : ptrs)
        if (p) hipFree(p);
    for (auto& t : pending) event_pool.push_back({t.start, t.stop});
    for (auto& e : event_pool) {
      hipEventDestroy(e.first);
      hipEventDestroy(e.second);
    }
  }
};

namespace {

bool scaled(const tn_plan_s* p) { return p->precision != TN_PREC_C64; }

// stride (elements) of bit q in tensor T's storage; 0 if absent
int64_t bit_stride(const Tensor& T, int q) {
  for (size_t i = 0; i < T.bits.size(); ++i)
    if (T.bits[i] == q) return int64_t(1) << i;
  for (size_t i = 0; i < T.sbits.size(); ++i)
    if (T.sbits[i] == q) return int64_t(1) << (T.bits.size() + i);
  return 0;
}

// stride of slice-local bit j for operand T (chunk buffers: per-slice tensors are
// stored [slice][elems]; sliced leaves carry the slice bits in their storage)
int64_t slice_stride(const tn_plan_s* p, const Tensor& T, int j) {
  if (!T.per_slice) return 0;
  if (T.leaf) return bit_stride(T, p->slice_bits[j]);
  return T.elems << j;
}

void fill_enum(TileEnum& en, std::vector<std::pair<int64_t, std::pair<int, int>>> bitsv,
               const std::vector<std::pair<int64_t, std::pair<int, int>>>& tail = {}) {
  // bitsv: (stride, (row increment, col increment)); sorted by stride, then `tail` appended as is
  std::stable_sort(bitsv.begin(), bitsv.end(),
                   [](const auto& a, const auto& b) { return a.first < b.first; });
  bitsv.insert(bitsv.end(), tail.begin(), tail.end());
  memset(&en, 0, sizeof(en));
  en.n = (int)bitsv.size();
  for (size_t j = 0; j < bitsv.size(); ++j) {
    en.stride[j] = bitsv[j].first;
    en.row[j] = bitsv[j].second.first;
    en.col[j] = bitsv[j].second.second;
  }
}

int contig_run(const TileEnum& en) {
  int r = 0;
  for (int j = 0; j < en.n; ++j) {
    if (en.stride[j] == (int64_t(1) << r)) ++r;
    else if (en.stride[j] == 0) continue;
    else break;
  }
  return r;
}

void build_desc(tn_plan_s* p, Step& st) {
  GettDesc& d = st.desc;
  memset(&d, 0, sizeof(d));
  const Tensor& A = p->tensors[st.ta];
  const Tensor& B = p->tensors[st.tb];
  const Tensor& C = p->tensors[st.tc];
  const int own = (int)st.bb.size();
  const int sb = st.per_slice ? p->s_bits : 0;
  d.own_bb = own;
  d.nbb = own + sb;
  d.mb = (int)st.mb.size();
  d.nb = (int)st.nb.size();
  d.kb = (int)st.kb.size();
  d.c_nbits = (int)C.bits.size();
  d.c_elems = C.elems;
  for (int j = 0; j < own; ++j) {
    d.a_b[j] = bit_stride(A, st.bb[j]);
    d.b_b[j] = bit_stride(B, st.bb[j]);
    d.c_b[j] = bit_stride(C, st.bb[j]);
  }
  for (int j = 0; j < sb; ++j) {
    d.a_b[own + j] = slice_stride(p, A, j);
    d.b_b[own + j] = slice_stride(p, B, j);
    d.c_b[own + j] = slice_stride(p, C, j);
  }
  for (int j = 0; j < d.mb; ++j) {
    d.a_m[j] = bit_stride(A, st.mb[j]);
    d.c_m[j] = bit_stride(C, st.mb[j]);
  }
  for (int j = 0; j < d.nb; ++j) {
    d.b_n[j] = bit_stride(B, st.nb[j]);
    d.c_n[j] = bit_stride(C, st.nb[j]);
  }
  for (int j = 0; j < d.kb; ++j) {
    d.a_k[j] = bit_stride(A, st.kb[j]);
    d.b_k[j] = bit_stride(B, st.kb[j]);
  }
  {
    const int k0 = std::min(d.kb, 4);   // bits inside one K stage of the MFMA kernels
    int64_t sa = 0, sb = 0;
    for (int t = 0; k0 + t < d.kb; ++t) {
      d.a_kd[t] = d.a_k[k0 + t] - sa;
      d.b_kd[t] = d.b_k[k0 + t] - sb;
      sa += d.a_k[k0 + t];
      sb += d.b_k[k0 + t];
    }
    d.a_kstep = k0 < d.kb ? d.a_k[k0] : 0;
    d.b_kstep = k0 < d.kb ? d.b_k[k0] : 0;
    d.k_linear = 1;
    for (int t = 0; k0 + t < d.kb; ++t)
      if (d.a_k[k0 + t] != (d.a_kstep << t) || d.b_k[k0 + t] != (d.b_kstep << t)) d.k_linear = 0;
  }
  for (size_t pos = 0; pos < C.bits.size(); ++pos) {
    const int q = C.bits[pos];
    int code = -1;
    for (int j = 0; j < own; ++j)
      if (st.bb[j] == q) code = (0 << 8) | j;
    for (int j = 0; j < d.mb; ++j)
      if (st.mb[j] == q) code = (1 << 8) | j;
    for (int j = 0; j < d.nb; ++j)
      if (st.nb[j] == q) code = (2 << 8) | j;
    d.c_pos[pos] = code;
  }
  for (int j = 0; j < sb; ++j) d.c_pos[C.bits.size() + j] = (0 << 8) | (own + j);
  // the global -> LDS copy path: both operands stored split, quads of consecutive k
  // adjacent in memory (one hi quad, one lo quad), whole 16-k stages, the 256x128 tile
  // id; full 256 x 128 tiles, or 512 x 64 / 512 x 32 tiles for steps with exactly 64 / 32
  // columns (which would leave half or three quarters of a 256 x 128 tile empty)
  const bool copy_path = (st.kernel == TN_K_MFMA_F16X3 || st.kernel == TN_K_MFMA_BF16X3) &&
                         st.tile == TN_TILE_256x128 && A.fmt == TN_FMT_SPLIT && B.fmt == TN_FMT_SPLIT &&
                         d.kb >= 4 && st.k_split_bits >= 4 && st.k_split_bits - 4 <= 30 && d.a_k[0] == 1 && d.a_k[1] == 2 && d.b_k[0] == 1 &&
                         d.b_k[1] == 2;
  st.dma = !copy_path ? 0
           : (d.mb >= 8 && d.nb >= 7) ? 1
           : (d.mb >= 9 && d.nb == 6) ? 2
           : (d.mb >= 9 && d.nb == 5) ? 3
                                      : 0;
  // tile enumerations for the MFMA kernels (the step's tile shape)
  int bm = 128, bn = 128, nt = 256;
  tn_tile_shape(st.tile, &bm, &bn, &nt);
  if (st.dma >= 2) {
    bm = 512;
    bn = st.dma == 2 ? 64 : 32;
  }
  const int lm = std::min(d.mb, ilog2_exact(bm)), ln = std::min(d.nb, ilog2_exact(bn)), lk = std::min(d.kb, 4);
  st.tiles_m_bits = d.mb - lm;
  st.tiles_n_bits = d.nb - ln;
  std::vector<std::pair<int64_t, std::pair<int, int>>> va, vb, vc, vpass;
  for (int j = 0; j < lm; ++j) va.push_back({d.a_m[j], {1 << j, 0}});
  for (int j = 0; j < lk; ++j) va.push_back({d.a_k[j], {0, 1 << j}});
  for (int j = 0; j < ln; ++j) vb.push_back({d.b_n[j], {1 << j, 0}});
  for (int j = 0; j < lk; ++j) vb.push_back({d.b_k[j], {0, 1 << j}});
  // the epilogue stages 64 rows at a time: local m bits >= 6 go last
  for (int j = 0; j < lm; ++j) (j < 6 ? vc : vpass).push_back({d.c_m[j], {1 << j, 0}});
  for (int j = 0; j < ln; ++j) vc.push_back({d.c_n[j], {0, 1 << j}});
  fill_enum(d.ea, va);
  fill_enum(d.eb, vb);
  fill_enum(d.ec, vc, vpass);
  st.a_contig = contig_run(d.ea);
  st.b_contig = contig_run(d.eb);
}

// Tile shape and K split of an MFMA step.
void set_tile(const tn_plan_s* p, Step& st, int tile) {
  const int bbits = (int)st.bb.size() + (st.per_slice ? p->s_bits : 0);
  const int mb = (int)st.mb.size(), nb = (int)st.nb.size(), kb = (int)st.kb.size();
  int bm, bn, nt;
  tn_tile_shape(tile, &bm, &bn, &nt);
  st.tile = tile;
  const int lm = std::min(mb, ilog2_exact(bm)), ln = std::min(nb, ilog2_exact(bn)), lk = std::min(kb, 4);
  st.tiles_m_bits = mb - lm;
  st.tiles_n_bits = nb - ln;
  const int tile_bits = st.tiles_m_bits + st.tiles_n_bits + bbits;
  int s = 0;
  // split K when the grid is small and K long: aim for >= 1024 blocks, >= 8 K stages per split
  while (tile_bits + s < 10 && kb - (s + 1) >= lk + 3) ++s;
  st.splits = 1 << s;
  st.k_split_bits = kb - s;
  st.scratch_elems = st.splits > 1 ? (int64_t(st.splits) << (bbits + mb + nb)) : 0;
}

// Tile id from the step's m and n bits (the shape heuristic).
int heuristic_tile(int mb, int nb) {
  if (nb >= 7 && mb >= 8) return TN_TILE_256x128;
  if (nb >= 7 && mb >= 7) return TN_TILE_128x128;
  if (mb >= 7) return TN_TILE_128x64;
  return TN_TILE_64x64;
}

// split_policy 2: every step runs split products on the MFMA kernels, except steps that
// read an intermediate of fewer than 4 elements (the split storage is blocked by 4)
bool forced_split(const tn_plan_s* p, const Step& st) {
  if (p->precision == TN_PREC_C64 || p->opts.split_policy != 2 || p->tensors.empty()) return false;
  for (int x : {st.ta, st.tb}) {
    const Tensor& T = p->tensors[x];
    if (!T.leaf && T.elems < 4) return false;
  }
  return true;
}

void choose_kernel(tn_plan_s* p, Step& st) {
  const int bbits = (int)st.bb.size() + (st.per_slice ? p->s_bits : 0);
  const int mb = (int)st.mb.size(), nb = (int)st.nb.size(), kb = (int)st.kb.size();
  if (forced_split(p, st)) {
    st.kernel = p->precision == TN_PREC_F16X3 ? TN_K_MFMA_F16X3 : TN_K_MFMA_BF16X3;
    st.dot = false;
    set_tile(p, st, heuristic_tile(mb, nb));
    return;
  }
  const bool small = (kb <= 6 && bbits + mb + nb <= 14) || (bbits + mb + nb + kb <= 16);
  // batched dot products (at most 4 output elements per batch, K >= 2^10): an MFMA tile
  // would be almost empty; one block per output element splits K instead
  const bool dot = mb + nb <= 2 && kb >= 10;
  if (small || dot) {
    st.kernel = TN_K_SMALL;
    st.dot = dot;
    st.splits = 1;
    return;
  }
  bool split_prec = false;
  if (p->precision != TN_PREC_C64) {
    if (p->opts.split_policy == 1) split_prec = kb >= 3;
    else split_prec = kb >= 4 && mb >= 5 && nb >= 4;
  }
  st.kernel = split_prec ? (p->precision == TN_PREC_F16X3 ? TN_K_MFMA_F16X3 : TN_K_MFMA_BF16X3)
                         : TN_K_MFMA_F32;
  set_tile(p, st, heuristic_tile(mb, nb));
}

// Offset (elements) in tensor T of the open bonds' values for bitstring key `key`:
// raw open labels contribute their bit's stride when the key's bit is set; a merged
// bond contributes the strides of the bits of its value, the index of the key's
// restriction to T's measured qubits among T's keys.
int64_t open_offset(const tn_plan_s* p, const Tensor& T, uint64_t key) {
  int64_t off = 0;
  if (T.merged >= 0) {
    const uint64_t r = key & T.sq;
    const auto it = std::lower_bound(T.key_value.begin(), T.key_value.end(), std::make_pair(r, int64_t(0)));
    const int64_t v = (it != T.key_value.end() && it->first == r) ? it->second : 0;   // always found
    const Label& L = p->labels[T.merged];
    for (int b = 0; b < L.nb; ++b)
      if ((v >> b) & 1) off += bit_stride(T, L.bit0 + b);
    return off;
  }
  for (int l : T.labels) {
    const Label& L = p->labels[l];
    if (L.qubit >= 0 && ((key >> L.qubit) & 1)) off += bit_stride(T, L.bit0);
  }
  return off;
}

// Tables of a sparse-einsum step: for each value f of the result's merged bond (padding
// values repeat f = 0), the offsets in A and B of the restrictions of keys[f].
void build_tables(tn_plan_s* p, Step& st) {
  const Tensor& A = p->tensors[st.ta];
  const Tensor& B = p->tensors[st.tb];
  const Tensor& C = p->tensors[st.tc];
  const int64_t ext = p->labels[st.tab_label].ext;
  st.tab_a.assign(ext, 0);
  st.tab_b.assign(ext, 0);
  for (size_t f = 0; f < C.keys.size(); ++f) {
    st.tab_a[f] = open_offset(p, A, C.keys[f]);
    st.tab_b[f] = open_offset(p, B, C.keys[f]);
  }
  for (int64_t f = (int64_t)C.keys.size(); f < ext; ++f) {
    st.tab_a[f] = st.tab_a[0];
    st.tab_b[f] = st.tab_b[0];
  }
  st.tab_a_max = *std::max_element(st.tab_a.begin(), st.tab_a.end());
  st.tab_b_max = *std::max_element(st.tab_b.begin(), st.tab_b.end());
  // Values are ordered by their restriction to A's qubits first, so runs of consecutive
  // values read the same slice of A.  Where those runs average 4 values or more, the MFMA
  // kernels take the values as the fastest part of the block index: the blocks resident
  // together then share each A tile through L2 (instead of every value streaming A again)
  // and read one B slice per value.
  int64_t changes = 0;
  for (size_t f = 1; f < C.keys.size(); ++f) changes += st.tab_a[f] != st.tab_a[f - 1] ? 1 : 0;
  st.values_first = C.keys.size() >= 64 && changes * 4 < (int64_t)C.keys.size() ? 1 : 0;
}

// Every address a kernel forms is a sum of per-bit strides.  Check, for every
// step and operand, that the largest reachable offset stays inside its buffer
// and that no two bits share a non-zero stride.
tn_status validate_steps(const tn_plan_s* p, const std::vector<Step>& steps) {
  const int64_t S = int64_t(1) << p->s_bits;
  for (size_t s = 0; s < steps.size(); ++s) {
    const Step& st = steps[s];
    const GettDesc& d = st.desc;
    struct Op {
      const Tensor* T;
      const int64_t* b;
      const int64_t* r;
      int nr;
      const int64_t* k;
      int nk;
    } ops[3] = {{&p->tensors[st.ta], d.a_b, d.a_m, d.mb, d.a_k, d.kb},
                {&p->tensors[st.tb], d.b_b, d.b_n, d.nb, d.b_k, d.kb},
                {&p->tensors[st.tc], d.c_b, d.c_m, d.mb, d.c_n, d.nb}};
    for (int o = 0; o < 3; ++o) {
      const Tensor& T = *ops[o].T;
      std::vector<int64_t> strides;
      for (int j = 0; j < d.nbb; ++j) strides.push_back(ops[o].b[j]);
      for (int j = 0; j < ops[o].nr; ++j) strides.push_back(ops[o].r[j]);
      for (int j = 0; j < ops[o].nk; ++j) strides.push_back(ops[o].k[j]);
      int64_t cap = T.leaf ? (T.elems << T.sbits.size()) : (T.per_slice ? T.elems * S : T.elems);
      int64_t mx = o == 0 ? st.tab_a_max : o == 1 ? st.tab_b_max : 0;   // sparse-einsum table offsets
      if (T.leaf && T.per_slice)  // slice bits above the chunk are a base offset
        for (int j = (st.per_slice ? p->s_bits : 0); j < p->n_slice_bits; ++j) mx += bit_stride(T, p->slice_bits[j]);
      std::set<int64_t> seen;
      for (int64_t v : strides) {
        if (v < 0 || (v & (v - 1)) != 0)
          return fail(TN_E_STATE, "internal: step " + std::to_string(s) + " has a stride that is not a power of two");
        if (v > 0 && !seen.insert(v).second)
          return fail(TN_E_STATE, "internal: step " + std::to_string(s) + " has aliased operand bits");
        mx += v;
      }
      if (mx >= cap)
        return fail(TN_E_STATE, "internal: step " + std::to_string(s) + " operand " + std::to_string(o) +
                                    " reaches offset " + std::to_string(mx) + " of " + std::to_string(cap));
      if (st.kernel != TN_K_SMALL && o < 2) {
        // the MFMA kernels keep operand-tile offsets (m or n bits plus k bits) in 32 bits
        int64_t tile_span = 0;
        for (int j = 0; j < ops[o].nr; ++j) tile_span += ops[o].r[j];
        for (int j = 0; j < ops[o].nk; ++j) tile_span += ops[o].k[j];
        if (tile_span > INT32_MAX)
          return fail(TN_E_UNSUPPORTED, "step " + std::to_string(s) + ": an operand spans more than 2^31 elements "
                                        "across its free and summed bits");
      }
    }
    if (st.kernel != TN_K_SMALL && st.splits > 1) {
      const int64_t need = int64_t(st.splits) << (d.nbb + d.mb + d.nb);
      if (need > st.scratch_elems || (!p->host_only && need > p->scratch_elems))
        return fail(TN_E_STATE, "internal: split-K scratch too small");
    }
  }
  return TN_OK;
}

tn_status validate_bounds(const tn_plan_s* p) { return validate_steps(p, p->steps); }

tn_status check(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(TN_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return TN_OK;
}

// device permutation of a bit-indexed tensor: in_pos[q], out_pos[q] are storage positions
tn_status permute_bits(const std::vector<int>& in_pos, const std::vector<int>& out_pos, const void* in,
                       void* out, hipStream_t s, PermDesc* d_desc_scratch) {
  const int n = (int)in_pos.size();
  PermDesc pd;
  memset(&pd, 0, sizeof(pd));
  // local bits: lowest input positions U lowest output positions
  std::vector<int> local;
  const int want = std::min(n, 6);
  for (int q = 0; q < n; ++q)
    if (in_pos[q] < want || out_pos[q] < want) local.push_back(q);
  while ((int)local.size() < std::min(n, PERM_LOCAL_MAX)) {
    // widen with the next lowest output positions
    int best = -1;
    for (int q = 0; q < n; ++q)
      if (std::find(local.begin(), local.end(), q) == local.end() && (best < 0 || out_pos[q] < out_pos[best])) best = q;
    if (best < 0) break;
    local.push_back(best);
  }
  // LDS position r holds the local bit of the r-th lowest input position, so a load
  // of two elements along input stride 1 fills two adjacent positions.  Positions
  // 5 and up also flip some of bits 1..4 (an XOR swizzle that keeps position pairs
  // together): output-order reads of a transpose then spread over the LDS banks
  // (at most 2-way conflicts for 2-D transposes and random bit permutations of
  // 28 bits, by enumeration of the access pattern, against 32-way unswizzled).
  std::sort(local.begin(), local.end(), [&](int a, int b) { return in_pos[a] < in_pos[b]; });
  static const int kSwizzle[PERM_LOCAL_MAX - 5] = {28, 30, 4, 26, 24, 18, 14};
  std::vector<std::pair<int64_t, std::pair<int, int>>> vi, vo;
  for (size_t r = 0; r < local.size(); ++r) {
    const int row = (1 << r) ^ (r >= 5 ? kSwizzle[r - 5] : 0);
    vi.push_back({int64_t(1) << in_pos[local[r]], {row, 0}});
    vo.push_back({int64_t(1) << out_pos[local[r]], {row, 0}});
  }
  fill_enum(pd.ein, vi);
  fill_enum(pd.eout, vo);
  int h = 0;
  for (int q = 0; q < n; ++q) {
    if (std::find(local.begin(), local.end(), q) != local.end()) continue;
    pd.h_in[h] = int64_t(1) << in_pos[q];
    pd.h_out[h] = int64_t(1) << out_pos[q];
    ++h;
  }
  pd.nh = h;
  // 16-byte accesses need aligned buffers (the lowest input and output bits are local)
  const int pairs = n >= 1 && ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
  const int first = 8 + pairs;   // enumeration bits below: the pair bit and the thread bits
  const int nl = pd.ein.n;
  pd.iters = nl > first ? 1 << (nl - first) : 1;
  for (int it = 0; it < pd.iters; ++it)
    for (int j = first; j < nl; ++j)
      if ((it >> (j - first)) & 1) {
        pd.it_in_off[it] += pd.ein.stride[j];
        pd.it_in_row[it] ^= pd.ein.row[j];
        pd.it_out_off[it] += pd.eout.stride[j];
        pd.it_out_row[it] ^= pd.eout.row[j];
      }
  tn_status st = check(hipMemcpyAsync(d_desc_scratch, &pd, sizeof(pd), hipMemcpyHostToDevice, s), "permute desc");
  if (st) return st;
  st = check(tn_launch_permute(d_desc_scratch, pairs, int64_t(1) << h, in, out, s), "permute launch");
  if (st) return st;
  return check(hipStreamSynchronize(s), "permute sync");
}

tn_status autotune(tn_plan_s* p);

tn_status plan_build(tn_plan_s* p, int32_t n_tensors, const int32_t* ranks, const int32_t* const* labels,
                     const int64_t* const* extents, const double* const* data, int32_t n_open,
                     const int32_t* open_labels, int32_t n_steps, const int32_t* path, int32_t n_sliced,
                     const int32_t* sliced_labels) {
  if (n_tensors < 1) return fail(TN_E_ARG, "n_tensors must be >= 1");
  if (!ranks || (!labels && n_tensors > 0) || !extents) return fail(TN_E_ARG, "null ranks/labels/extents");
  if (n_open < 0 || (n_open > 0 && !open_labels)) return fail(TN_E_ARG, "bad open labels");
  if (n_sliced < 0 || (n_sliced > 0 && !sliced_labels)) return fail(TN_E_ARG, "bad sliced labels");
  if (n_steps < 0 || (n_steps > 0 && !path)) return fail(TN_E_ARG, "bad path");
  if (!p->host_only && !data) return fail(TN_E_ARG, "null data");
  std::map<int, int> dense;
  // labels
  for (int t = 0; t < n_tensors; ++t) {
    if (ranks[t] < 0 || ranks[t] > 64) return fail(TN_E_ARG, "rank out of range");
    if (ranks[t] > 0 && (!labels[t] || !extents[t])) return fail(TN_E_ARG, "null labels/extents of a tensor");
    std::set<int> seen;
    for (int r = 0; r < ranks[t]; ++r) {
      const int l = labels[t][r];
      const int64_t e = extents[t][r];
      if (l < 0) return fail(TN_E_LABEL, "negative label id");
      if (!seen.insert(l).second) return fail(TN_E_LABEL, "label repeated within one tensor");
      if (e < 1) return fail(TN_E_LABEL, "extent must be >= 1");
      auto it = dense.find(l);
      if (it == dense.end()) {
        Label L;
        L.ext = e;
        L.user = l;
        L.nb = ilog2_exact(e);
        if (L.nb < 0) return fail(TN_E_UNSUPPORTED, "extent " + std::to_string(e) + " is not a power of two");
        dense[l] = (int)p->labels.size();
        p->labels.push_back(L);
      } else if (p->labels[it->second].ext != e) {
        return fail(TN_E_LABEL, "label " + std::to_string(l) + " has inconsistent extents");
      }
    }
  }
  std::vector<int> open_d;
  for (int i = 0; i < n_open; ++i) {
    auto it = dense.find(open_labels[i]);
    if (it == dense.end()) return fail(TN_E_LABEL, "open label " + std::to_string(open_labels[i]) + " is on no tensor");
    if (p->labels[it->second].open) return fail(TN_E_LABEL, "open label repeated");
    p->labels[it->second].open = true;
    open_d.push_back(it->second);
  }
  if (p->sparse) {
    if (n_open > 64) return fail(TN_E_UNSUPPORTED, "a sparse state measures at most 64 open labels");
    for (int i = 0; i < n_open; ++i) {
      Label& L = p->labels[open_d[i]];
      if (L.ext != 2) return fail(TN_E_UNSUPPORTED, "open labels of a sparse state must have extent 2");
      L.qubit = i;
      int on = 0;
      for (int t = 0; t < n_tensors; ++t)
        for (int r = 0; r < ranks[t]; ++r) on += labels[t][r] == open_labels[i] ? 1 : 0;
      if (on != 1) return fail(TN_E_UNSUPPORTED, "an open label of a sparse state must be on exactly one tensor");
    }
  }
  std::vector<int> sliced_d;
  for (int i = 0; i < n_sliced; ++i) {
    auto it = dense.find(sliced_labels[i]);
    if (it == dense.end()) return fail(TN_E_SLICE, "sliced label is on no tensor");
    Label& L = p->labels[it->second];
    if (L.open) return fail(TN_E_SLICE, "a sliced label may not be open");
    if (L.slice_pos >= 0) return fail(TN_E_SLICE, "sliced label repeated");
    L.slice_pos = i;
    sliced_d.push_back(it->second);
  }
  // bits
  p->n_bits = 0;
  for (auto& L : p->labels) {
    L.bit0 = p->n_bits;
    p->n_bits += L.nb;
  }
  // slice id bits, LSB first: last sliced label least significant
  for (int i = n_sliced - 1; i >= 0; --i) {
    const Label& L = p->labels[sliced_d[i]];
    for (int b = 0; b < L.nb; ++b) p->slice_bits.push_back(L.bit0 + b);
  }
  p->n_slice_bits = (int)p->slice_bits.size();
  if (p->n_slice_bits > 40) return fail(TN_E_UNSUPPORTED, "too many slice bits");
  p->n_slices = int64_t(1) << p->n_slice_bits;
  int amp_bits = 0;
  for (int l : open_d) amp_bits += p->labels[l].nb;
  if (!p->sparse && amp_bits > 30) return fail(TN_E_UNSUPPORTED, "too many output bits");
  if (!p->sparse) p->n_amp = int64_t(1) << amp_bits;

  // leaves (plus a unit scalar when the network is a single tensor)
  const bool single = n_tensors == 1;
  if (single) {
    if (n_steps != 0) return fail(TN_E_PATH, "a single tensor takes an empty path");
  } else if (n_steps != n_tensors - 1) {
    return fail(TN_E_PATH, "path must have n_tensors - 1 steps");
  }
  p->n_leaves = n_tensors + (single ? 1 : 0);
  for (int t = 0; t < n_tensors; ++t) {
    Tensor T;
    T.leaf = true;
    for (int r = ranks[t] - 1; r >= 0; --r) {
      const Label& L = p->labels[dense[labels[t][r]]];
      for (int b = 0; b < L.nb; ++b) T.user_layout.push_back(L.bit0 + b);
    }
    for (int r = 0; r < ranks[t]; ++r) {
      const int l = dense[labels[t][r]];
      if (p->labels[l].slice_pos >= 0) {
        if (p->labels[l].nb > 0) T.per_slice = true;
      } else {
        T.labels.push_back(l);
      }
      if (p->labels[l].qubit >= 0) T.sq |= uint64_t(1) << p->labels[l].qubit;
    }
    p->tensors.push_back(T);
  }
  if (single) {
    Tensor U;
    U.leaf = true;
    p->tensors.push_back(U);
  }
  // replay the path
  std::vector<int> slot(p->n_leaves);
  for (int i = 0; i < p->n_leaves; ++i) slot[i] = i;
  std::vector<int> count(p->labels.size(), 0);
  for (auto& T : p->tensors)
    for (int l : T.labels) count[l]++;
  std::vector<std::pair<int, int>> pairs;
  if (single) pairs.push_back({0, 1});
  for (int s = 0; s < n_steps; ++s) pairs.push_back({path[2 * s], path[2 * s + 1]});
  for (size_t s = 0; s < pairs.size(); ++s) {
    const int i = pairs[s].first, j = pairs[s].second;
    if (i < 0 || j < 0 || i >= p->n_leaves || j >= p->n_leaves || i == j)
      return fail(TN_E_PATH, "path step " + std::to_string(s) + " has an invalid slot");
    if (slot[i] < 0 || slot[j] < 0) return fail(TN_E_PATH, "path step " + std::to_string(s) + " uses a dead slot");
    Step st;
    st.slot_a = i;
    st.slot_b = j;
    st.ta = slot[i];
    st.tb = slot[j];
    const Tensor& A = p->tensors[st.ta];
    const Tensor& B = p->tensors[st.tb];
    for (int l : A.labels) count[l]--;
    for (int l : B.labels) count[l]--;
    std::set<int> sa(A.labels.begin(), A.labels.end()), sbs(B.labels.begin(), B.labels.end());
    std::set<int> all = sa;
    all.insert(sbs.begin(), sbs.end());
    Tensor C;
    // sparse einsum (Sec. 3.3): both operands hold open bonds of measured qubits; those
    // bonds are not classified but indexed through the step's tables
    const bool merge = p->sparse && A.sq != 0 && B.sq != 0;
    std::set<int> indexed;
    if (merge) {
      for (int l : A.labels)
        if (p->labels[l].open) st.ia_labels.push_back(l);
      for (int l : B.labels)
        if (p->labels[l].open) st.ib_labels.push_back(l);
      indexed.insert(st.ia_labels.begin(), st.ia_labels.end());
      indexed.insert(st.ib_labels.begin(), st.ib_labels.end());
    }
    for (int l : all) {
      if (indexed.count(l)) continue;
      const bool keep = p->labels[l].open || count[l] > 0;
      const bool ina = sa.count(l), inb = sbs.count(l);
      if (ina && inb) (keep ? st.lb : st.lk).push_back(l);
      else if (ina) (keep ? st.lm : st.lk).push_back(l);
      else (keep ? st.ln : st.lk).push_back(l);
      if (keep) C.labels.push_back(l);
    }
    if (merge) {
      // the merged bond: one value per distinct restriction of the bitstrings to the
      // union of the operands' measured qubits, padded to a power of two; values are
      // ordered by the restriction to A's qubits, then to B's, so that runs of consecutive
      // values read the same slice of A (the block order can then share it, build_tables)
      const uint64_t q = A.sq | B.sq;
      for (uint64_t k : p->bkeys) C.keys.push_back(k & q);
      std::sort(C.keys.begin(), C.keys.end());
      C.keys.erase(std::unique(C.keys.begin(), C.keys.end()), C.keys.end());
      const uint64_t qa = A.sq, qb = B.sq;
      std::sort(C.keys.begin(), C.keys.end(), [qa, qb](uint64_t x, uint64_t y) {
        return (x & qa) != (y & qa) ? (x & qa) < (y & qa) : (x & qb) < (y & qb);
      });
      for (size_t v = 0; v < C.keys.size(); ++v) C.key_value.push_back({C.keys[v], (int64_t)v});
      std::sort(C.key_value.begin(), C.key_value.end());
      Label L;
      while ((int64_t(1) << L.nb) < (int64_t)C.keys.size()) ++L.nb;
      L.ext = int64_t(1) << L.nb;
      L.open = true;
      L.merged = true;
      L.user = -1;
      L.bit0 = p->n_bits;
      p->n_bits += L.nb;
      const int ml = (int)p->labels.size();
      p->labels.push_back(L);
      count.push_back(0);
      st.lb.push_back(ml);
      C.labels.push_back(ml);
      st.tab_label = ml;
      C.sq = q;
      C.merged = ml;
    } else {
      const Tensor& O = A.sq != 0 ? A : B;
      C.sq = A.sq | B.sq;
      C.merged = O.merged;
      C.keys = O.keys;
      C.key_value = O.key_value;
    }
    for (int l : C.labels) count[l]++;
    C.per_slice = A.per_slice || B.per_slice;
    st.per_slice = C.per_slice;
    st.tc = (int)p->tensors.size();
    p->tensors.push_back(C);
    slot[i] = st.tc;
    slot[j] = -1;
    p->steps.push_back(st);
  }
  int live = 0;
  for (int i = 0; i < p->n_leaves; ++i)
    if (slot[i] >= 0) {
      ++live;
      p->root = slot[i];
    }
  if (live != 1) return fail(TN_E_PATH, "path does not reduce the network to one tensor");
  // sizes and cap
  for (auto& T : p->tensors) {
    int nb = 0;
    for (int l : T.labels) nb += p->labels[l].nb;
    if (nb > 36) return fail(TN_E_UNSUPPORTED, "tensor with more than 2^36 elements");
    T.elems = int64_t(1) << nb;
  }
  if (p->sparse) {
    if (p->tensors[p->root].elems > (int64_t(1) << 30)) return fail(TN_E_UNSUPPORTED, "too many output bits");
    p->n_amp = p->tensors[p->root].elems;
  }
  for (auto& st : p->steps) {
    p->max_intermediate = std::max(p->max_intermediate, p->tensors[st.tc].elems);
    if (p->opts.mem_cap_elems > 0 && p->tensors[st.tc].elems > p->opts.mem_cap_elems)
      return fail(TN_E_CAP, "intermediate of " + std::to_string(p->tensors[st.tc].elems) +
                                " elements exceeds the cap");
  }
  // layouts, root first
  {
    Tensor& R = p->tensors[p->root];
    R.bits.clear();
    if (p->sparse && R.merged >= 0) {
      const Label& L = p->labels[R.merged];
      for (int b = 0; b < L.nb; ++b) R.bits.push_back(L.bit0 + b);
    } else {
      const std::set<int> rl(R.labels.begin(), R.labels.end());
      for (int i = (int)open_d.size() - 1; i >= 0; --i) {
        if (p->sparse && !rl.count(open_d[i])) continue;
        const Label& L = p->labels[open_d[i]];
        for (int b = 0; b < L.nb; ++b) R.bits.push_back(L.bit0 + b);
      }
    }
    R.layout_set = true;
  }
  for (int s = (int)p->steps.size() - 1; s >= 0; --s) {
    Step& st = p->steps[s];
    const Tensor& C = p->tensors[st.tc];
    std::map<int, int> cpos;
    for (size_t i = 0; i < C.bits.size(); ++i) cpos[C.bits[i]] = (int)i;
    auto bits_of = [&](const std::vector<int>& ls) {
      std::vector<int> out;
      for (int l : ls)
        for (int b = 0; b < p->labels[l].nb; ++b) out.push_back(p->labels[l].bit0 + b);
      return out;
    };
    auto by_cpos = [&](std::vector<int> v) {
      std::sort(v.begin(), v.end(), [&](int a, int b) { return cpos.at(a) < cpos.at(b); });
      return v;
    };
    st.bb = by_cpos(bits_of(st.lb));
    if (st.tab_label >= 0) {   // the merged bond's bits are the lowest batch bits (table index)
      std::vector<int> tb = bits_of({st.tab_label}), rest;
      for (int q : st.bb)
        if (std::find(tb.begin(), tb.end(), q) == tb.end()) rest.push_back(q);
      st.bb = tb;
      st.bb.insert(st.bb.end(), rest.begin(), rest.end());
    }
    st.mb = by_cpos(bits_of(st.lm));
    st.nb = by_cpos(bits_of(st.ln));
    st.kb = bits_of(st.lk);
    std::sort(st.kb.begin(), st.kb.end());
    if ((int)st.bb.size() + p->s_bits > TN_MAXB - 8 || (int)st.mb.size() > TN_MAXR ||
        (int)st.nb.size() > TN_MAXR || (int)st.kb.size() > TN_MAXK)
      return fail(TN_E_UNSUPPORTED, "step has too many bits for the kernels");
    Tensor& A = p->tensors[st.ta];
    Tensor& B = p->tensors[st.tb];
    std::set<int> abits, bbits;
    for (int q : bits_of(A.labels)) abits.insert(q);
    for (int q : bits_of(B.labels)) bbits.insert(q);
    A.bits.clear();
    for (int q : st.kb)
      if (abits.count(q)) A.bits.push_back(q);
    for (int q : st.mb) A.bits.push_back(q);
    for (int q : st.bb)
      if (abits.count(q)) A.bits.push_back(q);
    for (int q : bits_of(st.ia_labels)) A.bits.push_back(q);   // open bonds the tables index
    B.bits.clear();
    for (int q : st.kb)
      if (bbits.count(q)) B.bits.push_back(q);
    for (int q : st.nb) B.bits.push_back(q);
    for (int q : st.bb)
      if (bbits.count(q)) B.bits.push_back(q);
    for (int q : bits_of(st.ib_labels)) B.bits.push_back(q);
    A.layout_set = B.layout_set = true;
  }
  // leaves: sliced bits on top, in slice-id order
  for (int t = 0; t < p->n_leaves; ++t) {
    Tensor& T = p->tensors[t];
    for (int q : p->slice_bits)
      if (std::find(T.user_layout.begin(), T.user_layout.end(), q) != T.user_layout.end()) T.sbits.push_back(q);
  }
  // slice chunk size: the caller's, else 8 slices, raised to 16 or 32 while the chunk's
  // per-slice arena stays within kAutoChunkBytes (larger chunks give the per-slice GEMMs more
  // batch; the per-slice arena grows linearly with the chunk, so its one-slice peak decides)
  int64_t want = p->opts.slice_batch > 0 ? p->opts.slice_batch : 8;
  if (p->opts.slice_batch > 0 && ilog2_exact(p->opts.slice_batch) < 0)
    return fail(TN_E_ARG, "slice_batch must be a power of two");
  if (p->opts.slice_batch <= 0 && p->n_slice_bits > 0) {
    constexpr double kAutoChunkBytes = 32.0 * (1ull << 30);
    Arena dry;
    std::map<int, int64_t> at;   // per-slice intermediates of the dry run -> offset
    for (const Step& st : p->steps) {
      if (!st.per_slice) continue;
      at[st.tc] = dry.alloc(p->tensors[st.tc].elems);
      for (int x : {st.ta, st.tb}) {
        auto it = at.find(x);
        if (it != at.end()) {
          dry.release(it->second, p->tensors[x].elems);
          at.erase(it);
        }
      }
    }
    const double per_slice = 8.0 * (double)dry.peak;
    while (want < 32 && 2.0 * (double)want * per_slice <= kAutoChunkBytes) want *= 2;
  }
  p->s_bits = 0;
  while ((int64_t(2) << p->s_bits) <= std::min<int64_t>(want, p->n_slices)) ++p->s_bits;
  if (p->n_slice_bits == 0) p->s_bits = 0;
  // kernels, descriptors and costs
  for (auto& st : p->steps) {
    choose_kernel(p, st);
    const Tensor& A = p->tensors[st.ta];
    const Tensor& B = p->tensors[st.tb];
    const Tensor& C = p->tensors[st.tc];
    int ub = (int)(st.bb.size() + st.mb.size() + st.nb.size() + st.kb.size());
    st.flops = 8.0 * std::ldexp(1.0, ub);
    st.bytes = 8.0 * ((double)A.elems + (double)B.elems + (double)C.elems);
    if (st.per_slice) {
      p->flops_ps += st.flops;
      p->bytes_ps += st.bytes;
    } else {
      p->flops_inv += st.flops;
      p->bytes_inv += st.bytes;
    }
  }
  // intermediates read by a split-precision MFMA step are stored split
  for (auto& st : p->steps) {
    if (st.kernel != TN_K_MFMA_F16X3 && st.kernel != TN_K_MFMA_BF16X3) continue;
    for (int x : {st.ta, st.tb})
      if (!p->tensors[x].leaf) p->tensors[x].fmt = TN_FMT_SPLIT;
  }
  for (const Tensor& T : p->tensors)   // the split format is blocked by 4 elements
    if (T.fmt == TN_FMT_SPLIT && (T.elems & 3) != 0)
      return fail(TN_E_STATE, "internal: a split-stored tensor has fewer than 4 elements");
  for (size_t s = 0; s < p->steps.size(); ++s)
    (p->steps[s].per_slice ? p->ps_order : p->inv_order).push_back((int)s);
  // memory: leaves, invariant arena, per-slice arena (S copies of each tensor)
  int64_t off = 0;
  for (int t = 0; t < p->n_leaves; ++t) {
    Tensor& T = p->tensors[t];
    T.arena = 0;
    T.offset = off;
    off += Arena::align(T.elems << T.sbits.size());
  }
  p->leaf_elems = std::max<int64_t>(off, 64);
  Arena inv, ps;
  for (int s : p->inv_order) {
    Step& st = p->steps[s];
    Tensor& C = p->tensors[st.tc];
    C.arena = 1;
    C.offset = inv.alloc(C.elems);
    for (int x : {st.ta, st.tb}) {
      Tensor& X = p->tensors[x];
      if (!X.leaf && X.arena == 1) inv.release(X.offset, X.elems);
    }
  }
  const int64_t S = int64_t(1) << p->s_bits;
  for (int s : p->ps_order) {
    Step& st = p->steps[s];
    Tensor& C = p->tensors[st.tc];
    C.arena = 2;
    C.offset = ps.alloc(C.elems * S);
    for (int x : {st.ta, st.tb}) {
      Tensor& X = p->tensors[x];
      if (!X.leaf && X.arena == 2) ps.release(X.offset, X.elems * S);
    }
  }
  p->inv_elems = std::max<int64_t>(inv.peak, 64);
  p->ps_elems = std::max<int64_t>(ps.peak, 64);
  if (p->sparse) {
    for (auto& st : p->steps)
      if (st.tab_label >= 0) {
        build_tables(p, st);
        p->tab_elems += 2 * p->labels[st.tab_label].ext;
      }
    const Tensor& R = p->tensors[p->root];
    for (uint64_t k : p->bkeys) p->amp_index.push_back(open_offset(p, R, k));
  }
  for (auto& st : p->steps) build_desc(p, st);
  p->S = (int)S;
  for (auto& st : p->steps) p->scratch_elems = std::max(p->scratch_elems, st.scratch_elems);
  if (tn_status vb = validate_bounds(p)) return vb;
  // a caller-owned workspace reserves split-K scratch for any tile a step may be given later
  int64_t scratch_any = p->scratch_elems;
  for (const Step& st0 : p->steps) {
    if (st0.kernel == TN_K_SMALL) continue;
    for (int tile = 0; tile < TN_N_TILES; ++tile) {
      Step c = st0;
      set_tile(p, c, tile);
      scratch_any = std::max(scratch_any, c.scratch_elems);
    }
  }
  const size_t nt = p->tensors.size();
  int64_t max_leaf = 1;
  for (int t = 0; t < p->n_leaves; ++t) max_leaf = std::max(max_leaf, p->tensors[t].elems << p->tensors[t].sbits.size());
  const size_t dev_bytes[] = {(size_t)p->leaf_elems * 8, (size_t)p->inv_elems * 8, (size_t)p->ps_elems * 8,
                              sizeof(GettDesc) * std::max<size_t>(p->steps.size(), 1) + sizeof(PermDesc),
                              nt * 4, nt * S * 4, nt * 4, nt * S * 4, (size_t)p->n_amp * 16,
                              (size_t)p->n_amp * 16 * S, 64, (size_t)scratch_any * 8, (size_t)max_leaf * 8,
                              (size_t)p->tab_elems * 8};
  p->ws_need = 0;
  for (size_t b : dev_bytes) p->ws_need += (int64_t)((b + 255) & ~size_t(255));
  if (p->host_only) return TN_OK;

  // ---- device setup ----
  hipStream_t s = p->stream;
  if (p->opts.workspace) {
    if (p->opts.workspace_bytes < p->ws_need)
      return fail(TN_E_NOMEM, "workspace of " + std::to_string(p->opts.workspace_bytes) + " bytes is too small: the plan needs " +
                                  std::to_string(p->ws_need));
    p->own_memory = false;
    p->ws = reinterpret_cast<char*>(p->opts.workspace);
    p->ws_size = (size_t)p->opts.workspace_bytes;
    if ((reinterpret_cast<uintptr_t>(p->ws) & 255) != 0) return fail(TN_E_ARG, "workspace must be 256-byte aligned");
    p->scratch_elems = scratch_any;
  }
  auto dmalloc = [&](void** ptr, size_t bytes) -> tn_status {
    if (!p->own_memory) {
      const size_t b = (bytes + 255) & ~size_t(255);
      if (p->ws_used + b > p->ws_size) return fail(TN_E_NOMEM, "workspace too small");
      *ptr = p->ws + p->ws_used;
      p->ws_used += b;
      p->device_bytes += b;
      return TN_OK;
    }
    if (hipMalloc(ptr, bytes) != hipSuccess) {
      hipGetLastError();
      return fail(TN_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    p->device_bytes += bytes;
    return TN_OK;
  };
  auto dfree = [&](void* ptr) {
    if (p->own_memory) hipFree(ptr);
  };
  tn_status st;
  if ((st = dmalloc((void**)&p->d_leaves, p->leaf_elems * 8))) return st;
  if ((st = dmalloc((void**)&p->d_inv, p->inv_elems * 8))) return st;
  if ((st = dmalloc((void**)&p->d_ps, p->ps_elems * 8))) return st;
  if ((st = dmalloc((void**)&p->d_desc, sizeof(GettDesc) * std::max<size_t>(p->steps.size(), 1) + sizeof(PermDesc)))) return st;
  if ((st = dmalloc((void**)&p->d_max_inv, nt * 4))) return st;
  if ((st = dmalloc((void**)&p->d_max_ps, nt * S * 4))) return st;
  if ((st = dmalloc((void**)&p->d_exp_inv, nt * 4))) return st;
  if ((st = dmalloc((void**)&p->d_exp_ps, nt * S * 4))) return st;
  if ((st = dmalloc((void**)&p->d_acc, p->n_amp * 16))) return st;
  if ((st = dmalloc((void**)&p->d_part, p->n_amp * 16 * S))) return st;
  if ((st = dmalloc((void**)&p->d_flag, 64))) return st;
  if (p->scratch_elems > 0 && (st = dmalloc((void**)&p->d_scratch, p->scratch_elems * 8))) return st;
  if (p->tab_elems > 0) {
    if ((st = dmalloc((void**)&p->d_tabs, p->tab_elems * 8))) return st;
    std::vector<int64_t> all;
    for (auto& stp : p->steps)
      if (stp.tab_label >= 0) {
        stp.d_tab_a = p->d_tabs + all.size();
        all.insert(all.end(), stp.tab_a.begin(), stp.tab_a.end());
        stp.d_tab_b = p->d_tabs + all.size();
        all.insert(all.end(), stp.tab_b.begin(), stp.tab_b.end());
      }
    if ((st = check(hipMemcpyAsync(p->d_tabs, all.data(), all.size() * 8, hipMemcpyHostToDevice, s), "table upload")))
      return st;
    if ((st = check(hipStreamSynchronize(s), "table upload sync"))) return st;
  }
  if ((st = check(hipMemsetAsync(p->d_acc, 0, p->n_amp * 16, s), "memset acc"))) return st;
  if ((st = check(hipMemsetAsync(p->d_flag, 0, 64, s), "memset flag"))) return st;
  if ((st = check(hipMemsetAsync(p->d_max_inv, 0, nt * 4, s), "memset max"))) return st;
  if ((st = check(hipMemsetAsync(p->d_exp_inv, 0, nt * 4, s), "memset exp"))) return st;
  if ((st = check(hipMemsetAsync(p->d_exp_ps, 0, nt * S * 4, s), "memset exp"))) return st;
  std::vector<GettDesc> descs(p->steps.size());
  for (size_t i = 0; i < p->steps.size(); ++i) descs[i] = p->steps[i].desc;
  if (!descs.empty() &&
      (st = check(hipMemcpyAsync(p->d_desc, descs.data(), sizeof(GettDesc) * descs.size(), hipMemcpyHostToDevice, s),
                  "desc upload")))
    return st;
  PermDesc* d_perm = reinterpret_cast<PermDesc*>(p->d_desc + std::max<size_t>(p->steps.size(), 1));
  // leaves: upload complex128 -> complex64 staging, then permute on the device
  float* d_stage = nullptr;
  if ((st = dmalloc((void**)&d_stage, max_leaf * 8))) return st;
  std::vector<float> host;
  for (int t = 0; t < p->n_leaves; ++t) {
    Tensor& T = p->tensors[t];
    const int64_t n = T.elems << T.sbits.size();
    host.assign(2 * n, 0.f);
    if (t < n_tensors) {
      if (!data[t]) {
        dfree(d_stage);
        return fail(TN_E_ARG, "null data for a tensor");
      }
      for (int64_t i = 0; i < 2 * n; ++i) host[i] = (float)data[t][i];
    } else {
      host[0] = 1.f;  // unit scalar
    }
    st = check(hipMemcpyAsync(d_stage, host.data(), n * 8, hipMemcpyHostToDevice, s), "leaf upload");
    if (!st) st = check(hipStreamSynchronize(s), "leaf upload sync");
    if (st) {
      dfree(d_stage);
      return st;
    }
    // user layout -> planned layout (bits then sliced bits)
    std::vector<int> full = T.bits;
    full.insert(full.end(), T.sbits.begin(), T.sbits.end());
    if (full.size() != T.user_layout.size()) {
      dfree(d_stage);
      return fail(TN_E_STATE, "internal: leaf layout size mismatch");
    }
    std::vector<int> in_pos(full.size()), out_pos(full.size());
    for (size_t q = 0; q < full.size(); ++q) {
      out_pos[q] = (int)q;
      in_pos[q] = (int)(std::find(T.user_layout.begin(), T.user_layout.end(), full[q]) - T.user_layout.begin());
    }
    float* dst = p->d_leaves + 2 * T.offset;
    if (full.empty()) {
      st = check(hipMemcpyAsync(dst, d_stage, 8, hipMemcpyDeviceToDevice, s), "scalar leaf");
    } else {
      st = permute_bits(in_pos, out_pos, d_stage, dst, s, d_perm);
    }
    if (st) {
      dfree(d_stage);
      return st;
    }
    if (scaled(p)) {
      st = check(tn_launch_absmax(dst, n, p->d_max_inv + t, s), "leaf max");
      if (st) {
        dfree(d_stage);
        return st;
      }
    }
  }
  st = check(hipStreamSynchronize(s), "setup sync");
  dfree(d_stage);
  if (p->own_memory) p->device_bytes -= max_leaf * 8;
  if (st) return st;
  if (p->opts.tuning == 1) {
    // the arenas start zeroed; tuning then runs the steps in order (autotune)
    if ((st = check(hipMemsetAsync(p->d_inv, 0, p->inv_elems * 8, s), "arena clear"))) return st;
    if ((st = check(hipMemsetAsync(p->d_ps, 0, p->ps_elems * 8, s), "arena clear"))) return st;
    if ((st = check(hipMemsetAsync(p->d_max_ps, 0, nt * S * 4, s), "max clear"))) return st;
    st = autotune(p);
  }
  return st;
}

const float* tensor_ptr(const tn_plan_s* p, const Tensor& T) {
  if (T.arena == 0) return p->d_leaves + 2 * T.offset;
  if (T.arena == 1) return p->d_inv + 2 * T.offset;
  return p->d_ps + 2 * T.offset;
}

// chunk offset of a sliced leaf for the slice bits above the chunk
int64_t leaf_chunk_offset(const tn_plan_s* p, const Tensor& T, int64_t base, int chunk_bits) {
  int64_t off = 0;
  for (int j = chunk_bits; j < p->n_slice_bits; ++j)
    if ((base >> j) & 1) off += bit_stride(T, p->slice_bits[j]);
  return off;
}

// Main launch of step s, followed by its split-K reduction when `rg` is set; with
// record_steps both are bracketed by one pair of events (the step's time).
tn_status timed_launch(tn_plan_s* p, int s, int kind, const GettDesc* d, const GettArgs& g, int64_t blocks,
                       const char* what, const GettArgs* rg, int64_t rblocks) {
  const int tile = p->steps[s].tile;
  auto launch = [&]() -> tn_status {
    tn_status r = check(tn_launch_gett(kind, tile, d, g, blocks, p->stream), what);
    if (!r && rg) r = check(tn_launch_gett(TN_K_SPLITK_REDUCE, 0, d, *rg, rblocks, p->stream), "split-K reduce");
    return r;
  };
  if (!p->opts.record_steps) return launch();
  std::pair<hipEvent_t, hipEvent_t> ev;
  if (!p->event_pool.empty()) {
    ev = p->event_pool.back();
    p->event_pool.pop_back();
  } else {
    tn_status st = check(hipEventCreate(&ev.first), "event create");
    if (!st) st = check(hipEventCreate(&ev.second), "event create");
    if (st) return st;
  }
  tn_status st = check(hipEventRecord(ev.first, p->stream), "event record");
  if (!st) st = launch();
  if (!st) st = check(hipEventRecord(ev.second, p->stream), "event record");
  p->pending.push_back({s, ev.first, ev.second});
  return st;
}

// One launch-equivalent of the contraction: a kernel launch in the ordinary
// path, an instance of the persistent executor in a group.
struct Launch {
  int kind = TN_K_SMALL;
  int tile = 0;
  int step = -1;           // step index for a step's main launch (timed), else -1
  const GettDesc* desc = nullptr;
  GettArgs g{};
  ReduceArgs r{};
  uint32_t* fill_ptr = nullptr;
  int64_t fill_n = 0;
  int64_t elems = 0;       // element-wise kinds: elements covered
  int64_t blocks = 0;      // MFMA kinds: tile blocks
  int64_t nblocks(int threads) const {
    if (kind == TN_K_SMALL && g.dot) return elems;   // one block per output element
    return (kind == TN_K_MFMA_F32 || kind == TN_K_MFMA_F16X3 || kind == TN_K_MFMA_BF16X3)
               ? blocks
               : (elems + threads - 1) / threads;
  }
};

// Launches of step `st` (descriptor d) for one chunk: the main launch and, with
// split K, its reduction.
void step_launches(const tn_plan_s* p, const Step& st, const GettDesc* d, int s, int64_t chunk_base, int chunk_bits,
                   std::vector<Launch>& out) {
  const Tensor& A = p->tensors[st.ta];
  const Tensor& B = p->tensors[st.tb];
  const Tensor& C = p->tensors[st.tc];
  Launch L;
  GettArgs& g = L.g;
  memset(&g, 0, sizeof(g));
  g.A = tensor_ptr(p, A) + 2 * (A.leaf ? leaf_chunk_offset(p, A, chunk_base, chunk_bits) : 0);
  g.B = tensor_ptr(p, B) + 2 * (B.leaf ? leaf_chunk_offset(p, B, chunk_base, chunk_bits) : 0);
  g.C = const_cast<float*>(tensor_ptr(p, C));
  const int S = p->S;
  auto slots = [&](const Tensor& T, int id, const uint32_t*& mx, const int32_t*& ex, int& ps) {
    if (T.per_slice && !T.leaf) {
      mx = p->d_max_ps + (int64_t)id * S;
      ex = p->d_exp_ps + (int64_t)id * S;
      ps = 1;
    } else {
      mx = p->d_max_inv + id;
      ex = p->d_exp_inv + id;
      ps = 0;
    }
  };
  const int32_t* ec;
  const uint32_t* mc;
  slots(A, st.ta, g.maxA, g.expA, g.a_ps);
  slots(B, st.tb, g.maxB, g.expB, g.b_ps);
  slots(C, st.tc, mc, ec, g.c_ps);
  g.scale_mode = scaled(p) ? 1 : 0;
  if (g.scale_mode) {
    g.maxC = const_cast<uint32_t*>(mc);
    g.expC = const_cast<int32_t*>(ec);
  }
  g.target_exp = (st.kernel == TN_K_MFMA_F16X3 || st.kernel == TN_K_MFMA_BF16X3) ? 14 : 0;
  g.chunk_bits = st.per_slice ? chunk_bits : 0;
  g.fa = A.fmt;
  g.fb = B.fmt;
  g.fc = C.fmt;
  g.split_bf16 = p->precision == TN_PREC_BF16X3 ? 1 : 0;
  g.dma = st.dma;
  g.terms = st.terms;
  if (st.tab_label >= 0) {
    g.tab_a = st.d_tab_a;
    g.tab_b = st.d_tab_b;
    g.tab_bits = p->labels[st.tab_label].nb;
    g.values_first = st.values_first;
  }
  L.desc = d;
  L.step = s;
  L.kind = st.kernel;
  L.tile = st.tile;
  const int64_t c_total = int64_t(1) << (C.bits.size() + g.chunk_bits);
  if (st.kernel == TN_K_SMALL) {
    g.dot = st.dot ? 1 : 0;
    L.elems = c_total;
    out.push_back(L);
    return;
  }
  const int bbits = (int)st.bb.size() + g.chunk_bits;
  g.splits = st.splits;
  g.k_split_bits = st.k_split_bits;
  g.tiles_m_bits = st.tiles_m_bits;
  g.tiles_n_bits = st.tiles_n_bits;
  L.blocks = (int64_t(st.splits)) << (st.tiles_m_bits + st.tiles_n_bits + bbits);
  if (st.splits > 1) {
    g.scratch = p->d_scratch;
    g.write_scratch = 1;
    out.push_back(L);
    Launch R = L;
    R.g.write_scratch = 0;
    R.kind = TN_K_SPLITK_REDUCE;
    R.step = -1;
    R.elems = c_total;
    out.push_back(R);
    return;
  }
  out.push_back(L);
}

Launch fill_launch(uint32_t* ptr, int64_t n) {
  Launch L;
  L.kind = TN_K_FILL;
  L.fill_ptr = ptr;
  L.fill_n = n;
  L.elems = n;
  return L;
}

// Launches of the slice-independent phase.
void invariant_launches(const tn_plan_s* p, const std::vector<Step>& steps, const GettDesc* d_desc,
                        std::vector<Launch>& out) {
  if (scaled(p)) {
    const int64_t nt = (int64_t)p->tensors.size();
    if (nt > p->n_leaves) out.push_back(fill_launch(p->d_max_inv + p->n_leaves, nt - p->n_leaves));
  }
  for (int s : p->inv_order) step_launches(p, steps[s], d_desc + s, s, 0, 0, out);
}

// Launches of one chunk of 2^bits slices starting at base (aligned); the chunk
// ends by adding into the accumulator, or writing partials when partial_out is set.
void chunk_launches(const tn_plan_s* p, const std::vector<Step>& steps, const GettDesc* d_desc, int64_t base,
                    int bits, double* partial_out, std::vector<Launch>& out) {
  if (scaled(p) && !p->ps_order.empty())
    out.push_back(fill_launch(p->d_max_ps, (int64_t)p->tensors.size() * p->S));
  for (int s : p->ps_order) step_launches(p, steps[s], d_desc + s, s, base, bits, out);
  const Tensor& R = p->tensors[p->root];
  Launch L;
  L.kind = TN_K_SLICE_REDUCE;
  ReduceArgs& r = L.r;
  memset(&r, 0, sizeof(r));
  r.root = tensor_ptr(p, R);
  if (scaled(p)) r.exp = R.per_slice ? p->d_exp_ps + (int64_t)p->root * p->S : p->d_exp_inv + p->root;
  r.acc = p->d_acc;
  r.out = partial_out;
  r.flag = p->d_flag;
  r.n_amp = p->n_amp;
  r.n_slices = 1 << bits;
  L.elems = p->n_amp;
  out.push_back(L);
}

// Aligned power-of-two chunks of [first, first + n), each at most 2^s_bits slices.
std::vector<std::pair<int64_t, int>> chunks_of(const tn_plan_s* p, int64_t first, int64_t n) {
  std::vector<std::pair<int64_t, int>> out;
  int64_t cur = first;
  const int64_t end = first + n;
  while (cur < end) {
    int bits = 0;
    while (bits < p->s_bits && (cur & ((int64_t(2) << bits) - 1)) == 0 && cur + (int64_t(2) << bits) <= end) ++bits;
    out.push_back({cur, bits});
    cur += int64_t(1) << bits;
  }
  return out;
}

// Issue launches on stream `st`; with `timed` (the plan's own stream only), step
// launches are bracketed by events when options.record_steps is set.
tn_status execute_on(tn_plan_s* p, const std::vector<Launch>& ls, hipStream_t st, bool timed) {
  for (size_t i = 0; i < ls.size(); ++i) {
    const Launch& L = ls[i];
    tn_status r = TN_OK;
    if (timed && L.step >= 0 && L.kind != TN_K_SMALL && i + 1 < ls.size() && ls[i + 1].kind == TN_K_SPLITK_REDUCE) {
      const Launch& R = ls[++i];
      r = timed_launch(p, L.step, L.kind, L.desc, L.g, L.nblocks(256), "step", &R.g, R.nblocks(256));
      if (r) return r;
      continue;
    }
    switch (L.kind) {
      case TN_K_FILL: r = check(tn_launch_fill_u32(L.fill_ptr, 0, L.fill_n, st), "fill"); break;
      case TN_K_SLICE_REDUCE: r = check(tn_launch_slice_reduce(L.r, st), "slice reduce"); break;
      case TN_K_SPLITK_REDUCE:
        r = check(tn_launch_gett(TN_K_SPLITK_REDUCE, 0, L.desc, L.g, L.nblocks(256), st), "split-K reduce");
        break;
      default:
        r = (timed && L.step >= 0) ? timed_launch(p, L.step, L.kind, L.desc, L.g, L.nblocks(256), "step", nullptr, 0)
                                   : check(tn_launch_gett(L.kind, L.tile, L.desc, L.g, L.nblocks(256), st), "step");
    }
    if (r) return r;
  }
  return TN_OK;
}

tn_status execute(tn_plan_s* p, const std::vector<Launch>& ls) { return execute_on(p, ls, p->stream, true); }

tn_status run_step(tn_plan_s* p, int s, int64_t chunk_base, int chunk_bits) {
  std::vector<Launch> ls;
  step_launches(p, p->steps[s], p->d_desc + s, s, chunk_base, chunk_bits, ls);
  return execute(p, ls);
}

// ---------------------------------------------------------------------------
// Autotuner: time each MFMA step with every tile shape on the device and keep
// the fastest.  Choices are cached per step signature for the process.
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;

std::string step_signature(const tn_plan_s* p, const Step& st) {
  char buf[160];
  const Tensor& A = p->tensors[st.ta];
  const Tensor& B = p->tensors[st.tb];
  const Tensor& C = p->tensors[st.tc];
  snprintf(buf, sizeof(buf), "k%d b%d m%d n%d k%d s%d f%d%d%d c%d%d", st.kernel,
           (int)st.bb.size() + (st.per_slice ? p->s_bits : 0), (int)st.mb.size(), (int)st.nb.size(),
           (int)st.kb.size(), st.per_slice ? 1 : 0, A.fmt, B.fmt, C.fmt, st.a_contig, st.b_contig);
  return buf;
}

tn_status ensure_scratch(tn_plan_s* p, int64_t elems) {
  if (elems <= p->scratch_elems) return TN_OK;
  if (!p->own_memory) return fail(TN_E_NOMEM, "split-K scratch beyond the workspace reservation");
  tn_status st = check(hipStreamSynchronize(p->stream), "scratch sync");
  if (st) return st;
  if (p->d_scratch) {
    hipFree(p->d_scratch);
    p->device_bytes -= p->scratch_elems * 8;
    p->d_scratch = nullptr;
  }
  if (hipMalloc((void**)&p->d_scratch, elems * 8) != hipSuccess) {
    hipGetLastError();
    p->scratch_elems = 0;
    return fail(TN_E_NOMEM, "split-K scratch allocation failed");
  }
  p->device_bytes += elems * 8;
  p->scratch_elems = elems;
  return TN_OK;
}

tn_status apply_tile(tn_plan_s* p, int s, int tile) {
  Step& st = p->steps[s];
  ++p->epoch;
  set_tile(p, st, tile);
  build_desc(p, st);
  tn_status r = ensure_scratch(p, st.scratch_elems);
  if (r) return r;
  return check(hipMemcpyAsync(p->d_desc + s, &st.desc, sizeof(GettDesc), hipMemcpyHostToDevice, p->stream),
               "desc upload");
}

// tuning_cache file: one "signature<TAB>tile" line per measured step signature.
void load_tuning_cache(const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return;   // a missing file is an empty cache
  char line[256];
  std::lock_guard<std::mutex> lk(g_tune_mu);
  while (fgets(line, sizeof(line), f)) {
    char* tab = strchr(line, '\t');
    if (!tab) continue;
    *tab = 0;
    char* end = nullptr;
    const long tile = strtol(tab + 1, &end, 10);
    if (end == tab + 1 || tile < 0 || tile >= TN_N_TILES) continue;
    g_tune_cache[line] = (int)tile;
  }
  fclose(f);
}

tn_status save_tuning_cache(const char* path) {
  std::map<std::string, int> all;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    all = g_tune_cache;
  }
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return fail(TN_E_ARG, std::string("tuning_cache: cannot write ") + tmp);
  bool ok = true;
  for (const auto& kv : all) ok = ok && fprintf(f, "%s\t%d\n", kv.first.c_str(), kv.second) > 0;
  ok = (fclose(f) == 0) && ok;
  if (!ok || rename(tmp.c_str(), path) != 0) {
    remove(tmp.c_str());
    return fail(TN_E_ARG, std::string("tuning_cache: cannot write ") + path);
  }
  return TN_OK;
}

tn_status autotune(tn_plan_s* p) {
  if (p->opts.tuning_cache) load_tuning_cache(p->opts.tuning_cache);
  hipEvent_t e0, e1;
  tn_status r = check(hipEventCreate(&e0), "event");
  if (r) return r;
  if ((r = check(hipEventCreate(&e1), "event"))) {
    hipEventDestroy(e0);
    return r;
  }
  const int keep_record = p->opts.record_steps;
  p->opts.record_steps = 0;
  // Steps run in path order on slice chunk 0, each once whether timed or not, so that
  // every timed step reads the real intermediates of its operands (the clock the chip
  // holds under a load depends on the data it multiplies).
  for (size_t s = 0; s < p->steps.size() && !r; ++s) {
    Step& st = p->steps[s];
    const int bits = st.per_slice ? p->s_bits : 0;
    if (st.kernel == TN_K_SMALL) {
      r = run_step(p, (int)s, 0, bits);
      continue;
    }
    const std::string sig = step_signature(p, st);
    int cached = -1;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_cache.find(sig);
      if (it != g_tune_cache.end()) cached = it->second;
    }
    if (cached >= 0) {
      r = apply_tile(p, (int)s, cached);
      if (!r) r = run_step(p, (int)s, 0, bits);
      continue;
    }
    int best = st.tile;
    float best_ms = 1e30f;
    for (int tile = 0; tile < TN_N_TILES && !r; ++tile) {
      if ((r = apply_tile(p, (int)s, tile))) break;
      if ((r = run_step(p, (int)s, 0, bits))) break;   // warm-up
      if ((r = check(hipEventRecord(e0, p->stream), "event"))) break;
      for (int rep = 0; rep < 2 && !r; ++rep) r = run_step(p, (int)s, 0, bits);
      if (r || (r = check(hipEventRecord(e1, p->stream), "event"))) break;
      if ((r = check(hipEventSynchronize(e1), "event sync"))) break;
      float ms = 0.f;
      if ((r = check(hipEventElapsedTime(&ms, e0, e1), "event time"))) break;
      if (ms < best_ms) {
        best_ms = ms;
        best = tile;
      }
    }
    if (!r) r = apply_tile(p, (int)s, best);
    if (!r) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune_cache[sig] = best;
    }
  }
  p->opts.record_steps = keep_record;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (!r) r = check(hipStreamSynchronize(p->stream), "tuning sync");
  if (!r) r = validate_bounds(p);
  if (!r && p->opts.tuning_cache) r = save_tuning_cache(p->opts.tuning_cache);
  return r;
}

// Cost-model features of a step run with `tile` (layout in include/tn.h).
void step_features(const tn_plan_s* p, const Step& st0, int tile, float* f) {
  Step st = st0;
  const bool mfma = st.kernel != TN_K_SMALL;
  if (mfma && tile >= 0 && tile != st.tile) {
    set_tile(p, st, tile);
    build_desc(const_cast<tn_plan_s*>(p), st);
  }
  const Tensor& A = p->tensors[st.ta];
  const Tensor& B = p->tensors[st.tb];
  const Tensor& C = p->tensors[st.tc];
  const int bb = (int)st.bb.size() + (st.per_slice ? p->s_bits : 0);
  const int mb = (int)st.mb.size(), nb = (int)st.nb.size(), kb = (int)st.kb.size();
  for (int i = 0; i < TN_COST_FEATURES; ++i) f[i] = 0.f;
  f[0] = (float)bb;
  f[1] = (float)mb;
  f[2] = (float)nb;
  f[3] = (float)kb;
  f[4] = (float)(3 + bb + mb + nb + kb);
  const double elems = std::ldexp(1.0, bb + mb + kb) + std::ldexp(1.0, bb + kb + nb) + std::ldexp(1.0, bb + mb + nb);
  f[5] = (float)std::log2(8.0 * elems);
  f[6] = f[4] - f[5];
  f[11] = st.per_slice ? 1.f : 0.f;
  f[12 + std::min(std::max(st.kernel, 0), 3)] = 1.f;
  if (mfma) {
    int bm = 128, bn = 128, nt = 256;
    tn_tile_shape(st.tile, &bm, &bn, &nt);
    if (st.dma >= 2) {   // the copy path's 512 x 64 / 512 x 32 layouts of the 256x128 tile id
      bm = 512;
      bn = st.dma == 2 ? 64 : 32;
    }
    const int sb = ilog2_exact(st.splits);
    f[7] = (float)st.tiles_m_bits;
    f[8] = (float)st.tiles_n_bits;
    f[9] = (float)sb;
    f[10] = (float)(bb + st.tiles_m_bits + st.tiles_n_bits + sb);
    f[16 + st.tile] = 1.f;
    f[20] = (float)st.a_contig;
    f[21] = (float)st.b_contig;
    f[22] = (float)contig_run(st.desc.ec);
    f[26] = (float)std::min(0, mb - ilog2_exact(bm));
    f[27] = (float)std::min(0, nb - ilog2_exact(bn));
    f[28] = (float)(st.k_split_bits - 4);
  } else {
    // one thread per output element in blocks of 256
    f[10] = (float)std::max(0, bb + mb + nb - 8);
  }
  f[23] = A.fmt == TN_FMT_SPLIT ? 1.f : 0.f;
  f[24] = B.fmt == TN_FMT_SPLIT ? 1.f : 0.f;
  f[25] = C.fmt == TN_FMT_SPLIT ? 1.f : 0.f;
}

// Re-tile one MFMA step; device plans also upload its descriptor.
tn_status retile_step(tn_plan_s* p, int s, int tile) {
  if (!p->host_only) return apply_tile(p, s, tile);
  Step& st = p->steps[s];
  ++p->epoch;
  set_tile(p, st, tile);
  build_desc(p, st);
  return TN_OK;
}

}  // namespace

extern "C" {

const char* tn_status_string(tn_status s) {
  switch (s) {
    case TN_OK: return "TN_OK";
    case TN_E_ARG: return "TN_E_ARG";
    case TN_E_LABEL: return "TN_E_LABEL";
    case TN_E_PATH: return "TN_E_PATH";
    case TN_E_SLICE: return "TN_E_SLICE";
    case TN_E_CAP: return "TN_E_CAP";
    case TN_E_NOMEM: return "TN_E_NOMEM";
    case TN_E_DEVICE: return "TN_E_DEVICE";
    case TN_E_STATE: return "TN_E_STATE";
    case TN_E_UNSUPPORTED: return "TN_E_UNSUPPORTED";
    case TN_E_NUMERIC: return "TN_E_NUMERIC";
  }
  return "unknown status";
}

const char* tn_last_error_message(void) { return g_err.c_str(); }

}  // extern "C"

namespace {
tn_status create_plan(tn_plan* out, int32_t n_tensors, const int32_t* ranks, const int32_t* const* labels,
                      const int64_t* const* extents, const double* const* data, int32_t n_open,
                      const int32_t* open_labels, int32_t n_steps, const int32_t* path, int32_t n_sliced,
                      const int32_t* sliced_labels, int64_t n_bitstrings, const uint8_t* bitstrings,
                      const tn_options* opts) {
  if (!out) return fail(TN_E_ARG, "null output pointer");
  *out = nullptr;
  tn_plan_s* p = new (std::nothrow) tn_plan_s();
  if (!p) return fail(TN_E_NOMEM, "host allocation failed");
  if (bitstrings) {
    if (n_bitstrings < 1 || n_open < 1) {
      delete p;
      return fail(TN_E_ARG, "a sparse state needs at least one bitstring and one open label");
    }
    if (n_open > 64) {
      delete p;
      return fail(TN_E_UNSUPPORTED, "a sparse state measures at most 64 open labels");
    }
    p->sparse = true;
    p->bkeys.resize(n_bitstrings);   // may throw: the entry points turn that into TN_E_NOMEM
    for (int64_t i = 0; i < n_bitstrings; ++i) {
      uint64_t k = 0;
      for (int32_t c = 0; c < n_open; ++c) {
        const uint8_t v = bitstrings[i * n_open + c];
        if (v > 1) {
          delete p;
          return fail(TN_E_ARG, "bitstring values must be 0 or 1");
        }
        k |= uint64_t(v) << c;
      }
      p->bkeys[i] = k;
    }
  }
  if (opts) {
    if (opts->struct_size < (int32_t)offsetof(tn_options, deterministic)) {
      delete p;
      return fail(TN_E_ARG, "tn_options.struct_size too small");
    }
    memcpy(&p->opts, opts, std::min<size_t>(sizeof(tn_options), (size_t)opts->struct_size));
  }
  if (p->opts.deterministic != 0 && p->opts.deterministic != 1) {
    delete p;
    return fail(TN_E_ARG, "tn_options.deterministic must be 0 or 1");
  }
  if (p->opts.tuning < 0 || p->opts.tuning > 2 || (p->opts.tuning == 2 && !p->opts.cost_model)) {
    delete p;
    return fail(TN_E_ARG, "tn_options.tuning must be 0, 1 or 2 (2 needs cost_model)");
  }
  if (p->opts.split_policy < 0 || p->opts.split_policy > 2) {
    delete p;
    return fail(TN_E_ARG, "tn_options.split_policy must be 0, 1 or 2");
  }
  p->host_only = p->opts.host_only != 0;
  p->stream = reinterpret_cast<hipStream_t>(p->opts.stream);
  p->precision = p->opts.precision;
  if (p->precision < TN_PREC_C64 || p->precision > TN_PREC_BF16X3) {
    delete p;
    return fail(TN_E_ARG, "unknown precision");
  }
  g_err.clear();
  tn_status st = plan_build(p, n_tensors, ranks, labels, extents, data, n_open, open_labels, n_steps, path,
                            n_sliced, sliced_labels);
  if (st == TN_OK && p->opts.tuning == 2) st = tn_plan_tune_with_model(p, p->opts.cost_model, nullptr, 0);
  p->opts.cost_model = nullptr;   // borrowed for creation only
  p->opts.tuning_cache = nullptr;
  if (st != TN_OK) {
    std::string keep = g_err;
    delete p;
    g_err = keep;
    return st;
  }
  *out = p;
  return TN_OK;
}
}  // namespace

extern "C" {

tn_status tn_plan_create(tn_plan* out, int32_t n_tensors, const int32_t* ranks, const int32_t* const* labels,
                         const int64_t* const* extents, const double* const* data, int32_t n_open,
                         const int32_t* open_labels, int32_t n_steps, const int32_t* path, int32_t n_sliced,
                         const int32_t* sliced_labels, const tn_options* opts) {
  TN_TRY
  return create_plan(out, n_tensors, ranks, labels, extents, data, n_open, open_labels, n_steps, path, n_sliced,
                     sliced_labels, 0, nullptr, opts);
  TN_CATCH
}

tn_status tn_plan_create_sparse(tn_plan* out, int32_t n_tensors, const int32_t* ranks, const int32_t* const* labels,
                                const int64_t* const* extents, const double* const* data, int32_t n_open,
                                const int32_t* open_labels, int32_t n_steps, const int32_t* path, int32_t n_sliced,
                                const int32_t* sliced_labels, int64_t n_bitstrings, const uint8_t* bitstrings,
                                const tn_options* opts) {
  TN_TRY
  if (!bitstrings) return fail(TN_E_ARG, "null bitstrings");
  return create_plan(out, n_tensors, ranks, labels, extents, data, n_open, open_labels, n_steps, path, n_sliced,
                     sliced_labels, n_bitstrings, bitstrings, opts);
  TN_CATCH
}

tn_status tn_plan_sparse_index(tn_plan p, int64_t* index, int64_t n_bitstrings) {
  TN_TRY
  if (!p || !index) return fail(TN_E_ARG, "null argument");
  if (!p->sparse) return fail(TN_E_STATE, "the plan has no sparse state");
  if (n_bitstrings != (int64_t)p->amp_index.size()) return fail(TN_E_ARG, "n_bitstrings does not match the plan");
  std::copy(p->amp_index.begin(), p->amp_index.end(), index);
  return TN_OK;
  TN_CATCH
}

void tn_plan_destroy(tn_plan plan) {
  TN_TRY_VOID
  delete plan;
  TN_CATCH_VOID
}

tn_status tn_plan_describe(tn_plan p, tn_plan_info* out) {
  TN_TRY
  if (!p || !out) return fail(TN_E_ARG, "null argument");
  memset(out, 0, sizeof(*out));
  out->n_slices = p->n_slices;
  out->n_amplitudes = p->n_amp;
  out->n_steps = (int32_t)p->steps.size();
  out->n_slice_steps = (int32_t)p->ps_order.size();
  out->flops_per_slice = p->flops_ps;
  out->flops_invariant = p->flops_inv;
  out->bytes_per_slice = p->bytes_ps;
  out->bytes_invariant = p->bytes_inv;
  out->max_intermediate = p->max_intermediate;
  out->workspace_bytes = p->host_only ? p->ws_need : (int64_t)p->device_bytes;
  out->slice_batch = p->S;
  out->precision = p->precision;
  return TN_OK;
  TN_CATCH
}

tn_status tn_plan_steps(tn_plan p, tn_step_info* steps, int32_t cap) {
  TN_TRY
  if (!p || (!steps && cap > 0) || cap < 0) return fail(TN_E_ARG, "bad arguments");
  const int n = std::min<int>(cap, (int)p->steps.size());
  for (int i = 0; i < n; ++i) {
    const Step& st = p->steps[i];
    tn_step_info& o = steps[i];
    memset(&o, 0, sizeof(o));
    o.slot_a = st.slot_a;
    o.slot_b = st.slot_b;
    o.per_slice = st.per_slice;
    o.kernel = st.kernel == TN_K_SMALL ? 0 : st.kernel == TN_K_MFMA_F32 ? 1 : st.kernel == TN_K_MFMA_F16X3 ? 2 : 3;
    o.batch = int64_t(1) << st.bb.size();
    o.m = int64_t(1) << st.mb.size();
    o.n = int64_t(1) << st.nb.size();
    o.k = int64_t(1) << st.kb.size();
    o.split_k = st.splits;
    int bm = 1, bn = 1, nt = 0;
    if (st.kernel != TN_K_SMALL) tn_tile_shape(st.tile, &bm, &bn, &nt);
    if (st.dma >= 2) {
      bm = 512;
      bn = st.dma == 2 ? 64 : 32;
    }
    o.tile_m = (int)std::min<int64_t>(o.m, bm);
    o.tile_n = (int)std::min<int64_t>(o.n, bn);
    o.a_contig = st.a_contig;
    o.b_contig = st.b_contig;
    o.flops = st.flops;
    o.terms = (st.kernel == TN_K_MFMA_F16X3 || st.kernel == TN_K_MFMA_BF16X3) ? st.terms : 0;
    o.merged_bits = st.tab_label >= 0 ? p->labels[st.tab_label].nb : -1;
    o.values_first = st.values_first;
    o.bytes = st.bytes;
    o.tile = st.kernel == TN_K_SMALL ? -1 : st.tile;
    o.lds_copy = st.dma;
  }
  return TN_OK;
  TN_CATCH
}

tn_status tn_plan_step_times(tn_plan p, double* ms_total, int64_t* launches, int32_t cap) {
  TN_TRY
  if (!p || cap < 0) return fail(TN_E_ARG, "bad arguments");
  if (p->host_only || !p->opts.record_steps) return fail(TN_E_STATE, "step recording is off");
  tn_status st = check(hipStreamSynchronize(p->stream), "stream sync");
  if (st) return st;
  p->step_ms.resize(p->steps.size(), 0.0);
  p->step_launches.resize(p->steps.size(), 0);
  for (auto& t : p->pending) {
    float ms = 0.f;
    if (!st) st = check(hipEventElapsedTime(&ms, t.start, t.stop), "event elapsed");
    p->step_ms[t.step] += ms;
    p->step_launches[t.step] += 1;
    p->event_pool.push_back({t.start, t.stop});
  }
  p->pending.clear();
  if (st) return st;
  const int n = std::min<int>(cap, (int)p->steps.size());
  for (int i = 0; i < n; ++i) {
    if (ms_total) ms_total[i] = p->step_ms[i];
    if (launches) launches[i] = p->step_launches[i];
  }
  std::fill(p->step_ms.begin(), p->step_ms.end(), 0.0);
  std::fill(p->step_launches.begin(), p->step_launches.end(), 0);
  return TN_OK;
  TN_CATCH
}

tn_status tn_plan_step_features(tn_plan p, int32_t step, int32_t tile, float* out, int32_t cap) {
  TN_TRY
  if (!p || !out || cap < TN_COST_FEATURES) return fail(TN_E_ARG, "bad arguments");
  if (step < 0 || step >= (int32_t)p->steps.size()) return fail(TN_E_ARG, "step out of range");
  if (tile < -1 || tile >= TN_N_TILES) return fail(TN_E_ARG, "tile id out of range");
  step_features(p, p->steps[step], tile, out);
  return TN_OK;
  TN_CATCH
}

tn_status tn_plan_set_tile(tn_plan p, int32_t step, int32_t tile) {
  TN_TRY
  if (!p) return fail(TN_E_ARG, "null plan");
  if (step < 0 || step >= (int32_t)p->steps.size()) return fail(TN_E_ARG, "step out of range");
  if (tile < 0 || tile >= TN_N_TILES) return fail(TN_E_ARG, "tile id out of range");
  if (p->steps[step].kernel == TN_K_SMALL) return fail(TN_E_ARG, "step runs on the small kernel (no tile)");
  tn_status st = retile_step(p, step, tile);
  if (!st) st = validate_steps(p, p->steps);
  return st;
  TN_CATCH
}

tn_status tn_plan_set_step_terms(tn_plan p, int32_t step, int32_t terms) {
  TN_TRY
  if (!p) return fail(TN_E_ARG, "null plan");
  if (step < 0 || step >= (int32_t)p->steps.size()) return fail(TN_E_ARG, "step out of range");
  Step& st = p->steps[step];
  if (st.kernel != TN_K_MFMA_F16X3 && st.kernel != TN_K_MFMA_BF16X3)
    return fail(TN_E_ARG, "step does not run a split-precision kernel");
  if (terms != 1 && terms != 3) return fail(TN_E_ARG, "terms must be 1 or 3");
  if (st.terms != terms) ++p->epoch;
  st.terms = terms;
  return TN_OK;
  TN_CATCH
}

tn_status tn_plan_tune_with_model(tn_plan p, tn_costmodel model, float* predicted_us, int32_t cap) {
  TN_TRY
  if (!p || !model) return fail(TN_E_ARG, "null argument");
  int32_t nf = 0;
  tn_status st = tn_costmodel_describe(model, &nf, nullptr, nullptr);
  if (st) return st;
  if (nf != TN_COST_FEATURES) return fail(TN_E_ARG, "model must take the step features as input");
  const int n = (int)p->steps.size();
  // every (step, tile) candidate in one batch; small-kernel steps get one row
  std::vector<float> X;
  std::vector<std::pair<int, int>> rows;
  for (int s = 0; s < n; ++s) {
    const bool mfma = p->steps[s].kernel != TN_K_SMALL;
    for (int t = 0; t < (mfma ? TN_N_TILES : 1); ++t) {
      const size_t o = X.size();
      X.resize(o + TN_COST_FEATURES);
      step_features(p, p->steps[s], mfma ? t : -1, X.data() + o);
      rows.push_back({s, mfma ? t : -1});
    }
  }
  std::vector<float> y(rows.size());
  if ((st = tn_costmodel_predict(model, X.data(), (int64_t)rows.size(), y.data()))) return st;
  std::vector<int> best(n, -1);
  std::vector<float> best_y(n, 1e30f);
  for (size_t r = 0; r < rows.size(); ++r) {
    const int s = rows[r].first;
    if (y[r] < best_y[s]) {
      best_y[s] = y[r];
      best[s] = rows[r].second;
    }
  }
  for (int s = 0; s < n && !st; ++s)
    if (best[s] >= 0 && best[s] != p->steps[s].tile) st = retile_step(p, s, best[s]);
  if (!st) st = validate_steps(p, p->steps);
  if (!st && predicted_us)
    for (int s = 0; s < n && s < cap; ++s) predicted_us[s] = std::exp(best_y[s]);
  return st;
  TN_CATCH
}

}  // extern "C"

namespace {

// A pairwise step of 2^bb x 2^mb x 2^nb x 2^kb complex extents laid out the way a plan lays
// out intermediates for their consumer: k innermost in both operands (A: k, m, batch bits;
// B: k, n, batch bits; C: n, m, batch bits, lowest first), operands and result stored split
// when the step runs a split kernel; kernel and K split by the planner's own rules.
void canonical_step(tn_plan_s& tmp, Step& st, int32_t precision, int bb, int mb, int nb, int kb) {
  tmp.precision = precision;
  tmp.host_only = true;
  for (int j = 0; j < bb; ++j) st.bb.push_back(j);
  for (int j = 0; j < mb; ++j) st.mb.push_back(bb + j);
  for (int j = 0; j < nb; ++j) st.nb.push_back(bb + mb + j);
  for (int j = 0; j < kb; ++j) st.kb.push_back(bb + mb + nb + j);
  Tensor TA, TB, TC;
  TA.bits = st.kb;
  TA.bits.insert(TA.bits.end(), st.mb.begin(), st.mb.end());
  TA.bits.insert(TA.bits.end(), st.bb.begin(), st.bb.end());
  TB.bits = st.kb;
  TB.bits.insert(TB.bits.end(), st.nb.begin(), st.nb.end());
  TB.bits.insert(TB.bits.end(), st.bb.begin(), st.bb.end());
  TC.bits = st.nb;
  TC.bits.insert(TC.bits.end(), st.mb.begin(), st.mb.end());
  TC.bits.insert(TC.bits.end(), st.bb.begin(), st.bb.end());
  TA.elems = int64_t(1) << TA.bits.size();
  TB.elems = int64_t(1) << TB.bits.size();
  TC.elems = int64_t(1) << TC.bits.size();
  tmp.tensors = {TA, TB, TC};
  st.ta = 0;
  st.tb = 1;
  st.tc = 2;
  choose_kernel(&tmp, st);
  if (st.kernel == TN_K_MFMA_F16X3 || st.kernel == TN_K_MFMA_BF16X3)
    for (auto& T : tmp.tensors) T.fmt = TN_FMT_SPLIT;
  if (st.kernel != TN_K_SMALL) build_desc(&tmp, st);
}

}  // namespace

extern "C" {

tn_status tn_costmodel_predict_shapes(tn_costmodel model, int32_t precision, const int32_t* shapes, int64_t n,
                                      float* us) {
  TN_TRY
  if (!model || n < 0 || (n > 0 && (!shapes || !us))) return fail(TN_E_ARG, "bad arguments");
  if (precision < 0 || precision > 2) return fail(TN_E_ARG, "unknown precision");
  int32_t nf = 0;
  tn_status st = tn_costmodel_describe(model, &nf, nullptr, nullptr);
  if (st) return st;
  if (nf != TN_COST_FEATURES) return fail(TN_E_ARG, "model must take the step features as input");
  std::vector<float> X;
  std::vector<int64_t> owner;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t* s = shapes + 4 * i;
    for (int j = 0; j < 4; ++j)
      if (s[j] < 0 || s[j] > 30) return fail(TN_E_UNSUPPORTED, "shape bits must lie in 0..30");
    if (s[0] > 16) return fail(TN_E_UNSUPPORTED, "at most 16 batch bits");
    tn_plan_s tmp;
    Step step;
    canonical_step(tmp, step, precision, s[0], s[1], s[2], s[3]);
    const bool mfma = step.kernel != TN_K_SMALL;
    for (int t = 0; t < (mfma ? TN_N_TILES : 1); ++t) {
      const size_t o = X.size();
      X.resize(o + TN_COST_FEATURES);
      step_features(&tmp, step, mfma ? t : -1, X.data() + o);
      owner.push_back(i);
    }
  }
  if (n == 0) return TN_OK;
  std::vector<float> y(owner.size());
  if ((st = tn_costmodel_predict(model, X.data(), (int64_t)owner.size(), y.data()))) return st;
  std::vector<float> best(n, 1e30f);
  for (size_t r = 0; r < owner.size(); ++r) best[owner[r]] = std::min(best[owner[r]], y[r]);
  for (int64_t i = 0; i < n; ++i) us[i] = std::exp(best[i]);
  return TN_OK;
  TN_CATCH
}

}  // extern "C"

namespace {

// Per-slice amplitudes of the given slices, true scale, complex128 interleaved, on the
// host (the accumulator is untouched).  Synchronous.
tn_status partials_to_host(tn_plan_s* p, const int64_t* ids, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i)
    if (ids[i] < 0 || ids[i] >= p->n_slices) return fail(TN_E_SLICE, "slice id out of range");
  if (n == 0) return TN_OK;
  std::vector<Launch> ls;
  invariant_launches(p, p->steps, p->d_desc, ls);
  tn_status st = execute(p, ls);
  if (st) return st;
  for (int64_t i = 0; i < n; ++i) {
    ls.clear();
    chunk_launches(p, p->steps, p->d_desc, ids[i], 0, p->d_part, ls);
    if ((st = execute(p, ls))) return st;
    if ((st = check(hipMemcpyAsync(out + 2 * p->n_amp * i, p->d_part, p->n_amp * 16, hipMemcpyDeviceToHost, p->stream),
                    "partials copy")))
      return st;
  }
  st = check(hipStreamSynchronize(p->stream), "partials sync");
  if (st) return st;
  int32_t flag = 0;
  st = check(hipMemcpy(&flag, p->d_flag, 4, hipMemcpyDeviceToHost), "flag copy");
  if (st) return st;
  if (flag) return fail(TN_E_NUMERIC, "Inf or NaN in a slice result");
  return TN_OK;
}

// Time of every step's launches over one chunk of slices (the plan's chunk size, from
// slice 0), measured with events on the plan's stream; the chunk's amplitudes go to the
// partials buffer, so the accumulator is untouched.  Records of the caller's own step
// timing (options.record_steps) are kept aside meanwhile.
tn_status measure_step_ms(tn_plan_s* p, std::vector<double>& ms) {
  std::vector<tn_plan_s::Timing> keep;
  keep.swap(p->pending);
  const int keep_rec = p->opts.record_steps;
  p->opts.record_steps = 1;
  std::vector<Launch> ls;
  invariant_launches(p, p->steps, p->d_desc, ls);
  chunk_launches(p, p->steps, p->d_desc, 0, p->s_bits, p->d_part, ls);
  tn_status st = execute(p, ls);
  p->opts.record_steps = keep_rec;
  if (!st) st = check(hipStreamSynchronize(p->stream), "timing sync");
  ms.assign(p->steps.size(), 0.0);
  for (auto& t : p->pending) {
    float x = 0.f;
    if (!st) st = check(hipEventElapsedTime(&x, t.start, t.stop), "event elapsed");
    ms[t.step] += x;
    p->event_pool.push_back({t.start, t.stop});
  }
  p->pending.swap(keep);
  return st;
}

// The split-precision steps, costliest first (Sec. 4.3 ranks contractions by their
// actual computation time): by measured time over one chunk, or by flops per
// contraction (slice-dependent steps count once per slice).  Ties keep step order.
tn_status rank_split_steps(tn_plan_s* p, bool by_time, std::vector<int>& rank) {
  std::vector<double> cost(p->steps.size(), 0.0);
  if (by_time) {
    tn_status st = measure_step_ms(p, cost);
    if (st) return st;
  } else {
    for (size_t i = 0; i < p->steps.size(); ++i)
      cost[i] = p->steps[i].flops * (p->steps[i].per_slice ? (double)p->n_slices : 1.0);
  }
  rank.clear();
  for (size_t i = 0; i < p->steps.size(); ++i)
    if (p->steps[i].kernel == TN_K_MFMA_F16X3 || p->steps[i].kernel == TN_K_MFMA_BF16X3) rank.push_back((int)i);
  std::stable_sort(rank.begin(), rank.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  return TN_OK;
}

}  // namespace

extern "C" {

tn_status tn_contract_slices(tn_plan p, int64_t first, int64_t n) {
  TN_TRY
  if (!p) return fail(TN_E_ARG, "null plan");
  if (p->host_only) return fail(TN_E_STATE, "host-only plan");
  if (first < 0 || n < 0 || first + n > p->n_slices) return fail(TN_E_SLICE, "slice range out of bounds");
  if (n == 0) return TN_OK;
  std::vector<Launch> ls;
  invariant_launches(p, p->steps, p->d_desc, ls);
  for (auto& c : chunks_of(p, first, n)) chunk_launches(p, p->steps, p->d_desc, c.first, c.second, nullptr, ls);
  tn_status st = execute(p, ls);
  if (st) return st;
  p->slices_acc += n;
  return TN_OK;
  TN_CATCH
}

tn_status tn_slice_partials(tn_plan p, const int64_t* ids, int64_t n, double* out) {
  TN_TRY
  if (!p || (n > 0 && (!ids || !out)) || n < 0) return fail(TN_E_ARG, "bad arguments");
  if (p->host_only) return fail(TN_E_STATE, "host-only plan");
  return partials_to_host(p, ids, n, out);
  TN_CATCH
}

tn_status tn_plan_rank_split_steps(tn_plan p, int32_t by_time, int32_t* order, int32_t cap, int32_t* n_split) {
  TN_TRY
  if (!p || cap < 0 || (cap > 0 && !order)) return fail(TN_E_ARG, "bad arguments");
  if (by_time && p->host_only) return fail(TN_E_STATE, "ranking by measured time needs a device plan");
  std::vector<int> rank;
  tn_status st = rank_split_steps(p, by_time != 0, rank);
  if (st) return st;
  for (int i = 0; i < cap && i < (int)rank.size(); ++i) order[i] = rank[i];
  if (n_split) *n_split = (int32_t)rank.size();
  return TN_OK;
  TN_CATCH
}

tn_status tn_plan_choose_single_products(tn_plan p, double budget, const int64_t* ids, int64_t n_ids,
                                         int32_t* k_chosen, double* eps_l2sq) {
  TN_TRY
  if (!p || !ids || n_ids < 1 || !(budget >= 0.0)) return fail(TN_E_ARG, "bad arguments");
  if (p->host_only) return fail(TN_E_STATE, "host-only plan");
  for (int64_t i = 0; i < n_ids; ++i)
    if (ids[i] < 0 || ids[i] >= p->n_slices) return fail(TN_E_SLICE, "slice id out of range");
  std::vector<int> rank;
  tn_status st = rank_split_steps(p, true, rank);
  if (st) return st;
  if (rank.empty()) return fail(TN_E_STATE, "the plan has no split-precision step");
  auto set_top = [&](int k) {
    for (size_t i = 0; i < rank.size(); ++i) {
      Step& s = p->steps[rank[i]];
      const int terms = (int)i < k ? 1 : 3;
      if (s.terms != terms) ++p->epoch;
      s.terms = terms;
    }
  };
  // reference: three products on every step
  set_top(0);
  const size_t len = (size_t)(2 * p->n_amp * n_ids);
  std::vector<double> ref(len), cur(len);
  if ((st = partials_to_host(p, ids, n_ids, ref.data()))) return st;
  double l2_ref = 0.0;
  for (double x : ref) l2_ref += x * x;
  int best_k = 0;
  double best_eps = 0.0;
  const int n_split = (int)rank.size();
  for (int k = 1; k <= n_split;) {
    set_top(k);
    if ((st = partials_to_host(p, ids, n_ids, cur.data()))) break;
    double l2 = 0.0;
    for (double x : cur) l2 += x * x;
    const double eps = l2_ref > 0.0 ? std::fabs(l2 - l2_ref) / l2_ref : 0.0;
    if (!(eps <= budget)) break;
    best_k = k;
    best_eps = eps;
    if (k == n_split) break;
    // candidate k grow by about 1.5x (1, 2, 3, 4, 6, 9, ...), always ending at n_split
    k = std::min(n_split, std::max(k + 1, (k * 3) / 2));
  }
  set_top(best_k);
  if (st) return st;
  if (k_chosen) *k_chosen = best_k;
  if (eps_l2sq) *eps_l2sq = best_eps;
  return TN_OK;
  TN_CATCH
}

tn_status tn_amplitudes(tn_plan p, double* out, int64_t n_amp, int64_t* slices_accumulated) {
  TN_TRY
  if (!p || !out) return fail(TN_E_ARG, "null argument");
  if (p->host_only) return fail(TN_E_STATE, "host-only plan");
  if (n_amp != p->n_amp) return fail(TN_E_ARG, "n_amp does not match the plan's output size");
  tn_status st = check(hipStreamSynchronize(p->stream), "stream sync");
  if (st) return st;
  int32_t flag = 0;
  if ((st = check(hipMemcpy(&flag, p->d_flag, 4, hipMemcpyDeviceToHost), "flag copy"))) return st;
  if (flag) return fail(TN_E_NUMERIC, "Inf or NaN reached a slice result");
  if ((st = check(hipMemcpy(out, p->d_acc, n_amp * 16, hipMemcpyDeviceToHost), "accumulator copy"))) return st;
  if (slices_accumulated) *slices_accumulated = p->slices_acc;
  return TN_OK;
  TN_CATCH
}

tn_status tn_plan_xeb(tn_plan p, int32_t n_qubits, int32_t n_bins, double x_lo, double x_hi, tn_xeb_stats* stats,
                      int64_t* hist) {
  TN_TRY
  if (!p || !stats || n_qubits < 0 || n_qubits > 1000 || n_bins < 0 || n_bins > (1 << 20) ||
      (n_bins > 0 && (!hist || !(x_hi > x_lo))))
    return fail(TN_E_ARG, "bad arguments");
  if (p->host_only) return fail(TN_E_STATE, "host-only plan");
  tn_status st = check(hipStreamSynchronize(p->stream), "stream sync");
  if (st) return st;
  int32_t flag = 0;
  if ((st = check(hipMemcpy(&flag, p->d_flag, 4, hipMemcpyDeviceToHost), "flag copy"))) return st;
  if (flag) return fail(TN_E_NUMERIC, "Inf or NaN reached a slice result");
  // samples: one per bitstring of a sparse-state plan (repeats count again), else every amplitude
  const int64_t m = p->sparse ? (int64_t)p->amp_index.size() : p->n_amp;
  const int64_t blocks = (m + 255) / 256;
  const size_t idx_bytes = p->sparse ? (size_t)m * 8 : 0;
  const size_t part_bytes = (size_t)blocks * 16, hist_bytes = (size_t)n_bins * 8;
  char* buf = nullptr;
  if (hipMalloc((void**)&buf, idx_bytes + part_bytes + hist_bytes + 16) != hipSuccess) {
    hipGetLastError();
    return fail(TN_E_NOMEM, "xeb buffers: device allocation failed");
  }
  int64_t* d_idx = p->sparse ? reinterpret_cast<int64_t*>(buf) : nullptr;
  double* d_part = reinterpret_cast<double*>(buf + idx_bytes);
  unsigned long long* d_hist = reinterpret_cast<unsigned long long*>(buf + idx_bytes + part_bytes);
  double* d_out = reinterpret_cast<double*>(buf + idx_bytes + part_bytes + hist_bytes);
  if (d_idx) st = check(hipMemcpyAsync(d_idx, p->amp_index.data(), idx_bytes, hipMemcpyHostToDevice, p->stream),
                        "index upload");
  if (!st && n_bins > 0) st = check(tn_launch_fill_u32(d_hist, 0, (int64_t)n_bins * 2, p->stream), "hist clear");
  const double log_d = n_qubits * std::log(2.0);
  if (!st)
    st = check(tn_launch_xeb(p->d_acc, d_idx, m, log_d, n_bins, x_lo, x_hi, d_part, d_hist, d_out, p->stream),
               "xeb kernels");
  double sums[2] = {0.0, 0.0};
  std::vector<unsigned long long> h(n_bins);
  if (!st) st = check(hipMemcpyAsync(sums, d_out, 16, hipMemcpyDeviceToHost, p->stream), "xeb copy");
  if (!st && n_bins > 0)
    st = check(hipMemcpyAsync(h.data(), d_hist, hist_bytes, hipMemcpyDeviceToHost, p->stream), "hist copy");
  tn_status st2 = check(hipStreamSynchronize(p->stream), "xeb sync");
  hipFree(buf);
  if (st) return st;
  if (st2) return st2;
  const double D = std::ldexp(1.0, n_qubits);
  memset(stats, 0, sizeof(*stats));
  stats->samples = m;
  stats->sum_p = sums[0];
  stats->sum_p2 = sums[1];
  stats->mean_dp = m > 0 ? D * sums[0] / (double)m : 0.0;
  stats->mean_dp2 = m > 0 ? D * D * sums[1] / (double)m : 0.0;
  stats->lxeb = stats->mean_dp - 1.0;
  for (int i = 0; i < n_bins; ++i) hist[i] = (int64_t)h[i];
  return TN_OK;
  TN_CATCH
}

tn_status tn_accumulator_set(tn_plan p, const double* acc, int64_t n_amp, int64_t slices_accumulated) {
  TN_TRY
  if (!p || !acc) return fail(TN_E_ARG, "null argument");
  if (p->host_only) return fail(TN_E_STATE, "host-only plan");
  if (n_amp != p->n_amp) return fail(TN_E_ARG, "n_amp does not match the plan's output size");
  if (slices_accumulated < 0) return fail(TN_E_ARG, "negative slice count");
  tn_status st = check(hipStreamSynchronize(p->stream), "stream sync");
  if (st) return st;
  if ((st = check(hipMemcpy(p->d_acc, acc, n_amp * 16, hipMemcpyHostToDevice), "accumulator copy"))) return st;
  p->slices_acc = slices_accumulated;
  return TN_OK;
  TN_CATCH
}

tn_status tn_reset(tn_plan p) {
  TN_TRY
  if (!p) return fail(TN_E_ARG, "null plan");
  if (p->host_only) return fail(TN_E_STATE, "host-only plan");
  tn_status st = check(hipMemsetAsync(p->d_acc, 0, p->n_amp * 16, p->stream), "reset");
  if (st) return st;
  if ((st = check(hipMemsetAsync(p->d_flag, 0, 4, p->stream), "reset"))) return st;
  p->slices_acc = 0;
  return check(hipStreamSynchronize(p->stream), "reset sync");
  TN_CATCH
}

// ---------------------------------------------------------------------------
// Batching form (tn_group_*)
// ---------------------------------------------------------------------------
}  // extern "C"

struct tn_group_s {
  std::vector<tn_plan_s*> plans;
  int precision = 0;
  int n_branches = 1;
  hipStream_t stream = nullptr;              // capture and replay stream
  hipStream_t user_stream = nullptr;
  std::vector<hipStream_t> branch;           // fork streams used while capturing
  std::vector<hipEvent_t> branch_done;
  hipEvent_t fork = nullptr, ev = nullptr;
  struct Cached {
    std::vector<int64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* d_batch = nullptr;                 // task and block tables of the batched launches
    int64_t n_kernels = 0;
    int32_t n_branches = 0;
    void release() {
      if (exec) hipGraphExecDestroy(exec);
      if (graph) hipGraphDestroy(graph);
      if (d_batch) hipFree(d_batch);
      exec = nullptr;
      graph = nullptr;
      d_batch = nullptr;
    }
  };
  std::vector<Cached> cache;
  int64_t last_kernels = 0;
  int32_t last_branches = 0;

  ~tn_group_s() {
    if (stream) hipStreamSynchronize(stream);
    for (auto& c : cache) c.release();
    for (auto e : branch_done)
      if (e) hipEventDestroy(e);
    for (auto b : branch)
      if (b) hipStreamDestroy(b);
    if (fork) hipEventDestroy(fork);
    if (ev) hipEventDestroy(ev);
    if (stream) hipStreamDestroy(stream);
  }
};

namespace {

// Capture every plan's launch chain for the ranges in `key` into one graph:
// plans are assigned to branches longest-processing-time first (by flops), and
// branches fork from and join into the group stream.  Within a branch the plans'
// chains advance in rounds: round r holds the r-th launch of each of the branch's
// plans (launches of different plans are independent, and a plan's launches stay
// in order because rounds do).  The element-wise launches of a round (small
// steps, split-K sums, FP64 slice sums, fills) go out as one batched launch; its
// MFMA launches follow it one by one.
constexpr int64_t kMaxBranchNodes = 8192;

tn_status group_build(tn_group_s* G, const std::vector<int64_t>& key, tn_group_s::Cached& C) {
  const int P = (int)G->plans.size();
  std::vector<std::vector<Launch>> chains(P);
  std::vector<std::pair<double, int>> work;
  for (int i = 0; i < P; ++i) {
    tn_plan_s* p = G->plans[i];
    const int64_t first = key[3 * i], n = key[3 * i + 1];
    if (n == 0) continue;
    invariant_launches(p, p->steps, p->d_desc, chains[i]);
    for (auto& c : chunks_of(p, first, n)) chunk_launches(p, p->steps, p->d_desc, c.first, c.second, nullptr, chains[i]);
    work.push_back({p->flops_inv + p->flops_ps * (double)n + 1.0, i});
  }
  std::sort(work.begin(), work.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
    return a.first != b.first ? a.first > b.first : a.second < b.second;
  });
  const int B = std::max(1, std::min<int>(G->n_branches, (int)work.size()));
  std::vector<double> load(B, 0.0);
  std::vector<std::vector<int>> assign(B);
  for (auto& w : work) {
    const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[b] += w.first;
    assign[b].push_back(w.second);
  }
  struct Round {
    int64_t task0 = 0, ntask = 0, block0 = 0, nblock = 0;
    std::vector<std::pair<int, const Launch*>> single;   // (plan, launch) issued on their own
  };
  std::vector<std::vector<Round>> rounds(B);
  std::vector<BatchTask> tasks;
  std::vector<int32_t> block_task;
  for (int b = 0; b < B; ++b) {
    size_t len = 0;
    for (int i : assign[b]) len = std::max(len, chains[i].size());
    for (size_t r = 0; r < len; ++r) {
      Round R;
      std::vector<std::pair<int, const Launch*>> batch;
      for (int i : assign[b]) {
        if (r >= chains[i].size()) continue;
        const Launch& L = chains[i][r];
        const bool elementwise = (L.kind == TN_K_SMALL && !L.g.dot) || L.kind == TN_K_SPLITK_REDUCE ||
                                 L.kind == TN_K_SLICE_REDUCE || L.kind == TN_K_FILL;
        if (elementwise && L.nblocks(256) > 0) batch.push_back({i, &L});
        else R.single.push_back({i, &L});
      }
      if (batch.size() == 1) {
        R.single.insert(R.single.begin(), batch[0]);
        batch.clear();
      }
      R.task0 = (int64_t)tasks.size();
      R.block0 = (int64_t)block_task.size();
      for (auto& e : batch) {
        const Launch& L = *e.second;
        BatchTask t;
        memset(&t, 0, sizeof(t));
        t.kind = L.kind;
        t.first_block = R.nblock;
        t.desc = L.desc;
        t.g = L.g;
        t.r = L.r;
        t.fill_ptr = L.fill_ptr;
        t.fill_n = L.fill_n;
        const int64_t nb = L.nblocks(256);
        block_task.insert(block_task.end(), (size_t)nb, (int32_t)R.ntask);
        tasks.push_back(t);
        ++R.ntask;
        R.nblock += nb;
      }
      rounds[b].push_back(std::move(R));
    }
  }
  // Longest chain of kernel nodes in one branch.  A capture with a 74k-node branch ended the
  // process during capture or instantiation (cause not established); graphs are kept to at
  // most kMaxBranchNodes nodes per branch, and larger ranges must be split by the caller.
  for (int b = 0; b < B; ++b) {
    int64_t nodes = 0;
    for (const Round& R : rounds[b]) nodes += (R.ntask > 0 ? 1 : 0) + (int64_t)R.single.size();
    if (nodes > kMaxBranchNodes)
      return fail(TN_E_UNSUPPORTED, "group graph branch of " + std::to_string(nodes) + " kernel nodes (at most " +
                                        std::to_string(kMaxBranchNodes) + "): contract fewer slices per call");
  }
  const BatchTask* d_tasks = nullptr;
  const int32_t* d_block_task = nullptr;
  if (!tasks.empty()) {
    const size_t tb = tasks.size() * sizeof(BatchTask), bb = block_task.size() * sizeof(int32_t);
    if (hipMalloc(&C.d_batch, tb + bb) != hipSuccess) {
      hipGetLastError();
      return fail(TN_E_NOMEM, "group task tables: device allocation failed");
    }
    // on the group's stream (after any replay still running there), finished before capture
    tn_status st = check(hipMemcpyAsync(C.d_batch, tasks.data(), tb, hipMemcpyHostToDevice, G->stream),
                         "task table upload");
    if (!st)
      st = check(hipMemcpyAsync(static_cast<char*>(C.d_batch) + tb, block_task.data(), bb, hipMemcpyHostToDevice,
                                G->stream),
                 "block table upload");
    if (!st) st = check(hipStreamSynchronize(G->stream), "task table sync");
    if (st) return st;
    d_tasks = static_cast<const BatchTask*>(C.d_batch);
    d_block_task = reinterpret_cast<const int32_t*>(static_cast<const char*>(C.d_batch) + tb);
  }
  C.key = key;
  C.n_kernels = 0;
  C.n_branches = B;
  tn_status st = check(hipStreamBeginCapture(G->stream, hipStreamCaptureModeThreadLocal), "begin capture");
  if (st) return st;
  st = check(hipEventRecord(G->fork, G->stream), "fork");
  std::vector<Launch> one(1);
  for (int b = 0; b < B && !st; ++b) {
    st = check(hipStreamWaitEvent(G->branch[b], G->fork, 0), "fork wait");
    for (const Round& R : rounds[b]) {
      if (st) break;
      if (R.ntask > 0) {
        st = check(tn_launch_batch(d_tasks + R.task0, d_block_task + R.block0, R.nblock, G->branch[b]),
                   "batched launch");
        ++C.n_kernels;
      }
      for (auto& e : R.single) {
        if (st) break;
        one[0] = *e.second;
        st = execute_on(G->plans[e.first], one, G->branch[b], false);
        ++C.n_kernels;
      }
    }
    if (!st) st = check(hipEventRecord(G->branch_done[b], G->branch[b]), "join");
    if (!st) st = check(hipStreamWaitEvent(G->stream, G->branch_done[b], 0), "join wait");
  }
  hipGraph_t graph = nullptr;
  const tn_status end = check(hipStreamEndCapture(G->stream, &graph), "end capture");
  if (st || end) {
    if (graph) hipGraphDestroy(graph);
    return st ? st : end;
  }
  C.graph = graph;
  return check(hipGraphInstantiate(&C.exec, graph, nullptr, nullptr, 0), "graph instantiate");
}

}  // namespace

extern "C" {

tn_status tn_group_create(tn_group* out, const tn_plan* plans, int32_t n, const tn_options* opts) {
  TN_TRY
  if (!out || !plans || n < 1) return fail(TN_E_ARG, "bad arguments");
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) return fail(TN_E_ARG, "null plan");
    if (plans[i]->host_only) return fail(TN_E_STATE, "host-only plan in a group");
    if (plans[i]->precision != plans[0]->precision) return fail(TN_E_ARG, "plans of a group must share a precision");
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return fail(TN_E_ARG, "a plan appears twice in a group");
  }
  if (opts && opts->struct_size < (int32_t)offsetof(tn_options, deterministic))
    return fail(TN_E_ARG, "tn_options.struct_size too small");
  tn_group_s* G = new (std::nothrow) tn_group_s();
  if (!G) return fail(TN_E_NOMEM, "host allocation failed");
  G->precision = plans[0]->precision;
  G->n_branches = std::min(n, 8);
  if (opts) {
    G->user_stream = reinterpret_cast<hipStream_t>(opts->stream);
    if (opts->slice_batch > 0) G->n_branches = std::min<int>(opts->slice_batch, n);
  }
  for (int i = 0; i < n; ++i) G->plans.push_back(plans[i]);
  tn_status st = check(tn_prepare_kernels(), "kernel attributes");
  if (!st) st = check(hipStreamCreateWithFlags(&G->stream, hipStreamNonBlocking), "group stream");
  if (!st) st = check(hipEventCreateWithFlags(&G->ev, hipEventDisableTiming), "group event");
  if (!st) st = check(hipEventCreateWithFlags(&G->fork, hipEventDisableTiming), "group event");
  for (int b = 0; b < G->n_branches && !st; ++b) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    st = check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "branch stream");
    if (!st) G->branch.push_back(s);
    if (!st) st = check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "branch event");
    if (!st) G->branch_done.push_back(e);
  }
  if (st) {
    std::string keep = g_err;
    delete G;
    g_err = keep;
    return st;
  }
  *out = G;
  return TN_OK;
  TN_CATCH
}

}  // extern "C"

namespace {

// The captured graph of plan ranges [first[i], first[i] + count[i]) for the plans' current
// configurations: from the group's cache, else captured now (graphs of earlier plan
// configurations are dropped after their last replay has finished).
tn_status group_graph(tn_group G, const int64_t* first, const int64_t* count, tn_group_s::Cached** out) {
  if (!G || !first || !count) return fail(TN_E_ARG, "bad arguments");
  const int P = (int)G->plans.size();
  // graphs are cached per set of ranges and per plan configuration: a plan re-tiled since
  // a capture has new descriptors in device memory that its old kernels must not read
  std::vector<int64_t> key(3 * P);
  for (int i = 0; i < P; ++i) {
    if (first[i] < 0 || count[i] < 0 || first[i] + count[i] > G->plans[i]->n_slices)
      return fail(TN_E_SLICE, "slice range out of bounds for plan " + std::to_string(i));
    key[3 * i] = first[i];
    key[3 * i + 1] = count[i];
    key[3 * i + 2] = G->plans[i]->epoch;
  }
  tn_group_s::Cached* C = nullptr;
  for (auto& c : G->cache)
    if (c.key == key) C = &c;
  if (!C) {
    bool synced = false;
    for (size_t j = 0; j < G->cache.size();) {
      bool stale = false;
      for (int i = 0; i < P; ++i) stale = stale || G->cache[j].key[3 * i + 2] != key[3 * i + 2];
      if (stale) {
        if (!synced) {
          tn_status st = check(hipStreamSynchronize(G->stream), "group sync");
          if (st) return st;
          synced = true;
        }
        G->cache[j].release();
        G->cache.erase(G->cache.begin() + j);
      } else {
        ++j;
      }
    }
    G->cache.emplace_back();
    C = &G->cache.back();
    tn_status st = group_build(G, key, *C);
    if (st) {
      C->release();
      G->cache.pop_back();
      return st;
    }
  }
  *out = C;
  return TN_OK;
}

}  // namespace

extern "C" {

tn_status tn_group_prepare(tn_group G, const int64_t* first, const int64_t* count) {
  TN_TRY
  tn_group_s::Cached* C = nullptr;
  tn_status st = group_graph(G, first, count, &C);
  if (st) return st;
  G->last_kernels = C->n_kernels;
  G->last_branches = C->n_branches;
  return TN_OK;
  TN_CATCH
}

tn_status tn_group_contract(tn_group G, const int64_t* first, const int64_t* count) {
  TN_TRY
  tn_group_s::Cached* C = nullptr;
  tn_status st0 = group_graph(G, first, count, &C);
  if (st0) return st0;
  const int P = (int)G->plans.size();
  G->last_kernels = C->n_kernels;
  G->last_branches = C->n_branches;
  tn_status st = TN_OK;
  // after every plan's pending work (and the caller's stream) ...
  for (int i = 0; i < P && !st; ++i) {
    st = check(hipEventRecord(G->ev, G->plans[i]->stream), "event");
    if (!st) st = check(hipStreamWaitEvent(G->stream, G->ev, 0), "wait");
  }
  if (!st && G->user_stream) {
    st = check(hipEventRecord(G->ev, G->user_stream), "event");
    if (!st) st = check(hipStreamWaitEvent(G->stream, G->ev, 0), "wait");
  }
  if (!st) st = check(hipGraphLaunch(C->exec, G->stream), "graph launch");
  // ... and before anything later on those streams
  if (!st) st = check(hipEventRecord(G->ev, G->stream), "event");
  for (int i = 0; i < P && !st; ++i) st = check(hipStreamWaitEvent(G->plans[i]->stream, G->ev, 0), "wait");
  if (!st && G->user_stream) st = check(hipStreamWaitEvent(G->user_stream, G->ev, 0), "wait");
  if (st) return st;
  for (int i = 0; i < P; ++i) G->plans[i]->slices_acc += count[i];
  return TN_OK;
  TN_CATCH
}

tn_status tn_group_describe(tn_group G, int64_t* n_kernels, int32_t* n_branches) {
  TN_TRY
  if (!G) return fail(TN_E_ARG, "null group");
  if (n_kernels) *n_kernels = G->last_kernels;
  if (n_branches) *n_branches = G->last_branches;
  return TN_OK;
  TN_CATCH
}

void tn_group_destroy(tn_group G) {
  TN_TRY_VOID
  delete G;
  TN_CATCH_VOID
}

}  // extern "C"

namespace {

// The product C = A B of tn_gemm, planned as one contraction step with row-major
// operands (batch bits on top).
struct GemmPlan {
  tn_plan_s tmp;
  Step st;
  int bb = 0, mb = 0, nb = 0, kb = 0;
  size_t desc_bytes = 0, slot_bytes = 256, scratch_bytes = 0;
  size_t total_bytes() const { return desc_bytes + slot_bytes + scratch_bytes; }
};

tn_status gemm_plan(GemmPlan& G, int32_t precision, int64_t batch, int64_t m, int64_t n, int64_t k, const void* A,
                    const void* B, void* C) {
  G.bb = ilog2_exact(batch);
  G.mb = ilog2_exact(m);
  G.nb = ilog2_exact(n);
  G.kb = ilog2_exact(k);
  const int bb = G.bb, mb = G.mb, nb = G.nb, kb = G.kb;
  if (!A || !B || !C) return fail(TN_E_ARG, "null pointer");
  if (bb < 0 || mb < 0 || nb < 0 || kb < 0) return fail(TN_E_UNSUPPORTED, "dimensions must be powers of two");
  if (precision < 0 || precision > 2) return fail(TN_E_ARG, "unknown precision");
  if (bb > 16 || mb > 30 || nb > 30 || kb > 30 || bb + mb + nb > 34) return fail(TN_E_UNSUPPORTED, "too large");
  tn_plan_s& tmp = G.tmp;
  Step& st = G.st;
  tmp.precision = precision;
  tmp.opts.split_policy = 1;
  tmp.host_only = true;
  for (int j = 0; j < bb; ++j) st.bb.push_back(j);
  for (int j = 0; j < mb; ++j) st.mb.push_back(bb + j);
  for (int j = 0; j < nb; ++j) st.nb.push_back(bb + mb + j);
  for (int j = 0; j < kb; ++j) st.kb.push_back(bb + mb + nb + j);
  Tensor TA, TB, TC;
  TA.bits = st.kb;
  TA.bits.insert(TA.bits.end(), st.mb.begin(), st.mb.end());
  TA.bits.insert(TA.bits.end(), st.bb.begin(), st.bb.end());
  TB.bits = st.nb;
  TB.bits.insert(TB.bits.end(), st.kb.begin(), st.kb.end());
  TB.bits.insert(TB.bits.end(), st.bb.begin(), st.bb.end());
  TC.bits = st.nb;
  TC.bits.insert(TC.bits.end(), st.mb.begin(), st.mb.end());
  TC.bits.insert(TC.bits.end(), st.bb.begin(), st.bb.end());
  TA.elems = int64_t(1) << TA.bits.size();
  TB.elems = int64_t(1) << TB.bits.size();
  TC.elems = int64_t(1) << TC.bits.size();
  tmp.tensors = {TA, TB, TC};
  st.ta = 0;
  st.tb = 1;
  st.tc = 2;
  choose_kernel(&tmp, st);
  if (precision != 0 && st.kernel != (precision == 1 ? TN_K_MFMA_F16X3 : TN_K_MFMA_BF16X3)) {
    // keep the split arithmetic on every diagnostic problem
    st.kernel = precision == 1 ? TN_K_MFMA_F16X3 : TN_K_MFMA_BF16X3;
    set_tile(&tmp, st, mb >= 7 ? TN_TILE_128x64 : TN_TILE_64x64);
  }
  const char* tile_env = getenv("TN_GEMM_TILE");
  if (tile_env && st.kernel != TN_K_SMALL) set_tile(&tmp, st, atoi(tile_env) % TN_N_TILES);
  build_desc(&tmp, st);
  // device scratch: desc, max/exp slots, split partials
  G.desc_bytes = (sizeof(GettDesc) + 255) & ~size_t(255);
  G.scratch_bytes = st.kernel != TN_K_SMALL && st.splits > 1 ? (size_t)st.scratch_elems * 8 : 0;
  return TN_OK;
}

// Issue the product on stream s with `buf` (device, G.total_bytes()) as its scratch:
// the descriptor, the max / exponent slots (cleared by a fill kernel) and the K-split
// partials.  Asynchronous.
tn_status gemm_issue(const GemmPlan& G, int32_t precision, const void* A, const void* B, void* C, char* buf,
                     hipStream_t s) {
  const Step& st = G.st;
  const int bb = G.bb, mb = G.mb, nb = G.nb, kb = G.kb;
  const int64_t batch = int64_t(1) << bb, m = int64_t(1) << mb, n = int64_t(1) << nb, k = int64_t(1) << kb;
  GettDesc* dd = reinterpret_cast<GettDesc*>(buf);
  uint32_t* slots = reinterpret_cast<uint32_t*>(buf + G.desc_bytes);  // maxA maxB maxC expA expB expC
  tn_status r = check(hipMemcpyAsync(dd, &st.desc, sizeof(GettDesc), hipMemcpyHostToDevice, s), "desc");
  if (!r) r = check(tn_launch_fill_u32(slots, 0, (int64_t)(G.slot_bytes / 4), s), "slots");
  GettArgs g;
  memset(&g, 0, sizeof(g));
  g.A = reinterpret_cast<const float*>(A);
  g.B = reinterpret_cast<const float*>(B);
  g.C = reinterpret_cast<float*>(C);
  if (precision != 0) {
    if (!r) r = check(tn_launch_absmax(A, batch * m * k, slots + 0, s), "max A");
    if (!r) r = check(tn_launch_absmax(B, batch * k * n, slots + 1, s), "max B");
    g.scale_mode = 1;
    g.maxA = slots + 0;
    g.maxB = slots + 1;
    g.maxC = slots + 2;
    g.expA = reinterpret_cast<int32_t*>(slots + 3);
    g.expB = reinterpret_cast<int32_t*>(slots + 4);
    g.expC = reinterpret_cast<int32_t*>(slots + 5);
    g.target_exp = (st.kernel == TN_K_MFMA_F16X3 || st.kernel == TN_K_MFMA_BF16X3) ? 14 : 0;
    g.split_bf16 = precision == TN_PREC_BF16X3 ? 1 : 0;
  }
  const GettDesc* d = dd;
  if (!r) {
    if (st.kernel == TN_K_SMALL) {
      g.dot = st.dot ? 1 : 0;
      const int64_t outs = int64_t(1) << (bb + mb + nb);
      r = check(tn_launch_gett(TN_K_SMALL, 0, d, g, st.dot ? outs : (outs + 255) / 256, s), "gemm");
    } else {
      g.splits = st.splits;
      g.k_split_bits = st.k_split_bits;
      g.tiles_m_bits = st.tiles_m_bits;
      g.tiles_n_bits = st.tiles_n_bits;
      const int64_t blocks = int64_t(st.splits) << (st.tiles_m_bits + st.tiles_n_bits + bb);
      if (st.splits > 1) {
        g.scratch = reinterpret_cast<float*>(buf + G.desc_bytes + G.slot_bytes);
        g.write_scratch = 1;
        r = check(tn_launch_gett(st.kernel, st.tile, d, g, blocks, s), "gemm");
        g.write_scratch = 0;
        if (!r)
          r = check(tn_launch_gett(TN_K_SPLITK_REDUCE, 0, d, g, ((int64_t(1) << (bb + mb + nb)) + 255) / 256, s),
                    "gemm reduce");
      } else {
        r = check(tn_launch_gett(st.kernel, st.tile, d, g, blocks, s), "gemm");
      }
    }
  }
  if (!r && precision != 0)
    r = check(tn_launch_scale_pow2(C, batch * m * n, reinterpret_cast<int32_t*>(slots + 5), s), "rescale");
  return r;
}

}  // namespace

extern "C" {

tn_status tn_gemm(int32_t precision, int64_t batch, int64_t m, int64_t n, int64_t k, const void* A, const void* B,
                  void* C, void* stream) {
  TN_TRY
  GemmPlan G;
  tn_status r = gemm_plan(G, precision, batch, m, n, k, A, B, C);
  if (r) return r;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* buf = nullptr;
  if (hipMalloc((void**)&buf, G.total_bytes()) != hipSuccess) {
    hipGetLastError();
    return fail(TN_E_NOMEM, "scratch allocation failed");
  }
  r = gemm_issue(G, precision, A, B, C, buf, s);
  tn_status r2 = check(hipStreamSynchronize(s), "gemm sync");
  hipFree(buf);
  return r ? r : r2;
  TN_CATCH
}

}  // extern "C"

// Scratch of tn_gemm_noalloc.  Each GPU holds its own copy for the life of the process.
// Its host-side name is not a device address: host code uses only the address that
// hipGetSymbolAddress returns for the current device (noalloc_scratch below).
static __device__ __align__(256) char scratch[TN_GEMM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up on the first call
// made with that device current.
tn_status noalloc_scratch(char** out) {
  int dev = -1;
  tn_status r = check(hipGetDevice(&dev), "hipGetDevice");
  if (r) return r;
  if (dev < 0 || dev >= kMaxDevices) return fail(TN_E_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    r = check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch symbol address");
    if (r) return r;
    if (!p) return fail(TN_E_DEVICE, "scratch symbol has no device address");
    g_noalloc_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return TN_OK;
}

}  // namespace

extern "C" {

tn_status tn_gemm_noalloc(int32_t precision, int64_t batch, int64_t m, int64_t n, int64_t k, const void* A,
                          const void* B, void* C, void* stream) {
  TN_TRY
  GemmPlan G;
  tn_status r = gemm_plan(G, precision, batch, m, n, k, A, B, C);
  if (r) return r;
  if (G.total_bytes() > TN_GEMM_NOALLOC_SCRATCH_BYTES)
    return fail(TN_E_NOMEM, "tn_gemm_noalloc: the product needs " + std::to_string(G.total_bytes()) +
                                " bytes of scratch, more than the fixed " +
                                std::to_string((size_t)TN_GEMM_NOALLOC_SCRATCH_BYTES) + " bytes");
  char* buf = nullptr;
  r = noalloc_scratch(&buf);
  if (r) return r;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  r = gemm_issue(G, precision, A, B, C, buf, s);
  tn_status r2 = check(hipStreamSynchronize(s), "gemm sync");
  return r ? r : r2;
  TN_CATCH
}

tn_status tn_permute(int32_t rank, const int64_t* dims, const int32_t* perm, const void* in, void* out,
                     void* stream) {
  TN_TRY
  if (rank < 0 || rank > 32 || (rank > 0 && (!dims || !perm)) || !in || !out) return fail(TN_E_ARG, "bad arguments");
  std::vector<int> nb(rank), bit0(rank);
  int total = 0;
  for (int r = 0; r < rank; ++r) {
    nb[r] = ilog2_exact(dims[r]);
    if (nb[r] < 0) return fail(TN_E_UNSUPPORTED, "dims must be powers of two");
    bit0[r] = total;
    total += nb[r];
  }
  if (total > 40) return fail(TN_E_UNSUPPORTED, "tensor too large");
  std::vector<int> used(rank, 0);
  for (int r = 0; r < rank; ++r) {
    if (perm[r] < 0 || perm[r] >= rank || used[perm[r]]) return fail(TN_E_ARG, "perm is not a permutation");
    used[perm[r]] = 1;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // input position of (axis r, bit b): row-major, last axis least significant
  std::vector<int> in_pos(total), out_pos(total);
  int pos = 0;
  for (int r = rank - 1; r >= 0; --r)
    for (int b = 0; b < nb[r]; ++b) in_pos[bit0[r] + b] = pos++;
  pos = 0;
  for (int r = rank - 1; r >= 0; --r) {
    const int ax = perm[r];
    for (int b = 0; b < nb[ax]; ++b) out_pos[bit0[ax] + b] = pos++;
  }
  if (total == 0) {
    tn_status r = check(hipMemcpyAsync(out, in, 8, hipMemcpyDeviceToDevice, s), "copy");
    tn_status r2 = check(hipStreamSynchronize(s), "sync");
    return r ? r : r2;
  }
  PermDesc* d = nullptr;
  if (hipMalloc((void**)&d, sizeof(PermDesc)) != hipSuccess) {
    hipGetLastError();
    return fail(TN_E_NOMEM, "desc allocation failed");
  }
  tn_status r = permute_bits(in_pos, out_pos, in, out, s, d);
  hipFree(d);
  return r;
  TN_CATCH
}

}  // extern "C"
