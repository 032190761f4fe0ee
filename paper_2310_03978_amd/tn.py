"""ctypes binding of the C ABI in include/tn.h (argument marshalling only).

Every contraction step runs in the HIP library ``_lib/libtnmi.so``; nothing
here computes amplitudes.  Importing this module raises ImportError when the
library has not been built, so a missing extension fails loudly instead of
falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# One HIP runtime per process: torch ships its own libamdhip64.so.7.  Loaded first, it
# satisfies the library's dependency on that soname; loaded after the library, a second
# runtime would come in beside /opt/rocm's and the two would not share devices' state.
try:
    import torch  # noqa: F401
except ImportError:
    pass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libtnmi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                      "(run __graft_entry__.build() or python paper_2310_03978_amd/build.py)")

_lib = ctypes.CDLL(LIB_PATH)

TN_PREC_C64, TN_PREC_F16X3, TN_PREC_BF16X3 = 0, 1, 2
PRECISIONS = {"c64": TN_PREC_C64, "f16x3": TN_PREC_F16X3, "bf16x3": TN_PREC_BF16X3}

STATUS = {0: "TN_OK", -1: "TN_E_ARG", -2: "TN_E_LABEL", -3: "TN_E_PATH", -4: "TN_E_SLICE",
          -5: "TN_E_CAP", -6: "TN_E_NOMEM", -7: "TN_E_DEVICE", -8: "TN_E_STATE",
          -9: "TN_E_UNSUPPORTED", -10: "TN_E_NUMERIC"}

EXPORTED = ["tn_plan_create", "tn_plan_create_sparse", "tn_plan_sparse_index", "tn_plan_destroy", "tn_plan_describe", "tn_plan_steps",
            "tn_plan_step_times", "tn_contract_slices", "tn_slice_partials", "tn_amplitudes", "tn_accumulator_set",
            "tn_reset", "tn_group_create", "tn_group_contract", "tn_group_prepare", "tn_group_describe",
            "tn_group_destroy", "tn_plan_step_features", "tn_plan_set_tile", "tn_plan_set_step_terms",
            "tn_plan_tune_with_model", "tn_plan_rank_split_steps", "tn_plan_choose_single_products",
            "tn_plan_xeb", "tn_costmodel_create", "tn_costmodel_destroy",
            "tn_costmodel_describe", "tn_costmodel_set_normalization", "tn_costmodel_get_params",
            "tn_costmodel_set_params", "tn_costmodel_predict", "tn_costmodel_gradient",
            "tn_costmodel_adam_step", "tn_costmodel_train", "tn_costmodel_predict_shapes", "tn_gemm", "tn_gemm_noalloc", "tn_permute",
            "tn_status_string", "tn_last_error_message"]

TN_COST_FEATURES = 29
TN_N_TILE_SHAPES = 4


class TnError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class tn_options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("mem_cap_elems", ctypes.c_int64), ("stream", ctypes.c_void_p),
                ("slice_batch", ctypes.c_int32), ("host_only", ctypes.c_int32),
                ("split_policy", ctypes.c_int32), ("record_steps", ctypes.c_int32),
                ("tuning", ctypes.c_int32), ("deterministic", ctypes.c_int32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_int64),
                ("tuning_cache", ctypes.c_char_p), ("cost_model", ctypes.c_void_p)]


class tn_plan_info(ctypes.Structure):
    _fields_ = [("n_slices", ctypes.c_int64), ("n_amplitudes", ctypes.c_int64),
                ("n_steps", ctypes.c_int32), ("n_slice_steps", ctypes.c_int32),
                ("flops_per_slice", ctypes.c_double), ("flops_invariant", ctypes.c_double),
                ("bytes_per_slice", ctypes.c_double), ("bytes_invariant", ctypes.c_double),
                ("max_intermediate", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("slice_batch", ctypes.c_int32), ("precision", ctypes.c_int32)]


class tn_xeb_stats(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int64), ("sum_p", ctypes.c_double), ("sum_p2", ctypes.c_double),
                ("mean_dp", ctypes.c_double), ("mean_dp2", ctypes.c_double), ("lxeb", ctypes.c_double)]


class tn_step_info(ctypes.Structure):
    _fields_ = [("slot_a", ctypes.c_int32), ("slot_b", ctypes.c_int32),
                ("per_slice", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("batch", ctypes.c_int64), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("k", ctypes.c_int64), ("split_k", ctypes.c_int32), ("tile_m", ctypes.c_int32),
                ("tile_n", ctypes.c_int32), ("a_contig", ctypes.c_int32),
                ("b_contig", ctypes.c_int32), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double), ("tile", ctypes.c_int32), ("lds_copy", ctypes.c_int32),
                ("terms", ctypes.c_int32), ("merged_bits", ctypes.c_int32),
                ("values_first", ctypes.c_int32)]


_P = ctypes.POINTER
_lib.tn_plan_create.argtypes = [_P(ctypes.c_void_p), ctypes.c_int32, _P(ctypes.c_int32),
                                _P(_P(ctypes.c_int32)), _P(_P(ctypes.c_int64)),
                                _P(_P(ctypes.c_double)), ctypes.c_int32, _P(ctypes.c_int32),
                                ctypes.c_int32, _P(ctypes.c_int32), ctypes.c_int32,
                                _P(ctypes.c_int32), _P(tn_options)]
_lib.tn_plan_create.restype = ctypes.c_int
_lib.tn_plan_create_sparse.argtypes = [_P(ctypes.c_void_p), ctypes.c_int32, _P(ctypes.c_int32),
                                       _P(_P(ctypes.c_int32)), _P(_P(ctypes.c_int64)),
                                       _P(_P(ctypes.c_double)), ctypes.c_int32, _P(ctypes.c_int32),
                                       ctypes.c_int32, _P(ctypes.c_int32), ctypes.c_int32,
                                       _P(ctypes.c_int32), ctypes.c_int64, _P(ctypes.c_uint8), _P(tn_options)]
_lib.tn_plan_create_sparse.restype = ctypes.c_int
_lib.tn_plan_sparse_index.argtypes = [ctypes.c_void_p, _P(ctypes.c_int64), ctypes.c_int64]
_lib.tn_plan_sparse_index.restype = ctypes.c_int
_lib.tn_plan_destroy.argtypes = [ctypes.c_void_p]
_lib.tn_plan_destroy.restype = None
_lib.tn_plan_describe.argtypes = [ctypes.c_void_p, _P(tn_plan_info)]
_lib.tn_plan_describe.restype = ctypes.c_int
_lib.tn_plan_steps.argtypes = [ctypes.c_void_p, _P(tn_step_info), ctypes.c_int32]
_lib.tn_plan_steps.restype = ctypes.c_int
_lib.tn_plan_step_times.argtypes = [ctypes.c_void_p, _P(ctypes.c_double), _P(ctypes.c_int64),
                                    ctypes.c_int32]
_lib.tn_plan_step_times.restype = ctypes.c_int
_lib.tn_contract_slices.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64]
_lib.tn_contract_slices.restype = ctypes.c_int
_lib.tn_slice_partials.argtypes = [ctypes.c_void_p, _P(ctypes.c_int64), ctypes.c_int64,
                                   _P(ctypes.c_double)]
_lib.tn_slice_partials.restype = ctypes.c_int
_lib.tn_amplitudes.argtypes = [ctypes.c_void_p, _P(ctypes.c_double), ctypes.c_int64,
                               _P(ctypes.c_int64)]
_lib.tn_amplitudes.restype = ctypes.c_int
_lib.tn_plan_xeb.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                             _P(tn_xeb_stats), _P(ctypes.c_int64)]
_lib.tn_plan_xeb.restype = ctypes.c_int
_lib.tn_accumulator_set.argtypes = [ctypes.c_void_p, _P(ctypes.c_double), ctypes.c_int64,
                                    ctypes.c_int64]
_lib.tn_accumulator_set.restype = ctypes.c_int
_lib.tn_reset.argtypes = [ctypes.c_void_p]
_lib.tn_reset.restype = ctypes.c_int
_lib.tn_group_create.argtypes = [_P(ctypes.c_void_p), _P(ctypes.c_void_p), ctypes.c_int32,
                                 _P(tn_options)]
_lib.tn_group_create.restype = ctypes.c_int
_lib.tn_group_contract.argtypes = [ctypes.c_void_p, _P(ctypes.c_int64), _P(ctypes.c_int64)]
_lib.tn_group_contract.restype = ctypes.c_int
_lib.tn_group_prepare.argtypes = [ctypes.c_void_p, _P(ctypes.c_int64), _P(ctypes.c_int64)]
_lib.tn_group_prepare.restype = ctypes.c_int
_lib.tn_group_describe.argtypes = [ctypes.c_void_p, _P(ctypes.c_int64), _P(ctypes.c_int32)]
_lib.tn_group_describe.restype = ctypes.c_int
_lib.tn_group_destroy.argtypes = [ctypes.c_void_p]
_lib.tn_group_destroy.restype = None
_F32P = _P(ctypes.c_float)
_lib.tn_plan_step_features.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, _F32P,
                                       ctypes.c_int32]
_lib.tn_plan_step_features.restype = ctypes.c_int
_lib.tn_plan_set_tile.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
_lib.tn_plan_set_tile.restype = ctypes.c_int
_lib.tn_plan_set_step_terms.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
_lib.tn_plan_set_step_terms.restype = ctypes.c_int
_lib.tn_plan_tune_with_model.argtypes = [ctypes.c_void_p, ctypes.c_void_p, _F32P, ctypes.c_int32]
_lib.tn_plan_tune_with_model.restype = ctypes.c_int
_lib.tn_plan_rank_split_steps.argtypes = [ctypes.c_void_p, ctypes.c_int32, _P(ctypes.c_int32), ctypes.c_int32,
                                          _P(ctypes.c_int32)]
_lib.tn_plan_rank_split_steps.restype = ctypes.c_int
_lib.tn_plan_choose_single_products.argtypes = [ctypes.c_void_p, ctypes.c_double, _P(ctypes.c_int64),
                                                ctypes.c_int64, _P(ctypes.c_int32), _P(ctypes.c_double)]
_lib.tn_plan_choose_single_products.restype = ctypes.c_int
_lib.tn_costmodel_create.argtypes = [_P(ctypes.c_void_p), ctypes.c_int32, ctypes.c_uint64]
_lib.tn_costmodel_create.restype = ctypes.c_int
_lib.tn_costmodel_destroy.argtypes = [ctypes.c_void_p]
_lib.tn_costmodel_destroy.restype = None
_lib.tn_costmodel_describe.argtypes = [ctypes.c_void_p, _P(ctypes.c_int32), _P(ctypes.c_int32),
                                       _P(ctypes.c_int64)]
_lib.tn_costmodel_describe.restype = ctypes.c_int
_lib.tn_costmodel_set_normalization.argtypes = [ctypes.c_void_p, _F32P, _F32P]
_lib.tn_costmodel_set_normalization.restype = ctypes.c_int
_lib.tn_costmodel_get_params.argtypes = [ctypes.c_void_p, _F32P, ctypes.c_int64]
_lib.tn_costmodel_get_params.restype = ctypes.c_int
_lib.tn_costmodel_set_params.argtypes = [ctypes.c_void_p, _F32P, ctypes.c_int64]
_lib.tn_costmodel_set_params.restype = ctypes.c_int
_lib.tn_costmodel_predict.argtypes = [ctypes.c_void_p, _F32P, ctypes.c_int64, _F32P]
_lib.tn_costmodel_predict.restype = ctypes.c_int
_lib.tn_costmodel_predict_shapes.argtypes = [ctypes.c_void_p, ctypes.c_int32, _P(ctypes.c_int32), ctypes.c_int64,
                                              _F32P]
_lib.tn_costmodel_predict_shapes.restype = ctypes.c_int
_lib.tn_costmodel_gradient.argtypes = [ctypes.c_void_p, _F32P, _F32P, ctypes.c_int64, _F32P, _F32P]
_lib.tn_costmodel_gradient.restype = ctypes.c_int
_lib.tn_costmodel_adam_step.argtypes = [ctypes.c_void_p, _F32P, ctypes.c_int64, ctypes.c_float]
_lib.tn_costmodel_adam_step.restype = ctypes.c_int
_lib.tn_costmodel_train.argtypes = [ctypes.c_void_p, _F32P, _F32P, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_float, ctypes.c_uint64, _F32P]
_lib.tn_costmodel_train.restype = ctypes.c_int
_lib.tn_gemm.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                         ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                         ctypes.c_void_p]
_lib.tn_gemm.restype = ctypes.c_int
_lib.tn_gemm_noalloc.argtypes = _lib.tn_gemm.argtypes
_lib.tn_gemm_noalloc.restype = ctypes.c_int
_lib.tn_permute.argtypes = [ctypes.c_int32, _P(ctypes.c_int64), _P(ctypes.c_int32),
                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
_lib.tn_permute.restype = ctypes.c_int
_lib.tn_status_string.argtypes = [ctypes.c_int]
_lib.tn_status_string.restype = ctypes.c_char_p
_lib.tn_last_error_message.argtypes = []
_lib.tn_last_error_message.restype = ctypes.c_char_p


def _check(status: int):
    if status != 0:
        raise TnError(status, _lib.tn_last_error_message().decode())


def exported_symbols() -> list:
    return [name for name in EXPORTED if hasattr(_lib, name)]


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def tn_plan_create(tensors, labels, open_labels, path, sliced_labels=(), precision="c64",
                   mem_cap_elems: int = 0, stream=None, slice_batch: int = 0,
                   host_only: bool = False, split_policy: int = 0, record_steps: bool = False,
                   tuning: int = 0, workspace=None, bitstrings=None, tuning_cache=None,
                   cost_model=None, deterministic: int = 1):
    """Create a plan; returns an opaque handle (int).  Leaves are copied.  With bitstrings
    (uint8 [count, n_open]) a sparse-state plan (tn_plan_create_sparse).  tuning = 2 takes
    the tiles from cost_model (a model handle)."""
    n = len(labels)
    ranks = (ctypes.c_int32 * n)(*[len(l) for l in labels])
    lab_arrays = [(ctypes.c_int32 * max(len(l), 1))(*l) for l in labels]
    if tensors is None:
        shapes = None
    else:
        shapes = [tuple(np.shape(t)) for t in tensors]
    ext_arrays = []
    for t, l in enumerate(labels):
        if shapes is not None:
            ext = shapes[t]
        else:
            raise ValueError("tensors are required to know the extents")
        ext_arrays.append((ctypes.c_int64 * max(len(l), 1))(*ext))
    lab_pp = (_P(ctypes.c_int32) * n)(*[ctypes.cast(a, _P(ctypes.c_int32)) for a in lab_arrays])
    ext_pp = (_P(ctypes.c_int64) * n)(*[ctypes.cast(a, _P(ctypes.c_int64)) for a in ext_arrays])
    keep = []
    if host_only:
        data_pp = None
    else:
        arrs = [np.ascontiguousarray(np.asarray(t, dtype=np.complex128)).view(np.float64)
                for t in tensors]
        keep = arrs
        data_pp = (_P(ctypes.c_double) * n)(*[a.ctypes.data_as(_P(ctypes.c_double)) for a in arrs])
    op = (ctypes.c_int32 * max(len(open_labels), 1))(*open_labels)
    flat = [x for pair in path for x in pair]
    pa = (ctypes.c_int32 * max(len(flat), 1))(*flat)
    sl = (ctypes.c_int32 * max(len(sliced_labels), 1))(*sliced_labels)
    opts = tn_options()
    opts.struct_size = ctypes.sizeof(tn_options)
    opts.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    opts.mem_cap_elems = int(mem_cap_elems)
    opts.stream = _stream_handle(stream)
    opts.slice_batch = int(slice_batch)
    opts.host_only = 1 if host_only else 0
    opts.split_policy = int(split_policy)
    opts.record_steps = 1 if record_steps else 0
    opts.tuning = int(tuning)
    opts.deterministic = int(deterministic)
    opts.tuning_cache = None if tuning_cache is None else os.fsencode(tuning_cache)
    opts.cost_model = cost_model
    if workspace is not None:   # a device tensor: its memory, caller-owned
        opts.workspace = int(workspace.data_ptr())
        opts.workspace_bytes = int(workspace.numel() * workspace.element_size())
    handle = ctypes.c_void_p()
    if bitstrings is None:
        status = _lib.tn_plan_create(ctypes.byref(handle), n, ranks, lab_pp, ext_pp, data_pp,
                                     len(open_labels), op, len(path), pa, len(sliced_labels), sl,
                                     ctypes.byref(opts))
    else:
        bits = np.ascontiguousarray(np.asarray(bitstrings, dtype=np.uint8))
        if bits.ndim != 2 or bits.shape[1] != len(open_labels):
            raise ValueError("bitstrings must be (count, n_open)")
        keep.append(bits)
        status = _lib.tn_plan_create_sparse(ctypes.byref(handle), n, ranks, lab_pp, ext_pp, data_pp,
                                            len(open_labels), op, len(path), pa, len(sliced_labels), sl,
                                            bits.shape[0], bits.ctypes.data_as(_P(ctypes.c_uint8)),
                                            ctypes.byref(opts))
    del keep
    _check(status)
    return handle.value


def tn_plan_destroy(plan):
    _lib.tn_plan_destroy(plan)


def tn_plan_sparse_index(plan, n_bitstrings: int) -> np.ndarray:
    idx = np.zeros(max(int(n_bitstrings), 1), dtype=np.int64)
    _check(_lib.tn_plan_sparse_index(plan, idx.ctypes.data_as(_P(ctypes.c_int64)), int(n_bitstrings)))
    return idx[:n_bitstrings]


def tn_plan_describe(plan) -> dict:
    info = tn_plan_info()
    _check(_lib.tn_plan_describe(plan, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in tn_plan_info._fields_}


def tn_plan_steps(plan) -> list:
    n = tn_plan_describe(plan)["n_steps"]
    arr = (tn_step_info * max(n, 1))()
    _check(_lib.tn_plan_steps(plan, arr, n))
    return [{name: getattr(arr[i], name) for name, _ in tn_step_info._fields_} for i in range(n)]


def tn_plan_step_times(plan):
    """(ms_total, launches) numpy arrays per step, recorded since the last call."""
    n = tn_plan_describe(plan)["n_steps"]
    ms = np.zeros(max(n, 1), dtype=np.float64)
    cnt = np.zeros(max(n, 1), dtype=np.int64)
    _check(_lib.tn_plan_step_times(plan, ms.ctypes.data_as(_P(ctypes.c_double)),
                                   cnt.ctypes.data_as(_P(ctypes.c_int64)), n))
    return ms[:n], cnt[:n]


def tn_contract_slices(plan, first_slice: int, n_slices: int):
    _check(_lib.tn_contract_slices(plan, int(first_slice), int(n_slices)))


def tn_slice_partials(plan, slice_ids) -> np.ndarray:
    ids = np.ascontiguousarray(np.asarray(slice_ids, dtype=np.int64))
    n_amp = tn_plan_describe(plan)["n_amplitudes"]
    out = np.zeros((len(ids), n_amp), dtype=np.complex128)
    _check(_lib.tn_slice_partials(plan, ids.ctypes.data_as(_P(ctypes.c_int64)), len(ids),
                                  out.view(np.float64).ctypes.data_as(_P(ctypes.c_double))))
    return out


def tn_amplitudes(plan):
    n_amp = tn_plan_describe(plan)["n_amplitudes"]
    out = np.zeros(n_amp, dtype=np.complex128)
    count = ctypes.c_int64()
    _check(_lib.tn_amplitudes(plan, out.view(np.float64).ctypes.data_as(_P(ctypes.c_double)),
                              n_amp, ctypes.byref(count)))
    return out, count.value


def tn_plan_xeb(plan, n_qubits: int, n_bins: int = 0, x_lo: float = -6.0, x_hi: float = 3.0):
    """(stats dict, histogram int64 array) of the accumulated amplitudes (tn_plan_xeb)."""
    st = tn_xeb_stats()
    hist = np.zeros(max(int(n_bins), 1), dtype=np.int64)
    _check(_lib.tn_plan_xeb(plan, int(n_qubits), int(n_bins), float(x_lo), float(x_hi), ctypes.byref(st),
                            hist.ctypes.data_as(_P(ctypes.c_int64)) if n_bins > 0 else None))
    return {name: getattr(st, name) for name, _ in tn_xeb_stats._fields_}, hist[:n_bins]


def tn_accumulator_set(plan, acc, slices_accumulated: int):
    acc = np.ascontiguousarray(np.asarray(acc, dtype=np.complex128))
    _check(_lib.tn_accumulator_set(plan, acc.view(np.float64).ctypes.data_as(_P(ctypes.c_double)),
                                   acc.size, int(slices_accumulated)))


def tn_reset(plan):
    _check(_lib.tn_reset(plan))


def tn_group_create(plans, stream=None, branches: int = 0):
    """Group plan handles; each tn_group_contract call replays one captured graph."""
    arr = (ctypes.c_void_p * len(plans))(*plans)
    opts = tn_options()
    opts.struct_size = ctypes.sizeof(tn_options)
    opts.stream = _stream_handle(stream)
    opts.slice_batch = int(branches)
    handle = ctypes.c_void_p()
    _check(_lib.tn_group_create(ctypes.byref(handle), arr, len(plans), ctypes.byref(opts)))
    return handle.value


def tn_group_contract(group, first, count):
    f = (ctypes.c_int64 * len(first))(*[int(x) for x in first])
    c = (ctypes.c_int64 * len(count))(*[int(x) for x in count])
    _check(_lib.tn_group_contract(group, f, c))


def tn_group_prepare(group, first, count):
    f = (ctypes.c_int64 * len(first))(*[int(x) for x in first])
    c = (ctypes.c_int64 * len(count))(*[int(x) for x in count])
    _check(_lib.tn_group_prepare(group, f, c))


def tn_group_describe(group) -> dict:
    nk, nb = ctypes.c_int64(), ctypes.c_int32()
    _check(_lib.tn_group_describe(group, ctypes.byref(nk), ctypes.byref(nb)))
    return {"n_kernels": nk.value, "n_branches": nb.value}


def tn_group_destroy(group):
    _lib.tn_group_destroy(group)


class Group:
    """Owning wrapper around a group of plans (the plans must outlive it)."""

    handle = None

    def __init__(self, plans, stream=None, branches: int = 0):
        self.plans = list(plans)
        self.handle = tn_group_create([p.handle for p in self.plans], stream, branches)

    def _ranges(self, first, count):
        if first is None:
            first = [0] * len(self.plans)
        if count is None:
            count = [p.describe()["n_slices"] - f for p, f in zip(self.plans, first)]
        return first, count

    def contract(self, first=None, count=None):
        tn_group_contract(self.handle, *self._ranges(first, count))

    def prepare(self, first=None, count=None):
        """Capture the graph of these ranges without launching it (a later contract replays)."""
        tn_group_prepare(self.handle, *self._ranges(first, count))

    def describe(self):
        return tn_group_describe(self.handle)

    def close(self):
        if self.handle:
            tn_group_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _f32(x, shape=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    if shape is not None and a.shape != shape:
        a = a.reshape(shape)
    return a


def _fp(a):
    return a.ctypes.data_as(_F32P)


def tn_plan_step_features(plan, step: int, tile: int = -1) -> np.ndarray:
    out = np.zeros(TN_COST_FEATURES, dtype=np.float32)
    _check(_lib.tn_plan_step_features(plan, int(step), int(tile), _fp(out), TN_COST_FEATURES))
    return out


def tn_plan_set_tile(plan, step: int, tile: int):
    _check(_lib.tn_plan_set_tile(plan, int(step), int(tile)))


def tn_plan_set_step_terms(plan, step: int, terms: int):
    _check(_lib.tn_plan_set_step_terms(plan, int(step), int(terms)))


def tn_plan_rank_split_steps(plan, by_time: bool) -> list:
    n = tn_plan_describe(plan)["n_steps"]
    order = (ctypes.c_int32 * max(n, 1))()
    count = ctypes.c_int32()
    _check(_lib.tn_plan_rank_split_steps(plan, 1 if by_time else 0, order, n, ctypes.byref(count)))
    return [int(order[i]) for i in range(count.value)]


def tn_plan_choose_single_products(plan, budget: float, slice_ids):
    """(k, eps_l2sq): the plan keeps single products on its top k split steps."""
    ids = np.ascontiguousarray(np.asarray(slice_ids, dtype=np.int64))
    k, eps = ctypes.c_int32(), ctypes.c_double()
    _check(_lib.tn_plan_choose_single_products(plan, float(budget), ids.ctypes.data_as(_P(ctypes.c_int64)),
                                               len(ids), ctypes.byref(k), ctypes.byref(eps)))
    return k.value, eps.value


def tn_plan_tune_with_model(plan, model) -> np.ndarray:
    n = tn_plan_describe(plan)["n_steps"]
    out = np.zeros(max(n, 1), dtype=np.float32)
    _check(_lib.tn_plan_tune_with_model(plan, model, _fp(out), n))
    return out[:n]


def tn_costmodel_create(n_features: int, seed: int = 0):
    handle = ctypes.c_void_p()
    _check(_lib.tn_costmodel_create(ctypes.byref(handle), int(n_features), int(seed)))
    return handle.value


def tn_costmodel_destroy(model):
    _lib.tn_costmodel_destroy(model)


def tn_costmodel_describe(model):
    f, h, p = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(_lib.tn_costmodel_describe(model, ctypes.byref(f), ctypes.byref(h), ctypes.byref(p)))
    return f.value, h.value, p.value


def tn_costmodel_set_normalization(model, mean, std):
    m, s = _f32(mean), _f32(std)
    _check(_lib.tn_costmodel_set_normalization(model, _fp(m), _fp(s)))


def tn_costmodel_get_params(model, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.float32)
    _check(_lib.tn_costmodel_get_params(model, _fp(out), n))
    return out


def tn_costmodel_set_params(model, theta):
    t = _f32(theta)
    _check(_lib.tn_costmodel_set_params(model, _fp(t), t.size))


def tn_costmodel_predict(model, X) -> np.ndarray:
    X = _f32(X)
    n = X.shape[0] if X.ndim == 2 else 0
    y = np.zeros(max(n, 1), dtype=np.float32)
    _check(_lib.tn_costmodel_predict(model, _fp(X), n, _fp(y)))
    return y[:n]


def tn_costmodel_predict_shapes(model, precision, shapes) -> np.ndarray:
    """Predicted microseconds per launch of canonical steps; shapes: (n, 4) ints (b, m, n, k bits)."""
    sh = np.ascontiguousarray(np.asarray(shapes, dtype=np.int32).reshape(-1, 4))
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    n = sh.shape[0]
    us = np.zeros(max(n, 1), dtype=np.float32)
    _check(_lib.tn_costmodel_predict_shapes(model, prec, sh.ctypes.data_as(_P(ctypes.c_int32)), n, _fp(us)))
    return us[:n]


def tn_costmodel_gradient(model, X, t):
    X, t = _f32(X), _f32(t)
    _, _, n_params = tn_costmodel_describe(model)
    g = np.zeros(n_params, dtype=np.float32)
    loss = ctypes.c_float()
    _check(_lib.tn_costmodel_gradient(model, _fp(X), _fp(t), X.shape[0], _fp(g), ctypes.byref(loss)))
    return g, float(loss.value)


def tn_costmodel_adam_step(model, grad, lr: float):
    g = _f32(grad)
    _check(_lib.tn_costmodel_adam_step(model, _fp(g), g.size, float(lr)))


def tn_costmodel_train(model, X, t, epochs: int, batch: int, lr: float, seed: int = 0) -> float:
    X, t = _f32(X), _f32(t)
    loss = ctypes.c_float()
    _check(_lib.tn_costmodel_train(model, _fp(X), _fp(t), X.shape[0], int(epochs), int(batch),
                                   float(lr), int(seed), ctypes.byref(loss)))
    return float(loss.value)


def tn_gemm(A, B, C, precision="c64", stream=None, noalloc=False):
    """C[b] = A[b] @ B[b] on device complex64 torch tensors of shape (b, m, k), (b, k, n), (b, m, n).

    noalloc=True calls tn_gemm_noalloc: the same product with the library's fixed per-device
    scratch array instead of an allocation (TN_GEMM_NOALLOC_SCRATCH_BYTES at most)."""
    b, m, k = A.shape
    n = B.shape[2]
    if tuple(B.shape) != (b, k, n) or tuple(C.shape) != (b, m, n):
        raise ValueError("shape mismatch")
    for x in (A, B, C):
        if not x.is_contiguous() or str(x.dtype) != "torch.complex64" or x.device.type != "cuda":
            raise ValueError("operands must be contiguous complex64 device tensors")
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    fn = _lib.tn_gemm_noalloc if noalloc else _lib.tn_gemm
    _check(fn(prec, b, m, n, k, A.data_ptr(), B.data_ptr(), C.data_ptr(), _stream_handle(stream)))


def tn_permute(x, perm, out, stream=None):
    """out = x.permute(perm) (contiguous) on device complex64 torch tensors."""
    rank = x.dim()
    if out.numel() != x.numel() or not x.is_contiguous() or not out.is_contiguous():
        raise ValueError("bad tensors")
    dims = (ctypes.c_int64 * max(rank, 1))(*x.shape)
    pm = (ctypes.c_int32 * max(rank, 1))(*perm)
    _check(_lib.tn_permute(rank, dims, pm, x.data_ptr(), out.data_ptr(), _stream_handle(stream)))


class Plan:
    """Owning wrapper around a plan handle.

    tuning: 0 = tile shapes from the shape heuristic, 1 = measured autotuning at creation,
    2 = tiles chosen by a learned step-time model (all in the library); for tuning = 2 the
    model is ``cost_model`` (a CostModel or handle) or, when none is given, the model shipped
    with the package."""

    handle = None
    sparse_index = None

    def __init__(self, tensors, labels, open_labels, path, sliced_labels=(), **kw):
        self.workspace = kw.get("workspace")   # kept alive for the plan's lifetime
        shipped = None
        if kw.get("tuning", 0) == 2:
            model = kw.get("cost_model")
            if model is None:
                from .costmodel import CostModel
                shipped = model = CostModel.load()
            kw["cost_model"] = getattr(model, "handle", model)
        try:
            self.handle = tn_plan_create(tensors, labels, open_labels, path, sliced_labels, **kw)
        finally:
            if shipped is not None:
                shipped.close()
        bits = kw.get("bitstrings")
        self.sparse_index = None if bits is None else tn_plan_sparse_index(self.handle, len(bits))

    def close(self):
        if self.handle:
            tn_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def describe(self):
        return tn_plan_describe(self.handle)

    def steps(self):
        return tn_plan_steps(self.handle)

    def contract(self, first=0, n=None):
        if n is None:
            n = self.describe()["n_slices"] - first
        tn_contract_slices(self.handle, first, n)

    def amplitudes(self):
        """(amplitudes, slices accumulated); for a sparse-state plan one amplitude per
        bitstring, in the order given."""
        amps, count = tn_amplitudes(self.handle)
        if self.sparse_index is not None:
            amps = amps[self.sparse_index]
        return amps, count

    def step_times(self):
        return tn_plan_step_times(self.handle)

    def xeb(self, n_qubits, n_bins=0, x_lo=-6.0, x_hi=3.0):
        """LXEB statistics and the Porter-Thomas histogram of the accumulated amplitudes."""
        return tn_plan_xeb(self.handle, n_qubits, n_bins, x_lo, x_hi)

    def partials(self, ids):
        out = tn_slice_partials(self.handle, ids)
        if self.sparse_index is not None:
            out = out[:, self.sparse_index]
        return out

    def reset(self):
        tn_reset(self.handle)

    def set_accumulator(self, acc, slices):
        tn_accumulator_set(self.handle, acc, slices)

    def step_features(self, step, tile=-1):
        return tn_plan_step_features(self.handle, step, tile)

    def set_tile(self, step, tile):
        tn_plan_set_tile(self.handle, step, tile)

    def set_step_terms(self, step, terms):
        tn_plan_set_step_terms(self.handle, step, terms)

    def rank_split_steps(self, by_time=True):
        """Split steps costliest first (measured time, or flops per contraction)."""
        return tn_plan_rank_split_steps(self.handle, by_time)

    def single_product_top(self, k, by_time=True):
        """Run the top k split steps of the library's ranking as hi*hi only, the others as
        three products; returns their indices."""
        order = self.rank_split_steps(by_time)
        for i, s in enumerate(order):
            tn_plan_set_step_terms(self.handle, s, 1 if i < k else 3)
        return order[:k]

    def choose_single_products(self, budget, slice_ids):
        """Largest top-k set of single-product steps under an epsilon_L2^2 budget: (k, eps)."""
        return tn_plan_choose_single_products(self.handle, budget, slice_ids)

    def tune_with_model(self, model):
        """Tile every MFMA step by the model's predicted time; returns predicted us per step."""
        return tn_plan_tune_with_model(self.handle, getattr(model, "handle", model))
