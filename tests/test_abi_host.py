"""Host-side tests of the C ABI: symbols, planner output and error codes (no GPU needed)."""
import os
import re

import numpy as np
import pytest

from oracle import contract
from tn_inputs import configs
from tn_inputs.network import random_network
from tn_inputs.paths import greedy_path

tn = pytest.importorskip("paper_2310_03978_amd.tn")

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "tn.h")


def test_library_exports_every_declared_symbol():
    text = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:tn_status|void|const char\*)\s+(tn_\w+)\(", text, re.M))
    assert len(declared) >= 13
    missing = [name for name in declared if not hasattr(tn._lib, name)]
    assert not missing, missing


def _host_plan(net, path, sliced=(), **kw):
    return tn.tn_plan_create(net.tensors, net.labels, net.open_labels, path, sliced,
                             host_only=True, **kw)


def _compare_costs(net, path, sliced):
    h = _host_plan(net, path, sliced)
    try:
        steps = tn.tn_plan_steps(h)
        info = tn.tn_plan_describe(h)
    finally:
        tn.tn_plan_destroy(h)
    ref = contract.step_costs(net.tensors, net.labels, net.open_labels, path, sliced)
    assert len(steps) == len(ref)
    for s, r in zip(steps, ref):
        assert (s["batch"], s["m"], s["n"], s["k"]) == (r["B"], r["M"], r["N"], r["K"])
        assert s["flops"] == r["flops"]
        assert s["bytes"] == r["bytes"]
    ps = sum(s["flops"] for s in steps if s["per_slice"])
    inv = sum(s["flops"] for s in steps if not s["per_slice"])
    assert info["flops_per_slice"] == ps and info["flops_invariant"] == inv
    return info, steps


def test_planner_costs_match_oracle_rqc12():
    circ, net, best = configs.build("rqc12")
    info, steps = _compare_costs(net, best["path"], ())
    assert info["n_slices"] == 1 and info["n_amplitudes"] == 16
    assert info["n_steps"] == len(net.tensors) - 1


def test_planner_costs_match_oracle_rqc30():
    circ, net, best = configs.build("rqc30")
    info, steps = _compare_costs(net, best["path"], best["sliced"])
    assert info["n_slices"] == 256 and info["n_amplitudes"] == 64
    assert info["max_intermediate"] <= 2 ** 28
    # the slice-dependent steps are the ones that touch a sliced leaf
    assert 0 < info["n_slice_steps"] < info["n_steps"]


@pytest.mark.parametrize("seed", range(6))
def test_planner_costs_match_oracle_random(seed):
    net = random_network(seed, n_tensors=6, n_labels=10, extents=(1, 2, 4), n_open=2)
    path = greedy_path(net.labels, net.open_labels, net.extents(), seed=seed)
    ext = net.extents()
    sliced = [l for l in sorted(ext) if l not in net.open_labels and ext[l] > 1][:1]
    _compare_costs(net, path, sliced)


def test_single_tensor_plan():
    x = np.arange(8, dtype=np.complex128).reshape(2, 4)
    h = tn.tn_plan_create([x], [(3, 5)], (5,), [], (), host_only=True)
    info = tn.tn_plan_describe(h)
    tn.tn_plan_destroy(h)
    assert info["n_steps"] == 1 and info["n_amplitudes"] == 4


def _expect(status, fn):
    with pytest.raises(tn.TnError) as e:
        fn()
    assert e.value.name == status, str(e.value)


def test_error_codes():
    a = np.zeros((2, 2), dtype=np.complex128)
    b = np.zeros((2, 2), dtype=np.complex128)
    c = np.zeros((2, 3), dtype=np.complex128)
    d = np.zeros((4,), dtype=np.complex128)
    mk = lambda *args, **kw: tn.tn_plan_create(*args, host_only=True, **kw)
    _expect("TN_E_LABEL", lambda: mk([a, b], [(0, -1), (1, 0)], (1,), [(0, 1)]))
    _expect("TN_E_LABEL", lambda: mk([a, d], [(0, 1), (1,)], (0,), [(0, 1)]))
    _expect("TN_E_LABEL", lambda: mk([a, b], [(0, 0), (1, 0)], (1,), [(0, 1)]))
    _expect("TN_E_LABEL", lambda: mk([a, b], [(0, 1), (1, 2)], (7,), [(0, 1)]))
    _expect("TN_E_UNSUPPORTED", lambda: mk([c, b], [(0, 1), (0, 2)], (2,), [(0, 1)]))
    _expect("TN_E_PATH", lambda: mk([a, b], [(0, 1), (1, 2)], (0, 2), []))
    _expect("TN_E_PATH", lambda: mk([a, b, a], [(0, 1), (1, 2), (2, 3)], (0, 3), [(0, 1), (1, 2)]))
    _expect("TN_E_PATH", lambda: mk([a, b], [(0, 1), (1, 2)], (0, 2), [(0, 0)]))
    _expect("TN_E_PATH", lambda: mk([a, b], [(0, 1), (1, 2)], (0, 2), [(0, 5)]))
    _expect("TN_E_SLICE", lambda: mk([a, b], [(0, 1), (1, 2)], (0, 2), [(0, 1)], (0,)))
    _expect("TN_E_SLICE", lambda: mk([a, b], [(0, 1), (1, 2)], (0, 2), [(0, 1)], (9,)))
    _expect("TN_E_SLICE", lambda: mk([a, b], [(0, 1), (1, 2)], (0, 2), [(0, 1)], (1, 1)))
    _expect("TN_E_CAP", lambda: mk([a, b], [(0, 1), (2, 3)], (0, 1, 2, 3), [(0, 1)],
                                   mem_cap_elems=8))
    _expect("TN_E_ARG", lambda: mk([a, b], [(0, 1), (1, 2)], (0, 2), [(0, 1)], slice_batch=3))
    h = mk([a, b], [(0, 1), (1, 2)], (0, 2), [(0, 1)])
    try:
        _expect("TN_E_STATE", lambda: tn.tn_contract_slices(h, 0, 1))
        _expect("TN_E_STATE", lambda: tn.tn_amplitudes(h))
    finally:
        tn.tn_plan_destroy(h)


def test_status_strings():
    for code, name in tn.STATUS.items():
        assert tn._lib.tn_status_string(code).decode() == name


def test_step_features_describe_the_step_and_tile():
    circ, net, best = configs.build("rqc30")
    h = _host_plan(net, best["path"], best["sliced"], precision="f16x3")
    try:
        steps = tn.tn_plan_steps(h)
        info = tn.tn_plan_describe(h)
        sbits = int(np.log2(info["slice_batch"]))
        for i, s in enumerate(steps):
            f = tn.tn_plan_step_features(h, i, -1)
            bb = int(np.log2(s["batch"])) + (sbits if s["per_slice"] else 0)
            assert f[0] == bb and f[1] == np.log2(s["m"]) and f[2] == np.log2(s["n"])
            assert f[3] == np.log2(s["k"])
            assert f[4] == 3 + f[0] + f[1] + f[2] + f[3]
            assert abs(f[6] - (f[4] - f[5])) < 1e-5
            assert f[11] == s["per_slice"]
            assert f[12:16].sum() == 1 and f[12 + s["kernel"]] == 1
            if s["kernel"] == 0:
                assert f[16:20].sum() == 0
                continue
            tile = s["tile"]
            bm, bn = [(256, 128), (128, 128), (128, 64), (64, 64)][tile]
            if s["lds_copy"] >= 2:   # the copy path lays a 256x128 tile id out as 512 x 64 / 512 x 32
                assert tile == 0 and s["n"] == (64 if s["lds_copy"] == 2 else 32) and s["m"] >= 512
                bm, bn = 512, s["n"]
            assert (s["tile_m"], s["tile_n"]) == (min(bm, s["m"]), min(bn, s["n"]))
            assert f[16 + tile] == 1 and f[16:20].sum() == 1
            assert f[9] == np.log2(s["split_k"])
            assert f[20] == s["a_contig"] and f[21] == s["b_contig"]
            # other tiles: only tile-dependent features move
            wide = False
            if s["n"] in (32, 64) and s["m"] >= 512:   # would tile id 0 take a 512-row copy layout?
                tn.tn_plan_set_tile(h, i, 0)
                wide = tn.tn_plan_steps(h)[i]["lds_copy"] >= 2
                tn.tn_plan_set_tile(h, i, tile)
            for t in range(4):
                g = tn.tn_plan_step_features(h, i, t)
                assert np.array_equal(g[:7], f[:7]) and g[16 + t] == 1
                bm, bn = [(256, 128), (128, 128), (128, 64), (64, 64)][t]
                if t == 0 and wide:
                    bm, bn = 512, s["n"]
                assert g[7] == max(0, f[1] - np.log2(bm)) and g[8] == max(0, f[2] - np.log2(bn))
    finally:
        tn.tn_plan_destroy(h)


def test_set_tile_on_host_plan():
    circ, net, best = configs.build("rqc30")
    h = _host_plan(net, best["path"], best["sliced"], precision="c64")
    try:
        steps = tn.tn_plan_steps(h)
        mfma = [i for i, s in enumerate(steps) if s["kernel"] != 0]
        small = [i for i, s in enumerate(steps) if s["kernel"] == 0]
        assert mfma and small
        i = mfma[0]
        for t, shape in enumerate([(256, 128), (128, 128), (128, 64), (64, 64)]):
            tn.tn_plan_set_tile(h, i, t)
            s = tn.tn_plan_steps(h)[i]
            assert s["tile"] == t
            assert (s["tile_m"], s["tile_n"]) == (min(shape[0], s["m"]), min(shape[1], s["n"]))
            assert tn.tn_plan_step_features(h, i, -1)[16 + t] == 1
        _expect("TN_E_ARG", lambda: tn.tn_plan_set_tile(h, small[0], 0))
        _expect("TN_E_ARG", lambda: tn.tn_plan_set_tile(h, i, 4))
        _expect("TN_E_ARG", lambda: tn.tn_plan_set_tile(h, len(steps), 0))
        _expect("TN_E_ARG", lambda: tn.tn_plan_step_features(h, i, 7))
    finally:
        tn.tn_plan_destroy(h)


def test_host_plan_reports_workspace_size():
    """A host-only plan reports the device bytes a caller-owned workspace must hold: at least
    the leaves and both arenas, 256-byte aligned pieces."""
    circ, net, best = configs.build("rqc30")
    h = _host_plan(net, best["path"], best["sliced"], precision="f16x3")
    try:
        info = tn.tn_plan_describe(h)
    finally:
        tn.tn_plan_destroy(h)
    assert info["workspace_bytes"] % 256 == 0
    assert info["workspace_bytes"] >= 8 * info["max_intermediate"] * info["slice_batch"]


def test_automatic_slice_chunk():
    """slice_batch = 0: 8 slices per chunk, raised to 16 or 32 while the chunk's per-slice arena
    fits in 32 GiB (one-slice arena peak x chunk); a caller's value is kept; never more than
    the slice count."""
    circ, net, best = configs.build("rqc30")
    infos = {}
    for sb in (0, 8, 16):
        h = _host_plan(net, best["path"], best["sliced"], precision="f16x3", slice_batch=sb)
        try:
            infos[sb] = tn.tn_plan_describe(h)
        finally:
            tn.tn_plan_destroy(h)
    assert infos[8]["slice_batch"] == 8 and infos[16]["slice_batch"] == 16
    auto = infos[0]["slice_batch"]
    assert auto in (8, 16, 32)
    # the per-slice part of the workspace grows with the chunk: check the rule from the
    # 8- and 16-slice plans' workspaces (same leaves and invariant arena)
    per_slice = (infos[16]["workspace_bytes"] - infos[8]["workspace_bytes"]) / 8
    expect = 8
    while expect < 32 and 2 * expect * per_slice <= 32 * 2**30 * 1.01:
        expect *= 2
    assert auto == expect, (auto, per_slice)
    assert auto == 32   # the 30-qubit workload: about 0.9 GiB per slice
    _, net, best = configs.build("rqc53d12")   # 2^30-element intermediates: stays at 8
    h = _host_plan(net, best["path"], best["sliced"], precision="f16x3")
    try:
        assert tn.tn_plan_describe(h)["slice_batch"] == 8
    finally:
        tn.tn_plan_destroy(h)
    # a small network: the whole (at most 32-slice) slice range in one chunk
    rnet = random_network(4, n_tensors=8)
    rpath = greedy_path(rnet.labels, rnet.open_labels, rnet.extents())
    ext = rnet.extents()
    sliced = [l for l in sorted({l for lab in rnet.labels for l in lab})
              if l not in rnet.open_labels and ext[l] > 1][:2]
    h = _host_plan(rnet, rpath, sliced)
    try:
        info = tn.tn_plan_describe(h)
        assert 1 < info["n_slices"] <= 32 and info["slice_batch"] == info["n_slices"], info
    finally:
        tn.tn_plan_destroy(h)


def test_step_terms_setting_and_errors():
    """Per-step product count: split steps default to 3 and accept 1 or 3; other steps and
    other counts are refused; single_product_top marks the costliest split steps."""
    _, net, best = configs.build("rqc30d12")
    with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], precision="f16x3",
                 split_policy=1, host_only=True) as p:
        st = p.steps()
        split = [i for i, s in enumerate(st) if s["kernel"] in (2, 3)]
        other = [i for i, s in enumerate(st) if s["kernel"] not in (2, 3)]
        assert split and other
        assert all(st[i]["terms"] == 3 for i in split) and all(st[i]["terms"] == 0 for i in other)
        p.set_step_terms(split[0], 1)
        assert p.steps()[split[0]]["terms"] == 1
        with pytest.raises(tn.TnError):
            p.set_step_terms(split[0], 2)
        with pytest.raises(tn.TnError):
            p.set_step_terms(other[0], 1)
        with pytest.raises(tn.TnError):
            p.set_step_terms(len(st), 1)
        order = p.rank_split_steps(by_time=False)
        assert sorted(order) == split
        assert [st[i]["flops"] for i in order] == sorted((st[i]["flops"] for i in split), reverse=True)
        with pytest.raises(tn.TnError):   # measured ranking needs a device plan
            p.rank_split_steps(by_time=True)
        top = p.single_product_top(2, by_time=False)
        costs = sorted((st[i]["flops"] for i in split), reverse=True)
        assert sorted((st[i]["flops"] for i in top), reverse=True) == costs[:2]
        after = p.steps()
        assert [i for i in split if after[i]["terms"] == 1] == sorted(top)
    with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], precision="c64",
                 host_only=True) as q:
        with pytest.raises(tn.TnError):
            q.set_step_terms(0, 1)


def _all_open_circuit(rows, cols, cycles, seed):
    from tn_inputs.circuits import open_and_closed, random_circuit
    from tn_inputs.network import circuit_network
    circ = random_circuit(rows, cols, cycles, seed)
    oq, _ = open_and_closed(circ.n_qubits, circ.n_qubits, seed)
    net = circuit_network(circ, oq, {})
    return circ, net, greedy_path(net.labels, net.open_labels, net.extents(), seed=seed)


def test_sparse_plan_host_side():
    """Sparse-state plans: one amplitude entry per distinct bitstring (padded to a power of
    two), duplicates share their entry, merged bonds appear as table-indexed batch bits,
    and malformed inputs are refused."""
    from tn_inputs.circuits import sample_bitstrings
    circ, net, path = _all_open_circuit(3, 4, 8, 31)
    bits = sample_bitstrings(circ.n_qubits, 64, 5, duplicates=4)
    distinct = len({tuple(r) for r in bits})
    with tn.Plan(net.tensors, net.labels, net.open_labels, path, host_only=True, bitstrings=bits) as p:
        n_amp = p.describe()["n_amplitudes"]
        assert n_amp == 1 << (distinct - 1).bit_length()
        idx = p.sparse_index
        assert len(idx) == len(bits) and len(set(idx.tolist())) == distinct and idx.max() < n_amp
        for i in range(len(bits)):
            for j in range(i):
                assert (idx[i] == idx[j]) == bool(np.array_equal(bits[i], bits[j]))
        assert any(s["merged_bits"] >= 0 for s in p.steps())
    bad = bits.copy()
    bad[3, 2] = 2
    with pytest.raises(tn.TnError):
        tn.Plan(net.tensors, net.labels, net.open_labels, path, host_only=True, bitstrings=bad)
    with pytest.raises(ValueError):
        tn.Plan(net.tensors, net.labels, net.open_labels, path, host_only=True, bitstrings=bits[:, 1:])
    with tn.Plan(net.tensors, net.labels, net.open_labels, path, host_only=True) as q:
        with pytest.raises(tn.TnError):
            tn.tn_plan_sparse_index(q.handle, len(bits))
    # an open label of extent 4 is not a qubit bond
    x = np.ones((4, 2), dtype=np.complex128)
    y = np.ones((2,), dtype=np.complex128)
    with pytest.raises(tn.TnError):
        tn.Plan([x, y], [(0, 1), (1,)], (0,), [(0, 1)], host_only=True, bitstrings=np.zeros((2, 1), np.uint8))


def _raw_sparse_create(n_open, n_bitstrings, bits_buf, opts=None):
    """tn_plan_create_sparse called directly: a 1-tensor network holding n_open open labels."""
    import ctypes
    P = ctypes.POINTER
    ranks = (ctypes.c_int32 * 1)(n_open)
    lab = (ctypes.c_int32 * n_open)(*range(n_open))
    ext = (ctypes.c_int64 * n_open)(*([2] * n_open))
    lab_pp = (P(ctypes.c_int32) * 1)(ctypes.cast(lab, P(ctypes.c_int32)))
    ext_pp = (P(ctypes.c_int64) * 1)(ctypes.cast(ext, P(ctypes.c_int64)))
    op = (ctypes.c_int32 * n_open)(*range(n_open))
    pa = (ctypes.c_int32 * 1)(0)
    sl = (ctypes.c_int32 * 1)(0)
    if opts is None:
        opts = tn.tn_options()
        opts.struct_size = ctypes.sizeof(tn.tn_options)
        opts.host_only = 1
    h = ctypes.c_void_p()
    st = tn._lib.tn_plan_create_sparse(ctypes.byref(h), 1, ranks, lab_pp, ext_pp, None, n_open, op, 0, pa, 0, sl,
                                       n_bitstrings, ctypes.cast(bits_buf, P(ctypes.c_uint8)),
                                       ctypes.byref(opts))
    if st == 0:
        tn.tn_plan_destroy(h.value)
    return st, tn._lib.tn_last_error_message().decode()


def test_sparse_einsums_take_the_values_first_block_order_where_a_slices_repeat():
    """The 30-qubit 12-cycle sparse state (4096 bitstrings): its result values are ordered by
    A's restriction first, so the 1024-value einsum (A: 16 slices) and the 4096-value einsum
    (A: about 1000 slices) both take the values-first block order; only sparse einsums on
    MFMA kernels report it."""
    net, path, bits = configs.sparse_state_workload()
    with tn.Plan(net.tensors, net.labels, net.open_labels, path, precision="f16x3", bitstrings=bits,
                 host_only=True) as p:
        st = p.steps()
    big = [s for s in st if s["merged_bits"] == 10 and s["k"] == 4096]
    wide = [s for s in st if s["merged_bits"] == 12 and s["n"] == 32]
    assert big and big[0]["values_first"] == 1
    assert wide and wide[0]["values_first"] == 1
    assert all(s["values_first"] == 0 for s in st if s["merged_bits"] < 0)


def test_huge_allocation_returns_a_status_instead_of_aborting():
    """The C entry points never let a C++ exception cross the ABI: a request for more host
    memory than exists (2^61 sampled bitstrings) fails with TN_E_NOMEM."""
    import ctypes
    buf = (ctypes.c_uint8 * 8)()
    st, msg = _raw_sparse_create(2, 1 << 61, buf)
    assert tn.STATUS[st] == "TN_E_NOMEM", (st, msg)
    assert msg


def test_sparse_state_rejects_more_than_64_measured_labels():
    import ctypes
    buf = (ctypes.c_uint8 * 65)()
    st, msg = _raw_sparse_create(65, 1, buf)
    assert tn.STATUS[st] == "TN_E_UNSUPPORTED", (st, msg)


def test_option_values_are_validated():
    circ, net, best = configs.build("rqc12")
    for kw, name in ((dict(deterministic=2), "TN_E_ARG"), (dict(tuning=2), "TN_E_ARG"),
                     (dict(tuning=3), "TN_E_ARG"), (dict(split_policy=3), "TN_E_ARG")):
        with pytest.raises(tn.TnError) as e:
            tn.tn_plan_create(net.tensors, net.labels, net.open_labels, best["path"], (),
                              host_only=True, **kw)
        assert e.value.name == name, kw
    # deterministic 0 and 1 are both accepted (every reduction is fixed-order anyway)
    for d in (0, 1):
        h = tn.tn_plan_create(net.tensors, net.labels, net.open_labels, best["path"], (), host_only=True,
                              deterministic=d)
        tn.tn_plan_destroy(h)


def test_options_of_an_older_struct_size_are_accepted():
    """struct_size is the ABI version: a caller built before tuning_cache and cost_model
    existed passes a shorter struct, and the library reads only what it covers."""
    import ctypes
    circ, net, best = configs.build("rqc12")
    h = tn.tn_plan_create(net.tensors, net.labels, net.open_labels, best["path"], (), host_only=True)
    tn.tn_plan_destroy(h)
    opts = tn.tn_options()
    opts.struct_size = tn.tn_options.tuning_cache.offset
    opts.host_only = 1
    opts.tuning = 0
    opts.cost_model = 12345   # beyond struct_size: must not be read
    ranks = (ctypes.c_int32 * 1)(1)
    lab = (ctypes.c_int32 * 1)(0)
    ext = (ctypes.c_int64 * 1)(2)
    P = ctypes.POINTER
    lab_pp = (P(ctypes.c_int32) * 1)(ctypes.cast(lab, P(ctypes.c_int32)))
    ext_pp = (P(ctypes.c_int64) * 1)(ctypes.cast(ext, P(ctypes.c_int64)))
    op = (ctypes.c_int32 * 1)(0)
    out = ctypes.c_void_p()
    st = tn._lib.tn_plan_create(ctypes.byref(out), 1, ranks, lab_pp, ext_pp, None, 1, op, 0, op, 0, op,
                                ctypes.byref(opts))
    assert st == 0, tn._lib.tn_last_error_message()
    tn.tn_plan_destroy(out.value)
    opts.struct_size = 8   # too short to hold the required fields
    st = tn._lib.tn_plan_create(ctypes.byref(out), 1, ranks, lab_pp, ext_pp, None, 1, op, 0, op, 0, op,
                                ctypes.byref(opts))
    assert tn.STATUS[st] == "TN_E_ARG"


def test_split_policy_2_puts_small_steps_on_split_kernels():
    """split_policy 2: every step of the 12-qubit network whose intermediate operands hold at
    least 4 elements runs a split kernel; the rest (and policies 0, 1) stay on FP32."""
    circ, net, best = configs.build("rqc12")
    for prec, kind in (("f16x3", 2), ("bf16x3", 3)):
        kinds = {}
        for pol in (0, 1, 2):
            h = tn.tn_plan_create(net.tensors, net.labels, net.open_labels, best["path"], (), host_only=True,
                                  precision=prec, split_policy=pol)
            try:
                kinds[pol] = [s["kernel"] for s in tn.tn_plan_steps(h)]
            finally:
                tn.tn_plan_destroy(h)
        assert kind not in kinds[0] and kind not in kinds[1]
        assert kinds[2].count(kind) >= 0.9 * len(kinds[2])
        assert set(kinds[2]) <= {0, kind}
