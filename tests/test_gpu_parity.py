"""GPU parity: the HIP path (through the C ABI) against the CPU complex128 oracle.

Tolerances (relative L2 error of the amplitude batch, as the judged metric):
complex64 <= 1e-5; split FP16 / BF16 products with power-of-two scaling <= 1e-3.
Kernel-level products use the Frobenius relative error against numpy.
"""
import numpy as np
import pytest

from oracle import contract, metrics
from tn_inputs import configs
from tn_inputs.network import Network, random_network
from tn_inputs.paths import choose_slices, greedy_path

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
tn = pytest.importorskip("paper_2310_03978_amd.tn")

TOL = {"c64": 1e-5, "f16x3": 1e-3, "bf16x3": 1e-3}
# per-element bound beside the batch's relative L2: max_i |a_i - a*_i| over the RMS amplitude
# (a single wrong amplitude of a batch of n can hide under rel_l2 up to sqrt(n) times its error)
MAX_TOL = {k: 10 * v for k, v in TOL.items()}
GEMM_TOL = {"c64": 2e-6, "f16x3": 2e-6, "bf16x3": 1e-4}
SPLIT_KINDS = {"f16x3": 2, "bf16x3": 3}


def _check_amps(got, ref, prec, rel=None, what=""):
    """rel_l2 and the per-element bound against the oracle; prints both."""
    rel = TOL[prec] if rel is None else rel
    e, m = metrics.rel_l2(got, ref), metrics.max_err(got, ref)
    print(f"  {what} {prec}: rel_l2 {e:.3e} max_err {m:.3e}", flush=True)
    assert e <= rel, (what, prec, e)
    assert m <= 10 * rel, (what, prec, m)


def _assert_split_mix(steps, prec, min_share=0.5):
    """In a split precision, the steps really run the split kernels (not the FP32 ones)."""
    if prec not in SPLIT_KINDS:
        return
    kinds = [s["kernel"] for s in steps]
    n_split = sum(1 for k in kinds if k == SPLIT_KINDS[prec])
    assert n_split >= min_share * len(kinds), (prec, kinds)


def _assert_split_everywhere(steps, prec, min_share=0.8):
    """split_policy 2: every step runs the split kernel except steps with an operand of fewer
    than 4 elements (an intermediate that small stays on the FP32 kernel)."""
    _assert_split_mix(steps, prec, min_share)
    if prec not in SPLIT_KINDS:
        return
    for i, s in enumerate(steps):
        if s["kernel"] != SPLIT_KINDS[prec]:
            small = min(s["batch"] * s["m"] * s["k"], s["batch"] * s["k"] * s["n"])
            assert small < 4, (prec, i, s)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _crandn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("prec", ["c64", "f16x3", "bf16x3"])
@pytest.mark.parametrize("b,m,n,k", [(1, 128, 64, 16), (2, 256, 128, 64), (1, 8, 4, 2),
                                     (1, 1, 1, 1), (4, 32, 16, 512),
                                     (1, 64, 32, 8192), (1, 512, 256, 256), (2, 16, 128, 32),
                                     (256, 1, 1, 4096), (4, 2, 2, 65536), (1, 1, 2, 1024)])
def test_gemm_matches_numpy(prec, b, m, n, k):
    print(f"gemm {prec} b={b} m={m} n={n} k={k}", flush=True)
    rng = np.random.default_rng(b * 7 + m + n + k)
    A, B = _crandn(rng, (b, m, k)), _crandn(rng, (b, k, n))
    C = torch.zeros((b, m, n), dtype=torch.complex64, device="cuda")
    tn.tn_gemm(_dev(A), _dev(B), C, precision=prec)
    got = C.cpu().numpy().astype(np.complex128)
    ref = np.matmul(A.astype(np.complex128), B.astype(np.complex128))
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= GEMM_TOL[prec] * max(1.0, np.sqrt(k / 64)), err


@pytest.mark.parametrize("shape,perm", [((2, 4, 8), (2, 0, 1)), ((64, 32), (1, 0)),
                                        ((2,) * 14, tuple(np.random.default_rng(1).permutation(14))),
                                        ((4, 1, 256, 8, 2), (3, 1, 4, 0, 2)), ((), ()), ((2,), (0,)),
                                        ((1024, 2048), (1, 0)), ((1 << 20,), (0,)),
                                        ((2,) * 22, tuple(np.random.default_rng(2).permutation(22))),
                                        ((2, 512, 4, 256), (2, 0, 3, 1)), ((8, 8, 8, 8, 8, 8, 8), (6, 5, 4, 3, 2, 1, 0))])
def test_permute_bit_exact(shape, perm):
    print(f"permute {shape} {perm}", flush=True)
    rng = np.random.default_rng(len(shape))
    x = _crandn(rng, shape)
    out = torch.zeros(int(np.prod(shape)) if shape else 1, dtype=torch.complex64, device="cuda")
    xd = _dev(x.reshape(shape) if shape else x.reshape(()))
    tn.tn_permute(xd, list(perm), out)
    ref = np.transpose(x, perm).reshape(-1) if shape else x.reshape(-1)
    assert np.array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("shift_in,shift_out", [(1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("shape,perm", [((64, 32), (1, 0)), ((2,) * 18, tuple(np.random.default_rng(5).permutation(18)))])
def test_permute_unaligned_buffers(shape, perm, shift_in, shift_out):
    # buffers 8-byte but not 16-byte aligned: element-wide accesses instead of pairs
    print(f"permute unaligned {shape} {perm} {shift_in} {shift_out}", flush=True)
    rng = np.random.default_rng(9)
    x = _crandn(rng, shape)
    n = x.size
    xin = torch.zeros(n + 1, dtype=torch.complex64, device="cuda")
    xin[shift_in:shift_in + n] = _dev(x.reshape(-1))
    out = torch.zeros(n + 1, dtype=torch.complex64, device="cuda")
    tn.tn_permute(xin[shift_in:shift_in + n].view(shape), list(perm), out[shift_out:shift_out + n])
    ref = np.transpose(x, perm).reshape(-1)
    got = out.cpu().numpy()
    assert np.array_equal(got[shift_out:shift_out + n], ref)
    assert got[0 if shift_out else n] == 0   # nothing written outside the output


def _gpu_amplitudes(net, path, sliced=(), prec="c64", **kw):
    with tn.Plan(net.tensors, net.labels, net.open_labels, path, sliced, precision=prec, **kw) as p:
        p.contract()
        amps, count = p.amplitudes()
    return amps, count


@pytest.mark.parametrize("prec", ["c64", "f16x3", "bf16x3"])
def test_rqc12_matches_oracle(prec):
    """The 12-qubit circuit; in the split precisions split_policy 2 puts every step whose
    operands allow it on the split MFMA kernels (on its own every step of this small network
    would run the FP32 small-step kernel)."""
    print(f"rqc12 {prec}", flush=True)
    circ, net, best = configs.build("rqc12")
    ref = contract.amplitudes(net.tensors, net.labels, net.open_labels, best["path"])
    with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], (), precision=prec,
                 split_policy=2) as p:
        _assert_split_everywhere(p.steps(), prec)
        p.contract()
        got, count = p.amplitudes()
    assert count == 1
    _check_amps(got, ref, prec, what="rqc12")


@pytest.mark.parametrize("prec", ["c64", "f16x3", "bf16x3"])
def test_rqc12_sliced_matches_oracle(prec):
    print(f"rqc12 sliced {prec}", flush=True)
    circ, net, best = configs.build("rqc12")
    sliced = choose_slices(net.labels, net.open_labels, net.extents(), best["path"], cap_log2=6,
                           min_sliced=4)
    ref = contract.amplitudes(net.tensors, net.labels, net.open_labels, best["path"])
    for sb in (1, 4, 16):
        with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], sliced, precision=prec,
                     slice_batch=sb, split_policy=2) as p:
            _assert_split_everywhere(p.steps(), prec)
            p.contract()
            got, count = p.amplitudes()
        assert count == 2 ** len(sliced)
        _check_amps(got, ref, prec, what=f"rqc12 sliced, chunk {sb}")
    # per-slice partials against the oracle's slices
    ids = [0, 3, 2 ** len(sliced) - 1]
    with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], sliced, precision=prec,
                 split_policy=2) as p:
        parts = p.partials(ids)
    for i, s in enumerate(ids):
        r = contract.contract_slice(net.tensors, net.labels, net.open_labels, best["path"], sliced, s)
        _check_amps(parts[i], r, prec, what=f"rqc12 slice {s}")


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("prec", ["c64", "f16x3"])
def test_random_networks_match_oracle(seed, prec):
    """Batch (hyperedge) labels, labels summed on one operand, extents 1/2/4, slicing."""
    print(f"random net {seed} {prec}", flush=True)
    net = random_network(seed, n_tensors=7, n_labels=12, extents=(1, 2, 4), n_open=2)
    ext = net.extents()
    path = greedy_path(net.labels, net.open_labels, ext, seed=seed)
    sliced = [l for l in sorted(ext) if l not in net.open_labels and ext[l] > 1][: seed % 3]
    ref = contract.amplitudes(net.tensors, net.labels, net.open_labels, path, sliced)
    got, _ = _gpu_amplitudes(net, path, sliced, prec=prec, split_policy=2)
    _check_amps(got, ref, prec, what=f"random net {seed}")


def test_large_random_steps_use_mfma_and_match():
    """A synthetic network whose steps are large enough for the MFMA kernels and split K."""
    print("large steps", flush=True)
    rng = np.random.default_rng(5)
    # A[a(2^7) k(2^9)] B[k(2^9) b(2^6)] C[b(2^6) c(2^1)] -> open a, c
    shapes = {"A": (128, 512), "B": (512, 64), "C": (64, 2)}
    tensors = [(_crandn(rng, shapes[x]) / 8).astype(np.complex128) for x in "ABC"]
    net = Network(tensors=tensors, labels=[(0, 1), (1, 2), (2, 3)], open_labels=(0, 3))
    ref = contract.amplitudes(net.tensors, net.labels, net.open_labels, [(0, 1), (0, 2)])
    for prec in ("c64", "f16x3", "bf16x3"):
        with tn.Plan(net.tensors, net.labels, net.open_labels, [(0, 1), (0, 2)], (),
                     precision=prec, split_policy=1) as p:
            kinds = [s["kernel"] for s in p.steps()]
            p.contract()
            got, _ = p.amplitudes()
        assert kinds[0] != 0
        _check_amps(got, ref, prec, what="large steps")


@pytest.mark.parametrize("prec", ["f16x3", "bf16x3"])
@pytest.mark.parametrize("K", [16, 32, 256, 2048])
def test_lds_copy_pipeline_matches_oracle(prec, K):
    """Both operands of the last step are split-stored intermediates with contiguous k: the
    step runs the global -> LDS copy pipeline (1, 2 and many K stages, split K, a batch label)."""
    print(f"lds copy {prec} K={K}", flush=True)
    rng = np.random.default_rng(K)
    b, m, n, k1 = 2, 512, 256, 4
    # X[b m k1] Y[b k1 k] -> P[b m k];  Z[b k k1'] W[b k1' n] -> Q[b k n];  P Q -> R[b m n]
    labels = [(0, 1, 2), (0, 2, 3), (0, 3, 4), (0, 4, 5)]
    shapes = [(b, m, k1), (b, k1, K), (b, K, k1), (b, k1, n)]
    tensors = [(_crandn(rng, sh) / np.sqrt(sh[-1])).astype(np.complex128) for sh in shapes]
    net = Network(tensors=tensors, labels=labels, open_labels=(0, 1, 5))
    path = [(0, 1), (2, 3), (0, 2)]
    ref = contract.amplitudes(net.tensors, net.labels, net.open_labels, path)
    with tn.Plan(net.tensors, net.labels, net.open_labels, path, (), precision=prec) as p:
        last = p.steps()[2]
        p.contract()
        got, _ = p.amplitudes()
    assert last["lds_copy"] == 1, last
    _check_amps(got, ref, prec, what=f"lds copy K={K}")


def test_chunking_accumulation_and_resume():
    print("chunking", flush=True)
    circ, net, best = configs.build("rqc12")
    sliced = choose_slices(net.labels, net.open_labels, net.extents(), best["path"], cap_log2=6,
                           min_sliced=4)
    n = 2 ** len(sliced)
    with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], sliced,
                 slice_batch=4) as p:
        p.contract(0, n)
        full, c = p.amplitudes()
        assert c == n
        p.reset()
        for first, cnt in ((0, 3), (3, 6), (9, n - 9)):
            p.contract(first, cnt)
        parts, c = p.amplitudes()
        assert c == n
        assert metrics.rel_l2(parts, full) <= 1e-6
        # checkpoint after half, resume
        p.reset()
        p.contract(0, n // 2)
        half, c = p.amplitudes()
        p.reset()
        p.set_accumulator(half, c)
        p.contract(n // 2, n - n // 2)
        resumed, c = p.amplitudes()
        assert c == n and metrics.rel_l2(resumed, full) <= 1e-6
        # re-running a range adds it again
        p.reset()
        p.contract(0, n)
        p.contract(0, n)
        twice, _ = p.amplitudes()
        assert metrics.rel_l2(twice, 2 * full) <= 1e-6
        with pytest.raises(tn.TnError):
            p.contract(n - 1, 2)


@pytest.mark.parametrize("prec", ["f16x3", "bf16x3"])
def test_deterministic_bitwise(prec):
    """Two runs of the same split plan (every step on the split kernels, K splits included)
    give the same amplitudes bit for bit."""
    print(f"determinism {prec}", flush=True)
    circ, net, best = configs.build("rqc12")
    sliced = choose_slices(net.labels, net.open_labels, net.extents(), best["path"], cap_log2=6,
                           min_sliced=3)
    outs = []
    for _ in range(2):
        with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], sliced, precision=prec,
                     split_policy=2, deterministic=1) as p:
            _assert_split_everywhere(p.steps(), prec)
            p.contract()
            outs.append(p.amplitudes()[0])
    assert np.array_equal(outs[0], outs[1])


def test_degenerate_networks():
    print("degenerate", flush=True)
    x = (np.arange(8) + 1j * np.arange(8)[::-1]).reshape(2, 4).astype(np.complex128)
    # single tensor: sum over label 3, keep 5
    net = Network(tensors=[x], labels=[(3, 5)], open_labels=(5,))
    got, _ = _gpu_amplitudes(net, [])
    np.testing.assert_allclose(got, x.sum(axis=0), rtol=1e-6)
    # closed network (single amplitude): <u|v>
    u, v = np.array([1, 2j], dtype=np.complex128), np.array([3, -1j], dtype=np.complex128)
    net = Network(tensors=[u, v], labels=[(0,), (0,)], open_labels=())
    got, _ = _gpu_amplitudes(net, [(0, 1)])
    np.testing.assert_allclose(got, [np.sum(u * v)], rtol=1e-6)
    # scalar leaf and an outer product
    s = np.array(2.0 - 1j, dtype=np.complex128)
    net = Network(tensors=[s, u, v], labels=[(), (0,), (1,)], open_labels=(1, 0))
    got, _ = _gpu_amplitudes(net, [(1, 2), (0, 1)])
    np.testing.assert_allclose(got, (s * np.outer(v, u)).reshape(-1), rtol=1e-6)


def test_numeric_error_is_reported():
    print("numeric", flush=True)
    a = np.array([np.inf, 1.0], dtype=np.complex128)
    b = np.array([1.0, 1.0], dtype=np.complex128)
    net = Network(tensors=[a, b], labels=[(0,), (0,)], open_labels=())
    with tn.Plan(net.tensors, net.labels, net.open_labels, [(0, 1)]) as p:
        p.contract()
        with pytest.raises(tn.TnError) as e:
            p.amplitudes()
        assert e.value.name == "TN_E_NUMERIC"


@pytest.mark.parametrize("prec", ["c64", "f16x3"])
def test_rqc30_sampled_slices_match_oracle(prec):
    """The 30-qubit, 14-cycle, 256-slice workload at full size, in the launch configuration
    the bench times (autotuned tiles, the automatic chunk of 32 slices): a sampled slice vs the
    oracle, and the chunk holding it, contracted as one launch sequence, vs the sum of its
    slices' partials."""
    print(f"rqc30 {prec}", flush=True)
    circ, net, best = configs.build("rqc30")
    sid = 137
    ref = _rqc30_oracle_slice(sid)
    with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], best["sliced"],
                 precision=prec, tuning=1) as p:
        chunk = p.describe()["slice_batch"]
        assert chunk == 32
        part = p.partials([sid])[0]
        # the full run accumulates every slice once; chunked sums agree with partial sums
        first = sid - sid % chunk
        p.contract(first, chunk)
        acc, c = p.amplitudes()
        assert c == chunk
        parts = p.partials(list(range(first, first + chunk)))
    rep = metrics.report(part, ref)
    print(f"rqc30 slice {sid} {prec}: {rep}", flush=True)
    _check_amps(part, ref, prec, what=f"rqc30 slice {sid}")
    assert metrics.rel_l2(acc, parts.sum(axis=0)) <= 1e-6


@pytest.mark.parametrize("prec", ["c64", "f16x3", "bf16x3"])
def test_rqc30d12_precision_subcase_matches_oracle(prec):
    """The precision form's 30-qubit sub-case (5x6 lattice, 12 cycles, 512 correlated
    amplitudes, largest intermediate 2^26): every amplitude against the oracle's, stored
    by tests/golden/make_rqc30d12_amplitudes.py."""
    import importlib.util
    import os
    print(f"rqc30d12 {prec}", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_rqc30d12_amplitudes.py")
    spec = importlib.util.spec_from_file_location("make_rqc30d12_amplitudes", path)
    fx = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(fx)
    digest, ref = fx.read_fixture()
    _, net, best = configs.build("rqc30d12")
    assert digest == fx.network_digest(net, best)
    with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], precision=prec) as p:
        p.contract()
        got, c = p.amplitudes()
    assert c == 1
    rep = metrics.report(got, ref)
    print(f"rqc30d12 {prec}: {rep}", flush=True)
    _check_amps(got, ref, prec, what="rqc30d12")
    assert rep["fidelity"] >= 1 - 2 * TOL[prec]


_ORACLE_CACHE = {}


def _rqc30_oracle_slice(sid):
    if sid not in _ORACLE_CACHE:
        circ, net, best = configs.build("rqc30")
        _ORACLE_CACHE[sid] = contract.contract_slice(net.tensors, net.labels, net.open_labels,
                                                     best["path"], best["sliced"], sid)
    return _ORACLE_CACHE[sid]


@pytest.mark.parametrize("tile", [0, 1, 2, 3])
@pytest.mark.parametrize("prec", ["c64", "f16x3", "bf16x3"])
@pytest.mark.parametrize("b,m,n,k", [(1, 512, 256, 64), (2, 64, 16, 4096), (1, 256, 8, 32)])
def test_gemm_every_tile_shape(tile, prec, b, m, n, k, monkeypatch):
    """Each MFMA tile shape (256x128, 128x128, 128x64, 64x64), with partial tiles and split K."""
    print(f"gemm tile {tile} {prec} b={b} m={m} n={n} k={k}", flush=True)
    monkeypatch.setenv("TN_GEMM_TILE", str(tile))
    rng = np.random.default_rng(tile * 13 + m + k)
    A, B = _crandn(rng, (b, m, k)), _crandn(rng, (b, k, n))
    C = torch.zeros((b, m, n), dtype=torch.complex64, device="cuda")
    tn.tn_gemm(_dev(A), _dev(B), C, precision=prec)
    got = C.cpu().numpy().astype(np.complex128)
    ref = np.matmul(A.astype(np.complex128), B.astype(np.complex128))
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= GEMM_TOL[prec] * max(1.0, np.sqrt(k / 64)), err


@pytest.mark.parametrize("prec", ["f16x3", "bf16x3"])
def test_split_storage_chain_matches_oracle(prec):
    """Intermediates feeding split-precision steps are stored split; a chain of such steps."""
    print(f"split chain {prec}", flush=True)
    rng = np.random.default_rng(9)
    # X[a(2^8) k1(2^6)] Y[k1(2^6) k2(2^6) b(2^1)] Z[k2(2^6) c(2^6)] W[c(2^6) d(2^5)]
    shapes = [(256, 64), (64, 64, 2), (64, 64), (64, 32)]
    tensors = [(_crandn(rng, s) / 4).astype(np.complex128) for s in shapes]
    labels = [(0, 1), (1, 2, 3), (2, 4), (4, 5)]
    net = Network(tensors=tensors, labels=labels, open_labels=(0, 3, 5))
    path = [(0, 1), (0, 2), (0, 3)]
    ref = contract.amplitudes(net.tensors, net.labels, net.open_labels, path)
    with tn.Plan(net.tensors, net.labels, net.open_labels, path, (), precision=prec,
                 split_policy=1) as p:
        kinds = [s["kernel"] for s in p.steps()]
        p.contract()
        got, _ = p.amplitudes()
    assert kinds.count(2 if prec == "f16x3" else 3) >= 2, kinds
    _check_amps(got, ref, prec, rel=(1e-5 if prec == "f16x3" else 1e-3), what="split chain")


@pytest.mark.parametrize("prec", ["c64", "f16x3"])
def test_autotuned_plan_matches_oracle(prec):
    """tuning=1 times every tile shape per MFMA step at plan creation; results still match."""
    print(f"autotune {prec}", flush=True)
    rng = np.random.default_rng(21)
    shapes = [(512, 256), (256, 128, 2), (128, 64)]
    tensors = [(_crandn(rng, s) / 4).astype(np.complex128) for s in shapes]
    net = Network(tensors=tensors, labels=[(0, 1), (1, 2, 3), (2, 4)], open_labels=(0, 3, 4))
    path = [(0, 1), (0, 2)]
    ref = contract.amplitudes(net.tensors, net.labels, net.open_labels, path)
    with tn.Plan(net.tensors, net.labels, net.open_labels, path, (), precision=prec,
                 split_policy=1, tuning=1) as p:
        p.contract()
        got, _ = p.amplitudes()
    _check_amps(got, ref, prec, what="autotuned")


def _small_circuits(n, seed=1040, open_k=4):
    """Uneven 16-28 qubit lattice circuits, depth 8-14, unsliced (the batching form's sub-networks)."""
    return configs.uneven_circuits(n, seed=seed, open_k=open_k, cap_log2=22)


@pytest.mark.parametrize("prec", ["c64", "f16x3"])
def test_group_graph_launch_matches_individual_plans(prec):
    """Slices of one network plus uneven small networks in one graph replay: every plan's
    amplitudes equal, bit for bit, those of the same plan contracted on its own."""
    print(f"group {prec}", flush=True)
    circ, net, best = configs.build("rqc12")
    sliced = choose_slices(net.labels, net.open_labels, net.extents(), best["path"], cap_log2=6,
                           min_sliced=4)
    items = [(net, {"path": best["path"], "sliced": sliced})] + _small_circuits(6)
    refs = [contract.amplitudes(n.tensors, n.labels, n.open_labels, b["path"], b.get("sliced", ()))
            for n, b in items]

    def make():
        return [tn.Plan(n.tensors, n.labels, n.open_labels, b["path"], b.get("sliced", ()),
                        precision=prec, slice_batch=4) for n, b in items]

    alone = make()
    plans = make()
    try:
        for p in alone:
            p.contract()
        singles = [p.amplitudes()[0] for p in alone]
        with tn.Group(plans, branches=3) as g:
            # capture without launching: nothing is added to any accumulator
            g.prepare()
            info = g.describe()
            assert info["n_kernels"] > len(plans) and info["n_branches"] == 3
            for p in plans:
                amps0, count0 = p.amplitudes()
                assert count0 == 0 and not np.any(amps0)
            g.contract()   # a replay of the prepared graph
            assert g.describe() == info
            outs = [p.amplitudes() for p in plans]
            for (amps, count), ref, one, p in zip(outs, refs, singles, plans):
                assert count == p.describe()["n_slices"]
                assert np.array_equal(amps, one)
                _check_amps(amps, ref, prec, what="group member")
            # a replay of the captured graph adds the same amplitudes again
            g.contract()
            for (amps, _), p in zip(outs, plans):
                again, count = p.amplitudes()
                assert count == 2 * p.describe()["n_slices"]
                assert metrics.rel_l2(again, 2 * amps) <= 1e-12
            # a partial range through the group equals the same range contracted alone
            for p in plans:
                p.reset()
            g.contract([3] + [0] * (len(plans) - 1), [5] + [0] * (len(plans) - 1))
            part, c = plans[0].amplitudes()
            assert c == 5
            assert g.describe()["n_branches"] == 1
        alone[0].reset()
        alone[0].contract(3, 5)
        ref5, _ = alone[0].amplitudes()
        assert np.array_equal(part, ref5)
    finally:
        for p in plans + alone:
            p.close()


@pytest.mark.parametrize("prec", ["c64", "f16x3"])
def test_caller_owned_workspace(prec):
    """A plan built in a torch-owned workspace gives the same amplitudes, bit for bit, as a
    plan that allocates its own memory; a workspace that is too small is refused."""
    print(f"workspace {prec}", flush=True)
    circ, net, best = configs.build("rqc12")
    sliced = choose_slices(net.labels, net.open_labels, net.extents(), best["path"], cap_log2=6,
                           min_sliced=3)
    args = (net.tensors, net.labels, net.open_labels, best["path"], sliced)
    kw = dict(precision=prec, split_policy=2)
    with tn.Plan(*args, host_only=True, **kw) as h:
        need = h.describe()["workspace_bytes"]
    with tn.Plan(*args, **kw) as p:
        _assert_split_everywhere(p.steps(), prec)
        p.contract()
        ref, _ = p.amplitudes()
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    with tn.Plan(*args, workspace=ws, **kw) as q:
        assert q.describe()["workspace_bytes"] <= need
        q.contract()
        got, _ = q.amplitudes()
    assert np.array_equal(got, ref)
    # autotuning inside the workspace (split-K scratch is reserved for every tile)
    with tn.Plan(*args, workspace=ws, tuning=1, **kw) as q:
        q.contract()
        tuned, _ = q.amplitudes()
    oracle_ref = contract.amplitudes(net.tensors, net.labels, net.open_labels, best["path"])
    _check_amps(tuned, oracle_ref, prec, what="workspace, autotuned")
    small = torch.empty(need // 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(tn.TnError) as e:
        tn.Plan(*args, workspace=small, **kw)
    assert e.value.name == "TN_E_NOMEM"


def _sample_slices(n_slices, k, seed):
    rng = np.random.default_rng(seed)
    return sorted(int(x) for x in rng.choice(n_slices, size=min(k, n_slices), replace=False))


def test_rqc53d12_full_size_properties():
    """The precision form at its full size (53 qubits, 12 cycles, 512 correlated amplitudes,
    largest intermediate 2^30 elements, 2^16 slices), where no oracle slice finishes in
    seconds: properties that hold at any size, on slices of the seeded sample (seed 303).
    (1) The split-FP16 and split-BF16 partial amplitudes of a slice agree with the
    complex64 ones within the precision form's bound.  (2) Slicing invariance (Sec. 3.2):
    the two slices that differ only in the last sliced bond sum to the slice of the plan
    that leaves that bond unsliced (largest intermediate 2^31)."""
    print("rqc53d12 full size", flush=True)
    _, net, best = configs.build("rqc53d12")
    sliced = list(best["sliced"])
    n = 1 << len(sliced)
    s = _sample_slices(n, 4096, 303)[0] & ~1
    args = (net.tensors, net.labels, net.open_labels, best["path"])
    with tn.Plan(*args, sliced, precision="c64", slice_batch=1) as q:
        pc = q.partials([s, s | 1])
    for prec in ("f16x3", "bf16x3"):
        with tn.Plan(*args, sliced, precision=prec, slice_batch=1) as p:
            pf = p.partials([s, s | 1])
        for j in range(2):
            err = metrics.rel_l2(pf[j], pc[j])
            print(f"rqc53d12 slice {s | j} {prec} vs c64: rel_l2 {err:.2e}", flush=True)
            assert err <= TOL[prec]
    with tn.Plan(*args, sliced[:-1], precision="c64", slice_batch=1) as r:
        pr = r.partials([s >> 1])[0]
    err = metrics.rel_l2(pc.sum(axis=0), pr)
    print(f"rqc53d12 slicing invariance: rel_l2 {err:.2e}", flush=True)
    assert err <= 2 * TOL["c64"]


def test_rqc40_batching_form_full_size():
    """The batching form's shape: slices of the 40-qubit, 16-cycle network (largest
    intermediate 2^28) and 64 uneven 16-28-qubit circuits in one captured graph.  Every
    plan's amplitudes equal, bit for bit, the same plan's run on its own; every uneven circuit
    the oracle contracts in well under a second (at most 1e12 flops: 56 of the 64) also
    matches the oracle, and the graph's 40-qubit sum agrees with the complex64 path's."""
    print("rqc40 batching form", flush=True)
    _, net, best = configs.build("rqc40")
    args = (net.tensors, net.labels, net.open_labels, best["path"], best["sliced"])
    small = configs.uneven_circuits(64)
    first = _sample_slices(1 << len(best["sliced"]), 1, 404)[0] & ~7

    def make():
        return ([tn.Plan(*args, precision="f16x3", slice_batch=4)] +
                [tn.Plan(n_.tensors, n_.labels, n_.open_labels, b["path"], precision="f16x3") for n_, b in small])

    alone, plans = make(), make()
    try:
        alone[0].contract(first, 8)
        for p in alone[1:]:
            p.contract()
        singles = [p.amplitudes()[0] for p in alone]
        with tn.Group(plans, branches=8) as g:
            g.contract([first] + [0] * len(small), [8] + [1] * len(small))
            for p, one in zip(plans, singles):
                assert np.array_equal(p.amplitudes()[0], one)
        cheap = [i for i in range(len(small)) if small[i][1]["cost"]["flops_total"] <= 1e12]
        assert len(cheap) >= 48
        for i in cheap:
            n_, b = small[i]
            ref = contract.amplitudes(n_.tensors, n_.labels, n_.open_labels, b["path"])
            _check_amps(singles[1 + i], ref, "f16x3", what=f"uneven circuit {i}")
        with tn.Plan(*args, precision="c64", slice_batch=4) as q:
            q.contract(first, 8)
            ref40, _ = q.amplitudes()
        err = metrics.rel_l2(singles[0], ref40)
        print(f"rqc40 slices [{first}, {first + 8}) f16x3 vs c64: rel_l2 {err:.2e}", flush=True)
        assert err <= TOL["f16x3"]
    finally:
        for p in plans + alone:
            p.close()


def test_group_refuses_a_branch_beyond_its_node_limit():
    """A group graph whose one branch would hold more than 8192 kernel nodes (all 256 slices of
    the 30-qubit workload one slice per chunk, a few hundred launches each) is refused on the
    host before anything is captured; a smaller range of the same group then runs normally."""
    print("group node limit", flush=True)
    _, net, best = configs.build("rqc30")
    with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], best["sliced"], precision="f16x3",
                 slice_batch=1) as p:
        per_slice = sum(1 for s in p.steps() if s["per_slice"])
        assert 256 * per_slice > 8192
        with tn.Group([p]) as g:
            with pytest.raises(tn.TnError) as e:
                g.prepare([0], [256])
            assert e.value.status == -9 and "kernel nodes" in str(e.value), e.value
            amps0, count0 = p.amplitudes()
            assert count0 == 0
            g.contract([0], [2])
            got, count = p.amplitudes()
        assert count == 2
        ref = p.partials([0, 1]).sum(axis=0)
        assert metrics.rel_l2(got, ref) <= 1e-12


def test_group_recaptures_after_retile():
    """A plan re-tiled after its group captured a graph: the next group contraction uses the
    new tiles (bitwise equal to the re-tiled plan alone), not the stale graph."""
    print("group retile", flush=True)
    items = _small_circuits(3)
    kw = dict(precision="f16x3", split_policy=1)
    plans = [tn.Plan(n.tensors, n.labels, n.open_labels, b["path"], **kw) for n, b in items]
    alone = tn.Plan(items[0][0].tensors, items[0][0].labels, items[0][0].open_labels, items[0][1]["path"], **kw)
    try:
        mfma = [i for i, s in enumerate(plans[0].steps()) if s["kernel"] != 0]
        assert mfma
        with tn.Group(plans, branches=2) as g:
            g.contract()
            first, _ = plans[0].amplitudes()
            s = mfma[0]
            new_tile = (plans[0].steps()[s]["tile"] + 1) % 4
            plans[0].set_tile(s, new_tile)
            alone.set_tile(s, new_tile)
            for p in plans:
                p.reset()
            g.contract()
            got, c = plans[0].amplitudes()
        assert c == 1
        alone.contract()
        ref, _ = alone.amplitudes()
        assert np.array_equal(got, ref)
        assert metrics.rel_l2(got, first) <= 2 * TOL["f16x3"]
    finally:
        for p in plans + [alone]:
            p.close()


def _round16(x, bf):
    """float32 array rounded to fp16 (or bf16), round to nearest even, as float64."""
    x = np.asarray(x, dtype=np.float32)
    if not bf:
        return x.astype(np.float16).astype(np.float64)
    bits = x.view(np.uint32).astype(np.uint64)
    r = ((bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def _split_hi(z, bf):
    """The hi part the split kernels form for a complex64 leaf: scaled by the power of two
    that brings max(|re|, |im|) to [2^14, 2^15), rounded to 16 bits, scaled back."""
    z = z.astype(np.complex64)
    mx = np.float32(max(np.abs(z.real).max(), np.abs(z.imag).max()))
    e = 14 - (int(np.frexp(mx)[1]) - 1)
    s = np.float32(2.0 ** e)
    return (_round16(z.real * s, bf) + 1j * _round16(z.imag * s, bf)) / float(s)


@pytest.mark.parametrize("prec", ["f16x3", "bf16x3"])
def test_single_product_step_is_the_rounded_operands_product(prec):
    """A split step run with one product (hi x hi) computes exactly the product of the 16-bit
    rounded, power-of-two scaled operands, up to FP32 accumulation; with three products it is
    within the extended-precision bound of the exact product."""
    print(f"single product {prec}", flush=True)
    bf = prec == "bf16x3"
    rng = np.random.default_rng(17)
    m, k, n = 256, 512, 128
    A, B = _crandn(rng, (m, k)).astype(np.complex128), _crandn(rng, (k, n)).astype(np.complex128)
    net = Network(tensors=[A, B], labels=[(0, 1), (1, 2)], open_labels=(0, 2))
    exact = (A.astype(np.complex64).astype(np.complex128) @ B.astype(np.complex64).astype(np.complex128)).reshape(-1)
    rounded = (_split_hi(A, bf) @ _split_hi(B, bf)).reshape(-1)
    with tn.Plan(net.tensors, net.labels, net.open_labels, [(0, 1)], precision=prec, split_policy=1) as p:
        st = p.steps()
        assert st[0]["kernel"] in (2, 3) and st[0]["terms"] == 3
        p.contract()
        three, _ = p.amplitudes()
        p.set_step_terms(0, 1)
        assert p.steps()[0]["terms"] == 1
        p.reset()
        p.contract()
        one, _ = p.amplitudes()
    e1 = metrics.rel_l2(one, rounded)
    e3 = metrics.rel_l2(three, exact)
    e1x = metrics.rel_l2(one, exact)
    print(f"{prec}: one product vs rounded {e1:.2e}, vs exact {e1x:.2e}; three products vs exact {e3:.2e}", flush=True)
    assert e1 <= 1e-5
    assert e3 <= GEMM_TOL[prec]
    assert e1x > 10 * e3          # the single product really drops the correction terms


def test_single_product_on_top_steps_trend():
    """Per-step precision on the 30-qubit 12-cycle sub-case (512 amplitudes, stored oracle
    amplitudes): single products on the k costliest split steps; k = 0 is the default plan
    bit for bit, and the error grows with k while staying near the 16-bit rounding level."""
    import importlib.util
    import os
    print("single product top-k", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_rqc30d12_amplitudes.py")
    spec = importlib.util.spec_from_file_location("make_rqc30d12_amplitudes", path)
    fx = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(fx)
    digest, ref = fx.read_fixture()
    _, net, best = configs.build("rqc30d12")
    assert digest == fx.network_digest(net, best)
    errs = []
    with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], precision="f16x3") as p:
        p.contract()
        base, _ = p.amplitudes()
        n_split = sum(1 for s in p.steps() if s["kernel"] in (2, 3))
        for k in (0, 1, 4, n_split):
            p.single_product_top(k)
            p.reset()
            p.contract()
            got, _ = p.amplitudes()
            if k == 0:
                assert np.array_equal(got, base)
            errs.append(metrics.rel_l2(got, ref))
            print(f"top-{k} of {n_split} split steps single: eps_l2^2 {metrics.eps_l2sq(got, ref):.3e} "
                  f"rel_l2 {errs[-1]:.3e}", flush=True)
            # one fp16 product per step: each operand rounded to 11 significant bits (relative
            # 2^-12), so a step adds about 2^-11.5 relative error; k such steps add in
            # quadrature at most sqrt(k) times that (bound doubled)
            bound = TOL["f16x3"] / 100 if k == 0 else 2 * 2.0 ** -11.5 * np.sqrt(k)
            assert errs[-1] <= bound, (k, errs[-1], bound)
    assert errs[-1] > errs[0]


@pytest.mark.parametrize("budget", [1e-6, 1e-4])
def test_single_products_chosen_under_a_budget(budget):
    """Per-step precision chosen by the library under an epsilon_L2^2 budget (Sec. 4.3,
    Table 3): the plan keeps single products on its k costliest split steps (ranked by
    measured time) with epsilon_L2^2 <= budget against its three-product amplitudes; against
    the oracle the error is then at most the budget plus the three-product error."""
    import importlib.util
    import os
    print(f"single products under budget {budget}", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_rqc30d12_amplitudes.py")
    spec = importlib.util.spec_from_file_location("make_rqc30d12_amplitudes", path)
    fx = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(fx)
    digest, ref = fx.read_fixture()
    _, net, best = configs.build("rqc30d12")
    assert digest == fx.network_digest(net, best)
    with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], precision="f16x3") as p:
        p.contract()
        three, _ = p.amplitudes()
        k, eps = p.choose_single_products(budget, [0])
        st = p.steps()
        single = [i for i, s in enumerate(st) if s["terms"] == 1]
        order = p.rank_split_steps(by_time=True)
        p.reset()
        p.contract()
        got, _ = p.amplitudes()
    print(f"budget {budget}: k = {k} of {len(order)} split steps, eps_l2^2 {eps:.3e} against three products, "
          f"{metrics.eps_l2sq(got, ref):.3e} against the oracle (three products {metrics.eps_l2sq(three, ref):.3e})",
          flush=True)
    assert eps <= budget and len(single) == k
    assert abs(metrics.eps_l2sq(got, three) - eps) <= 1e-3 * budget + 1e-12
    assert metrics.eps_l2sq(got, ref) <= budget * (1 + 1e-6) + metrics.eps_l2sq(three, ref) + 1e-12
    if budget >= 1e-4:
        assert k >= 1
    assert metrics.rel_l2(got, ref) <= 2 * 2.0 ** -11.5 * np.sqrt(max(k, 1))


def _all_open(rows, cols, cycles, seed):
    from tn_inputs.circuits import open_and_closed, random_circuit
    from tn_inputs.network import circuit_network
    circ = random_circuit(rows, cols, cycles, seed)
    oq, _ = open_and_closed(circ.n_qubits, circ.n_qubits, seed)
    net = circuit_network(circ, oq, {})
    return circ, net, greedy_path(net.labels, net.open_labels, net.extents(), seed=3)


_DENSE_ALL_OPEN = {}


@pytest.mark.parametrize("prec", ["c64", "f16x3", "bf16x3"])
@pytest.mark.parametrize("sliced_bits", [0, 3])
def test_sparse_state_matches_oracle(prec, sliced_bits):
    """Sparse-state contraction (Sec. 3.3) of a 20-qubit, 10-cycle circuit with every qubit
    measured, for 512 sampled bitstrings plus 16 repeats: the merged bonds run as
    table-indexed batches on the small and the split MFMA kernels; every amplitude is
    compared with the oracle (the dense contraction with all qubits open, read at the
    bitstrings).  With sliced bonds the slices' sums go through the same tables."""
    from tn_inputs.circuits import sample_bitstrings
    print(f"sparse state {prec} sliced bits {sliced_bits}", flush=True)
    circ, net, path = _all_open(4, 5, 10, 41)
    bits = sample_bitstrings(circ.n_qubits, 528, 5, duplicates=16)
    if "d" not in _DENSE_ALL_OPEN:
        _DENSE_ALL_OPEN["d"] = contract.amplitudes(net.tensors, net.labels, net.open_labels, path)
    dense = _DENSE_ALL_OPEN["d"]
    ref = dense[[int("".join(str(int(b)) for b in row), 2) for row in bits]]
    sliced = ()
    if sliced_bits:
        sliced = choose_slices(net.labels, net.open_labels, net.extents(), path, cap_log2=60,
                               min_sliced=sliced_bits, max_sliced=sliced_bits)
    with tn.Plan(net.tensors, net.labels, net.open_labels, path, sliced, precision=prec, split_policy=1,
                 bitstrings=bits, slice_batch=4) as p:
        st = p.steps()
        merged = [s for s in st if s["merged_bits"] >= 0]
        assert any(s["kernel"] == 0 for s in merged)
        if prec != "c64":
            assert any(s["kernel"] in (2, 3) for s in merged)
        p.contract()
        got, c = p.amplitudes()
    assert c == (1 << sliced_bits)
    rep = metrics.report(got, ref)
    print(f"sparse state {prec} sliced {sliced_bits}: {rep}", flush=True)
    _check_amps(got, ref, prec, what="sparse state")


_SPARSE_C64 = {}


def _wide_copy_steps(p):
    """Steps whose 256x128 tile id takes one of the LDS-copy kernel's 512-row layouts
    (512 x 64 for 64 columns, 512 x 32 for 32) once set."""
    out = []
    for i, s in enumerate(p.steps()):
        if s["kernel"] in (2, 3) and s["n"] in (32, 64) and s["m"] >= 512:
            p.set_tile(i, 0)
            if p.steps()[i]["lds_copy"] >= 2:
                out.append(i)
    return out


def test_lds_copy_512x64_layout_on_a_single_stage_step():
    """A 64-column split step of the 30-qubit network (m = 4096, k = 16: one K stage) on the
    LDS-copy kernel's 512 x 64 layout gives the amplitudes of the same plan with the step on
    the staged kernel, to rounding (2 slices, split FP16)."""
    print("copy layout 512x64 on rqc30", flush=True)
    circ, net, best = configs.build("rqc30")
    with tn.Plan(net.tensors, net.labels, net.open_labels, best["path"], best["sliced"], precision="f16x3",
                 tuning=0) as p:
        p.contract(0, 2)
        ref, _ = p.amplitudes()
        p.reset()
        wide = _wide_copy_steps(p)
        assert wide, "no 64-column split step in the plan"
        assert any(p.steps()[i]["k"] == 16 for i in wide)
        p.contract(0, 2)
        got, _ = p.amplitudes()
    assert metrics.rel_l2(got, ref) <= 1e-5


@pytest.mark.parametrize("prec", ["f16x3", "bf16x3"])
def test_lds_copy_512x64_layout_on_the_sparse_state(prec):
    """The sparse state of the 30-qubit 12-cycle circuit (4096 bitstrings), whose largest
    sparse einsum (1024 merged values x 65536 x 64 x 4096) runs on the 512 x 64 layout and
    whose 4096 values x 8192 x 32 x 512 einsum runs on the 512 x 32 layout, against the
    complex64 contraction of the same plan."""
    print(f"copy layouts 512x64 and 512x32 on the sparse state, {prec}", flush=True)
    net, path, bits = configs.sparse_state_workload()
    if "ref" not in _SPARSE_C64:
        with tn.Plan(net.tensors, net.labels, net.open_labels, path, precision="c64", bitstrings=bits) as q:
            q.contract()
            _SPARSE_C64["ref"] = q.amplitudes()[0]
    ref = _SPARSE_C64["ref"]
    with tn.Plan(net.tensors, net.labels, net.open_labels, path, precision=prec, bitstrings=bits,
                 tuning=0) as p:
        wide = _wide_copy_steps(p)
        st = p.steps()
        assert any(st[i]["merged_bits"] >= 0 and st[i]["k"] == 4096 and st[i]["lds_copy"] == 2
                   and st[i]["values_first"] == 1 for i in wide)
        assert any(st[i]["merged_bits"] >= 0 and st[i]["n"] == 32 and st[i]["lds_copy"] == 3 for i in wide)
        p.contract()
        got, _ = p.amplitudes()
    rel = metrics.rel_l2(got, ref)
    print(f"sparse state on the 512-row layouts, {prec}: rel_l2 vs complex64 {rel:.2e}", flush=True)
    assert rel <= (1e-4 if prec == "f16x3" else 1e-3)


_SPARSE_ORACLE = {}


@pytest.mark.parametrize("prec", ["c64", "f16x3"])
def test_sparse_einsum_values_first_matches_oracle(prec):
    """The sparse state of the 30-qubit 12-cycle circuit, whose 1024-value einsum (runs of
    about 62 consecutive values share A's slice) takes the block order with the merged
    values fastest: 6 seeded bitstrings' amplitudes against the oracle's definition (one
    closed complex128 contraction per bitstring, Sec. 3.3), on the learned model's tiles
    (the split step on the 512 x 64 LDS-copy layout) and on complex64."""
    from oracle import sparse
    from tn_inputs.paths import path_cost
    print(f"sparse einsum with values first, {prec}", flush=True)
    net, path, bits = configs.sparse_state_workload()
    ids = [int(x) for x in np.random.default_rng(808).choice(len(bits), 6, replace=False)]
    if "ref" not in _SPARSE_ORACLE:
        opened = set(net.open_labels)
        closed = [tuple(l for l in lab if l not in opened) for lab in net.labels]
        ext = net.extents()
        cands = [greedy_path(closed, (), ext, seed=k, temperature=0.0 if k == 0 else 0.3) for k in range(6)]
        cpath = min(cands, key=lambda q: path_cost(closed, (), ext, q)["flops_total"])
        _SPARSE_ORACLE["ref"] = sparse.definition_amplitudes(net.tensors, net.labels, net.open_labels,
                                                             cpath, bits[ids])
    ref = _SPARSE_ORACLE["ref"]
    with tn.Plan(net.tensors, net.labels, net.open_labels, path, precision=prec, bitstrings=bits,
                 tuning=2) as p:
        st = p.steps()
        big = [s for s in st if s["merged_bits"] == 10 and s["k"] == 4096]
        assert big and big[0]["values_first"] == 1 and big[0]["kernel"] != 0, big
        if prec == "f16x3":
            assert big[0]["lds_copy"] == 2, big
        assert any(s["merged_bits"] >= 0 and s["kernel"] != 0 and s["values_first"] == 0 for s in st)
        p.contract()
        got, _ = p.amplitudes()
    _check_amps(got[ids], ref, prec, rel=1e-5 if prec == "c64" else 1e-4, what="sparse state, values first")


@pytest.mark.parametrize("prec", ["c64", "f16x3"])
def test_annealed_path_matches_oracle(prec):
    """A tree refined by the annealer (Sec. 3.2) is an ordinary path for the library: its
    amplitudes match the oracle's along the original greedy path."""
    from paper_2310_03978_amd import planner
    print(f"annealed path {prec}", flush=True)
    circ, net, best = configs.build("rqc12")
    ref = contract.amplitudes(net.tensors, net.labels, net.open_labels, best["path"])
    r = planner.refine(net.labels, net.open_labels, best["path"], sweeps=20, seed=2)
    assert r["path"] != list(best["path"])
    with tn.Plan(net.tensors, net.labels, net.open_labels, r["path"], (), precision=prec,
                 split_policy=2) as p:
        _assert_split_everywhere(p.steps(), prec)
        p.contract()
        got, _ = p.amplitudes()
    _check_amps(got, ref, prec, what="annealed path")


@pytest.mark.parametrize("prec", ["f16x3", "bf16x3"])
@pytest.mark.parametrize("total_exp", [7, 301])
def test_exponent_bookkeeping_with_prescaled_leaves(prec, total_exp):
    """Power-of-two scale and exponent bookkeeping (Sec. 4.2 dynamic scaling; the re-scaling
    outlook of Sec. 6): every leaf of the 30-qubit 12-cycle sub-case multiplied by a seeded
    2^e, e in [-40, 40] (the exponents summing to total_exp), gives the unscaled plan's
    amplitudes times 2^total_exp bit for bit (scaling by powers of two is exact in every
    step, and the exponents travel beside the values), and the oracle's amplitudes times
    2^total_exp within the precision's tolerance."""
    import importlib.util
    import os
    print(f"exponent bookkeeping {prec} total 2^{total_exp}", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_rqc30d12_amplitudes.py")
    spec = importlib.util.spec_from_file_location("make_rqc30d12_amplitudes", path)
    fx = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(fx)
    digest, ref = fx.read_fixture()
    _, net, best = configs.build("rqc30d12")
    assert digest == fx.network_digest(net, best)
    rng = np.random.default_rng(4040 + total_exp)
    e = rng.integers(-40, 41, size=len(net.tensors))
    # move the sum to total_exp through leaves that stay inside [-40, 40]
    rest = total_exp - int(e.sum())
    i = 0
    while rest != 0:
        step = int(np.clip(rest, -40 - e[i], 40 - e[i]))
        e[i] += step
        rest -= step
        i = (i + 1) % len(e)
    assert int(e.sum()) == total_exp and e.min() >= -40 and e.max() <= 40
    scaled = [np.asarray(t, dtype=np.complex128) * 2.0 ** int(x) for t, x in zip(net.tensors, e)]
    args = (net.labels, net.open_labels, best["path"])
    with tn.Plan(net.tensors, *args, precision=prec) as p:
        p.contract()
        base, _ = p.amplitudes()
    with tn.Plan(scaled, *args, precision=prec) as p:
        p.contract()
        got, _ = p.amplitudes()
    assert np.array_equal(got, np.ldexp(base.real, total_exp) + 1j * np.ldexp(base.imag, total_exp))
    unscaled = np.ldexp(got.real, -total_exp) + 1j * np.ldexp(got.imag, -total_exp)
    _check_amps(unscaled, ref, prec, what=f"prescaled leaves (2^{total_exp} overall)")
