"""tn_gemm_noalloc (the product with the library's fixed per-device scratch array, for
callers that cannot allocate device memory) against tn_gemm on the same operands.

Both run the same kernels, so the results must be equal bit for bit.  Two calls in a row
per precision, the second with a smaller problem, so the second runs on an array that still
holds the first call's slots and K-split partials; a third problem whose scratch is above
the fixed size must be refused before anything is launched.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
tn = pytest.importorskip("paper_2310_03978_amd.tn")

# (batch, m, n, k): 256 x 128 output with k = 8192 splits K 64 ways (16 MiB of partials);
# the second, smaller product splits K 8 ways
CALLS = [(1, 256, 128, 8192), (2, 64, 32, 2048)]
GEMM_TOL = {"c64": 2e-6, "f16x3": 2e-6, "bf16x3": 1e-4}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _operands(seed, b, m, n, k):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((b, m, k)) + 1j * rng.standard_normal((b, m, k))).astype(np.complex64)
    B = (rng.standard_normal((b, k, n)) + 1j * rng.standard_normal((b, k, n))).astype(np.complex64)
    return A, B


@pytest.mark.parametrize("prec", ["c64", "f16x3", "bf16x3"])
def test_gemm_noalloc_matches_gemm(prec):
    for i, (b, m, n, k) in enumerate(CALLS):
        print(f"gemm_noalloc {prec} call {i}: b={b} m={m} n={n} k={k}", flush=True)
        A, B = _operands(1000 + i, b, m, n, k)
        dA, dB = torch.from_numpy(A).to("cuda"), torch.from_numpy(B).to("cuda")
        ref = torch.zeros((b, m, n), dtype=torch.complex64, device="cuda")
        got = torch.full((b, m, n), complex(7.0, -7.0), dtype=torch.complex64, device="cuda")
        tn.tn_gemm(dA, dB, ref, precision=prec)
        tn.tn_gemm(dA, dB, got, precision=prec, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(got.view(torch.float32), ref.view(torch.float32)), (prec, i)
        exact = np.matmul(A.astype(np.complex128), B.astype(np.complex128))
        err = np.linalg.norm(got.cpu().numpy() - exact) / np.linalg.norm(exact)
        print(f"  rel err vs complex128 {err:.3e}", flush=True)
        assert err <= GEMM_TOL[prec] * max(1.0, np.sqrt(k / 64)), err


def test_gemm_noalloc_refuses_oversized_scratch():
    # 1024 x 1024 output with k = 4096 splits K 32 ways: 256 MiB of partials, above the array
    b, m, n, k = 1, 1024, 1024, 4096
    A = torch.zeros((b, m, k), dtype=torch.complex64, device="cuda")
    B = torch.zeros((b, k, n), dtype=torch.complex64, device="cuda")
    C = torch.full((b, m, n), complex(3.0, 1.0), dtype=torch.complex64, device="cuda")
    with pytest.raises(tn.TnError) as e:
        tn.tn_gemm(A, B, C, precision="f16x3", noalloc=True)
    assert e.value.status == -6 and "scratch" in str(e.value), e.value
    torch.cuda.synchronize()
    assert bool((C == complex(3.0, 1.0)).all())
