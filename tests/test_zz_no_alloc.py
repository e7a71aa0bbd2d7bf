"""The allocation-free matvec (ipm_normal_matvec_noalloc) against ipm_normal_matvec, through the
C ABI: the same kernels on the same inputs, so the results must agree bit for bit; two calls in
a row with the second on a smaller input (the shared scratch keeps the first call's partials);
dense FP64, ragged BF16 and CSR A; a need beyond the static scratch is IPM_ERR_ARG."""
import numpy as np
import pytest
import scipy.sparse as sp

import lpgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P = None


@pytest.fixture(scope="module")
def ctx():
    global P
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_08722_amd as mod
    P = mod
    c = mod.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _pair(ctx, A, m, n, seed):
    rng = np.random.default_rng(seed)
    d2 = dev(np.exp(rng.uniform(-4, 4, n)))
    v = dev(rng.standard_normal(m))
    ref = P.ipm_normal_matvec(ctx, A, d2, v)
    q = torch.full((m,), float("nan"), dtype=torch.float64, device="cuda:0")
    P.ipm_normal_matvec_noalloc(ctx, A, d2, v, q)
    torch.cuda.synchronize()
    return q.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_matches_the_allocating_matvec_twice(ctx):
    # first call: 500 x 100000 FP64 (every block of the odd grid writes 500 partials)
    rng = np.random.default_rng(0)
    A1 = P.Matrix.from_numpy(rng.standard_normal((500, 100_000)))
    q, ref = _pair(ctx, A1, 500, 100_000, 1)
    assert np.array_equal(q, ref)
    # second call, smaller: 37 x 1001 BF16 (fewer blocks and rows than the partials left behind)
    A2 = P.Matrix.from_numpy(lpgen.bf16_round(rng.standard_normal((37, 1001))), dtype=torch.bfloat16)
    q, ref = _pair(ctx, A2, 37, 1001, 2)
    assert np.array_equal(q, ref)
    # CSR A (column pass over the CSC mirror, row pass over CSR)
    S = sp.random(300, 20_000, density=2e-3, random_state=3, format="csr")
    A3 = P.SparseMatrix.from_scipy(S)
    q, ref = _pair(ctx, A3, 300, 20_000, 3)
    assert np.array_equal(q, ref)
    # and the first shape again after the smaller ones
    q, ref = _pair(ctx, A1, 500, 100_000, 4)
    assert np.array_equal(q, ref)


def test_noalloc_rejects_a_need_beyond_the_scratch(ctx):
    # BF16 with 6000 rows takes the re-read pass: 511 blocks x 6000 rows of partials > 16 MB
    m, n = 6000, 40_000
    A = P.Matrix(torch.zeros((m, n), dtype=torch.bfloat16, device="cuda:0"), n)
    d2 = torch.ones(n, dtype=torch.float64, device="cuda:0")
    v = torch.ones(m, dtype=torch.float64, device="cuda:0")
    q = torch.zeros(m, dtype=torch.float64, device="cuda:0")
    with pytest.raises(P.IpmError) as ei:
        P.ipm_normal_matvec_noalloc(ctx, A, d2, v, q)
    assert ei.value.code == -1 and "scratch" in str(ei.value)
    assert float(q.abs().sum()) == 0.0
