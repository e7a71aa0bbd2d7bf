"""The largest one-GPU dense workload at full size: A 2000 x 2*10^6, i.i.d. N(0, 1) rounded to
BF16 (8 GB), with an FP64 copy of the same values (32 GB) for the plain form; sketch w = 16000,
s = 2; generated in device memory.

The oracle's IPM is out of reach here (its normal matrix costs 8e12 flops per iteration), so the
checks are: the CG matvec over both storages element by element against its definition
A (d^2 o (A^T v)) evaluated on the host in FP64 from the stored values; sampled rows of the
sketch against the oracle's sketch of the same rows; and for the plain and the mixed solve the
stop test recomputed on the host in FP64 and the duality sandwich of the generator's witness
pair. The host evaluations stream A in column blocks.
"""
import numpy as np
import pytest

from oracle import sketch as osk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P = None
M_, N_, W_, S_ = 2000, 2_000_000, 16000, 2
BLOCK = 1 << 17
EPS = np.finfo(float).eps


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


@pytest.fixture(scope="module")
def lp(ctx):
    from lpgen import device as gdev
    print(f"\ngenerating the {M_} x {N_} BF16 LP (seed 0) and its FP64 copy in device memory", flush=True)
    out = gdev.dense_lp(M_, N_, seed=0, storage="bf16")
    torch.cuda.synchronize()
    yield out
    del out
    torch.cuda.empty_cache()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def column_blocks(lp):
    """(j0, j1, A[:, j0:j1] as FP64 on the host): the stored BF16 values, exactly."""
    for j0 in range(0, N_, BLOCK):
        j1 = min(N_, j0 + BLOCK)
        yield j0, j1, host(lp.A[:, j0:j1].to(torch.float64))


def test_matvec_both_storages(ctx, lp):
    rng = np.random.default_rng(1)
    d2 = np.exp(rng.uniform(-6, 6, N_))
    v = rng.standard_normal(M_)
    ref = np.zeros(M_)
    bound = np.zeros(M_)
    for j0, j1, Ab in column_blocks(lp):
        ref += Ab @ (d2[j0:j1] * (Ab.T @ v))
        aa = np.abs(Ab)
        bound += aa @ (d2[j0:j1] * (aa.T @ np.abs(v)))
    dev = lambda a: torch.from_numpy(a).to("cuda:0")  # noqa: E731
    for name, Amat in (("bf16", P.Matrix(lp.A, N_)), ("f64", P.Matrix(lp.A64, N_))):
        q = host(P.ipm_normal_matvec(ctx, Amat, dev(d2), dev(v)))
        err = np.max(np.abs(q - ref) / bound)
        print(f"\n{name} storage: largest error / summation bound scale {err:.2e}", flush=True)
        # FP64 accumulation over exactly stored values: only the summation order differs
        assert np.all(np.abs(q - ref) <= 64 * EPS * (M_ + np.sqrt(N_)) * bound)


def test_sketch_sampled_rows(ctx, lp):
    """B = A D W acts row by row: 24 sampled rows of the GPU's B (both storages, FP64 and FP32
    B) against the oracle's sketch of the same rows of A."""
    rng = np.random.default_rng(2)
    d = np.exp(rng.uniform(-3, 3, N_))
    rows = np.sort(rng.choice(M_, size=24, replace=False))
    Ar = host(lp.A[torch.from_numpy(rows).to("cuda:0")][:, :N_].to(torch.float64))
    ref = osk.sketch_ADW(Ar, d, W_, S_, 5, 3)
    Wm = osk.sketch_matrix(N_, W_, S_, 5, 3)
    bound = np.asarray((abs(Wm).T @ (np.abs(Ar) * d).T).T)
    dd = torch.from_numpy(d).to("cuda:0")
    idx = torch.from_numpy(rows).to("cuda:0")
    for Amat in (P.Matrix(lp.A, N_), P.Matrix(lp.A64, N_)):
        B = P.ipm_sketch(ctx, Amat, dd, 5, 3, W_, S_)
        Bs = host(B[idx])
        del B
        assert np.all(np.abs(Bs - ref) <= 32 * EPS * np.sqrt(N_) * bound + 1e-300)
    B32 = P.ipm_sketch(ctx, P.Matrix(lp.A, N_), dd, 5, 3, W_, S_, out_dtype=torch.float32)
    Bs = host(B32[idx])
    del B32
    # FP64 accumulation, then at most a few FP32 roundings (one per column chunk added atomically)
    assert np.all(np.abs(Bs - ref) <= 4 * 2.0 ** -24 * bound + 32 * EPS * np.sqrt(N_) * bound)


def _check_solution(lp, res, label):
    """Stop test and duality sandwich recomputed on the host in FP64 from the stored A."""
    b, c = host(lp.b), host(lp.c)
    x, y, s = host(res.state.x), host(res.state.y), host(res.state.s)
    assert np.all(x > 0) and np.all(s > 0)
    Ax = np.zeros(M_)
    rd2 = 0.0
    for j0, j1, Ab in column_blocks(lp):
        Ax += Ab @ x[j0:j1]
        r = Ab.T @ y + s[j0:j1] - c[j0:j1]
        rd2 += float(r @ r)
    obj, dual = float(c @ x), float(b @ y)
    relgap = abs(obj - dual) / (1 + abs(obj))
    rp = np.linalg.norm(Ax - b) / (1 + np.linalg.norm(b))
    rd = np.sqrt(rd2) / (1 + np.linalg.norm(c))
    print(f"\n{label}: {res.iterations} IPM iterations, objective {obj:.12e}, relgap {relgap:.2e}, "
          f"rp {rp:.2e}, rd {rd:.2e} (host FP64)", flush=True)
    assert relgap <= 1e-8 and rp <= 1e-8 and rd <= 1e-8
    lo, hi = float(b @ host(lp.y0)), float(c @ host(lp.x0))
    assert lo - 1e-8 * abs(lo) <= obj <= hi + 1e-8 * abs(hi)
    return obj


@pytest.mark.timeout(600)
def test_plain_and_mixed_solves(ctx, lp):
    plain = P.solve(ctx, P.Problem(P.Matrix(lp.A64, N_), lp.b, lp.c), P.Params(w=W_, s=S_, seed=0))
    assert plain.converged
    op = _check_solution(lp, plain, "plain FP64")
    mixed = P.solve(ctx, P.Problem(P.Matrix(lp.A, N_), lp.b, lp.c),
                    P.Params(w=W_, s=S_, seed=0, precision=P.IPM_MIXED))
    assert mixed.converged
    om = _check_solution(lp, mixed, "mixed BF16")
    # both objectives are upper bounds of the optimum within their own relative gap (<= 1e-8)
    assert abs(op - om) <= 1e-8 * (1 + abs(op))
    assert abs(plain.iterations - mixed.iterations) <= 3
