"""Parity of the Gaussian sketch (params.sketch = IPM_SKETCH_GAUSSIAN; the experiments' sketching
matrix, Section 7) with the oracle: B = A D W element by element (both sides generate W from the
same counter-based definition; they differ only in the rounding of log and cos), the IPM step
in lock-step, solves against HiGHS, and the 500 x 100000 workload's sketch on sampled rows and
its solve against the sparse-embedding solve."""
import numpy as np
import pytest
from scipy.optimize import linprog

import lockstep
import lpgen
from oracle import ipm as oipm
from oracle import sketch as osk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P = None
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _ref_and_bound(A, d, w, seed, k, chunk=4096):
    """The oracle's A diag(d) W (its sketch_gaussian, chunk by chunk) and |A| diag(d) |W| (the
    scale of the summation error), from one generation of each chunk of W."""
    m, n = A.shape
    ref, bound = np.zeros((m, w)), np.zeros((m, w))
    for j0 in range(0, n, chunk):
        j1 = min(n, j0 + chunk)
        Wc = osk.gaussian_rows(j0, j1, w, seed, k)
        Ad = A[:, j0:j1] * d[j0:j1]
        ref += Ad @ Wc
        bound += np.abs(Ad) @ np.abs(Wc)
    return ref, bound


@pytest.mark.parametrize("m,n,w,dtype", [(50, 2000, 200, "f64"), (37, 1001, 74, "f64"), (130, 5003, 500, "f32"),
                                         (300, 20011, 1200, "bf16"), (1, 300, 7, "f64"), (257, 4096, 129, "f64")])
def test_gaussian_sketch_parity(ctx, m, n, w, dtype):
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n))
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    if dtype == "bf16":
        A = lpgen.bf16_round(A)
    elif dtype == "f32":
        A = lpgen.f32_round(A)
    d = np.exp(rng.uniform(-2, 2, n))
    B = host(P.ipm_sketch_gaussian(ctx, P.Matrix.from_numpy(A, dtype=tdt), dev(d), 11, 3, w))
    ref, bound = _ref_and_bound(A, d, w, 11, 3)
    assert np.allclose(ref, osk.sketch_gaussian(A, d, w, 11, 3), rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    assert np.all(np.abs(B - ref) <= 64 * EPS * np.sqrt(n) * bound + 1e-300)


def test_gaussian_sketch_rejects_csr(ctx):
    import scipy.sparse as sp
    A = sp.random(10, 200, density=0.1, random_state=1, format="csr")
    with pytest.raises(P.IpmError) as ei:
        P.ipm_sketch_gaussian(ctx, P.SparseMatrix.from_scipy(A), dev(np.ones(200)), 0, 0, 40)
    assert ei.value.code == -1


@pytest.mark.parametrize("vcorr", [1, 0])
def test_gaussian_lockstep(ctx, vcorr):
    lp = lpgen.dense_lp(30, 1500, seed=8)
    prob = P.Problem.from_lp(lp)
    oprm = oipm.Params(w=120, s=2, seed=4, sketch=1, vcorr=bool(vcorr))
    gprm = P.Params(w=120, s=2, seed=4, sketch=1, vcorr=vcorr)
    _, _, conv = lockstep.run(P, ctx, lp.A, lp.b, lp.c, prob, oprm, gprm, 200,
                              label=f"Gaussian sketch, v {'on' if vcorr else 'off'}")
    assert conv


@pytest.mark.parametrize("m,n,precision", [(20, 800, 0), (60, 6000, 0), (60, 6000, 1)])
def test_gaussian_solve_matches_highs(ctx, m, n, precision):
    lp = lpgen.dense_lp(m, n, seed=m)
    dt = torch.float64 if precision == 0 else torch.float32
    A = lp.A if precision == 0 else lpgen.f32_round(lp.A)
    b = lp.b if precision == 0 else A @ lp.x0
    c = lp.c if precision == 0 else A.T @ lp.y0 + lp.s0
    prob = P.Problem(P.Matrix.from_numpy(A, dtype=dt), dev(b), dev(c))
    res = P.solve(ctx, prob, P.Params(w=4 * m, s=2, seed=2, sketch=1, precision=precision))
    ref = linprog(c, A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    assert res.converged
    obj = float(c @ host(res.state.x))
    # an upper bound of the optimum within the solve's relative gap (<= 1e-8)
    assert abs(obj - ref.fun) <= 1e-8 * (1 + abs(ref.fun))


def test_gaussian_full_size(ctx):
    """500 x 100000 (the bench workload), w = 2000: sampled rows of the sketch against the oracle,
    and the Gaussian-sketch solve against the sparse-embedding solve and the host KKT check."""
    lp = lpgen.workload("dense_500x100000", seed=0)
    prob = P.Problem.from_lp(lp)
    rng = np.random.default_rng(3)
    d = np.exp(rng.uniform(-3, 3, lp.n))
    B = host(P.ipm_sketch_gaussian(ctx, prob.A, dev(d), 5, 2, 2000))
    rows = np.sort(rng.choice(lp.m, size=12, replace=False))
    ref, bound = _ref_and_bound(lp.A[rows], d, 2000, 5, 2)
    assert np.all(np.abs(B[rows] - ref) <= 64 * EPS * np.sqrt(lp.n) * bound)
    g = P.solve(ctx, prob, P.Params(w=2000, s=2, seed=0, sketch=1))
    sp_ = P.solve(ctx, prob, P.Params(w=2000, s=2, seed=0))
    assert g.converged and sp_.converged
    x, y, s = host(g.state.x), host(g.state.y), host(g.state.s)
    og, osp = float(lp.c @ x), float(lp.c @ host(sp_.state.x))
    assert abs(og - float(lp.b @ y)) <= 1e-8 * (1 + abs(og))
    assert np.linalg.norm(lp.A @ x - lp.b) <= 1e-8 * (1 + np.linalg.norm(lp.b))
    # both are upper bounds of the optimum within their own relative gap (<= 1e-8)
    assert abs(og - osp) <= 1e-8 * (1 + abs(osp))
    cg_g = sum(i["pcg_iters"] for i in g.infos if i["rc"] != 1)
    cg_s = sum(i["pcg_iters"] for i in sp_.infos if i["rc"] != 1)
    print(f"\nGaussian: {g.iterations} IPM / {cg_g} CG iterations; sparse: {sp_.iterations} / {cg_s}", flush=True)
