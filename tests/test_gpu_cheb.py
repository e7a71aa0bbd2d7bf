"""Parity of the Chebyshev solver (params.solver = IPM_SOLVER_CHEBYSHEV; Section 3.2) with the
oracle: the solve alone (same CG probe, same Ritz interval, same recurrence) against
oracle.ipm.pcg_chebyshev, the IPM step in lock-step, solves against HiGHS (dense and CSR), and
the 500 x 100000 workload against its CG solve."""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.optimize import linprog

import lockstep
import lpgen
from oracle import ipm as oipm
from oracle import sketch as osk

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


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("m,n,w,spread", [(50, 2000, 200, 5.0), (120, 9001, 480, 8.0), (37, 1001, 74, 3.0)])
def test_chebyshev_solve_parity(ctx, m, n, w, spread):
    rng = np.random.default_rng(m)
    A = rng.standard_normal((m, n))
    d2 = np.exp(rng.uniform(-spread, spread, n))
    B = osk.sketch_ADW(A, np.sqrt(d2), w, 2, 3, 0)
    L = np.linalg.cholesky(B @ B.T)
    Linv = sla.solve_triangular(L, np.eye(m), lower=True)
    p = rng.standard_normal(m)
    M = (A * d2) @ A.T
    ores = oipm.pcg_chebyshev(lambda v: M @ v, L, p, 1e-10, 500)
    prm = P.Params(w=w, s=2, solver=1)
    dy, info = P.ipm_pcg_solve(ctx, P.Matrix.from_numpy(A), dev(d2), dev(Linv), dev(p), prm)
    assert info["status"] == 0 and ores.status == oipm.OK
    assert ores.interval                                  # the probe did not already converge
    assert abs(info["iters"] - ores.iters) <= max(2, 0.05 * ores.iters)
    # the true preconditioned residual of the GPU solution meets the tolerance
    g = host(dy)
    rr = sla.solve_triangular(L, p - M @ g, lower=True)
    assert np.linalg.norm(rr) <= 1e-10 * np.linalg.norm(sla.solve_triangular(L, p, lower=True)) * 1.05
    assert np.linalg.norm(g - ores.dy) <= 1e-8 * np.linalg.norm(ores.dy)


@pytest.mark.parametrize("sparse", [False, True])
def test_chebyshev_lockstep(ctx, sparse):
    lp = lpgen.sparse_lp(40, 3000, 0.02, seed=3) if sparse else lpgen.dense_lp(30, 1500, seed=9)
    A = P.SparseMatrix.from_scipy(lp.A) if sparse else P.Matrix.from_numpy(lp.A)
    prob = P.Problem(A, dev(lp.b), dev(lp.c))
    w = 4 * lp.m
    oprm = oipm.Params(w=w, s=2, seed=2, solver=1)
    gprm = P.Params(w=w, s=2, seed=2, solver=1)
    _, _, conv = lockstep.run(P, ctx, lp.A, lp.b, lp.c, prob, oprm, gprm, 200, pcg_slack=2,
                              label=f"Chebyshev, {'CSR' if sparse else 'dense'}")
    assert conv


@pytest.mark.parametrize("m,n,sparse", [(20, 800, False), (60, 6000, False), (60, 8000, True)])
def test_chebyshev_solve_matches_highs(ctx, m, n, sparse):
    lp = lpgen.sparse_lp(m, n, 0.01, seed=m) if sparse else lpgen.dense_lp(m, n, seed=m)
    A = P.SparseMatrix.from_scipy(lp.A) if sparse else P.Matrix.from_numpy(lp.A)
    prob = P.Problem(A, dev(lp.b), dev(lp.c))
    res = P.solve(ctx, prob, P.Params(w=4 * m, s=2, seed=2, solver=1))
    Ad = lp.A.toarray() if sparse else lp.A
    ref = linprog(lp.c, A_eq=Ad, b_eq=lp.b, bounds=(0, None), method="highs")
    assert res.converged
    obj = float(lp.c @ host(res.state.x))
    # an upper bound of the optimum within the solve's relative gap (<= 1e-8)
    assert abs(obj - ref.fun) <= 1e-8 * (1 + abs(ref.fun))


def test_chebyshev_full_size(ctx):
    lp = lpgen.workload("dense_500x100000", seed=0)
    prob = P.Problem.from_lp(lp)
    ch = P.solve(ctx, prob, P.Params(w=2000, s=2, seed=0, solver=1))
    cg = P.solve(ctx, prob, P.Params(w=2000, s=2, seed=0))
    assert ch.converged and cg.converged
    o1, o0 = float(lp.c @ host(ch.state.x)), float(lp.c @ host(cg.state.x))
    # both are upper bounds of the optimum within their own relative gap (<= 1e-8)
    assert abs(o1 - o0) <= 1e-8 * (1 + abs(o0))
    n1 = sum(i["pcg_iters"] for i in ch.infos if i["rc"] != 1)
    n0 = sum(i["pcg_iters"] for i in cg.infos if i["rc"] != 1)
    print(f"\nChebyshev: {ch.iterations} IPM / {n1} inner iterations; CG: {cg.iterations} / {n0}", flush=True)
