"""Parity of the library's feasible IPM (Algorithm 2, params.feasible = 1) with the oracle's.

Lock-step from a point off A x = b (so that the feasible right-hand side p = A x -
sigma mu A S^-1 1 differs from the infeasible method's), dense and CSR; full solves from the
generator's strictly feasible pair against the HiGHS optimum, with every iterate inside
N(gamma) and the residuals kept at rounding level; the 500 x 100000 workload's feasible solve
against its infeasible one.
"""
import numpy as np
import pytest
from scipy.optimize import linprog

import lockstep
import lpgen
from oracle import ipm as oipm

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


def _start(lp, perturb=0.0, seed=0):
    rng = np.random.default_rng(seed)
    x = lp.x0 * (1.0 + perturb * rng.uniform(-1.0, 1.0, lp.n))
    return oipm.feasible_state(lp.A, x, lp.y0, lp.s0)


def _gpu_state(st):
    return P.State(dev(st.x), dev(st.y), dev(st.s), st.k, st.mu0, st.r0norm)


def _problem(lp, sparse):
    A = P.SparseMatrix.from_scipy(lp.A) if sparse else P.Matrix.from_numpy(lp.A)
    return P.Problem(A, dev(lp.b), dev(lp.c))


@pytest.mark.parametrize("sparse", [False, True])
def test_feasible_lockstep(ctx, sparse):
    lp = lpgen.sparse_lp(40, 3000, 0.02, seed=4) if sparse else lpgen.dense_lp(30, 1500, seed=4)
    prob = _problem(lp, sparse)
    oprm = oipm.Params(w=120 if not sparse else 160, s=2, seed=6, feasible=True)
    gprm = P.Params(w=oprm.w, s=2, seed=6, feasible=1)
    st = _start(lp, perturb=1e-3)

    def keeps_ax(old, gst, ginfo, oinfo):
        # the feasible step keeps A x where it was (A dx = 0): r_p does not contract
        assert np.linalg.norm(lp.A @ host(gst.x) - lp.A @ old.x) <= 1e-9 * np.linalg.norm(lp.A @ old.x)

    # the start is off A x = b and the feasible method keeps A x fixed, so r_p stays at its
    # starting level and the stop test is never met: 40 steps (mu falls by about 1e-9)
    recs, _, _ = lockstep.run(P, ctx, lp.A, lp.b, lp.c, prob, oprm, gprm, 40, st=st, check=keeps_ax,
                              label=f"feasible, {'CSR' if sparse else 'dense'}")
    assert len(recs) == 40


@pytest.mark.parametrize("m,n,sparse", [(20, 400, False), (60, 6000, True), (100, 20000, False)])
def test_feasible_solve_matches_highs(ctx, m, n, sparse):
    lp = lpgen.sparse_lp(m, n, 0.01, seed=m) if sparse else lpgen.dense_lp(m, n, seed=m)
    prob = _problem(lp, sparse)
    prm = P.Params(w=4 * m, s=2, seed=3, feasible=1)
    inside = []

    def cb(st, info):
        x, s = host(st.x), host(st.s)
        mu = float(x @ s) / n
        inside.append(bool(np.all(x * s >= (1.0 - prm.gamma) * mu * (1 - 1e-12))))

    res = P.solve(ctx, prob, prm, st=_gpu_state(_start(lp)), callback=cb)
    assert res.converged and all(inside)
    ref = linprog(lp.c, A_eq=lp.A, b_eq=lp.b, bounds=(0, None), method="highs")
    obj = float(lp.c @ host(res.state.x))
    assert abs(obj - ref.fun) <= 1e-8 * (1 + abs(ref.fun))
    last = res.infos[-1]
    assert last["rp_rel"] <= 1e-9 and last["rd_rel"] <= 1e-9


def test_feasible_against_infeasible_full_size(ctx):
    """Algorithm 2 from the witness pair and Algorithm 3 from x = s = 1, y = 0 on the
    500 x 100000 workload reach the same optimum."""
    lp = lpgen.workload("dense_500x100000", seed=0)
    prob = P.Problem.from_lp(lp)
    feas = P.solve(ctx, prob, P.Params(w=2000, s=2, seed=0, feasible=1), st=_gpu_state(_start(lp)))
    infeas = P.solve(ctx, prob, P.Params(w=2000, s=2, seed=0))
    assert feas.converged and infeas.converged
    of, oi = float(lp.c @ host(feas.state.x)), float(lp.c @ host(infeas.state.x))
    print(f"\nfeasible: {feas.iterations} iterations, infeasible: {infeas.iterations}", flush=True)
    # both are upper bounds of the optimum within their own relative gap (<= 1e-8)
    assert abs(of - oi) <= 1e-8 * (1 + abs(oi))
