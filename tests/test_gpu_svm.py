"""The v-correction ablation on l1-SVM LPs (Section 7, the no-correction comparison) through the
C ABI: lock-step parity with the oracle with the perturbation v on and off, and solves at the
experiments' four shapes (Table 1) with v on and off reaching the same optimum; the smallest
shape against HiGHS."""
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


@pytest.mark.parametrize("vcorr", [1, 0])
def test_svm_lockstep(ctx, vcorr):
    lp = lpgen.svm_lp(30, 300, seed=2)
    prob = P.Problem.from_lp(lp)
    oprm = oipm.Params(w=120, s=2, seed=5, vcorr=bool(vcorr))
    gprm = P.Params(w=120, s=2, seed=5, vcorr=vcorr)

    def v_on_off(old, gst, ginfo, oinfo):
        assert (ginfo["vnorm"] > 0) == bool(vcorr)

    _, _, conv = lockstep.run(P, ctx, lp.A, lp.b, lp.c, prob, oprm, gprm, 200, check=v_on_off,
                              label=f"l1-SVM 30x300, v {'on' if vcorr else 'off'}")
    assert conv


def _kkt(lp, res):
    x, y, s = host(res.state.x), host(res.state.y), host(res.state.s)
    obj, dual = float(lp.c @ x), float(lp.b @ y)
    assert abs(obj - dual) / (1 + abs(obj)) <= 1e-8
    assert np.linalg.norm(lp.A @ x - lp.b) / (1 + np.linalg.norm(lp.b)) <= 1e-8
    assert np.linalg.norm(lp.A.T @ y + s - lp.c) / (1 + np.linalg.norm(lp.c)) <= 1e-8
    return obj


@pytest.mark.parametrize("name", list(lpgen.SVM_SHAPES))
def test_svm_shapes_with_and_without_v(ctx, name):
    sh = lpgen.SVM_SHAPES[name]
    lp = lpgen.svm_lp(sh["m"], sh["N"], seed=0)
    prob = P.Problem.from_lp(lp)
    on = P.solve(ctx, prob, P.Params(w=sh["w"], s=2, seed=0, vcorr=1))
    off = P.solve(ctx, prob, P.Params(w=sh["w"], s=2, seed=0, vcorr=0))
    assert on.converged and off.converged
    o1, o0 = _kkt(lp, on), _kkt(lp, off)
    # both are upper bounds of the optimum within their own relative gap (<= 1e-8)
    assert abs(o1 - o0) <= 1e-8 * (1 + abs(o1))
    if name == "arcene":
        ref = linprog(lp.c, A_eq=lp.A, b_eq=lp.b, bounds=(0, None), method="highs")
        assert abs(o1 - ref.fun) <= 1e-8 * (1 + abs(ref.fun))
    print(f"\n{name}: outer iterations with v {on.iterations}, without v {off.iterations}", flush=True)
