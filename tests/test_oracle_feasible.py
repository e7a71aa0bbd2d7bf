"""Pins of the oracle's feasible IPM (Algorithm 2, Section 4) against the identities and the
optimum the paper fixes: the Newton system eq. iip_3_f (A dx = 0, A^T dy + ds = 0,
X ds + S dx = -XS1 + sigma mu 1 - v), dx^T ds = 0, the duality measure along the step
(Lemma maxalpha0 (b)), iterates inside N(gamma) (eq. neigh), and the LP optimum (HiGHS)."""
import numpy as np
import pytest
from scipy.optimize import linprog

import lpgen
from oracle import ipm as oipm


def _start(lp, perturb=0.0, seed=0):
    rng = np.random.default_rng(seed)
    x = lp.x0 * (1.0 + perturb * rng.uniform(-1.0, 1.0, lp.n))
    return oipm.feasible_state(lp.A, x, lp.y0, lp.s0)


@pytest.mark.parametrize("mode", ["exact", "sketch"])
def test_feasible_newton_system(mode):
    # x perturbed off A x = b, so that a right-hand side built from b (Algorithm 3's) would
    # give A dx = -r_p instead of 0
    lp = lpgen.dense_lp(20, 300, seed=3)
    st = _start(lp, perturb=1e-3)
    prm = oipm.Params(w=80, s=2, seed=1, feasible=True)
    new, info = oipm.step(lp.A, lp.b, lp.c, st, prm, mode, keep=True)
    assert info.status >= 0
    e = info.extra
    dx, dy, ds, v = e["dx"], e["dy"], e["ds"], e["v"]
    x, s = st.x, st.s
    mu = float(x @ s) / lp.n
    scale = np.linalg.norm(lp.A, 2) * np.linalg.norm(dx)
    assert np.linalg.norm(lp.A @ dx) <= 1e-9 * scale
    assert np.linalg.norm(lp.A.T @ dy + ds) <= 1e-12 * np.linalg.norm(ds)
    lhs = x * ds + s * dx
    rhs = -x * s + prm.sigma * mu - v
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(x * s)
    assert abs(dx @ ds) <= 1e-9 * np.linalg.norm(dx) * np.linalg.norm(ds)
    if mode == "sketch":
        assert np.linalg.norm(v) > 0.0


def test_feasible_rhs_from_b_would_fail_the_pin():
    """The A dx = 0 pin is sensitive to the right-hand side: the same direction built from
    p = b - sigma mu A S^-1 1 (right only at an exactly feasible x) violates it by ~||r_p||."""
    lp = lpgen.dense_lp(20, 300, seed=3)
    st = _start(lp, perturb=1e-3)
    x, s = st.x, st.s
    mu = float(x @ s) / lp.n
    d2 = x / s
    M = oipm.normal_matrix(lp.A, d2)
    for p, ok in ((oipm.rhs_p_feasible(lp.A, x, s, 0.5, mu), True),
                  (lp.b - 0.5 * mu * (lp.A @ (1.0 / s)), False)):
        dy = np.linalg.solve(M, p)
        ds = -(lp.A.T @ dy)
        dx = -x + 0.5 * mu / s - d2 * ds
        err = np.linalg.norm(lp.A @ dx)
        rp = np.linalg.norm(lp.A @ x - lp.b)
        if ok:
            assert err <= 1e-9 * rp
        else:
            assert err >= 0.5 * rp


def test_feasible_duality_measure_along_the_step():
    lp = lpgen.dense_lp(15, 200, seed=5)
    st = _start(lp)
    prm = oipm.Params(w=60, s=2, seed=2, feasible=True)
    for _ in range(4):
        new, info = oipm.step(lp.A, lp.b, lp.c, st, prm, "sketch", keep=True)
        v = info.extra["v"]
        mu = float(st.x @ st.s) / lp.n
        a = info.alpha
        want = (1.0 - a * (1.0 - prm.sigma)) * mu - a * v.sum() / lp.n
        got = float(new.x @ new.s) / lp.n
        assert got == pytest.approx(want, rel=1e-10)
        st = new


@pytest.mark.parametrize("m,n,seed", [(10, 120, 0), (30, 600, 1)])
def test_feasible_solve_reaches_the_optimum(m, n, seed):
    lp = lpgen.dense_lp(m, n, seed=seed)
    prm = oipm.Params(w=4 * m, s=2, seed=seed, feasible=True)
    inside = []

    def cb(st, info):
        mu = float(st.x @ st.s) / n
        inside.append(bool(np.all(st.x * st.s >= (1.0 - prm.gamma) * mu * (1 - 1e-12))))

    res = oipm.solve(lp.A, lp.b, lp.c, prm, "sketch", st=_start(lp), callback=cb)
    assert res.converged and all(inside)
    ref = linprog(lp.c, A_eq=lp.A, b_eq=lp.b, bounds=(0, None), method="highs")
    obj = float(lp.c @ res.state.x)
    assert abs(obj - ref.fun) <= 1e-8 * (1 + abs(ref.fun))
    # started feasible, the iterates stay feasible up to rounding
    last = res.infos[-1]
    assert last.rp_rel <= 1e-9 and last.rd_rel <= 1e-9
