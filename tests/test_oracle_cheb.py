"""Pins of the oracle's Chebyshev iteration (Section 3.2) and of its eigenvalue estimate:
the residual bound of Gutknecht's Theorem 1.6.2 (eq. cs) per iteration with exact spectral
bounds, a one-step solve for a single-eigenvalue spectrum, Lanczos Ritz values (exact after m
CG steps, interlaced before), convergence of the CG-probe + Chebyshev solver to the tolerance
on a sketch-preconditioned normal matrix, and the IPM's optimum with it."""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.optimize import linprog

import lpgen
from oracle import ipm as oipm
from oracle import sketch as osk


def _diag_system(lams, seed=0):
    rng = np.random.default_rng(seed)
    m = lams.size
    Qo, _ = np.linalg.qr(rng.standard_normal((m, m)))
    M = (Qo * lams) @ Qo.T
    return M, rng.standard_normal(m)


@pytest.mark.parametrize("kappa", [4.0, 9.0, 100.0])
def test_chebyshev_residual_bound(kappa):
    m = 60
    lams = np.concatenate([[1.0, kappa], np.random.default_rng(1).uniform(1.0, kappa, m - 2)])
    M, p = _diag_system(lams)
    L = np.eye(m)                       # Q = I: the preconditioned matrix is M itself
    U = kappa
    dy, r, it, status, hist = oipm.chebyshev(lambda v: M @ v, L, p, 1.0, kappa, 1e-300, 40, np.zeros(m),
                                             p.copy(), float(p @ p), [float(np.linalg.norm(p))])
    assert it == 40
    q = (np.sqrt(U) + 1) / (np.sqrt(U) - 1)
    for t, res in enumerate(hist):
        bound = 2.0 / (q ** t + q ** (-t))
        assert res <= bound * hist[0] * (1 + 1e-9) + 1e-300, (t, res / hist[0], bound)
    # the recursive residual is the true one
    assert np.linalg.norm(r - (p - M @ dy)) <= 1e-10 * np.linalg.norm(p)


def test_chebyshev_single_eigenvalue_one_step():
    m = 20
    M, p = _diag_system(np.full(m, 3.0))
    dy, r, it, status, hist = oipm.chebyshev(lambda v: M @ v, np.eye(m), p, 3.0, 3.0, 1e-12, 10, np.zeros(m),
                                             p.copy(), float(p @ p), [float(np.linalg.norm(p))])
    assert it == 1 and status == oipm.OK
    assert np.allclose(dy, p / 3.0, rtol=1e-14, atol=1e-14)


def test_lanczos_ritz_values():
    rng = np.random.default_rng(3)
    m = 12
    lams = np.sort(rng.uniform(0.5, 5.0, m))
    M, p = _diag_system(lams, seed=4)
    L = np.linalg.cholesky(np.diag(rng.uniform(0.5, 2.0, m)))   # a non-trivial preconditioner
    K = sla.solve_triangular(L, sla.solve_triangular(L, M, lower=True).T, lower=True)   # L^-1 M L^-T
    ev = np.linalg.eigvalsh(K)
    full = oipm.pcg(lambda v: M @ v, L, p, 0.0, m)
    ritz = oipm.lanczos_ritz(full.alphas, full.history)
    assert np.allclose(ritz, ev, rtol=1e-8)
    part = oipm.pcg(lambda v: M @ v, L, p, 0.0, 5)
    rp = oipm.lanczos_ritz(part.alphas, part.history)
    assert rp.size == 5 and rp[0] >= ev[0] * (1 - 1e-12) and rp[-1] <= ev[-1] * (1 + 1e-12)


def test_pcg_chebyshev_meets_the_tolerance():
    lp = lpgen.dense_lp(40, 2000, seed=2)
    rng = np.random.default_rng(5)
    d2 = np.exp(rng.uniform(-4, 4, 2000))
    M = (lp.A * d2) @ lp.A.T
    B = osk.sketch_ADW(lp.A, np.sqrt(d2), 160, 2, 7, 1)
    L = np.linalg.cholesky(B @ B.T)
    p = rng.standard_normal(40)
    res = oipm.pcg_chebyshev(lambda v: M @ v, L, p, 1e-10, 500)
    assert res.status == oipm.OK and res.interval and res.iters > 10
    lo, hi = res.interval
    K = sla.solve_triangular(L, sla.solve_triangular(L, M, lower=True).T, lower=True)
    ev = np.linalg.eigvalsh(K)
    assert lo <= ev[0] and hi >= ev[-1]            # the margins cover the true spectrum here
    true = sla.solve_triangular(L, p - M @ res.dy, lower=True)
    ref = sla.solve_triangular(L, p, lower=True)
    assert np.linalg.norm(true) <= 1e-10 * np.linalg.norm(ref) * 1.01
    cg = oipm.pcg(lambda v: M @ v, L, p, 1e-10, 500)
    assert cg.iters <= res.iters                    # CG is optimal in the Krylov space


def test_chebyshev_ipm_reaches_the_optimum():
    lp = lpgen.dense_lp(20, 500, seed=7)
    res = oipm.solve(lp.A, lp.b, lp.c, oipm.Params(w=80, s=2, seed=1, solver=1), "sketch")
    ref = linprog(lp.c, A_eq=lp.A, b_eq=lp.b, bounds=(0, None), method="highs")
    assert res.converged
    assert abs(float(lp.c @ res.state.x) - ref.fun) <= 1e-8 * (1 + abs(ref.fun))
