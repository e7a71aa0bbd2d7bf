"""Pins of the oracle against what the paper and the mathematics fix (CPU only).

Each test names the passage or the fact it pins. None of them retypes the
oracle's own formula: they use brute force, closed forms, identities the
paper proves, library routines on special cases, or published reference
values.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.optimize import linprog

import lpgen
from oracle import ipm, sketch, vertex


def interior_point(lp, seed=7, scale=1.0):
    """A random strictly positive, infeasible point (x, y, s)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.2, 2.0, lp.n) * scale
    s = rng.uniform(0.2, 2.0, lp.n) * scale
    y = rng.standard_normal(lp.m)
    return x, y, s


def state_at(lp, x, y, s, k=0):
    st0 = ipm.initial_state(lp.A, lp.b, lp.c)
    return ipm.State(x.copy(), y.copy(), s.copy(), k, st0.mu0, st0.r0norm)


# ------------------------------------------------------------------ sketch (Section 2)

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden_rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [line.split() for line in f if line.strip() and not line.startswith("#")]


def test_splitmix64_reference_outputs():
    """SplitMix64 (Steele, Lea, Flood 2014) published reference outputs (tests/golden)."""
    rows = _golden_rows("splitmix64_reference.txt")
    assert len(rows) == 2
    for seed, *outs in rows:
        assert sketch.splitmix64_stream(int(seed), len(outs)) == [int(o) for o in outs]


@pytest.mark.parametrize("n,w,s", [(1000, 40, 1), (1000, 40, 2), (997, 36, 4)])
def test_sketch_structure(n, w, s):
    """Each row of W: s nonzeros, one per bucket block, +-1/sqrt(s), unit norm (Section 2)."""
    W = sketch.sketch_matrix(n, w, s, seed=3, k=5).toarray()
    nz = W != 0
    assert np.all(nz.sum(axis=1) == s)
    blk = w // s
    for r in range(s):
        assert np.all(nz[:, r * blk:(r + 1) * blk].sum(axis=1) == 1)
    assert np.allclose(np.abs(W[nz]), 1 / np.sqrt(s))
    assert np.allclose((W * W).sum(axis=1), 1.0)
    # buckets and signs are spread out: every bucket used, both signs used
    assert np.all(nz.sum(axis=0) > 0)
    assert 0.4 < (W[nz] > 0).mean() < 0.6


def test_sketch_redrawn_per_iteration():
    """Algorithm 3, step 2 draws a fresh W every iteration."""
    b0, _ = sketch.buckets_signs(500, 64, 2, seed=1, k=0)
    b1, _ = sketch.buckets_signs(500, 64, 2, seed=1, k=1)
    assert (b0 != b1).mean() > 0.9


def test_sketch_ADW_brute_force():
    """B = A D W by an explicit triple loop over rows, columns and copies."""
    rng = np.random.default_rng(0)
    m, n, w, s = 3, 40, 12, 3
    A = rng.standard_normal((m, n))
    d = rng.uniform(0.1, 3.0, n)
    B = sketch.sketch_ADW(A, d, w, s, seed=11, k=4)
    bucket, sign = sketch.buckets_signs(n, w, s, seed=11, k=4)
    Bb = np.zeros((m, w))
    for i in range(m):
        for j in range(n):
            for r in range(s):
                Bb[i, bucket[j, r]] += A[i, j] * d[j] * sign[j, r] / np.sqrt(s)
    assert np.allclose(B, Bb, rtol=1e-14, atol=1e-14)


def test_sketch_WWt_mean_is_identity():
    """E[W W^T] = I for the +-1/sqrt(s) embedding (diagonal exact, off-diagonal -> 0)."""
    n, w, s = 60, 16, 2
    acc = np.zeros((n, n))
    T = 400
    for seed in range(T):
        W = sketch.sketch_matrix(n, w, s, seed=seed, k=0).toarray()
        acc += W @ W.T
    acc /= T
    assert np.allclose(np.diag(acc), 1.0)
    off = acc - np.diag(np.diag(acc))
    assert np.abs(off).max() < 0.12   # ~ 4 standard errors of 1/sqrt(w*T) spread


# ------------------------------------------------------------------ right-hand side (Section 5)

def test_p_matches_paper_form():
    """p = -r_p - sigma mu A S^-1 1 + A x - A D^2 r_d (Section 5) equals b - A(sigma mu/s + d^2 r_d)."""
    lp = lpgen.tiny_lp(6, 40, 2)
    x, y, s = interior_point(lp)
    rp, rd = ipm.residuals(lp.A, lp.b, lp.c, x, y, s)
    mu = x @ s / lp.n
    p1 = ipm.rhs_p(lp.A, lp.b, x, s, rd, 0.5, mu)
    p2 = ipm.rhs_p_paper_form(lp.A, lp.b, x, s, rd, 0.5, mu)
    assert np.allclose(p1, p2, rtol=1e-12, atol=1e-12 * np.abs(p1).max())


def test_first_direction_closed_form():
    """At x = s = 1, y = 0: D = I, mu = 1, M = A A^T, p = b - A(sigma + 1 - c)."""
    lp = lpgen.tiny_lp(5, 30, 3)
    st = ipm.initial_state(lp.A, lp.b, lp.c)
    prm = ipm.Params()
    _, info = ipm.step(lp.A, lp.b, lp.c, st, prm, mode="exact", keep=True)
    p = lp.b - lp.A @ (prm.sigma + 1.0 - lp.c)
    dy = np.linalg.solve(lp.A @ lp.A.T, p)
    assert np.allclose(info.extra["p"], p, rtol=1e-13, atol=1e-12)
    assert np.allclose(info.extra["dy"], dy, rtol=1e-10, atol=1e-11)
    ds = -(1.0 - lp.c) - lp.A.T @ dy
    assert np.allclose(info.extra["ds"], ds, rtol=1e-10, atol=1e-10)


# ------------------------------------------------------------------ Newton system identities

@pytest.mark.parametrize("mode,maxit,kind", [("exact", 500, 0), ("sketch", 500, 0), ("sketch", 1, 0), ("sketch", 3, 0),
                                             ("sketch", 1, 1), ("sketch", 500, 1)])
def test_newton_system_identities(mode, maxit, kind):
    """A dx = -r_p, A^T dy + ds = -r_d, X ds + S dx = -XS1 + sigma mu 1 - v (eq. iip_3).

    Holds for any dy once v satisfies A S^-1 v = A D^2 A^T dy - p, so also for a
    1-iteration PCG (Section 4, eq. addl; Lemma fullrankR).
    """
    lp = lpgen.tiny_lp(8, 120, 4)
    x, y, s = interior_point(lp, seed=5)
    st = state_at(lp, x, y, s)
    prm = ipm.Params(w=32, s=2, seed=9, maxit_pcg=maxit, sketch=kind)
    _, info = ipm.step(lp.A, lp.b, lp.c, st, prm, mode=mode, keep=True)
    e = info.extra
    A = lp.A
    mu = x @ s / lp.n
    sc = np.abs(e["p"]).max() + np.abs(A).max() * (np.abs(e["dx"]).max() + 1)
    assert np.allclose(A @ e["dx"], -e["rp"], atol=1e-11 * sc)
    assert np.allclose(A.T @ e["dy"] + e["ds"], -e["rd"], atol=1e-12 * sc)
    rhs = -x * s + prm.sigma * mu - e["v"]
    assert np.allclose(x * e["ds"] + s * e["dx"], rhs, atol=1e-11 * (1 + np.abs(rhs).max()))


@pytest.mark.parametrize("kind", [0, 1])
def test_v_invariant_and_norm_bound(kind):
    """A S^-1 v = M dy - p exactly (Lemma fullrankR) and ||v|| <= sqrt(3 n mu) ||f|| (Lemma v),
    for the sparse embedding (kind 0) and the Gaussian sketch (kind 1)."""
    lp = lpgen.tiny_lp(10, 400, 5)
    x, y, s = interior_point(lp, seed=8)
    st = state_at(lp, x, y, s)
    # large sketch so the embedding condition holds (w.h.p.)
    prm = ipm.Params(w=800, s=8, seed=2, maxit_pcg=2, sketch=kind)
    _, info = ipm.step(lp.A, lp.b, lp.c, st, prm, mode="sketch", keep=True)
    e = info.extra
    A = lp.A
    rhat = A @ (e["d2"] * (A.T @ e["dy"])) - e["p"]
    lhs = A @ (e["v"] / s)
    assert np.linalg.norm(lhs - rhat) <= 1e-12 * np.linalg.norm(e["p"])
    f = sla.solve_triangular(e["L"], rhat, lower=True)   # Q^{-1/2}-norm of the residual
    mu = x @ s / lp.n
    assert np.linalg.norm(e["v"]) <= np.sqrt(3 * lp.n * mu) * np.linalg.norm(f)


def test_residual_contraction_is_exact():
    """r_p and r_d shrink by exactly (1 - alpha) even with an inexact dy (Sections 4-5)."""
    lp = lpgen.tiny_lp(8, 200, 6)
    st = ipm.initial_state(lp.A, lp.b, lp.c)
    prm = ipm.Params(w=32, s=2, seed=1, maxit_pcg=1)
    new, info = ipm.step(lp.A, lp.b, lp.c, st, prm, mode="sketch", keep=True)
    a = info.alpha
    assert 0 < a <= 1
    rp1, rd1 = ipm.residuals(lp.A, lp.b, lp.c, new.x, new.y, new.s)
    rp0, rd0 = info.extra["rp"], info.extra["rd"]
    assert np.allclose(rp1, (1 - a) * rp0, atol=1e-11 * np.abs(rp0).max())
    assert np.allclose(rd1, (1 - a) * rd0, atol=1e-12 * np.abs(rd0).max())
    # without the correction the primal residual drifts by alpha (M dy - p)
    prm2 = ipm.Params(w=32, s=2, seed=1, maxit_pcg=1, vcorr=False)
    new2, info2 = ipm.step(lp.A, lp.b, lp.c, st, prm2, mode="sketch", keep=True)
    rp2, _ = ipm.residuals(lp.A, lp.b, lp.c, new2.x, new2.y, new2.s)
    assert np.linalg.norm(rp2 - (1 - info2.alpha) * rp0) > 1e-6 * np.linalg.norm(rp0)


# ------------------------------------------------------------------ PCG (Algorithm 1, Section 3)

def _normal(lp, d2):
    return (lp.A * d2) @ lp.A.T


def test_pcg_with_exact_preconditioner_takes_one_iteration():
    """Q = A D^2 A^T makes the preconditioned matrix the identity: CG stops after 1 step."""
    lp = lpgen.tiny_lp(12, 300, 7)
    rng = np.random.default_rng(1)
    d2 = rng.uniform(0.01, 100.0, lp.n)
    M = _normal(lp, d2)
    L = np.linalg.cholesky(M)
    p = rng.standard_normal(lp.m)
    res = ipm.pcg(lambda v: M @ v, L, p, tol=1e-10, maxit=50)
    assert res.iters == 1 and res.status == ipm.OK
    assert np.allclose(res.dy, np.linalg.solve(M, p), rtol=1e-9)


def _sketched(lp, d2, w, s, seed):
    B = sketch.sketch_ADW(lp.A, np.sqrt(d2), w, s, seed, 0)
    Q = B @ B.T
    L = np.linalg.cholesky(Q)
    M = _normal(lp, d2)
    Li = np.linalg.inv(L)
    ev = np.linalg.eigvalsh(Li @ M @ Li.T)
    return M, L, ev


def test_spectral_condition_lemma_cond3():
    """Eigenvalues of Q^{-1/2} A D^2 A^T Q^{-1/2} lie in [2/(2+zeta), 2/(2-zeta)], zeta = 1/2
    (eq. pdcond1, Lemma cond3), for a wide sparse embedding (w = 100 m, s = 8)."""
    lp = lpgen.tiny_lp(20, 2000, 8)
    rng = np.random.default_rng(2)
    d2 = np.exp(rng.uniform(-4, 4, lp.n))
    zeta = 0.5
    for seed in range(3):
        _, _, ev = _sketched(lp, d2, 2000, 8, seed)
        assert ev.min() >= 2 / (2 + zeta) and ev.max() <= 2 / (2 - zeta)


def test_cg_residual_monotone_lemma_prev1():
    """||f_j|| <= (kappa^2 - 1)/2 ||f_{j-1}|| (Lemma prev1) with kappa^2 of Q^{-1/2} A D."""
    lp = lpgen.tiny_lp(20, 2000, 9)
    rng = np.random.default_rng(3)
    d2 = np.exp(rng.uniform(-3, 3, lp.n))
    M, L, ev = _sketched(lp, d2, 2000, 8, 1)
    kappa2 = ev.max() / ev.min()
    assert kappa2 < 3
    p = rng.standard_normal(lp.m)
    res = ipm.pcg(lambda v: M @ v, L, p, tol=1e-12, maxit=100)
    h = np.array(res.history)
    assert np.all(h[1:] <= (kappa2 - 1) / 2 * h[:-1] * (1 + 1e-9))
    # and the reported residual is the paper's ||Q^{-1/2}(M dy - p)||
    f = sla.solve_triangular(L, M @ res.dy - p, lower=True)
    assert np.linalg.norm(f) <= 1e-12 * np.linalg.norm(sla.solve_triangular(L, p, lower=True)) * 10


def test_pcg_energy_error_matches_tolerance():
    """PCG stops with ||f|| <= tol ||Q^{-1/2} p|| and an M-norm error consistent with it."""
    lp = lpgen.tiny_lp(30, 1500, 10)
    rng = np.random.default_rng(4)
    d2 = np.exp(rng.uniform(-5, 5, lp.n))
    M, L, ev = _sketched(lp, d2, 120, 2, 3)
    p = rng.standard_normal(lp.m)
    tol = 1e-10
    res = ipm.pcg(lambda v: M @ v, L, p, tol=tol, maxit=500)
    assert res.status == ipm.OK
    f = sla.solve_triangular(L, M @ res.dy - p, lower=True)
    fp = sla.solve_triangular(L, p, lower=True)
    assert np.linalg.norm(f) <= 10 * tol * np.linalg.norm(fp)
    x = np.linalg.solve(M, p)
    e = res.dy - x
    # ||e||_M = ||Q^{-1/2} M^{1/2}... ||: bounded via the preconditioned spectrum
    en = np.sqrt(e @ M @ e)
    assert en <= 10 * tol * np.linalg.norm(fp) / np.sqrt(ev.min())


def test_pcg_warm_start_multiple_of_solution_needs_no_iteration():
    """Any nonzero multiple of the exact solution, negative ones included, is scaled back to
    the solution by the energy-optimal factor: CG stops before its first iteration."""
    lp = lpgen.tiny_lp(15, 400, 11)
    rng = np.random.default_rng(5)
    d2 = np.exp(rng.uniform(-3, 3, lp.n))
    M, L, _ = _sketched(lp, d2, 60, 2, 1)
    p = rng.standard_normal(lp.m)
    xs = np.linalg.solve(M, p)
    for c in (-3.0, 1e-3, 7.5):
        res = ipm.pcg(lambda v: M @ v, L, p, tol=1e-10, maxit=100, dy0=c * xs)
        assert res.warm_used and res.iters == 0
        assert np.allclose(res.dy, xs, rtol=1e-9)
    # a direction M-orthogonal to the solution carries no information: beta = 0, zero start
    z = rng.standard_normal(lp.m)
    z -= (z @ M @ xs) / (xs @ M @ xs) * xs
    res = ipm.pcg(lambda v: M @ v, L, p, tol=1e-10, maxit=100, dy0=z)
    cold = ipm.pcg(lambda v: M @ v, L, p, tol=1e-10, maxit=100)
    assert not res.warm_used and res.iters == cold.iters


def test_pcg_warm_start_never_increases_the_energy_error():
    """The scaled warm start is the best multiple of dy0 in the M-norm, so its error is at most
    that of dy0 itself and of the zero start (minimisation over a line through 0)."""
    lp = lpgen.tiny_lp(15, 400, 12)
    rng = np.random.default_rng(6)
    d2 = np.exp(rng.uniform(-3, 3, lp.n))
    M, L, _ = _sketched(lp, d2, 60, 2, 2)
    p = rng.standard_normal(lp.m)
    xs = np.linalg.solve(M, p)
    enorm = lambda e: np.sqrt(e @ M @ e)
    for t in range(20):
        dy0 = xs * rng.uniform(0.0, 3.0) + rng.standard_normal(lp.m) * rng.uniform(0, 2) * np.linalg.norm(xs)
        res = ipm.pcg(lambda v: M @ v, L, p, tol=1e-10, maxit=0, dy0=dy0)
        e = enorm(res.dy - xs)
        assert e <= enorm(dy0 - xs) * (1 + 1e-12) and e <= enorm(xs) * (1 + 1e-12)
        # brute force over a grid of multiples
        grid = np.linspace(-3, 3, 601)
        best = min(enorm(g * dy0 - xs) for g in grid)
        if res.warm_used:
            assert e <= best * (1 + 1e-9)


def test_pcg_two_candidates_span_the_solution():
    """Two candidates whose span holds the solution give it exactly: no CG iteration."""
    lp = lpgen.tiny_lp(15, 400, 13)
    rng = np.random.default_rng(7)
    d2 = np.exp(rng.uniform(-3, 3, lp.n))
    M, L, _ = _sketched(lp, d2, 60, 2, 3)
    p = rng.standard_normal(lp.m)
    xs = np.linalg.solve(M, p)
    v1 = rng.standard_normal(lp.m)
    v2 = 2.5 * xs - 0.7 * v1
    res = ipm.pcg(lambda v: M @ v, L, p, tol=1e-10, maxit=100, dy0=np.stack([v1, v2], axis=1))
    assert res.warm_used and res.iters == 0
    assert np.allclose(res.dy, xs, rtol=1e-8)


def test_pcg_two_candidates_beat_each_alone():
    """The two-candidate start is the M-norm best point of the plane (brute force over a grid)
    and so no worse than either candidate's best multiple."""
    lp = lpgen.tiny_lp(15, 400, 14)
    rng = np.random.default_rng(8)
    d2 = np.exp(rng.uniform(-3, 3, lp.n))
    M, L, _ = _sketched(lp, d2, 60, 2, 4)
    p = rng.standard_normal(lp.m)
    xs = np.linalg.solve(M, p)
    enorm = lambda e: np.sqrt(e @ M @ e)
    for t in range(10):
        v1 = xs + rng.standard_normal(lp.m) * np.linalg.norm(xs) * rng.uniform(0.1, 2)
        v2 = xs * rng.uniform(-1, 1) + rng.standard_normal(lp.m) * np.linalg.norm(xs)
        two = ipm.pcg(lambda v: M @ v, L, p, tol=1e-10, maxit=0, dy0=np.stack([v1, v2], axis=1))
        e2 = enorm(two.dy - xs)
        for v in (v1, v2):
            one = ipm.pcg(lambda u: M @ u, L, p, tol=1e-10, maxit=0, dy0=v)
            assert e2 <= enorm(one.dy - xs) * (1 + 1e-10)
        grid = np.linspace(-3, 3, 121)
        best = min(enorm(a * v1 + b * v2 - xs) for a in grid for b in grid)
        assert e2 <= best * (1 + 1e-10)
    # parallel candidates fall back to the first one's best multiple
    v1 = rng.standard_normal(lp.m)
    par = ipm.pcg(lambda v: M @ v, L, p, tol=1e-10, maxit=0, dy0=np.stack([v1, -2 * v1], axis=1))
    one = ipm.pcg(lambda v: M @ v, L, p, tol=1e-10, maxit=0, dy0=v1)
    assert par.warm_used == one.warm_used and np.allclose(par.dy, one.dy, rtol=1e-12)


def test_shifted_cholesky_special_cases():
    """SPD Q: the plain factor (library routine). Q = B B^T with B of numerical rank < m: the
    factor of Q + delta I with delta = u trace(Q) 100^j. A Q with a large negative eigenvalue:
    none."""
    rng = np.random.default_rng(9)
    B = rng.standard_normal((20, 60))
    Q = B @ B.T
    L, d = ipm.shifted_cholesky(Q, 2)
    assert d == 0.0 and np.allclose(L, np.linalg.cholesky(Q), rtol=1e-13, atol=1e-13)
    U, _ = np.linalg.qr(rng.standard_normal((20, 20)))
    sv = np.logspace(0, -12, 20)
    B = (U * sv) @ rng.standard_normal((20, 60)) / np.sqrt(60)
    B[5] = B[4]                                   # an exactly repeated row: Q is singular
    Q = B @ B.T
    L, d = ipm.shifted_cholesky(Q, 2)
    assert L is not None and d > 0.0
    assert d in (np.finfo(float).eps / 2 * np.trace(Q) * f for f in (1.0, 100.0))
    assert np.linalg.norm(L @ L.T - (Q + d * np.eye(20))) <= 1e-14 * np.linalg.norm(Q)
    Qn = Q - 1e-3 * np.trace(Q) * np.outer(U[:, 0], U[:, 0])
    L, d = ipm.shifted_cholesky(Qn, 2)
    assert L is None


def test_sparse_matrix_branches_match_dense():
    """The sparse (CSR) branches of the oracle give what the dense ones give on the densified
    matrix: normal matrix, sketch, and whole IPM steps."""
    lp = lpgen.sparse_lp(30, 900, 0.05, seed=4)
    Ad = lp.A.toarray()
    rng = np.random.default_rng(3)
    d2 = np.exp(rng.uniform(-3, 3, lp.n))
    assert np.allclose(ipm.normal_matrix(lp.A, d2), ipm.normal_matrix(Ad, d2), rtol=1e-13, atol=1e-12)
    assert np.allclose(sketch.sketch_ADW(lp.A, np.sqrt(d2), 120, 2, 5, 1),
                       sketch.sketch_ADW(Ad, np.sqrt(d2), 120, 2, 5, 1), rtol=1e-13, atol=1e-13)
    prm = ipm.Params(w=120, s=2, seed=2)
    st_s = ipm.initial_state(lp.A, lp.b, lp.c)
    st_d = ipm.initial_state(Ad, lp.b, lp.c)
    for _ in range(5):     # direct-solver steps: identical up to summation order
        st_s, _ = ipm.step(lp.A, lp.b, lp.c, st_s, prm, "exact")
        st_d, _ = ipm.step(Ad, lp.b, lp.c, st_d, prm, "exact")
        assert np.allclose(st_s.x, st_d.x, rtol=1e-11)
    # one sketch step from the same point: CG counts may differ by one through rounding
    new_s, inf_s = ipm.step(lp.A, lp.b, lp.c, st_s, prm, "sketch")
    new_d, inf_d = ipm.step(Ad, lp.b, lp.c, st_s, prm, "sketch")
    assert abs(inf_s.pcg_iters - inf_d.pcg_iters) <= 1
    assert np.allclose(new_s.x, new_d.x, rtol=1e-7)


def test_sparse_lp_optimum_matches_highs():
    """Sparse LP like the 1000 x 10^6 workload (uniform pattern, no empty column): the
    direct-solver IPM's optimum equals HiGHS's."""
    lp = lpgen.sparse_lp(40, 3000, 0.02, seed=6)
    assert np.all(lp.A.getnnz(axis=0) > 0)
    res = ipm.solve(lp.A, lp.b, lp.c, ipm.Params(), "exact")
    assert res.converged
    ref = linprog(lp.c, A_eq=lp.A, b_eq=lp.b, bounds=(0, None), method="highs")
    obj = float(lp.c @ res.state.x)
    assert abs(obj - ref.fun) <= 1e-8 * (1 + abs(ref.fun))


# ------------------------------------------------------------------ step lengths (Algorithm 3, steps 6-7)

def _constraints(x, s, dx, ds, gamma, mu0, r0n, rn, a):
    xa, sa = x + a * dx, s + a * ds
    mua = xa @ sa / x.size
    ok = np.all(xa > 0) and np.all(sa > 0) and np.all(xa * sa >= (1 - gamma) * mua - 1e-15)
    ok = ok and ((1 - a) * rn / r0n <= mua / mu0 + 1e-15)
    return ok, mua


def test_step_lengths_brute_force():
    """alpha_max is where the segment leaves N(gamma); alpha_bar minimises mu on [0, alpha_max]."""
    lp = lpgen.tiny_lp(6, 80, 11)
    st = ipm.initial_state(lp.A, lp.b, lp.c)
    prm = ipm.Params(w=24, s=2, seed=4)
    checked = 0
    for _ in range(12):
        new, info = ipm.step(lp.A, lp.b, lp.c, st, prm, mode="sketch", keep=True)
        e = info.extra
        rn = np.sqrt(e["rp"] @ e["rp"] + e["rd"] @ e["rd"])
        grid = np.linspace(0, info.alpha_max, 2001)
        vals = [_constraints(st.x, st.s, e["dx"], e["ds"], prm.gamma, st.mu0, st.r0norm, rn, a)
                for a in grid]
        assert all(v[0] for v in vals), "a point inside [0, alpha_max] leaves N(gamma)"
        mus = np.array([v[1] for v in vals])
        mu_bar = (st.x + info.alpha * e["dx"]) @ (st.s + info.alpha * e["ds"]) / lp.n
        assert mu_bar <= mus.min() * (1 + 1e-12) + 1e-300
        if info.alpha_max < 1:
            unbacked = info.alpha_max / prm.theta
            beyond = np.linspace(unbacked, min(1.0, unbacked * 1.002 + 1e-9), 50)[1:]
            assert not all(_constraints(st.x, st.s, e["dx"], e["ds"], prm.gamma, st.mu0,
                                        st.r0norm, rn, a)[0] for a in beyond)
            checked += 1
        st = new
    assert checked >= 1


def test_first_exit_roots():
    """Closed-form first exit of c + b a + a2 a^2 checked against dense sampling."""
    rng = np.random.default_rng(5)
    for _ in range(500):
        c0, b0, a0 = rng.uniform(0, 2), rng.normal(), rng.normal()
        r = float(ipm.first_exit(c0, b0, a0))
        grid = np.linspace(0, 5, 200001)
        vals = c0 + b0 * grid + a0 * grid * grid
        neg = np.nonzero(vals < -1e-12)[0]
        expect = grid[neg[0]] if neg.size else np.inf
        if np.isinf(expect):
            assert r >= 5 - 1e-4
        else:
            assert abs(r - expect) <= 5e-5 * max(1, expect)


def test_xs_identity_lemma_maxalpha0():
    """x(a) o s(a) = (1-a) x o s + a sigma mu 1 - a v + a^2 dx o ds (Lemma maxalpha0)."""
    lp = lpgen.tiny_lp(8, 150, 12)
    x, y, s = interior_point(lp, seed=3)
    st = state_at(lp, x, y, s)
    prm = ipm.Params(w=40, s=2, seed=5, maxit_pcg=2)
    _, info = ipm.step(lp.A, lp.b, lp.c, st, prm, mode="sketch", keep=True)
    e = info.extra
    mu = x @ s / lp.n
    for a in (0.1, 0.5, 0.9):
        lhs = (x + a * e["dx"]) * (s + a * e["ds"])
        rhs = (1 - a) * x * s + a * prm.sigma * mu - a * e["v"] + a * a * e["dx"] * e["ds"]
        assert np.allclose(lhs, rhs, rtol=1e-11, atol=1e-11)


# ------------------------------------------------------------------ LP optimum

@pytest.mark.parametrize("m,n,seed", [(2, 6, 0), (3, 8, 1), (3, 9, 2), (4, 10, 3), (4, 11, 4)])
@pytest.mark.parametrize("mode", ["exact", "sketch"])
def test_optimum_vs_vertex_enumeration(m, n, seed, mode):
    """Brute-force optimum over all basic feasible solutions (fundamental theorem of LP)."""
    lp = lpgen.tiny_lp(m, n, seed)
    opt, xs = vertex.lp_optimum(lp.A, lp.b, lp.c)
    prm = ipm.Params(w=4 * m, s=2, seed=seed)
    res = ipm.solve(lp.A, lp.b, lp.c, prm, mode)
    assert res.converged
    obj = float(lp.c @ res.state.x)
    assert abs(obj - opt) <= 1e-7 * (1 + abs(opt))
    if len(xs) == 1:
        assert np.allclose(res.state.x, xs[0], atol=1e-6 * (1 + np.abs(xs[0]).max()))


def test_optimum_closed_form_single_constraint():
    """m = 1, a > 0, b > 0: optimum b * min_j c_j / a_j."""
    rng = np.random.default_rng(6)
    n = 50
    a = rng.uniform(0.5, 2.0, n)
    c = rng.uniform(0.1, 3.0, n)
    A = a[None, :]
    b = np.array([3.0])
    for mode in ("exact", "sketch"):
        res = ipm.solve(A, b, c, ipm.Params(w=4, s=2, seed=1), mode)
        assert res.converged
        opt = b[0] * np.min(c / a)
        assert abs(c @ res.state.x - opt) <= 1e-7 * (1 + opt)


def test_optimum_closed_form_square():
    """n = m: the only feasible point is A^{-1} b (here the generator's x0 > 0)."""
    lp = lpgen.tiny_lp(6, 6, 13)
    for mode in ("exact", "sketch"):
        res = ipm.solve(lp.A, lp.b, lp.c, ipm.Params(w=24, s=2, seed=2), mode)
        assert res.converged
        assert np.allclose(res.state.x, np.linalg.solve(lp.A, lp.b), rtol=1e-6, atol=1e-6)


def test_dense_50x2000_matches_highs_and_duality_sandwich():
    """Objective of the 50 x 2000 workload vs scipy's HiGHS; b^T y0 <= opt <= c^T x0."""
    lp = lpgen.workload("dense_50x2000")
    ref = linprog(lp.c, A_eq=lp.A, b_eq=lp.b, bounds=(0, None), method="highs")
    assert ref.status == 0
    opt = ref.fun
    assert lp.b @ lp.y0 <= opt <= lp.c @ lp.x0
    for mode in ("exact", "sketch"):
        res = ipm.solve(lp.A, lp.b, lp.c, ipm.Params(w=200, s=1, seed=0), mode)
        assert res.converged
        st = res.state
        assert abs(lp.c @ st.x - opt) <= 1e-8 * (1 + abs(opt))
        # KKT at exit: positivity and small complementarity
        assert np.all(st.x > 0) and np.all(st.s > 0)
        assert (st.x @ st.s) / lp.n <= 1e-8 * (1 + abs(opt))


def test_iterates_stay_in_neighbourhood_and_counts_match():
    """Every iterate lies in N(gamma) (Section 5); sketch and direct IPM take equal
    outer-iteration counts (the qualitative claim of Table 1)."""
    lp = lpgen.tiny_lp(15, 600, 14)
    prm = ipm.Params(w=60, s=2, seed=3)
    seen = []

    def cb(st, info):
        seen.append(ipm.State(st.x.copy(), st.y.copy(), st.s.copy(), st.k, st.mu0, st.r0norm))

    res_s = ipm.solve(lp.A, lp.b, lp.c, prm, "sketch", callback=cb)
    res_e = ipm.solve(lp.A, lp.b, lp.c, prm, "exact")
    assert res_s.converged and res_e.converged
    assert abs(len(res_s.infos) - len(res_e.infos)) <= 1
    for st in seen:
        mu = st.x @ st.s / lp.n
        assert np.all(st.x * st.s >= (1 - prm.gamma) * mu * (1 - 1e-9))
        rp, rd = ipm.residuals(lp.A, lp.b, lp.c, st.x, st.y, st.s)
        rn = np.sqrt(rp @ rp + rd @ rd)
        assert rn / st.r0norm <= mu / st.mu0 * (1 + 1e-7) + 1e-14


# ------------------------------------------------------------------ planted mistakes are caught

def test_planted_sign_error_in_p_is_caught(monkeypatch):
    """A sign slip in the d^2 r_d term of p breaks the closed-form first direction."""
    def bad(A, b, x, s, rd, sigma, mu):
        return b - A @ (sigma * mu / s - (x / s) * rd)
    monkeypatch.setattr(ipm, "rhs_p", bad)
    lp = lpgen.tiny_lp(5, 30, 3)
    st = ipm.initial_state(lp.A, lp.b, lp.c)
    _, info = ipm.step(lp.A, lp.b, lp.c, st, ipm.Params(), mode="exact", keep=True)
    p = lp.b - lp.A @ (0.5 + 1.0 - lp.c)
    assert not np.allclose(info.extra["p"], p, rtol=1e-6)


def test_planted_transposed_sketch_is_caught():
    """Using W's buckets with the wrong copy index breaks the brute-force sketch pin."""
    rng = np.random.default_rng(0)
    A = rng.standard_normal((3, 40))
    d = rng.uniform(0.1, 3.0, 40)
    bucket, sign = sketch.buckets_signs(40, 12, 3, seed=11, k=4)
    Bb = np.zeros((3, 12))
    for j in range(40):
        for r in range(3):
            Bb[:, bucket[j, (r + 1) % 3]] += A[:, j] * d[j] * sign[j, r] / np.sqrt(3)
    assert not np.allclose(sketch.sketch_ADW(A, d, 12, 3, 11, 4), Bb)


def _near_dependent_lp(near: bool):
    """6 x 600 LP from the generic rule; with ``near`` its second row is the first plus 1e-10 noise,
    so kappa(A D) ~ 1e10 and every draw's Q = B B^T is beyond 1/u."""
    rng = np.random.default_rng(5)
    m, n = 6, 600
    A = rng.standard_normal((m, n))
    if near:
        A[1] = A[0] + 1e-10 * rng.standard_normal(n)
    x0 = rng.uniform(0.5, 1.5, n)
    y0, s0 = rng.standard_normal(m), rng.uniform(0.5, 1.5, n)
    return A, A @ x0, A.T @ y0 + s0


@pytest.mark.parametrize("near", [True, False])
def test_redraw_rule_keeps_shifted_redraw(near):
    """Redraws (reading of the failed-solve case): CG capped at 2 iterations fails on every draw.
    When Q factors only with a shift on every draw (kappa(AD) itself beyond sqrt(1/u)), the first
    redraw is kept (2 attempts, shift > 0); with a well-conditioned A all max_redraws + 1 draws are
    tried (4 attempts, no shift)."""
    A, b, c = _near_dependent_lp(near)
    st = ipm.initial_state(A, b, c)
    st, _ = ipm.step(A, b, c, st, ipm.Params(w=24, s=2, seed=1), "sketch")
    _, info = ipm.step(A, b, c, st, ipm.Params(w=24, s=2, seed=1, maxit_pcg=2), "sketch")
    assert info.pcg_status == ipm.PCG_MAXIT
    if near:
        assert info.extra["attempts"] == 2 and info.extra["w_used"] == 48 and info.extra["shift"] > 0
    else:
        assert info.extra["attempts"] == 4 and info.extra["w_used"] == 192 and info.extra["shift"] == 0
