"""Pins of the oracle's Gaussian sketch (the paper's experimental choice, Section 7) against what
the definition and the mathematics fix: single entries recomputed from SplitMix64 and
Box-Muller with Python integers and the math module, the normal distribution (moments and a
Kolmogorov-Smirnov test), E[W W^T] = I, the Marchenko-Pastur edges of B B^T for an orthonormal A,
and the chunked sketch against the dense product."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import sketch as osk


def test_entries_from_the_definition():
    seed, k, w = 12345, 7, 37
    W = osk.gaussian_rows(3, 6, w, seed, k)
    key = osk.mix64_int(((seed ^ osk.mix64_int(k)) + osk.GAUSS_DOMAIN) % 2 ** 64)
    for (j, c) in ((3, 0), (4, 17), (5, 36)):
        e = j * w + c
        h1 = osk.mix64_int((key + (2 * e + 1) * osk.PHI) % 2 ** 64)
        h2 = osk.mix64_int((key + (2 * e + 2) * osk.PHI) % 2 ** 64)
        u1 = ((h1 >> 11) + 1) / 2.0 ** 53
        u2 = (h2 >> 11) / 2.0 ** 53
        z = math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)
        assert W[j - 3, c] == pytest.approx(z / math.sqrt(w), rel=1e-15, abs=1e-300)


def test_normal_distribution():
    z = osk.gaussian_rows(0, 1000, 2000, 3, 1).ravel() * math.sqrt(2000)   # 2e6 deviates
    N = z.size
    assert abs(z.mean()) < 5 / math.sqrt(N)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / N)
    assert abs(stats.kurtosis(z, fisher=False) - 3.0) < 5 * math.sqrt(24.0 / N)
    assert stats.kstest(z[:200000], "norm").pvalue > 1e-4


def test_expected_gram_is_identity_and_draws_differ():
    n, w = 40, 20000
    W = osk.gaussian_rows(0, n, w, 9, 2)
    G = W @ W.T
    assert np.max(np.abs(np.diag(G) - 1.0)) < 6 * math.sqrt(2.0 / w)
    assert np.max(np.abs(G - np.diag(np.diag(G)))) < 6 / math.sqrt(w)
    assert not np.allclose(W, osk.gaussian_rows(0, n, w, 9, 3))
    assert np.array_equal(W, osk.gaussian_rows(0, n, w, 9, 2))


def test_marchenko_pastur_edges():
    # A with orthonormal rows: B B^T = (A W)(A W)^T has the spectrum of a Wishart matrix with
    # aspect ratio m / w, whose edges are (1 -+ sqrt(m / w))^2
    m, n, w = 60, 3000, 1200
    Q, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((n, m)))
    B = osk.sketch_gaussian(Q.T, np.ones(n), w, 5, 0, chunk=700)
    ev = np.linalg.eigvalsh(B @ B.T)
    r = math.sqrt(m / w)
    assert (1 - r) ** 2 * 0.85 < ev.min() < (1 - r) ** 2 * 1.2
    assert (1 + r) ** 2 * 0.85 < ev.max() < (1 + r) ** 2 * 1.15


def test_chunked_sketch_and_apply_match_dense():
    rng = np.random.default_rng(1)
    m, n, w = 7, 1001, 50
    A = rng.standard_normal((m, n))
    d = np.exp(rng.uniform(-2, 2, n))
    W = osk.gaussian_rows(0, n, w, 4, 6)
    assert np.allclose(osk.sketch_gaussian(A, d, w, 4, 6, chunk=97), (A * d) @ W, rtol=1e-13, atol=1e-13)
    u = rng.standard_normal(w)
    assert np.allclose(osk.gaussian_apply(u, n, w, 4, 6, chunk=89), W @ u, rtol=1e-13, atol=1e-13)


def test_gaussian_sketch_ipm_reaches_the_optimum():
    import lpgen
    from scipy.optimize import linprog
    from oracle import ipm as oipm
    lp = lpgen.dense_lp(20, 500, seed=7)
    res = oipm.solve(lp.A, lp.b, lp.c, oipm.Params(w=80, s=2, seed=1, sketch=1), "sketch")
    ref = linprog(lp.c, A_eq=lp.A, b_eq=lp.b, bounds=(0, None), method="highs")
    assert res.converged
    assert abs(float(lp.c @ res.state.x) - ref.fun) <= 1e-8 * (1 + abs(ref.fun))
