"""Parity of the sparse (CSR) path with the FP64 oracle on seeded sparse LPs (uniform random
pattern, N(0, 1) values; the method's cost is stated in nnz(A), Sections 3 and 4).

The matvec and the sketch are compared element by element against the oracle's routines with
FP64 summation bounds; the IPM step in lockstep with the oracle's step on the same scipy matrix;
solves against the oracle's optimum. The full-size cases are the 1000 x 10^6 matrix with density
10^-3 and the 5000 x 2*10^6 matrix with density 5*10^-4 (BF16 values), solved in the plain form
(FP64 copy of the same values) and the mixed form.
"""
import numpy as np
import pytest
import scipy.sparse as sp

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


_TDT = {"f64": "float64", "f32": "float32", "bf16": "bfloat16"}


def _round(vals, storage):
    if storage == "bf16":
        return lpgen.bf16_round(vals)
    if storage == "f32":
        return lpgen.f32_round(vals)
    return vals


def _random_csr(m, n, density, seed, storage, empty_rows=(), empty_cols=()):
    """Uniform pattern with chosen rows / columns emptied (edge cases of the row and column
    passes), values N(0, 1) rounded to the storage type."""
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=density, random_state=rng, data_rvs=rng.standard_normal, format="lil")
    for i in empty_rows:
        A[i, :] = 0
    for j in empty_cols:
        A[:, j] = 0
    A = A.tocsr()
    A.eliminate_zeros()
    A.data = _round(A.data, storage)
    return A


def _smat(A, storage):
    return P.SparseMatrix.from_scipy(A, dtype=getattr(torch, _TDT[storage]))


# ------------------------------------------------------------------------- matvec pass

@pytest.mark.parametrize("m,n,density,storage", [(1, 300, 0.05, "f64"), (7, 33, 0.3, "f64"),
                                                 (50, 2000, 0.02, "f64"), (130, 5003, 0.01, "f32"),
                                                 (300, 20011, 0.003, "bf16"), (1000, 30001, 0.001, "bf16"),
                                                 (64, 4096, 0.5, "f64")])
def test_csr_matvec(ctx, m, n, density, storage):
    A = _random_csr(m, n, density, m + n, storage, empty_rows=(0,) if m > 4 else (),
                    empty_cols=(1, n - 1))
    rng = np.random.default_rng(3)
    d2 = np.exp(rng.uniform(-6, 6, n))
    v = rng.standard_normal(m)
    q = host(P.ipm_normal_matvec(ctx, _smat(A, storage), dev(d2), dev(v)))
    ref = oipm.normal_matrix(A, d2) @ v
    absA = abs(A)
    bound = absA @ (d2 * (absA.T @ np.abs(v)))
    assert np.all(np.abs(q - ref) <= 64 * EPS * (m + np.sqrt(n)) * bound + 1e-300)
    if m > 4:
        assert q[0] == 0.0        # an empty row of A gives an exactly zero row of A D^2 A^T


def test_csr_matvec_matches_dense_pass(ctx):
    """The sparse passes and the dense strip pass on the same values agree to rounding."""
    A = _random_csr(200, 7001, 0.05, 11, "f64")
    rng = np.random.default_rng(4)
    d2 = np.exp(rng.uniform(-3, 3, 7001))
    v = rng.standard_normal(200)
    qs = host(P.ipm_normal_matvec(ctx, _smat(A, "f64"), dev(d2), dev(v)))
    qd = host(P.ipm_normal_matvec(ctx, P.Matrix.from_numpy(A.toarray()), dev(d2), dev(v)))
    absA = abs(A)
    bound = absA @ (d2 * (absA.T @ np.abs(v)))
    assert np.all(np.abs(qs - qd) <= 128 * EPS * (200 + np.sqrt(7001)) * bound + 1e-300)


# ------------------------------------------------------------------------- sketch

@pytest.mark.parametrize("m,n,density,storage,w,s,out", [(50, 2000, 0.02, "f64", 200, 1, "f64"),
                                                         (37, 1001, 0.05, "f64", 74, 2, "f64"),
                                                         (300, 20011, 0.003, "bf16", 1200, 2, "f32"),
                                                         (20, 3000, 0.01, "f32", 60000, 2, "f64"),
                                                         (10, 5000, 0.01, "f64", 48000, 3, "f32")])
def test_csr_sketch(ctx, m, n, density, storage, w, s, out):
    A = _random_csr(m, n, density, 7 * m + n, storage, empty_rows=(m - 1,))
    rng = np.random.default_rng(5)
    d = np.exp(rng.uniform(-3, 3, n))
    odt = torch.float64 if out == "f64" else torch.float32
    B = host(P.ipm_sketch(ctx, _smat(A, storage), dev(d), 9, 4, w, s, out_dtype=odt))
    ref = osk.sketch_ADW(A, d, w, s, 9, 4)
    Wm = osk.sketch_matrix(n, w, s, 9, 4)
    bound = np.asarray((abs(Wm).T @ (abs(A) @ sp.diags(d)).T).T.todense())
    tol = 32 * EPS * np.sqrt(n) if out == "f64" else 2.0 ** -23
    assert np.all(np.abs(B - ref) <= tol * bound + 1e-300)
    assert np.all(B[m - 1] == 0.0)


# ------------------------------------------------------------------------- IPM step and solve

def _gpu_state(st):
    return P.State(dev(st.x), dev(st.y), dev(st.s), st.k, st.mu0, st.r0norm)


def _lockstep(ctx, lp, storage, oprm, gprm, steps, label=""):
    """Lock-step (tests/lockstep.py: dy in the energy norm, alpha, x and s entry by entry)."""
    prob = P.Problem(_smat(lp.A, storage), dev(lp.b), dev(lp.c))
    recs, _, conv = lockstep.run(P, ctx, lp.A, lp.b, lp.c, prob, oprm, gprm, steps, label=label)
    return recs, conv


@pytest.mark.parametrize("m,n,density,w,s,seed", [(40, 3000, 0.02, 160, 2, 0), (23, 1003, 0.05, 92, 1, 5),
                                                  (100, 20000, 0.004, 400, 2, 2)])
def test_sparse_step_lockstep(ctx, m, n, density, w, s, seed):
    lp = lpgen.sparse_lp(m, n, density, seed=seed)
    _, conv = _lockstep(ctx, lp, "f64", oipm.Params(w=w, s=s, seed=seed), P.Params(w=w, s=s, seed=seed),
                        steps=200, label=f"csr {m}x{n}")
    assert conv


@pytest.mark.parametrize("m,n,density,w,s,storage,prec", [(40, 3000, 0.02, 160, 2, "f64", "plain"),
                                                          (60, 8000, 0.01, 240, 2, "bf16", "plain"),
                                                          (60, 8000, 0.01, 240, 2, "bf16", "mixed"),
                                                          (30, 4000, 0.01, 120, 2, "f32", "f32acc")])
def test_sparse_solve_matches_oracle(ctx, m, n, density, w, s, storage, prec):
    lp = lpgen.sparse_lp(m, n, density, seed=m, storage=storage)
    precision = {"plain": P.IPM_PLAIN, "mixed": P.IPM_MIXED, "f32acc": P.IPM_MIXED_F32ACC}[prec]
    dt = "f64" if prec == "plain" else storage
    res = P.solve(ctx, P.Problem(_smat(lp.A, dt), dev(lp.b), dev(lp.c)),
                  P.Params(w=w, s=s, seed=1, precision=precision))
    ores = oipm.solve(lp.A, lp.b, lp.c, oipm.Params(), "exact")
    assert res.converged and ores.converged
    obj, oobj = float(lp.c @ host(res.state.x)), float(lp.c @ ores.state.x)
    # both objectives are upper bounds of the optimum within their own relative gap (<= 1e-8)
    assert abs(obj - oobj) <= 1e-8 * (1 + abs(oobj))
    last = res.infos[-1]
    assert max(last["relgap"], last["rp_rel"], last["rd_rel"]) <= 1e-8


def test_sparse_and_dense_layouts_take_the_same_steps(ctx):
    """The same LP stored as CSR and as a dense matrix, each step taken from the same point: the
    same draws of W, so the measured quantities agree to rounding and the new iterates to the CG
    tolerance."""
    lp = lpgen.sparse_lp(30, 2000, 0.03, seed=9)
    prm = P.Params(w=120, s=2, seed=3)
    ps = P.Problem(_smat(lp.A, "f64"), dev(lp.b), dev(lp.c))
    pd = P.Problem(P.Matrix.from_numpy(lp.A.toarray()), dev(lp.b), dev(lp.c))
    sd = P.State.initial(30, 2000)
    for k in range(8):
        ss = P.State(sd.x.clone(), sd.y.clone(), sd.s.clone(), sd.k, sd.mu0, sd.r0norm)
        a = P.ipm_step(ctx, ps, ss, prm)
        b = P.ipm_step(ctx, pd, sd, prm)
        assert a["rc"] == b["rc"]
        for key in ("mu", "relgap", "rp_rel", "rd_rel"):
            assert a[key] == pytest.approx(b[key], rel=1e-11, abs=1e-15)
        assert abs(a["pcg_iters"] - b["pcg_iters"]) <= 1
        for name in ("x", "y", "s"):
            g, o = host(getattr(ss, name)), host(getattr(sd, name))
            assert np.linalg.norm(g - o) <= 1e-8 * np.linalg.norm(o), (k, name)


def test_sparse_argument_errors(ctx):
    A = _random_csr(10, 100, 0.1, 1, "f64")
    M = _smat(A, "f64")
    c = M.c()
    c.row_ptr = None
    import ctypes
    d = dev(np.ones(100))
    B = torch.empty((10, 40), dtype=torch.float64, device="cuda:0")
    rc = ctx.lib.ipm_sketch(ctx.h, ctypes.byref(c), d.data_ptr(), 0, 0, 40, 2, 0, B.data_ptr())
    assert rc == -1
    c = M.c()
    c.layout = 7
    rc = ctx.lib.ipm_sketch(ctx.h, ctypes.byref(c), d.data_ptr(), 0, 0, 40, 2, 0, B.data_ptr())
    assert rc == -1


# ------------------------------------------------------------------------- full size

def _golden(key, lp):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_optima.json")
    ref = json.load(open(path))[key]
    fp = ref["fingerprint"]
    row0 = lp.A[0].toarray().ravel()
    assert np.allclose(lp.b[:4], fp["b"], rtol=1e-12) and np.allclose(lp.c[:4], fp["c"], rtol=1e-12)
    assert np.abs(row0).sum() == pytest.approx(fp["row0_abs_sum"], rel=1e-12)
    assert ref["converged"]
    return ref


@pytest.fixture(scope="module")
def lp_csr1k():
    print("\ngenerating the 1000 x 1e6 sparse LP (density 1e-3, BF16 values)", flush=True)
    lp = lpgen.workload("csr_1000x1000000")
    # the oracle's direct-solver optimum of this LP, written by tests/golden/make_oracle_optima.py
    return lp, _golden("csr_1000x1000000/0", lp)["objective"]


def test_csr_1000x1000000_matvec_and_sketch(ctx, lp_csr1k):
    lp, _ = lp_csr1k
    m, n = lp.A.shape
    rng = np.random.default_rng(8)
    d = np.exp(rng.uniform(-3, 3, n))
    M = _smat(lp.A, "bf16")
    v = rng.standard_normal(m)
    q = host(P.ipm_normal_matvec(ctx, M, dev(d * d), dev(v)))
    ref = oipm.normal_matrix(lp.A, d * d) @ v
    absA = abs(lp.A)
    bound = absA @ (d * d * (absA.T @ np.abs(v)))
    assert np.all(np.abs(q - ref) <= 64 * EPS * (m + np.sqrt(n)) * bound)
    B = host(P.ipm_sketch(ctx, M, dev(d), 0, 3, 4000, 2))
    Bref = osk.sketch_ADW(lp.A, d, 4000, 2, 0, 3)
    assert np.max(np.abs(B - Bref)) <= 1e-12 * np.max(np.abs(Bref))


def _check(lp, res):
    A = lp.A
    x, y, s = host(res.state.x), host(res.state.y), host(res.state.s)
    assert np.all(x > 0) and np.all(s > 0)
    obj, dual = float(lp.c @ x), float(lp.b @ y)
    assert abs(obj - dual) / (1 + abs(obj)) <= 1e-8
    assert np.linalg.norm(A @ x - lp.b) / (1 + np.linalg.norm(lp.b)) <= 1e-8
    assert np.linalg.norm(A.T @ y + s - lp.c) / (1 + np.linalg.norm(lp.c)) <= 1e-8
    return obj


def test_csr_1000x1000000_solves(ctx, lp_csr1k):
    lp, opt = lp_csr1k
    prob64 = P.Problem(_smat(lp.A, "f64"), dev(lp.b), dev(lp.c))
    prob16 = P.Problem(_smat(lp.A, "bf16"), dev(lp.b), dev(lp.c))
    plain = P.solve(ctx, prob64, P.Params(w=4000, s=2, seed=0))
    mixed = P.solve(ctx, prob16, P.Params(w=4000, s=2, seed=0, precision=P.IPM_MIXED))
    assert plain.converged and mixed.converged
    for res in (plain, mixed):
        obj = _check(lp, res)
        # both are upper bounds of the optimum within their own relative gap (<= 1e-8)
        assert abs(obj - opt) <= 1e-8 * (1 + abs(opt))
    print(f"\nplain {plain.iterations} iterations, mixed {mixed.iterations}", flush=True)


# ------------------------------------------------------------------------- 5000 x 2e6 (Gram-dominated)

@pytest.fixture(scope="module")
def lp_csr5k():
    print("\ngenerating the 5000 x 2e6 sparse LP (density 5e-4, BF16 values)", flush=True)
    return lpgen.workload("csr_5000x2000000")


def test_csr_5000x2000000_matvec_and_sketch(ctx, lp_csr5k):
    lp = lp_csr5k
    m, n = lp.A.shape
    rng = np.random.default_rng(9)
    d = np.exp(rng.uniform(-3, 3, n))
    M = _smat(lp.A, "bf16")
    v = rng.standard_normal(m)
    q = host(P.ipm_normal_matvec(ctx, M, dev(d * d), dev(v)))
    ref = oipm.normal_matrix(lp.A, d * d) @ v
    absA = abs(lp.A)
    bound = absA @ (d * d * (absA.T @ np.abs(v)))
    assert np.all(np.abs(q - ref) <= 64 * EPS * (m + np.sqrt(n)) * bound)
    # the sketch acts row by row (B = A D W), so sampled rows of B are checked against the
    # oracle's sketch of the same rows of A
    B = P.ipm_sketch(ctx, M, dev(d), 0, 5, 40000, 2)
    rows = np.sort(rng.choice(m, size=200, replace=False))
    Bs = host(B[torch.from_numpy(rows).to("cuda:0")])
    del B
    Bref = osk.sketch_ADW(lp.A[rows], d, 40000, 2, 0, 5)
    assert np.max(np.abs(Bs - Bref)) <= 1e-12 * np.max(np.abs(Bref))


def test_csr_5000x2000000_solves(ctx, lp_csr5k):
    lp = lp_csr5k
    prob64 = P.Problem(_smat(lp.A, "f64"), dev(lp.b), dev(lp.c))
    prob16 = P.Problem(_smat(lp.A, "bf16"), dev(lp.b), dev(lp.c))
    plain = P.solve(ctx, prob64, P.Params(w=40000, s=2, seed=0))
    print(f"\nplain {plain.iterations} iterations", flush=True)
    mixed = P.solve(ctx, prob16, P.Params(w=40000, s=2, seed=0, precision=P.IPM_MIXED))
    print(f"mixed {mixed.iterations} iterations", flush=True)
    assert plain.converged and mixed.converged
    op, om = _check(lp, plain), _check(lp, mixed)
    lo, hi = float(lp.b @ lp.y0), float(lp.c @ lp.x0)
    for obj in (op, om):
        assert lo - 1e-8 * abs(lo) <= obj <= hi + 1e-8 * abs(hi)
    # the oracle's direct-solver optimum of this LP (tests/golden/make_oracle_optima.py): every
    # objective is an upper bound of the optimum within its own relative gap (<= 1e-8)
    opt = _golden("csr_5000x2000000/0", lp)["objective"]
    for name, obj in (("plain", op), ("mixed", om)):
        err = abs(obj - opt) / (1 + abs(opt))
        print(f"{name}: objective rel. difference to the oracle {err:.2e}", flush=True)
        assert err <= 1e-8
