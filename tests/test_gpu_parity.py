"""Parity of the HIP library (through its C ABI) with the FP64 oracle on the same seeded inputs.

Every comparison is element by element against the oracle or, for the LP optimum, against
quantities the oracle tests pin independently. Tolerances are stated per test with the
reason.
"""
import numpy as np
import pytest
import scipy.linalg as sla

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
    return t.detach().cpu().numpy()


def rand_lp_matrix(m, n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, n))


# ------------------------------------------------------------------------- matvec pass

@pytest.mark.parametrize("m,n", [(1, 100), (7, 33), (50, 2000), (37, 1001), (130, 5003), (500, 20011),
                                 (257, 4096), (1000, 3000)])
def test_normal_matvec_fp64(ctx, m, n):
    A = rand_lp_matrix(m, n, m * 7 + n)
    rng = np.random.default_rng(1)
    d2 = np.exp(rng.uniform(-6, 6, n))
    v = rng.standard_normal(m)
    q = host(P.ipm_normal_matvec(ctx, P.Matrix.from_numpy(A), dev(d2), dev(v)))
    ref = A @ (d2 * (A.T @ v))
    # FP64 summation bound: |error| <= c * eps * |A| (d2 * |A|^T |v|) with c ~ m + n
    bound = np.abs(A) @ (d2 * (np.abs(A).T @ np.abs(v)))
    assert np.all(np.abs(q - ref) <= 64 * np.finfo(float).eps * (m + np.sqrt(n)) * bound + 1e-300)


@pytest.mark.parametrize("m,n,dtype", [(60, 3001, "f32"), (60, 3001, "bf16"), (1500, 4003, "f64"),
                                       (2000, 3001, "f32"), (2000, 5003, "bf16"), (513, 1999, "bf16"),
                                       (1000, 1777, "bf16")])
def test_normal_matvec_low_storage(ctx, m, n, dtype):
    A = rand_lp_matrix(m, n, 5)
    if dtype == "bf16":
        A, tdt = lpgen.bf16_round(A), torch.bfloat16
    elif dtype == "f32":
        A, tdt = lpgen.f32_round(A), torch.float32
    else:
        tdt = torch.float64
    rng = np.random.default_rng(2)
    d2 = np.exp(rng.uniform(-3, 3, n))
    v = rng.standard_normal(m)
    q = host(P.ipm_normal_matvec(ctx, P.Matrix.from_numpy(A, dtype=tdt), dev(d2), dev(v)))
    ref = A @ (d2 * (A.T @ v))
    bound = np.abs(A) @ (d2 * (np.abs(A).T @ np.abs(v)))
    # storage is exact (values are representable); accumulation is FP64
    assert np.all(np.abs(q - ref) <= 64 * np.finfo(float).eps * (m + np.sqrt(n)) * bound)


# ------------------------------------------------------------------------- sketch

@pytest.mark.parametrize("m,n,w,s,seed,k", [(50, 2000, 200, 1, 0, 0), (37, 1001, 96, 3, 5, 7),
                                            (5, 40, 12, 3, 11, 4), (64, 5000, 256, 8, 2, 1),
                                            (500, 20000, 2000, 2, 9, 3), (3, 17, 4, 2, 1, 0),
                                            (20, 5000, 48000, 2, 3, 1), (7, 3001, 30000, 3, 2, 0),
                                            # column chunks added atomically: two rows per block with an
                                            # odd last row block; one row per block at two and at one
                                            # block per CU (w = 6000 and 12000); short last chunks
                                            (101, 30001, 4000, 2, 4, 2), (60, 50001, 6000, 2, 7, 1),
                                            (30, 40000, 12000, 3, 1, 0)])
def test_sketch_parity(ctx, m, n, w, s, seed, k):
    A = rand_lp_matrix(m, n, 100 + m)
    rng = np.random.default_rng(3)
    d = np.exp(rng.uniform(-2, 2, n))
    B = host(P.ipm_sketch(ctx, P.Matrix.from_numpy(A), dev(d), seed, k, w, s))
    ref = osk.sketch_ADW(A, d, w, s, seed, k)
    # each bucket sums ~ n*s/w terms; only the summation order differs
    W = osk.sketch_matrix(n, w, s, seed, k)
    bound = np.asarray((abs(W).T @ (np.abs(A) * d).T).T)
    assert np.all(np.abs(B - ref) <= 32 * np.finfo(float).eps * np.sqrt(n) * bound + 1e-300)


@pytest.mark.parametrize("m,n,w,s", [(37, 30011, 9000, 2), (10, 20011, 12000, 3), (9, 30001, 16000, 2),
                                     (2000, 20011, 16000, 2)])
def test_sketch_bf16_one_row_blocks(ctx, m, n, w, s):
    """BF16 A whose w buckets fill a block's LDS (one row per block, d / sqrt(s) from the per-call
    vector): column chunks added atomically at small m, one pass over the columns at m = 2000."""
    A = lpgen.bf16_round(rand_lp_matrix(m, n, 31))
    d = np.exp(np.random.default_rng(5).uniform(-2, 2, n))
    B = host(P.ipm_sketch(ctx, P.Matrix.from_numpy(A, dtype=torch.bfloat16), dev(d), 6, 3, w, s))
    ref = osk.sketch_ADW(A, d, w, s, 6, 3)
    W = osk.sketch_matrix(n, w, s, 6, 3)
    bound = np.asarray((abs(W).T @ (np.abs(A) * d).T).T)
    assert np.all(np.abs(B - ref) <= 32 * np.finfo(float).eps * np.sqrt(n) * bound + 1e-300)


@pytest.mark.parametrize("dt,ld", [("f64", 20016), ("f32", 20016), ("bf16", 20016), ("f64", 20014)])
@pytest.mark.parametrize("m,n,w,s,out", [(9, 20011, 16000, 2, "f64"), (300, 20013, 9000, 1, "f32"),
                                         (3, 5, 9000, 2, "f64")])
def test_sketch_one_row_blocks_row_strides(ctx, dt, ld, m, n, w, s, out):
    """One row per block with the buckets and signs from the per-call packed table: the pipelined
    four-column kernel for FP32 and BF16 A (ragged last quad of columns), the per-column kernel for
    FP64 A (row strides of 4k and 4k + 2 elements); s = 1 and 2, column chunks added atomically
    (m = 9) and one pass (m = 300); five columns (one ragged quad, most lanes without a column)."""
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dt]
    A = rand_lp_matrix(m, n, 41)
    if dt == "bf16":
        A = lpgen.bf16_round(A)
    elif dt == "f32":
        A = lpgen.f32_round(A)
    pad = torch.full((m, ld), float("nan"), dtype=torch.float64)   # the padding is never read
    pad[:, :n] = torch.from_numpy(A)
    mat = P.Matrix(pad.to(tdt).to("cuda:0").contiguous(), n)
    d = np.exp(np.random.default_rng(7).uniform(-2, 2, n))
    odt = torch.float64 if out == "f64" else torch.float32
    B = host(P.ipm_sketch(ctx, mat, dev(d), 9, 4, w, s, out_dtype=odt))
    ref = osk.sketch_ADW(A, d, w, s, 9, 4)
    W = osk.sketch_matrix(n, w, s, 9, 4)
    bound = np.asarray((abs(W).T @ (np.abs(A) * d).T).T)
    tol = 32 * np.finfo(float).eps * np.sqrt(n) * bound + (4 * 2.0 ** -24 * bound if out == "f32" else 0)
    assert np.all(np.abs(B - ref) <= tol + 1e-300)


@pytest.mark.parametrize("m,n,w,s", [(40, 3000, 160, 2), (130, 7001, 520, 2), (9, 4000, 50000, 2)])
def test_sketch_fp32_output(ctx, m, n, w, s):
    """FP32 B: accumulated in FP64, stored rounded to FP32 (w = 50000 takes the bucket-range path)."""
    A = rand_lp_matrix(m, n, 8)
    d = np.exp(np.random.default_rng(4).uniform(-1, 1, n))
    B = host(P.ipm_sketch(ctx, P.Matrix.from_numpy(A), dev(d), 3, 2, w, s, out_dtype=torch.float32))
    ref = osk.sketch_ADW(A, d, w, s, 3, 2)
    W = osk.sketch_matrix(n, w, s, 3, 2)
    bound = np.asarray((abs(W).T @ (np.abs(A) * d).T).T)
    # FP64 accumulation, then at most a few FP32 roundings (one per column chunk added atomically)
    assert np.all(np.abs(B - ref) <= 4 * 2.0 ** -24 * bound + 32 * np.finfo(float).eps * np.sqrt(n) * bound)


# ------------------------------------------------------------------------- factor

@pytest.mark.parametrize("m,w", [(1, 4), (50, 200), (64, 128), (65, 130), (130, 520), (200, 400), (500, 2000)])
def test_precond_factor(ctx, m, w):
    rng = np.random.default_rng(m)
    B = rng.standard_normal((m, w)) * np.exp(rng.uniform(-2, 2, (m, 1)))
    L, Linv = P.ipm_precond_factor(ctx, dev(B))
    L, Linv = np.tril(host(L)), host(Linv)
    Q = B @ B.T
    Lref = np.linalg.cholesky(Q)
    kap = np.linalg.cond(Lref)
    assert np.linalg.norm(L - Lref) <= 1e-13 * kap * np.linalg.norm(Lref)
    assert np.allclose(np.triu(Linv, 1), 0.0)
    assert np.linalg.norm(Linv @ Lref - np.eye(m)) <= 1e-13 * kap * kap * np.sqrt(m)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gpu_preconditioned_spectrum_lemma_cond3(ctx, seed):
    """The spectral condition the method relies on (eq. pdcond1, Lemma cond3), on the GPU's own
    sketch and factor: with a wide embedding (w = 100 m, s = 8) the eigenvalues of
    X A D^2 A^T X^T (X = L^{-1} from ipm_precond_factor of B = ipm_sketch) lie in
    [2/(2+zeta), 2/(2-zeta)], zeta = 1/2, and equal the oracle's for the same W."""
    lp = lpgen.tiny_lp(20, 2000, 8)
    rng = np.random.default_rng(2)
    d2 = np.exp(rng.uniform(-4, 4, lp.n))
    B = P.ipm_sketch(ctx, P.Matrix.from_numpy(lp.A), dev(np.sqrt(d2)), seed, 0, 2000, 8)
    _, Linv = P.ipm_precond_factor(ctx, B)
    X = host(Linv)
    M = (lp.A * d2) @ lp.A.T
    ev = np.linalg.eigvalsh(X @ M @ X.T)
    zeta = 0.5
    assert ev.min() >= 2 / (2 + zeta) and ev.max() <= 2 / (2 - zeta)
    Bo = osk.sketch_ADW(lp.A, np.sqrt(d2), 2000, 8, seed, 0)
    Lo = np.linalg.cholesky(Bo @ Bo.T)
    evo = np.linalg.eigvalsh(sla.solve_triangular(Lo, sla.solve_triangular(Lo, M, lower=True).T, lower=True))
    assert np.allclose(ev, evo, rtol=1e-9, atol=0)


@pytest.mark.parametrize("r", [16, 17, 70])
def test_precond_factor_reports_bad_pivot(ctx, r):
    """A zero row of B makes pivot r of Q = B B^T exactly zero: IPM_ERR_NOT_SPD with bad_pivot = r
    (the diagonal blocks eliminate two columns per step: r even is a step's first pivot, r odd
    its second; r = 70 lies in the second 64-column block)."""
    import ctypes
    rng = np.random.default_rng(0)
    B = rng.standard_normal((80, 160))
    B[r] = 0.0
    with pytest.raises(P.IpmError) as ei:
        P.ipm_precond_factor(ctx, dev(B))
    assert ei.value.code == -3
    Bd = dev(B)
    Linv = torch.empty((80, 80), dtype=torch.float64, device="cuda:0")
    bad = ctypes.c_int64(-2)
    rc = ctx.lib.ipm_precond_factor(ctx.h, 80, 160, P.IPM_F64, ctypes.c_void_p(Bd.data_ptr()), None,
                                    ctypes.c_void_p(Linv.data_ptr()), ctypes.byref(bad))
    assert rc == -3 and bad.value == r


# ------------------------------------------------------------------------- PCG

def _pcg_case(m=50, n=2000, w=200, s=2, seed=0):
    A = rand_lp_matrix(m, n, 31)
    rng = np.random.default_rng(seed)
    d2 = np.exp(rng.uniform(-5, 5, n))
    B = osk.sketch_ADW(A, np.sqrt(d2), w, s, seed, 0)
    L = np.linalg.cholesky(B @ B.T)
    p = rng.standard_normal(m)
    return A, d2, L, p


@pytest.mark.parametrize("maxit", [500, 1, 3])
def test_pcg_parity(ctx, maxit):
    A, d2, L, p = _pcg_case()
    Linv = np.linalg.inv(L)
    prm = P.Params(w=200, s=2, maxit_pcg=maxit)
    dy, info = P.ipm_pcg_solve(ctx, P.Matrix.from_numpy(A), dev(d2), dev(np.tril(Linv)), dev(p), prm)
    dy = host(dy)
    M = (A * d2) @ A.T
    ref = oipm.pcg(lambda v: M @ v, L, p, 1e-10, maxit)
    assert abs(info["iters"] - ref.iters) <= 1
    if maxit < 10:
        assert info["iters"] == ref.iters
        assert info["status"] == 2
    e = dy - ref.dy
    en = np.sqrt(e @ M @ e) / np.sqrt(ref.dy @ M @ ref.dy)
    assert en <= (1e-8 if maxit >= 10 else 1e-12)
    # the paper's residual ||Q^{-1/2}(M dy - p)|| recomputed by the oracle
    f = sla.solve_triangular(L, M @ dy - p, lower=True)
    fp = sla.solve_triangular(L, p, lower=True)
    if maxit >= 10:
        assert np.linalg.norm(f) <= 1e-10 * np.linalg.norm(fp) * 1.01 + 1e-12 * np.linalg.norm(fp)


def test_pcg_warm_start(ctx):
    A, d2, L, p = _pcg_case(seed=4)
    Linv = np.tril(np.linalg.inv(L))
    M = (A * d2) @ A.T
    xs = np.linalg.solve(M, p)
    prm = P.Params(w=200, s=2)
    good = xs * (1 + 1e-4 * np.random.default_rng(0).standard_normal(xs.size))
    dy_w, info_w = P.ipm_pcg_solve(ctx, P.Matrix.from_numpy(A), dev(d2), dev(Linv), dev(p), prm, dy0=dev(good))
    _, info_c = P.ipm_pcg_solve(ctx, P.Matrix.from_numpy(A), dev(d2), dev(Linv), dev(p), prm)
    assert info_w["warm_used"] == 1 and info_w["iters"] < info_c["iters"]
    ref = oipm.pcg(lambda v: M @ v, L, p, 1e-10, 500, dy0=good)
    assert abs(info_w["iters"] - ref.iters) <= 1
    # a multiple of the solution is scaled back to it (energy-optimal factor): no iteration
    dy_s, info_s = P.ipm_pcg_solve(ctx, P.Matrix.from_numpy(A), dev(d2), dev(Linv), dev(p), prm,
                                   dy0=dev(-3.0 * xs))
    assert info_s["warm_used"] == 1 and info_s["iters"] == 0
    assert np.allclose(host(dy_s), xs, rtol=1e-8)
    # a direction M-orthogonal to the solution gets beta = 0 and is rejected
    z = np.random.default_rng(1).standard_normal(xs.size)
    z -= (z @ M @ xs) / (xs @ M @ xs) * xs
    _, info_b = P.ipm_pcg_solve(ctx, P.Matrix.from_numpy(A), dev(d2), dev(Linv), dev(p), prm, dy0=dev(z))
    assert info_b["warm_used"] == 0 and abs(info_b["iters"] - info_c["iters"]) <= 1


# ------------------------------------------------------------------------- IPM step and solve

def _gpu_state(st):
    return P.State(dev(st.x), dev(st.y), dev(st.s), st.k, st.mu0, st.r0norm)


def _lockstep(ctx, lp, oprm, gprm, steps, label=""):
    """Lock-step through the whole solve (or ``steps`` steps): see tests/lockstep.py for what is
    compared and the bounds."""
    recs, _, conv = lockstep.run(P, ctx, lp.A, lp.b, lp.c, P.Problem.from_lp(lp), oprm, gprm, steps, label=label)
    return recs, conv


def test_step_lockstep_dense_50x2000(ctx):
    """Every iteration of the 50 x 2000 workload (s = 1, w = 200) to the oracle's stop test."""
    lp = lpgen.workload("dense_50x2000")
    recs, conv = _lockstep(ctx, lp, oipm.Params(w=200, s=1, seed=0), P.Params(w=200, s=1, seed=0), steps=200,
                           label="dense_50x2000")
    assert conv and len(recs) >= 25


def test_step_lockstep_ragged(ctx):
    lp = lpgen.dense_lp(23, 1003, seed=5)
    recs, conv = _lockstep(ctx, lp, oipm.Params(w=92, s=2, seed=7), P.Params(w=92, s=2, seed=7), steps=200,
                           label="dense 23x1003")
    assert conv


@pytest.mark.parametrize("near", [True, False])
def test_redraw_rule_matches_oracle(ctx, near):
    """CG capped at 2 iterations fails on every draw. With a well-conditioned A all four draws are
    tried, as in the oracle's step. With nearly dependent rows (kappa(Q) ~ 1e20) whether a draw's
    Cholesky needs a shift is decided by rounding noise in the pivot, so the GPU and the oracle may
    stop at different draws; the GPU must stop before the last draw only on a redraw that needed
    a shift."""
    rng = np.random.default_rng(5)
    m, n = 6, 600
    A = rng.standard_normal((m, n))
    if near:
        A[1] = A[0] + 1e-10 * rng.standard_normal(n)
    x0 = rng.uniform(0.5, 1.5, n)
    y0, s0 = rng.standard_normal(m), rng.uniform(0.5, 1.5, n)
    b, c = A @ x0, A.T @ y0 + s0
    st = oipm.initial_state(A, b, c)
    st, _ = oipm.step(A, b, c, st, oipm.Params(w=24, s=2, seed=1), "sketch")
    _, oinfo = oipm.step(A, b, c, st, oipm.Params(w=24, s=2, seed=1, maxit_pcg=2), "sketch")
    prob = P.Problem(P.Matrix.from_numpy(A), dev(b), dev(c))
    ginfo = P.ipm_step(ctx, prob, _gpu_state(st), P.Params(w=24, s=2, seed=1, maxit_pcg=2))
    assert ginfo["pcg_status"] == oinfo.pcg_status == oipm.PCG_MAXIT
    assert ginfo["w_used"] == 24 << (ginfo["attempts"] - 1)
    if near:
        assert ginfo["attempts"] == 4 or (ginfo["attempts"] >= 2 and ginfo["shift"] > 0)
    else:
        assert ginfo["attempts"] == oinfo.extra["attempts"] == 4
        assert ginfo["shift"] == oinfo.extra["shift"] == 0


def test_solve_dense_50x2000_matches_oracle(ctx):
    lp = lpgen.workload("dense_50x2000")
    res = P.solve(ctx, P.Problem.from_lp(lp), P.Params(w=200, s=1, seed=0))
    ores = oipm.solve(lp.A, lp.b, lp.c, oipm.Params(w=200, s=1, seed=0), "sketch")
    assert res.converged and ores.converged
    assert abs(res.iterations - len(ores.infos) + 1) <= 1
    x = host(res.state.x)
    obj = float(lp.c @ x)
    oobj = float(lp.c @ ores.state.x)
    assert abs(obj - oobj) <= 1e-8 * (1 + abs(oobj))
    last = res.infos[-1]
    assert max(last["relgap"], last["rp_rel"], last["rd_rel"]) <= 1e-8
    assert np.linalg.norm(x - ores.state.x) <= 1e-5 * np.linalg.norm(ores.state.x)


@pytest.mark.parametrize("m,n,w,s", [(1, 50, 4, 2), (6, 6, 24, 2), (4, 11, 8, 1), (20, 2000, 2000, 8)])
def test_solve_edge_shapes(ctx, m, n, w, s):
    if m == 1:
        rng = np.random.default_rng(6)
        a = rng.uniform(0.5, 2.0, n)
        c = rng.uniform(0.1, 3.0, n)
        A, b = a[None, :], np.array([3.0])
        lp = lpgen.LP(A, b, c, None, None, None)
        opt = 3.0 * np.min(c / a)
    else:
        lp = lpgen.dense_lp(m, n, seed=m + n)
        ores = oipm.solve(lp.A, lp.b, lp.c, oipm.Params(w=w, s=s), "exact")
        opt = float(lp.c @ ores.state.x)
    res = P.solve(ctx, P.Problem.from_lp(lp), P.Params(w=w, s=s))
    assert res.converged
    obj = float(lp.c @ host(res.state.x))
    # both objectives are upper bounds of the optimum within their own relative gap (<= 1e-8)
    assert abs(obj - opt) <= 1e-8 * (1 + abs(opt))


def test_argument_errors(ctx):
    lp = lpgen.dense_lp(10, 100, seed=1)
    prob = P.Problem.from_lp(lp)
    for bad in (P.Params(w=8, s=2), P.Params(w=30, s=4), P.Params(w=40, s=9)):
        st = P.State.initial(10, 100)
        with pytest.raises(P.IpmError) as ei:
            P.ipm_step(ctx, prob, st, bad)
        assert ei.value.code == -1
        assert float(st.x.sum()) == 100.0   # untouched


@pytest.mark.parametrize("dtype,mmax", [("f64", 2048), ("f32", 2048), ("bf16", 6400)])
def test_dense_row_limit(ctx, dtype, mmax):
    """The largest m a dense A accepts (the strip pass keeps all m rows of a column strip on
    chip): the matvec at that m, with a ragged n, against the definition; one row more is
    IPM_ERR_ARG."""
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    rnd = {"f64": lambda a: a, "f32": lpgen.f32_round, "bf16": lpgen.bf16_round}[dtype]
    n = mmax + 1003
    A = rnd(rand_lp_matrix(mmax, n, mmax))
    rng = np.random.default_rng(4)
    d2 = np.exp(rng.uniform(-3, 3, n))
    v = rng.standard_normal(mmax)
    q = host(P.ipm_normal_matvec(ctx, P.Matrix.from_numpy(A, dtype=tdt), dev(d2), dev(v)))
    ref = A @ (d2 * (A.T @ v))
    bound = np.abs(A) @ (d2 * (np.abs(A).T @ np.abs(v)))
    assert np.all(np.abs(q - ref) <= 64 * np.finfo(float).eps * (mmax + np.sqrt(n)) * bound)
    del A
    big = P.Matrix.from_numpy(np.ones((mmax + 1, mmax + 8)), dtype=tdt)
    with pytest.raises(P.IpmError) as ei:
        P.ipm_normal_matvec(ctx, big, dev(np.ones(mmax + 8)), dev(np.ones(mmax + 1)))
    assert ei.value.code == -1 and "limit" in str(ei.value)


def test_step_rejects_oversized_dense_before_device_work(ctx):
    m, n = 2049, 2100
    prob = P.Problem(P.Matrix.from_numpy(np.ones((m, n))), dev(np.ones(m)), dev(np.ones(n)))
    st = P.State.initial(m, n)
    with pytest.raises(P.IpmError) as ei:
        P.ipm_step(ctx, prob, st, P.Params(w=2 * m, s=2))
    assert ei.value.code == -1
    assert float(st.x.sum()) == n and float(st.y.abs().sum()) == 0.0   # untouched


def test_method_option_errors(ctx):
    """Out-of-range method switches (feasible, solver, sketch) and a non-zero reserved field
    are IPM_ERR_ARG, with the state untouched; m > n is rejected."""
    from dataclasses import replace
    lp = lpgen.dense_lp(10, 100, seed=1)
    prob = P.Problem.from_lp(lp)
    base = P.Params(w=40, s=2)

    class Reserved(P.Params):
        def c(self):
            cp = super().c()
            cp.reserved = 1
            return cp

    for bad in (replace(base, feasible=2), replace(base, solver=2), replace(base, solver=-1),
                replace(base, sketch=2), Reserved(w=40, s=2)):
        st = P.State.initial(10, 100)
        with pytest.raises(P.IpmError) as ei:
            P.ipm_step(ctx, prob, st, bad)
        assert ei.value.code == -1
        assert float(st.x.sum()) == 100.0
    tall = P.Matrix.from_numpy(np.ones((12, 8)))
    with pytest.raises(P.IpmError) as ei:
        P.ipm_normal_matvec(ctx, tall, dev(np.ones(8)), dev(np.ones(12)))
    assert ei.value.code == -1


_LP500 = {}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("chunk", range(5))
def test_dense_500x100000_lockstep_every_iteration(ctx, chunk):
    """The bench workload (500 x 100000, w = 2000, s = 2, seed 0) in lock-step with the oracle,
    every iteration to the oracle's stop test: 12 steps per test, the oracle's iterate carried
    from one test to the next."""
    if chunk == 0:
        print("\ngenerating dense_500x100000 seed 0", flush=True)
        _LP500.clear()
        _LP500["lp"] = lpgen.workload("dense_500x100000", seed=0)
        _LP500["st"] = None
    lp = _LP500["lp"]
    if _LP500.get("converged"):
        return
    recs, st, conv = lockstep.run(P, ctx, lp.A, lp.b, lp.c, P.Problem.from_lp(lp), oipm.Params(w=2000, s=2, seed=0),
                                  P.Params(w=2000, s=2, seed=0), 12, st=_LP500["st"],
                                  label=f"dense_500x100000 seed 0, steps {12 * chunk}-")
    _LP500["st"], _LP500["converged"] = st, conv
    if chunk == 4:
        assert conv, "the oracle's solve should stop within 60 iterations"
        del _LP500["lp"]


def _golden_optimum(key):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_optima.json")
    return json.load(open(path))[key]


def _check_fingerprint(lp, fp):
    row0 = lp.A[0].toarray().ravel() if hasattr(lp.A, "toarray") else np.asarray(lp.A[0])
    assert np.allclose(lp.b[:4], fp["b"], rtol=1e-12) and np.allclose(lp.c[:4], fp["c"], rtol=1e-12)
    assert row0.sum() == pytest.approx(fp["row0_sum"], rel=1e-12, abs=1e-9)
    assert np.abs(row0).sum() == pytest.approx(fp["row0_abs_sum"], rel=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_dense_500x100000_solve_matches_oracle(ctx, seed):
    """Seeds 0-4 of the 500 x 100000 workload: the GPU's plain FP64 solve against the oracle's
    direct-solver optimum (tests/golden/oracle_optima.json, written by make_oracle_optima.py from
    the oracle alone). Both objectives are upper bounds of the optimum within their own gap, so
    with both relative gaps <= 1e-8 they agree to 1e-8 relative."""
    ref = _golden_optimum(f"dense_500x100000/{seed}")
    lp = lpgen.workload("dense_500x100000", seed=seed)
    _check_fingerprint(lp, ref["fingerprint"])
    res = P.solve(ctx, P.Problem.from_lp(lp), P.Params(w=2000, s=2, seed=seed))
    assert res.converged and ref["converged"]
    x, y, s_ = host(res.state.x), host(res.state.y), host(res.state.s)
    obj = float(lp.c @ x)
    # the stop test recomputed on the host
    assert (obj - float(lp.b @ y)) / (1 + abs(obj)) <= 1e-8
    assert np.linalg.norm(lp.A @ x - lp.b) / (1 + np.linalg.norm(lp.b)) <= 1e-8
    assert np.linalg.norm(lp.A.T @ y + s_ - lp.c) / (1 + np.linalg.norm(lp.c)) <= 1e-8
    assert np.all(x > 0) and np.all(s_ > 0)
    err = abs(obj - ref["objective"]) / (1 + abs(ref["objective"]))
    print(f"\nseed {seed}: GPU {res.iterations} iterations, oracle {ref['iterations']}, "
          f"objective rel. difference {err:.2e}")
    assert err <= 1e-8
    assert abs(res.iterations - ref["iterations"]) <= 2


def test_dense_ld_limit_rejected_before_device_work(ctx):
    """The strip passes address the rows of a 64-row (here 32-row) group with a 32-bit element
    offset: a dense A whose row stride would overflow it is IPM_ERR_ARG before any device access
    (the descriptor points at a 16-byte aligned one-element buffer, never read)."""
    import ctypes
    buf = torch.zeros(2, dtype=torch.float64, device="cuda:0")
    d2 = torch.ones(4, dtype=torch.float64, device="cuda:0")
    m = 100                                      # 256-thread blocks, 32 rows per group
    # FP64 strips are 16 columns wide: 31 ld + 16 must stay below 2^32
    ld = ((1 << 32) - 1 - 16) // 31 + 1
    ld += ld % 2                                 # a 16-byte multiple, so only the offset limit fails
    assert 31 * ld + 16 > (1 << 32) - 1 and 31 * (ld - 2) + 16 <= (1 << 32) - 1
    Ac = P.native.IpmMatrix(m, ld, ld, 0, 0, buf.data_ptr())
    rc = ctx.lib.ipm_normal_matvec(ctx.h, ctypes.byref(Ac), buf.data_ptr(), d2.data_ptr(), d2.data_ptr())
    assert rc == -1 and "ld=" in ctx.lib.ipm_last_error(ctx.h).decode()
    # 1025 <= m <= 2048: a 64-row group's bytes must fit the 32-bit range of a buffer descriptor
    m = 1500
    ld = 1 << 23                                 # 64 * ld * 8 bytes = 2^32
    Ac = P.native.IpmMatrix(m, ld, ld, 0, 0, buf.data_ptr())
    rc = ctx.lib.ipm_normal_matvec(ctx.h, ctypes.byref(Ac), buf.data_ptr(), d2.data_ptr(), d2.data_ptr())
    assert rc == -1 and "ld=" in ctx.lib.ipm_last_error(ctx.h).decode()


def test_row_limit_of_the_cg_kernels(ctx):
    """m above the CG kernels' LDS limit (two FP64 m-vectors per block) is IPM_ERR_ARG for a CSR
    A and for the factor, before device work."""
    import ctypes
    m, n = 10237, 10240
    z64 = torch.zeros(m + 1, dtype=torch.int64, device="cuda:0")
    zc = torch.zeros(n + 1, dtype=torch.int64, device="cuda:0")
    zi = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    v = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    Ac = P.native.IpmMatrix(m, n, 0, 1, 0, v.data_ptr(), 0, z64.data_ptr(), zi.data_ptr(), v.data_ptr(),
                            zc.data_ptr(), zi.data_ptr())
    rc = ctx.lib.ipm_normal_matvec(ctx.h, ctypes.byref(Ac), v.data_ptr(), v.data_ptr(), v.data_ptr())
    assert rc == -1 and "limit" in ctx.lib.ipm_last_error(ctx.h).decode()
    bad = ctypes.c_int64(0)
    rc = ctx.lib.ipm_precond_factor(ctx.h, m, m, 0, v.data_ptr(), None, v.data_ptr(), ctypes.byref(bad))
    assert rc == -1
