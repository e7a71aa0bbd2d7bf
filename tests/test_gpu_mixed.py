"""The mixed-precision forms and the warm starts of the HIP library, through its C ABI, against
the FP64 oracle.

Mixed forms: A is stored in FP32 or BF16 (the stored values define the LP, so both sides solve
the same problem) and the sketch B is accumulated and stored in FP32. IPM_MIXED runs one CG
with FP64-accumulated matvecs; IPM_MIXED_F32ACC accumulates the inner CG matvecs in FP32 and
applies the stop test to the residual recomputed with FP64 accumulation (iterative
refinement). The bar is the plain method's: the paper's preconditioned residual (eq. pdcond2)
recomputed by the oracle below tol_pcg, and the LP optimum within 1e-8. The FP64-oracle error
of each result is printed.
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

TDT = {"f64": None, "f32": "float32", "bf16": "bfloat16"}


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


def tdtype(storage):
    return getattr(torch, TDT[storage]) if TDT[storage] else torch.float64


def rounded(A, storage):
    return {"f64": A, "f32": lpgen.f32_round(A), "bf16": lpgen.bf16_round(A)}[storage]


def _case(m, n, w, s, storage, seed, spread=5.0):
    rng = np.random.default_rng(seed)
    A = rounded(rng.standard_normal((m, n)), storage)
    d2 = np.exp(rng.uniform(-spread, spread, n))
    B = osk.sketch_ADW(A, np.sqrt(d2), w, s, seed, 0)
    L = np.linalg.cholesky(B @ B.T)
    p = rng.standard_normal(m)
    return A, d2, L, p


# ------------------------------------------------------------------------- mixed CG

@pytest.mark.parametrize("m,n,w,storage", [(50, 2000, 200, "f32"), (50, 2000, 200, "bf16"),
                                           (37, 3001, 148, "bf16"), (130, 5003, 520, "f32"),
                                           (500, 20011, 2000, "bf16"), (2000, 12007, 8000, "f32"),
                                           (64, 4096, 256, "f64")])
def test_pcg_mixed_meets_the_fp64_residual_bound(ctx, m, n, w, storage):
    A, d2, L, p = _case(m, n, w, 2, storage, seed=m + n)
    Linv = np.tril(np.linalg.inv(L))
    prm = P.Params(w=w, s=2, precision=P.IPM_MIXED_F32ACC)
    Am = P.Matrix.from_numpy(A, dtype=tdtype(storage))
    dy, info = P.ipm_pcg_solve(ctx, Am, dev(d2), dev(Linv), dev(p), prm)
    dy = host(dy)
    M = (A * d2) @ A.T
    f = sla.solve_triangular(L, M @ dy - p, lower=True)
    fp = sla.solve_triangular(L, p, lower=True)
    rel = np.linalg.norm(f) / np.linalg.norm(fp)
    xs = np.linalg.solve(M, p)
    e = dy - xs
    en = np.sqrt(e @ M @ e) / np.sqrt(xs @ M @ xs)
    print(f"mixed CG {m}x{n} {storage}: iters {info['iters']} rounds {info['rounds']} "
          f"relres(oracle) {rel:.3e} energy err {en:.3e}")
    assert info["status"] == 0
    # the library's FP64-recomputed residual and the oracle's agree, and meet tol
    # (the two recomputations differ only by FP64 rounding of the residual, ~1e-12 relative)
    assert rel <= 1e-10 * 1.01 + 1e-12
    assert info["relres"] == pytest.approx(rel, rel=1e-2, abs=2e-12)
    # error in the M-norm: at most the preconditioned residual times sqrt(kappa(L^-1 M L^-T))
    ev = np.linalg.eigvalsh(sla.solve_triangular(L, sla.solve_triangular(L, M, lower=True).T, lower=True))
    assert en <= 1e-10 * np.sqrt(ev[-1] / ev[0]) * 1.01
    if storage != "f64":
        assert info["rounds"] >= 2    # FP32 inner solves alone cannot reach 1e-10


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_pcg_fp64_accumulation_on_low_storage(ctx, storage):
    """IPM_MIXED's CG: one solve with FP64-accumulated matvecs over the stored values, the same
    iterates as the plain CG on the widened matrix."""
    A, d2, L, p = _case(500, 20011, 2000, 2, storage, seed=11)
    Linv = dev(np.tril(np.linalg.inv(L)))
    dy, info = P.ipm_pcg_solve(ctx, P.Matrix.from_numpy(A, dtype=tdtype(storage)), dev(d2), Linv, dev(p),
                               P.Params(w=2000, s=2, precision=P.IPM_MIXED))
    dyw, infow = P.ipm_pcg_solve(ctx, P.Matrix.from_numpy(A), dev(d2), Linv, dev(p), P.Params(w=2000, s=2))
    assert info["rounds"] == 1 and abs(info["iters"] - infow["iters"]) <= 1
    M = (A * d2) @ A.T
    f = sla.solve_triangular(L, M @ host(dy) - p, lower=True)
    assert np.linalg.norm(f) <= 1e-10 * 1.01 * np.linalg.norm(sla.solve_triangular(L, p, lower=True))
    e = host(dy) - host(dyw)
    assert np.sqrt(e @ M @ e) <= 1e-8 * np.sqrt(host(dyw) @ M @ host(dyw))


def test_pcg_mixed_plain_iteration_budget(ctx):
    """The mixed form's total inner CG count stays within a small factor of the plain count."""
    A, d2, L, p = _case(500, 20011, 2000, 2, "bf16", seed=3)
    Linv = dev(np.tril(np.linalg.inv(L)))
    Am = P.Matrix.from_numpy(A, dtype=torch.bfloat16)
    _, plain = P.ipm_pcg_solve(ctx, Am, dev(d2), Linv, dev(p), P.Params(w=2000, s=2))
    _, mixed = P.ipm_pcg_solve(ctx, Am, dev(d2), Linv, dev(p),
                               P.Params(w=2000, s=2, precision=P.IPM_MIXED_F32ACC))
    print(f"plain {plain['iters']} mixed {mixed['iters']} in {mixed['rounds']} rounds")
    assert mixed["iters"] <= 2 * plain["iters"] + 10


def test_pcg_mixed_warm_start(ctx):
    A, d2, L, p = _case(50, 2000, 200, 2, "bf16", seed=4)
    Linv = dev(np.tril(np.linalg.inv(L)))
    M = (A * d2) @ A.T
    xs = np.linalg.solve(M, p)
    Am = P.Matrix.from_numpy(A, dtype=torch.bfloat16)
    prm = P.Params(w=200, s=2, precision=P.IPM_MIXED_F32ACC)
    good = xs * (1 + 1e-6 * np.random.default_rng(0).standard_normal(xs.size))
    dw, iw = P.ipm_pcg_solve(ctx, Am, dev(d2), Linv, dev(p), prm, dy0=dev(good))
    _, ic = P.ipm_pcg_solve(ctx, Am, dev(d2), Linv, dev(p), prm)
    assert iw["warm_used"] == 1 and iw["iters"] < ic["iters"]
    f = sla.solve_triangular(L, M @ host(dw) - p, lower=True)
    assert np.linalg.norm(f) <= 1e-10 * 1.001 * np.linalg.norm(sla.solve_triangular(L, p, lower=True))
    ds, is_ = P.ipm_pcg_solve(ctx, Am, dev(d2), Linv, dev(p), prm, dy0=dev(-3.0 * xs))
    assert is_["warm_used"] == 1 and is_["iters"] == 0 and is_["rounds"] == 0
    assert np.allclose(host(ds), xs, rtol=1e-8)
    z = np.random.default_rng(1).standard_normal(xs.size)
    z -= (z @ M @ xs) / (xs @ M @ xs) * xs
    _, ib = P.ipm_pcg_solve(ctx, Am, dev(d2), Linv, dev(p), prm, dy0=dev(z))
    assert ib["warm_used"] == 0 and ib["iters"] == ic["iters"]


# ------------------------------------------------------------------------- mixed IPM

def _lockstep(ctx, lp, oprm, gprm, steps, rtol_state):
    """Lock-step (tests/lockstep.py) of a mixed form against the FP64 oracle on the same rounded
    LP. The CG of every form stops on the FP64-accumulated residual at the same tolerance, so dy
    is held to the plain form's energy-norm bound; B is stored in FP32 (a preconditioner, and a
    perturbation v, that differ from the oracle's by FP32 rounding), so the step length is held
    to rtol_state relative and x, s to rtol_state of their update's size. The FP32-accumulated
    form counts the inner iterations of its refinement rounds, so its CG count is not compared."""
    prob = P.Problem.from_lp(lp, dtype=tdtype(lp.storage))
    recs, _, conv = lockstep.run(P, ctx, lp.A, lp.b, lp.c, prob, oprm, gprm, steps, state_tol=rtol_state,
                                 alpha_tol=rtol_state, count_check=gprm.precision != P.IPM_MIXED_F32ACC,
                                 label=f"mixed form {gprm.precision}, {lp.name}")
    return recs, conv


PREC = {"mixed": "IPM_MIXED", "f32acc": "IPM_MIXED_F32ACC"}


@pytest.mark.parametrize("prec", ["mixed", "f32acc"])
@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_step_lockstep_mixed(ctx, storage, prec):
    lp = lpgen.dense_lp(50, 2000, seed=0, storage=storage)
    oprm = oipm.Params(w=200, s=2, seed=1)
    gprm = P.Params(w=200, s=2, seed=1, precision=getattr(P, PREC[prec]))
    # both sides solve to the same preconditioned residual; the directions differ by at most
    # that much, amplified by the step's sensitivity, so states agree far below the stop tolerance
    _, conv = _lockstep(ctx, lp, oprm, gprm, steps=200, rtol_state=1e-7)
    assert conv


@pytest.mark.parametrize("prec", ["mixed", "f32acc"])
@pytest.mark.parametrize("m,n,w,storage,seed", [(50, 2000, 200, "f32", 0), (50, 2000, 200, "bf16", 1),
                                                (23, 1003, 92, "bf16", 5), (300, 20000, 1200, "f32", 2),
                                                (700, 15001, 2800, "bf16", 3)])
def test_solve_mixed_matches_oracle(ctx, m, n, w, storage, seed, prec):
    lp = lpgen.dense_lp(m, n, seed=seed, storage=storage)
    prob = P.Problem.from_lp(lp, dtype=tdtype(storage))
    res = P.solve(ctx, prob, P.Params(w=w, s=2, seed=seed, precision=getattr(P, PREC[prec])))
    ores = oipm.solve(lp.A, lp.b, lp.c, oipm.Params(w=w, s=2, seed=seed), "exact")
    assert res.converged and ores.converged
    x = host(res.state.x)
    obj, oobj = float(lp.c @ x), float(lp.c @ ores.state.x)
    err = abs(obj - oobj) / (1 + abs(oobj))
    xerr = np.linalg.norm(x - ores.state.x) / np.linalg.norm(ores.state.x)
    print(f"mixed solve {lp.name}: iterations {res.iterations} (oracle {len(ores.infos) - 1}), "
          f"objective error {err:.2e}, x error {xerr:.2e}, "
          f"rounds/step {np.mean([i['refine_rounds'] for i in res.infos[:-1]]):.2f}")
    assert err <= 1e-8
    assert abs(res.iterations - (len(ores.infos) - 1)) <= 2
    last = res.infos[-1]
    assert max(last["relgap"], last["rp_rel"], last["rd_rel"]) <= 1e-8
    # stop test recomputed by the oracle on the returned point
    y, s = host(res.state.y), host(res.state.s)
    assert np.linalg.norm(lp.A @ x - lp.b) / (1 + np.linalg.norm(lp.b)) <= 1e-8
    assert np.linalg.norm(lp.A.T @ y + s - lp.c) / (1 + np.linalg.norm(lp.c)) <= 1e-8


# ------------------------------------------------------------------------- warm starts

@pytest.mark.parametrize("precision", ["plain", "mixed", "f32acc"])
def test_solve_warm_prev(ctx, precision):
    lp = lpgen.dense_lp(50, 2000, seed=2, storage="f64" if precision == "plain" else "bf16")
    prob = P.Problem.from_lp(lp, dtype=tdtype(lp.storage))
    prec = getattr(P, PREC[precision]) if precision in PREC else P.IPM_PLAIN
    cold = P.solve(ctx, prob, P.Params(w=200, s=2, precision=prec))
    warm = P.solve(ctx, prob, P.Params(w=200, s=2, precision=prec, warm_start=P.IPM_WARM_PREV))
    assert cold.converged and warm.converged
    oc = float(lp.c @ host(cold.state.x))
    ow = float(lp.c @ host(warm.state.x))
    # both are upper bounds of the optimum within their own relative gap (<= 1e-8)
    assert abs(oc - ow) <= 1e-8 * (1 + abs(oc))
    used = sum(i["warm_used"] for i in warm.infos)
    print(f"{precision}: cold CG {sum(i['pcg_iters'] for i in cold.infos)}, "
          f"prev-warm CG {sum(i['pcg_iters'] for i in warm.infos)}, warm kept in {used} steps")
    assert used >= 1


def test_step_warm_given_matches_oracle(ctx):
    """A warm start equal to the exact Newton solution: both sides keep it and take the same step."""
    lp = lpgen.dense_lp(40, 1500, seed=9)
    prob = P.Problem.from_lp(lp)
    oprm = oipm.Params(w=160, s=2, seed=3)
    gprm = P.Params(w=160, s=2, seed=3, warm_start=P.IPM_WARM_GIVEN)
    st = oipm.initial_state(lp.A, lp.b, lp.c)
    for _ in range(3):
        st, _ = oipm.step(lp.A, lp.b, lp.c, st, oprm, "sketch")
    d2 = st.x / st.s
    M = (lp.A * d2) @ lp.A.T
    _, rd = oipm.residuals(lp.A, lp.b, lp.c, st.x, st.y, st.s)
    p = oipm.rhs_p(lp.A, lp.b, st.x, st.s, rd, oprm.sigma, float(st.x @ st.s) / lp.n)
    dy0 = np.linalg.solve(M, p)
    gst = P.State(dev(st.x), dev(st.y), dev(st.s), st.k, st.mu0, st.r0norm)
    ginfo = P.ipm_step_warm(ctx, prob, gst, gprm, dev(dy0))
    new, oinfo = oipm.step(lp.A, lp.b, lp.c, st, oprm, "sketch", dy0=dy0, keep=True)
    assert ginfo["warm_used"] == 1 and oinfo.extra["pcg"].warm_used
    assert ginfo["pcg_iters"] == oinfo.pcg_iters
    for name in ("x", "y", "s"):
        g, o = host(getattr(gst, name)), getattr(new, name)
        assert np.linalg.norm(g - o) <= 1e-9 * np.linalg.norm(o)
    # the accepted direction is retrievable and is the one the update used
    dy = host(P.ipm_last_dy(ctx, lp.m))
    assert np.linalg.norm(ginfo["alpha"] * dy - (host(gst.y) - st.y)) <= 1e-12 * (1 + np.linalg.norm(st.y))
    assert ginfo["dy_norm"] == pytest.approx(np.linalg.norm(dy), rel=1e-12)


@pytest.mark.parametrize("precision", ["plain", "mixed", "f32acc"])
def test_step_two_candidates_matches_oracle(ctx, precision):
    """Two candidates whose span holds the Newton solution: both sides start from it (no CG
    iteration) and take the same step."""
    lp = lpgen.dense_lp(40, 1500, seed=10, storage="f64" if precision == "plain" else "bf16")
    prob = P.Problem.from_lp(lp, dtype=tdtype(lp.storage))
    oprm = oipm.Params(w=160, s=2, seed=4)
    gprm = P.Params(w=160, s=2, seed=4, warm_start=P.IPM_WARM_GIVEN,
                    precision=getattr(P, PREC[precision]) if precision in PREC else P.IPM_PLAIN)
    st = oipm.initial_state(lp.A, lp.b, lp.c)
    for _ in range(4):
        st, _ = oipm.step(lp.A, lp.b, lp.c, st, oprm, "sketch")
    d2 = st.x / st.s
    _, rd = oipm.residuals(lp.A, lp.b, lp.c, st.x, st.y, st.s)
    p = oipm.rhs_p(lp.A, lp.b, st.x, st.s, rd, oprm.sigma, float(st.x @ st.s) / lp.n)
    xs = np.linalg.solve((lp.A * d2) @ lp.A.T, p)
    v1 = np.random.default_rng(2).standard_normal(lp.m)
    cands = np.stack([v1, 2.5 * xs - 0.7 * v1])
    gst = P.State(dev(st.x), dev(st.y), dev(st.s), st.k, st.mu0, st.r0norm)
    ginfo = P.ipm_step_warm(ctx, prob, gst, gprm, dev(cands))
    new, oinfo = oipm.step(lp.A, lp.b, lp.c, st, oprm, "sketch", dy0=cands.T.copy(), keep=True)
    assert ginfo["warm_used"] == 1 and oinfo.extra["pcg"].warm_used
    assert ginfo["pcg_iters"] == 0 and oinfo.pcg_iters == 0
    for name in ("x", "y", "s"):
        g, o = host(getattr(gst, name)), getattr(new, name)
        assert np.linalg.norm(g - o) <= 1e-9 * np.linalg.norm(o)


# (m, n, storage, layout): every strip-pass instance family the paired product of the two
# candidates runs on (256-thread blocks; 512 threads with 12 and 32 rows per thread, the last
# one per storage type) and the sparse column/row passes; n leaves a ragged last strip
_PAIR_CASES = [(40, 1500, "f64", "dense"), (300, 5003, "f32", "dense"), (700, 4001, "bf16", "dense"),
               (2000, 20011, "f64", "dense"), (2000, 20011, "f32", "dense"), (2000, 12007, "bf16", "dense"),
               (200, 6000, "f64", "csr")]


@pytest.mark.parametrize("m,n,storage,layout", _PAIR_CASES, ids=[f"{c[3]}_{c[0]}x{c[1]}_{c[2]}" for c in _PAIR_CASES])
def test_step_two_generic_candidates_match_oracle(ctx, m, n, storage, layout):
    """Two generic candidates (a perturbed Newton solution and a random vector): the GPU computes
    both products M v_k in one paired pass over A; its step (CG from the M-norm-optimal
    combination, then the update) matches the oracle's, whose products are two plain matvecs."""
    if layout == "csr":
        lp = lpgen.sparse_lp(m, n, 0.02, seed=13, storage=storage)
    else:
        lp = lpgen.dense_lp(m, n, seed=13, storage=storage)
    prob = P.Problem.from_lp(lp, dtype=tdtype(storage))
    w = 4 * m
    oprm = oipm.Params(w=w, s=2, seed=5)
    gprm = P.Params(w=w, s=2, seed=5, warm_start=P.IPM_WARM_GIVEN)
    st = oipm.initial_state(lp.A, lp.b, lp.c)
    for _ in range(4):
        st, _ = oipm.step(lp.A, lp.b, lp.c, st, oprm, "sketch")
    d2 = st.x / st.s
    _, rd = oipm.residuals(lp.A, lp.b, lp.c, st.x, st.y, st.s)
    p = oipm.rhs_p(lp.A, lp.b, st.x, st.s, rd, oprm.sigma, float(st.x @ st.s) / lp.n)
    Mm = oipm.normal_matrix(lp.A, d2)
    xs = np.linalg.solve(Mm, p)
    rng = np.random.default_rng(3)
    v1 = xs + 0.3 * np.linalg.norm(xs) / np.sqrt(m) * rng.standard_normal(m)
    v2 = rng.standard_normal(m)
    cands = np.stack([v1, v2])
    gst = P.State(dev(st.x), dev(st.y), dev(st.s), st.k, st.mu0, st.r0norm)
    ginfo = P.ipm_step_warm(ctx, prob, gst, gprm, dev(cands))
    new, oinfo = oipm.step(lp.A, lp.b, lp.c, st, oprm, "sketch", dy0=cands.T.copy(), keep=True)
    print(f"\n{layout} {m}x{n} {storage}: CG GPU {ginfo['pcg_iters']} oracle {oinfo.pcg_iters}, "
          f"warm kept GPU {ginfo['warm_used']} oracle {int(oinfo.extra['pcg'].warm_used)}")
    assert ginfo["warm_used"] == 1 and oinfo.extra["pcg"].warm_used
    assert ginfo["pcg_iters"] == oinfo.pcg_iters
    assert ginfo["alpha"] == pytest.approx(oinfo.alpha, rel=1e-10, abs=1e-12)
    for name in ("x", "y", "s"):
        g, o = host(getattr(gst, name)), getattr(new, name)
        assert np.linalg.norm(g - o) <= 1e-9 * np.linalg.norm(o), name


def test_warm_given_needs_dy0(ctx):
    lp = lpgen.dense_lp(10, 100, seed=1)
    prob = P.Problem.from_lp(lp)
    st = P.State.initial(10, 100)
    with pytest.raises(P.IpmError) as ei:
        P.ipm_step(ctx, prob, st, P.Params(w=40, s=2, warm_start=P.IPM_WARM_GIVEN))
    assert ei.value.code == -1
    with pytest.raises(P.IpmError):
        P.ipm_step(ctx, prob, st, P.Params(w=40, s=2, precision=5))
    with pytest.raises(P.IpmError):
        P.ipm_step(ctx, prob, st, P.Params(w=40, s=2, inner_tol=0.0))
