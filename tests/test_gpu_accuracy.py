"""Accuracy of the mixed-precision forms against the FP64 oracle, per result.

For each workload (the sparse 1000 x 10^6 and 5000 x 2*10^6 LPs and the dense 500 x 10^5 LP,
all with A stored in BF16: the stored values define the LP both sides solve) and each form (plain
FP64 arithmetic on the stored values, IPM_MIXED, IPM_MIXED_F32ACC), one whole solve to the stop
test; at sampled iterations the accepted dy is compared with the exact Newton direction
dy* = M^{-1} p (M = A D^2 A^T, p the right-hand side of the normal equations, Section 1 and
eq. ipm_inf) that the oracle computes in FP64 by Cholesky at the GPU's own iterate:
    energy error  ||dy - dy*||_M / ||dy*||_M,     Euclidean error  ||dy - dy*|| / ||dy*||.
The final objective is compared with the oracle's optimum of the same LP (tests/golden), the
final relative gap is the GPU's own. The table is printed; the asserts hold every form to the
plain method's bar: optimum within 1e-8, and at each sampled iteration dy within
    tol_pcg * 10^3 + m u kappa(M)
of dy*: the CG's stop test bounds the energy error by tol_pcg sqrt(kappa(Q^{-1} M)) (below
10^3 for the sketches here), and both FP64 sides carry rounding errors of order m u kappa(M)
(u = 2^-53; the Cholesky solve's backward error, and the residual the CG's stop test reads),
which dominate late in the IPM, where kappa(M) grows past 10^10. kappa(M) is estimated by
power and inverse iteration (a lower estimate).
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import lpgen
from oracle import ipm as oipm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
OPTIMA = json.load(open(os.path.join(HERE, "golden", "oracle_optima.json")))
P = None

# (workload, seed, iteration sampling period): dy* costs a dense m x m Cholesky of the oracle's
# normal matrix per sampled iteration
CASES = [("csr_1000x1000000", 0, 3), ("csr_5000x2000000", 0, 8), ("dense_500x100000_bf16", 0, 3)]
FORMS = ("plain", "mixed", "f32acc")
_LP = {}


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


def host(t):
    return t.detach().cpu().numpy()


def _lp(name, seed):
    key = (name, seed)
    if key not in _LP:
        _LP.clear()
        _LP[key] = lpgen.workload(name, seed=seed)
    return _LP[key]


def _exact_dy(A, b, c, x, y, s, sigma):
    """dy* = M^{-1} p at the iterate (x, y, s), by Cholesky of the FP64 normal matrix; with M and
    an estimate of kappa(M) (30 steps of power iteration and of inverse iteration)."""
    mu = float(x @ s) / x.size
    _, rd = oipm.residuals(A, b, c, x, y, s)
    p = oipm.rhs_p(A, b, x, s, rd, sigma, mu)
    M = oipm.normal_matrix(A, x / s)
    cf = sla.cho_factor(M, lower=True)
    rng = np.random.default_rng(0)
    hi, lo = rng.standard_normal(M.shape[0]), rng.standard_normal(M.shape[0])
    for _ in range(30):
        hi = M @ hi
        hi /= np.linalg.norm(hi)
        lo = sla.cho_solve(cf, lo)
        lo /= np.linalg.norm(lo)
    kappa = float(hi @ (M @ hi)) / float(lo @ (M @ lo))
    return sla.cho_solve(cf, p), M, kappa


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("name,seed,period", CASES, ids=[f"{c[0]}/{c[1]}" for c in CASES])
def test_form_accuracy_against_oracle(ctx, name, seed, period, form):
    lp = _lp(name, seed)
    opt = OPTIMA[f"{name}/{seed}"]
    assert float(lp.b[0]) == opt["fingerprint"]["b"][0]   # the LP the optimum was computed for
    w, s = lp.meta["w"], lp.meta["s"]
    prec = {"plain": P.IPM_PLAIN, "mixed": P.IPM_MIXED, "f32acc": P.IPM_MIXED_F32ACC}[form]
    prm = P.Params(w=w, s=s, seed=0, precision=prec)
    prob = P.Problem.from_lp(lp, dtype=torch.bfloat16)
    m, n = lp.m, lp.n
    st = P.State.initial(m, n)
    rows, converged, last = [], False, None
    for k in range(200):
        xk, yk, sk = host(st.x), host(st.y), host(st.s)
        info = P.ipm_step(ctx, prob, st, prm)
        if info["rc"] == P.IPM_CONVERGED:
            converged, last = True, info
            break
        if k % period == 0:
            dy = host(P.ipm_last_dy(ctx, m))
            dys, M, kap = _exact_dy(lp.A, lp.b, lp.c, xk, yk, sk, prm.sigma)
            d = dy - dys
            e_m = float(np.sqrt(max(d @ (M @ d), 0.0) / (dys @ (M @ dys))))
            e_2 = float(np.linalg.norm(d) / np.linalg.norm(dys))
            rows.append((k, e_m, e_2, info["pcg_iters"], info["refine_rounds"], kap))
    assert converged
    obj = float(lp.c @ host(st.x))
    obj_err = abs(obj - opt["objective"]) / (1 + abs(opt["objective"]))
    em = np.array([r[1] for r in rows])
    e2 = np.array([r[2] for r in rows])
    print(f"\n{name}/{seed} {form}: {st.k} iterations, objective {obj:.12e} (oracle {opt['objective']:.12e}, "
          f"rel. diff {obj_err:.2e}), relgap {last['relgap']:.2e}; dy vs the oracle's exact dy at "
          f"{len(rows)} iterations: energy error median {np.median(em):.2e} max {em.max():.2e}, "
          f"Euclidean error median {np.median(e2):.2e} max {e2.max():.2e}")
    for k, a, b_, it, rr, kap in rows:
        print(f"  k={k:3d}  kappa(M) {kap:.1e}  energy {a:.2e}  euclid {b_:.2e}  CG {it}  rounds {rr}")
    assert obj_err <= 1e-8
    assert last["relgap"] <= 1e-8
    u = 2.0 ** -53
    for k, a, _, _, _, kap in rows:
        assert a <= prm.tol_pcg * 1e3 + m * u * kap, (k, a, kap)
