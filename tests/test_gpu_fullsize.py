"""Full-size checks on the ill-conditioned 2000 x 200000 family (A = U diag(sigma) V^T, sigma
log-spaced 1..1e4, FP32 storage, w = 8000, s = 2), generated in device memory.

At this size the oracle's IPM is out of reach, so the checks are: the CG matvec and the sketch
element by element against the oracle's own FP64 routines on the host, and for full solves of the
plain and mixed forms the stop test recomputed on the host in FP64, the duality sandwich of the
generator's witness pair, and agreement of the two forms' objectives.
"""
import numpy as np
import pytest

from oracle import sketch as osk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P = None
M_, N_, W_, S_ = 2000, 200_000, 8000, 2


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


@pytest.fixture(scope="module")
def lp(ctx):
    from lpgen import device as gdev
    print(f"\ngenerating the {M_} x {N_} ill-conditioned LP (seed 64) in device memory", flush=True)
    out = gdev.illcond_lp(M_, N_, seed=64, storage="f32")
    torch.cuda.synchronize()
    return out


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def test_matvec_full_size(ctx, lp):
    rng = np.random.default_rng(1)
    d2 = np.exp(rng.uniform(-6, 6, N_))
    v = rng.standard_normal(M_)
    A = host(lp.A[:, :N_])                       # the stored FP32 values, exactly
    dev = lambda a: torch.from_numpy(a).to("cuda:0")
    for Amat in (P.Matrix(lp.A, N_), P.Matrix(lp.A64, N_)):
        q = host(P.ipm_normal_matvec(ctx, Amat, dev(d2), dev(v)))
        ref = A @ (d2 * (A.T @ v))
        bound = np.abs(A) @ (d2 * (np.abs(A).T @ np.abs(v)))
        assert np.all(np.abs(q - ref) <= 64 * np.finfo(float).eps * (M_ + np.sqrt(N_)) * bound)


def test_sketch_full_size(ctx, lp):
    rng = np.random.default_rng(2)
    d = np.exp(rng.uniform(-3, 3, N_))
    A = host(lp.A[:, :N_])
    B = host(P.ipm_sketch(ctx, P.Matrix(lp.A64, N_), torch.from_numpy(d).to("cuda:0"), 5, 3, W_, S_))
    ref = osk.sketch_ADW(A, d, W_, S_, 5, 3)
    Wm = osk.sketch_matrix(N_, W_, S_, 5, 3)
    bound = np.asarray((abs(Wm).T @ (np.abs(A) * d).T).T)
    assert np.all(np.abs(B - ref) <= 32 * np.finfo(float).eps * np.sqrt(N_) * bound + 1e-300)


def _check_solution(lp, res):
    A = host(lp.A[:, :N_])
    b, c = host(lp.b), host(lp.c)
    x, y, s = host(res.state.x), host(res.state.y), host(res.state.s)
    assert np.all(x > 0) and np.all(s > 0)
    obj, dual = float(c @ x), float(b @ y)
    assert abs(obj - dual) / (1 + abs(obj)) <= 1e-8
    assert np.linalg.norm(A @ x - b) / (1 + np.linalg.norm(b)) <= 1e-8
    assert np.linalg.norm(A.T @ y + s - c) / (1 + np.linalg.norm(c)) <= 1e-8
    # weak duality with the generator's strictly feasible pair: b^T y0 <= opt <= c^T x0
    lo, hi = float(b @ host(lp.y0)), float(c @ host(lp.x0))
    assert lo - 1e-8 * abs(lo) <= obj <= hi + 1e-8 * abs(hi)
    return obj


def test_full_size_solves_plain_and_mixed(ctx, lp):
    plain = P.solve(ctx, P.Problem(P.Matrix(lp.A64, N_), lp.b, lp.c), P.Params(w=W_, s=S_, seed=0))
    mixed = P.solve(ctx, P.Problem(P.Matrix(lp.A, N_), lp.b, lp.c),
                    P.Params(w=W_, s=S_, seed=0, precision=P.IPM_MIXED))
    assert plain.converged and mixed.converged
    op, om = _check_solution(lp, plain), _check_solution(lp, mixed)
    print(f"\nplain: {plain.iterations} iterations, mixed: {mixed.iterations} iterations, "
          f"objective difference {abs(op - om) / (1 + abs(op)):.2e}")
    # each solve stops at relative gap <= 1e-8 with x feasible to rounding, so each objective is
    # an upper bound of the optimum within 1e-8 (relative), and the two agree to 1e-8
    assert abs(op - om) <= 1e-8 * (1 + abs(op))
    assert abs(plain.iterations - mixed.iterations) <= 5
