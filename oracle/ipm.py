"""Infeasible long-step IPM with a sketch-preconditioned CG normal-equations solve.

TEST INFRASTRUCTURE (oracle). Plain FP64 NumPy/SciPy, written from the paper:

* LP and dual (Section 1, eqs. primal and dual); normal equations
  A D^2 A^T dy = p with D = X^{1/2} S^{-1/2} (Section 1, eq. normal).
* Residuals r_p = A x - b, r_d = A^T y + s - c (Section 5, eq. ipm_residuals).
* Right-hand side p = -r_p - sigma mu A S^{-1} 1 + A x - A D^2 r_d (Section 5,
  below eq. ipm_inf). -r_p + A x equals b, so it is evaluated as
  p = b - A (sigma mu / s + d^2 * r_d); a test checks the two forms agree.
* Algorithm 1 (Section 3): B = A D W, Q = B B^T (eqn. pdprecond), CG on the
  preconditioned system (eq. precond_alt). Q^{-1/2} from the SVD of B and a
  Cholesky factor L of Q give the same CG iterates, and the paper's residual
  norm ||Q^{-1/2} r|| equals ||L^{-1} r||, so Cholesky replaces the SVD.
  Stopping: ||L^{-1} r_j|| <= tol * ||L^{-1} p|| (eq. pdcond2 with a tolerance
  in place of the fixed iteration count t).
* Params.sketch = 1 replaces the sparse embedding by a Gaussian W (the experiments' choice,
  Section 7; oracle.sketch.gaussian_rows), the same W serving Q and v.
* Perturbation v = (XS)^{1/2} W (ADW)^+ (A D^2 A^T dy - p) (Section 4,
  eq. compv) with (ADW)^+ = B^T Q^{-1} since B has full row rank (Lemma
  fullrankR). The residual is the true one, recomputed from dy.
* Directions (Section 5, eq. ipm_inf): ds = -r_d - A^T dy,
  dx = -x + sigma mu / s - d^2 * ds - v / s.
* Step lengths (Algorithm 3, steps 6-7): alpha_max is the end of the
  connected segment [0, alpha] that stays in the infeasible neighbourhood
  N(gamma) = {x_i s_i >= (1-gamma) mu, ||r|| / ||r0|| <= mu / mu0} (Section 5),
  with a backoff theta when it is below 1; alpha_bar minimises mu(alpha) on
  [0, alpha_max]. Update (Algorithm 3, step 8).
* Feasible variant (Params.feasible; Algorithm 2, Section 4) from a strictly
  feasible point: p = A x - sigma mu A S^{-1} 1 (eqn. pdef), ds = -A^T dy
  (eq. dels), the same dx with v (eq. delxhat), and the neighbourhood
  N(gamma) = {x_i s_i >= (1-gamma) mu} without a residual term (eq. neigh);
  alpha_bar minimises (x + alpha dx)^T (s + alpha ds) on [0, alpha_max].

Where the paper is silent the following readings apply (both the oracle and
the GPU library implement them): gamma = 0.9, sigma = 0.5, theta = 0.9999;
the neighbourhood's residual term uses the exact contraction r(alpha) =
(1 - alpha) r that the perturbation v guarantees; a constraint already
violated by rounding at alpha = 0 is only kept from getting worse; the stop
test is relative gap, primal and dual residual all <= gap_tol; CG stops early
when its preconditioned residual drops by less than 1 % over 10 iterations.

Parity unpinned: two policies here are this implementation's, not the paper's
(which draws W once per iteration and runs a fixed number of CG steps), and no
value the paper prints or mathematics fixes pins them: the CG stagnation guard
above, and the redraw rule (sketch_size, sketch_seed and the loop in step: a
draw whose CG fails is redrawn with w doubled, s >= 2 and a shifted seed; a
redrawn W whose Q factors only with a shift is kept). Their tests check the
oracle's own behaviour and that the GPU follows it.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Callable, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .sketch import gaussian_apply, sketch_ADW, sketch_gaussian, sketch_matrix

# status values (oracle-side names)
OK = 0
CONVERGED = 1
PCG_MAXIT = 2
PCG_STAGNATED = 3
ERR_NOT_SPD = -3
ERR_BREAKDOWN = -4
ERR_STALL = -5


@dataclass
class Params:
    sigma: float = 0.5
    gamma: float = 0.9
    theta: float = 0.9999
    tol_pcg: float = 1e-10
    maxit_pcg: int = 500
    gap_tol: float = 1e-8
    maxit_ipm: int = 200
    w: int = 0
    s: int = 2
    seed: int = 0
    vcorr: bool = True
    stag_window: int = 10
    stag_ratio: float = 0.99
    min_step: float = 1e-14
    max_redraws: int = 3
    max_shifts: int = 3
    feasible: bool = False      # Algorithm 2 instead of Algorithm 3
    sketch: int = 0             # 0: sparse embedding (Section 2); 1: Gaussian W (Section 7)
    solver: int = 0             # 0: CG; 1: Chebyshev iteration after a CG probe (Section 3.2)
    cheb_probe: int = 10


@dataclass
class State:
    x: np.ndarray
    y: np.ndarray
    s: np.ndarray
    k: int = 0
    mu0: float = 0.0
    r0norm: float = 0.0


@dataclass
class StepInfo:
    status: int = OK
    k: int = 0
    mu: float = 0.0
    gap: float = 0.0
    relgap: float = 0.0
    rp_rel: float = 0.0
    rd_rel: float = 0.0
    obj: float = 0.0
    alpha_max: float = 0.0
    alpha: float = 0.0
    pcg_iters: int = 0
    pcg_status: int = OK
    pcg_relres: float = 0.0
    vnorm: float = 0.0
    extra: dict = field(default_factory=dict)


def initial_state(A: np.ndarray, b: np.ndarray, c: np.ndarray) -> State:
    """x = s = 1, y = 0; mu0 and ||r0|| taken at this point (start of Algorithm 3)."""
    m, n = A.shape
    st = State(np.ones(n), np.zeros(m), np.ones(n), 0)
    rp, rd = residuals(A, b, c, st.x, st.y, st.s)
    st.mu0 = float(st.x @ st.s / n)
    st.r0norm = float(np.sqrt(rp @ rp + rd @ rd))
    return st


def feasible_state(A, x0: np.ndarray, y0: np.ndarray, s0: np.ndarray) -> State:
    """A strictly feasible start (x0, y0, s0) for Algorithm 2; mu0 taken there, no residual
    reference (the feasible neighbourhood has no residual term)."""
    n = A.shape[1]
    return State(x0.copy(), y0.copy(), s0.copy(), 0, float(x0 @ s0 / n), 0.0)


def normal_matrix(A, d2) -> np.ndarray:
    """M = A diag(d2) A^T as a dense m x m array (A dense or scipy sparse)."""
    if sp.issparse(A):
        return (A.multiply(d2[None, :]).tocsr() @ A.T).toarray()
    return (A * d2) @ A.T


def residuals(A, b, c, x, y, s):
    """Primal and dual residuals (Section 5, eq. ipm_residuals); r_p in R^m, r_d in R^n."""
    return A @ x - b, A.T @ y + s - c


def rhs_p(A, b, x, s, rd, sigma, mu):
    """p = b - A (sigma mu / s + d^2 r_d), the infeasible right-hand side of Section 5."""
    return b - A @ (sigma * mu / s + (x / s) * rd)


def rhs_p_feasible(A, x, s, sigma, mu):
    """p = -sigma mu A S^{-1} 1 + A x, the feasible right-hand side (Section 4, eqn. pdef)."""
    return A @ x - sigma * mu * (A @ (1.0 / s))


def rhs_p_paper_form(A, b, x, s, rd, sigma, mu):
    """p = -r_p - sigma mu A S^{-1} 1 + A x - A D^2 r_d exactly as printed (Section 5)."""
    rp = A @ x - b
    return -rp - sigma * mu * (A @ (1.0 / s)) + A @ x - A @ ((x / s) * rd)


def stop_metrics(A, b, c, x, y, s, rp, rd):
    """Duality gap and relative residuals used by the stop test."""
    ctx = float(c @ x)
    gap = ctx - float(b @ y)
    return dict(
        gap=gap,
        relgap=abs(gap) / (1.0 + abs(ctx)),
        rp_rel=float(np.linalg.norm(rp)) / (1.0 + float(np.linalg.norm(b))),
        rd_rel=float(np.linalg.norm(rd)) / (1.0 + float(np.linalg.norm(c))),
        obj=ctx,
    )


# ---------------------------------------------------------------- PCG (Algorithm 1)

@dataclass
class PCGResult:
    dy: np.ndarray
    iters: int
    status: int
    relres: float            # ||L^{-1} r|| / ||L^{-1} p|| at exit (recursive residual)
    history: list            # ||L^{-1} r_j|| for j = 0..iters
    rho_star: float          # ||L^{-1} p||^2
    warm_used: bool = False
    alphas: list = field(default_factory=list)   # CG step lengths alpha_j (for Lanczos estimates)
    r: Optional[np.ndarray] = None               # recursive residual p - M dy at exit
    interval: tuple = ()                         # Chebyshev: the eigenvalue interval used


def pcg(matvec: Callable, L: np.ndarray, p: np.ndarray, tol: float, maxit: int,
        dy0: Optional[np.ndarray] = None, stag_window: int = 10,
        stag_ratio: float = 0.99) -> PCGResult:
    """CG on Q^{-1/2} M Q^{-1/2} z = Q^{-1/2} p written with the preconditioner Q = L L^T.

    ``matvec(v)`` applies M = A D^2 A^T. The residual norm reported is the
    paper's ||f|| = ||Q^{-1/2}(M dy - p)|| = ||L^{-1} r|| (Section 3.1).

    Warm start (not in the paper): dy0 holds one candidate vector (shape (m,))
    or two (shape (m, 2)). The initial iterate is their combination V c
    closest to the solution in the M-norm, c solving the Galerkin system
    (V^T M V) c = V^T p. Two candidates whose Gram determinant is at most
    1e-8 a11 a22 (nearly parallel in the M-norm) or with a non-positive
    M-norm are reduced to one: beta = v^T p / v^T M v for the first with a
    positive M-norm (beta = 0 if none). The iterate is kept only if its
    preconditioned residual is smaller than that of 0, so the stop test,
    relative to ||L^{-1} p||, is unchanged.
    """
    def lsolve(r):
        return sla.solve_triangular(L, r, lower=True)

    def ltsolve(wv):
        return sla.solve_triangular(L, wv, lower=True, trans="T")

    m = p.shape[0]
    wp = lsolve(p)
    rho_star = float(wp @ wp)
    dy = np.zeros(m)
    r = p.copy()
    wv = wp
    warm_used = False
    if dy0 is not None:
        V = dy0.reshape(m, -1)
        Q = np.stack([matvec(V[:, i]) for i in range(V.shape[1])], axis=1)
        G = V.T @ Q
        rhs = V.T @ p
        coef = np.zeros(V.shape[1])
        if V.shape[1] == 2 and G[0, 0] > 0 and G[1, 1] > 0 and \
                G[0, 0] * G[1, 1] - G[0, 1] * G[1, 0] > 1e-8 * G[0, 0] * G[1, 1]:
            coef = np.linalg.solve(G, rhs)
        else:
            for i in range(V.shape[1]):
                if G[i, i] > 0:
                    coef[i] = rhs[i] / G[i, i]
                    break
        r0 = p - Q @ coef
        w0 = lsolve(r0)
        if float(w0 @ w0) < rho_star:
            dy, r, wv, warm_used = V @ coef, r0, w0, True
    rho = float(wv @ wv)
    hist = [np.sqrt(rho)]
    thresh = tol * np.sqrt(rho_star)
    if np.sqrt(rho) <= thresh:
        rel = np.sqrt(rho / rho_star) if rho_star > 0 else 0.0
        return PCGResult(dy, 0, OK, rel, hist, rho_star, warm_used, [], r)
    z = ltsolve(wv)
    d = z.copy()
    status = PCG_MAXIT
    it = 0
    alphas = []
    while it < maxit:
        q = matvec(d)
        dq = float(d @ q)
        if not dq > 0.0:
            status = ERR_BREAKDOWN
            break
        alpha = rho / dq
        alphas.append(alpha)
        dy = dy + alpha * d
        r = r - alpha * q
        wv = lsolve(r)
        rho_new = float(wv @ wv)
        it += 1
        hist.append(np.sqrt(rho_new))
        if np.sqrt(rho_new) <= thresh:
            status = OK
            break
        if it >= stag_window and hist[-1] > stag_ratio * hist[-1 - stag_window]:
            status = PCG_STAGNATED
            break
        z = ltsolve(wv)
        d = z + (rho_new / rho) * d
        rho = rho_new
    return PCGResult(dy, it, status, hist[-1] / np.sqrt(rho_star), hist, rho_star, warm_used, alphas, r)


def lanczos_ritz(alphas, history) -> np.ndarray:
    """Eigenvalues of the Lanczos tridiagonal T_k that k CG steps build (the Ritz values of the
    preconditioned matrix): with beta_j = rho_{j+1} / rho_j (rho_j = history[j]^2),
    T[0,0] = 1/alpha_0, T[j,j] = 1/alpha_j + beta_{j-1}/alpha_{j-1},
    T[j,j+1] = T[j+1,j] = sqrt(beta_j)/alpha_j."""
    k = len(alphas)
    a = np.asarray(alphas, dtype=float)
    h = np.asarray(history[:k + 1], dtype=float)
    beta = (h[1:] / h[:-1]) ** 2                  # beta_0 .. beta_{k-1}
    diag = 1.0 / a
    diag[1:] += beta[:-1] / a[:-1]
    off = np.sqrt(beta[:-1]) / a[:-1]
    return sla.eigvalsh_tridiagonal(diag, off)


def chebyshev(matvec: Callable, L: np.ndarray, p: np.ndarray, lo: float, hi: float, tol: float, maxit: int,
              dy: np.ndarray, r: np.ndarray, rho_star: float, history: list, start_it: int = 0,
              stag_window: int = 10, stag_ratio: float = 0.99):
    """Preconditioned Chebyshev iteration (Section 3.2) for the eigenvalue interval [lo, hi] of
    Q^{-1} M, continuing from dy with residual r = p - M dy; the three-term recurrence in
    correction form, theta = (hi + lo)/2, delta = (hi - lo)/2, s = delta/theta:
        omega_1 = 1, omega_2 = 1 / (1 - s^2/2), omega_{t+1} = 1 / (1 - s^2 omega_t / 4),
        dx_t = (omega_{t+1}/theta) Q^{-1} r_t + (omega_{t+1} - 1) dx_{t-1},
        dy += dx_t, r -= M dx_t.
    No inner products enter the recurrence; ||L^{-1} r|| is only measured for the stop test.
    Returns (dy, r, iterations, status, history)."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    s2 = (delta / theta) ** 2
    thresh = tol * np.sqrt(rho_star)
    hist = list(history)
    dx = np.zeros_like(dy)
    omega = 1.0
    t = 0
    status = PCG_MAXIT
    while True:
        wv = sla.solve_triangular(L, r, lower=True)
        res = float(np.sqrt(wv @ wv))
        it = start_it + t
        if t > 0:
            hist.append(res)
        if res <= thresh:
            status = OK
            break
        if t > 0 and it >= stag_window and hist[-1] > stag_ratio * hist[-1 - stag_window]:
            status = PCG_STAGNATED
            break
        if it >= maxit:
            status = PCG_MAXIT
            break
        z = sla.solve_triangular(L, wv, lower=True, trans="T")
        omega = 1.0 if t == 0 else (1.0 / (1.0 - 0.5 * s2) if t == 1 else 1.0 / (1.0 - 0.25 * s2 * omega))
        dx = (omega / theta) * z + (omega - 1.0) * dx
        dy = dy + dx
        r = r - matvec(dx)
        t += 1
    return dy, r, start_it + t, status, hist


def pcg_chebyshev(matvec: Callable, L: np.ndarray, p: np.ndarray, tol: float, maxit: int,
                  dy0: Optional[np.ndarray] = None, probe: int = 10, lo_factor: float = 0.5,
                  hi_factor: float = 1.1, stag_window: int = 10, stag_ratio: float = 0.99) -> PCGResult:
    """Chebyshev iteration in place of CG (Section 3.2). Its eigenvalue interval comes from
    Lemma cond3 when the sketch meets eq. pdcond1; at practical sketch sizes it is estimated:
    ``probe`` CG steps run first and the extreme Ritz values theta_min, theta_max of their
    Lanczos tridiagonal give [lo_factor theta_min, hi_factor theta_max] (theta_max approaches
    lambda_max from below, theta_min overestimates lambda_min, hence the margins). Chebyshev
    then continues from the CG iterate."""
    res = pcg(matvec, L, p, tol, min(probe, maxit), dy0=dy0, stag_window=stag_window, stag_ratio=stag_ratio)
    if res.status != PCG_MAXIT or res.iters < probe or res.iters >= maxit:
        return res
    ritz = lanczos_ritz(res.alphas, res.history)
    lo, hi = lo_factor * float(ritz[0]), hi_factor * float(ritz[-1])
    dy, r, it, status, hist = chebyshev(matvec, L, p, lo, hi, tol, maxit, res.dy, res.r, res.rho_star,
                                        res.history, start_it=res.iters, stag_window=stag_window,
                                        stag_ratio=stag_ratio)
    return PCGResult(dy, it, status, hist[-1] / np.sqrt(res.rho_star), hist, res.rho_star, res.warm_used,
                     res.alphas, r, (lo, hi))


# ---------------------------------------------------------------- step lengths

def first_exit(cq, bq, aq):
    """Smallest alpha > 0 at which cq + bq*alpha + aq*alpha^2 drops below min(cq, 0).

    Vectorised over arrays; returns +inf where that never happens. A constraint
    already violated at 0 by rounding (cq < 0) is measured against its value
    at 0, i.e. cq is taken as 0 after shifting.
    """
    cq = np.maximum(np.asarray(cq, dtype=np.float64), 0.0)
    bq = np.asarray(bq, dtype=np.float64)
    aq = np.asarray(aq, dtype=np.float64)
    cq, bq, aq = np.broadcast_arrays(cq, bq, aq)
    out = np.full(cq.shape, np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        # c == 0: alpha*(b + a alpha)
        z = cq == 0.0
        zneg = z & ((bq < 0) | ((bq == 0) & (aq < 0)))
        out[zneg] = 0.0
        zpos = z & ~zneg & (aq < 0)
        out[zpos] = -bq[zpos] / aq[zpos]
        # c > 0, linear
        lin = (~z) & (aq == 0.0) & (bq < 0)
        out[lin] = -cq[lin] / bq[lin]
        # c > 0, quadratic
        qd = (~z) & (aq != 0.0)
        disc = bq * bq - 4.0 * aq * cq
        ok = qd & (disc >= 0)
        sq = np.sqrt(np.where(ok, disc, 0.0))
        qq = -0.5 * (bq + np.copysign(sq, bq))
        r1 = np.where(ok, qq / aq, np.inf)
        r2 = np.where(ok & (qq != 0), cq / qq, np.inf)
        r1 = np.where(r1 > 0, r1, np.inf)
        r2 = np.where(r2 > 0, r2, np.inf)
        out[qd] = np.minimum(r1, r2)[qd]
    return out


def step_lengths(x, s, dx, ds, gamma, theta, mu0, r0norm, rnorm):
    """alpha_max and alpha_bar of Algorithm 3, steps 6-7 (closed form).

    mu(alpha) = (x^T s + alpha a1 + alpha^2 a2) / n with a1 = x^T ds + s^T dx,
    a2 = dx^T ds; x_i(alpha) s_i(alpha) = x_i s_i + alpha (x_i ds_i + s_i dx_i)
    + alpha^2 dx_i ds_i.
    """
    n = x.shape[0]
    xs = float(x @ s)
    a1 = float(x @ ds + s @ dx)
    a2 = float(dx @ ds)
    mu = xs / n
    g = 1.0 - gamma
    roots = [
        first_exit(x * s - g * mu, x * ds + s * dx - g * a1 / n, dx * ds - g * a2 / n).min(),
        first_exit(x, dx, 0.0).min(),
        first_exit(s, ds, 0.0).min(),
    ]
    if r0norm > 0:
        rho = rnorm / r0norm
        roots.append(float(first_exit(xs / (n * mu0) - rho, a1 / (n * mu0) + rho, a2 / (n * mu0))))
    amax = min(1.0, min(roots))
    if amax < 1.0:
        amax *= theta
    if a2 > 0:
        abar = min(max(-a1 / (2.0 * a2), 0.0), amax)
    else:
        abar = amax if (a1 * amax + a2 * amax * amax) <= 0.0 else 0.0
    return amax, abar, dict(a1=a1, a2=a2)


# ---------------------------------------------------------------- sketch redraws

def sketch_size(w: int, s: int, attempt: int):
    """(w, s) of redraw ``attempt``: w doubles per redraw, s is at least 2 after the first."""
    if attempt == 0:
        return w, s
    return w << attempt, max(s, 2)


def sketch_seed(seed: int, attempt: int) -> int:
    """Seed of redraw ``attempt``; the first draw uses the caller's seed unchanged."""
    return seed if attempt == 0 else (seed + attempt * 0x632BE59BD9B4E019) & ((1 << 64) - 1)


# ---------------------------------------------------------------- one IPM iteration

def shifted_cholesky(Q: np.ndarray, max_shifts: int):
    """Cholesky factor of Q, or of Q + delta I when Q's factorization breaks down.

    Q = B B^T formed in FP64 squares the condition number of B = A D W, so a Q whose B is
    still numerically full rank can fail to factor; Algorithm 1 takes Q^{-1/2} from the SVD of
    B, which has no such loss. On breakdown the shift delta_j = u trace(Q) 100^j
    (u = 2^-53, j = 0 .. max_shifts-1; trace(Q) >= ||Q||_2, so delta_0 is the rounding level of
    Q's largest entries) is tried in turn. Returns (L, delta), delta = 0 without a shift, or
    (None, 0) when every shift fails.
    """
    try:
        return sla.cholesky(Q, lower=True), 0.0
    except np.linalg.LinAlgError:
        pass
    m = Q.shape[0]
    base = np.finfo(float).eps / 2 * float(np.trace(Q))
    for j in range(max_shifts):
        delta = base * 100.0 ** j
        try:
            return sla.cholesky(Q + delta * np.eye(m), lower=True), delta
        except np.linalg.LinAlgError:
            continue
    return None, 0.0


def step(A, b, c, st: State, prm: Params, mode: str = "sketch", dy0=None,
         keep: bool = False) -> tuple:
    """One iteration of Algorithm 3 (Algorithm 2 when prm.feasible) from state ``st``; returns
    (new_state, StepInfo).

    mode "exact": A D^2 A^T dy = p solved by Cholesky, v = 0 (IPM with a direct
    solver). mode "sketch": Algorithm 1 with the hash sketch of oracle.sketch and
    the perturbation v of eq. compv (v = 0 if prm.vcorr is False).
    If the stop test already holds, the state is returned unchanged with
    status CONVERGED.
    """
    x, y, s = st.x, st.y, st.s
    m, n = A.shape
    mu = float(x @ s) / n
    rp, rd = residuals(A, b, c, x, y, s)
    met = stop_metrics(A, b, c, x, y, s, rp, rd)
    info = StepInfo(k=st.k, mu=mu, gap=met["gap"], relgap=met["relgap"],
                    rp_rel=met["rp_rel"], rd_rel=met["rd_rel"], obj=met["obj"])
    if max(met["relgap"], met["rp_rel"], met["rd_rel"]) <= prm.gap_tol:
        info.status = CONVERGED
        return st, info
    d2 = x / s
    p = rhs_p_feasible(A, x, s, prm.sigma, mu) if prm.feasible else rhs_p(A, b, x, s, rd, prm.sigma, mu)

    def matvec(v):
        return A @ (d2 * (A.T @ v))

    v = np.zeros(n)
    if mode == "exact":
        Mmat = normal_matrix(A, d2)
        try:
            L = sla.cholesky(Mmat, lower=True)
        except np.linalg.LinAlgError:
            info.status = ERR_NOT_SPD
            return st, info
        dy = sla.cho_solve((L, True), p)
    else:
        # Redraws: the accepted draw is the last one tried; a draw whose Q is not SPD is
        # skipped unless it is the last allowed one (then the step fails). A redrawn W (w
        # doubled, s >= 2) whose Q still factors only with a shift is kept whatever CG did: the
        # shift means kappa(Q) = kappa(ADW)^2 is beyond 1/u, and once the draw is a good
        # embedding kappa(ADW) tracks kappa(AD), which further draws do not change. A first draw
        # that needs a shift is redrawn: with s = 1 or a narrow W the draw itself can leave B
        # nearly rank deficient.
        res = None
        for attempt in range(prm.max_redraws + 1):
            w, sk = sketch_size(prm.w, prm.s, attempt)
            key = sketch_seed(prm.seed, attempt)
            if prm.sketch == 1:
                B = sketch_gaussian(A, np.sqrt(d2), w, key, st.k)
            else:
                B = sketch_ADW(A, np.sqrt(d2), w, sk, key, st.k)
            Q = B @ B.T
            L, shift = shifted_cholesky(Q, prm.max_shifts)
            if L is None:
                if attempt == prm.max_redraws:
                    info.status = ERR_NOT_SPD
                    info.extra.update(attempts=attempt + 1)
                    return st, info
                continue
            if prm.solver == 1:
                res = pcg_chebyshev(matvec, L, p, prm.tol_pcg, prm.maxit_pcg, dy0=dy0, probe=prm.cheb_probe,
                                    stag_window=prm.stag_window, stag_ratio=prm.stag_ratio)
            else:
                res = pcg(matvec, L, p, prm.tol_pcg, prm.maxit_pcg, dy0=dy0,
                          stag_window=prm.stag_window, stag_ratio=prm.stag_ratio)
            if res.status in (OK, ERR_BREAKDOWN) or (shift > 0.0 and attempt > 0):
                break
        info.extra.update(attempts=attempt + 1, w_used=w, s_used=sk, shift=shift)
        info.pcg_iters, info.pcg_status, info.pcg_relres = res.iters, res.status, res.relres
        if res.status == ERR_BREAKDOWN:
            info.status = ERR_BREAKDOWN
            return st, info
        dy = res.dy
        if prm.vcorr:
            rhat = matvec(dy) - p
            gq = sla.cho_solve((L, True), rhat)
            u = B.T @ gq
            if prm.sketch == 1:
                v = np.sqrt(x * s) * gaussian_apply(u, n, w, key, st.k)
            else:
                W = sketch_matrix(n, w, sk, key, st.k)
                v = np.sqrt(x * s) * (W @ u)
        if keep:
            info.extra.update(B=B, Q=Q, L=L, pcg=res)
    ds = -(A.T @ dy) if prm.feasible else -rd - A.T @ dy
    dx = -x + prm.sigma * mu / s - d2 * ds - v / s
    rnorm = float(np.sqrt(rp @ rp + rd @ rd))
    r0ref = 0.0 if prm.feasible else st.r0norm     # no residual term in the feasible N(gamma)
    amax, abar, aux = step_lengths(x, s, dx, ds, prm.gamma, prm.theta, st.mu0, r0ref, rnorm)
    info.alpha_max, info.alpha = amax, abar
    info.vnorm = float(np.linalg.norm(v))
    if keep:
        info.extra.update(p=p, dy=dy, dx=dx, ds=ds, v=v, d2=d2, rp=rp, rd=rd, **aux)
    if abar < prm.min_step:
        info.status = ERR_STALL
        return st, info
    new = State(x + abar * dx, y + abar * dy, s + abar * ds, st.k + 1, st.mu0, st.r0norm)
    if info.status == OK and mode != "exact":
        info.status = info.pcg_status if info.pcg_status > 0 else OK
    return new, info


@dataclass
class SolveResult:
    state: State
    infos: list
    converged: bool
    status: int


def solve(A, b, c, prm: Params, mode: str = "sketch", st: Optional[State] = None,
          callback=None) -> SolveResult:
    """Run Algorithm 3 from x = s = 1, y = 0 (or Algorithm 2 from ``st``, which must then be
    strictly feasible, when prm.feasible) until the stop test holds or maxit_ipm."""
    st = initial_state(A, b, c) if st is None else st
    infos = []
    for _ in range(prm.maxit_ipm + 1):
        new, info = step(A, b, c, st, prm, mode)
        infos.append(info)
        if callback is not None:
            callback(st, info)
        if info.status == CONVERGED:
            return SolveResult(st, infos, True, CONVERGED)
        if info.status < 0:
            return SolveResult(st, infos, False, info.status)
        st = new
    return SolveResult(st, infos, False, OK)


def with_params(prm: Params, **kw) -> Params:
    return replace(prm, **kw)
