"""Lock-step comparison of the library's ipm_step with the oracle's step (test helper, imported by
the GPU tests).

Every step starts both sides from the oracle's iterate, so rounding differences never compound
across steps. Both sides draw the same W (the hash definition of the sparse embedding), form the
same Q and run CG to the same preconditioned-residual tolerance, so per step they compute the
same quantities up to rounding:

- the stop metrics (mu, relative gap and residuals) to 1e-11 relative;
- dy, in the energy norm of M = A D^2 A^T: ||D A^T (dy_gpu - dy_oracle)|| / ||D A^T dy_oracle||.
  A vector with ||L^-1 (p - M dy)|| <= tau ||L^-1 p|| (eq. pdcond2) has a relative energy-norm
  error of at most tau sqrt(kappa(P)), P = L^-1 M L^-T (the preconditioned matrix; from
  r^T M^-1 r <= ||L^-1 r||^2 / lambda_min(P) and p^T M^-1 p >= ||L^-1 p||^2 / lambda_max(P)).
  tau is each side's true residual for the oracle's p, M and L, recomputed in FP64 (it includes
  CG's drift from its recursive residual and the rounding of p, which cancels late in the IPM),
  so the two sides differ by at most (tau_gpu + tau_oracle) sqrt(kappa(P)). Asserted as at most
  the larger of 1e-8 and twice that bound while the oracle's kappa(M) <= 1e5; beyond, where
  FP64 itself loses digits in proportion to kappa(M) (measured: 1e-8 to 4e-8 at kappa(M) = 3e5
  to 6e5 on 40 x 3000 and 30 x 300 LPs with CG residuals of 1e-13), stated;
- the step length alpha_bar: |d alpha| <= 1e-10 under the same condition;
- x and s entry by entry: beyond what the two sides' dy and alpha differences propagate
  (e = |A|^T |dy_gpu - dy_oracle|: s_j moves by alpha e_j and x_j by alpha d_j^2 e_j, both by
  |d alpha| |ds_j| or |d alpha| |dx_j|), an entry may differ by at most 1e-8 of the size of the
  update that produced it, |x_j| + alpha |dx_j| (the same for s). A norm over n entries would be
  dominated by the O(1) basic entries; this test sees a wrong non-basic entry of 1e-9 as well as
  a wrong basic one. Asserted under the same condition; y is compared as an m-vector, norm-wise,
  beyond the propagated alpha ||d dy|| + |d alpha| ||dy||.

A step whose two sides accepted different draws of W (CG stagnating on one side only, which
finite-precision CG on an ill-conditioned system can do) is stated, not asserted.

Iteration counts are not a parity quantity (CG in finite precision; counts may differ by a few
once the preconditioned system is ill-conditioned); they are compared within 10 %, and the
number of draws of W must agree, under the same condition. The stop metrics are compared at every
step: mu to 1e-11 relative, the relative gap and residuals to 1e-11 relative or 1e-13 absolute
(near the optimum c^T x - b^T y cancels, and each side rounds it at about u |c^T x|).
"""
from __future__ import annotations

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import ipm as oipm

KAPPA_GATE = 1e5
DY_FLOOR = 1e-8
ALPHA_TOL = 1e-10
STATE_TOL = 1e-8


def _host(t):
    return t.detach().cpu().numpy()


def _entry_err(g, o, old, upd, propagated):
    """Largest difference beyond the propagated part, relative to the update's size."""
    scale = np.abs(old) + np.abs(upd)
    excess = np.maximum(np.abs(g - o) - propagated, 0.0)
    return float(np.max(excess / np.maximum(scale, 1e-300)))


def run(P, ctx, A, b, c, prob, oprm, gprm, steps, st=None, state_tol=STATE_TOL, alpha_tol=ALPHA_TOL,
        kappa_gate=KAPPA_GATE, pcg_slack=2, count_check=True, check=None, label=""):
    """Lock-step from ``st`` (default: the oracle's start) for up to ``steps`` steps or until the
    oracle's stop test holds. ``check(old_state, gpu_state, gpu_info, oracle_info)`` runs extra
    per-step assertions. Returns (records, final oracle state, converged)."""
    import torch
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")  # noqa: E731
    st = oipm.initial_state(A, b, c) if st is None else st
    m = A.shape[0]
    recs = []
    try:
        return _run(P, ctx, A, b, c, prob, oprm, gprm, steps, st, m, dev, recs, state_tol, alpha_tol,
                    kappa_gate, pcg_slack, count_check, check, label)
    except AssertionError:
        _print(recs, label + " (failed)")
        raise


def _run(P, ctx, A, b, c, prob, oprm, gprm, steps, st, m, dev, recs, state_tol, alpha_tol, kappa_gate,
         pcg_slack, count_check, check, label):
    for _ in range(steps):
        gst = P.State(dev(st.x), dev(st.y), dev(st.s), st.k, st.mu0, st.r0norm)
        ginfo = P.ipm_step(ctx, prob, gst, gprm)
        new, oinfo = oipm.step(A, b, c, st, oprm, "sketch", keep=True)
        assert oinfo.status >= 0 and ginfo["rc"] >= 0, (st.k, oinfo.status, ginfo["rc"])
        for key, ab in (("mu", 0.0), ("relgap", 1e-13), ("rp_rel", 1e-13), ("rd_rel", 1e-13)):
            assert ginfo[key] == pytest.approx(getattr(oinfo, key), rel=1e-11, abs=ab), \
                (st.k, key, ginfo[key], getattr(oinfo, key))
        if oinfo.status == oipm.CONVERGED:
            assert ginfo["rc"] == 1
            _print(recs, label)
            return recs, st, True
        ex = oinfo.extra
        d2 = ex["d2"]
        Mm = oipm.normal_matrix(A, d2)
        kappa = float(np.linalg.cond(Mm))
        Lo = ex["L"]
        Pm = sla.solve_triangular(Lo, sla.solve_triangular(Lo, Mm, lower=True).T, lower=True)
        ev = np.linalg.eigvalsh(0.5 * (Pm + Pm.T))
        kappa_pre = float(ev[-1] / max(ev[0], 1e-300))
        dy_g = _host(P.ipm_last_dy(ctx, m))
        # each side's true preconditioned residual for the oracle's system, recomputed in FP64
        fp = np.linalg.norm(sla.solve_triangular(Lo, ex["p"], lower=True))
        tau_g = float(np.linalg.norm(sla.solve_triangular(Lo, ex["p"] - Mm @ dy_g, lower=True)) / fp)
        tau_o = float(np.linalg.norm(sla.solve_triangular(Lo, ex["p"] - Mm @ ex["dy"], lower=True)) / fp)
        dy_bound = 2.0 * (tau_g + tau_o) * np.sqrt(kappa_pre)
        e = A.T @ (dy_g - ex["dy"])
        ref = A.T @ ex["dy"]
        dy_energy = float(np.sqrt(np.sum(d2 * e * e)) / np.sqrt(np.sum(d2 * ref * ref)))
        dy_2 = float(np.linalg.norm(dy_g - ex["dy"]) / np.linalg.norm(ex["dy"]))
        a = oinfo.alpha
        da = abs(ginfo["alpha"] - a)
        xg, yg, sg = _host(gst.x), _host(gst.y), _host(gst.s)
        eprop = abs(A).T @ np.abs(dy_g - ex["dy"])
        attempts = (ginfo["attempts"], ex.get("attempts", 1))
        rec = dict(k=st.k, kappa=kappa, kappa_pre=kappa_pre, relres=(tau_g, tau_o), dy_bound=dy_bound,
                   pcg_gpu=ginfo["pcg_iters"], pcg_oracle=oinfo.pcg_iters, attempts=attempts,
                   pcg_status=(ginfo["pcg_status"], oinfo.pcg_status), dy_energy=dy_energy, dy_2=dy_2,
                   dalpha=da, alpha=a,
                   x_entry=_entry_err(xg, new.x, st.x, a * ex["dx"], a * d2 * eprop + da * np.abs(ex["dx"])),
                   s_entry=_entry_err(sg, new.s, st.s, a * ex["ds"], a * eprop + da * np.abs(ex["ds"])),
                   y_norm=float(max(np.linalg.norm(yg - new.y) - 2.0 * (a * np.linalg.norm(dy_g - ex["dy"]) +
                                                                       da * np.linalg.norm(ex["dy"])), 0.0)
                                / max(np.linalg.norm(new.y), 1e-300)))
        recs.append(rec)
        if check is not None:
            check(st, gst, ginfo, oinfo)
        assert ginfo["pcg_relres"] <= oprm.tol_pcg or ginfo["pcg_status"] > 0, rec
        if kappa <= kappa_gate and attempts[0] == attempts[1]:
            if count_check:
                assert abs(ginfo["pcg_iters"] - oinfo.pcg_iters) <= max(pcg_slack, 0.1 * oinfo.pcg_iters), \
                    (label, rec)
            assert dy_energy <= max(DY_FLOOR, dy_bound), (label, rec)
            assert rec["dalpha"] <= alpha_tol * max(1.0, a), (label, rec)
            assert rec["x_entry"] <= state_tol and rec["s_entry"] <= state_tol, (label, rec)
            assert rec["y_norm"] <= state_tol, (label, rec)
        st = new
    _print(recs, label)
    return recs, st, False


def _print(recs, label):
    if not recs:
        return
    print(f"\nlock-step {label}: k, kappa(M), kappa(P), CG gpu/oracle, relres gpu/oracle, dy energy err "
          f"(bound), dy 2-norm err, |d alpha|, x entry err, s entry err")
    for r in recs:
        flag = "" if r["kappa"] <= KAPPA_GATE else "  (stated: kappa > 1e5)"
        if r["attempts"][0] != r["attempts"][1]:
            flag += f"  (stated: draws of W gpu/oracle {r['attempts'][0]}/{r['attempts'][1]})"
        print(f"  {r['k']:3d} {r['kappa']:9.2e} {r['kappa_pre']:9.2e} {r['pcg_gpu']:3d}/{r['pcg_oracle']:3d} "
              f"{r['relres'][0]:8.1e}/{r['relres'][1]:8.1e} {r['dy_energy']:9.2e} ({r['dy_bound']:8.1e}) "
              f"{r['dy_2']:9.2e} {r['dalpha']:9.2e} {r['x_entry']:9.2e} {r['s_entry']:9.2e}{flag}", flush=True)
