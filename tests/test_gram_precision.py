"""Why the mixed form's Gram Q = B B^T accumulates in FP64 although B is stored in FP32 (CPU,
oracle only): on an ill-conditioned family (kappa(A) = 1e4, so kappa(A D^2 A^T) passes 1e8 at
once and 1e12 later) the FP64 Gram of the FP32-rounded sketch still preconditions A D^2 A^T to a
small condition number, while the same Gram summed in FP32 is not positive definite within a
few IPM iterations."""
import numpy as np
import pytest

import lpgen
from oracle import ipm as oipm
from oracle import sketch as osk


def _preconditioned_kappa(Q, M):
    try:
        L = np.linalg.cholesky(Q)
    except np.linalg.LinAlgError:
        return np.inf
    Li = np.linalg.inv(L)
    P = Li @ M @ Li.T
    e = np.linalg.eigvalsh(0.5 * (P + P.T))
    return e[-1] / e[0] if e[0] > 0 else np.inf


def test_fp32_gram_fails_where_fp64_gram_preconditions():
    lp = lpgen.illcond_lp(100, 10000, seed=3, cond=1e4)
    prm = oipm.Params(w=4000, s=2, seed=1)
    st = oipm.initial_state(lp.A, lp.b, lp.c)
    k64, k32 = [], []
    for k in range(8):
        d2 = st.x / st.s
        M = oipm.normal_matrix(lp.A, d2)
        B = osk.sketch_ADW(lp.A, np.sqrt(d2), prm.w, prm.s, prm.seed, k).astype(np.float32)
        B64 = B.astype(np.float64)
        k64.append(_preconditioned_kappa(B64 @ B64.T, M))
        k32.append(_preconditioned_kappa((B @ B.T).astype(np.float64), M))
        st, _ = oipm.step(lp.A, lp.b, lp.c, st, prm, "sketch")
    print(f"\nkappa of the preconditioned matrix, FP64 Gram: {np.round(k64, 2)}; FP32 Gram: {k32}")
    assert max(k64) < 20.0
    assert sum(np.isinf(k32[2:])) >= 3
