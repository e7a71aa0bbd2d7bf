"""The l1-SVM LP generator (the experiments' application, Section 7 and the appendix on SVMs)
checked against what the formulation fixes: the LP optimum found by HiGHS is a separating w
with margin 1 whose l1 norm is the optimal value, and the oracle's IPM with and without the
v-correction reaches that optimum."""
import os

import numpy as np
import pytest
from scipy.optimize import linprog

import lpgen
from oracle import ipm as oipm


def test_svm_lp_is_the_l1_svm():
    lp = lpgen.svm_lp(25, 120, seed=4)
    m, N = 25, 120
    assert lp.A.shape == (m, 2 * N + m)
    ref = linprog(lp.c, A_eq=lp.A, b_eq=lp.b, bounds=(0, None), method="highs")
    assert ref.status == 0
    w = ref.x[:N] - ref.x[N:2 * N]
    X, y = lp.meta["features"], lp.meta["labels"]
    assert np.min(y * (X @ w)) >= 1 - 1e-9                  # every point outside the margin
    assert abs(np.abs(w).sum() - ref.fun) <= 1e-9 * ref.fun  # objective = ||w||_1
    # no smaller l1 norm separates: scaling the optimum down breaks the margin
    assert np.min(y * (X @ (0.99 * w))) < 1


@pytest.mark.parametrize("vcorr", [True, False])
def test_oracle_solves_svm_lp(vcorr):
    lp = lpgen.svm_lp(20, 100, seed=1)
    ref = linprog(lp.c, A_eq=lp.A, b_eq=lp.b, bounds=(0, None), method="highs")
    res = oipm.solve(lp.A, lp.b, lp.c, oipm.Params(w=80, s=2, seed=0, vcorr=vcorr), "sketch")
    assert res.converged
    assert abs(float(lp.c @ res.state.x) - ref.fun) <= 1e-7 * (1 + abs(ref.fun))


def test_svm_shapes_are_table1():
    """The four l1-SVM shapes and sketch widths are those Table 1 prints (tests/golden)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1_svm_shapes.txt")
    with open(path) as f:
        rows = [line.split() for line in f if line.strip() and not line.startswith("#")]
    assert {r[0]: dict(m=int(r[1]), N=int(r[2]), w=int(r[3])) for r in rows} == lpgen.SVM_SHAPES
