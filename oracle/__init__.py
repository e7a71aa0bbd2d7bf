"""Oracle for the sketch-preconditioned infeasible interior point method.

TEST INFRASTRUCTURE. Only the test suite, the entry point's smoke check and
the benchmark's CPU-baseline leg may import this package. The product path
(the HIP library and its Python binding) never imports, calls or links it,
and it never imports the product.

Plain, slow, FP64 NumPy/SciPy code written from the paper (Chowdhury,
Dexter, London, Avron, Drineas: "Faster Randomized Interior Point Methods
for Tall/Wide Linear Programs"):

* ``oracle.sketch``  - the sparse embedding W (Section 2) and the sketch A D W
  (Algorithm 1, step 1).
* ``oracle.ipm``     - the infeasible long-step IPM (Algorithm 3, Section 5):
  residuals, right-hand side p, the normal equations solved exactly by
  Cholesky ("IPM with a direct solver") or by preconditioned CG with
  Q = (ADW)(ADW)^T (Algorithm 1, Section 3), the perturbation v (eq. compv),
  step lengths and the update.
* ``oracle.vertex``  - brute-force vertex enumeration for tiny LPs (the
  independent pin of the LP optimum).
* ``oracle.mlp``     - FP64 reference of the warm-start MLP (not in the paper).

Readings of passages the paper leaves open are listed in the repository's
design notes; each function's docstring names the passage it follows.
"""
from . import sketch, ipm, vertex, mlp  # noqa: F401
