"""Seeded synthetic LP generators shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the interior point method. It only draws
inputs: a constraint matrix ``A`` (m x n, m << n, full row rank with
probability 1), and a strictly feasible primal/dual pair from which the
right-hand sides are built, so the LP

    min c^T x  s.t.  A x = b, x >= 0          (primal, Section 1)
    max b^T y  s.t.  A^T y + s = c, s >= 0     (dual, Section 1)

is feasible and bounded by construction:

    x0 ~ U(0.5, 1.5)^n,  b = A x0,
    y0 ~ N(0, 1)^m,  s0 ~ U(0.5, 1.5)^n,  c = A^T y0 + s0.

Draw order with ``numpy.random.default_rng(seed)``: A (pattern first for
sparse A), then x0, y0, s0.

The paper's own workloads are l1-SVM LPs on UCI data sets (Section 7,
Table 1); those data sets are not used. The shapes here extend the paper's
m << n regime; the values follow the recipe above.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = ["LP", "dense_lp", "sparse_lp", "svm_lp", "tiny_lp", "workload", "bf16_round", "f32_round",
           "WORKLOADS", "SVM_SHAPES", "mlp_init"]


@dataclass
class LP:
    """A standard-form LP ``min c^T x, A x = b, x >= 0`` plus its generator's witness pair."""
    A: np.ndarray            # (m, n) float64 row-major (values may be bf16/fp32-representable)
    b: np.ndarray            # (m,) float64
    c: np.ndarray            # (n,) float64
    x0: np.ndarray           # strictly feasible primal witness
    y0: np.ndarray           # dual witness
    s0: np.ndarray           # strictly positive dual slack witness
    storage: str = "f64"     # element type the GPU path stores A in: "f64" | "f32" | "bf16"
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even); returned as float64.

    Used so that the BF16-stored matrix *is* the problem: both precisions then
    solve the same LP.
    """
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16) << np.uint64(16)
    return (u.astype(np.uint32).view(np.float32)).astype(np.float64)


def f32_round(a: np.ndarray) -> np.ndarray:
    """Round to the nearest float32; returned as float64."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _witness(rng: np.random.Generator, A: np.ndarray):
    m, n = A.shape
    x0 = rng.uniform(0.5, 1.5, size=n)
    y0 = rng.standard_normal(m)
    s0 = rng.uniform(0.5, 1.5, size=n)
    b = A @ x0
    c = A.T @ y0 + s0
    return b, c, x0, y0, s0


def dense_lp(m: int, n: int, seed: int = 0, storage: str = "f64", name: str = "") -> LP:
    """Dense LP with A i.i.d. N(0, 1), rounded to ``storage`` precision."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    if storage == "bf16":
        A = bf16_round(A)
    elif storage == "f32":
        A = f32_round(A)
    b, c, x0, y0, s0 = _witness(rng, A)
    return LP(A, b, c, x0, y0, s0, storage=storage, name=name or f"dense{m}x{n}s{seed}")


def sparse_lp(m: int, n: int, density: float, seed: int = 0, storage: str = "f64", name: str = "") -> LP:
    """Sparse LP, A in CSR (scipy.sparse.csr_matrix): round(density m n) positions drawn uniformly
    without replacement, then one random row added to every column left empty (so no column of
    A is zero); values N(0, 1) rounded to ``storage``. Draw order: pattern, fill rows, values,
    then the witness pair."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    k = int(round(density * m * n))
    flat = rng.choice(m * n, size=k, replace=False)
    rows, cols = flat // n, flat % n
    has = np.zeros(n, dtype=bool)
    has[cols] = True
    empty = np.flatnonzero(~has)
    rows = np.concatenate([rows, rng.integers(0, m, size=empty.size)])
    cols = np.concatenate([cols, empty])
    vals = rng.standard_normal(rows.size)
    if storage == "bf16":
        vals = bf16_round(vals)
    elif storage == "f32":
        vals = f32_round(vals)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    A.sum_duplicates()
    A.sort_indices()
    b, c, x0, y0, s0 = _witness(rng, A)
    return LP(A, b, c, x0, y0, s0, storage=storage, name=name or f"sparse{m}x{n}s{seed}")


def svm_lp(m: int, N: int, seed: int = 0, k: int = 10, density: float = 1.0, name: str = "") -> LP:
    """l1-regularised SVM as a standard-form LP (the experiments' application, Section 7 and the
    appendix on SVMs), on synthetic data: m training points x_i in R^N with N(0, 1) features
    (a fraction ``density`` of them nonzero), labels y_i = sign(x_i^T beta) for a k-sparse
    N(0, 1) beta (separable through the origin, so the LP is feasible). Variables w+, w- (N each)
    and surplus t (m): minimise 1^T (w+ + w-) subject to y_i x_i^T (w+ - w-) - t_i = 1,
    (w+, w-, t) >= 0, i.e. A = [Y X, -Y X, -I] (m x (2N + m)), b = 1, c = [1, 1, 0]. The bias b'
    of the SVM is left out (its split into two free parts with zero cost would make the optimal
    face unbounded). Draw order: beta's support, beta, features (pattern first when sparse).
    No witness pair is drawn (x0, y0, s0 are None)."""
    rng = np.random.default_rng(seed)
    supp = rng.choice(N, size=min(k, N), replace=False)
    beta = np.zeros(N)
    beta[supp] = rng.standard_normal(supp.size)
    if density < 1.0:
        mask = rng.random((m, N)) < density
        X = np.where(mask, rng.standard_normal((m, N)), 0.0)
    else:
        X = rng.standard_normal((m, N))
    y = np.sign(X @ beta)
    y[y == 0] = 1.0
    YX = y[:, None] * X
    A = np.hstack([YX, -YX, -np.eye(m)])
    b = np.ones(m)
    c = np.concatenate([np.ones(2 * N), np.zeros(m)])
    lp = LP(A, b, c, None, None, None, storage="f64", name=name or f"svm{m}x{N}s{seed}")
    lp.meta.update(features=X, labels=y)
    return lp


# The experiments' four l1-SVM shapes (m training points x N features) and sketch widths
# (Section 7, Table 1); synthetic stand-ins for the UCI data sets named there.
SVM_SHAPES = {
    "arcene": dict(m=100, N=10_000, w=200),
    "dexter": dict(m=300, N=20_000, w=500),
    "drivface": dict(m=606, N=6400, w=1000),
    "gene_rna": dict(m=801, N=20_531, w=2000),
}


def tiny_lp(m: int, n: int, seed: int) -> LP:
    """Small dense LP for brute-force checks (same recipe as ``dense_lp``)."""
    return dense_lp(m, n, seed, name=f"tiny{m}x{n}s{seed}")


def illcond_lp(m: int, n: int, seed: int = 0, matrix_seed: int = 1000,
               cond: float = 1e4, storage: str = "f32") -> LP:
    """A = U diag(sigma) V^T with Haar U (m x m), V (n x m) orthonormal columns,
    sigma log-spaced from 1 to ``cond``; A is drawn once from ``matrix_seed`` and
    (b, c) from ``seed``."""
    rng_a = np.random.default_rng(matrix_seed)
    G = rng_a.standard_normal((m, m))
    U, R = np.linalg.qr(G)
    U = U * np.sign(np.diag(R))
    H = rng_a.standard_normal((n, m))
    V, R2 = np.linalg.qr(H)
    V = V * np.sign(np.diag(R2))
    sig = np.logspace(0.0, np.log10(cond), m)
    A = (U * sig) @ V.T
    A = f32_round(A) if storage == "f32" else (bf16_round(A) if storage == "bf16" else A)
    rng = np.random.default_rng(seed)
    b, c, x0, y0, s0 = _witness(rng, A)
    return LP(A, b, c, x0, y0, s0, storage=storage, name=f"illcond{m}x{n}s{seed}")


# Workload table: (kind, m, n, storage, sketch width w, nonzeros per sketch row s, seeds)
WORKLOADS = {
    "dense_50x2000": dict(kind="dense", m=50, n=2000, storage="f64", w=200, s=1, seeds=[0]),
    "dense_500x100000": dict(kind="dense", m=500, n=100_000, storage="f64", w=2000, s=2, seeds=[0, 1, 2, 3, 4]),
    # the same generator with A rounded to BF16 (the mixed forms' accuracy on a dense workload)
    "dense_500x100000_bf16": dict(kind="dense", m=500, n=100_000, storage="bf16", w=2000, s=2, seeds=[0]),
    "csr_1000x1000000": dict(kind="csr", m=1000, n=1_000_000, storage="bf16", w=4000, s=2, seeds=[0],
                             density=1e-3),
    "illcond_2000x200000": dict(kind="illcond", m=2000, n=200_000, storage="f32", w=8000, s=2,
                                seeds=list(range(80))),
    "dense_2000x2000000": dict(kind="dense", m=2000, n=2_000_000, storage="bf16", w=16000, s=2, seeds=[0]),
    "csr_5000x2000000": dict(kind="csr", m=5000, n=2_000_000, storage="bf16", w=40000, s=2, seeds=[0],
                             density=5e-4),
}


def workload(name: str, seed: Optional[int] = None) -> LP:
    """Build the named workload (a key of WORKLOADS) at ``seed`` (defaults to its first seed)."""
    cfg = WORKLOADS[name]
    sd = cfg["seeds"][0] if seed is None else seed
    if cfg["kind"] == "illcond":
        lp = illcond_lp(cfg["m"], cfg["n"], seed=sd, storage=cfg["storage"])
    elif cfg["kind"] == "csr":
        lp = sparse_lp(cfg["m"], cfg["n"], cfg["density"], seed=sd, storage=cfg["storage"],
                       name=f"{name}_s{sd}")
    else:
        lp = dense_lp(cfg["m"], cfg["n"], seed=sd, storage=cfg["storage"], name=f"{name}_s{sd}")
    lp.meta.update(w=cfg["w"], s=cfg["s"], workload=name, seed=sd)
    return lp


def mlp_init(n_in: int, n_hidden: int, n_out: int, seed: int = 0, out_scale: float = 0.01) -> np.ndarray:
    """Initial weights of the warm-start network, flat in the layout W1 [H x I], b1 [H],
    W2 [H x H], b2 [H], W3 [O x H], b3 [O]: W1, W2 ~ N(0, 2 / fan_in) (He et al., 2015),
    W3 ~ N(0, out_scale^2 / H), biases 0. Returned as float32-representable float64."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((n_hidden, n_in)) * np.sqrt(2.0 / n_in)
    W2 = rng.standard_normal((n_hidden, n_hidden)) * np.sqrt(2.0 / n_hidden)
    W3 = rng.standard_normal((n_out, n_hidden)) * (out_scale / np.sqrt(n_hidden))
    theta = np.concatenate([W1.ravel(), np.zeros(n_hidden), W2.ravel(), np.zeros(n_hidden),
                            W3.ravel(), np.zeros(n_out)])
    return f32_round(theta)
