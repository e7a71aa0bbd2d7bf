"""Seeded LP generators that draw directly in device memory (torch on a ROCm device), for the
large workloads whose host generation would take minutes.

Same recipe as the host generators in ``lpgen`` (A, then x0 ~ U(0.5, 1.5)^n, b = A x0,
y0 ~ N(0, 1)^m, s0 ~ U(0.5, 1.5)^n, c = A^T y0 + s0), with torch's device generator seeded by
``seed``; the values therefore differ from the host generators' for the same seed. The stored
low-precision matrix defines the LP (b and c are computed from its values in FP64), and the FP64
copy holds the same values widened. No arithmetic of the interior point method is done here.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _torch():
    import torch
    return torch


@dataclass
class DeviceLP:
    A: object                 # (m, ld) storage dtype, row-major, columns >= n are zero
    n: int
    b: object                 # (m,) float64
    c: object                 # (n,) float64
    x0: object
    y0: object
    s0: object
    storage: str
    A64: object = None        # (m, ld64) float64 copy of the same values (plain form)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.A.shape[0]


_DT = {"f64": "float64", "f32": "float32", "bf16": "bfloat16"}


def _padded(m, n, dtype, device):
    torch = _torch()
    esz = torch.empty((), dtype=dtype).element_size()
    align = 128 // esz
    ld = ((n + align - 1) // align) * align
    return torch.zeros((m, ld), dtype=dtype, device=device)


def _finish(A_vals, storage, seed, device, widen, name):
    """A_vals: (m, n) float32/float64 device tensor holding the matrix before rounding."""
    torch = _torch()
    m, n = A_vals.shape
    dt = getattr(torch, _DT[storage])
    A = _padded(m, n, dt, device)
    A[:, :n] = A_vals.to(dt)
    del A_vals
    A64 = _padded(m, n, torch.float64, device)
    A64[:, :n] = A[:, :n].to(torch.float64)
    b, c, x0, y0, s0 = _rhs(A64, n, seed, device)
    lp = DeviceLP(A, n, b, c, x0, y0, s0, storage, A64 if widen else None, name)
    if not widen:
        del A64
    return lp


def _rhs(A64, n, seed, device):
    """The witness pair x0 ~ U(0.5, 1.5)^n, y0 ~ N(0, 1)^m, s0 ~ U(0.5, 1.5)^n (generator seeded
    by seed + 7919) and b = A x0, c = A^T y0 + s0 in FP64."""
    torch = _torch()
    m = A64.shape[0]
    g = torch.Generator(device=device)
    g.manual_seed(seed + 7919)
    x0 = torch.rand(n, generator=g, dtype=torch.float64, device=device) + 0.5
    y0 = torch.randn(m, generator=g, dtype=torch.float64, device=device)
    s0 = torch.rand(n, generator=g, dtype=torch.float64, device=device) + 0.5
    b = A64[:, :n] @ x0
    c = A64[:, :n].T @ y0 + s0
    return b, c, x0, y0, s0


def with_seed(lp: DeviceLP, seed: int) -> DeviceLP:
    """The LP of the same family with (b, c) from ``seed``: the same A (and FP64 copy, which must
    be present), a new witness pair. Equal to building the family member at ``seed`` with the
    same matrix seed, without drawing A again."""
    if lp.A64 is None:
        raise ValueError("with_seed needs the FP64 copy of A")
    b, c, x0, y0, s0 = _rhs(lp.A64, lp.n, seed, lp.A.device)
    return DeviceLP(lp.A, lp.n, b, c, x0, y0, s0, lp.storage, lp.A64, f"{lp.name}_rhs{seed}")


def dense_lp(m: int, n: int, seed: int = 0, storage: str = "bf16", device: str = "cuda:0",
             widen: bool = True, matrix_seed=None) -> DeviceLP:
    """A i.i.d. N(0, 1) rounded to ``storage`` (round to nearest even), drawn from ``matrix_seed``
    (default: ``seed``); (b, c) from ``seed``."""
    torch = _torch()
    g = torch.Generator(device=device)
    g.manual_seed(seed if matrix_seed is None else matrix_seed)
    A = torch.randn((m, n), generator=g, dtype=torch.float32, device=device)
    return _finish(A, storage, seed, device, widen, f"dense{m}x{n}{storage}s{seed}")


_ILLCOND_CACHE = {}


def illcond_matrix(m: int, n: int, matrix_seed: int = 1000, cond: float = 1e4, device: str = "cuda:0"):
    """U diag(sigma) V^T (FP64): U Haar (QR of a Gaussian, signs fixed by diag(R) > 0), V with
    Haar-distributed orthonormal columns (V = H R^-1, R the Cholesky factor of H^T H with a
    positive diagonal, i.e. the QR of the Gaussian H), sigma log-spaced from 1 to cond."""
    key = (m, n, matrix_seed, cond, device)
    if key in _ILLCOND_CACHE:
        return _ILLCOND_CACHE[key]
    torch = _torch()
    g = torch.Generator(device=device)
    g.manual_seed(matrix_seed)
    G = torch.randn((m, m), generator=g, dtype=torch.float64, device=device)
    U, R = torch.linalg.qr(G)
    U = U * torch.sign(torch.diagonal(R))
    del G, R
    H = torch.randn((n, m), generator=g, dtype=torch.float64, device=device)
    Rc = torch.linalg.cholesky(H.T @ H, upper=True)
    # R is m x m and well conditioned (H is a tall Gaussian): V = H R^-1 as a product
    Rinv = torch.linalg.solve_triangular(Rc, torch.eye(m, dtype=torch.float64, device=device), upper=True)
    V = H @ Rinv
    del H, Rc, Rinv
    sig = torch.logspace(0.0, float(np.log10(cond)), m, dtype=torch.float64, device=device)
    A = (U * sig) @ V.T
    del V, U
    _ILLCOND_CACHE.clear()
    _ILLCOND_CACHE[key] = A
    return A


def illcond_lp(m: int, n: int, seed: int = 0, matrix_seed: int = 1000, cond: float = 1e4,
               storage: str = "f32", device: str = "cuda:0", widen: bool = True) -> DeviceLP:
    """One fixed ill-conditioned A (from ``matrix_seed``) with (b, c) drawn from ``seed``."""
    A = illcond_matrix(m, n, matrix_seed, cond, device)
    return _finish(A.clone(), storage, seed, device, widen, f"illcond{m}x{n}{storage}s{seed}")
