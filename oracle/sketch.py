"""Sparse embedding W and the sketch B = A D W (oracle; test infrastructure only).

Section 2 of the paper uses a sparse embedding W in R^{n x w} with a small
number of signed nonzeros per row; Algorithm 1 (step 1) forms A D W. The
paper fixes neither the bucket rule, the scaling nor the random source, so
this reading is used (the GPU library implements the same definition
independently):

* Each row j of W has exactly ``s`` nonzeros, one in each of ``s`` disjoint
  bucket blocks of width ``w / s`` (so they are distinct); ``s`` must divide
  ``w``.
* Copy r of row j sits in bucket ``r*(w/s) + floor(hi32(h) * (w/s) / 2^32)``
  with value ``+1/sqrt(s)`` if bit 0 of h is 0, else ``-1/sqrt(s)``.
  Every row then has unit norm, so E[W W^T] = I.
* h is the j-th output of a SplitMix64 stream (Steele, Lea, Flood 2014)
  whose start state is ``K[k, r] = mix64((seed ^ mix64(k)) + (r+1)*phi)``:
  ``h = mix64(K[k, r] + (j+1)*phi)``, with phi = 0x9E3779B97F4A7C15 and mix64
  the SplitMix64 output function. j is 0-based, k is the IPM iteration, so W
  is redrawn every iteration (Algorithm 3, step 2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

MASK64 = (1 << 64) - 1
PHI = 0x9E3779B97F4A7C15


def mix64_int(z: int) -> int:
    """SplitMix64 output function on a Python int (mod 2^64)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrap-around arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def splitmix64_stream(state: int, count: int) -> list:
    """First ``count`` outputs of SplitMix64 started at ``state``."""
    out = []
    for _ in range(count):
        state = (state + PHI) & MASK64
        out.append(mix64_int(state))
    return out


def stream_keys(seed: int, k: int, s: int) -> list:
    """Per-copy stream start states K[k, r], r = 0..s-1."""
    base = (seed ^ mix64_int(k)) & MASK64
    return [mix64_int((base + (r + 1) * PHI) & MASK64) for r in range(s)]


def buckets_signs(n: int, w: int, s: int, seed: int, k: int):
    """Bucket index (n, s) int64 and sign (n, s) float64 (+-1) of every nonzero of W."""
    if w % s != 0:
        raise ValueError("s must divide w")
    blk = w // s
    keys = stream_keys(seed, k, s)
    j = np.arange(n, dtype=np.uint64)
    bucket = np.empty((n, s), dtype=np.int64)
    sign = np.empty((n, s), dtype=np.float64)
    with np.errstate(over="ignore"):
        jphi = (j + np.uint64(1)) * np.uint64(PHI)
        for r in range(s):
            h = mix64(np.uint64(keys[r]) + jphi)
            hi = h >> np.uint64(32)
            bucket[:, r] = r * blk + ((hi * np.uint64(blk)) >> np.uint64(32)).astype(np.int64)
            sign[:, r] = np.where((h & np.uint64(1)) == 0, 1.0, -1.0)
    return bucket, sign


def sketch_matrix(n: int, w: int, s: int, seed: int, k: int) -> sp.csr_matrix:
    """W as a sparse n x w matrix with entries +-1/sqrt(s)."""
    bucket, sign = buckets_signs(n, w, s, seed, k)
    rows = np.repeat(np.arange(n), s)
    vals = (sign / np.sqrt(s)).ravel()
    return sp.csr_matrix((vals, (rows, bucket.ravel())), shape=(n, w))


def sketch_ADW(A: np.ndarray, d: np.ndarray, w: int, s: int, seed: int, k: int) -> np.ndarray:
    """B = A diag(d) W (Algorithm 1, step 1; eqn. pdprecond builds Q = B B^T).

    A library sparse product serves as the step: (A diag(d)) times the sparse W.
    """
    W = sketch_matrix(A.shape[1], w, s, seed, k)
    if sp.issparse(A):
        return np.asarray((W.T @ A.multiply(d[None, :]).tocsr().T).T.toarray())
    return np.asarray((W.T @ (A * d).T).T)


# ---------------------------------------------------------------- Gaussian sketch

# A Gaussian sketching matrix is the paper's experimental choice (Section 7; Section 6 notes
# that it gives the same accuracy guarantees at a higher cost of forming A D W). Reading: W has
# i.i.d. N(0, 1/w) entries, so E[W W^T] = I like the sparse embedding. Entry (j, c) (0-based,
# row-major index e = j w + c) takes outputs 2e and 2e+1 of the SplitMix64 stream started at
# K = mix64((seed ^ mix64(k)) + GAUSS_DOMAIN) and turns them into one normal deviate with the
# Box-Muller transform (Box and Muller, 1958):
#     u1 = ((h1 >> 11) + 1) 2^-53 in (0, 1],  u2 = (h2 >> 11) 2^-53 in [0, 1),
#     z  = sqrt(-2 ln u1) cos(2 pi u2),       W[j, c] = z / sqrt(w).
# The GPU library implements the same definition with its own code.
GAUSS_DOMAIN = 0xD1B54A32D192ED03


def gaussian_key(seed: int, k: int) -> int:
    """Stream start state of the Gaussian sketch of IPM iteration k."""
    return mix64_int(((seed ^ mix64_int(k)) + GAUSS_DOMAIN) & MASK64)


def gaussian_rows(j0: int, j1: int, w: int, seed: int, k: int) -> np.ndarray:
    """Rows j0..j1-1 of the Gaussian W (dense (j1 - j0) x w, FP64)."""
    key = np.uint64(gaussian_key(seed, k))
    e = (np.arange(j0, j1, dtype=np.uint64)[:, None] * np.uint64(w)
         + np.arange(w, dtype=np.uint64)[None, :])
    with np.errstate(over="ignore"):
        h1 = mix64(key + (np.uint64(2) * e + np.uint64(1)) * np.uint64(PHI))
        h2 = mix64(key + (np.uint64(2) * e + np.uint64(2)) * np.uint64(PHI))
    u1 = ((h1 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (h2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return z / np.sqrt(w)


def sketch_gaussian(A, d: np.ndarray, w: int, seed: int, k: int, chunk: int = 2048) -> np.ndarray:
    """B = A diag(d) W for the Gaussian W of iteration k (m x w, FP64), W formed by row chunks."""
    m, n = A.shape
    B = np.zeros((m, w))
    for j0 in range(0, n, chunk):
        j1 = min(n, j0 + chunk)
        Ad = A[:, j0:j1] @ sp.diags(d[j0:j1]) if sp.issparse(A) else A[:, j0:j1] * d[j0:j1]
        B += np.asarray(Ad @ gaussian_rows(j0, j1, w, seed, k))
    return B


def gaussian_apply(u: np.ndarray, n: int, w: int, seed: int, k: int, chunk: int = 2048) -> np.ndarray:
    """W u for the Gaussian W of iteration k (n-vector)."""
    out = np.empty(n)
    for j0 in range(0, n, chunk):
        j1 = min(n, j0 + chunk)
        out[j0:j1] = gaussian_rows(j0, j1, w, seed, k) @ u
    return out
