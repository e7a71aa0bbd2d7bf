"""Learned warm start of the CG solve (a further form of the method, not in the paper).

TEST INFRASTRUCTURE (oracle). Plain FP64 NumPy reference of what the HIP kernels compute.

At IPM iteration k >= 1 a small network maps the previous accepted direction dy_{k-1}, summary
statistics of log d^2 at the current iterate (d^2 = x / s, Section 1, eq. normal) and the
iteration index to a second candidate direction for the normal equations A D^2 A^T dy = p. The
CG solve starts from the combination of dy_{k-1} and that candidate closest to the solution in
the M-norm (oracle.ipm.pcg with two candidates), keeps its own stop test (eq. pdcond2, relative
to ||Q^{-1/2} p||) and falls back to the zero start when the combination's preconditioned
residual is not smaller, so the network changes iteration counts only.

Features (m + 18 entries):
    u = dy_{k-1} / ||dy_{k-1}||                                     (m)
    0.1 * log ||dy_{k-1}||
    0.1 * [mean, std, min, max] of l = log(x / s) over the n columns
    0.1 * 12 quantiles of l at levels i / 13 (i = 1..12), read from a 64-bin histogram of l on
          [min, max] with linear interpolation inside the bin
    k / kmax
Network (width H): h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3.
Candidate: ||dy_{k-1}|| * y (its scale does not matter to the combination).
Training target: the part of the new direction that dy_{k-1} misses,
    t_k = (dy_k - (u^T dy_k) u) / ||dy_{k-1}||;
if y points along t_k, the span of dy_{k-1} and y contains dy_k. Only the direction of y
matters: with the squared sine of the angle between output and target,
    e_b = 1 - (y_b^T t_b)^2 / (||y_b||^2 ||t_b||^2),
a warm start with relative error sqrt(e) saves about log(1 / e) / (2 log(1 / rho)) CG iterations
(rho the CG contraction factor), so the loss over a batch of B samples is the mean log error
    (1 / B) sum_b log(e_b + EPS),   EPS = 1e-10.
Optimiser: Adam (Kingma and Ba, 2015), bias-corrected moments.
Flat parameter layout: W1 [H x I] row-major, b1 [H], W2 [H x H], b2 [H], W3 [O x H], b3 [O]
with I = m + 18 inputs and O = m outputs.
"""
from __future__ import annotations

import numpy as np

N_EXTRA = 18
N_BINS = 64
LEVELS = np.arange(1, 13) / 13.0
STAT_SCALE = 0.1
EPS = 1e-10


def shapes(n_in: int, n_hidden: int, n_out: int):
    return [("W1", (n_hidden, n_in)), ("b1", (n_hidden,)), ("W2", (n_hidden, n_hidden)),
            ("b2", (n_hidden,)), ("W3", (n_out, n_hidden)), ("b3", (n_out,))]


def param_count(n_in: int, n_hidden: int, n_out: int) -> int:
    return sum(int(np.prod(s)) for _, s in shapes(n_in, n_hidden, n_out))


def unpack(theta: np.ndarray, n_in: int, n_hidden: int, n_out: int) -> dict:
    out, o = {}, 0
    for name, shp in shapes(n_in, n_hidden, n_out):
        k = int(np.prod(shp))
        out[name] = theta[o:o + k].reshape(shp)
        o += k
    return out


def pack(parts: dict, n_in: int, n_hidden: int, n_out: int) -> np.ndarray:
    return np.concatenate([parts[name].ravel() for name, _ in shapes(n_in, n_hidden, n_out)])


# ------------------------------------------------------------------ features

def hist_quantiles(l: np.ndarray, levels=LEVELS, nbins: int = N_BINS) -> np.ndarray:
    """Quantiles of l read from an nbins-bin histogram on [min, max], linear inside a bin.

    Bin of v: floor((v - lo) / (hi - lo) * nbins), clamped to nbins - 1. For level q the
    target count is q n; the first nonempty bin b whose cumulative count reaches it gives
    lo + (b + (q n - count below b) / count in b) * (hi - lo) / nbins.
    """
    lo, hi = float(l.min()), float(l.max())
    n = l.size
    if not hi > lo:
        return np.full(len(levels), lo)
    idx = np.floor((l - lo) / (hi - lo) * nbins).astype(np.int64)
    idx = np.minimum(idx, nbins - 1)
    counts = np.bincount(idx, minlength=nbins)
    width = (hi - lo) / nbins
    out = []
    for q in levels:
        target = q * n
        below = 0
        val = hi
        for b in range(nbins):
            c = counts[b]
            if c > 0 and below + c >= target:
                val = lo + (b + (target - below) / c) * width
                break
            below += c
        out.append(val)
    return np.array(out)


def features(dy_prev: np.ndarray, x: np.ndarray, s: np.ndarray, k: int, kmax: int) -> np.ndarray:
    """Feature vector (m + 18) of iteration k (see the module docstring)."""
    nrm = float(np.linalg.norm(dy_prev))
    u = dy_prev / nrm if nrm > 0 else np.zeros_like(dy_prev)
    l = np.log(x / s)
    mean = float(np.mean(l))
    std = float(np.sqrt(np.mean((l - mean) ** 2)))
    stats = [mean, std, float(l.min()), float(l.max())] + list(hist_quantiles(l))
    lognrm = np.log(nrm) if nrm > 0 else 0.0
    return np.concatenate([u, [STAT_SCALE * lognrm], STAT_SCALE * np.array(stats), [k / kmax]])


# ------------------------------------------------------------------ network

def forward(theta: np.ndarray, X: np.ndarray, n_hidden: int, n_out: int):
    """Outputs Y (B x O) for inputs X (B x I) and the activations the backward pass needs."""
    n_in = X.shape[1]
    P = unpack(theta, n_in, n_hidden, n_out)
    Z1 = X @ P["W1"].T + P["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ P["W2"].T + P["b2"]
    H2 = np.maximum(Z2, 0.0)
    Y = H2 @ P["W3"].T + P["b3"]
    return Y, dict(Z1=Z1, H1=H1, Z2=Z2, H2=H2)


def sin2(Y: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Per row, 1 - cos^2 of the angle between y and t."""
    a = np.sum(Y * T, axis=1)
    return 1.0 - a * a / (np.sum(Y * Y, axis=1) * np.sum(T * T, axis=1))


def loss(Y: np.ndarray, T: np.ndarray) -> float:
    """Mean over the batch of log(sin^2(angle(y, t)) + EPS)."""
    return float(np.mean(np.log(sin2(Y, T) + EPS)))


def backward(theta: np.ndarray, X: np.ndarray, T: np.ndarray, n_hidden: int, n_out: int):
    """(loss, gradient of the loss with respect to the flat parameters), by the chain rule."""
    n_in = X.shape[1]
    P = unpack(theta, n_in, n_hidden, n_out)
    Y, c = forward(theta, X, n_hidden, n_out)
    B = X.shape[0]
    # d/dy log(e + EPS) = (de/dy) / (e + EPS), e = 1 - a^2 / (yy tt), a = y^T t,
    # yy = ||y||^2, tt = ||t||^2: de/dy = 2 a / (yy tt) (a / yy y - t)
    a = np.sum(Y * T, axis=1)[:, None]
    yy = np.sum(Y * Y, axis=1)[:, None]
    tt = np.sum(T * T, axis=1)[:, None]
    e = 1.0 - a * a / (yy * tt)
    dY = (2.0 * a / (B * yy * tt * (e + EPS))) * (a / yy * Y - T)
    g = {"W3": dY.T @ c["H2"], "b3": dY.sum(axis=0)}
    dZ2 = (dY @ P["W3"]) * (c["Z2"] > 0)
    g["W2"] = dZ2.T @ c["H1"]
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ P["W2"]) * (c["Z1"] > 0)
    g["W1"] = dZ1.T @ X
    g["b1"] = dZ1.sum(axis=0)
    return loss(Y, T), pack(g, n_in, n_hidden, n_out)


def adam(theta, grad, m1, m2, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step (t >= 1); returns new (theta, m1, m2)."""
    m1 = beta1 * m1 + (1.0 - beta1) * grad
    m2 = beta2 * m2 + (1.0 - beta2) * grad * grad
    mhat = m1 / (1.0 - beta1 ** t)
    vhat = m2 / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m1, m2


def target(dy_prev: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """Training target of one sample: (dy - (u^T dy) u) / ||dy_prev||, u = dy_prev / ||dy_prev||."""
    nrm = float(np.linalg.norm(dy_prev))
    u = dy_prev / nrm
    return (dy - (u @ dy) * u) / nrm


def predict(theta: np.ndarray, dy_prev, x, s, k: int, kmax: int, n_hidden: int) -> np.ndarray:
    """Second warm-start candidate ||dy_{k-1}|| * y for iteration k."""
    f = features(dy_prev, x, s, k, kmax)
    Y, _ = forward(theta, f[None, :], n_hidden, dy_prev.size)
    return float(np.linalg.norm(dy_prev)) * Y[0]
