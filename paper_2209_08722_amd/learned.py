"""Learned warm start of the CG solve: binding of the ipm_mlp_* entry points, trajectory
collection from the plain IPM and the training loop (Adam over shuffled mini-batches).

Every forward, backward, optimiser and feature computation runs in the library's HIP kernels;
this module marshals arguments, gathers rows into batches and orders the calls.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

from . import native
from .native import IpmMlp

N_EXTRA = 18


def _torch():
    import torch
    return torch


def _p(t):
    return None if t is None else t.data_ptr()


class Mlp:
    """Network parameters, gradient and Adam moments (FP32, on the device)."""

    def __init__(self, n_in: int, n_hidden: int, n_out: int, theta, device: int = 0):
        torch = _torch()
        lib = native.load()
        self.n_in, self.n_hidden, self.n_out = int(n_in), int(n_hidden), int(n_out)
        count = lib.ipm_mlp_param_count(self.n_in, self.n_hidden, self.n_out)
        if count < 1:
            raise ValueError("bad network shape")
        theta = torch.as_tensor(theta, dtype=torch.float32).reshape(-1)
        if theta.numel() != count:
            raise ValueError(f"expected {count} parameters, got {theta.numel()}")
        dev = f"cuda:{device}"
        self.params = theta.to(dev).contiguous()
        self.grad = torch.zeros_like(self.params)
        self.m1 = torch.zeros_like(self.params)
        self.m2 = torch.zeros_like(self.params)
        self.t = 0

    @property
    def count(self) -> int:
        return self.params.numel()

    def c(self) -> IpmMlp:
        return IpmMlp(self.n_in, self.n_hidden, self.n_out, 0, self.params.data_ptr())


def ipm_mlp_features(ctx, dy_prev, x, s, k: int, kmax: int):
    torch = _torch()
    m = dy_prev.numel()
    feat = torch.empty(m + N_EXTRA, dtype=torch.float32, device=dy_prev.device)
    ctx.check(ctx.lib.ipm_mlp_features(ctx.h, m, x.numel(), _p(dy_prev), _p(x), _p(s), k, kmax, _p(feat)))
    return feat


def ipm_mlp_target(ctx, dy_prev, dy):
    torch = _torch()
    t = torch.empty(dy.numel(), dtype=torch.float32, device=dy.device)
    ctx.check(ctx.lib.ipm_mlp_target(ctx.h, dy.numel(), _p(dy_prev), _p(dy), _p(t)))
    return t


def ipm_mlp_forward(ctx, net: Mlp, X):
    torch = _torch()
    X = X.contiguous()
    Y = torch.empty((X.shape[0], net.n_out), dtype=torch.float32, device=X.device)
    c = net.c()
    ctx.check(ctx.lib.ipm_mlp_forward(ctx.h, ctypes.byref(c), X.shape[0], _p(X), _p(Y)))
    return Y


def ipm_mlp_backward(ctx, net: Mlp, X, T, want_loss: bool = True):
    """Gradient of the batch loss into net.grad; returns the loss (or None)."""
    c = net.c()
    loss = ctypes.c_double()
    ctx.check(ctx.lib.ipm_mlp_backward(ctx.h, ctypes.byref(c), X.shape[0], _p(X.contiguous()), _p(T.contiguous()),
                                       _p(net.grad), ctypes.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def ipm_mlp_adam(ctx, net: Mlp, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    net.t += 1
    ctx.check(ctx.lib.ipm_mlp_adam(ctx.h, net.count, _p(net.params), _p(net.grad), _p(net.m1), _p(net.m2), net.t,
                                   lr, beta1, beta2, eps))


def ipm_mlp_predict(ctx, net: Mlp, dy_prev, x, s, k: int, kmax: int):
    """The network's warm-start candidate ||dy_prev|| y (FP64, m)."""
    torch = _torch()
    dy0 = torch.empty(net.n_out, dtype=torch.float64, device=dy_prev.device)
    return mlp_predict_into(ctx, net, dy_prev, x, s, k, kmax, dy0)


def mlp_predict_into(ctx, net: Mlp, dy_prev, x, s, k: int, kmax: int, out):
    c = net.c()
    ctx.check(ctx.lib.ipm_mlp_predict(ctx.h, ctypes.byref(c), x.numel(), _p(dy_prev), _p(x), _p(s), k, kmax,
                                      _p(out)))
    return out


@dataclass
class Trajectories:
    X: object       # (N, m + 18) float32 features
    T: object       # (N, m) float32 targets: the part of dy_k that dy_{k-1} misses
    solves: int
    iterations: int      # IPM iterations
    cg_iterations: int   # CG iterations of those solves


def collect(ctx, problems, params, kmax: int = 200, maxit: int = 200) -> Trajectories:
    """Run the plain IPM (zero-start CG) on each problem; sample k >= 1 pairs the features at
    iteration k's start with the direction that iteration accepted."""
    from . import IPM_CONVERGED, State, ipm_last_dy, ipm_step
    torch = _torch()
    feats, targets, iters, cg = [], [], 0, 0
    for prob in problems:
        st = State.initial(prob.A.m, prob.A.n, prob.b.device.index or 0)
        prev = None
        for k in range(maxit + 1):
            f = ipm_mlp_features(ctx, prev, st.x, st.s, k, kmax) if prev is not None else None
            info = ipm_step(ctx, prob, st, params)
            if info["rc"] == IPM_CONVERGED:
                break
            cg += info["pcg_iters"]
            dy = ipm_last_dy(ctx, prob.A.m, prob.b.device.index or 0)
            if prev is not None:
                feats.append(f)
                targets.append(ipm_mlp_target(ctx, prev, dy))
            prev = dy
            iters += 1
    X = torch.stack(feats) if feats else None
    T = torch.stack(targets) if targets else None
    return Trajectories(X, T, len(problems), iters, cg)


def train(ctx, net: Mlp, X, T, epochs: int = 50, batch: int = 64, lr: float = 1e-3, seed: int = 0):
    """Adam over shuffled mini-batches; returns the full-data loss after each epoch."""
    torch = _torch()
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    n = X.shape[0]
    history = []
    for _ in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        for i in range(0, n, batch):
            idx = perm[i:i + batch]
            ipm_mlp_backward(ctx, net, X.index_select(0, idx), T.index_select(0, idx), want_loss=False)
            ipm_mlp_adam(ctx, net, lr)
        history.append(evaluate(ctx, net, X, T))
    return history


def evaluate(ctx, net: Mlp, X, T) -> float:
    """Mean loss over the rows of X (the gradient buffer is overwritten)."""
    total, n = 0.0, X.shape[0]
    for i in range(0, n, 4096):
        total += ipm_mlp_backward(ctx, net, X[i:i + 4096], T[i:i + 4096]) * min(4096, n - i)
    return total / n
