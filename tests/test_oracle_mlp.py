"""Pins of the warm-start network's FP64 oracle (CPU only): library routines on the same
network (torch.nn and torch.optim in float64), central finite differences, closed forms of
the histogram quantiles and special cases of the features."""
import numpy as np
import pytest

import lpgen
from oracle import mlp

torch = pytest.importorskip("torch")


def _net(n_in, H, n_out, seed):
    theta = lpgen.mlp_init(n_in, H, n_out, seed, out_scale=0.5)
    rng = np.random.default_rng(seed + 1)
    theta = theta + 0.05 * rng.standard_normal(theta.size)   # nonzero biases too
    return theta


def _torch_model(theta, n_in, H, n_out):
    P = mlp.unpack(theta, n_in, H, n_out)
    lin = [torch.nn.Linear(n_in, H), torch.nn.Linear(H, H), torch.nn.Linear(H, n_out)]
    for layer, (w, b) in zip(lin, (("W1", "b1"), ("W2", "b2"), ("W3", "b3"))):
        layer.double()
        with torch.no_grad():
            layer.weight.copy_(torch.from_numpy(P[w]))
            layer.bias.copy_(torch.from_numpy(P[b]))
    return lin


def _torch_loss(lin, X, T, n_out):
    h = torch.relu(lin[0](X))
    h = torch.relu(lin[1](h))
    y = lin[2](h)
    # the loss as a minimisation over the scale, solved by torch's least squares
    beta = torch.linalg.lstsq(y[:, :, None], T[:, :, None]).solution[:, 0, 0]
    e = ((beta[:, None] * y - T) ** 2).sum(1) / (T * T).sum(1)
    return torch.log(e + mlp.EPS).mean(), y


@pytest.mark.parametrize("n_out,H,B", [(5, 7, 3), (30, 16, 8), (50, 64, 1)])
def test_forward_backward_match_torch(n_out, H, B):
    n_in = n_out + mlp.N_EXTRA
    theta = _net(n_in, H, n_out, n_out)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((B, n_in))
    T = rng.standard_normal((B, n_out))
    lin = _torch_model(theta, n_in, H, n_out)
    Xt, Tt = torch.from_numpy(X), torch.from_numpy(T)
    lt, yt = _torch_loss(lin, Xt, Tt, n_out)
    lt.backward()
    Y, _ = mlp.forward(theta, X, H, n_out)
    assert np.allclose(Y, yt.detach().numpy(), rtol=1e-13, atol=1e-13)
    lo, g = mlp.backward(theta, X, T, H, n_out)
    assert lo == pytest.approx(lt.item(), rel=1e-13)
    gt = {"W1": lin[0].weight.grad, "b1": lin[0].bias.grad, "W2": lin[1].weight.grad,
          "b2": lin[1].bias.grad, "W3": lin[2].weight.grad, "b3": lin[2].bias.grad}
    ref = mlp.pack({k: v.numpy() for k, v in gt.items()}, n_in, H, n_out)
    assert np.allclose(g, ref, rtol=1e-12, atol=1e-14)


def test_backward_matches_central_differences():
    n_out, H, B = 6, 9, 4
    n_in = n_out + mlp.N_EXTRA
    theta = _net(n_in, H, n_out, 11)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((B, n_in))
    T = rng.standard_normal((B, n_out))
    _, g = mlp.backward(theta, X, T, H, n_out)
    h = 1e-6
    num = np.empty_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        num[i] = (mlp.loss(mlp.forward(theta + e, X, H, n_out)[0], T)
                  - mlp.loss(mlp.forward(theta - e, X, H, n_out)[0], T)) / (2 * h)
    assert np.linalg.norm(g - num) <= 1e-6 * np.linalg.norm(num)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(40)
    p = torch.nn.Parameter(torch.from_numpy(theta.copy()))
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m1 = np.zeros_like(theta)
    m2 = np.zeros_like(theta)
    for t in range(1, 8):
        g = rng.standard_normal(40) * (10.0 ** rng.uniform(-4, 1, 40))
        p.grad = torch.from_numpy(g.copy())
        opt.step()
        theta, m1, m2 = mlp.adam(theta, g, m1, m2, t, lr=1e-2)
        assert np.allclose(theta, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_histogram_quantiles_on_a_uniform_grid():
    """Evenly spaced data: the histogram quantile is exact up to the data spacing."""
    l = np.linspace(-7.0, 11.0, 64001)
    q = mlp.hist_quantiles(l)
    ref = np.quantile(l, mlp.LEVELS)
    assert np.max(np.abs(q - ref)) <= 2 * 18.0 / 64000


@pytest.mark.parametrize("dist", ["normal", "lognormal", "bimodal"])
def test_histogram_quantiles_within_one_bin(dist):
    """For any data the histogram quantile lies in the bin of the exact quantile (or the
    adjacent one when the quantile falls on a bin edge), so the error is at most one bin width."""
    rng = np.random.default_rng(6)
    l = {"normal": rng.standard_normal(5000), "lognormal": np.exp(rng.standard_normal(5000)),
         "bimodal": np.concatenate([rng.normal(-20, 1, 3000), rng.normal(15, 3, 2000)])}[dist]
    q = mlp.hist_quantiles(l)
    ref = np.quantile(l, mlp.LEVELS)
    width = (l.max() - l.min()) / mlp.N_BINS
    assert np.all(np.abs(q - ref) <= width * (1 + 1e-9))
    assert np.all(np.diff(q) >= 0)


def test_histogram_quantiles_constant_data():
    assert np.all(mlp.hist_quantiles(np.full(10, 2.5)) == 2.5)


def test_features_layout_and_statistics():
    rng = np.random.default_rng(7)
    m, n = 9, 500
    dy = rng.standard_normal(m) * 3.0
    x = rng.uniform(0.1, 5, n)
    s = rng.uniform(0.1, 5, n)
    f = mlp.features(dy, x, s, k=7, kmax=200)
    assert f.size == m + mlp.N_EXTRA
    assert np.linalg.norm(f[:m]) == pytest.approx(1.0)
    assert np.allclose(f[:m] * np.linalg.norm(dy), dy)
    assert f[m] == pytest.approx(0.1 * np.log(np.linalg.norm(dy)))
    l = np.log(x) - np.log(s)
    st = 0.1 * np.array([np.mean(l), np.std(l), l.min(), l.max()])
    assert np.allclose(f[m + 1:m + 5], st, rtol=1e-12)
    assert np.all(np.diff(f[m + 5:m + 17]) >= 0)
    assert f[m + 3] <= f[m + 5] and f[m + 16] <= f[m + 4]
    assert f[-1] == 7 / 200


def test_target_completes_the_previous_direction():
    """The target is orthogonal to the previous direction, and the previous direction and the
    target span the new direction (least squares over the pair leaves no residual)."""
    rng = np.random.default_rng(8)
    prev, dy = rng.standard_normal(12), rng.standard_normal(12)
    t = mlp.target(prev, dy)
    assert abs(t @ prev) <= 1e-13 * np.linalg.norm(t) * np.linalg.norm(prev)
    V = np.stack([prev, t], axis=1)
    c, *_ = np.linalg.lstsq(V, dy, rcond=None)
    assert np.linalg.norm(V @ c - dy) <= 1e-12 * np.linalg.norm(dy)
