"""Pins of the FP64 network oracle: analytic gradients against central finite differences."""
import numpy as np

from oracle import mlp


def _net(rng, dims):
    return [(rng.standard_normal((a, b)) / np.sqrt(a), rng.standard_normal(b) * 0.1) for a, b in zip(dims, dims[1:])]


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(5)
    params = _net(rng, [5, 7, 6, 9])
    x = rng.standard_normal((4, 5))
    t = rng.standard_normal((4, 9))
    grads = mlp.backward(params, x, t)
    h = 1e-6
    for l, (w, b) in enumerate(params):
        for arr, g in ((w, grads[l][0]), (b, grads[l][1])):
            for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]:
                old = arr[idx]
                arr[idx] = old + h
                lp = mlp.loss(mlp.forward(params, x)[0][-1], t)
                arr[idx] = old - h
                lm = mlp.loss(mlp.forward(params, x)[0][-1], t)
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(fd)), (l, idx, fd, g[idx])


def test_silu_grad_is_the_derivative():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.silu_grad(z))) < 1e-8


def test_loss_is_zero_at_target_and_scale_free():
    rng = np.random.default_rng(6)
    t = rng.standard_normal((3, 10))
    assert mlp.loss(t, t) == 0.0
    y = t + rng.standard_normal((3, 10))
    assert abs(mlp.loss(10 * y, 10 * t) - mlp.loss(y, t)) < 1e-12
