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


# Adam (Kingma & Ba 2015): with bias-corrected moments m_k/(1-b1^k) and v_k/(1-b2^k), a gradient that
# stays constant from zero moments gives m_hat = g and v_hat = g^2 exactly, so every step moves a
# weight by lr g / (|g| + eps).  A wrong bias correction (missing, or with the step count frozen) scales
# the step by (1 - b1^k)/sqrt(1 - b2^k) or its inverse; eps under the square root gives
# lr g / sqrt(g^2 + eps), visibly different at |g| ~ sqrt(eps); swapped decay rates change m and v.

def test_adam_first_step_from_zero_moments_is_lr_g_over_abs_g_plus_eps():
    g = np.array([3.0, -0.5, 1e-4, -2e-4, 0.0])
    w0 = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    w1, m1, v1 = mlp.adam_step(w0, g, np.zeros(5), np.zeros(5), 1, lr=0.01)
    np.testing.assert_allclose(w1, w0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15, atol=0)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-15, atol=0)


def test_adam_constant_gradient_moves_every_step_by_the_same_amount():
    g = np.array([0.7, -1.3, 1e-4, -3e-4])
    lr, b1, b2, eps = 0.003, 0.9, 0.999, 1e-8
    w = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    for k in range(1, 26):
        w, m, v = mlp.adam_step(w, g, m, v, k, lr=lr, b1=b1, b2=b2, eps=eps)
        # moments are exponential averages of a constant: (1 - b^k) g and (1 - b^k) g^2
        np.testing.assert_allclose(m, (1 - b1 ** k) * g, rtol=1e-13)
        np.testing.assert_allclose(v, (1 - b2 ** k) * g * g, rtol=1e-12)
        np.testing.assert_allclose(w, -k * lr * g / (np.abs(g) + eps), rtol=1e-12)
    # eps under the square root would have moved the small weights by about 30 % less
    assert abs(w[2]) > 1.3 * 25 * lr * 1e-4 / np.sqrt(1e-8 + 1e-8)


def test_adam_alternating_gradient_closed_form():
    # g_k = (-1)^(k+1) g: m_k = (1 - b1) sum_j b1^(k-j) g_j = (-1)^(k+1) (1 - b1) g (1 - (-b1)^k) / (1 + b1)
    # and v_k = (1 - b2^k) g^2, so the k-th step is lr (m_k / (1 - b1^k)) / (g + eps)
    g = 0.25
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    w, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    for k in range(1, 8):
        gk = g if k % 2 else -g
        w_prev = w.copy()
        w, m, v = mlp.adam_step(w, np.array([gk]), m, v, k, lr=lr, b1=b1, b2=b2, eps=eps)
        mk = (-1) ** (k + 1) * (1 - b1) * g * (1 - (-b1) ** k) / (1 + b1)
        np.testing.assert_allclose(m, mk, rtol=1e-13)
        m_hat = mk / (1 - b1 ** k)
        np.testing.assert_allclose(w_prev - w, lr * m_hat / (g + eps), rtol=1e-12)
