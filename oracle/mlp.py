"""FP64 forward and backward of the kernel-surrogate network (test infrastructure only).

The network is not in the paper; it is the learned kernel generator this library adds.  Layers:
z_l = a_{l-1} W_l + b_l, a_l = SiLU(z_l) = z_l / (1 + exp(-z_l)) for hidden layers, output y = z_L.
Loss: L = (1/B) sum_b |y_b - t_b|^2 / |t_b|^2.  Gradients by the chain rule, written out.
"""
import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x):
    """params: list of (W [d_in][d_out], b [d_out]); returns (pre-activations, activations)."""
    pre, act = [], [np.asarray(x, dtype=np.float64)]
    for i, (w, b) in enumerate(params):
        z = act[-1] @ w + b
        pre.append(z)
        if i + 1 < len(params):
            act.append(silu(z))
    return pre, act


def loss(y, t):
    return float(np.mean(np.sum((y - t) ** 2, axis=1) / np.sum(t ** 2, axis=1)))


def loss_grad(y, t):
    return 2.0 * (y - t) / (y.shape[0] * np.sum(t ** 2, axis=1, keepdims=True))


def backward(params, x, t):
    """Gradients [(dW_l, db_l)] of the loss at x, t."""
    pre, act = forward(params, x)
    g = loss_grad(pre[-1], t)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        grads[l] = (act[l].T @ g, g.sum(axis=0))
        if l > 0:
            g = (g @ params[l][0].T) * silu_grad(pre[l - 1])
    return grads


def adam_step(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, bias-corrected moments); returns (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
