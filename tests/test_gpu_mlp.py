"""The surrogate network's HIP kernels against the FP64 oracle, layer by layer, fed with the GPU's
own bfloat16 operands (so the float32 accumulations are what is compared)."""
import numpy as np
import pytest

from oracle import mlp as omlp

torch = pytest.importorskip("torch")
pg = pytest.importorskip("paper_2206_15117_amd.polgrid")

pytestmark = pytest.mark.gpu


def f64(t):
    torch.cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_forward_layer_by_layer():
    net = pg.MLP(20, 64, 2, 300, max_batch=64, seed=11)
    gen = torch.Generator(device="cuda").manual_seed(1)
    x = torch.randn((37, 20), device="cuda", generator=gen)  # ragged against the 64-row tiles
    y = net.forward(x)   # the output layer writes y directly
    for l in range(3):
        a = f64(net.copy(pg.MLP_ACT, l, 37))
        w = f64(net.copy(pg.MLP_W_BF16, l))
        b = f64(net.copy(pg.MLP_B, l))
        z = f64(y) if l == 2 else f64(net.copy(pg.MLP_PRE, l, 37))
        assert rel(z, a @ w + b) < 1e-5, l
        if l < 2:  # next layer's input is SiLU of this pre-activation rounded to bfloat16
            nxt = f64(net.copy(pg.MLP_ACT, l + 1, 37))
            assert np.max(np.abs(nxt - omlp.silu(z))) <= 2 ** -8 * np.max(np.abs(omlp.silu(z))) + 1e-6
    # a training step's own forward leaves the output in the network's buffer: the same bits
    net.train_step(x, torch.zeros_like(y), lr=0.0, update=False)
    assert rel(f64(y), f64(net.copy(pg.MLP_PRE, 2, 37))) == 0.0


def test_backward_layer_by_layer_with_split_k():
    net = pg.MLP(20, 48, 1, 20000, max_batch=16, seed=12)  # wide output: split-K input gradient
    gen = torch.Generator(device="cuda").manual_seed(2)
    x = torch.randn((16, 20), device="cuda", generator=gen)
    t = torch.randn((16, 20000), device="cuda", generator=gen)
    loss = net.train_step(x, t, lr=0.0, update=False)
    y = f64(net.copy(pg.MLP_PRE, 1, 16))
    tt = f64(t)
    assert abs(float(loss.item()) - omlp.loss(y, tt)) < 1e-5 * omlp.loss(y, tt)
    gy = f64(net.copy(pg.MLP_GY, 0, 16))
    assert rel(gy, omlp.loss_grad(y, tt)) < 1e-5
    gyb = f64(net.copy(pg.MLP_GY_BF16, 0, 16))
    a1 = f64(net.copy(pg.MLP_ACT, 1, 16))
    assert rel(f64(net.copy(pg.MLP_GW, 1)), a1.T @ gyb) < 1e-5
    assert rel(f64(net.copy(pg.MLP_GB, 1)), gy.sum(axis=0)) < 1e-5
    w1 = f64(net.copy(pg.MLP_W_BF16, 1))
    z0 = f64(net.copy(pg.MLP_PRE, 0, 16))
    gz = f64(net.copy(pg.MLP_GZ, 0, 16))
    assert rel(gz, (gyb @ w1.T) * omlp.silu_grad(z0)) < 1e-5
    gzb = f64(net.copy(pg.MLP_GZ_BF16, 0, 16))
    x0 = f64(net.copy(pg.MLP_ACT, 0, 16))
    assert rel(f64(net.copy(pg.MLP_GW, 0)), x0.T @ gzb) < 1e-5
    assert rel(f64(net.copy(pg.MLP_GB, 0)), gz.sum(axis=0)) < 1e-5


def test_full_backward_close_to_fp64_oracle():
    """All layers against exact FP64 backprop of the same bfloat16 weights; the GPU rounds
    intermediate gradients to bfloat16 for its products, hence the 2e-2 bound."""
    net = pg.MLP(20, 32, 3, 500, max_batch=24, seed=13)
    gen = torch.Generator(device="cuda").manual_seed(3)
    x = torch.randn((24, 20), device="cuda", generator=gen)
    t = torch.randn((24, 500), device="cuda", generator=gen)
    net.train_step(x, t, lr=0.0, update=False)
    params = [(f64(net.copy(pg.MLP_W_BF16, l)), f64(net.copy(pg.MLP_B, l))) for l in range(4)]
    grads = omlp.backward(params, f64(net.copy(pg.MLP_ACT, 0, 24)), f64(t))
    for l in range(4):
        assert rel(f64(net.copy(pg.MLP_GW, l)), grads[l][0]) < 2e-2, l
        assert rel(f64(net.copy(pg.MLP_GB, l)), grads[l][1]) < 2e-2, l


def test_adam_update_matches_oracle():
    net = pg.MLP(8, 16, 1, 40, max_batch=8, seed=14)
    gen = torch.Generator(device="cuda").manual_seed(4)
    x = torch.randn((8, 8), device="cuda", generator=gen)
    t = torch.randn((8, 40), device="cuda", generator=gen)
    w0 = f64(net.copy(pg.MLP_W, 1))
    net.train_step(x, t, lr=0.0, update=False)
    g = f64(net.copy(pg.MLP_GW, 1))
    net.train_step(x, t, lr=1e-2, update=True)  # same gradient (weights unchanged by the first call)
    want, _, _ = omlp.adam_step(w0, g, np.zeros_like(g), np.zeros_like(g), 1, 1e-2)
    assert np.max(np.abs(f64(net.copy(pg.MLP_W, 1)) - want)) < 1e-6


def test_adam_three_steps_with_moments_match_oracle():
    """Steps 1-3 from zero moments, each with that step's gradient: weights and both moments follow
    the oracle's Adam (bias corrections and decay rates act once the moments are non-zero)."""
    net = pg.MLP(8, 16, 1, 40, max_batch=8, seed=16)
    gen = torch.Generator(device="cuda").manual_seed(6)
    x = torch.randn((8, 8), device="cuda", generator=gen)
    t = torch.randn((8, 40), device="cuda", generator=gen)
    w = f64(net.copy(pg.MLP_W, 1))
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for step in range(1, 4):
        net.train_step(x, t, lr=1e-2, update=True)
        g = f64(net.copy(pg.MLP_GW, 1))  # the gradient this step's update used
        w, m, v = omlp.adam_step(w, g, m, v, step, 1e-2)
        assert np.max(np.abs(f64(net.copy(pg.MLP_MW, 1)) - m)) <= 1e-6 * max(np.max(np.abs(m)), 1e-30), step
        assert np.max(np.abs(f64(net.copy(pg.MLP_VW, 1)) - v)) <= 1e-5 * max(np.max(np.abs(v)), 1e-30), step
        assert np.max(np.abs(f64(net.copy(pg.MLP_W, 1)) - w)) < 1e-6, step
        # continue from the device's state so float32 rounding does not accumulate across steps
        w, m, v = f64(net.copy(pg.MLP_W, 1)), f64(net.copy(pg.MLP_MW, 1)), f64(net.copy(pg.MLP_VW, 1))


def test_training_reduces_loss():
    net = pg.MLP(20, 64, 3, 2048, max_batch=64, seed=15)
    gen = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randn((64, 20), device="cuda", generator=gen)
    basis = torch.randn((20, 2048), device="cuda", generator=gen)
    t = torch.tanh(x @ basis / 4)
    first = float(net.train_step(x, t, lr=3e-3).item())
    for _ in range(300):
        last = float(net.train_step(x, t, lr=3e-3).item())
    assert last < 0.2 * first, (first, last)
