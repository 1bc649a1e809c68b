"""Checkpoints on the device: kernel sets and surrogate networks saved to safetensors files and
restored.  A restored kernel set has the identical table and grids bit-identically (reproducible
gridding mode); a restored network has the identical weights, Adam moments and step, and training
resumed from the file follows the run that never stopped."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pg = pytest.importorskip("paper_2206_15117_amd.polgrid")
from paper_2206_15117_amd import checkpoint  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("storage", [pg.STORE_F32, pg.STORE_F16])
def test_kernel_set_round_trip(tmp_path, storage):
    w = synth.scaled_config2(5000, n=256, nplanes=8, mk=64, support=[16, 12, 10, 8, 8, 10, 12, 16])
    jones = synth.jones_on_lattice(w.beam, w.geom.mk, w.geom.fov)
    k = pg.make_kernels(w.geom, 4, pg.KIND_GRID, jones=jones, eps_null=w.eps_null, storage=storage)
    path = str(tmp_path / "kernels.safetensors")
    checkpoint.save_kernels(k, path)
    k2 = checkpoint.load_kernels(path)
    assert (k2.npol, k2.kind, k2.storage, k2.os, k2.n, k2.nplanes) == (k.npol, k.kind, k.storage, k.os, k.n, k.nplanes)
    assert np.array_equal(k2.plane_offset, k.plane_offset)
    assert np.array_equal(k2.aa_pixels, k.aa_pixels)
    a, b = k.table(), k2.table()
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.uint8) if a.dtype != torch.complex64 else torch.view_as_real(a),
                       b.view(torch.uint8) if b.dtype != torch.complex64 else torch.view_as_real(b))
    vis = dev(synth.random_vis(w.nvis, 4, np.random.default_rng(3)))
    g1 = pg.grid(pg.plan(k, dev(w.uvw), max_chunk=200), k, vis, deterministic=True)
    g2 = pg.grid(pg.plan(k2, dev(w.uvw), max_chunk=200), k2, vis, deterministic=True)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(g1), torch.view_as_real(g2))


def _batches(n_in, n_out, steps, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return [(torch.randn((64, n_in), device="cuda", generator=g), torch.randn((64, n_out), device="cuda", generator=g))
            for _ in range(steps)]


def test_network_round_trip_and_resume(tmp_path):
    n_in, n_out = 24, 300
    net = pg.MLP(n_in, 64, 3, n_out, 64, seed=5)
    first, second = _batches(n_in, n_out, 4, 1), _batches(n_in, n_out, 4, 2)
    for x, t in first:
        net.train_step(x, t, 1e-3)
    path = str(tmp_path / "net.safetensors")
    scale = np.linspace(0.5, 2.0, 16)
    checkpoint.save_network(net, path, extra={"cell_scale": scale, "note": "test"})
    net2, extra = checkpoint.load_network(path)
    assert np.allclose(extra["cell_scale"], scale) and extra["note"] == "test"
    assert net2.dims == net.dims and net2.step == net.step == 4
    for layer in range(4):
        for what in (pg.MLP_W, pg.MLP_W_BF16, pg.MLP_B, pg.MLP_MW, pg.MLP_VW, pg.MLP_MB, pg.MLP_VB):
            assert torch.equal(net.copy(what, layer), net2.copy(what, layer)), (layer, what)
    x0 = first[0][0]
    assert torch.equal(net.forward(x0), net2.forward(x0))
    for x, t in second:
        net.train_step(x, t, 1e-3)
        net2.train_step(x, t, 1e-3)
    torch.cuda.synchronize()
    assert net2.step == net.step == 8
    for layer in range(4):
        a, b = net.copy(pg.MLP_W, layer), net2.copy(pg.MLP_W, layer)
        assert float((a - b).norm() / a.norm()) < 1e-6, layer


def test_weights_only_checkpoint_starts_a_fresh_optimiser(tmp_path):
    net = pg.MLP(8, 32, 2, 40, 32, seed=2)
    for x, t in _batches(8, 40, 3, 4)[:3]:
        net.train_step(x[:32], t[:32], 1e-3)
    path = str(tmp_path / "w.safetensors")
    checkpoint.save_network(net, path, training_state=False)
    net2, _ = checkpoint.load_network(path, max_batch=16)
    assert net2.step == 0 and net2.max_batch == 16
    assert torch.equal(net.copy(pg.MLP_W, 2), net2.copy(pg.MLP_W, 2))
    assert float(net2.copy(pg.MLP_MW, 0).abs().max()) == 0.0


def test_set_rejects_bad_arguments():
    net = pg.MLP(8, 32, 2, 40, 32, seed=2)
    with pytest.raises(ValueError):
        net.set(pg.MLP_W, 0, torch.zeros((32, 8), device="cuda"))
    with pytest.raises(pg.PolgridError):
        pg._check(pg.lib().pg_mlp_set(net._h, pg.MLP_GW, 0, torch.zeros(8 * 32, device="cuda").data_ptr(), None))
    with pytest.raises(pg.PolgridError):
        net.step = -1
