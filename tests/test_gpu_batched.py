"""The batched launch against the oracle, per field, plus HIP-graph replay."""
import numpy as np
import pytest

import synth
from oracle import gridding, kernels, mueller

torch = pytest.importorskip("torch")
pg = pytest.importorskip("paper_2206_15117_amd.polgrid")

pytestmark = pytest.mark.gpu
TOL = 1e-5


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _fields(storage=pg.STORE_F32):
    specs = [dict(nvis=3000, n=128, nplanes=4, support=[12, 8, 8, 12], seed=1),
             dict(nvis=12000, n=256, nplanes=8, support=[16, 12, 10, 8, 8, 10, 12, 16], seed=2),
             dict(nvis=500, n=128, nplanes=3, support=[10, 8, 10], seed=3)]
    out = []
    for sp in specs:
        w = synth.scaled_config2(sp["nvis"], n=sp["n"], nplanes=sp["nplanes"], mk=32,
                                 support=sp["support"], seed=synth.SEED_BASE + 20 + sp["seed"])
        g = w.geom
        jones = synth.jones_on_lattice(w.beam, g.mk, g.fov)
        kg = pg.make_kernels(g, 4, pg.KIND_GRID, jones=jones, eps_null=w.eps_null, storage=storage)
        kd = pg.make_kernels(g, 4, pg.KIND_DEGRID, jones=jones, storage=storage)
        tg = kernels.make_tables(g, mueller.phi_grid(jones, w.eps_null))
        td = kernels.make_tables(g, mueller.phi_degrid(jones))
        if storage == pg.STORE_F16:
            tg, td = kernels.round_tables(tg, np.float16), kernels.round_tables(td, np.float16)
        rng = np.random.default_rng(sp["seed"])
        vis = synth.random_vis(w.nvis, 4, rng)
        uvw = torch.from_numpy(w.uvw).cuda()
        out.append(dict(w=w, kg=kg, kd=kd, tg=tg, td=td, vis=vis, pg_=pg.plan(kg, uvw, max_chunk=97),
                        pd=pg.plan(kd, uvw, max_chunk=97)))
    return out


@pytest.fixture(scope="module")
def fields():
    return _fields()


@pytest.mark.parametrize("storage", [pg.STORE_F32, pg.STORE_F16])
def test_batched_grid_and_degrid_match_oracle(storage, fields):
    fs = fields if storage == pg.STORE_F32 else _fields(pg.STORE_F16)
    vis = [torch.from_numpy(f["vis"]).cuda() for f in fs]
    grids = [torch.empty((4, f["w"].geom.n, f["w"].geom.n), dtype=torch.complex64, device="cuda") for f in fs]
    b = pg.batch([(f["pg_"], f["kg"], v, g) for f, v, g in zip(fs, vis, grids)])
    assert b.work_items == sum(f["pg_"].n_items for f in fs)
    b.grid()
    for f, g in zip(fs, grids):
        want = gridding.grid(f["w"].geom, f["tg"], f["w"].uvw, f["vis"])
        assert rel(g.cpu().numpy(), want) < TOL
    rng = np.random.default_rng(9)
    gin = [(rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape)).astype(np.complex64) for g in grids]
    outs = [torch.empty((f["w"].nvis, 4), dtype=torch.complex64, device="cuda") for f in fs]
    gd = [torch.from_numpy(x).cuda() for x in gin]
    bd = pg.batch([(f["pd"], f["kd"], o, g) for f, o, g in zip(fs, outs, gd)])
    bd.degrid()
    for f, o, x in zip(fs, outs, gin):
        want = gridding.degrid(f["w"].geom, f["td"], f["w"].uvw, x)
        assert rel(o.cpu().numpy(), want) < TOL


@pytest.mark.parametrize("storage,planes,waves", [(pg.STORE_F32, 1, 8), (pg.STORE_F32, 0, 4), (pg.STORE_F16, 2, 16)])
def test_batched_shared_tap_gridder(storage, planes, waves):
    """The shared-tap gridder over a batch (the first field's plan selects it, with its output
    planes per workgroup and waves) against the oracle per field, and against single launches."""
    fs = _fields(storage)
    fs[0]["pg_"].set_launch(3, waves, waves, 1, planes)
    vis = [torch.from_numpy(f["vis"]).cuda() for f in fs]
    grids = [torch.empty((4, f["w"].geom.n, f["w"].geom.n), dtype=torch.complex64, device="cuda") for f in fs]
    b = pg.batch([(f["pg_"], f["kg"], v, g) for f, v, g in zip(fs, vis, grids)])
    b.grid(fftshift=True)
    n_sign = [(-1.0) ** (np.arange(f["w"].geom.n)[:, None] + np.arange(f["w"].geom.n)[None, :]) for f in fs]
    for f, v, g, sg in zip(fs, vis, grids, n_sign):
        want = gridding.grid(f["w"].geom, f["tg"], f["w"].uvw, f["vis"]) * sg[None]
        for q in range(4):
            assert rel(g.cpu().numpy()[q], want[q]) < TOL, q
        one = pg.grid(f["pg_"], f["kg"], v, fftshift=True, variant=pg.VARIANT_SHARED)
        assert rel(g.cpu().numpy(), one.cpu().numpy()) < 1e-6


def test_batched_equals_single_field_launches(fields):
    vis = [torch.from_numpy(f["vis"]).cuda() for f in fields]
    grids = [torch.empty((4, f["w"].geom.n, f["w"].geom.n), dtype=torch.complex64, device="cuda") for f in fields]
    b = pg.batch([(f["pg_"], f["kg"], v, g) for f, v, g in zip(fields, vis, grids)])
    b.grid(fftshift=True)
    for f, v, g in zip(fields, vis, grids):
        one = pg.grid(f["pg_"], f["kg"], v, fftshift=True)
        assert rel(g.cpu().numpy(), one.cpu().numpy()) < 1e-6


def test_graph_replay_matches_eager(fields):
    """grid (batched) -> FFT -> taper captured in one HIP graph; every replay equals eager."""
    vis = [torch.from_numpy(f["vis"]).cuda() for f in fields]
    grids = [torch.empty((4, f["w"].geom.n, f["w"].geom.n), dtype=torch.complex64, device="cuda") for f in fields]
    imgs = [torch.empty((4, f["w"].geom.n, f["w"].geom.n), dtype=torch.float32, device="cuda") for f in fields]
    b = pg.batch([(f["pg_"], f["kg"], v, g) for f, v, g in zip(fields, vis, grids)])

    def pipeline():
        b.grid(fftshift=True)
        for f, g, im in zip(fields, grids, imgs):
            pg.taper(f["kg"], torch.fft.fft2(g), im, pg.TAPER_IMAGE, float(f["pg_"].n_kept))

    pipeline()
    torch.cuda.synchronize()
    eager = [im.clone() for im in imgs]
    eager_grids = [g.clone() for g in grids]
    masks = [torch.from_numpy(np.outer(f["kg"].aa_pixels, f["kg"].aa_pixels) >= 1e-2).cuda() for f in fields]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pipeline()  # warm-up on the capture stream (rocFFT plans, kernel attributes)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        pipeline()
    for rep in range(3):
        for im in imgs:
            im.fill_(-7.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        # float-atomic flush order differs between runs (~1e-7); edge pixels are divided by AA^2
        # down to ~4e-8, so images are compared where AA(l) AA(m) >= 1e-2, grids everywhere
        for e, im, ok in zip(eager, imgs, masks):
            assert float((im[:, ok] - e[:, ok]).norm() / e[:, ok].norm()) < 1e-5, rep
        for e, g in zip(eager_grids, grids):
            assert float((g - e).norm() / e.norm()) < 1e-6, rep
        _ = torch.randn(1000, device="cuda").sum().item()  # eager work between replays


def test_batch_with_empty_and_dropped_fields(fields):
    f = fields[0]
    empty = pg.plan(f["kg"], torch.zeros((0, 3), dtype=torch.float64, device="cuda"))
    far = pg.plan(f["kg"], torch.full((10, 3), 1e9, dtype=torch.float64, device="cuda"))
    g0 = torch.ones((4, 128, 128), dtype=torch.complex64, device="cuda")
    g1 = torch.ones((4, 128, 128), dtype=torch.complex64, device="cuda")
    v1 = torch.ones((10, 4), dtype=torch.complex64, device="cuda")
    b = pg.batch([(empty, f["kg"], None, g0), (far, f["kg"], v1, g1)])
    assert b.work_items == 0
    b.grid()
    assert float(g0.abs().max()) == 0.0 and float(g1.abs().max()) == 0.0
    b.degrid()
    assert float(v1.abs().max()) == 0.0


def test_batch_rejects_mixed_npol(fields):
    f = fields[0]
    w1 = synth.config1(nvis=100)
    k1 = pg.make_kernels(w1.geom, 1, pg.KIND_GRID)
    p1 = pg.plan(k1, torch.from_numpy(w1.uvw).cuda())
    g = torch.empty((1, 256, 256), dtype=torch.complex64, device="cuda")
    v = torch.empty((100, 1), dtype=torch.complex64, device="cuda")
    g4 = torch.empty((4, 128, 128), dtype=torch.complex64, device="cuda")
    with pytest.raises(pg.PolgridError, match="npol"):
        pg.batch([(f["pg_"], f["kg"], torch.from_numpy(f["vis"]).cuda(), g4), (p1, k1, v, g)])


# ------------------------------------------------------------------ full size: 16 fields, 16.1M rows

def test_full_size_batched_fields_sampled():
    """The 16-field workload (4096^2 x 4 each, float16 tables, 16.1M rows) in the benchmark's launch
    configuration: one grid launch over all fields with visibilities that are zero except a seeded
    sample of every field (rows of its densest plane and of its first populated plane); every
    field's grid against the oracle (its tables rounded to float16); then one degrid launch, the
    sampled rows of every field against the oracle."""
    from oracle import geometry
    from oracle_pool import tables_for_tasks
    from paper_2206_15117_amd import autotune

    pg.use_torch_allocator(True)
    ws = synth.config3()
    nf = len(ws)
    n = ws[0].geom.n
    check = list(range(nf))
    rng = np.random.default_rng(31)
    fields, samples, tasks = [], {}, []
    for f, w in enumerate(ws):
        launch = autotune.apply(w.geom, 4, pg.STORE_F16)
        g = launch.geom
        w.geom = g
        jones = synth.jones_on_lattice(w.beam, g.mk, g.fov)
        # the batched gridder's own tiles (the tables do not depend on them)
        kg = pg.make_kernels(autotune.batch_grid_geom(launch), 4, pg.KIND_GRID, jones=jones, eps_null=0.2,
                             storage=pg.STORE_F16)
        kd = pg.make_kernels(g, 4, pg.KIND_DEGRID, jones=jones, storage=pg.STORE_F16)
        uvw = torch.from_numpy(w.uvw).cuda()
        pgr, pdg = autotune.batch_plans(kg, kd, uvw, launch)
        vis = np.zeros((w.nvis, 4), np.complex64)
        if f in check:
            loc = geometry.locate(g, w.uvw)
            cnt = np.bincount(loc["plane"][loc["keep"]], minlength=g.nplanes)
            planes = sorted({int(np.argmax(cnt)), int(np.flatnonzero(cnt)[0])})
            s = np.sort(np.concatenate([rng.choice(np.flatnonzero((loc["plane"] == q) & loc["keep"]),
                                                   min(30, int(cnt[q])), replace=False) for q in planes]))
            vis[s] = synth.random_vis(len(s), 4, rng)
            samples[f] = s
            pgrid, pdeg = mueller.phi_grid(jones, 0.2), mueller.phi_degrid(jones)
            tasks += [(f, kind, q, (g, phi, q)) for kind, phi in ((0, pgrid), (1, pdeg)) for q in planes]
        fields.append(dict(w=w, kg=kg, kd=kd, pg_=pgr, pd=pdg, vis=torch.from_numpy(vis).cuda()))
    got_tabs = tables_for_tasks([t[3] for t in tasks], "16 fields")
    tabs = {f: ([None] * ws[f].geom.nplanes, [None] * ws[f].geom.nplanes) for f in check}
    for (f, kind, q, _), t in zip(tasks, got_tabs):
        tabs[f][kind][q] = t
    tabs = {f: (kernels.round_tables(a, np.float16), kernels.round_tables(b, np.float16)) for f, (a, b) in tabs.items()}
    grids = torch.empty((nf, 4, n, n), dtype=torch.complex64, device="cuda")
    b = pg.batch([(f["pg_"], f["kg"], f["vis"], grids[i]) for i, f in enumerate(fields)])
    b.grid(fftshift=True)
    sign = ((-1.0) ** (np.arange(n)[:, None] + np.arange(n)[None, :]))[None]
    for i in range(nf):
        if i in check:
            w = fields[i]["w"]
            s = samples[i]
            want = gridding.grid(w.geom, tabs[i][0], w.uvw[s], fields[i]["vis"].cpu().numpy()[s]) * sign
            got = grids[i].cpu().numpy()
            for q in range(4):
                assert rel(got[q], want[q]) < TOL, (i, q)
        else:
            assert float(grids[i].abs().max()) == 0.0, i
    gen = torch.Generator(device="cuda").manual_seed(32)
    gin = torch.randn((nf, 4, n, n), dtype=torch.complex64, device="cuda", generator=gen)
    outs = [torch.empty((f["w"].nvis, 4), dtype=torch.complex64, device="cuda") for f in fields]
    bd = pg.batch([(f["pd"], f["kd"], outs[i], gin[i]) for i, f in enumerate(fields)])
    bd.degrid(fftshift=True)
    for i in check:
        w = fields[i]["w"]
        s = samples[i]
        want = gridding.degrid(w.geom, tabs[i][1], w.uvw[s], gin[i].cpu().numpy().astype(np.complex128) * sign)
        got = outs[i].cpu().numpy()[s]
        for c in range(4):
            assert rel(got[:, c], want[:, c]) < TOL, (i, c)
