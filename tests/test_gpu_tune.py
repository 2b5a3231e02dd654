"""Scheduling knobs and the autotuner (GPU, through the C ABI).

The cell side, the dense-cell threshold and the PGD graph length change only
the schedule: every setting, including the extremes (every cell dense, every
cell sparse, cells four times r_v), gives the same stream bytes, labels,
active pairs and float64 coordinates, equal to the oracle's; the autotuner
picks one of its candidates, leaves it on the context, and the results
after tuning are those from before."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

SETTINGS = [(100, 32, 8), (150, 8, 4), (200, 128, 16), (125, 1, 32), (400, 4096, 1)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2604_18801_amd as pcc
    assert torch.cuda.is_available()
    c = pcc.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _pairs(ctx):
    i = ctx.debug_fetch(0, "active_i")
    j = ctx.debug_fetch(0, "active_j")
    t = ctx.debug_fetch(0, "active_type")
    o = np.lexsort((j, i))
    return i[o], j[o], t[o]


def _set(ctx, pct, dense, graph):
    ctx.set_option("cell_pct", pct)
    ctx.set_option("dense_cell", dense)
    ctx.set_option("graph_iters", graph)


def _small_periodic(seed=5):
    # a box of five r_v-cells per side: cells of 2 r_v or more fall back to
    # three per side
    rng = np.random.default_rng(seed)
    L, b, xi = 1.2, 0.2, 0.01
    orig = rng.uniform(0.0, L, size=(3, 600)).astype(np.float32)
    recon = (orig + rng.uniform(-0.9 * xi, 0.9 * xi, size=orig.shape)).astype(np.float32)
    recon = np.mod(recon, np.float32(L)).astype(np.float32)
    recon = np.where(np.abs(recon.astype(np.float64) - orig) > xi, orig, recon).astype(np.float32)
    return orig, recon, b, xi, (L, L, L)


@pytest.mark.parametrize("mode", ["sc", "hf"])
def test_knobs_do_not_change_results(ctx, mode):
    w = synth.cosmology(24, seed=6, xi=0.05)
    ref = oracle.correct(w.orig, w.recon, w.b, w.xi, mode=mode, box=w.box, max_iters=60)
    base = None
    for pct, dense, graph in SETTINGS:
        print("case cosmology24", mode, "cell_pct", pct, "dense", dense, "graph", graph, flush=True)
        _set(ctx, pct, dense, graph)
        s, lab, st = ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, mode=mode, box=w.box,
                                 debug_xyz=True, max_iters=60)
        got = (s, lab.cpu().numpy(), st["debug_xyz"], _pairs(ctx), st["iters"])
        np.testing.assert_array_equal(got[1], ref.labels)
        np.testing.assert_array_equal(got[2], ref.p)
        np.testing.assert_array_equal(got[3][0], ref.a_i)
        np.testing.assert_array_equal(got[3][1], ref.a_j)
        assert got[4] == ref.iters
        if base is None:
            base = got
        else:
            assert got[0] == base[0]
    _set(ctx, 100, 32, 8)


def test_cells_fall_back_to_three_per_periodic_axis(ctx):
    orig, recon, b, xi, box = _small_periodic()
    ref = oracle.correct(orig, recon, b, xi, mode="vp", box=box)
    for pct in (100, 200, 400):
        print("case small periodic box, cell_pct", pct, flush=True)
        ctx.set_option("cell_pct", pct)
        s, lab, st = ctx.correct(_dev(orig), _dev(recon), b, xi, mode="vp", box=box,
                                 debug_xyz=True)
        np.testing.assert_array_equal(lab.cpu().numpy(), ref.labels)
        np.testing.assert_array_equal(st["debug_xyz"], ref.p)
        assert st["n_pairs"] == ref.stats["n_pairs"]
    ctx.set_option("cell_pct", 100)


def test_autotune_keeps_results(ctx):
    import paper_2604_18801_amd as pcc
    ws = [synth.md_block(n, 3_100_000 + k) for k, n in enumerate((20000, 45000, 12000, 80000))]
    jobs = [dict(orig=_dev(w.orig), recon=_dev(w.recon), b=w.b, xi=w.xi, mode="hf", box=w.box)
            for w in ws]
    print("case autotune on 4 MD blocks", flush=True)
    before = ctx.correct_batch(jobs)
    rep = ctx.autotune(jobs)
    assert len(rep["trials"]) == 20
    assert rep["cell_pct"] in (100, 125, 150, 200) and rep["dense_cell"] in (16, 32, 64, 128)
    assert rep["graph_iters"] in (4, 8, 16, 32)
    assert all(t["ms"] > 0 for t in rep["trials"])
    assert ctx.get_option("cell_pct") == rep["cell_pct"]
    assert ctx.get_option("dense_cell") == rep["dense_cell"]
    assert ctx.get_option("graph_iters") == rep["graph_iters"]
    after = ctx.correct_batch(jobs)
    for (s0, b0, l0, st0), (s1, b1, l1, st1) in zip(before, after):
        assert s0 == s1 and b0 == b1
        np.testing.assert_array_equal(l0.cpu().numpy(), l1.cpu().numpy())
        assert st0["iters"] == st1["iters"]
    # a tuned context hands its knobs to the workers of a server
    srv = pcc.Server(ctx)
    try:
        tk = srv.submit(**jobs[0])
        s2, b2, l2, _ = srv.wait(tk)
        assert s2 == before[0][0] and b2 == before[0][1]
    finally:
        srv.close()
    _set(ctx, 100, 32, 8)


def test_invalid_knob_values(ctx):
    import paper_2604_18801_amd as pcc
    print("case invalid knob values", flush=True)
    for key, v in (("cell_pct", 99), ("cell_pct", 401), ("dense_cell", 0), ("dense_cell", 5000)):
        with pytest.raises(pcc.PccError):
            ctx.set_option(key, v)
    assert ctx.get_option("cell_pct") == 100 and ctx.get_option("dense_cell") == 32


def test_kernel_timing_with_graphs(ctx):
    # timed graph replays: the same results, and one timed PGD step per step
    # launched (the first one directly, then whole graphs of graph_iters)
    w = synth.cosmology(24, seed=8, xi=0.05)
    print("case kernel timing on cosmology24", flush=True)
    s0, l0, st0 = ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, box=w.box, debug_xyz=True)
    ctx.set_option("kernel_timing", 1)
    try:
        s1, l1, st1 = ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, box=w.box,
                                  debug_xyz=True)
    finally:
        ctx.set_option("kernel_timing", 0)
    assert s0 == s1 and st0["iters"] == st1["iters"]
    np.testing.assert_array_equal(st0["debug_xyz"], st1["debug_xyz"])
    g = ctx.get_option("graph_iters")
    n = st1["kernel_launches"]["pgd_step"]
    assert n >= st1["iters"] + 1 and (n - 1) % g == 0, (n, st1["iters"], g)
    assert st1["kernel_launches"]["pgd_finalize"] == 1
    assert st1["kernel_ms"]["pgd_step"] > 0 and st1["kernel_ms"]["pair_classify"] > 0
