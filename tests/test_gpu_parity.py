"""GPU parity of the gfx950 path (through the C ABI) against the CPU oracle.

Bit-exact: FoF and safe labels, active pair sets and their types, editable
sets, iteration counts.  Float64 coordinates before quantisation: within
1e-4 * xi per coordinate after every iteration (per-iteration through
max_iters = k).  Every stream is decoded by both decoders and the method's
guarantees are checked on the result.
"""
import numpy as np
import pytest

import oracle
import golden_cases
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4


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


def _pairs(ctx, job=0):
    i = ctx.debug_fetch(job, "active_i")
    j = ctx.debug_fetch(job, "active_j")
    t = ctx.debug_fetch(job, "active_type")
    order = np.lexsort((j, i))
    return i[order], j[order], t[order]


def _run(ctx, w, mode, **kw):
    print("case", w.name, "n", w.n, "mode", mode, kw, flush=True)
    stream, lab, st = ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, mode=mode, box=w.box,
                                  debug_xyz=True, **kw)
    return stream, lab.cpu().numpy(), st


def _compare(ctx, w, mode, **kw):
    ref = oracle.correct(w.orig, w.recon, w.b, w.xi, mode=mode, box=w.box, **kw)
    stream, lab, st = _run(ctx, w, mode, **kw)
    np.testing.assert_array_equal(lab, ref.labels)
    np.testing.assert_array_equal(ctx.debug_fetch(0, "safe_labels"), ref.safe_labels)
    ai, aj, at = _pairs(ctx)
    np.testing.assert_array_equal(ai, ref.a_i)
    np.testing.assert_array_equal(aj, ref.a_j)
    np.testing.assert_array_equal(at, ref.a_type)
    np.testing.assert_array_equal(np.sort(ctx.debug_fetch(0, "editable")), ref.e_ids)
    for k in ("n_pairs", "n_safe", "n_pb", "n_pc", "n_active", "n_editable", "viol0"):
        assert st[k] == ref.stats[k], (k, st[k], ref.stats[k])
    assert st["iters"] == ref.iters and st["status"] == ref.status
    dp = np.abs(st["debug_xyz"] - ref.p).max() if w.n else 0.0
    assert dp <= TOL * w.xi, dp
    _check_loss(st, ref)
    return ref, stream, st


# The loss of Eq. 3 is a float64 sum over the violated pairs; the GPU adds
# per-wave partials in a fixed order, the oracle adds pair by pair, so the two
# sums differ by rounding only: a relative 1e-12 bounds it for the pair
# counts here (each of n additions errs by at most 2^-53 relative).
LOSS_RTOL = 1e-12


def _check_loss(st, ref):
    for k in ("loss0", "loss_final"):
        a, b = st[k], ref.stats[k]
        assert abs(a - b) <= LOSS_RTOL * abs(b), (k, a, b)


@pytest.mark.parametrize("case", golden_cases.load(), ids=lambda c: c["name"])
def test_golden_fixtures(ctx, case):
    pos = case["points"]
    for mode in ("vp", "sc", "hf"):
        stream, lab, st = ctx.correct(_dev(pos), _dev(pos), case["b"], case["xi"], mode=mode,
                                      box=case["box"])
        np.testing.assert_array_equal(lab.cpu().numpy(), case["fof"])
        np.testing.assert_array_equal(ctx.debug_fetch(0, "safe_labels"), case["safe"])
        ai, aj, _ = _pairs(ctx)
        assert sorted(zip(ai.tolist(), aj.tolist())) == case["active"][mode], mode


@pytest.mark.parametrize("mode", ["vp", "sc", "hf"])
def test_plain_workload_full_parity(ctx, mode):
    import paper_2604_18801_amd as pcc
    w = synth.plain_blobs()
    ref, stream, st = _compare(ctx, w, mode)
    assert st["status"] == 0 and st["viol_final"] == 0
    # both decoders on both streams; guarantees on the result
    xg = pcc.decode(stream, w.recon)
    np.testing.assert_array_equal(xg, oracle.decode(stream, w.recon))
    np.testing.assert_array_equal(pcc.decode(ref.stream, w.recon), oracle.decode(ref.stream, w.recon))
    assert np.abs(xg.astype(np.float64) - w.orig).max() <= w.xi
    np.testing.assert_array_equal(oracle.fof_labels(xg, w.b, w.box), ref.labels)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 10, 25, 60])
def test_plain_workload_per_iteration(ctx, k):
    w = synth.plain_blobs()
    ref = oracle.correct(w.orig, w.recon, w.b, w.xi, mode="vp", max_iters=k)
    _, _, st = _run(ctx, w, "vp", max_iters=k)
    assert st["iters"] == ref.iters == k
    assert np.abs(st["debug_xyz"] - ref.p).max() <= TOL * w.xi


@pytest.mark.parametrize("mode,k", [("hf", 0), ("sc", 30), ("vp", 30)])
def test_periodic_cosmology_parity(ctx, mode, k):
    w = synth.cosmology(32, xi=0.05)
    _compare(ctx, w, mode, max_iters=k)


def _threshold_pairs(layout, seed=5):
    """Isolated pairs whose distances sit within a few float32 ulps of the
    three class thresholds b - 2 sqrt(3) xi, b and b + 2 sqrt(3) xi (Sec. 3.1),
    about half of them straddling a face of the periodic box.  layout:
    'box' (periodic, coordinates in [0, L)), 'shifted' (periodic, coordinates
    in [-L/2, L/2)) or 'open'."""
    rng = np.random.default_rng(seed)
    b, xi, L = 0.2, 0.02, 12.0
    r3 = 2.0 * np.sqrt(3.0) * xi
    thr = np.array([b - r3, b, b + r3])
    g = np.arange(12) + 0.5
    c = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    m = len(c)
    if layout != "open":
        c[c == 0.5] = 0.0  # the first layer on every axis sits on the box face
    d = thr[np.arange(m) % 3] * (1.0 + rng.integers(-8, 9, m) * 2.0 ** -20)
    u = rng.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    p = np.concatenate([c - 0.5 * d[:, None] * u, c + 0.5 * d[:, None] * u])
    if layout != "open":
        p = np.mod(p, L)
        if layout == "shifted":
            p -= 0.5 * L
    p = p[rng.permutation(len(p))]
    orig = np.ascontiguousarray(p.T.astype(np.float32))
    if layout == "box":
        orig[orig >= np.float32(L)] = 0.0
    box = (0.0, 0.0, 0.0) if layout == "open" else (L, L, L)
    return synth.Workload("thr_" + layout, orig, synth.grid_reconstruction(orig, xi), b, xi, box)


@pytest.mark.parametrize("layout", ["box", "shifted", "open"])
@pytest.mark.parametrize("mode", ["vp", "hf"])
def test_pair_classes_at_the_thresholds(ctx, layout, mode):
    """The float32 classification with guard bands (and the per-cell
    periodic images inside the box) gives the oracle's classes for pairs at
    the thresholds, inside and outside the box and on open axes."""
    w = _threshold_pairs(layout)
    ref, stream, st = _compare(ctx, w, mode)
    assert ref.stats["n_pb"] > 0 and ref.stats["n_pc"] > 0 and ref.stats["n_safe"] > 0


@pytest.mark.parametrize("layout", ["box", "shifted", "open"])
def test_pair_classes_at_the_thresholds_in_dense_units(ctx, layout):
    """The same pairs with every cell taken as a dense unit: partners are
    staged with their image shift added and culled against the box of the
    unit's homes, so the pairs right at r_v test that no partner within r_v
    of a home is dropped."""
    old = ctx.get_option("dense_cell")
    ctx.set_option("dense_cell", 1)
    try:
        w = _threshold_pairs(layout, seed=11)
        for mode in ("vp", "hf"):
            print("case thr dense", layout, mode, flush=True)
            ref, stream, st = _compare(ctx, w, mode)
            assert ref.stats["n_pc"] > 0
    finally:
        ctx.set_option("dense_cell", old)


@pytest.mark.parametrize("m", [8, 32])
def test_bit_depths(ctx, m):
    import paper_2604_18801_amd as pcc
    w = synth.plain_blobs(8192, seed=9)
    ref, stream, st = _compare(ctx, w, "hf", m_bits=m)
    x = pcc.decode(stream, w.recon)
    assert np.abs(x.astype(np.float64) - w.orig).max() <= w.xi
    np.testing.assert_array_equal(oracle.fof_labels(x, w.b, w.box), ref.labels)


def test_sgd_and_paper_margins(ctx):
    w = synth.plain_blobs(4096, seed=5)
    _compare(ctx, w, "hf", optimizer="sgd", lr=0.05, max_iters=40)
    _compare(ctx, w, "sc", margin="paper", max_iters=40)


def test_edge_cases(ctx):
    import paper_2604_18801_amd as pcc
    z = np.zeros((3, 0), np.float32)
    stream, lab, st = ctx.correct(_dev(z), _dev(z), 0.1, 0.01)
    assert st["status"] == 0 and st["n_pairs"] == 0 and len(stream) >= 64
    assert pcc.decode(stream, z).shape == (3, 0)
    one = np.array([[0.5], [0.5], [0.5]], np.float32)
    stream, lab, st = ctx.correct(_dev(one), _dev(one), 0.1, 0.01)
    assert lab.cpu().numpy().tolist() == [0] and st["n_flagged"] == 0
    # all particles on one point: one component, no created pair
    same = np.full((3, 300), 0.25, np.float32)
    w = synth.Workload("same", same, same.copy(), 0.1, 0.01, (0.0, 0.0, 0.0))
    _compare(ctx, w, "hf")
    # xi = 0: no vulnerable pair
    w0 = synth.plain_blobs(4096, seed=2)
    w0 = synth.Workload("exact", w0.orig, w0.orig.copy(), w0.b, 0.0, (0.0, 0.0, 0.0))
    ref, stream, st = _compare(ctx, w0, "vp")
    assert st["n_active"] == 0 and st["n_flagged"] == 0
    # two particles, each side of the threshold
    for w in (synth.Workload("pair_pb", np.array([[0, 0.2421875], [0, 0], [0, 0]], np.float32),
                             np.array([[-0.015625, 0.2578125], [0, 0], [0, 0]], np.float32),
                             0.25, 0.02, (0.0, 0.0, 0.0)),
              synth.Workload("pair_pc0", np.array([[0, 0.28125], [0, 0], [0, 0]], np.float32),
                             np.array([[0.140625, 0.140625], [0, 0], [0, 0]], np.float32),
                             0.25, 0.15, (0.0, 0.0, 0.0))):
        _compare(ctx, w, "vp")


def test_error_statuses(ctx):
    import paper_2604_18801_amd as pcc
    w = synth.plain_blobs(2000, seed=3)
    bad = w.recon.copy()
    bad[1, 7] = w.orig[1, 7] + np.float32(3 * w.xi)
    with pytest.raises(pcc.PccError) as e:
        ctx.correct(_dev(w.orig), _dev(bad), w.b, w.xi)
    assert e.value.status == -5
    nan = w.orig.copy()
    nan[0, 3] = np.nan
    with pytest.raises(pcc.PccError) as e:
        ctx.correct(_dev(nan), _dev(w.recon), w.b, w.xi)
    assert e.value.status == -1
    with pytest.raises(pcc.PccError) as e:
        ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, m_bits=7)
    assert e.value.status == -1
    with pytest.raises(pcc.PccError) as e:
        ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, stream_cap=16)
    assert e.value.status == -4
    # the context keeps working after errors
    _compare(ctx, w, "hf")


def test_determinism(ctx):
    w = synth.cosmology(32, seed=7, xi=0.05)
    s1, l1, st1 = _run(ctx, w, "hf")
    s2, l2, st2 = _run(ctx, w, "hf")
    assert s1 == s2
    np.testing.assert_array_equal(l1, l2)
    np.testing.assert_array_equal(st1["debug_xyz"], st2["debug_xyz"])


def test_fof_labels_entry_point(ctx):
    for w in (synth.plain_blobs(), synth.cosmology(32, xi=0.05)):
        lab = ctx.fof_labels(_dev(w.orig), w.b, w.box).cpu().numpy()
        np.testing.assert_array_equal(lab, oracle.fof_labels(w.orig, w.b, w.box))
        lab = ctx.fof_labels(w.orig, w.b, w.box)  # host memory
        np.testing.assert_array_equal(lab, oracle.fof_labels(w.orig, w.b, w.box))


def test_batch_equals_single_calls(ctx):
    ws = [synth.plain_blobs(3000 + 1000 * k, seed=30 + k) for k in range(3)]
    ws.append(synth.cosmology(20, seed=40, xi=0.05))
    ws.append(synth.Workload("empty", np.zeros((3, 0), np.float32), np.zeros((3, 0), np.float32),
                             0.1, 0.01, (0.0, 0.0, 0.0)))
    modes = ["vp", "sc", "hf", "hf", "vp"]
    jobs = [dict(orig=_dev(w.orig), recon=_dev(w.recon), b=w.b, xi=w.xi, mode=m, box=w.box,
                 debug_xyz=True) for w, m in zip(ws, modes)]
    out = ctx.correct_batch(jobs)
    for (status, stream, lab, st), w, m in zip(out, ws, modes):
        s1, l1, st1 = _run(ctx, w, m)
        assert status == st1["status"]
        assert stream == s1
        np.testing.assert_array_equal(lab.cpu().numpy(), l1)
        np.testing.assert_array_equal(st["debug_xyz"], st1["debug_xyz"])
        assert st["iters"] == st1["iters"] and st["n_active"] == st1["n_active"]


@pytest.mark.parametrize("mode", ["vp", "sc", "hf"])
def test_trajectory_is_bitwise_the_oracles(ctx, mode):
    # rows summed in increasing partner index, host pow for the bias
    # corrections, correctly rounded division and square root: the float64
    # iterates are the oracle's to the last bit
    w = synth.plain_blobs()
    ref = oracle.correct(w.orig, w.recon, w.b, w.xi, mode=mode)
    _, _, st = _run(ctx, w, mode)
    assert st["iters"] == ref.iters
    np.testing.assert_array_equal(st["debug_xyz"], ref.p)


@pytest.mark.parametrize("k", [1, 2, 7, 40, 0])
def test_active_set_steps_are_exact(ctx, k):
    # rows that are fixed points of a step are skipped; the iterates stay
    # the oracle's to the last bit at every stopping point (k = 0: no cap)
    w = synth.cosmology(32, seed=4, xi=0.05)
    kw = {"max_iters": k} if k else {}
    ref = oracle.correct(w.orig, w.recon, w.b, w.xi, mode="hf", box=w.box, **kw)
    _, lab, st = _run(ctx, w, "hf", **kw)
    np.testing.assert_array_equal(lab, ref.labels)
    assert st["iters"] == ref.iters and st["status"] == ref.status
    np.testing.assert_array_equal(st["debug_xyz"], ref.p)
    ne, steps = st["n_editable"], st["iters"] + 1
    # the first step evaluates every row; no step evaluates more
    assert ne <= st["pgd_rows_evaluated"] <= steps * ne
    assert 2 * st["n_active"] <= st["pgd_incidences_evaluated"] <= steps * 2 * st["n_active"]
    if k == 0:
        assert st["pgd_rows_evaluated"] < steps * ne


@pytest.mark.parametrize("mode", ["vp", "sc", "hf"])
def test_slotted_and_exact_pair_paths_agree(ctx, mode):
    # the write pass either fills slots sized by the pair classes (then
    # compacts them) or writes at offsets counted in a pass of its own
    import paper_2604_18801_amd as pcc
    w = synth.cosmology(24, seed=9, xi=0.05)
    print("case slotted vs exact", mode, flush=True)
    ex = pcc.Context(0)
    try:
        ex.set_option("exact_pairs", 1)
        s1, l1, st1 = ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, mode=mode, box=w.box,
                                  debug_xyz=True, max_iters=40)
        p1 = _pairs(ctx)
        s2, l2, st2 = ex.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, mode=mode, box=w.box,
                                 debug_xyz=True, max_iters=40)
        p2 = _pairs(ex)
    finally:
        ex.close()
    assert s1 == s2
    np.testing.assert_array_equal(l1.cpu().numpy(), l2.cpu().numpy())
    np.testing.assert_array_equal(st1["debug_xyz"], st2["debug_xyz"])
    for a, b in zip(p1, p2):
        np.testing.assert_array_equal(a, b)
    assert st1["iters"] == st2["iters"] and st1["n_active"] == st2["n_active"]


@pytest.mark.parametrize("mode", ["hf", "vp"])
def test_loss_tolerance_stop_matches_oracle(ctx, mode):
    # Alg. 1's eps_L: both sides stop at the first iterate whose tightened
    # loss is <= eps_L.  eps_L is placed between two consecutive losses of the
    # run without a tolerance, far (relative 1e-6) from every evaluated loss,
    # so the rounding difference of the two sums cannot change the decision.
    w = synth.plain_blobs(8192, seed=21)
    full = oracle.correct(w.orig, w.recon, w.b, w.xi, mode=mode, box=w.box)
    hist = np.asarray(full.loss_hist)
    assert full.status == 0 and full.iters > 8
    k = full.iters // 2
    while hist[k] >= hist[k - 1]:
        k += 1
    tol = float(np.sqrt(hist[k - 1] * hist[k]))
    stop = int(np.argmax(hist <= tol))
    assert np.all(np.abs(hist[:stop + 1] - tol) > 1e-6 * tol)
    ref = oracle.correct(w.orig, w.recon, w.b, w.xi, mode=mode, box=w.box, loss_tol=tol)
    assert ref.iters == stop and ref.status == 0 and ref.stats["viol_final"] > 0
    _, lab, st = _run(ctx, w, mode, loss_tol=tol)
    np.testing.assert_array_equal(lab, ref.labels)
    assert st["iters"] == ref.iters and st["status"] == 0
    assert st["viol_final"] == ref.stats["viol_final"] and st["viol0"] == ref.stats["viol0"]
    _check_loss(st, ref)
    assert st["loss_final"] <= tol
    np.testing.assert_array_equal(st["debug_xyz"], ref.p)


@pytest.mark.parametrize("k", [1, 3, 20])
def test_loss_per_iteration_matches_oracle(ctx, k):
    # the loss of the last evaluated iterate at several caps, in a run whose
    # rows span many PGD tiles and waves
    w = synth.cosmology(24, seed=13, xi=0.05)
    ref = oracle.correct(w.orig, w.recon, w.b, w.xi, mode="hf", box=w.box, max_iters=k)
    _, _, st = _run(ctx, w, "hf", max_iters=k)
    assert st["iters"] == ref.iters == k
    assert ref.stats["loss_final"] > 0
    _check_loss(st, ref)
    assert st["loss_final"] == pytest.approx(ref.loss_hist[-1], rel=LOSS_RTOL)


def test_batch_with_mixed_caps_equals_single_calls(ctx):
    # jobs of one call with different iteration caps (and so different
    # lengths of Adam's bias-correction table), the short cap first
    ws = [synth.plain_blobs(4000, seed=50), synth.plain_blobs(5000, seed=51),
          synth.plain_blobs(3000, seed=52)]
    caps = [50, 0, 7]
    jobs = [dict(orig=_dev(w.orig), recon=_dev(w.recon), b=w.b, xi=w.xi, mode="hf", box=w.box,
                 debug_xyz=True, opts={"max_iters": c} if c else {}) for w, c in zip(ws, caps)]
    out = ctx.correct_batch(jobs)
    for (status, stream, lab, st), w, c in zip(out, ws, caps):
        kw = {"max_iters": c} if c else {}
        s1, l1, st1 = _run(ctx, w, "hf", **kw)
        ref = oracle.correct(w.orig, w.recon, w.b, w.xi, mode="hf", box=w.box, **kw)
        assert status == st1["status"] == ref.status
        assert st["iters"] == st1["iters"] == ref.iters
        assert stream == s1
        np.testing.assert_array_equal(st["debug_xyz"], st1["debug_xyz"])
        np.testing.assert_array_equal(st["debug_xyz"], ref.p)


def test_iteration_cap_above_the_limit_is_rejected(ctx):
    import paper_2604_18801_amd as pcc
    w = synth.plain_blobs(2000, seed=3)
    with pytest.raises(pcc.PccError) as e:
        ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, max_iters=(1 << 31) + 1)
    assert e.value.status == -1
    # betas whose bias corrections stay below 1 for longer than the table
    # the library keeps, with a cap beyond it
    with pytest.raises(pcc.PccError) as e:
        ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, beta2=1.0 - 1e-12,
                    max_iters=1 << 30)
    assert e.value.status == -1
    # at the limit with the default betas the table ends where both
    # corrections reach 1: the call runs as with the default cap
    a = ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, max_iters=1 << 31, debug_xyz=True)
    b = ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, debug_xyz=True)
    assert a[0] == b[0] and a[2]["iters"] == b[2]["iters"]


@pytest.mark.parametrize("mode,cap", [("vp", 0), ("sc", 0), ("hf", 0), ("hf", 9)])
def test_loss_trace_matches_oracle(ctx, mode, cap):
    # the per-evaluation trace of Alg. 1's loop (loss of Eq. 3 and violated
    # constraints at every iterate): the loss-against-iteration curve; the
    # plain workload converges in about 100 steps in every mode
    w = synth.plain_blobs() if cap == 0 else synth.cosmology(24, seed=12, xi=0.05)
    kw = {"max_iters": cap} if cap else {}
    ref = oracle.correct(w.orig, w.recon, w.b, w.xi, mode=mode, box=w.box, **kw)
    print("case trace", mode, cap, flush=True)
    _, _, st = ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, mode=mode, box=w.box,
                           trace=100000, **kw)
    assert len(st["loss_trace"]) == ref.iters + 1 == len(ref.loss_hist)
    np.testing.assert_array_equal(st["viol_trace"], ref.viol_hist)
    scale = np.maximum(np.abs(ref.loss_hist), 1e-300)
    assert np.all(np.abs(st["loss_trace"] - ref.loss_hist) <= LOSS_RTOL * scale)
    assert st["loss_trace"][0] == st["loss0"] and st["loss_trace"][-1] == st["loss_final"]
    # a trace shorter than the run keeps its first entries
    _, _, st5 = ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, mode=mode, box=w.box,
                            trace=5, **kw)
    np.testing.assert_array_equal(st5["viol_trace"], ref.viol_hist[:5])


@pytest.mark.parametrize("kind,mode", [("plain", "vp"), ("plain", "hf"), ("cosmo", "hf"),
                                       ("cosmo", "sc"), ("md", "hf"), ("sph", "sc")])
def test_workspace_query_bounds_the_call(ctx, kind, mode):
    # the footprint the served form admits by is at least the workspace the
    # full call then takes, and within a small factor of it
    w = {"plain": lambda: synth.plain_blobs(),
         "cosmo": lambda: synth.cosmology(32, seed=13, xi=0.05),
         "md": lambda: synth.md_block(40000, 14),
         "sph": lambda: synth.sph_voids(30000, 15)}[kind]()
    kw = {"max_iters": 50} if mode != "hf" else {}
    print("case workspace query", kind, mode, flush=True)
    q = ctx.workspace_query(_dev(w.orig), _dev(w.recon), w.b, w.xi, mode=mode, box=w.box, **kw)
    ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, mode=mode, box=w.box, **kw)
    hw = ctx.workspace_high_water()
    assert 0 < hw <= q <= 8 * hw + (4 << 20), (hw, q)


def test_cell_list_tables_stay_in_bounds(ctx):
    # the cell starts and forward-neighbour ranges every pair pass indexes:
    # starts strictly increasing from 0 to n; nine particle ranges per cell,
    # each empty or running between two cell starts
    def check(cs, nb, n):
        u = len(cs) - 1
        assert cs[0] == 0 and cs[-1] == n and np.all(np.diff(cs) >= 1)
        assert len(nb) == 2 * 9 * u
        lo, hi = nb[0::2], nb[1::2]
        assert np.all(lo <= hi) and np.all(hi <= n)
        full = hi > lo
        assert np.all(np.isin(lo[full], cs)) and np.all(np.isin(hi[full], cs))
    cases = [(synth.cosmology(24, seed=16, xi=0.05), "hf"), (synth.md_block(30000, 17), "sc"),
             (synth.plain_blobs(), "vp"), (synth.plain_blobs(2, seed=18), "hf")]
    for w, m in cases:
        print("case cell tables", w.name, flush=True)
        ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, mode=m, box=w.box, max_iters=5)
        check(ctx.debug_fetch(0, "cell_start").astype(np.int64),
              ctx.debug_fetch(0, "neighbors").astype(np.int64), w.n)
    # several jobs in one index space
    ws = [synth.plain_blobs(3000, seed=19), synth.cosmology(16, seed=20, xi=0.05)]
    ctx.correct_batch([dict(orig=_dev(w.orig), recon=_dev(w.recon), b=w.b, xi=w.xi, mode="hf",
                            box=w.box) for w in ws])
    check(ctx.debug_fetch(0, "cell_start").astype(np.int64),
          ctx.debug_fetch(1, "neighbors").astype(np.int64), sum(w.n for w in ws))
