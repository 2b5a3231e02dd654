"""The batched and served forms against the CPU oracle, job by job.

Each job of a mixed batch (plain, periodic cosmology, MD droplets, SPH voids;
VP, SC and HF) and each job of a served sample of the 2,000-job stream (its
own kinds, sizes, xi/b and mode draw, at the stream's Adam step 0.005 b and
an iteration cap) is compared with oracle.correct on that job alone: FoF
and safe labels, active pairs and their types, editable set, iteration
count and status bit-exact; float64 coordinates within 1e-4 xi (in fact
bitwise); the stream decoded by both decoders keeps the labels (when the
job converged) and the error box."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4
MODES = ("vp", "sc", "hf")


@pytest.fixture(scope="module")
def ctx():
    import paper_2604_18801_amd as pcc
    c = pcc.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _check_job(w, mode, res, ref, pairs=None):
    import paper_2604_18801_amd as pcc
    status, stream, lab, st = res
    lab = lab.cpu().numpy() if hasattr(lab, "cpu") else lab
    assert status == ref.status, (w.name, mode, status, ref.status)
    np.testing.assert_array_equal(lab, ref.labels)
    assert st["iters"] == ref.iters, (w.name, mode, st["iters"], ref.iters)
    for k in ("n_pairs", "n_safe", "n_pb", "n_pc", "n_active", "n_editable", "viol0"):
        assert st[k] == ref.stats[k], (w.name, mode, k, st[k], ref.stats[k])
    if pairs is not None:
        ai, aj, at, safe, ed = pairs
        order = np.lexsort((aj, ai))
        np.testing.assert_array_equal(ai[order], ref.a_i)
        np.testing.assert_array_equal(aj[order], ref.a_j)
        np.testing.assert_array_equal(at[order], ref.a_type)
        np.testing.assert_array_equal(safe, ref.safe_labels)
        np.testing.assert_array_equal(np.sort(ed), ref.e_ids)
    if w.n:
        dp = np.abs(st["debug_xyz"] - ref.p).max()
        assert dp <= TOL * w.xi, (w.name, mode, dp)
        x = pcc.decode(stream, w.recon)
        np.testing.assert_array_equal(x, oracle.decode(stream, w.recon))
        assert np.abs(x.astype(np.float64) - w.orig.astype(np.float64)).max() <= w.xi
        if ref.status == 0:
            np.testing.assert_array_equal(oracle.fof_labels(x, w.b, w.box), ref.labels)


def _batch_mix():
    ws = [synth.plain_blobs(4096, seed=81),
          synth.cosmology(24, seed=82, xi=0.05),
          synth.md_block(12000, 83),
          synth.sph_voids(9000, 84),
          synth.md_block(20000, 85),
          synth.cosmology(20, seed=86, xi=0.03),
          synth.sph_voids(6000, 87, xi=0.06),
          synth.plain_blobs(2048, seed=88)]
    modes = ["vp", "hf", "hf", "sc", "sc", "vp", "hf", "hf"]
    return ws, modes


def test_batch_jobs_equal_the_oracle(ctx):
    ws, modes = _batch_mix()
    jobs = [dict(orig=_dev(w.orig), recon=_dev(w.recon), b=w.b, xi=w.xi, mode=m, box=w.box,
                 debug_xyz=True) for w, m in zip(ws, modes)]
    print("case batch of %d mixed jobs" % len(jobs), flush=True)
    out = ctx.correct_batch(jobs)
    for k, (w, m) in enumerate(zip(ws, modes)):
        print("case batch job", k, w.name, m, flush=True)
        ref = oracle.correct(w.orig, w.recon, w.b, w.xi, mode=m, box=w.box)
        pairs = (ctx.debug_fetch(k, "active_i"), ctx.debug_fetch(k, "active_j"),
                 ctx.debug_fetch(k, "active_type"), ctx.debug_fetch(k, "safe_labels"),
                 ctx.debug_fetch(k, "editable"))
        _check_job(w, m, out[k], ref, pairs)


# small jobs of the 2,000-job served stream, one per (kind, mode) present
# among them: cosmology VP / SC / HF, SPH VP / SC / HF, MD VP / SC / HF
SERVED_SAMPLE = (149, 617, 666, 301, 1976, 378, 677, 1753, 1860)
SERVED_CAP = 400


def _served_sample():
    specs = synth.served_jobs(2000)
    return [(specs[j], synth.make_job(specs[j])) for j in SERVED_SAMPLE]


def test_served_sample_equals_the_oracle(ctx):
    import paper_2604_18801_amd as pcc
    sample = _served_sample()
    srv = pcc.Server(ctx, n_streams=2, max_inflight=4)
    try:
        tickets = []
        for s, w in sample:
            print("case served job", s["seed"] - 4_000_000, s["kind"], MODES[s["mode"]], w.n,
                  flush=True)
            tickets.append(srv.submit(orig=_dev(w.orig), recon=_dev(w.recon), b=w.b, xi=w.xi,
                                      mode=MODES[s["mode"]], box=w.box, debug_xyz=True,
                                      opts={"lr": 0.005 * w.b, "max_iters": SERVED_CAP}))
        srv.drain()
        results = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for (s, w), res in zip(sample, results):
        m = MODES[s["mode"]]
        ref = oracle.correct(w.orig, w.recon, w.b, w.xi, mode=m, box=w.box, lr=0.005 * w.b,
                             max_iters=SERVED_CAP)
        _check_job(w, m, res, ref)


def test_served_sample_in_one_batch_equals_the_oracle(ctx):
    sample = _served_sample()
    jobs = [dict(orig=_dev(w.orig), recon=_dev(w.recon), b=w.b, xi=w.xi, mode=MODES[s["mode"]],
                 box=w.box, debug_xyz=True, opts={"lr": 0.005 * w.b, "max_iters": SERVED_CAP})
            for s, w in sample]
    print("case served sample as one batch", flush=True)
    out = ctx.correct_batch(jobs)
    for k, (s, w) in enumerate(sample):
        m = MODES[s["mode"]]
        ref = oracle.correct(w.orig, w.recon, w.b, w.xi, mode=m, box=w.box, lr=0.005 * w.b,
                             max_iters=SERVED_CAP)
        pairs = (ctx.debug_fetch(k, "active_i"), ctx.debug_fetch(k, "active_j"),
                 ctx.debug_fetch(k, "active_type"), ctx.debug_fetch(k, "safe_labels"),
                 ctx.debug_fetch(k, "editable"))
        _check_job(w, m, out[k], ref, pairs)
