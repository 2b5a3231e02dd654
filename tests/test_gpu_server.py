"""Served form (the pcc_server_* calls through the C ABI): every job's
results equal those of a plain call on that job alone, whatever batch it
ran in; timestamps are ordered; a queued job can be cancelled; an invalid
job fails alone."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2604_18801_amd as pcc
    c = pcc.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _mix():
    ws = [synth.plain_blobs(2000 + 1500 * k, seed=50 + k) for k in range(4)]
    ws.append(synth.cosmology(16, seed=60, xi=0.05))
    ws.append(synth.md_block(3000, seed=61))
    ws.append(synth.sph_voids(4000, seed=62))
    ws.append(synth.Workload("empty", np.zeros((3, 0), np.float32), np.zeros((3, 0), np.float32),
                             0.1, 0.01, (0.0, 0.0, 0.0)))
    modes = ["vp", "sc", "hf", "hf", "hf", "sc", "vp", "hf"]
    return ws, modes


def _job(w, m, **kw):
    return dict(orig=_dev(w.orig), recon=_dev(w.recon), b=w.b, xi=w.xi, mode=m, box=w.box, **kw)


@pytest.mark.parametrize("n_streams,max_inflight", [(1, 0), (2, 3), (3, 1)])
def test_served_results_equal_single_calls(ctx, n_streams, max_inflight):
    import paper_2604_18801_amd as pcc
    print("case served mix n_streams", n_streams, "max_inflight", max_inflight, flush=True)
    ws, modes = _mix()
    srv = pcc.Server(ctx, n_streams=n_streams, max_inflight=max_inflight)
    try:
        tickets = [srv.submit(**_job(w, m)) for w, m in zip(ws, modes)]
        srv.drain()
        results = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for (status, stream, lab, st), w, m in zip(results, ws, modes):
        s1, l1, st1 = ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, mode=m, box=w.box)
        assert status == st1["status"], (w.name, m)
        assert stream == s1, (w.name, m)
        np.testing.assert_array_equal(lab.cpu().numpy(), l1.cpu().numpy())
        assert st["iters"] == st1["iters"] and st["n_active"] == st1["n_active"]
        assert 0.0 <= st["t_submit_ms"] <= st["t_start_ms"] <= st["t_finish_ms"]
        assert 1 <= st["batch_jobs"] <= (max_inflight or 256)
        assert 0 <= st["worker"] < n_streams


def test_cancel_poll_and_failures(ctx):
    import paper_2604_18801_amd as pcc
    print("case served cancel / poll / invalid job", flush=True)
    big = synth.cosmology(40, seed=70, xi=0.05)
    small = synth.plain_blobs(3000, seed=71)
    srv = pcc.Server(ctx, n_streams=1, max_inflight=1)
    try:
        t_big = srv.submit(**_job(big, "hf"))
        t_bad = srv.submit(**_job(small, "hf", opts={"m_bits": 12}))
        t_small = srv.submit(**_job(small, "sc"))
        t_cancel = srv.submit(**_job(small, "vp"))
        assert srv.poll(t_small) is None  # queued behind the big job
        cancelled = srv.cancel(t_cancel)
        r_big = srv.wait(t_big)
        r_bad = srv.wait(t_bad)
        r_small = srv.wait(t_small)
        r_cancel = srv.wait(t_cancel)
    finally:
        srv.close()
    assert r_big[0] == 0
    assert r_bad[0] == -1
    assert r_small[0] in (0, 1)
    s1, _, st1 = ctx.correct(_dev(small.orig), _dev(small.recon), small.b, small.xi, mode="sc")
    assert r_small[1] == s1
    if cancelled:
        assert r_cancel[0] == -7
    else:
        s2, _, _ = ctx.correct(_dev(small.orig), _dev(small.recon), small.b, small.xi, mode="vp")
        assert r_cancel[1] == s2


def test_arrivals_join_while_another_job_iterates(ctx):
    # iteration-level continuous batching: small jobs submitted while a long
    # job is iterating start, iterate beside it in the shared loop and
    # finish before it; every result equals the job run alone (plain call)
    # and the oracle's
    import oracle
    import paper_2604_18801_amd as pcc
    big = synth.cosmology(40, seed=90, xi=0.05)
    smalls = [synth.plain_blobs(2500 + 700 * k, seed=91 + k) for k in range(4)]
    modes = ["hf", "sc", "vp", "hf"]
    big_opts = {"max_iters": 3000}
    srv = pcc.Server(ctx, n_streams=2, max_inflight=1)
    try:
        print("case served: long VP job, then four small jobs", flush=True)
        t_big = srv.submit(**_job(big, "vp", opts=big_opts))
        ts = [srv.submit(**_job(w, m)) for w, m in zip(smalls, modes)]
        rs = [srv.wait(t) for t in ts]
        r_big = srv.wait(t_big)
    finally:
        srv.close()
    fin_big = r_big[3]["t_finish_ms"]
    for r in rs:
        assert r[3]["t_start_ms"] < fin_big and r[3]["t_finish_ms"] < fin_big, (r[3], r_big[3])
    s1, l1, st1 = ctx.correct(_dev(big.orig), _dev(big.recon), big.b, big.xi, mode="vp",
                              box=big.box, **big_opts)
    assert r_big[0] == st1["status"] and r_big[1] == s1 and r_big[3]["iters"] == st1["iters"]
    np.testing.assert_array_equal(r_big[2].cpu().numpy(), l1.cpu().numpy())
    for (status, stream, lab, st), w, m in zip(rs, smalls, modes):
        ref = oracle.correct(w.orig, w.recon, w.b, w.xi, mode=m, box=w.box)
        assert status == ref.status and st["iters"] == ref.iters, (w.name, m)
        np.testing.assert_array_equal(lab.cpu().numpy(), ref.labels)
        s2, _, _ = ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, mode=m, box=w.box)
        assert stream == s2
