"""Failure handling forced from the host (GPU, through the C ABI): a
workspace allocation made to fail at different points of a call returns
PCC_E_OUT_OF_MEMORY with nothing left running, and the context then gives
the results of an undisturbed call; a server whose batch runs out of memory
retries its jobs one by one and every result equals the plain call's."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2604_18801_amd as pcc
    assert torch.cuda.is_available()
    c = pcc.Context(0)
    yield c
    pcc.inject_alloc_failure(-1)
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_allocation_failures_at_every_stage(ctx):
    import paper_2604_18801_amd as pcc
    w = synth.cosmology(20, seed=12, xi=0.05)
    o, r = _dev(w.orig), _dev(w.recon)
    s0, l0, st0 = ctx.correct(o, r, w.b, w.xi, box=w.box, debug_xyz=True)
    # how many workspace allocations one call makes
    pcc.inject_alloc_failure(1 << 40)
    ctx.correct(o, r, w.b, w.xi, box=w.box)
    n_alloc = (1 << 40) - pcc.alloc_failure_countdown()
    pcc.inject_alloc_failure(-1)
    assert n_alloc > 10
    for k in sorted({0, 1, n_alloc // 4, n_alloc // 2, (3 * n_alloc) // 4, n_alloc - 1}):
        print("case allocation", k, "of", n_alloc, "fails", flush=True)
        pcc.inject_alloc_failure(k)
        with pytest.raises(pcc.PccError) as ei:
            ctx.correct(o, r, w.b, w.xi, box=w.box)
        assert ei.value.status == -2
        assert pcc.alloc_failure_countdown() < 0  # the hook switched itself off
        s1, l1, st1 = ctx.correct(o, r, w.b, w.xi, box=w.box, debug_xyz=True)
        assert s1 == s0
        np.testing.assert_array_equal(l1.cpu().numpy(), l0.cpu().numpy())
        np.testing.assert_array_equal(st1["debug_xyz"], st0["debug_xyz"])


def test_server_retries_a_batch_that_ran_out_of_memory(ctx):
    import paper_2604_18801_amd as pcc
    ws = [synth.md_block(n, 3_200_000 + k) for k, n in enumerate((15000, 30000, 22000))]
    jobs = [dict(orig=_dev(w.orig), recon=_dev(w.recon), b=w.b, xi=w.xi, mode="hf", box=w.box)
            for w in ws]
    ref = [ctx.correct(j["orig"], j["recon"], j["b"], j["xi"], mode="hf", box=j["box"])
           for j in jobs]
    print("case server batch out of memory", flush=True)
    srv = pcc.Server(ctx, n_streams=1)
    try:
        pcc.inject_alloc_failure(3)
        tks = [srv.submit(**j) for j in jobs]
        out = [srv.wait(t) for t in tks]
    finally:
        pcc.inject_alloc_failure(-1)
        srv.close()
    for (status, stream, lab, st), (s0, l0, _) in zip(out, ref):
        assert status >= 0
        assert stream == s0
        np.testing.assert_array_equal(lab.cpu().numpy(), l0.cpu().numpy())
