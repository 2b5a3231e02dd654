"""The allocation-free FoF entry point (pcc_fof_labels_noalloc) against the
allocating one (pcc_fof_labels) and against the oracle: bitwise equal labels
on two calls in a row, the second with a smaller input (the static scratch
keeps the first call's contents), with device and host inputs; the scratch
bound it states holds; sizes beyond it are refused before any device work;
the calls take no device memory."""
import numpy as np
import pytest

import oracle
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


def _check_bound(n):
    import paper_2604_18801_amd as pcc
    used = pcc.noalloc_high_water()
    assert 0 < used <= 256 * n + (1 << 20), (n, used)


def test_two_calls_shrinking_device(ctx):
    import torch
    big = synth.cosmology(64, seed=5, xi=0.05)      # 262,144 points, periodic
    small = synth.plain_blobs(32768, seed=6)        # open box
    for w in (big, small):
        print("case noalloc device n=%d" % w.n, flush=True)
        pts = _dev(w.orig)
        lab = ctx.fof_labels_noalloc(pts, w.b, w.box)
        torch.cuda.synchronize()
        _check_bound(w.n)
        ref = ctx.fof_labels(pts, w.b, w.box)
        np.testing.assert_array_equal(lab.cpu().numpy(), ref.cpu().numpy())
        np.testing.assert_array_equal(lab.cpu().numpy(), oracle.fof_labels(w.orig, w.b, w.box))


def test_two_calls_shrinking_host(ctx):
    big = synth.md_block(200_000, 3_000_017)
    small = synth.sph_voids(20_000, 77)
    for w in (big, small):
        print("case noalloc host n=%d" % w.n, flush=True)
        lab = ctx.fof_labels_noalloc(w.orig, w.b, w.box)
        _check_bound(w.n)
        np.testing.assert_array_equal(lab, ctx.fof_labels(w.orig, w.b, w.box))
        np.testing.assert_array_equal(lab, oracle.fof_labels(w.orig, w.b, w.box))


def test_largest_size_and_refusal(ctx):
    import paper_2604_18801_amd as pcc
    nmax = pcc.fof_labels_noalloc_max_n()
    assert nmax == 520192
    # uniform points at the largest accepted size, dense enough for pairs
    rng = np.random.default_rng(9)
    side = float(nmax) ** (1.0 / 3.0)
    pts = np.ascontiguousarray((rng.random((3, nmax)) * side).astype(np.float32))
    print("case noalloc n=max", flush=True)
    lab = ctx.fof_labels_noalloc(_dev(pts), 0.2, (0.0, 0.0, 0.0))
    _check_bound(nmax)
    np.testing.assert_array_equal(lab.cpu().numpy(),
                                  ctx.fof_labels(_dev(pts), 0.2).cpu().numpy())
    over = np.zeros((3, nmax + 1), dtype=np.float32)
    with pytest.raises(pcc.PccError) as e:
        ctx.fof_labels_noalloc(over, 0.2)
    assert e.value.status == -1 and "static scratch" in str(e.value)
    # empty and single-point inputs
    assert ctx.fof_labels_noalloc(np.zeros((3, 0), np.float32), 0.2).shape == (0,)
    assert list(ctx.fof_labels_noalloc(np.zeros((3, 1), np.float32), 0.2)) == [0]


def test_no_device_memory_taken(ctx):
    import torch
    w = synth.plain_blobs(32768, seed=8)
    pts = _dev(w.orig)
    lab = torch.empty(w.n, dtype=torch.int32, device="cuda")
    ctx.fof_labels_noalloc(pts, w.b, w.box, labels=lab)  # loads every kernel once
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        ctx.fof_labels_noalloc(pts, w.b, w.box, labels=lab)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    np.testing.assert_array_equal(lab.cpu().numpy(), oracle.fof_labels(w.orig, w.b, w.box))
