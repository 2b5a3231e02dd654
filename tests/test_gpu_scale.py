"""GPU results at scale (2M-particle cosmology snapshot), checked against the
oracle where it finishes in seconds and through properties that hold at any
size: exact labels, the class of every active pair, complete vulnerable-pair
sets for sampled particles (exhaustive search over all N), and the
guarantees of the decoded stream."""
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


@pytest.fixture(scope="module")
def snap():
    return synth.cosmology(128, seed=1, xi=0.05)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _d2(pos, i, j, box):
    x = pos.astype(np.float64)
    out = np.zeros(len(i))
    parts = []
    for a in range(3):
        d = x[a][i] - x[a][j]
        L = box[a]
        if L > 0:
            d = np.where(d > 0.5 * L, d - L, d)
            d = np.where(d < -0.5 * L, d + L, d)
        parts.append(d)
    out = (parts[0] * parts[0] + parts[1] * parts[1]) + parts[2] * parts[2]
    return out


def test_hf_labels_pairs_and_guarantees(ctx, snap):
    import paper_2604_18801_amd as pcc
    w = snap
    print("case cosmology128 hf", flush=True)
    stream, lab, st = ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, mode="hf", box=w.box)
    lab = lab.cpu().numpy()
    assert st["status"] == 0 and st["viol_final"] == 0
    ref = oracle.fof_labels(w.orig, w.b, w.box)
    np.testing.assert_array_equal(lab, ref)
    # every active pair is vulnerable and carries its class
    i = ctx.debug_fetch(0, "active_i")
    j = ctx.debug_fetch(0, "active_j")
    t = ctx.debug_fetch(0, "active_type")
    assert len(i) == st["n_active"] and np.all(i < j)
    d2 = _d2(w.orig, i, j, w.box)
    c = oracle.constants(w.b, w.xi, maxabs=float(max(np.abs(w.orig).max(), np.abs(w.recon).max())))
    pb = (d2 > c["rs2"]) & (d2 <= c["b2"])
    pc = (d2 > c["b2"]) & (d2 <= c["rv2"])
    np.testing.assert_array_equal(t == 2, pb)
    np.testing.assert_array_equal(t == 3, pc)
    # created pairs only across halos
    assert np.all(ref[i[t == 3]] != ref[j[t == 3]])
    # decoded stream: inside the box and the same clusters (two FoF codes)
    x = pcc.decode(stream, w.recon)
    assert np.abs(x.astype(np.float64) - w.orig).max() <= w.xi
    lab2 = ctx.fof_labels(_dev(x), w.b, w.box).cpu().numpy()
    np.testing.assert_array_equal(lab2, ref)
    np.testing.assert_array_equal(oracle.fof_labels(x, w.b, w.box), ref)


def test_vulnerable_sets_of_sampled_particles_are_complete(ctx, snap):
    w = snap
    print("case cosmology128 vp max_iters=1", flush=True)
    ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, mode="vp", box=w.box, max_iters=1,
                labels=False)
    i = ctx.debug_fetch(0, "active_i")
    j = ctx.debug_fetch(0, "active_j")
    c = oracle.constants(w.b, w.xi, maxabs=float(max(np.abs(w.orig).max(), np.abs(w.recon).max())))
    rng = np.random.default_rng(5)
    sample = rng.choice(w.n, 48, replace=False)
    # partners of the sampled particles from the GPU pair list
    sel = np.isin(i, sample) | np.isin(j, sample)
    gi, gj = i[sel], j[sel]
    got = {s: set() for s in sample.tolist()}
    for a, b in zip(gi.tolist(), gj.tolist()):
        if a in got:
            got[a].add(b)
        if b in got:
            got[b].add(a)
    allidx = np.arange(w.n)
    for s in sample.tolist():
        d2 = _d2(w.orig, np.full(w.n, s), allidx, w.box)
        want = (d2 > c["rs2"]) & (d2 <= c["rv2"])
        want[s] = False
        assert got[s] == set(np.nonzero(want)[0].tolist()), s


def test_large_stream_decodes_with_both_decoders(ctx):
    # a payload of several MB is compressed in pieces (concatenated frames)
    import paper_2604_18801_amd as pcc
    w = synth.cosmology(96, seed=6, xi=0.05)
    print("case cosmology96 vp max_iters=3", flush=True)
    stream, _, st = ctx.correct(_dev(w.orig), _dev(w.recon), w.b, w.xi, mode="vp", box=w.box,
                                max_iters=3, labels=False)
    assert st["bytes_flags"] + st["bytes_codes"] > (1 << 20)
    x1 = pcc.decode(stream, w.recon)
    x2 = oracle.decode(stream, w.recon)
    np.testing.assert_array_equal(x1, x2)
    assert np.abs(x1.astype(np.float64) - w.orig).max() <= w.xi
    # the device decoder: one thread per chunk of the Huffman bitstream
    x3 = ctx.decode_device(stream, _dev(w.recon)).cpu().numpy()
    np.testing.assert_array_equal(x3, x1)
