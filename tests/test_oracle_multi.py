"""Multi-threshold correction in the oracle (the union of every linking
length's selected constraints, each with its own b -+ delta_t): one
threshold is the single correction; the active list is the tagged union of
the single-threshold selections; a pair selected at two thresholds is held
in the window between them; the decoded result keeps the FoF labels at every
linking length."""
import numpy as np

import oracle
import synth


def test_one_threshold_is_the_single_correction():
    w = synth.plain_blobs(4000, seed=3)
    a = oracle.correct(w.orig, w.recon, w.b, w.xi, mode="hf")
    m = oracle.correct(w.orig, w.recon, [w.b], w.xi, mode="hf")
    np.testing.assert_array_equal(a.p, m.p)
    np.testing.assert_array_equal(a.a_i, m.a_i)
    np.testing.assert_array_equal(m.a_thr, np.zeros_like(m.a_thr))
    np.testing.assert_array_equal(m.labels_all[0], a.labels)
    assert a.stream == m.stream and a.iters == m.iters


def test_active_list_is_the_tagged_union():
    w = synth.cosmology(16, seed=5, xi=0.05)
    bs = [0.17, 0.2, 0.23]
    m = oracle.correct(w.orig, w.recon, bs, w.xi, mode="hf", box=w.box, max_iters=1)
    rows = []
    for k, b in enumerate(bs):
        s = oracle.correct(w.orig, w.recon, b, w.xi, mode="hf", box=w.box, max_iters=1)
        rows += [(int(i), int(j), int(t), k) for i, j, t in zip(s.a_i, s.a_j, s.a_type)]
        np.testing.assert_array_equal(m.labels_all[k], s.labels)
    rows.sort(key=lambda r: (r[0], r[1], r[3]))
    got = list(zip(m.a_i.tolist(), m.a_j.tolist(), m.a_type.tolist(), m.a_thr.tolist()))
    assert got == rows


def test_pair_held_in_the_window_between_two_thresholds():
    # original distance 1.0: a potentially-created pair for b1 = 0.95 and a
    # potentially-broken link for b2 = 1.05 (2 sqrt 3 xi = 0.173); the
    # reconstruction stretches it to 1.08, which breaks the b2 link
    xi = 0.05
    orig = np.array([[0.0, 1.0], [0.0, 0.0], [0.0, 0.0]], dtype=np.float32)
    recon = np.array([[-0.04, 1.04], [0.0, 0.0], [0.0, 0.0]], dtype=np.float32)
    r = oracle.correct(orig, recon, [0.95, 1.05], xi, mode="vp")
    assert r.status == 0
    assert sorted(zip(r.a_type.tolist(), r.a_thr.tolist())) == [(2, 1), (3, 0)]
    x = oracle.decode(r.stream, recon).astype(np.float64)
    d = np.linalg.norm(x[:, 0] - x[:, 1])
    assert 0.95 < d <= 1.05
    assert np.abs(x - orig).max() <= xi


def test_decoded_result_keeps_every_threshold():
    w = synth.cosmology(16, seed=7, xi=0.03)
    bs = [0.16, 0.2, 0.24]
    for mode in ("hf", "sc"):
        r = oracle.correct(w.orig, w.recon, bs, w.xi, mode=mode, box=w.box)
        assert r.status == 0
        x = oracle.decode(r.stream, w.recon)
        assert np.abs(x.astype(np.float64) - w.orig).max() <= w.xi
        for k, b in enumerate(bs):
            np.testing.assert_array_equal(oracle.fof_labels(x, b, w.box), r.labels_all[k])
            np.testing.assert_array_equal(oracle.fof_labels(w.orig, b, w.box), r.labels_all[k])
