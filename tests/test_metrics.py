"""Query metrics of the evaluation (Sec. 4.1) against independent
definitions: scikit-learn's adjusted Rand index, hand-worked IoU and HMF
cases, and brute-force pair counting."""
import itertools

import numpy as np
import pytest

from paper_2604_18801_amd import metrics


def _canon(lab):
    # smallest member index per component, as the library returns
    lab = np.asarray(lab)
    out = np.empty_like(lab)
    for v in np.unique(lab):
        idx = np.flatnonzero(lab == v)
        out[idx] = idx.min()
    return out


def test_ari_matches_scikit_learn():
    sk = pytest.importorskip("sklearn.metrics")
    rng = np.random.default_rng(0)
    for n, k in [(50, 3), (200, 20), (1000, 7), (300, 300)]:
        a = _canon(rng.integers(0, k, n))
        b = _canon(np.where(rng.random(n) < 0.2, rng.integers(0, k, n), a))
        assert metrics.ari(a, b) == pytest.approx(sk.adjusted_rand_score(a, b), abs=1e-12)


def test_pair_counts_brute_force():
    rng = np.random.default_rng(1)
    a = _canon(rng.integers(0, 5, 40))
    b = _canon(rng.integers(0, 6, 40))
    tp = fp = fn = tn = 0
    for i, j in itertools.combinations(range(40), 2):
        sa, sb = a[i] == a[j], b[i] == b[j]
        tp += sa and sb
        fn += sa and not sb
        fp += sb and not sa
        tn += not sa and not sb
    assert metrics.pair_counts(a, b) == {"tp": tp, "fp": fp, "fn": fn, "tn": tn}


def test_identity_and_degenerate_cases():
    a = _canon(np.array([0, 0, 1, 1, 1, 5]))
    assert metrics.ari(a, a) == 1.0
    assert metrics.membership_errors(a, a) == 0
    assert metrics.mwm_iou(a, a, min_members=2) == 1.0
    single = np.arange(10)
    assert metrics.ari(single, single) == 1.0  # 0/0: identical partitions


def test_iou_hand_worked():
    # original halos: A = {0..5} (6), B = {6..9} (4); decompressed: A splits
    # into {0..3} and {4, 5} and B gains particle 10 (from a singleton)
    orig = np.array([0] * 6 + [6] * 4 + [10])
    dec = np.array([0] * 4 + [4] * 2 + [6] * 4 + [6])
    # IoU_A = max(4/6, 2/6) = 2/3; IoU_B = 4/5; mass-weighted (6, 4)
    want = (6 * (2 / 3) + 4 * (4 / 5)) / 10
    assert metrics.mwm_iou(orig, dec, min_members=4) == pytest.approx(want)
    assert metrics.membership_errors(orig, dec) == 3  # 4, 5 and 10


def test_hmf_hand_worked():
    # halos of 20, 20, 40 and 80 members (log10: 1.30, 1.30, 1.60, 1.90) in
    # volume 10, 3 bins over [log10 20, log10 80]
    sizes = [20, 20, 40, 80]
    lab = np.concatenate([np.full(s, k * 1000) for k, s in enumerate(sizes)] + [np.arange(5000, 5010)])
    edges, dn = metrics.hmf(lab, volume=10.0, bins=3, min_members=20)
    w = (np.log10(80) - np.log10(20)) / 3
    np.testing.assert_allclose(edges, np.log10(20) + w * np.arange(4))
    np.testing.assert_allclose(dn, np.array([2, 1, 1]) / (10.0 * w))
    r = metrics.hmf_relative_error(lab, lab, volume=10.0, bins=3)
    assert r["max_abs"] == 0.0 and r["bins"] == 3
