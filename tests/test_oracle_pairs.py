"""Pins of the oracle's pair search, classification and components.

Pinned against: hand-derived dyadic fixtures (tests/golden), an exhaustive
O(N^2) search and breadth-first components (tests/bruteforce.py).
"""
import numpy as np
import pytest

import oracle
import bruteforce as bf
import golden_cases
import synth


def _classes(d2, c):
    cls = np.zeros(len(d2), dtype=np.int8)
    if c["rs"] > 0:
        cls[d2 <= c["rs2"]] = 1
    cls[(cls == 0) & (d2 <= c["b2"])] = 2
    cls[(cls == 0) & (d2 <= c["rv2"])] = 3
    return cls


@pytest.mark.parametrize("case", golden_cases.load(), ids=lambda c: c["name"])
def test_golden_classes_labels_and_modes(case):
    pos, b, xi, box = case["points"], case["b"], case["xi"], case["box"]
    n = pos.shape[1]
    c = oracle.constants(b, xi, maxabs=1.0)
    i, j, d2 = oracle.pairs(pos, box, 1e9)  # every pair
    got = {(int(a), int(bb)): int(k) for a, bb, k in zip(i, j, oracle.classify(d2, c))}
    assert got == case["pairs"]
    vi, vj, vd = oracle.pairs(pos, box, c["rv2"])
    fof = oracle.components(n, vi, vj, vd, c, "fof")
    safe = oracle.components(n, vi, vj, vd, c, "safe")
    np.testing.assert_array_equal(fof, case["fof"])
    np.testing.assert_array_equal(safe, case["safe"])
    for mode in ("vp", "sc", "hf"):
        ai, aj, _ = oracle.select(mode, n, vi, vj, vd, c, safe, fof, pos, box)
        assert sorted(zip(ai.tolist(), aj.tolist())) == case["active"][mode], mode


def _cloud(rng, n, box, scale=1.0):
    pos = np.empty((3, n), np.float32)
    for a in range(3):
        L = box[a] if box[a] > 0 else scale
        pos[a] = (rng.random(n) * L).astype(np.float32)
    return pos


@pytest.mark.parametrize("seed", range(6))
def test_pairs_match_exhaustive_search(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(200, 1500))
    box = [(0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (1.0, 0.0, 2.0)][seed % 3]
    pos = _cloud(rng, n, box)
    # clustered part so that some cells are crowded
    pos[:, : n // 3] = (pos[:, :1] + rng.normal(0, 0.02, (3, n // 3))).astype(np.float32)
    if box[0] > 0:
        pos[0] = np.mod(pos[0], np.float32(box[0]))
        pos[0][pos[0] >= box[0]] = 0
    r = float(rng.uniform(0.02, 0.2))
    i, j, d2 = oracle.pairs(pos, box, r * r)
    bi, bj, bd = bf.all_pairs(pos, box, r * r)
    np.testing.assert_array_equal(i, bi)
    np.testing.assert_array_equal(j, bj)
    np.testing.assert_array_equal(d2, bd)


@pytest.mark.parametrize("seed", range(4))
def test_components_match_bfs(seed):
    rng = np.random.default_rng(100 + seed)
    n = 1200
    box = (1.0, 1.0, 1.0) if seed % 2 else (0.0, 0.0, 0.0)
    pos = _cloud(rng, n, box)
    b = 0.06
    xi = [0.001, 0.004, 0.01, 0.03][seed]
    c = oracle.constants(b, xi, maxabs=1.0)
    i, j, d2 = oracle.pairs(pos, box, c["rv2"])
    cls = oracle.classify(d2, c)
    np.testing.assert_array_equal(cls, _classes(d2, c))
    fof = oracle.components(n, i, j, d2, c, "fof")
    safe = oracle.components(n, i, j, d2, c, "safe")
    link = (cls == 1) | (cls == 2)
    np.testing.assert_array_equal(fof, bf.components(n, i[link], j[link]))
    np.testing.assert_array_equal(safe, bf.components(n, i[cls == 1], j[cls == 1]))
    if c["rs"] <= 0:
        np.testing.assert_array_equal(safe, np.arange(n))


def test_fof_labels_on_plain_workload_match_library_neighbour_search():
    from scipy.spatial import cKDTree
    w = synth.plain_blobs()
    lab = oracle.fof_labels(w.orig, w.b, w.box)
    x = w.orig.T.astype(np.float64)
    cand = cKDTree(x).query_pairs(w.b * (1 + 1e-6), output_type="ndarray")
    d = x[cand[:, 0]] - x[cand[:, 1]]
    d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    keep = cand[d2 <= w.b * w.b]
    np.testing.assert_array_equal(lab, bf.components(w.n, keep[:, 0], keep[:, 1]))
