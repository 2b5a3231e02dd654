"""Pins of the oracle's constraint selection (Sec. 3.2, Sec. 3.3).

VP and SC against their definitions evaluated on breadth-first labels; HF
against a library minimum spanning tree; the mode hierarchy and the forest
size as invariants.
"""
import numpy as np
import pytest

import oracle
import bruteforce as bf


def _setup(seed, n=1500, b=0.05, xi=0.006, box=(0.0, 0.0, 0.0)):
    rng = np.random.default_rng(seed)
    pos = rng.random((3, n)).astype(np.float32)
    k = n // 2
    centres = rng.random((8, 3))
    pos[:, :k] = (centres[rng.integers(0, 8, k)].T + rng.normal(0, 0.03, (3, k))).astype(np.float32)
    if box[0] > 0:
        pos = np.mod(pos, np.float32(1.0)).astype(np.float32)
        pos[pos >= 1.0] = 0
    rec = (pos + rng.uniform(-xi, xi, pos.shape)).astype(np.float32)
    rec = np.where(np.abs(rec.astype(np.float64) - pos) > xi, pos, rec).astype(np.float32)
    c = oracle.constants(b, xi, maxabs=2.0)
    i, j, d2 = oracle.pairs(pos, box, c["rv2"])
    cls = oracle.classify(d2, c)
    link = (cls == 1) | (cls == 2)
    fof = bf.components(n, i[link], j[link])
    safe = bf.components(n, i[cls == 1], j[cls == 1])
    return pos, rec, c, i, j, d2, cls, fof, safe, box


def _set(ai, aj):
    return set(zip(ai.tolist(), aj.tolist()))


@pytest.mark.parametrize("seed", range(5))
def test_modes_against_definitions(seed):
    box = (1.0, 1.0, 1.0) if seed % 2 else (0.0, 0.0, 0.0)
    xi = [0.002, 0.006, 0.01, 0.006, 0.02][seed]
    pos, rec, c, i, j, d2, cls, fof, safe, box = _setup(seed, xi=xi, box=box)
    n = pos.shape[1]
    vul = (cls == 2) | (cls == 3)
    V = _set(i[vul], j[vul])
    vp = oracle.select("vp", n, i, j, d2, c, safe, fof, rec, box)
    sc = oracle.select("sc", n, i, j, d2, c, safe, fof, rec, box)
    hf = oracle.select("hf", n, i, j, d2, c, safe, fof, rec, box)
    A_vp, A_sc, A_hf = _set(*vp[:2]), _set(*sc[:2]), _set(*hf[:2])
    assert A_vp == V
    assert A_sc == {(a, b) for (a, b) in V if safe[a] != safe[b]}
    assert A_hf <= A_sc <= A_vp
    # sorted by (i, j), types carried along
    for ai, aj, at in (vp, sc, hf):
        key = ai.astype(np.int64) * n + aj
        assert np.all(np.diff(key) > 0)
        cmap = {(a, b): k for a, b, k in zip(i.tolist(), j.tolist(), cls.tolist())}
        assert all(cmap[(a, b)] == t for a, b, t in zip(ai.tolist(), aj.tolist(), at.tolist()))
    # HF: potentially-created pairs kept exactly across halos
    pc_hf = {(a, b) for a, b, t in zip(*hf) if t == 3}
    assert pc_hf == {(a, b) for (a, b), k in zip(zip(i.tolist(), j.tolist()), cls.tolist())
                     if k == 3 and fof[a] != fof[b]}
    # HF forest = minimum spanning forest of the supernode multigraph
    cand = [(a, b) for (a, b), k in zip(zip(i.tolist(), j.tolist()), cls.tolist())
            if k == 2 and safe[a] != safe[b]]
    ca = np.array([p[0] for p in cand], dtype=np.int64)
    cb = np.array([p[1] for p in cand], dtype=np.int64)
    x = rec.astype(np.float64)
    if len(cand):
        dd = [bf.min_image(x[a][ca] - x[a][cb], box[a]) for a in range(3)]
        r2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2]
        viol0 = (r2 > c["bm2"]).astype(np.uint64)
        key = (viol0 << np.uint64(62)) | (ca.astype(np.uint64) << np.uint64(31)) | cb.astype(np.uint64)
        forest = bf.spanning_forest(n, safe[ca], safe[cb], key)
        F = {(int(ca[k]), int(cb[k])) for k in forest}
    else:
        F = set()
    pb_hf = {(a, b) for a, b, t in zip(*hf) if t == 2}
    assert pb_hf == F
    # forest size: one edge per merge of safe components into halos
    n_safe_comp = len(np.unique(safe))
    n_fof_comp = len(np.unique(fof))
    assert len(F) == n_safe_comp - n_fof_comp
    # safe links plus the forest reproduce the FoF partition
    sl = cls == 1
    ei = np.concatenate([i[sl], np.array([p[0] for p in F], dtype=np.uint32)])
    ej = np.concatenate([j[sl], np.array([p[1] for p in F], dtype=np.uint32)])
    np.testing.assert_array_equal(bf.components(n, ei, ej), fof)


def test_no_safe_links_makes_sc_equal_vp():
    pos, rec, c, i, j, d2, cls, fof, safe, box = _setup(7, b=0.05, xi=0.02)
    assert c["rs"] <= 0
    n = pos.shape[1]
    vp = oracle.select("vp", n, i, j, d2, c, safe, fof, rec, box)
    sc = oracle.select("sc", n, i, j, d2, c, safe, fof, rec, box)
    assert _set(*vp[:2]) == _set(*sc[:2])
