"""GPU results on the full 256^3 cosmology snapshot (16.8M particles, the
benchmark's workload and call), checked where the oracle cannot follow at
this size through exact sampled computations and properties that hold at any
size:

* the FoF component of sampled particles, found by breadth-first search over
  an independent k-d tree (scipy) with the exact link predicate, is exactly
  the set of particles carrying its label, and the label is the component's
  smallest index;
* the vulnerable pairs of sampled particles (exhaustive search over all N)
  with their classes: every active pair at a sampled particle is one of
  them with its class, halo-forest mode keeps every potentially created pair
  that joins two halos, and its potentially broken pairs join two safe
  components;
* every active pair of the call lies in the distance window of its class;
* the decoded stream keeps every label and the error box;
* complete FoF of the originals and of the decoded positions computed
  without the library (a scipy k-d tree proposes pairs within b(1 + 1e-9),
  the exact float64 link predicate keeps the links, scipy's connected
  components join them): both equal the returned labels;
* the safe components joined by the halo-forest constraints are exactly the
  FoF components (the forest spans every halo).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def run():
    import torch
    import paper_2604_18801_amd as pcc
    assert torch.cuda.is_available()
    print("case cosmology256 hf full size: generating", flush=True)
    w = synth.cosmology(256, seed=1, xi=0.05)
    ctx = pcc.Context(0)
    o = torch.from_numpy(w.orig).cuda()
    r = torch.from_numpy(w.recon).cuda()
    print("case cosmology256 hf full size: correcting", flush=True)
    stream, lab, st = ctx.correct(o, r, w.b, w.xi, mode="hf", box=w.box)
    pairs = (ctx.debug_fetch(0, "active_i"), ctx.debug_fetch(0, "active_j"),
             ctx.debug_fetch(0, "active_type"))
    safe = ctx.debug_fetch(0, "safe_labels")
    yield w, ctx, stream, lab.cpu().numpy(), st, pairs, safe
    ctx.close()


def _consts(w):
    two_sqrt3 = 2.0 * np.sqrt(3.0)
    rs = w.b - two_sqrt3 * w.xi
    rv = w.b + two_sqrt3 * w.xi
    return (rs * rs if rs > 0 else -1.0), w.b * w.b, rv * rv


def _axis(d, L):
    d = np.where(d > 0.5 * L, d - L, d)
    return np.where(d < -0.5 * L, d + L, d)


def _d2_to(x, k, idx, box):
    # squared minimum-image distance in float64 from float32 inputs, summed
    # as (dx dx + dy dy) + dz dz
    p = [_axis(x[a][idx].astype(np.float64) - np.float64(x[a][k]), box[a]) for a in range(3)]
    return (p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]


def test_status_and_active_pair_windows(run):
    w, ctx, stream, lab, st, (ai, aj, at), safe = run
    assert st["status"] == 0 and st["viol_final"] == 0
    rs2, b2, rv2 = _consts(w)
    x = w.orig.astype(np.float64)
    p = [_axis(x[a][ai] - x[a][aj], w.box[a]) for a in range(3)]
    d2 = (p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]
    pb = at == 2
    assert np.all(d2[pb] > rs2) and np.all(d2[pb] <= b2)
    assert np.all(d2[~pb] > b2) and np.all(d2[~pb] <= rv2)
    assert np.all(at[~pb] == 3)
    # halo forest: created pairs join two halos, broken ones two safe components
    assert np.all(lab[ai[~pb]] != lab[aj[~pb]])
    assert np.all(safe[ai[pb]] != safe[aj[pb]])


def test_sampled_components_are_exact(run):
    from scipy.spatial import cKDTree
    w, ctx, stream, lab, st, pairs, safe = run
    n = w.n
    L = w.box[0]
    pts = np.mod(w.orig.T.astype(np.float64), L)
    tree = cKDTree(pts, boxsize=L, balanced_tree=False, compact_nodes=False)
    b2 = w.b * w.b
    rng = np.random.default_rng(17)
    seeds = list(rng.choice(n, size=6, replace=False))
    # and members of the two largest components
    vals, counts = np.unique(lab, return_counts=True)
    seeds += [int(v) for v in vals[np.argsort(counts)[-2:]]]
    for s in seeds:
        print("case component of particle", s, flush=True)
        seen = np.zeros(n, dtype=bool)
        seen[s] = True
        frontier = np.array([s])
        while len(frontier):
            cand = tree.query_ball_point(pts[frontier], r=w.b * (1 + 1e-9))
            new = []
            for k, c in zip(frontier, cand):
                c = np.asarray(c, dtype=np.int64)
                c = c[~seen[c]]
                if len(c) == 0:
                    continue
                c = c[_d2_to(w.orig, k, c, w.box) <= b2]
                seen[c] = True
                new.append(c)
            frontier = np.concatenate(new) if new else np.array([], dtype=np.int64)
        comp = np.nonzero(seen)[0]
        assert np.all(lab[comp] == comp.min()), s
        assert np.count_nonzero(lab == comp.min()) == len(comp), s


def test_sampled_vulnerable_sets(run):
    w, ctx, stream, lab, st, (ai, aj, at), safe = run
    rs2, b2, rv2 = _consts(w)
    n = w.n
    lo = np.minimum(ai, aj).astype(np.int64)
    hi = np.maximum(ai, aj).astype(np.int64)
    rng = np.random.default_rng(23)
    for k in rng.choice(n, size=16, replace=False):
        k = int(k)
        d2 = _d2_to(w.orig, k, np.arange(n), w.box)
        d2[k] = np.inf
        vul = np.nonzero((d2 > rs2) & (d2 <= rv2))[0]
        cls = np.where(d2[vul] <= b2, 2, 3)
        at_k = (lo == k) | (hi == k)
        partner = np.where(lo[at_k] == k, hi[at_k], lo[at_k])
        ptype = at[at_k]
        # every active pair at k is one of its vulnerable pairs, with its class
        pos = np.searchsorted(vul, partner)
        assert np.all(pos < len(vul)) and np.all(vul[np.minimum(pos, len(vul) - 1)] == partner)
        np.testing.assert_array_equal(cls[pos], ptype)
        # every created pair across two halos is kept
        across = vul[(cls == 3) & (lab[vul] != lab[k])]
        assert set(across.tolist()) <= set(partner[ptype == 3].tolist())


def _independent_fof(pos, b, box):
    """Canonical FoF labels (smallest member index) with no library code."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    from scipy.spatial import cKDTree
    n = pos.shape[1]
    L = box[0]
    pts = np.mod(pos.T.astype(np.float64), L)
    pts[pts >= L] = 0.0  # a tiny negative coordinate can round up to L
    tree = cKDTree(pts, boxsize=L, balanced_tree=False, compact_nodes=False)
    p = tree.query_pairs(b * (1 + 1e-9), output_type="ndarray")
    del tree, pts
    x = pos.astype(np.float64)
    d2 = None
    for a in range(3):
        d = _axis(x[a][p[:, 0]] - x[a][p[:, 1]], box[a])
        d2 = d * d if d2 is None else d2 + d * d
    p = p[d2 <= b * b]
    del d2
    g = coo_matrix((np.ones(len(p), np.int8), (p[:, 0], p[:, 1])), shape=(n, n)).tocsr()
    del p
    _, comp = connected_components(g, directed=False)
    minid = np.full(comp.max() + 1, n, dtype=np.int64)
    np.minimum.at(minid, comp, np.arange(n))
    return minid[comp].astype(np.int32)


def test_complete_fof_without_the_library(run):
    import paper_2604_18801_amd as pcc
    w, ctx, stream, lab, st, pairs, safe = run
    print("case independent FoF of the originals", flush=True)
    np.testing.assert_array_equal(_independent_fof(w.orig, w.b, w.box), lab)
    print("case independent FoF of the decoded positions", flush=True)
    x = pcc.decode(stream, w.recon)
    np.testing.assert_array_equal(_independent_fof(x, w.b, w.box), lab)


def test_forest_spans_every_halo(run):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    w, ctx, stream, lab, st, (ai, aj, at), safe = run
    n = w.n
    pb = at == 2
    # nodes: particles; edges: every particle to its safe component's label
    # and every forest constraint
    u = np.concatenate([np.arange(n), ai[pb].astype(np.int64)])
    v = np.concatenate([safe.astype(np.int64), aj[pb].astype(np.int64)])
    g = coo_matrix((np.ones(len(u), np.int8), (u, v)), shape=(n, n)).tocsr()
    _, comp = connected_components(g, directed=False)
    minid = np.full(comp.max() + 1, n, dtype=np.int64)
    np.minimum.at(minid, comp, np.arange(n))
    np.testing.assert_array_equal(minid[comp].astype(np.int32), lab)


def test_decoded_stream_keeps_labels_and_box(run):
    import torch
    import paper_2604_18801_amd as pcc
    w, ctx, stream, lab, st, pairs, safe = run
    x = pcc.decode(stream, w.recon)
    assert np.abs(x.astype(np.float64) - w.orig.astype(np.float64)).max() <= w.xi
    lab2 = ctx.fof_labels(torch.from_numpy(x).cuda(), w.b, w.box).cpu().numpy()
    np.testing.assert_array_equal(lab2, lab)
