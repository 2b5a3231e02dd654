"""Independent brute-force checkers used to pin the oracle.

O(N^2) pair search, breadth-first components (scipy.sparse.csgraph) and a
library minimum spanning tree; none of this shares code with the oracle.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, minimum_spanning_tree


def min_image(d: np.ndarray, L: float) -> np.ndarray:
    if L > 0:
        d = np.where(d > 0.5 * L, d - L, d)
        d = np.where(d < -0.5 * L, d + L, d)
    return d


def all_pairs(pos: np.ndarray, box, r2: float):
    """Every pair i < j with squared distance <= r2, by exhaustive search."""
    x = pos.astype(np.float64)
    n = x.shape[1]
    I, J, D = [], [], []
    for s in range(0, n, 512):
        e = min(n, s + 512)
        dd = [min_image(x[a][s:e, None] - x[a][None, :], box[a]) for a in range(3)]
        d2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2]
        ii, jj = np.nonzero(d2 <= r2)
        ii = ii + s
        keep = jj > ii
        I.append(ii[keep])
        J.append(jj[keep])
        D.append(d2[ii[keep] - s, jj[keep]])
    i = np.concatenate(I).astype(np.uint32) if I else np.zeros(0, np.uint32)
    j = np.concatenate(J).astype(np.uint32) if J else np.zeros(0, np.uint32)
    d2 = np.concatenate(D) if D else np.zeros(0)
    order = np.lexsort((j, i))
    return i[order], j[order], d2[order]


def components(n: int, i: np.ndarray, j: np.ndarray) -> np.ndarray:
    """Labels = smallest member index of each connected component."""
    g = sp.coo_matrix((np.ones(len(i)), (i.astype(np.int64), j.astype(np.int64))), shape=(n, n))
    _, comp = connected_components(g, directed=False)
    lab = np.full(comp.max() + 1 if n else 0, n, dtype=np.int64)
    np.minimum.at(lab, comp, np.arange(n))
    return lab[comp].astype(np.int32)


def spanning_forest(n_nodes: int, u: np.ndarray, v: np.ndarray, key: np.ndarray) -> np.ndarray:
    """Indices of the edges of the minimum spanning forest of a multigraph
    with distinct edge keys (library MST on the lightest edge per node pair)."""
    if len(u) == 0:
        return np.zeros(0, dtype=np.int64)
    a = np.minimum(u, v).astype(np.int64)
    b = np.maximum(u, v).astype(np.int64)
    rank = np.empty(len(key), dtype=np.int64)
    rank[np.argsort(key, kind="stable")] = np.arange(len(key))
    # lightest edge per unordered node pair
    order = np.lexsort((rank, b, a))
    first = np.ones(len(order), dtype=bool)
    first[1:] = (a[order][1:] != a[order][:-1]) | (b[order][1:] != b[order][:-1])
    best = order[first]
    w = rank[best].astype(np.float64) + 1.0
    g = sp.coo_matrix((w, (a[best], b[best])), shape=(n_nodes, n_nodes)).tocsr()
    t = minimum_spanning_tree(g).tocoo()
    chosen = {}
    for k in best:
        chosen[(a[k], b[k])] = k
    return np.array(sorted(chosen[(int(min(p, q)), int(max(p, q)))] for p, q in zip(t.row, t.col)),
                    dtype=np.int64)
