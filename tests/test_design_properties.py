"""CPU checks of properties the GPU design relies on (no GPU, no library).

* The halo forest's chunk-local prefilter: keeping only the minimum spanning
  forest of each run of consecutive candidates loses no edge of the minimum
  spanning forest of all candidates (cycle property), and Boruvka rounds
  with "an edge is taken when it is the lightest of either end's component"
  find exactly the chunk's forest when a component's keys are distinct.
* The PGD owner sum over violated terms only: a row's gradient is a float64
  sum, starting at +0.0, of its violated terms in column order; a satisfied
  constraint contributes +0.0, and adding +0.0 never changes such a sum, so
  skipping the satisfied ones gives the same bits.
"""
import numpy as np
import pytest


def _kruskal(n, edges):
    """Minimum spanning forest (edge ids) of edges (key, u, v, id) by key."""
    par = list(range(n))

    def find(x):
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x

    kept = []
    for k, u, v, i in sorted(edges):
        a, b = find(u), find(v)
        if a != b:
            par[max(a, b)] = min(a, b)
            kept.append(i)
    return set(kept)


def _boruvka_rounds(n, edges):
    """The chunk kernel's rounds: every component offers its lightest live
    edge; an edge that is the lightest of either end's component is taken
    and its components joined; edges inside one component die."""
    par = list(range(n))

    def find(x):
        while par[x] != x:
            x = par[x]
        return x

    live = [e for e in edges if e[1] != e[2]]
    taken = set()
    while live:
        best = {}
        roots = []
        for k, u, v, i in live:
            ru, rv = find(u), find(v)
            roots.append((ru, rv))
            if ru == rv:
                continue
            best[ru] = min(best.get(ru, k), k)
            best[rv] = min(best.get(rv, k), k)
        sel = []
        rest = []
        for (k, u, v, i), (ru, rv) in zip(live, roots):
            if ru == rv:
                continue  # inside one component: dies
            if best[ru] == k or best[rv] == k:
                sel.append((ru, rv, i))
            else:
                rest.append((k, u, v, i))
        if not best:
            break  # every live edge died
        assert sel, "a round with edges between components takes at least one"
        for ru, rv, i in sel:
            a, b = find(ru), find(rv)
            assert a != b, "the round's lightest edges form a forest"
            par[max(a, b)] = min(a, b)
            taken.add(i)
        live = rest
    return taken


def _graph(rng, n, m, local):
    """Random multigraph with self-loops and distinct keys; with `local`, the
    edges come in runs around a moving centre (neighbouring homes), like the
    pair pass's candidate slots."""
    keys = rng.permutation(m).tolist()
    edges = []
    for i in range(m):
        if local:
            c = (i * n) // m
            u = int(np.clip(c + rng.integers(-6, 7), 0, n - 1))
            v = int(np.clip(c + rng.integers(-12, 13), 0, n - 1))
        else:
            u, v = (int(x) for x in rng.integers(0, n, 2))
        edges.append((keys[i], u, v, i))
    return edges


@pytest.mark.parametrize("local", [True, False])
@pytest.mark.parametrize("chunk", [7, 64, 256])
def test_chunk_local_forests_keep_the_global_forest(local, chunk):
    rng = np.random.default_rng(chunk + (1000 if local else 0))
    for trial in range(6):
        n = int(rng.integers(20, 400))
        m = int(rng.integers(n, 8 * n))
        edges = _graph(rng, n, m, local)
        whole = _kruskal(n, edges)
        kept = set()
        for s in range(0, m, chunk):
            part = edges[s:s + chunk]
            local_forest = _kruskal(n, part)
            # the kernel's rounds find the same forest as Kruskal
            assert _boruvka_rounds(n, part) == local_forest
            kept |= local_forest
        assert whole <= kept
        assert _kruskal(n, [e for e in edges if e[3] in kept]) == whole
        if local:
            assert len(kept) < m  # the prefilter drops something on such graphs


def test_parallel_edges_and_self_loops_keep_only_the_lightest():
    # two vertices joined by many parallel edges plus self-loops: the chunk
    # forest is the single lightest joining edge
    edges = [(10, 0, 1, 0), (3, 0, 1, 1), (7, 1, 0, 2), (1, 0, 0, 3), (5, 1, 1, 4)]
    assert _kruskal(2, edges) == {1}
    assert _boruvka_rounds(2, edges) == {1}


def test_sum_of_violated_terms_equals_the_full_sum_bitwise():
    rng = np.random.default_rng(7)
    for trial in range(2000):
        k = int(rng.integers(1, 200))
        terms = rng.normal(size=k) * 10.0 ** rng.integers(-30, 5, size=k)
        hit = rng.random(k) < rng.random()
        # violated terms may be any float64, -0.0 included; satisfied ones are +0.0
        terms[hit & (rng.random(k) < 0.05)] = -0.0
        full = np.float64(0.0)
        for t, h in zip(terms, hit):
            full = full + (t if h else np.float64(0.0))
        some = np.float64(0.0)
        for t, h in zip(terms, hit):
            if h:
                some = some + t
        assert full.tobytes() == some.tobytes()
        # a running sum that starts at +0.0 never becomes -0.0
        assert not (some == 0.0 and np.signbit(some))
