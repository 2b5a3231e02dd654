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


# ---------------------------------------------------------------------------
# Float32 classification of staged partners (dense pair units): the partner is
# staged as ps = fl(pj + shift), the displacement is fl(pi - ps) per axis and
# d^2 = fma(dz, dz, fma(dy, dy, fl(dx * dx))) in float32.  Outside the guard
# bands [(sqrt T - e)^2 (1 - 2^-17), (sqrt T + e)^2 (1 + 2^-17)] with
# e = 4 ulp_f32(max|x| + L + 1) the float32 class must be the exact float64
# class; and the gap to the box of a unit's homes, computed the same way, is
# never above any home's own float32 distance (no partner within r_v culled).
# Float32 rounding and the fused multiply-add are emulated exactly with
# rationals.
# ---------------------------------------------------------------------------
from fractions import Fraction


def _round_f32(x):
    """x (a Fraction) rounded to the nearest float32, ties to even."""
    if x == 0:
        return Fraction(0)
    s = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, -126)                    # subnormals share the smallest exponent
    q = a / Fraction(2) ** (e - 23)     # 24-bit significand scale
    n, r = divmod(q.numerator, q.denominator)
    if 2 * r > q.denominator or (2 * r == q.denominator and n % 2 == 1):
        n += 1
    return s * Fraction(n) * Fraction(2) ** (e - 23)


def _f32(x):
    return Fraction(float(np.float32(x)))


def _ulp_f32(x):
    return 2.0 ** (np.floor(np.log2(x)) - 23)


def _band(T, e):
    r = np.sqrt(T)
    lo = (r - e) ** 2 * (1 - 2.0 ** -17) if r > 2 * e else -1.0
    hi = (r + e) ** 2 * (1 + 2.0 ** -17)
    flo, fhi = np.float32(lo), np.float32(hi)
    if float(flo) > lo:
        flo = np.nextafter(flo, np.float32(-np.inf))
    if float(fhi) < hi:
        fhi = np.nextafter(fhi, np.float32(np.inf))
    return Fraction(float(flo)), Fraction(float(fhi))


def _d2_staged(pi, pj, sh):
    d = [_round_f32(pi[a] - _round_f32(pj[a] + sh[a])) for a in range(3)]
    return _round_f32(d[2] * d[2] + _round_f32(d[1] * d[1] + _round_f32(d[0] * d[0])))


def test_staged_float32_classes_match_the_exact_ones_outside_the_bands():
    rng = np.random.default_rng(11)
    L, b, xi = 512.0, 0.2, 0.05
    rs, rv = b - 2 * np.sqrt(3) * xi, b + 2 * np.sqrt(3) * xi
    e = 4 * _ulp_f32(L + L + 1)
    bands = [_band(T * T, e) for T in (rs, b, rv)]
    (rs_lo, rs_hi), (b_lo, b_hi), (rv_lo, rv_hi) = bands
    outside = 0
    for trial in range(3000):
        T = (rs, b, rv)[trial % 3]
        d = T * (1 + rng.normal() * 1e-4 * 10 ** rng.integers(0, 3))
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        # the home near a periodic face on x, so that some partners lie across it
        pi = np.array([np.float32(rng.uniform(0, L)) for _ in range(3)], np.float32)
        pi[0] = np.float32(L - 0.05) if trial % 2 else np.float32(0.05)
        q = pi.astype(np.float64) + d * u
        sh = np.where(q >= L, L, np.where(q < 0, -L, 0.0))
        pj = (q - sh).astype(np.float32)                # the partner inside [0, L)
        pj = np.where(pj >= np.float32(L), np.float32(0.0), pj)
        # the exact predicate: float64 minimum image of the float32 coordinates
        dx = pi.astype(np.float64) - pj.astype(np.float64)
        dx -= L * np.round(dx / L)
        exact = Fraction(float((dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2]))
        d2f = _d2_staged([_f32(x) for x in pi], [_f32(x) for x in pj], [Fraction(s) for s in sh])
        R2 = [Fraction(float(r * r)) for r in (rs, b, rv)]
        if d2f > rv_hi:
            assert exact > R2[2]
        elif d2f < rs_lo:
            assert exact <= R2[0]
        elif rs_hi < d2f < b_lo:
            assert R2[0] < exact <= R2[1]
        elif b_hi < d2f < rv_lo:
            assert R2[1] < exact <= R2[2]
        else:
            continue
        outside += 1
    assert outside > 100


def test_box_gap_never_exceeds_a_homes_distance():
    rng = np.random.default_rng(12)
    for trial in range(400):
        homes = rng.uniform(100, 100.5, size=(int(rng.integers(1, 9)), 3)).astype(np.float32)
        ps = (homes[0] + rng.normal(size=3).astype(np.float32) * np.float32(0.4)).astype(np.float32)
        lo, hi = homes.min(0), homes.max(0)
        gap = []
        for a in range(3):
            g1 = _round_f32(_f32(lo[a]) - _f32(ps[a]))
            g2 = _round_f32(_f32(ps[a]) - _f32(hi[a]))
            gap.append(max(g1, g2, Fraction(0)))
        bd2 = _round_f32(gap[2] * gap[2] + _round_f32(gap[1] * gap[1] + _round_f32(gap[0] * gap[0])))
        for h in homes:
            d = [_round_f32(_f32(h[a]) - _f32(ps[a])) for a in range(3)]
            d2 = _round_f32(d[2] * d[2] + _round_f32(d[1] * d[1] + _round_f32(d[0] * d[0])))
            assert bd2 <= d2
