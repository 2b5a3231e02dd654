"""Seeded generators for the synthetic workloads.

Every generator works in float64 and stores float32 (round to nearest even),
draws from ``numpy.random.default_rng(seed)`` and finally applies a seeded
random permutation so that particle order carries no spatial information.

The reconstruction that stands in for a base compressor's output is a uniform
grid quantiser of step 2*xi (an SZ-like linear quantiser with a zero predictor:
the worst case for clusters, because it collapses nearby particles onto the
same grid point).  Where float32 rounding would break the pointwise bound
|x_hat - x| <= xi, x_hat is stepped one float32 ulp towards x.

Workloads (sizes, distributions):
  * ``plain_blobs``   32,768 particles in the unit box, half uniform, half in
                      64 Gaussian blobs (sigma 0.01); b = 0.2/32, xi = 0.4 b.
  * ``cosmology``     n_side^3 particles in a periodic box of side n_side
                      (mean density 1): 60 % of the particles in halos whose
                      masses follow p(M) ~ M^-1.9 on [20, 20000] with an NFW
                      radial profile (concentration 5), the rest uniform.
  * ``md_block``      a Lennard-Jones-like vapour (0.02 / sigma^3) holding
                      liquid droplets (0.8 / sigma^3, jittered FCC lattice) of
                      log-normal radius; b = 1.5 sigma, xi = 0.05 sigma.
  * ``sph_voids``     a uniform fluid (density 1) with spherical voids of
                      radius 5 whose inside density is 1 % of the fluid's.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Optional, Tuple

import numpy as np

MODE_VP, MODE_SC, MODE_HF = 0, 1, 2


def _pieces(n: int, fn, piece: int = 1 << 18) -> None:
    """fn(a, b) over [0, n) in pieces, on threads (numpy releases the GIL).
    Only used for elementwise work, so the result does not depend on the
    split."""
    ranges = [(a, min(n, a + piece)) for a in range(0, n, piece)]
    if len(ranges) <= 1:
        for a, b in ranges:
            fn(a, b)
        return
    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex:
        for _ in ex.map(lambda r: fn(*r), ranges):
            pass


@dataclasses.dataclass
class Workload:
    name: str
    orig: np.ndarray          # (3, N) float32, C-contiguous (SoA x, y, z)
    recon: np.ndarray         # (3, N) float32, C-contiguous
    b: float                  # linking length
    xi: float                 # absolute pointwise error bound
    box: Tuple[float, float, float]  # periodic box side per axis, 0 = open
    mode: int = MODE_HF
    seed: int = 0
    meta: Dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.orig.shape[1])


# --------------------------------------------------------------------------
# reconstruction model
# --------------------------------------------------------------------------
def grid_reconstruction(orig: np.ndarray, xi: float) -> np.ndarray:
    """Grid quantiser of step 2*xi applied to float32 positions.

    Returns float32 positions with |x_hat - x| <= xi checked in float64.
    """
    orig = np.ascontiguousarray(orig)
    rec = np.empty_like(orig, dtype=np.float32)

    def work(a, b):
        o = orig[:, a:b]
        x64 = o.astype(np.float64)
        q = np.rint(x64 / (2.0 * xi))
        r = (q * (2.0 * xi)).astype(np.float32)
        bad = np.abs(r.astype(np.float64) - x64) > xi
        while bad.any():
            r[bad] = np.nextafter(r[bad], o[bad])
            bad = np.abs(r.astype(np.float64) - x64) > xi
        rec[:, a:b] = r

    _pieces(orig.shape[1], work)
    return rec


def _finish(name, pos64, rng, b, xi, box, mode, seed, meta, wrap=False):
    """Permute, store float32 SoA, build the reconstruction."""
    n = pos64.shape[0]
    perm = rng.permutation(n)
    orig = np.empty((3, n), dtype=np.float32)

    def work(a, b):
        o = pos64[perm[a:b]].T.astype(np.float32)
        if wrap:
            for k in range(3):
                L = np.float32(box[k])
                if L > 0:
                    # float32 rounding can land a wrapped value on L itself
                    o[k][o[k] >= L] -= L
                    o[k][o[k] < 0] += L
        orig[:, a:b] = o

    _pieces(n, work)
    recon = grid_reconstruction(orig, xi)
    return Workload(name=name, orig=orig, recon=recon, b=float(b), xi=float(xi),
                    box=tuple(float(v) for v in box), mode=mode, seed=seed,
                    meta=meta)


# --------------------------------------------------------------------------
# plain method workload
# --------------------------------------------------------------------------
def plain_blobs(n: int = 32768, seed: int = 0, n_blobs: int = 64,
                sigma: float = 0.01, xi_over_b: float = 0.4,
                mode: int = MODE_VP) -> Workload:
    rng = np.random.default_rng(seed)
    n_bg = n // 2
    n_bl = n - n_bg
    per = np.full(n_blobs, n_bl // n_blobs)
    per[: n_bl - per.sum()] += 1
    bg = rng.random((n_bg, 3))
    centres = rng.random((n_blobs, 3))
    blob = np.repeat(centres, per, axis=0) + rng.normal(0.0, sigma, (n_bl, 3))
    pos = np.concatenate([bg, blob])
    side = int(round(n ** (1.0 / 3.0)))
    b = 0.2 / side if side ** 3 == n else 0.2 * n ** (-1.0 / 3.0)
    xi = xi_over_b * b
    return _finish("plain_blobs_%d" % n, pos, rng, b, xi, (0.0, 0.0, 0.0), mode,
                   seed, {"n_blobs": n_blobs, "sigma": sigma})


# --------------------------------------------------------------------------
# cosmology-like workload
# --------------------------------------------------------------------------
def _nfw_mu(x):
    return np.log1p(x) - x / (1.0 + x)


def _halo_masses(rng, total: int, slope: float, mmin: float, mmax: float):
    """Power-law masses p(M) ~ M^-slope on [mmin, mmax] by inverse CDF,
    rounded, drawn until they hold ``total`` particles; the last is trimmed."""
    a = 1.0 - slope
    lo, hi = mmin ** a, mmax ** a
    out: List[np.ndarray] = []
    acc = 0
    while acc < total:
        u = rng.random(max(1024, int((total - acc) / 150) + 1024))
        m = np.rint((lo + u * (hi - lo)) ** (1.0 / a)).astype(np.int64)
        m = np.maximum(m, 1)
        out.append(m)
        acc += int(m.sum())
    m = np.concatenate(out)
    cs = np.cumsum(m)
    k = int(np.searchsorted(cs, total))  # first index with cs >= total
    m = m[: k + 1].copy()
    m[-1] -= int(cs[k] - total)
    return m


def cosmology(n_side: int = 256, seed: int = 1, xi: float = 0.05, b: float = 0.2,
              L: Optional[float] = None, n: Optional[int] = None,
              halo_frac: float = 0.6, slope: float = 1.9, mmin: float = 20,
              mmax: float = 20000, conc: float = 5.0, mode: int = MODE_HF,
              bisect_steps: int = 48) -> Workload:
    """Periodic cosmology-like snapshot at mean density 1.

    Halo particle radii solve mu(r/r_s) = u * mu(c) by bisection, with
    r_200 = (3 M / (4 pi 200))^(1/3) and r_s = r_200 / c.
    """
    if n is None:
        n = n_side ** 3
    if L is None:
        L = float(n) ** (1.0 / 3.0) if n != n_side ** 3 else float(n_side)
    rng = np.random.default_rng(seed)
    n_halo = int(round(halo_frac * n))
    masses = _halo_masses(rng, n_halo, slope, mmin, mmax)
    nh = masses.shape[0]
    centres = rng.random((nh, 3)) * L
    r200 = (3.0 * masses / (4.0 * math.pi * 200.0)) ** (1.0 / 3.0)
    rs = r200 / conc
    mu_c = _nfw_mu(conc)
    pos = np.empty((n, 3), dtype=np.float64)
    owner = np.repeat(np.arange(nh), masses)
    chunk = 1 << 22
    for s in range(0, n_halo, chunk):
        e = min(n_halo, s + chunk)
        # draws in a fixed order per chunk; the per-particle work below uses
        # no random numbers and runs on threads
        target = rng.random(e - s) * mu_c
        d = rng.normal(size=(e - s, 3))

        def work(a, b, s=s, target=target, d=d):
            h = owner[s + a:s + b]
            lo = np.zeros(b - a)
            hi = np.full(b - a, conc)
            tg = target[a:b]
            for _ in range(bisect_steps):
                mid = 0.5 * (lo + hi)
                below = _nfw_mu(mid) < tg
                lo = np.where(below, mid, lo)
                hi = np.where(below, hi, mid)
            r = 0.5 * (lo + hi) * rs[h]
            dd = d[a:b] / np.linalg.norm(d[a:b], axis=1, keepdims=True)
            pos[s + a:s + b] = np.mod(centres[h] + r[:, None] * dd, L)

        _pieces(e - s, work)
    pos[n_halo:] = rng.random((n - n_halo, 3)) * L
    return _finish("cosmology_%d" % n, pos, rng, b, xi, (L, L, L), mode, seed,
                   {"n_halos": int(nh), "L": L}, wrap=True)


# --------------------------------------------------------------------------
# molecular-dynamics-like workload
# --------------------------------------------------------------------------
def _within_any(p: np.ndarray, c: np.ndarray, r: np.ndarray, k: int = 8) -> np.ndarray:
    """For each point of p, whether |p - c_i| < r_i for some sphere i.  The
    distance is the same numpy expression for every (point, sphere) pair
    examined; a k-d tree only limits which pairs are examined (points with k
    or more spheres in reach are checked against all of them)."""
    out = np.zeros(p.shape[0], dtype=bool)
    if c.shape[0] == 0 or p.shape[0] == 0:
        return out
    from scipy.spatial import cKDTree
    kk = min(k, c.shape[0])
    _, idx = cKDTree(c).query(p, k=kk, distance_upper_bound=float(r.max()) * (1 + 1e-9) + 1e-9)
    idx = idx.reshape(p.shape[0], kk)
    valid = idx < c.shape[0]
    safe = np.where(valid, idx, 0)
    d = np.linalg.norm(p[:, None, :] - c[safe], axis=2)
    out = (valid & (d < r[safe])).any(axis=1)
    full = valid[:, -1]  # k spheres in reach: there may be more
    if full.any():
        q = p[full]
        hit = np.zeros(q.shape[0], dtype=bool)
        for s in range(0, c.shape[0], 64):
            dd = np.linalg.norm(q[:, None, :] - c[None, s:s + 64, :], axis=2)
            hit |= (dd < r[None, s:s + 64]).any(axis=1)
        out[full] = hit
    return out


def _random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def md_block(n: int, seed: int, b: float = 1.5, xi: float = 0.05,
             liquid_frac: float = 0.5, rho_l: float = 0.8, rho_v: float = 0.02,
             r_mu: float = math.log(8.0), r_s: float = 0.5, jitter: float = 0.05,
             mode: int = MODE_HF) -> Workload:
    """Vapour with liquid droplets on a jittered, randomly rotated FCC lattice."""
    rng = np.random.default_rng(seed)
    vol = n * (liquid_frac / rho_l + (1.0 - liquid_frac) / rho_v)
    L = vol ** (1.0 / 3.0)
    n_liq = int(round(liquid_frac * n))
    a = (4.0 / rho_l) ** (1.0 / 3.0)
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    drops_c: List[np.ndarray] = []
    drops_r: List[float] = []
    liquid: List[np.ndarray] = []
    have = 0
    while have < n_liq:
        R = float(np.exp(rng.normal(r_mu, r_s)))
        R = min(R, 0.45 * L)
        centre = None
        for _ in range(100):
            c = rng.uniform(R, L - R, 3)
            ok = True
            for c2, r2 in zip(drops_c, drops_r):
                if np.linalg.norm(c - c2) < R + r2 + 2.0 * b:
                    ok = False
                    break
            if ok:
                centre = c
                break
        if centre is None:
            centre = c
        k = int(math.ceil(R / a)) + 1
        g = np.arange(-k, k + 1)
        cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 1, 3)
        sites = ((cells + basis[None]) * a).reshape(-1, 3)
        sites = sites[np.linalg.norm(sites, axis=1) <= R]
        sites = sites @ _random_rotation(rng).T
        sites = sites + rng.normal(0.0, jitter, sites.shape)
        need = n_liq - have
        if sites.shape[0] > need:
            order = np.argsort(np.linalg.norm(sites, axis=1), kind="stable")
            sites = sites[order[:need]]
        liquid.append(sites + centre)
        drops_c.append(centre)
        drops_r.append(R)
        have += sites.shape[0]
    liq = np.concatenate(liquid) if liquid else np.zeros((0, 3))
    n_vap = n - liq.shape[0]
    dc = np.array(drops_c) if drops_c else np.zeros((0, 3))
    dr = np.array(drops_r) if drops_r else np.zeros(0)
    vap: List[np.ndarray] = []
    got = 0
    while got < n_vap:
        m = max(1024, int(1.3 * (n_vap - got)))
        p = rng.random((m, 3)) * L
        keep = ~_within_any(p, dc, dr + 1.0)
        p = p[keep][: n_vap - got]
        vap.append(p)
        got += p.shape[0]
    pos = np.concatenate([liq] + vap)
    return _finish("md_block_%d" % n, pos, rng, b, xi, (0.0, 0.0, 0.0), mode,
                   seed, {"n_droplets": len(drops_r), "L": L})


def md_batch_sizes(n_blocks: int = 256, seed: int = 3_000_000,
                   lo: float = 1e4, hi: float = 2e6) -> np.ndarray:
    """Log-uniform block sizes 10^U(log10 lo, log10 hi)."""
    rng = np.random.default_rng(seed)
    return np.rint(10.0 ** rng.uniform(math.log10(lo), math.log10(hi), n_blocks)).astype(np.int64)


# --------------------------------------------------------------------------
# SPH-like workload
# --------------------------------------------------------------------------
def sph_voids(n: int, seed: int, b: float = 0.2, xi: float = 0.05,
              void_r: float = 5.0, void_frac: float = 0.1, inside: float = 0.01,
              mode: int = MODE_HF) -> Workload:
    rng = np.random.default_rng(seed)
    L = float(n) ** (1.0 / 3.0)
    nv = max(1, int(round(void_frac * L ** 3 / (4.0 / 3.0 * math.pi * void_r ** 3))))
    vc = rng.random((nv, 3)) * L
    pts: List[np.ndarray] = []
    got = 0
    while got < n:
        m = max(1024, int(1.2 * (n - got)))
        p = rng.random((m, 3)) * L
        inv = _within_any(p, vc, np.full(nv, float(void_r)))
        keep = ~inv | (rng.random(m) < inside)
        p = p[keep][: n - got]
        pts.append(p)
        got += p.shape[0]
    pos = np.concatenate(pts)
    return _finish("sph_voids_%d" % n, pos, rng, b, xi, (0.0, 0.0, 0.0), mode,
                   seed, {"n_voids": nv, "L": L})


# --------------------------------------------------------------------------
# served job mix
# --------------------------------------------------------------------------
def served_jobs(n_jobs: int = 2000, seed: int = 4_000_000, median: float = 2e5,
                sigma: float = 1.0, lo: float = 1e4, hi: float = 1e7):
    """Job specs for the served stream: (kind, n, xi/b, mode, seed)."""
    rng = np.random.default_rng(seed)
    sizes = np.clip(np.rint(np.exp(rng.normal(math.log(median), sigma, n_jobs))), lo, hi).astype(np.int64)
    kinds = rng.integers(0, 3, n_jobs)
    ratio = rng.uniform(0.1, 0.5, n_jobs)
    modes = rng.integers(0, 3, n_jobs)
    return [dict(kind=("cosmology", "md", "sph")[int(k)], n=int(s), xi_over_b=float(r),
                 mode=int(m), seed=seed + j)
            for j, (k, s, r, m) in enumerate(zip(kinds, sizes, ratio, modes))]


def make_job(spec) -> Workload:
    n, kind = spec["n"], spec["kind"]
    if kind == "cosmology":
        b = 0.2
        return cosmology(n=n, seed=spec["seed"], b=b, xi=spec["xi_over_b"] * b,
                         mode=spec["mode"])
    if kind == "md":
        b = 1.5
        return md_block(n, spec["seed"], b=b, xi=spec["xi_over_b"] * b, mode=spec["mode"])
    b = 0.2
    return sph_voids(n, spec["seed"], b=b, xi=spec["xi_over_b"] * b, mode=spec["mode"])


# --------------------------------------------------------------------------
# sampling
# --------------------------------------------------------------------------
def sub_box(w: Workload, side: float, corner=(0.0, 0.0, 0.0)) -> Workload:
    """Particles of ``w`` whose original positions fall in a cube of the
    given side at ``corner``; the cut is treated as an open (non-periodic)
    domain.  Used for bounded samples of a large workload."""
    lo = np.asarray(corner, dtype=np.float64)[:, None]
    o = w.orig.astype(np.float64)
    sel = np.all((o >= lo) & (o < lo + side), axis=0)
    orig = np.ascontiguousarray(w.orig[:, sel])
    recon = np.ascontiguousarray(w.recon[:, sel])
    return Workload(name="%s_sub%g" % (w.name, side), orig=orig, recon=recon, b=w.b,
                    xi=w.xi, box=(0.0, 0.0, 0.0), mode=w.mode, seed=w.seed,
                    meta=dict(w.meta, sub_box=side))
