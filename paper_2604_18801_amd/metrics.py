"""Cluster-membership query metrics (Sec. 4.1, "Metrics"), on host label
arrays (canonical FoF labels as returned by the library):

* membership errors: particles whose canonical label differs;
* the adjusted Rand index of the pairwise query same_halo(p_i, p_j), from the
  pair counts TP, TN, FP, FN over all particle pairs (the paper's formula);
* IoU_i = max_j |H_i ∩ H'_j| / |H_i ∪ H'_j| for every original halo H_i,
  summarised as the mass-weighted mean (MWM-IoU);
* the halo mass function dn/dlog10 M with equal-width log bins, and its
  pointwise relative error against the original's.

Halos for IoU and the HMF are the FoF components with at least
``min_members`` particles (default 20, the size threshold the paper cites);
the ARI counts every component, singletons included, and the decompressed
halos H'_j are all components.  Particle mass is uniform, so M_i = |H_i|.
"""
from typing import Dict, Tuple

import numpy as np


def _as_int64(lab) -> np.ndarray:
    try:
        import torch
        if isinstance(lab, torch.Tensor):
            lab = lab.cpu().numpy()
    except ImportError:
        pass
    return np.asarray(lab).astype(np.int64, copy=False)


def membership_errors(orig_labels, dec_labels) -> int:
    """Particles whose canonical (smallest member index) label differs."""
    a, b = _as_int64(orig_labels), _as_int64(dec_labels)
    return int(np.count_nonzero(a != b))


def contingency(orig_labels, dec_labels) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Non-empty cells (original label, decompressed label, particle count)."""
    a, b = _as_int64(orig_labels), _as_int64(dec_labels)
    if a.size == 0:
        z = np.zeros(0, np.int64)
        return z, z, z
    m = int(b.max()) + 1
    u, cnt = np.unique(a * m + b, return_counts=True)
    return u // m, u % m, cnt.astype(np.int64)


def _pairs(c) -> int:
    c = c.astype(object)
    return int(np.sum(c * (c - 1) // 2)) if len(c) else 0


def pair_counts(orig_labels, dec_labels) -> Dict[str, int]:
    """TP, FP, FN, TN over all unordered particle pairs (exact integers)."""
    a, b = _as_int64(orig_labels), _as_int64(dec_labels)
    n = int(a.size)
    total = n * (n - 1) // 2
    _, ca = np.unique(a, return_counts=True)
    _, cb = np.unique(b, return_counts=True)
    _, _, nij = contingency(a, b)
    tp = _pairs(nij)
    same_a, same_b = _pairs(ca), _pairs(cb)
    fn = same_a - tp  # together in the original, split after
    fp = same_b - tp  # apart in the original, merged after
    tn = total - tp - fp - fn
    return {"tp": tp, "fp": fp, "fn": fn, "tn": tn}


def ari(orig_labels, dec_labels) -> float:
    """2(TP TN - FP FN) / ((TP+FN)(FN+TN) + (TP+FP)(FP+TN)); 1 when both
    partitions are identical (including the degenerate all-one-cluster or
    all-singleton cases, where the fraction is 0/0)."""
    p = pair_counts(orig_labels, dec_labels)
    tp, fp, fn, tn = p["tp"], p["fp"], p["fn"], p["tn"]
    den = (tp + fn) * (fn + tn) + (tp + fp) * (fp + tn)
    if den == 0:
        return 1.0
    return float(2 * (tp * tn - fp * fn)) / float(den)


def mwm_iou(orig_labels, dec_labels, min_members: int = 20) -> float:
    """Mass-weighted mean over original halos (>= min_members) of the best
    IoU with any decompressed component; 1.0 if there is no such halo."""
    a, b = _as_int64(orig_labels), _as_int64(dec_labels)
    la, sa = np.unique(a, return_counts=True)
    lb, sb = np.unique(b, return_counts=True)
    ia, ib, nij = contingency(a, b)
    size_a = sa[np.searchsorted(la, ia)]
    size_b = sb[np.searchsorted(lb, ib)]
    iou = nij / (size_a + size_b - nij)
    keep = size_a >= min_members
    if not np.any(keep):
        return 1.0
    # best IoU per original halo: cells sorted by original label
    ia_k, iou_k, size_k = ia[keep], iou[keep], size_a[keep]
    starts = np.r_[0, np.flatnonzero(np.diff(ia_k)) + 1]
    best = np.maximum.reduceat(iou_k, starts)
    mass = size_k[starts].astype(np.float64)
    return float(np.sum(mass * best) / np.sum(mass))


def halo_masses(labels, min_members: int = 20) -> np.ndarray:
    _, s = np.unique(_as_int64(labels), return_counts=True)
    return s[s >= min_members]


def hmf(labels, volume: float, bins: int = 50, min_members: int = 20, mass_range=None):
    """(bin edges in log10 M, dn/dlog10 M): halo counts per equal-width
    log10 bin divided by the volume and the bin width."""
    m = halo_masses(labels, min_members).astype(np.float64)
    if mass_range is None:
        mass_range = (float(m.min()), float(m.max())) if m.size else (min_members, min_members + 1)
    lo, hi = np.log10(mass_range[0]), np.log10(mass_range[1])
    if hi <= lo:
        hi = lo + 1e-9
    edges = np.linspace(lo, hi, bins + 1)
    counts, _ = np.histogram(np.log10(m) if m.size else m, bins=edges)
    return edges, counts / (float(volume) * (edges[1] - edges[0]))


def hmf_relative_error(orig_labels, dec_labels, volume: float, bins: int = 50,
                       min_members: int = 20) -> Dict[str, float]:
    """Pointwise relative error of the decompressed HMF against the original's
    on the original's bins (bins where the original is non-empty)."""
    m0 = halo_masses(orig_labels, min_members)
    if m0.size == 0:
        return {"max_abs": 0.0, "mean_abs": 0.0, "bins": 0}
    rng = (float(m0.min()), float(m0.max()))
    _, h0 = hmf(orig_labels, volume, bins, min_members, rng)
    _, h1 = hmf(dec_labels, volume, bins, min_members, rng)
    ok = h0 > 0
    rel = np.abs(h1[ok] - h0[ok]) / h0[ok]
    return {"max_abs": float(rel.max()), "mean_abs": float(rel.mean()), "bins": int(ok.sum())}


def all_metrics(orig_labels, dec_labels, volume: float, bins: int = 50,
                min_members: int = 20) -> Dict[str, float]:
    h = hmf_relative_error(orig_labels, dec_labels, volume, bins, min_members)
    return {"membership_errors": membership_errors(orig_labels, dec_labels),
            "ari": ari(orig_labels, dec_labels),
            "mwm_iou": mwm_iou(orig_labels, dec_labels, min_members),
            "hmf_rel_err_max": h["max_abs"], "hmf_rel_err_mean": h["mean_abs"]}
