"""Pins of the oracle's edit stream and of the end-to-end guarantees.

The decoder is pinned by a stream assembled here byte by byte from the
format; the encoder by round trips; the whole method by its theorems:
zero membership errors, every coordinate within xi, VP link preservation.
"""
import struct

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
import bruteforce as bf
import synth
from stream_cases import huffman_stream


def _fof(pos, b, box):
    """FoF labels by a library neighbour search plus the exact predicate."""
    x = pos.astype(np.float64).T
    if any(v > 0 for v in box):
        L = np.array([v if v > 0 else 0 for v in box])
        xx = np.mod(x, np.where(L > 0, L, np.inf))
        tree = cKDTree(xx, boxsize=np.where(L > 0, L, 1e300))
    else:
        tree = cKDTree(x)
    cand = tree.query_pairs(b * (1 + 1e-6), output_type="ndarray")
    if len(cand) == 0:
        return np.arange(x.shape[0], dtype=np.int32)
    d = [bf.min_image(x[cand[:, 0], a] - x[cand[:, 1], a], box[a]) for a in range(3)]
    d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    keep = cand[d2 <= b * b]
    return bf.components(x.shape[0], keep[:, 0], keep[:, 1])


def test_decoder_on_hand_assembled_stream():
    rec = np.array([[1.0, 2.0, 3.0, 4.0, 5.0], [0.5] * 5, [-1.0] * 5], dtype=np.float32)
    n, m = 5, 8
    xi = 0.25
    step, offset = 4 * xi / (2 ** m - 1), 2 * xi
    flags = bytes([0b00010010])  # particles 1 and 4
    codes = {0: [0, 255], 1: [128, 127], 2: [200, 1]}  # per axis, per flagged particle
    sym = bytes(codes[0] + codes[1] + codes[2])
    payload = flags + sym
    hdr = struct.pack("<IHBBQQddQQII", 0x45434350, 2, m, 0, n, 2, step, offset,
                      len(payload), len(payload), 8, 0)
    out = oracle.decode(hdr + payload, rec)
    expect = rec.copy()
    for a in range(3):
        for k, pid in enumerate((1, 4)):
            expect[a, pid] = np.float32(float(rec[a, pid]) + codes[a][k] * step - offset)
    np.testing.assert_array_equal(out, expect)


def test_decoder_on_hand_assembled_huffman_stream():
    rec = np.array([[1.0, 2.0, 3.0, 4.0], [0.5] * 4, [-1.0] * 4], dtype=np.float32)
    stream, step, offset, codes = huffman_stream([0, 9])
    out = oracle.decode(stream, rec)
    expect = rec.copy()
    for a in range(3):
        for k, pid in enumerate((0, 3)):
            expect[a, pid] = np.float32(float(rec[a, pid]) + codes[a][k] * step - offset)
    np.testing.assert_array_equal(out, expect)


def test_decoder_rejects_a_wrong_chunk_start():
    rec = np.zeros((3, 4), np.float32)
    stream, *_ = huffman_stream([0, 8])
    with pytest.raises(ValueError):
        oracle.decode(stream, rec)


@pytest.mark.parametrize("m", [8, 16, 32])
def test_round_trip_error_within_quantiser_bound(m):
    w = synth.plain_blobs()
    r = oracle.correct(w.orig, w.recon, w.b, w.xi, mode="hf", m_bits=m)
    assert r.status == 0
    x = oracle.decode(r.stream, w.recon)
    c = oracle.constants(w.b, w.xi, m_bits=m,
                         maxabs=float(max(np.abs(w.orig).max(), np.abs(w.recon).max())))
    moved = np.any(r.p != w.recon.astype(np.float64), axis=0)
    assert moved.sum() == r.stats["n_flagged"]
    np.testing.assert_array_equal(x[:, ~moved], w.recon[:, ~moved])
    err = np.abs(x.astype(np.float64) - r.p)
    assert err.max() <= c["delta_q"]
    assert np.abs(x.astype(np.float64) - w.orig).max() <= w.xi


@pytest.mark.parametrize("mode", ["vp", "sc", "hf"])
def test_plain_workload_end_to_end_guarantees(mode):
    w = synth.plain_blobs()
    r = oracle.correct(w.orig, w.recon, w.b, w.xi, mode=mode)
    assert r.status == 0 and r.stats["viol_final"] == 0
    x = oracle.decode(r.stream, w.recon)
    l0 = _fof(w.orig, w.b, w.box)
    np.testing.assert_array_equal(r.labels, l0)
    np.testing.assert_array_equal(_fof(x, w.b, w.box), l0)
    assert np.abs(x.astype(np.float64) - w.orig).max() <= w.xi
    assert np.any(_fof(w.recon, w.b, w.box) != l0)  # the raw reconstruction is wrong
    if mode == "vp":
        c = oracle.constants(w.b, w.xi, maxabs=1.5)
        i, j, d2 = oracle.pairs(w.orig, w.box, c["rv2"])
        xx = x.astype(np.float64)
        e2 = ((xx[0][i] - xx[0][j]) ** 2 + (xx[1][i] - xx[1][j]) ** 2) + (xx[2][i] - xx[2][j]) ** 2
        np.testing.assert_array_equal(d2 <= c["b2"], e2 <= c["b2"])


def test_periodic_cosmology_sample_end_to_end():
    w = synth.cosmology(24, xi=0.05)
    r = oracle.correct(w.orig, w.recon, w.b, w.xi, mode="hf", box=w.box)
    assert r.status == 0
    x = oracle.decode(r.stream, w.recon)
    l0 = _fof(w.orig, w.b, w.box)
    np.testing.assert_array_equal(r.labels, l0)
    np.testing.assert_array_equal(_fof(x, w.b, w.box), l0)
    assert np.abs(x.astype(np.float64) - w.orig).max() <= w.xi


def test_input_outside_bound_is_rejected():
    w = synth.plain_blobs(1000, seed=5)
    bad = w.recon.copy()
    bad[0, 0] = w.orig[0, 0] + np.float32(2 * w.xi)
    with pytest.raises(ValueError):
        oracle.correct(w.orig, bad, w.b, w.xi)
