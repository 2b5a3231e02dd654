"""Pins of the oracle's correction loop (Alg. 1, Eq. 3, Sec. 4.2 Adam).

Two-particle problems reduce to a scalar recurrence written independently
below; loop-structure and special-case properties pin the rest.
"""
import math

import numpy as np
import pytest

import oracle
import bruteforce as bf
import synth


def _two(x0, x1, r0, r1):
    orig = np.array([[x0, x1], [0, 0], [0, 0]], dtype=np.float32)
    rec = np.array([[r0, r1], [0, 0], [0, 0]], dtype=np.float32)
    return orig, rec


def _scalar_run(x0, x1, r0, r1, b, xi, kind, steps, opt="adam", lr=1e-3,
                b1=0.9, b2=0.999, eps=1e-8):
    """1-D, two particles, particle 1 to the right of particle 0.
    kind 'pb': pull together while the gap exceeds b - delta_t;
    kind 'pc': push apart while the gap is at most b + delta_t.
    Returns the iterates, the number of steps and the tightened loss of Eq. 3
    at every evaluation (the squared overshoot of the one pair, 0 once it is
    satisfied)."""
    c = oracle.constants(b, xi, maxabs=max(abs(x0), abs(x1), abs(r0), abs(r1)))
    q = [float(np.float32(r0)), float(np.float32(r1))]
    lo = [float(np.float32(x0)) - c["xi_p"], float(np.float32(x1)) - c["xi_p"]]
    hi = [float(np.float32(x0)) + c["xi_p"], float(np.float32(x1)) + c["xi_p"]]
    m = [0.0, 0.0]
    v = [0.0, 0.0]
    t = 0
    traj = [list(q)]
    losses = []
    while True:
        gap = q[1] - q[0]
        if kind == "pb":
            viol = gap * gap > c["bm2"]
            h = gap - c["bm"]
            g = [-2.0 * h, 2.0 * h]        # d gap / d q0 = -1
        else:
            viol = gap * gap <= c["bp2"]
            h = c["bp"] - abs(gap)
            s = 1.0 if gap > 0 else (-1.0 if gap < 0 else 1.0)
            g = [2.0 * h * s, -2.0 * h * s]
        losses.append(h * h if viol else 0.0)
        if not viol or t >= steps:
            break
        t += 1
        for k in range(2):
            if opt == "sgd":
                q[k] = q[k] - lr * g[k]
            else:
                m[k] = b1 * m[k] + (1.0 - b1) * g[k]
                v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k]
                mh = m[k] / (1.0 - math.pow(b1, t))
                vh = v[k] / (1.0 - math.pow(b2, t))
                q[k] = q[k] - lr * mh / (math.sqrt(vh) + eps)
            q[k] = min(max(q[k], lo[k]), hi[k])
        traj.append(list(q))
    return traj, t, losses


@pytest.mark.parametrize("opt", ["adam", "sgd"])
def test_two_particle_pull_together(opt):
    x0, x1, r0, r1 = 0.0, 0.2421875, -0.015625, 0.2578125
    b, xi = 0.25, 0.02
    lr = 1e-3 if opt == "adam" else 2e-2
    traj, steps, losses = _scalar_run(x0, x1, r0, r1, b, xi, "pb", 10000, opt=opt, lr=lr)
    assert steps > 3
    orig, rec = _two(x0, x1, r0, r1)
    for k in (1, 2, steps // 2, steps):
        r = oracle.correct(orig, rec, b, xi, mode="vp", max_iters=k, optimizer=opt, lr=lr)
        np.testing.assert_allclose(r.p[0], traj[k], rtol=0, atol=1e-15)
        assert np.all(r.p[1:] == 0)
    r = oracle.correct(orig, rec, b, xi, mode="vp", optimizer=opt, lr=lr)
    assert r.status == 0 and r.iters == steps
    assert len(r.loss_hist) == steps + 1 and r.viol_hist[-1] == 0
    # Eq. 3 at every evaluation: the squared overshoot of the one pair
    np.testing.assert_allclose(r.loss_hist, losses, rtol=1e-15, atol=0)
    assert losses[0] > 0 and losses[-1] == 0.0
    assert r.stats["loss0"] == r.loss_hist[0] and r.stats["loss_final"] == 0.0


def test_first_adam_step_closed_form():
    # at t = 1 the bias-corrected moments are g and g^2: the step is
    # lr * g / (|g| + eps) for every coordinate
    x0, x1, r0, r1 = 0.0, 0.2421875, -0.015625, 0.2578125
    b, xi = 0.25, 0.02
    orig, rec = _two(x0, x1, r0, r1)
    c = oracle.constants(b, xi, maxabs=0.3)
    r = oracle.correct(orig, rec, b, xi, mode="vp", max_iters=1)
    g = 2.0 * ((r1 - r0) - c["bm"])
    step = 1e-3 * g / (g + 1e-8)
    np.testing.assert_allclose(r.p[0], [r0 + step, r1 - step], rtol=0, atol=1e-16)


def test_two_particle_push_apart_from_collapsed_point():
    # both reconstructed onto one point: the created pair has distance 0 and
    # is pushed apart along the original direction
    x0, x1, r0, r1 = 0.0, 0.28125, 0.140625, 0.140625
    b, xi = 0.25, 0.15
    orig, rec = _two(x0, x1, r0, r1)
    traj, steps, losses = _scalar_run(x0, x1, r0, r1, b, xi, "pc", 10000)
    assert steps > 3
    for k in (1, 3, steps):
        r = oracle.correct(orig, rec, b, xi, mode="vp", max_iters=k)
        np.testing.assert_allclose(r.p[0], traj[k], rtol=0, atol=1e-15)
    r = oracle.correct(orig, rec, b, xi, mode="vp")
    assert r.iters == steps and r.status == 0
    np.testing.assert_allclose(r.loss_hist, losses, rtol=1e-15, atol=0)
    # at the collapsed start the overshoot is the whole of b + delta_t
    c = oracle.constants(b, xi, maxabs=0.3)
    assert r.loss_hist[0] == c["bp"] ** 2


def test_no_violation_means_no_iteration_and_no_edit():
    w = synth.plain_blobs(4096, seed=3)
    # exact reconstruction with a tiny bound: no pair is near the threshold
    r = oracle.correct(w.orig, w.orig, w.b, 1e-9, mode="vp")
    assert r.iters == 0 and r.status == 0
    assert r.stats["n_flagged"] == 0 and len(r.loss_hist) == 1
    assert np.all(r.p == w.orig.astype(np.float64))
    x = oracle.decode(r.stream, w.orig)
    np.testing.assert_array_equal(x, w.orig)


def test_exact_reconstruction_violates_only_pairs_within_margin():
    w = synth.plain_blobs(4096, seed=4)
    r = oracle.correct(w.orig, w.orig, w.b, w.xi, mode="vp", max_iters=1)
    c = oracle.constants(w.b, w.xi, maxabs=float(np.abs(w.orig).max()))
    i, j, d2 = bf.all_pairs(w.orig, w.box, c["rv2"])
    pb = (d2 > c["rs2"]) & (d2 <= c["b2"]) if c["rs"] > 0 else (d2 <= c["b2"])
    pc = (d2 > c["b2"])
    expect = int(np.sum(pb & (d2 > c["bm2"])) + np.sum(pc & (d2 <= c["bp2"])))
    assert r.stats["viol0"] == expect
    # Eq. 3 over the exhaustive pair list: each violated potentially broken
    # link adds (d - (b - delta_t))^2, each violated potentially created pair
    # ((b + delta_t) - d)^2
    d = np.sqrt(d2)
    h = np.concatenate([(d - c["bm"])[pb & (d2 > c["bm2"])], (c["bp"] - d)[pc & (d2 <= c["bp2"])]])
    assert h.size == expect and np.all(h >= 0)
    loss = math.fsum((h * h).tolist())
    assert loss > 0
    assert abs(r.stats["loss0"] - loss) <= 1e-12 * loss
    assert r.loss_hist[0] == r.stats["loss0"]


def test_loss_tolerance_stops_at_the_first_evaluation_below_it():
    # Alg. 1's eps_L: the loop ends at the first iterate whose tightened loss
    # is <= eps_L; up to there the run is the one without a tolerance
    w = synth.plain_blobs(4096, seed=5)
    full = oracle.correct(w.orig, w.recon, w.b, w.xi, mode="hf", box=w.box)
    assert full.status == 0 and full.iters > 10
    hist = np.asarray(full.loss_hist)
    k = full.iters // 2
    tol = float(np.sqrt(hist[k - 1] * hist[k])) if hist[k] < hist[k - 1] else float(hist[k])
    stop = int(np.argmax(hist <= tol))
    assert 0 < stop <= k
    r = oracle.correct(w.orig, w.recon, w.b, w.xi, mode="hf", box=w.box, loss_tol=tol)
    assert r.status == 0 and r.iters == stop
    assert r.stats["loss_final"] == hist[stop] <= tol
    np.testing.assert_array_equal(np.asarray(r.loss_hist), hist[:stop + 1])
    capped = oracle.correct(w.orig, w.recon, w.b, w.xi, mode="hf", box=w.box, max_iters=stop)
    np.testing.assert_array_equal(r.p, capped.p)


def test_iteration_cap_reports_not_converged_inside_the_box():
    w = synth.plain_blobs()
    r = oracle.correct(w.orig, w.recon, w.b, w.xi, mode="vp", max_iters=5)
    assert r.status == 1 and r.iters == 5 and r.stats["viol_final"] > 0
    c = oracle.constants(w.b, w.xi, maxabs=float(max(np.abs(w.orig).max(), np.abs(w.recon).max())))
    dev = np.abs(r.p[:, r.e_ids] - w.orig[:, r.e_ids].astype(np.float64))
    # the clamp bounds x -+ xi' are themselves rounded to double
    assert dev.max() <= c["xi_p"] + 4 * np.spacing(np.float64(np.abs(w.orig).max()))
    assert len(r.loss_hist) == 6
