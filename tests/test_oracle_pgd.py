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
                b1=0.9, b2=0.999, eps=1e-8, patience=0):
    """1-D, two particles, particle 1 to the right of particle 0.
    kind 'pb': pull together while the gap exceeds b - delta_t;
    kind 'pc': push apart while the gap is at most b + delta_t."""
    c = oracle.constants(b, xi, maxabs=max(abs(x0), abs(x1), abs(r0), abs(r1)))
    q = [float(np.float32(r0)), float(np.float32(r1))]
    lo = [float(np.float32(x0)) - c["xi_p"], float(np.float32(x1)) - c["xi_p"]]
    hi = [float(np.float32(x0)) + c["xi_p"], float(np.float32(x1)) + c["xi_p"]]
    m = [0.0, 0.0]
    v = [0.0, 0.0]
    t = 0
    traj = [list(q)]
    best, stall, scale = None, 0, 1.0
    while t < steps:
        gap = q[1] - q[0]
        if kind == "pb":
            if not gap * gap > c["bm2"]:
                break
            h = gap - c["bm"]
            g = [-2.0 * h, 2.0 * h]        # d gap / d q0 = -1
        else:
            if not gap * gap <= c["bp2"]:
                break
            h = c["bp"] - abs(gap)
            s = 1.0 if gap > 0 else (-1.0 if gap < 0 else 1.0)
            g = [2.0 * h * s, -2.0 * h * s]
        # plateau rule: one violated pair per evaluation here, so alpha is
        # halved after every `patience` evaluations that follow the first;
        # the verdict of this evaluation applies from the next step on
        step = lr * scale
        if patience > 0:
            if best is None:
                best, stall = 1, 0
            else:
                stall += 1
                if stall >= patience:
                    scale, stall = scale * 0.5, 0
        t += 1
        for k in range(2):
            if opt == "sgd":
                q[k] = q[k] - step * g[k]
            else:
                m[k] = b1 * m[k] + (1.0 - b1) * g[k]
                v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k]
                mh = m[k] / (1.0 - math.pow(b1, t))
                vh = v[k] / (1.0 - math.pow(b2, t))
                q[k] = q[k] - step * mh / (math.sqrt(vh) + eps)
            q[k] = min(max(q[k], lo[k]), hi[k])
        traj.append(list(q))
    return traj, t


@pytest.mark.parametrize("opt", ["adam", "sgd"])
def test_two_particle_pull_together(opt):
    x0, x1, r0, r1 = 0.0, 0.2421875, -0.015625, 0.2578125
    b, xi = 0.25, 0.02
    lr = 1e-3 if opt == "adam" else 2e-2
    traj, steps = _scalar_run(x0, x1, r0, r1, b, xi, "pb", 10000, opt=opt, lr=lr)
    assert steps > 3
    orig, rec = _two(x0, x1, r0, r1)
    for k in (1, 2, steps // 2, steps):
        r = oracle.correct(orig, rec, b, xi, mode="vp", max_iters=k, optimizer=opt, lr=lr)
        np.testing.assert_allclose(r.p[0], traj[k], rtol=0, atol=1e-15)
        assert np.all(r.p[1:] == 0)
    r = oracle.correct(orig, rec, b, xi, mode="vp", optimizer=opt, lr=lr)
    assert r.status == 0 and r.iters == steps
    assert len(r.loss_hist) == steps + 1 and r.viol_hist[-1] == 0


@pytest.mark.parametrize("opt", ["adam", "sgd"])
def test_plateau_rule_halves_the_step(opt):
    # the optional plateau rule against the scalar recurrence (one violated
    # pair: alpha halves every `patience` evaluations until it is satisfied);
    # a patience longer than the run leaves the paper's trajectory unchanged
    x0, x1, r0, r1 = 0.0, 0.2421875, -0.015625, 0.2578125
    b, xi = 0.25, 0.02
    lr = 1e-3 if opt == "adam" else 2e-2
    plain, psteps = _scalar_run(x0, x1, r0, r1, b, xi, "pb", 20000, opt=opt, lr=lr)
    patience = 2 * psteps // 3 + 1
    traj, steps = _scalar_run(x0, x1, r0, r1, b, xi, "pb", 20000, opt=opt, lr=lr,
                              patience=patience)
    assert 20000 > steps > psteps > 3
    orig, rec = _two(x0, x1, r0, r1)
    for k in sorted({1, patience, patience + 1, steps // 2, steps}):
        r = oracle.correct(orig, rec, b, xi, mode="vp", max_iters=k, optimizer=opt, lr=lr,
                           lr_patience=patience)
        np.testing.assert_allclose(r.p[0], traj[k], rtol=0, atol=1e-15)
    r = oracle.correct(orig, rec, b, xi, mode="vp", optimizer=opt, lr=lr, lr_patience=patience)
    assert r.status == 0 and r.iters == steps
    a = oracle.correct(orig, rec, b, xi, mode="vp", optimizer=opt, lr=lr, lr_patience=10 ** 6)
    z = oracle.correct(orig, rec, b, xi, mode="vp", optimizer=opt, lr=lr)
    np.testing.assert_array_equal(a.p, z.p)
    assert a.iters == z.iters == psteps


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
    traj, steps = _scalar_run(x0, x1, r0, r1, b, xi, "pc", 10000)
    assert steps > 3
    for k in (1, 3, steps):
        r = oracle.correct(orig, rec, b, xi, mode="vp", max_iters=k)
        np.testing.assert_allclose(r.p[0], traj[k], rtol=0, atol=1e-15)
    r = oracle.correct(orig, rec, b, xi, mode="vp")
    assert r.iters == steps and r.status == 0


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


def test_iteration_cap_reports_not_converged_inside_the_box():
    w = synth.plain_blobs()
    r = oracle.correct(w.orig, w.recon, w.b, w.xi, mode="vp", max_iters=5)
    assert r.status == 1 and r.iters == 5 and r.stats["viol_final"] > 0
    c = oracle.constants(w.b, w.xi, maxabs=float(max(np.abs(w.orig).max(), np.abs(w.recon).max())))
    dev = np.abs(r.p[:, r.e_ids] - w.orig[:, r.e_ids].astype(np.float64))
    # the clamp bounds x -+ xi' are themselves rounded to double
    assert dev.max() <= c["xi_p"] + 4 * np.spacing(np.float64(np.abs(w.orig).max()))
    assert len(r.loss_hist) == 6
