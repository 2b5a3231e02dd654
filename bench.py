#!/usr/bin/env python3
"""Benchmark of the correction pass on one MI355X.

A step is one full correction (cell build, pair passes and components,
constraint selection, editable set and CSR, PGD to convergence, edit
encoding including the host ZSTD stage) of one synthetic snapshot whose
inputs are already in HBM.  Default workload: the cosmology-like snapshot of
512^3 particles (periodic L = 512, 60 % in halos, b = 0.2, xi = 0.05),
halo-forest mode: the largest configuration that fits one GPU.  The value is
particles per second over the timed steps; it counts only when the decoded
stream has zero membership errors and no coordinate outside the error bound
(checked after the timed region).

After the headline, within a time budget, the same JSON line gathers:
  * xi_sweep     the same snapshot at xi = 0.02 and 0.1 (reconstruction
                 regenerated per xi), one call each;
  * batched_md   all 256 blocks of the batched MD workload in one batched
                 call (sizes 10^U(4, log10 2e6) atoms, 9.6e7 in total);
  * served       the first J jobs of the 2,000-job served stream with the
                 stream's own VP / SC / HF draw, Poisson arrivals at 0.7 of
                 the closed-loop job rate: p50 / p99 latency and particles/s;
  * cpu_baseline the oracle (plain single-threaded C) on the same generator
                 at 96^3 (periodic), and on the 32,768-particle plain
                 workload in all three modes.

Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "corrected particles/s at zero membership errors; p50/p99 job latency (served)"
T0 = time.perf_counter()


def log(*a):
    print("[bench %6.1fs]" % (time.perf_counter() - T0), *a, file=sys.stderr, flush=True)


def elapsed():
    return time.perf_counter() - T0


def snapshot(name):
    import synth
    if name == "cosmo256":
        return synth.cosmology(256, seed=1, xi=0.05), "cosmology-like 256^3, periodic L=256, b=0.2, xi=0.05"
    if name == "cosmo128":
        return synth.cosmology(128, seed=1, xi=0.05), "cosmology-like 128^3, periodic L=128, b=0.2, xi=0.05"
    if name == "plain":
        return synth.plain_blobs(), "plain 32768 particles, unit box, 64 blobs, b=0.2/32, xi=0.4b"
    if name.startswith("cosmo512"):
        xi = float(name.split("_")[1]) if "_" in name else 0.05
        return synth.cosmology(512, seed=2, xi=xi), "cosmology-like 512^3, periodic L=512, b=0.2, xi=%g" % xi
    raise SystemExit("unknown workload " + name)


def with_xi(w, xi):
    """The same originals with the reconstruction regenerated for xi."""
    import dataclasses
    import synth
    return dataclasses.replace(w, xi=float(xi), recon=synth.grid_reconstruction(w.orig, xi))


# algorithmic bytes of all launches of a kernel in one step
def kernel_bytes(name, st, n):
    if name == "pgd_step":
        # per evaluated row: position read and write (24 + 24 B), original
        # position (12 B), Adam moments read and written (96 B), row pointer
        # (4 B); per evaluated incidence: its column entry (4 B)
        return 160 * st["pgd_rows_evaluated"] + 4 * st["pgd_incidences_evaluated"]
    if name in ("pair_classify", "pair_count", "pair_write"):
        # sorted positions (16 B) and cell index (4 B) per particle, plus
        # the per-particle counts or the written pairs
        base = 20 * n + 4 * n
        if name == "pair_write":
            base += 9 * st["n_active"]
        return base
    return None


def recorded(kernel, what):
    """A per-launch figure from the committed rocprofv3 counter runs
    (profiles/traffic.json), if the kernel's source is unchanged since they
    were taken (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path)).get(kernel)
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, ValueError, KeyError, TypeError, AttributeError):
        return None
    if hashlib.sha1(src).hexdigest() != rec["source_sha1"]:
        return None
    if what == "traffic":
        return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    return rec.get(what)


def verify(ctx, w, stream, labels, bs=None):
    """Membership errors of the decoded stream (summed over the linking
    lengths bs when several were corrected; labels then has one row each)
    and box violations."""
    import numpy as np
    import torch
    import paper_2604_18801_amd as pcc
    x = pcc.decode(stream, w.recon)
    box_viol = int(np.count_nonzero(np.abs(x.astype(np.float64) - w.orig.astype(np.float64)) > w.xi))
    xd = torch.from_numpy(x).cuda()
    if bs is None:
        memb = int((ctx.fof_labels(xd, w.b, w.box) != labels).sum().item())
    else:
        memb = 0
        for k, b in enumerate(bs):
            memb += int((ctx.fof_labels(xd, b, w.box) != labels[k]).sum().item())
    del xd
    return memb, box_viol


def _percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def _verify_many(ctx, ws, results):
    """Membership errors and box violations summed over jobs (decoded stream,
    FoF of the decoded positions on the GPU against the labels)."""
    memb = boxv = 0
    for w, (status, stream, lab, st) in zip(ws, results):
        if status < 0 or w.n == 0:
            continue
        m, bv = verify(ctx, w, stream, lab)
        memb += m
        boxv += bv
    return memb, boxv


def _oracle_labels_check(ws, results, picks):
    """Labels of the picked jobs against the oracle's FoF (plain C on the
    host, independent of the library)."""
    import numpy as np
    import oracle
    bad = 0
    for k in picks:
        lab = results[k][2]
        lab = lab.cpu().numpy() if hasattr(lab, "cpu") else lab
        bad += int(np.count_nonzero(lab != oracle.fof_labels(ws[k].orig, ws[k].b, ws[k].box)))
    return bad


def tune(ctx, jobs, args, graph=True):
    """Autotuner (outside the timed region): the chosen scheduling knobs and
    the spread of the trials, or None with --no-autotune."""
    if args.no_autotune:
        return None
    t = time.perf_counter()
    rep = ctx.autotune(jobs, graph=graph)
    pair = [x["ms"] for x in rep["trials"] if x["kind"] == "pre_pgd_stages"]
    full = [x["ms"] for x in rep["trials"] if x["kind"] == "correction"]
    out = {"cell_pct": rep["cell_pct"], "dense_cell": rep["dense_cell"],
           "graph_iters": rep["graph_iters"],
           "pre_pgd_stages_ms": [round(min(pair), 2), round(max(pair), 2)] if pair else None,
           "correction_ms": [round(min(full), 2), round(max(full), 2)] if full else None,
           "trials": len(rep["trials"]), "s": round(time.perf_counter() - t, 2)}
    log("autotune: %s" % out)
    return out


# --------------------------------------------------------------------------
# generation of the many-job workloads in worker processes (before any GPU
# use in this process); every job is a pure function of its seed
# --------------------------------------------------------------------------
def _gen_md(arg):
    import synth
    n, seed = arg
    return synth.md_block(int(n), int(seed))


def _gen_served(spec):
    import synth
    return synth.make_job(spec)


def generate_many(fn, items, what):
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    t = time.perf_counter()
    workers = max(1, min(16, os.cpu_count() or 1, len(items)))
    out = []
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
        for k, w in enumerate(ex.map(fn, items, chunksize=1)):
            out.append(w)
            if (k + 1) % 64 == 0:
                log("  %s: %d of %d generated" % (what, k + 1, len(items)))
    log("generated %d %s (%d particles) in %.1f s on %d processes" % (
        len(out), what, sum(w.n for w in out), time.perf_counter() - t, workers))
    return out


# --------------------------------------------------------------------------
# the parts of the line
# --------------------------------------------------------------------------
def copy_probe(mib):
    """A plain device-to-device copy timed with HIP events: the achievable
    HBM ceiling beside the 8 TB/s peak (and the counter calibration)."""
    import torch
    nel = mib * (1 << 20) // 4
    src = torch.ones(nel, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 5
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return {"bytes_read": nel * 4, "bytes_written": nel * 4, "ms": round(ms, 3),
            "gbs": round(2 * nel * 4 / (ms / 1e3) / 1e9, 1),
            "frac_of_peak": round(2 * nel * 4 / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def snapshot_line(ctx, w, desc, args, bs=None):
    """The headline: K timed corrections of one resident snapshot."""
    import torch
    o = torch.from_numpy(w.orig).cuda()
    r = torch.from_numpy(w.recon).cuda()
    torch.cuda.synchronize()

    def step(mode=args.mode, **kw):
        if args.max_iters and "max_iters" not in kw:
            kw["max_iters"] = args.max_iters
        if bs:
            return ctx.correct_multi(o, r, bs, w.xi, mode=mode, box=w.box, **kw)
        return ctx.correct(o, r, w.b, w.xi, mode=mode, box=w.box, **kw)

    tjob = dict(orig=o, recon=r, b=w.b, xi=w.xi, mode=args.mode, box=w.box,
                opts={"max_iters": args.max_iters} if args.max_iters else {})
    # the graph length stays at its default here: the timed steps then launch
    # the PGD kernels exactly as the profiled run does
    tuned = tune(ctx, [tjob], args, graph=False) if not bs else None
    for k in range(args.warmup):
        t = time.perf_counter()
        _, _, st = step()
        log("warmup %d: %.1f ms, iters %d, status %d" % (k, 1e3 * (time.perf_counter() - t),
                                                          st["iters"], st["status"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.steps):
        stream, labels, st = step()
        stats.append(st)
        log("step %d: iters %d active %d editable %d flagged %d stream %d B" % (
            k, st["iters"], st["n_active"], st["n_editable"], st["n_flagged"], len(stream)))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = 1e3 * el / max(1, args.steps)
    value = w.n * args.steps / el

    # dominant kernel and its roofline
    kms, klaunch = {}, {}
    for st in stats:
        for name, v in st["kernel_ms"].items():
            kms[name] = kms.get(name, 0.0) + v
            klaunch[name] = klaunch.get(name, 0) + st["kernel_launches"][name]
    roofline = None
    if kms and max(kms.values()) > 0:
        dom = max(kms, key=kms.get)
        avg_s = kms[dom] / 1e3 / max(1, klaunch[dom])
        per_step = [kernel_bytes(dom, st, w.n) for st in stats]
        nbytes = None if None in per_step else sum(per_step) / max(1, klaunch[dom])
        if nbytes is not None and avg_s > 0:
            ach = nbytes / avg_s / 1e9
            tb = recorded(dom, "traffic")
            roofline = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                        "traffic": int(tb) if tb else None, "bytes_per_launch": int(nbytes),
                        "avg_launch_us": round(avg_s * 1e6, 2), "launches": int(klaunch[dom])}
        else:
            roofline = {"kernel": dom, "bound": "alu", "achieved": None, "peak": None,
                        "unit": None, "frac": None, "traffic": None,
                        "avg_launch_us": round(avg_s * 1e6, 2)}
    last = stats[-1]
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generator; no dataset)",
        "config": {"workload": desc, "n": w.n, "mode": args.mode, "b": bs or w.b, "xi": w.xi,
                   "max_iters": args.max_iters or None, "parallelism": "single GPU"},
        "status": last["status"], "iters": last["iters"], "n_active": last["n_active"],
        "n_editable": last["n_editable"], "n_flagged": last["n_flagged"],
        "pgd_rows_evaluated": last["pgd_rows_evaluated"],
        "pgd_incidences_evaluated": last["pgd_incidences_evaluated"],
        "stream_bytes": last["bytes_stream"],
        "autotune": tuned,
        "stage_ms": {k: round(v, 3) for k, v in last["t_stage_ms"].items()},
        "kernel_ms_per_step": {k: round(v / len(stats), 3) for k, v in kms.items()},
        # algorithmic GB/s of every kernel whose bytes per unit are defined
        "kernel_gbs": {k: round(sum(kernel_bytes(k, s, w.n) for s in stats) / (kms[k] / 1e3) / 1e9, 1)
                       for k in kms if kms[k] > 0 and kernel_bytes(k, stats[0], w.n) is not None},
        "roofline": roofline,
    }
    # VALU use of the pair passes (they are bound by candidate tests in the
    # halo cores, not by HBM): from the committed counter run, if current
    valu = {k: recorded(k, "valu") for k in ("pair_classify", "pair_write")}
    out["pair_pass_valu"] = {k: v for k, v in valu.items() if v} or None
    if not args.no_verify:
        memb, boxv = verify(ctx, w, stream, labels, bs)
        out["membership_errors"] = memb
        out["box_violations"] = boxv
        if memb or boxv or last["status"] != 0:
            out["value_valid"] = False
        log("verified: membership errors %d, box violations %d" % (memb, boxv))
    del o, r
    torch.cuda.synchronize()
    return out


def one_call(ctx, w, mode, max_iters, verify_it=True, warm=False):
    """One correction of a snapshot (optionally after an untimed one)."""
    import torch
    o = torch.from_numpy(w.orig).cuda()
    r = torch.from_numpy(w.recon).cuda()
    kw = {"max_iters": max_iters} if max_iters else {}
    if warm:
        ctx.correct(o, r, w.b, w.xi, mode=mode, box=w.box, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter()
    s, lab, st = ctx.correct(o, r, w.b, w.xi, mode=mode, box=w.box, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    e = {"xi": w.xi, "mode": mode, "max_iters": max_iters or None, "status": st["status"],
         "iters": st["iters"], "n_active": st["n_active"], "viol0": st["viol0"],
         "viol_final": st["viol_final"], "ms": round(1e3 * dt, 2),
         "particles_per_s": round(w.n / dt, 1), "warm_arena": bool(warm),
         "stage_ms": {k: round(v, 2) for k, v in st["t_stage_ms"].items()}}
    if verify_it:
        e["membership_errors"], e["box_violations"] = verify(ctx, w, s, lab)
    del o, r
    return e


def batched_line(ctx, ws, args):
    """All blocks in one pcc_correct_batch call: a step is that call."""
    import torch
    total = int(sum(w.n for w in ws))
    kw = {"max_iters": args.max_iters} if args.max_iters else {}
    jobs = [dict(orig=torch.from_numpy(w.orig).cuda(), recon=torch.from_numpy(w.recon).cuda(),
                 b=w.b, xi=w.xi, mode=args.md_mode, box=w.box, opts=kw) for w in ws]
    torch.cuda.synchronize()
    tuned = tune(ctx, jobs, args)
    for k in range(args.md_warmup):
        t = time.perf_counter()
        ctx.correct_batch(jobs)
        log("batched MD warmup %d: %.1f ms" % (k, 1e3 * (time.perf_counter() - t)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.md_steps):
        res = ctx.correct_batch(jobs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    statuses = [r[0] for r in res]
    out = {"value": round(total * args.md_steps / el, 1), "unit": "particles/s",
           "ms_per_step": round(1e3 * el / args.md_steps, 3), "steps": args.md_steps,
           "warmup": args.md_warmup,
           "workload": "batched MD: blocks 0..%d of the 256-block batch (sizes 10^U(4, log10 2e6)), "
                       "droplets on FCC in vapour, b=1.5, xi=0.05, non-periodic" % (len(ws) - 1),
           "blocks": len(ws), "atoms": total, "mode": args.md_mode, "autotune": tuned,
           "iters_max": int(max(r[3]["iters"] for r in res)),
           "not_converged": int(sum(1 for s in statuses if s == 1)),
           "failed": int(sum(1 for s in statuses if s < 0))}
    if not args.no_verify:
        out["membership_errors"], out["box_violations"] = _verify_many(ctx, ws, res)
        picks = sorted(set([0, len(ws) // 3, (2 * len(ws)) // 3, len(ws) - 1]))
        picks = [k for k in picks if ws[k].n <= 300_000] or [min(range(len(ws)), key=lambda k: ws[k].n)]
        out["oracle_label_mismatches"] = _oracle_labels_check(ws, res, picks)
        out["oracle_checked_blocks"] = picks
        if out["membership_errors"] or out["box_violations"] or out["failed"] \
                or out["oracle_label_mismatches"]:
            out["value_valid"] = False
    del jobs
    torch.cuda.synchronize()
    return out


def served_line(ctx, ws, specs, args):
    """Served stream: the jobs are device-resident.  A closed-loop pass (all
    jobs submitted at once) gives the sustained job rate mu; the timed pass
    submits the same jobs at Poisson arrivals of rate args.rate * mu.
    Latency = finish - arrival per job."""
    import numpy as np
    import torch
    import paper_2604_18801_amd as pcc
    total = int(sum(w.n for w in ws))
    modes = [int(w.mode) for w in ws]
    jobs = []
    for w in ws:
        # Adam's step in units of b: the paper's alpha = 1e-3 at b = 0.2 of
        # the mean spacing, i.e. alpha = 0.005 b (MD lengths are in sigma)
        kw = {"lr": 0.005 * w.b}
        if args.served_max_iters:
            kw["max_iters"] = args.served_max_iters
        jobs.append(dict(orig=torch.from_numpy(w.orig).cuda(), recon=torch.from_numpy(w.recon).cuda(),
                         b=w.b, xi=w.xi, mode=int(w.mode), box=w.box, opts=kw))
    torch.cuda.synchronize()
    srv = pcc.Server(ctx)

    def run(arrivals):
        # one loop submits the jobs that are due and collects the finished
        # ones (progress every 10 s)
        t_start = time.perf_counter()
        tickets, done = [], {}
        last = t_start
        while len(done) < len(jobs):
            now = time.perf_counter() - t_start
            while len(tickets) < len(jobs) and (arrivals is None or arrivals[len(tickets)] <= now):
                tickets.append(srv.submit(**jobs[len(tickets)]))
            for k, tk in enumerate(tickets):
                if k not in done:
                    r = srv.poll(tk)
                    if r is not None:
                        done[k] = r
            if time.perf_counter() - last > 10.0:
                last = time.perf_counter()
                log("  %d submitted, %d of %d finished after %.1f s" % (
                    len(tickets), len(done), len(jobs), last - t_start))
            time.sleep(0.005)
        return [done[k] for k in range(len(jobs))]

    t = time.perf_counter()
    res = run(None)
    closed = time.perf_counter() - t
    mu = len(jobs) / closed
    log("served closed loop: %d jobs in %.2f s (%.2f jobs/s)" % (len(jobs), closed, mu))
    lam = args.rate * mu
    rng = np.random.default_rng(4_000_001)
    arrivals = np.cumsum(rng.exponential(1.0 / lam, len(jobs)))
    t = time.perf_counter()
    res = run(arrivals)
    el = time.perf_counter() - t
    lat = [r[3]["t_finish_ms"] - r[3]["t_submit_ms"] for r in res]
    statuses = [r[0] for r in res]
    lat_mode = {}
    for k, m in enumerate(("vp", "sc", "hf")):
        lm = [x for x, md in zip(lat, modes) if md == k]
        if lm:
            lat_mode[m] = {"jobs": len(lm), "p50": round(_percentile(lm, 50), 2),
                           "p99": round(_percentile(lm, 99), 2)}
    out = {"value": round(total / el, 1), "unit": "particles/s", "ms": round(1e3 * el, 3),
           "workload": "served stream: jobs 0..%d of the 2000-job mix (cosmology-like, MD, "
                       "SPH-like; sizes LogNormal(ln 2e5, 1) clipped to [1e4, 1e7]; xi = b U(0.1, "
                       "0.5); modes drawn from VP/SC/HF)" % (len(jobs) - 1),
           "jobs": len(jobs), "particles": total, "arrival_rate_frac": args.rate,
           "adam_lr": "0.005 b", "max_iters": args.served_max_iters or 100000,
           "latency_ms": {"p50": round(_percentile(lat, 50), 2),
                          "p99": round(_percentile(lat, 99), 2), "max": round(max(lat), 2)},
           "latency_ms_by_mode": lat_mode,
           "closed_loop_jobs_per_s": round(mu, 3), "arrival_jobs_per_s": round(lam, 3),
           "mean_batch_jobs": round(float(np.mean([r[3]["batch_jobs"] for r in res])), 2),
           "iters_by_mode": {m: int(max([r[3]["iters"] for r, md in zip(res, modes) if md == k]
                                        or [0])) for k, m in enumerate(("vp", "sc", "hf"))},
           "not_converged": int(sum(1 for s in statuses if s == 1)),
           "failed": int(sum(1 for s in statuses if s < 0)),
           "parallelism": "single GPU, server"}
    srv.close()
    if args.detail:
        with open(args.detail, "w") as f:
            for s, w, r in zip(specs, ws, res):
                f.write(json.dumps({"kind": s["kind"], "n": w.n, "xi_over_b": round(s["xi_over_b"], 3),
                                    "mode": int(w.mode), "status": r[0], "iters": r[3]["iters"],
                                    "viol0": r[3]["viol0"], "viol_final": r[3]["viol_final"],
                                    "n_active": r[3]["n_active"],
                                    "latency_ms": round(r[3]["t_finish_ms"] - r[3]["t_submit_ms"], 2)})
                        + "\n")
    if not args.no_verify:
        out["membership_errors"], out["box_violations"] = _verify_many(ctx, ws, res)
        conv = [k for k in range(len(ws)) if statuses[k] == 0]
        capped = [k for k in range(len(ws)) if statuses[k] == 1]
        out["membership_errors_converged_jobs"] = _verify_many(
            ctx, [ws[k] for k in conv], [res[k] for k in conv])[0]
        out["membership_errors_capped_jobs"] = _verify_many(
            ctx, [ws[k] for k in capped], [res[k] for k in capped])[0]
        small = [k for k in range(len(ws)) if ws[k].n <= 200_000]
        picks = small[:: max(1, len(small) // 4)][:4]
        out["oracle_label_mismatches"] = _oracle_labels_check(ws, res, picks)
        out["oracle_checked_jobs"] = picks
        if out["membership_errors"] or out["box_violations"] or out["failed"] \
                or out["oracle_label_mismatches"]:
            out["value_valid"] = False
    del jobs
    torch.cuda.synchronize()
    return out


def cpu_baseline(side):
    """The oracle (plain single-threaded C, as it stands) on the same
    generator at a bounded size, periodic like the headline workload, HF."""
    import oracle
    import synth
    w = synth.cosmology(side, seed=2, xi=0.05)
    t0 = time.perf_counter()
    r = oracle.correct(w.orig, w.recon, w.b, w.xi, mode="hf", box=w.box)
    dt = time.perf_counter() - t0
    return {"value": round(w.n / dt, 1), "unit": "particles/s", "cores": 1, "kind": "oracle",
            "host_nproc": os.cpu_count(),
            "sample": "cosmology-like %d^3 (%d particles, periodic L=%d, the 512^3 generator's "
                      "density and halo mix), b=0.2, xi=0.05, HF, %d iterations, status %d, "
                      "%.2f s on one thread" % (side, w.n, side, r.iters, r.status, dt)}


def cpu_baseline_plain():
    import oracle
    import synth
    w = synth.plain_blobs()
    out = {}
    for m in ("vp", "sc", "hf"):
        t0 = time.perf_counter()
        r = oracle.correct(w.orig, w.recon, w.b, w.xi, mode=m, box=w.box)
        dt = time.perf_counter() - t0
        out[m] = {"particles_per_s": round(w.n / dt, 1), "s": round(dt, 3), "iters": r.iters,
                  "status": r.status}
    return {"workload": "plain 32768 particles, unit box, 64 blobs, b=0.2/32, xi=0.4b",
            "cores": 1, "kind": "oracle", "modes": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cosmo512",
                    help="headline snapshot (cosmo512[_xi], cosmo256, cosmo128, plain), or "
                         "md_batch / served alone")
    ap.add_argument("--mode", default="hf")
    ap.add_argument("--quick", action="store_true", help="the headline only")
    ap.add_argument("--time-budget", type=float, default=420.0,
                    help="extras are skipped (and say so) once this many seconds have passed")
    ap.add_argument("--xi-sweep", default="0.02,0.1",
                    help="cosmo512: also run these xi once each ('' for none)")
    ap.add_argument("--sweep-max-iters", type=int, default=1000)
    ap.add_argument("--cpu-side", type=int, default=96)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=2048,
                    help="size of the timed device copy (0: none)")
    ap.add_argument("--md-blocks", type=int, default=256,
                    help="batched MD: blocks 0..K-1 of the 256-block batch (0: skip)")
    ap.add_argument("--md-steps", type=int, default=2)
    ap.add_argument("--md-warmup", type=int, default=1)
    ap.add_argument("--md-mode", default="hf")
    ap.add_argument("--jobs", type=int, default=120,
                    help="served: first J jobs of the stream (0: skip)")
    ap.add_argument("--rate", type=float, default=0.7,
                    help="served: arrival rate as a fraction of the closed-loop job rate")
    ap.add_argument("--served-max-iters", type=int, default=2000,
                    help="served: per-job iteration cap (0: the library's safety cap)")
    ap.add_argument("--max-iters", type=int, default=0,
                    help="headline iteration cap (0: the library's safety cap)")
    ap.add_argument("--detail", default="", help="served: write one JSON row per job here")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default scheduling knobs instead of autotuning them first")
    ap.add_argument("--thresholds", default="",
                    help="comma-separated linking lengths: correct the snapshot for all of "
                         "them at once (pcc_correct_multi)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the correction pass is built and measured on a "
              "single MI355X here (multi-GPU sharding is a design note only); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.quick:
        args.xi_sweep, args.md_blocks, args.jobs, args.no_cpu_baseline = "", 0, 0, True
    alone = args.workload in ("md_batch", "served")

    # ---- inputs, all generated before this process touches the GPU ----
    import synth
    head = None
    if not alone:
        t = time.perf_counter()
        head = snapshot(args.workload)
        log("generated %s: n=%d in %.1f s" % (args.workload, head[0].n, time.perf_counter() - t))
    sweep = []
    if not alone and args.workload.startswith("cosmo512") and args.xi_sweep and not args.thresholds:
        for xi in [float(v) for v in args.xi_sweep.split(",") if v]:
            if xi != head[0].xi:
                sweep.append(with_xi(head[0], xi))
        log("reconstructions for xi %s ready" % [w.xi for w in sweep])
    md = []
    if args.workload == "md_batch" or (not alone and args.md_blocks > 0):
        sizes = synth.md_batch_sizes()[: (args.md_blocks or 32)]
        md = generate_many(_gen_md, [(int(n), 3_000_000 + k) for k, n in enumerate(sizes)],
                           "MD blocks")
    served, specs = [], []
    if args.workload == "served" or (not alone and args.jobs > 0):
        specs = synth.served_jobs(2000)[: (args.jobs or 120)]
        served = generate_many(_gen_served, specs, "served jobs")

    import torch  # noqa: F401
    import paper_2604_18801_amd as pcc
    ctx = pcc.Context(0)
    if not args.no_kernel_timing:
        ctx.set_option("kernel_timing", 1)

    if alone:
        if args.workload == "md_batch":
            body = batched_line(ctx, md, args)
        else:
            body = served_line(ctx, served, specs, args)
        out = {"metric": METRIC, "value": body.pop("value"), "unit": body.pop("unit"),
               "n_gpus": 1, "steps": body.get("steps", 1), "warmup": body.get("warmup", 1),
               "ms_per_step": body.get("ms_per_step", body.get("ms")), "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic (seeded generator; no dataset)",
               "config": {"workload": body.pop("workload"), "parallelism": "single GPU"},
               "roofline": None, "cpu_baseline": None}
        out.update(body)
        ctx.close()
        print(json.dumps(out), flush=True)
        return

    probe = copy_probe(args.copy_probe_mib) if args.copy_probe_mib > 0 else None
    if probe:
        log("copy probe: %s" % probe)
    w, desc = head
    bs = [float(v) for v in args.thresholds.split(",")] if args.thresholds else None
    if bs:
        desc += "; corrected at linking lengths %s at once" % ",".join("%g" % v for v in bs)
    out = snapshot_line(ctx, w, desc, args, bs)
    if probe:
        out["copy_probe"] = probe
    log("headline %.1f M particles/s (%.1f ms per correction)" % (out["value"] / 1e6,
                                                                   out["ms_per_step"]))

    def budget(what):
        if elapsed() > args.time_budget:
            log("skipping %s: %.0f s elapsed, budget %.0f s" % (what, elapsed(), args.time_budget))
            return {"skipped": "time budget (%.0f s elapsed of %.0f)" % (elapsed(), args.time_budget)}
        return None

    if sweep:
        res = {}
        for ws in sweep:
            res["%g" % ws.xi] = budget("xi=%g" % ws.xi) or one_call(
                ctx, ws, args.mode, args.sweep_max_iters, not args.no_verify, warm=ws.xi < 0.05)
            log("xi %g: %s" % (ws.xi, res["%g" % ws.xi]))
        out["xi_sweep"] = res
        del sweep
    if md:
        out["batched_md"] = budget("batched MD") or batched_line(ctx, md, args)
        log("batched MD: %s" % {k: v for k, v in out["batched_md"].items() if k != "autotune"})
        del md
    if served:
        out["served"] = budget("served") or served_line(ctx, served, specs, args)
        log("served: %s" % out["served"])
        del served
    ctx.close()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) on the %d^3 snapshot" % args.cpu_side)
        out["cpu_baseline"] = cpu_baseline(args.cpu_side)
        out["cpu_baseline_plain"] = cpu_baseline_plain()
    else:
        out["cpu_baseline"] = None
    log("done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
