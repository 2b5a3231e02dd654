"""Iteration-capped corrections and their query metrics: the synthetic
analogue of the paper's truncated-budget study (Sec. 4.3, ARI / MWM-IoU /
HMF at an iteration cap).  For each mode and cap the snapshot is corrected
with max_iters = cap, the stream is decoded on the GPU, the decoded
positions are clustered by FoF on the GPU, and the clusters are compared
with those of the original positions.  Cap 0 is the raw reconstruction
(no correction); cap "full" runs to convergence.

    python -m paper_2604_18801_amd.quality --workload cosmo128 --modes hf,sc \\
        --caps 0,1,3,10,30,100,1000,full

prints one JSON line per (mode, cap).
"""
import argparse
import json
import sys
import time

import numpy as np

from . import metrics


def _volume(w) -> float:
    if all(L > 0 for L in w.box):
        return float(np.prod(w.box))
    ext = w.orig.max(axis=1).astype(np.float64) - w.orig.min(axis=1).astype(np.float64)
    return float(np.prod(np.maximum(ext, 1e-30)))


def study(ctx, w, modes=("hf",), caps=(0, 1, 3, 10, 30, 100, None), bins=50, min_members=20,
          trace=False, **opts):
    """Yields a row of metrics for every (mode, cap) as it is measured;
    cap None = to convergence (or the library's safety cap).  With trace,
    each row also holds the loss of Eq. 3 and the violation count at every
    evaluation (the loss-against-iteration curve)."""
    import torch
    o = torch.from_numpy(np.ascontiguousarray(w.orig)).cuda()
    r = torch.from_numpy(np.ascontiguousarray(w.recon)).cuda()
    vol = _volume(w)
    lab0 = ctx.fof_labels(o, w.b, w.box).cpu().numpy()
    if 0 in caps:
        lab = ctx.fof_labels(r, w.b, w.box).cpu().numpy()
        row = {"mode": "none", "cap": 0, "iters": 0, "status": None}
        row.update(metrics.all_metrics(lab0, lab, vol, bins, min_members))
        yield row
    for mode in modes:
        for cap in caps:
            if cap == 0:
                continue
            kw = dict(opts)
            if cap is not None:
                kw["max_iters"] = int(cap)
            torch.cuda.synchronize()
            t = time.perf_counter()
            if trace:
                kw["trace"] = (int(cap) + 1) if cap is not None else 100001
            stream, _, st = ctx.correct(o, r, w.b, w.xi, mode=mode, box=w.box, labels=False, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            x = ctx.decode_device(stream, r)
            lab = ctx.fof_labels(x, w.b, w.box).cpu().numpy()
            box_viol = int(torch.count_nonzero(torch.abs(x.double() - o.double()) > w.xi).item())
            row = {"mode": mode, "cap": "full" if cap is None else int(cap), "iters": st["iters"],
                   "status": st["status"], "viol0": st["viol0"], "viol_final": st["viol_final"],
                   "loss0": st["loss0"], "loss_final": st["loss_final"],
                   "n_active": st["n_active"], "stream_bytes": len(stream),
                   "ms": round(1e3 * dt, 2), "box_violations": box_viol}
            row.update(metrics.all_metrics(lab0, lab, vol, bins, min_members))
            if trace:
                row["loss_trace"] = [float(v) for v in st["loss_trace"]]
                row["viol_trace"] = [int(v) for v in st["viol_trace"]]
            yield row


def _workload(name):
    import synth
    if name.startswith("cosmo"):
        side = int(name[5:] or 128)
        return synth.cosmology(side, seed=1, xi=0.05)
    if name == "md":
        return synth.md_block(400000, seed=3_000_000)
    if name == "sph":
        return synth.sph_voids(400000, seed=5)
    if name == "plain":
        return synth.plain_blobs()
    raise SystemExit("unknown workload " + name)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="cosmo128")
    ap.add_argument("--modes", default="hf,sc,vp")
    ap.add_argument("--caps", default="0,1,3,10,30,100,300,1000",
                    help="comma-separated caps; 0 = raw reconstruction, full = no cap")
    ap.add_argument("--bins", type=int, default=50)
    ap.add_argument("--min-members", type=int, default=20)
    ap.add_argument("--optimizer", default="adam", choices=("adam", "sgd"))
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--trace", action="store_true",
                    help="add the per-evaluation loss and violation count to every row")
    args = ap.parse_args(argv)
    import paper_2604_18801_amd as pcc
    w = _workload(args.workload)
    caps = tuple(None if c == "full" else int(c) for c in args.caps.split(","))
    ctx = pcc.Context(0)
    try:
        for row in study(ctx, w, modes=tuple(args.modes.split(",")), caps=caps, bins=args.bins,
                         min_members=args.min_members, trace=args.trace,
                         optimizer=args.optimizer, lr=args.lr):
            row["workload"] = args.workload
            row["optimizer"] = args.optimizer
            print(json.dumps(row), flush=True)
    finally:
        ctx.close()


if __name__ == "__main__":
    sys.exit(main())
