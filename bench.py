#!/usr/bin/env python3
"""Throughput benchmark: objects fitted per second on 64x64 Sersic stamps.

One step = the whole per-object pipeline (centroid, joint centroid +
ellipticity, 8-parameter Sersic fit) over one batch of synthetic stamps that
are already resident in GPU memory.  W untimed warm-up steps, then K timed
steps between two synchronisations.  Prints one JSON line on stdout; progress
goes to stderr.

    python bench.py [--steps K] [--warmup W] [--workload sersic64]

Extra fields: `roofline` for the fit kernel (timed with HIP events on the
stream it runs on), `cpu_baseline` (the FP64 oracle on a bounded sample of the
same workload, all host threads) and `parity` (GPU vs oracle on that sample).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work of one pixel in one LM sweep of the fit kernel (8 free
# parameters, Sersic): model + residual 31 FLOP, Jacobian 25, J^T r and chi^2
# 17, J^T J 63 (FMA = 2 FLOP), plus 4 transcendentals counted as 1 each.
FLOP_PER_PIXEL_SWEEP = {0xFF: 140.0}
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane-ops/s; one
# FP32 or FP64 FMA (2 FLOP) per lane-op without packed FP32 math.
ALU_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="sersic64")
    ap.add_argument("--count", type=int, default=None, help="stamps (default: the whole workload)")
    ap.add_argument("--cpu-sample", type=int, default=2048)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(stamps are independent; a shard per GPU would run the same kernels). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1203_0571_amd as shape
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    wl = synth.WORKLOADS[args.workload]
    t = time.time()
    batch = synth.make(args.workload, count=args.count)
    log("generated %d stamps of %s in %.1f s" % (batch.n, args.workload, time.time() - t))
    db = shape.DeviceBatch.from_host(batch, dev)
    opts = shape.default_opts()
    torch.cuda.synchronize()

    def step(events=None):
        rec0, _, _ = shape.centroid(db, opts)
        rec1, _, _ = shape.moments(db, rec0, opts)
        if events:
            events[0].record()
        fit = shape.fit_sersic(db, rec=rec1, opts=opts)
        if events:
            events[1].record()
        return fit

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        fit = step(evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fit_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    objs_per_s = batch.n * args.steps / elapsed
    log("%d steps in %.3f s: %.0f objects/s; fit kernel %.3f ms/launch"
        % (args.steps, elapsed, objs_per_s, fit_ms))

    sweeps = fit["sweeps"].cpu().numpy().astype(np.float64)
    status = fit["status"].cpu().numpy()
    npix = batch.sides.astype(np.float64) ** 2
    pixel_sweeps = float((sweeps * npix).sum())
    flops = pixel_sweeps * FLOP_PER_PIXEL_SWEEP[0xFF]
    achieved = flops / (fit_ms * 1e-3) / 1e12
    conv = float(((status & shape.ST_CONVERGED) != 0).mean())

    line = {
        "metric": "objects fitted/sec (64x64 Sersic stamps)",
        "value": round(objs_per_s, 1),
        "unit": "objects/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "stamps": batch.n,
                   "side": int(wl.side) if wl.side else "uneven", "storage": wl.storage,
                   "form": "plain", "free_params": 8, "max_iter_lm": opts.max_iter_lm,
                   "converged_fraction": round(conv, 4),
                   "mean_sweeps": round(float(sweeps.mean()), 3)},
        "roofline": {"bound": "alu", "kernel": "fit_kernel", "achieved": round(achieved, 3),
                     "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / ALU_PEAK_TFLOPS, 4), "traffic": None,
                     "launch_ms": round(fit_ms, 4),
                     "flop_per_pixel_sweep": FLOP_PER_PIXEL_SWEEP[0xFF],
                     "pixel_sweeps_per_launch": pixel_sweeps},
    }

    if not args.no_cpu:
        import oracle
        m = min(args.cpu_sample, batch.n)
        sub = synth.make(args.workload, count=m)
        oo = oracle.opts()
        t = time.perf_counter()
        ref = oracle.pipeline(sub, oo)
        cpu_s = time.perf_counter() - t
        line["cpu_baseline"] = {"value": round(m / cpu_s, 2), "unit": "objects/s",
                                "cores": int(ref["threads"]), "kind": "oracle",
                                "sample": "first %d stamps of %s, FP64 oracle, LM tol 1e-9, "
                                          "cap 200, %.1f s" % (m, args.workload, cpu_s)}
        g = {k: v[:m].cpu().numpy() for k, v in fit.items() if v is not None}
        both = ((g["status"] & shape.ST_CONVERGED) != 0) & \
               ((ref["status"][:, 2] & oracle.CONVERGED) != 0)
        d = np.abs(g["p"][both] - ref["p"][both])
        rel = np.abs(g["p"][both] / ref["p"][both] - 1)
        line["parity"] = {"sample": m, "both_converged": int(both.sum()),
                          "max_dxy_px": float(d[:, :2].max()) if both.any() else None,
                          "max_de": float(d[:, 2:4].max()) if both.any() else None,
                          "max_rel_re": float(rel[:, 4].max()) if both.any() else None,
                          "max_rel_n": float(rel[:, 5].max()) if both.any() else None,
                          "within_bars": float(((d[:, :2].max(1) <= 1e-3) &
                                                (d[:, 2:4].max(1) <= 1e-4) &
                                                (rel[:, 4:6].max(1) <= 1e-3)).mean())
                          if both.any() else None}
        log("cpu oracle: %d stamps in %.1f s on %d threads" % (m, cpu_s, ref["threads"]))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
