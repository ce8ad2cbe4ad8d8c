#!/usr/bin/env python3
"""Throughput benchmark: objects fitted per second on 64x64 Sersic stamps.

Workload: 262,144 stamps of 64x64 Sersic galaxies (n U(0.5,4), Re log-U(1.5,6),
e_i N(0,0.25) with |e| < 0.7, flux log-U(1e3,1e5), S/N log-U(20,200), sky 10),
seed 0.  Forms timed on the same stamps, all resident in GPU memory:

  plain       FP32 stamps; centroid, moments and the fused fit, 3 launches
  f16         FP16 stamps with a per-stamp power-of-two scale, same launches
  f16_queue   FP16 stamps; centroid, moments, then the work-queue fit with one
              hipGraph replay per LM iteration

One step = the whole per-object pipeline over all stamps.  W untimed warm-up
steps, then K timed steps between two synchronisations.  `value` is the form
with the most objects/s among those whose parity sample meets the bars; every
form is reported under config.forms.  Prints one JSON line on stdout; progress
goes to stderr.

Extra fields: `roofline` for the chosen form's fit kernel (its launch time from
HIP events on the stream it runs on), `cpu_baseline` (the FP64 oracle on a
bounded sample, all host threads) and `parity` (GPU vs oracle per form).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work of one pixel in one LM sweep of the fit (8 free
# parameters, Sersic), FMA = 2 FLOP, a transcendental 1: offsets and
# elliptical radius 9, profile 4 + 3 transcendentals, residual 3, Jacobian 24
# + 1 transcendental (a shared factor dm/dR^2, the N u products, eight
# columns), J^T J 63, J^T r and chi^2 17.
FLOP_PER_PIXEL_SWEEP = 124.0
# The same sweep in the moment form the row layout takes (a batch of one side
# dividing 64, 8 free parameters): R^2 in units of Re^2 along the column 5,
# profile 7 + 3 transcendentals, n column 3, residual 3, H_j = h u2^j 2,
# chi^2 and the gradient sums 15, the x0..e2 block's five moments 10, their
# sums against the Re, n, I0 and sky columns 21, the Re, n, I0, sky block 15
# -> 82 (the per-lane recombination once per sweep is not counted, as the
# reduction is not).
FLOP_PER_PIXEL_SWEEP_MOMENT = 82.0
# The adjoint's FP64 sweeps in the moment form (64 x 64 stamps): chi^2 and the
# gradient only -- R^2 4, profile 7 with 3 transcendentals, h (reciprocal and
# k7) 3, Re and n columns 4, residual 3, H_j 2, chi^2 2, the gradient sums 13,
# the row step 1 -> 39 (61 for the direct columns: the 124 above without
# J^T J); with J^T J as well (the LM's normal matrix) 86.
FLOP_PER_PIXEL_GRAD_MOMENT = 39.0
FLOP_PER_PIXEL_GRAD_DIRECT = 61.0
FLOP_PER_PIXEL_GRAD_JTJ_MOMENT = 86.0
# An a-priori estimate of the same work, made before the sweep was written:
# about 85 VALU operations per pixel and sweep, 150 FLOP with FMA = 2.
FLOP_PER_PIXEL_SWEEP_ESTIMATE = 150.0
# Per pixel per iteration of the other stages (FMA = 2, transcendental = 1):
# centroid sweep: offsets 2, R^2 3, weight 2, f W 2, three sums 5 -> 14;
# moments sweep: offsets 2, products 3, R^2 5, weight 2, f W 2, eleven
# moment sums 21 -> 35; star step (R^2 and f formed once per pixel): weight
# 5 (Moffat) or 2 (Gaussian), products 3, three sums 3 -> 11 (Moffat).
FLOP_PER_PIXEL_CENTROID = 14.0
FLOP_PER_PIXEL_MOMENTS = 35.0
FLOP_PER_PIXEL_STAR_MOFFAT = 11.0
# The 4-parameter sweep (Re, n free, I0 and sky columns): offsets and radius
# 9, profile 4 + 3 transcendentals, residual 3, Jacobian columns for Re and n
# 4, J^T J 15, J^T r and chi^2 9.
FLOP_PER_PIXEL_SWEEP_4 = 47.0
# MI355X HBM3E: 8 TB/s.
HBM_PEAK_GBS = 8000.0
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane-ops/s; one
# FP32 or FP64 FMA (2 FLOP) per lane-op without packed FP32 math.
ALU_PEAK_TFLOPS = 78.6
BARS = dict(x=1e-3, e=1e-4, rel=1e-3)


# Sources that make up the fit kernel and the frame detection; the HBM
# counters in profiles/ are used only while these are unchanged.
FIT_SOURCES = ["paper_1203_0571_amd/csrc/fit.hip", "paper_1203_0571_amd/csrc/lm.hpp",
               "paper_1203_0571_amd/csrc/sweep.hpp", "paper_1203_0571_amd/csrc/common.hpp",
               "paper_1203_0571_amd/csrc/bn_table.h", "paper_1203_0571_amd/csrc/kernels.hpp",
               "include/shape.h", "paper_1203_0571_amd/build.py"]
FRAME_SOURCES = ["paper_1203_0571_amd/csrc/frames.hip", "paper_1203_0571_amd/csrc/common.hpp",
                 "paper_1203_0571_amd/csrc/bn_table.h", "paper_1203_0571_amd/csrc/kernels.hpp",
                 "include/shape.h", "paper_1203_0571_amd/build.py"]
# Counter summaries holding the fit's FETCH_SIZE / WRITE_SIZE per workload
TRAFFIC_FILES = {"sersic64h": os.path.join(ROOT, "profiles", "fit_sersic64h_hbm_traffic.md"),
                 "plain48": os.path.join(ROOT, "profiles", "pipeline_plain48_counters.md"),
                 "uneven": os.path.join(ROOT, "profiles", "pipeline_uneven_counters.md")}
FRAME_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "frame_detect_frames512_hbm_traffic.md")


def sources_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(path, files, form=""):
    """HBM bytes per launch from a committed counter summary (FETCH_SIZE and
    WRITE_SIZE in KiB, each scaled by its copy calibration), or None if the
    summary is missing or the kernel's sources changed since it was taken."""
    try:
        text = open(path).read()
    except OSError:
        return None
    kv = {}
    for line in text.splitlines():
        if ":" in line and line.startswith("    "):
            k, v = line.strip().split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256_16") != sources_hash(files):
        return None
    sfx = "_" + form if form else ""
    if "fetch_kib" + sfx not in kv:
        return None
    return (float(kv["fetch_kib" + sfx]) * float(kv["fetch_scale"]) +
            float(kv["write_kib" + sfx]) * float(kv["write_scale"])) * 1024.0


def counter_kv(path, files):
    """The key: value block of a committed counter summary, or None if it is
    missing or the kernel's sources changed since the counters were taken."""
    try:
        text = open(path).read()
    except OSError:
        return None
    kv = {}
    for line in text.splitlines():
        if ":" in line and line.startswith("    "):
            k, v = line.strip().split(":", 1)
            kv[k.strip()] = v.strip()
    return kv if kv.get("source_sha256_16") == sources_hash(files) else None


VALU_FILE = os.path.join(ROOT, "profiles", "fit_sersic64h_valu.md")


def fit_valu_issue(form):
    """The 64 x 64 fit's measured VALU issue (wave64 instructions per SIMD per
    four cycles, from its committed counters) for the given form, or None."""
    kv = counter_kv(VALU_FILE, FIT_SOURCES)
    v = kv.get("valu_issue_" + form) if kv else None
    return float(v) if v is not None else None


def fit_traffic_bytes(workload, form):
    """HBM bytes per launch of the fit of `workload` in the given form (None
    where no counters were taken for that pair)."""
    path = TRAFFIC_FILES.get(workload)
    return counter_traffic(path, FIT_SOURCES, form) if path else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fit_parity_block(fit, ref, batch, m, mask=0xFF):
    """GPU fit vs the FP64 oracle on the first m stamps, by the parity rule of
    tests/parity_util.py: bars on stamps both sides fit to the interior,
    chi^2 / sigma_p / amplitudes there, every disagreement validated as a
    minimum of the oracle's chi^2 no worse than the oracle's."""
    import numpy as np
    from parity_util import fit_parity
    g = {k: v[:m].cpu().numpy() for k, v in fit.items() if hasattr(v, "cpu")}
    g["status"] = np.stack([np.zeros(m, np.uint32), np.zeros(m, np.uint32),
                            g["status"].astype(np.uint32)], 1)
    st, failures = fit_parity(g, ref, batch, mask)
    st.pop("alternatives", None)
    st["failures"] = len(failures)
    st["rule"] = ("bars |dxy|<=1e-3 px, |de|<=1e-4, rel Re,n<=1e-3 on stamps both fit to the "
                  "interior; chi^2, sigma_p, I0, sky checked there; each stamp outside the bars "
                  "must be a validated minimum of the oracle chi^2")
    return st


def sigma_units(p_a, p_b, perr, mask, both):
    """|p_a - p_b| / sigma_p over the fitted parameters on stamps `both`:
    p50, p99, max per parameter."""
    import numpy as np
    names = ["x0", "y0", "e1", "e2", "Re", "n", "I0", "sky"]
    out = {}
    for k in range(8):
        if not (mask >> k) & 1:
            continue
        z = np.abs(p_a[both, k] - p_b[both, k]) / perr[both, k]
        z = z[np.isfinite(z)]
        if z.size:
            out[names[k]] = [float(np.percentile(z, 50)), float(np.percentile(z, 99)),
                             float(z.max())]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--count", type=int, default=None, help="stamps (default: the whole workload)")
    ap.add_argument("--forms", default="plain,f16,f16_queue")
    ap.add_argument("--cpu-sample", type=int, default=16384)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration)")
    ap.add_argument("--workload", default="sersic64h",
                    choices=["sersic64h", "plain48", "uneven", "stars32", "frames512", "plain32x",
                             "sersic64"],
                    help="plain48: 100,000 48x48 Sersic stamps, 8-parameter fit, cap 30; "
                         "uneven: 1,000,000 stamps of side 16-128 (80%% Sersic, 20%% Moffat), "
                         "fused fit vs autotuned work queue; stars32: 1,048,576 32x32 Moffat "
                         "stars, sizes from weighted moments; frames512: 4,096 512x512 frames, "
                         "detection and 6 r50 cut-outs; plain32x: 262,144 32x32 Gaussian "
                         "galaxies, 4-parameter fit profiled vs unprofiled; sersic64: 65,536 "
                         "64x64 stamps, chi^2 forward and adjoint gradient")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(stamps are independent; a shard per GPU would run the same kernels). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import synth

    if args.workload == "uneven":
        return bench_uneven(args)
    if args.workload == "stars32":
        return bench_stars(args)
    if args.workload == "frames512":
        return bench_frames(args)
    if args.workload == "plain32x":
        return bench_profiled(args)
    if args.workload == "sersic64":
        return bench_adjoint(args)
    wl = args.workload      # sersic64h (FP16 + FP32 copies) or plain48 (FP32)
    side = 64 if wl == "sersic64h" else 48
    forms = [f for f in args.forms.split(",") if f]
    if wl == "plain48":
        forms = [f.replace("f16_queue", "queue") for f in forms if f != "f16"]
    # Stamps are generated (in worker processes) before this process touches
    # the GPU, so no worker is forked from a process with an initialised runtime.
    b16 = b32 = None
    n = 0
    if not args.copy_calibration:
        t = time.time()
        if any(f.startswith("f16") for f in forms):
            b16 = synth.make(wl, count=args.count)
        if "plain" in forms or "queue" in forms:
            b32 = synth.make(wl, count=args.count, storage="f32")
        n = (b16 or b32).n
        log("generated %d stamps (%dx%d) in %.1f s" % (n, side, side, time.time() - t))

    import torch

    import paper_1203_0571_amd as shape
    from paper_1203_0571_amd import autotune

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of %d bytes (read %d, write %d per copy)"
            % (nbytes, nbytes, nbytes))
        return

    opts = shape.default_opts()
    dbs = {}
    if b32 is not None:
        dbs["f32"] = shape.DeviceBatch.from_host(b32, dev)
    if b16 is not None:
        dbs["f16"] = shape.DeviceBatch.from_host(b16, dev)
    torch.cuda.synchronize()
    storage = {"plain": "f32", "queue": "f32", "f16": "f16", "f16_queue": "f16"}
    tuned = {}
    for form in forms:
        if form.endswith("queue"):
            db = dbs[storage[form]]
            r0, _, _ = shape.centroid(db, opts)
            r1, _, _ = shape.moments(db, r0, opts)
            t = time.time()
            tuned[form] = autotune.tune_queue(db, r1, opts, use_cache=False)
            log("autotune %s %.1f s: team %d, grid %d, drain at %.2f" % (
                form, time.time() - t, tuned[form]["cfg"].team, tuned[form]["cfg"].grid,
                tuned[form]["drain_frac"]))

    def step(form, events=None, want_perr=False):
        db = dbs[storage[form]]
        rec0, _, _ = shape.centroid(db, opts)
        rec1, _, _ = shape.moments(db, rec0, opts)
        if events:
            events[0].record()
        if form.endswith("queue"):
            fit = shape.fit_queue(db, rec=rec1, opts=opts, cfg=tuned[form]["cfg"], use_graph=True,
                                  drain_at=int(tuned[form]["drain_frac"] * n),
                                  want_perr=want_perr)
        else:
            fit = shape.fit_sersic(db, rec=rec1, opts=opts, want_perr=want_perr)
        if events:
            events[1].record()
        return fit

    results = {}
    for form in forms:
        for _ in range(args.warmup):
            step(form)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        t0 = time.perf_counter()
        for k in range(args.steps):
            fit = step(form, evs[k])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        fit_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        sweeps = fit["sweeps"].cpu().numpy().astype(np.float64)
        status = fit["status"].cpu().numpy()
        pixel_sweeps = float(sweeps.sum()) * side * side
        results[form] = dict(elapsed=elapsed, fit_ms=fit_ms, objs=n * args.steps / elapsed,
                             pixel_sweeps=pixel_sweeps,
                             conv=float(((status & shape.ST_CONVERGED) != 0).mean()),
                             mean_sweeps=float(sweeps.mean()))
        log("%-10s %d steps in %.3f s: %.0f objects/s; fit %.3f ms/step, %.4f converged"
            % (form, args.steps, elapsed, results[form]["objs"], fit_ms, results[form]["conv"]))
    # outputs with sigma_p for the parity leg (untimed)
    for form in forms:
        results[form]["fit"] = step(form, want_perr=True)
    torch.cuda.synchronize()

    par, cpu = {}, None
    if not args.no_cpu:
        import oracle
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        m = min(args.cpu_sample, n)
        refs, heads = {}, {}
        for key, bb in (("f16", b16), ("f32", b32)):
            if bb is None:
                continue
            heads[key] = bb.head(m)
            t = time.perf_counter()
            refs[key] = oracle.pipeline(heads[key], oracle.opts())
            cpu_s = time.perf_counter() - t
            log("cpu oracle (%s pixels): %d stamps in %.1f s on %d threads"
                % (key, m, cpu_s, refs[key]["threads"]))
            if cpu is None:
                cpu = {"value": round(m / cpu_s, 2), "unit": "objects/s",
                       "cores": int(refs[key]["threads"]), "kind": "oracle",
                       "sample": "first %d stamps of the workload (%s pixels, as FP64), FP64 "
                                 "oracle pipeline, LM tol 1e-9, cap 200, %.1f s"
                                 % (m, "FP16-stored" if key == "f16" else "FP32", cpu_s)}
        if cpu is not None:
            # the same oracle on one thread, comparable with the paper's
            # single-core timings (0.1 s centroid + ellipticity, 0.5 s fit per
            # object on a 2.2 GHz CPU, Sec. 4.1)
            m1 = min(1024, m)
            t = time.perf_counter()
            oracle.pipeline((b16 or b32).head(m1), oracle.opts(), threads=1)
            s1 = time.perf_counter() - t
            cpu["one_thread"] = {"value": round(m1 / s1, 2), "unit": "objects/s",
                                 "sample": "first %d stamps, %.1f s" % (m1, s1)}
            log("cpu oracle, one thread: %d stamps in %.1f s" % (m1, s1))
        done = {}
        for form in forms:
            key = storage[form]
            fit = results[form]["fit"]
            same = next((f for f in done if storage[f] == key and all(
                torch.equal(fit[k], results[f]["fit"][k]) for k in ("p", "chi2", "status"))), None)
            if same:
                par[form] = dict(par[same], identical_to=same)
                continue
            t = time.perf_counter()
            par[form] = fit_parity_block(fit, refs[key], heads[key], m)
            log("parity %s: %d failures, %d validated alternative minima (%.1f s)"
                % (form, par[form]["failures"], par[form]["validated_alternative_minima"],
                   time.perf_counter() - t))
            done[form] = True
        if "f16" in refs and "f32" in refs:
            # the FP16 storage itself: oracle on FP16 pixels vs oracle on FP32
            # pixels, in units of the standard errors, where both fit to the interior
            a, c = refs["f16"], refs["f32"]
            cl = lambda st: ((st[:, 2] & 1) != 0) & ((st[:, 2] & oracle.AT_BOUND) == 0)
            both = cl(a["status"]) & cl(c["status"])
            par["fp16_storage_effect_in_sigma"] = {
                "stamps": int(both.sum()), "p50_p99_max": sigma_units(a["p"], c["p"], c["perr"],
                                                                      0xFF, both)}
            # the error each FP16 form makes against the oracle on FP32 pixels
            for form in forms:
                if storage[form] != "f16":
                    continue
                g = {k: v[:m].cpu().numpy() for k, v in results[form]["fit"].items()
                     if hasattr(v, "cpu")}
                gst = g["status"].astype(np.uint32)
                bg = ((gst & 1) != 0) & ((gst & oracle.AT_BOUND) == 0) & cl(c["status"])
                par[form]["vs_oracle_on_fp32_pixels_in_sigma"] = {
                    "stamps": int(bg.sum()),
                    "p50_p99_max": sigma_units(g["p"].astype(np.float64), c["p"], c["perr"],
                                               0xFF, bg)}

    ok = [f for f in results if f not in par or par[f]["failures"] == 0]
    chosen = max(ok or list(results), key=lambda f: results[f]["objs"])
    rc = results[chosen]
    # 64 x 64 stamps take the row layout's moment form, 48 x 48 the direct
    # lane-stride walk
    flop_px = FLOP_PER_PIXEL_SWEEP_MOMENT if side == 64 else FLOP_PER_PIXEL_SWEEP
    rate = lambda f: rc["pixel_sweeps"] * f / (rc["fit_ms"] * 1e-3) / 1e12
    achieved = rate(flop_px)
    wl_desc = ("sersic64h: 262,144 x 64x64 Sersic stamps, seed 0" if wl == "sersic64h" else
               "plain48: 100,000 x 48x48 Sersic stamps, seed 0")
    line = {
        "metric": ("objects fitted/sec (64\u00d764 S\u00e9rsic stamps), chosen vs plain form at "
                   "fixed param error" if side == 64 else
                   "objects fitted/sec (%dx%d Sersic stamps)" % (side, side)),
        "value": round(rc["objs"], 1),
        "unit": "objects/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(rc["elapsed"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl_desc, "stamps": n, "chosen_form": chosen, "free_params": 8,
                   "storage": "f16 x per-stamp scale" if storage[chosen] == "f16" else "f32",
                   "max_iter_lm": opts.max_iter_lm,
                   "chosen_by": "most objects/s among the forms whose parity sample has no "
                                "failing stamp under the parity rule",
                   "forms": {f: {"objects_per_s": round(r["objs"], 1),
                                 "ms_per_step": round(r["elapsed"] / args.steps * 1e3, 4),
                                 "fit_ms": round(r["fit_ms"], 4),
                                 "converged_fraction": round(r["conv"], 4),
                                 "mean_sweeps": round(r["mean_sweeps"], 3)}
                             for f, r in results.items()}},
        "roofline": {"bound": "alu", "kernel": "fit (" + chosen + ")",
                     "achieved": round(achieved, 3), "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / ALU_PEAK_TFLOPS, 4),
                     "traffic": fit_traffic_bytes(wl, chosen),
                     "valu_issue": (fit_valu_issue(chosen) if wl == "sersic64h" else None),
                     "valu_issue_unit": "wave64 VALU instructions per SIMD per 4 cycles "
                                        "(SQ_INSTS_VALU / 1024 SIMDs / cycles x 4; 1 = one "
                                        "instruction per pipe pass), from the committed counters",
                     "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "launch_ms": round(rc["fit_ms"], 4),
                     "flop_per_pixel_sweep": flop_px,
                     "flop_count": ("the sweep's own formulation (%s), FMA = 2, transcendental = 1"
                                    % ("moment form" if side == 64 else "direct Jacobian columns")),
                     "pixel_sweeps_per_launch": rc["pixel_sweeps"],
                     "other_counts": {
                         "direct_columns": {"flop_per_pixel_sweep": FLOP_PER_PIXEL_SWEEP,
                                            "achieved": round(rate(FLOP_PER_PIXEL_SWEEP), 3),
                                            "frac": round(rate(FLOP_PER_PIXEL_SWEEP)
                                                          / ALU_PEAK_TFLOPS, 4)},
                         "a_priori_estimate": {"flop_per_pixel_sweep": FLOP_PER_PIXEL_SWEEP_ESTIMATE,
                                               "achieved": round(rate(FLOP_PER_PIXEL_SWEEP_ESTIMATE), 3),
                                               "frac": round(rate(FLOP_PER_PIXEL_SWEEP_ESTIMATE)
                                                             / ALU_PEAK_TFLOPS, 4)},
                         "note": "work of the direct formulation (Jacobian columns summed "
                                 "pixel by pixel) and an a-priori estimate of it, divided by "
                                 "the same time: the moment form does less arithmetic than "
                                 "either, so these can exceed 1"}},
    }
    if cpu:
        line["cpu_baseline"] = cpu
    if tuned:
        line["config"]["queue_cfg"] = {f: dict(team=t["cfg"].team, team_min_side=t["cfg"].team_min_side, chunk=t["cfg"].chunk,
                                               grid=t["cfg"].grid, drain_frac=t["drain_frac"])
                                       for f, t in tuned.items()}
    # context, not the target: the paper's single-core timings for this path
    line["paper_context"] = {"hardware": "single-core 2.2 GHz Intel CPU (Sec. 4.1)",
                             "seconds_per_object": {"centroid_and_ellipticity": 0.1,
                                                    "two_parameter_fit": 0.5,
                                                    "seven_parameter_brute_force": 6.0},
                             "objects_per_s": round(1.0 / 0.6, 3)}
    if par:
        line["parity"] = par
    print(json.dumps(line), flush=True)


def bench_uneven(args):
    """Uneven stamps: one fused launch in input order vs the work queue
    (largest first, autotuned teams, one hipGraph replay per LM iteration)."""
    import numpy as np

    import synth

    t = time.time()
    b = synth.make("uneven", count=args.count)
    log("generated %d uneven stamps (%.2f Gpx) in %.1f s"
        % (b.n, float((b.sides.astype(np.int64) ** 2).sum()) / 1e9, time.time() - t))

    import torch

    import paper_1203_0571_amd as shape
    from paper_1203_0571_amd import autotune

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    db = shape.DeviceBatch.from_host(b, dev)
    opts = shape.default_opts()
    # forms: "fused" (one launch in input order) and "queue"; --forms picks
    # among them (both when it names neither)
    forms = [f for f in args.forms.split(",") if f in ("fused", "queue")] or ["fused", "queue"]
    cfg, drain_at = None, 0
    if "queue" in forms:
        rec0, _, _ = shape.centroid(db, opts)
        rec1, _, _ = shape.moments(db, rec0, opts)
        t = time.time()
        tuned = autotune.tune_queue(db, rec1, opts, use_cache=False)
        cfg, drain_at = tuned["cfg"], int(tuned["drain_frac"] * db.n)
        log("autotune %.1f s: best %s drain %.2f" % (time.time() - t, dict(team=cfg.team, team_min_side=cfg.team_min_side, grid=cfg.grid, chunk=cfg.chunk), tuned["drain_frac"]))

    def step(form, ev=None):
        if ev:
            ev[0].record()
        r0, _, _ = shape.centroid(db, opts)
        if ev:
            ev[1].record()
        r1, _, _ = shape.moments(db, r0, opts)
        if ev:
            ev[2].record()
        if form == "queue":
            fit = shape.fit_queue(db, rec=r1, opts=opts, cfg=cfg, use_graph=True,
                                  drain_at=drain_at)
        else:
            fit = shape.fit_sersic(db, rec=r1, opts=opts)
        if ev:
            ev[3].record()
        return fit

    res = {}
    for form in forms:
        for _ in range(args.warmup):
            step(form)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
        t0 = time.perf_counter()
        for k in range(args.steps):
            fit = step(form, evs[k])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = fit["status"].cpu().numpy()
        sw = fit["sweeps"].cpu().numpy().astype(np.float64)
        span = lambda i: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs]))
        res[form] = dict(objs=b.n * args.steps / el, ms=el / args.steps * 1e3,
                         centroid_ms=span(0), moments_ms=span(1), fit_ms=span(2),
                         conv=float(((st & shape.ST_CONVERGED) != 0).mean()),
                         px_sweeps=float((sw * b.sides.astype(np.float64) ** 2).sum()))
        log("%-6s %.0f objects/s, centroid %.2f ms, moments %.2f ms, fit %.2f ms, converged %.4f"
            % (form, res[form]["objs"], res[form]["centroid_ms"], res[form]["moments_ms"],
               res[form]["fit_ms"], res[form]["conv"]))
    best = max(res, key=lambda f: res[f]["objs"])
    r = res[best]
    achieved = r["px_sweeps"] * FLOP_PER_PIXEL_SWEEP / (r["fit_ms"] * 1e-3) / 1e12
    line = {"metric": "objects fitted/sec (uneven stamps, side 16-128, 80% Sersic / 20% Moffat)",
            "value": round(r["objs"], 1), "unit": "objects/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms"], 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "uneven: %d stamps, seed 0" % b.n, "chosen_form": best,
                       "queue_cfg": (dict(team=cfg.team, team_min_side=cfg.team_min_side,
                                          grid=cfg.grid, chunk=cfg.chunk,
                                          drain_frac=tuned["drain_frac"]) if cfg else None),
                       "forms": {f: {k: round(v, 4) for k, v in x.items()} for f, x in res.items()}},
            "roofline": {"bound": "alu", "kernel": "fit (" + best + ")",
                         "achieved": round(achieved, 3), "peak": ALU_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(achieved / ALU_PEAK_TFLOPS, 4),
                         "traffic": fit_traffic_bytes("uneven", best),
                         "traffic_unit": "bytes per fit call (its Sersic and Moffat launches; "
                                         "FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                         "launch_ms": round(r["fit_ms"], 3)}}
    print(json.dumps(line), flush=True)


def bench_stars(args):
    """Star sizes (Sec. 4.2) on 32x32 Moffat stars: centroid, joint centre and
    ellipticity, then the Moffat weighted-moment estimator (beta, rd, I0)."""
    import numpy as np

    import synth

    t = time.time()
    b = synth.make("stars32", count=args.count)
    log("generated %d stars (32x32) in %.1f s" % (b.n, time.time() - t))

    import torch

    import paper_1203_0571_amd as shape

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    db = shape.DeviceBatch.from_host(b, dev)
    opts = shape.default_opts()
    npix = 32 * 32

    def step(ev=None):
        if ev:
            ev[0].record()
        r0, i0, _ = shape.centroid(db, opts)
        if ev:
            ev[1].record()
        r1, i1, _ = shape.moments(db, r0, opts)
        if ev:
            ev[2].record()
        out = shape.star_moments(db, r1, shape.STAR_MOFFAT, 1e-4, 20)
        if ev:
            ev[3].record()
        return i0, i1, out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        i0, i1, (out, i2, st) = step(evs[k])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = {name: float(np.mean([e[q].elapsed_time(e[q + 1]) for e in evs]))
          for q, name in enumerate(("centroid", "moments", "star_moments"))}
    its = [x.cpu().numpy().astype(np.float64) for x in (i0, i1, i2)]
    flop = {"centroid": its[0].sum() * npix * FLOP_PER_PIXEL_CENTROID,
            "moments": its[1].sum() * npix * FLOP_PER_PIXEL_MOMENTS,
            "star_moments": its[2].sum() * npix * FLOP_PER_PIXEL_STAR_MOFFAT}
    stv = st.cpu().numpy()
    conv = float(((stv & shape.ST_CONVERGED) != 0).mean())
    dom = max(ms, key=ms.get)
    achieved = flop[dom] / (ms[dom] * 1e-3) / 1e12
    log("stars: %.0f objects/s; %s; converged %.4f"
        % (b.n * args.steps / el, {k: round(v, 3) for k, v in ms.items()}, conv))
    line = {"metric": "star sizes measured/sec (32x32 Moffat stars, weighted moments)",
            "value": round(b.n * args.steps / el, 1), "unit": "objects/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(el / args.steps * 1e3, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "stars32: %d x 32x32 Moffat stars, seed 0" % b.n,
                       "kernel_ms": {k: round(v, 4) for k, v in ms.items()},
                       "mean_iters": {k: round(float(x.mean()), 3) for k, x in
                                      zip(("centroid", "moments", "star_moments"), its)},
                       "converged_fraction": round(conv, 4)},
            "roofline": {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3),
                         "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(achieved / ALU_PEAK_TFLOPS, 4), "traffic": None,
                         "launch_ms": round(ms[dom], 4),
                         "flop_per_pixel_step": {"centroid": FLOP_PER_PIXEL_CENTROID,
                                                 "moments": FLOP_PER_PIXEL_MOMENTS,
                                                 "star_moments": FLOP_PER_PIXEL_STAR_MOFFAT},
                         "per_kernel": {k: {"ms": round(ms[k], 4),
                                            "achieved": round(flop[k] / (ms[k] * 1e-3) / 1e12, 3),
                                            "frac": round(flop[k] / (ms[k] * 1e-3) / 1e12
                                                          / ALU_PEAK_TFLOPS, 4)}
                                        for k in ms}}}
    # the paper's remedy for the rd-beta degeneracy (Sec. 4.2.2): beta fixed,
    # here at the workload's mean (3.75), rd and I0 from r0 and r2
    r1 = shape.moments(db, shape.centroid(db, opts)[0], opts)[0]
    fb = []
    for k in range(args.warmup + args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fout, fit_, fst = shape.star_moments_beta(db, r1, 3.75, 1e-4, 20)
        e1.record()
        torch.cuda.synchronize()
        if k >= args.warmup:
            fb.append(e0.elapsed_time(e1))
    fstv = fst.cpu().numpy()
    line["config"]["fixed_beta"] = {
        "beta": 3.75, "kernel_ms": round(float(np.mean(fb)), 4),
        "mean_iters": round(float(fit_.float().mean().item()), 3),
        "converged_fraction": round(float(((fstv & shape.ST_CONVERGED) != 0).mean()), 4),
        "free_beta_status": {k: round(float(((stv & getattr(shape, "ST_" + k)) != 0).mean()), 4)
                             for k in ("CONVERGED", "SINGULAR", "MAX_ITER", "NONPOSITIVE_FLUX")}}
    log("fixed beta: %.3f ms, converged %.4f" % (np.mean(fb), line["config"]["fixed_beta"]["converged_fraction"]))
    if not args.no_cpu:
        import oracle
        m = min(args.cpu_sample * 16, b.n)
        t = time.perf_counter()
        ref = oracle.star_pipeline(b.head(m), oracle.MOFFAT, 1e-4, 20)
        cpu_s = time.perf_counter() - t
        line["cpu_baseline"] = {"value": round(m / cpu_s, 2), "unit": "objects/s",
                                "cores": int(ref["threads"]), "kind": "oracle",
                                "sample": "first %d stars, FP64 oracle chain, %.1f s" % (m, cpu_s)}
        g = out[:m].cpu().numpy().astype(np.float64)
        both = ((stv[:m] & 1) != 0) & ((ref["status"] & 1) != 0)
        rel = np.abs(g[both][:, :3] / ref["out"][both][:, :3] - 1)
        line["parity"] = {"sample": m, "both_converged": int(both.sum()),
                          "status_agree": float((stv[:m] == ref["status"]).mean()),
                          "max_rel_rd": float(rel[:, 0].max()) if both.any() else None,
                          "max_rel_beta": float(rel[:, 1].max()) if both.any() else None,
                          "max_rel_i0": float(rel[:, 2].max()) if both.any() else None,
                          "within_1e-3": float((rel.max(1) <= 1e-3).mean()) if both.any() else None}
    print(json.dumps(line), flush=True)


def bench_profiled(args):
    """The paper's split on the 32x32 Gaussian galaxies of the first benchmark
    configuration: centre and ellipticity from the moments, then (Re, n)
    searched with (I0, sky) profiled at every evaluation (linear_init 1), or
    all four searched by the same LM (linear_init 0)."""
    import numpy as np

    import synth

    t = time.time()
    b = synth.make("plain32x", count=args.count)
    log("generated %d stamps (32x32) in %.1f s" % (b.n, time.time() - t))

    import torch

    import paper_1203_0571_amd as shape

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    db = shape.DeviceBatch.from_host(b, dev)
    forms = {"profiled": shape.default_opts(free_mask=shape.MASK_SIZE),
             "unprofiled": shape.default_opts(free_mask=shape.MASK_SIZE, linear_init=0)}

    def step(o, ev=None):
        r0, _, _ = shape.centroid(db, o)
        r1, _, _ = shape.moments(db, r0, o)
        if ev:
            ev[0].record()
        fit = shape.fit_sersic(db, rec=r1, opts=o)
        if ev:
            ev[1].record()
        return fit

    res = {}
    for name, o in forms.items():
        for _ in range(args.warmup):
            step(o)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        t0 = time.perf_counter()
        for k in range(args.steps):
            fit = step(o, evs[k])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = fit["status"].cpu().numpy()
        sw = fit["sweeps"].cpu().numpy().astype(np.float64)
        res[name] = dict(fit=fit, objs=b.n * args.steps / el, ms=el / args.steps * 1e3,
                         fit_ms=float(np.mean([x.elapsed_time(y) for x, y in evs])),
                         conv=float(((st & shape.ST_CONVERGED) != 0).mean()),
                         mean_trials=float(fit["iters"].float().mean().item()),
                         mean_sweeps=float(sw.mean()), px_sweeps=float(sw.sum()) * 32 * 32)
        log("%-10s %.0f objects/s, fit %.3f ms, %.2f trials, converged %.4f"
            % (name, res[name]["objs"], res[name]["fit_ms"], res[name]["mean_trials"],
               res[name]["conv"]))
    r = res["profiled"]
    achieved = r["px_sweeps"] * FLOP_PER_PIXEL_SWEEP_4 / (r["fit_ms"] * 1e-3) / 1e12
    line = {"metric": "objects fitted/sec (32x32 Gaussian galaxies, (Re, n, I0, sky) fit)",
            "value": round(r["objs"], 1), "unit": "objects/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms"], 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "plain32x: %d x 32x32 Gaussian galaxies, seed 0" % b.n,
                       "chosen_form": "profiled",
                       "forms": {k: {q: round(v, 4) for q, v in x.items() if q != "fit"}
                                 for k, x in res.items()}},
            "roofline": {"bound": "alu", "kernel": "fit (profiled, 4 parameters)",
                         "achieved": round(achieved, 3), "peak": ALU_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(achieved / ALU_PEAK_TFLOPS, 4),
                         "traffic": None, "launch_ms": round(r["fit_ms"], 4),
                         "flop_per_pixel_sweep": FLOP_PER_PIXEL_SWEEP_4}}
    if not args.no_cpu:
        import oracle
        m = min(args.cpu_sample * 16, b.n)   # 32x32 stamps fit fast: ~15 s of oracle work
        sub = b.head(m)
        par = {}
        for name, li in (("profiled", 1), ("unprofiled", 0)):
            o = oracle.opts(free_mask=0xF0, linear_init=li)
            t = time.perf_counter()
            ref = oracle.pipeline(sub, o)
            cpu_s = time.perf_counter() - t
            if name == "profiled":
                line["cpu_baseline"] = {"value": round(m / cpu_s, 2), "unit": "objects/s",
                                        "cores": int(ref["threads"]), "kind": "oracle",
                                        "sample": "first %d stamps, FP64 oracle, LM tol 1e-9, "
                                                  "cap 200, %.1f s" % (m, cpu_s)}
            g = {k: v[:m].cpu().numpy() for k, v in res[name]["fit"].items() if hasattr(v, "cpu")}
            both = ((g["status"] & shape.ST_CONVERGED) != 0) & ((ref["status"][:, 2] & 1) != 0)
            rel = np.abs(g["p"][both, 4:6] / ref["p"][both, 4:6] - 1)
            par[name] = {"sample": m, "both_converged": int(both.sum()),
                         "max_rel_re": float(rel[:, 0].max()), "max_rel_n": float(rel[:, 1].max()),
                         "within_bars": float((rel.max(1) <= BARS["rel"]).mean()),
                         "oracle_mean_trials": float(ref["iters"][:, 2].mean())}
        line["parity"] = par
    print(json.dumps(line), flush=True)


def bench_adjoint(args):
    """chi^2 and its adjoint gradient (the FP64 instance of the sweep) on the
    65,536 64x64 Sersic stamps, at parameters away from the optimum; also the
    gradient through torch.autograd (SersicChi2)."""
    import numpy as np

    import synth

    t = time.time()
    b = synth.make("sersic64", count=args.count)
    log("generated %d stamps (64x64) in %.1f s" % (b.n, time.time() - t))
    rng = np.random.default_rng(42)
    p = b.truth.copy()
    p[:, 0:2] += rng.uniform(-0.3, 0.3, (b.n, 2))
    p[:, 4] *= rng.uniform(0.85, 1.15, b.n)
    p[:, 5] *= rng.uniform(0.85, 1.15, b.n)

    import torch

    import paper_1203_0571_amd as shape

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    db = shape.DeviceBatch.from_host(b, dev)
    pt = torch.from_numpy(p.astype(np.float32)).to(dev)
    calls = {"forward": lambda: shape.chi2_fwd(db, pt),
             "backward": lambda: shape.chi2_bwd(db, pt),
             "backward_jtj": lambda: shape.chi2_bwd(db, pt, want_normal=True)}
    ms = {}
    for name, fn in calls.items():
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms[name] = e0.elapsed_time(e1) / args.steps
    q = pt.clone().requires_grad_(True)
    for _ in range(args.warmup):
        shape.sersic_chi2(q, db).sum().backward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        q.grad = None
        shape.sersic_chi2(q, db).sum().backward()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    log("adjoint: %s ms per launch; autograd forward+backward %.3f ms"
        % ({k: round(v, 3) for k, v in ms.items()}, el / args.steps * 1e3))
    # the backward's algorithmic FLOP per pixel (chi^2 and the gradient in the
    # moment form, transcendentals counted once, as in the fit) against the
    # FP64 vector peak: the FP64 series for log2 / exp2 and the reciprocal's
    # Newton steps are what this instance spends beyond them
    rate = lambda f, k: b.n * 64 * 64 * f / (ms[k] * 1e-3) / 1e12
    achieved = rate(FLOP_PER_PIXEL_GRAD_MOMENT, "backward")
    line = {"metric": "chi^2 gradients/sec (64x64 Sersic stamps, adjoint)",
            "value": round(b.n * args.steps / el, 1), "unit": "gradients/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(el / args.steps * 1e3, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "sersic64: %d x 64x64 Sersic stamps, seed 0" % b.n,
                       "kernel_ms": {k: round(v, 4) for k, v in ms.items()},
                       "note": "value = forward + backward through torch.autograd"},
            "roofline": {"bound": "alu", "kernel": "chi2 backward (FP64)",
                         "achieved": round(achieved, 3), "peak": ALU_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(achieved / ALU_PEAK_TFLOPS, 4),
                         "traffic": None, "launch_ms": round(ms["backward"], 4),
                         "flop_per_pixel": FLOP_PER_PIXEL_GRAD_MOMENT,
                         "flop_count": "chi^2 and J^T r in the moment form, FMA = 2, "
                                       "transcendental = 1 (61 for the direct columns: frac %.4f)"
                                       % (rate(FLOP_PER_PIXEL_GRAD_DIRECT, "backward")
                                          / ALU_PEAK_TFLOPS),
                         "jtj_instance": {"flop_per_pixel": FLOP_PER_PIXEL_GRAD_JTJ_MOMENT,
                                          "launch_ms": round(ms["backward_jtj"], 4),
                                          "achieved": round(rate(FLOP_PER_PIXEL_GRAD_JTJ_MOMENT,
                                                                 "backward_jtj"), 3),
                                          "frac": round(rate(FLOP_PER_PIXEL_GRAD_JTJ_MOMENT,
                                                             "backward_jtj") / ALU_PEAK_TFLOPS, 4)}}}
    if not args.no_cpu:
        import oracle
        m = min(65536, b.n)   # ~13 s of oracle work on one thread
        t = time.perf_counter()
        for s_ in range(m):
            oracle.chi2(b.stamp(s_), float(b.sigma[s_]), p[s_].astype(np.float32).astype(np.float64),
                        want_grad=True)
        cpu_s = time.perf_counter() - t
        line["cpu_baseline"] = {"value": round(m / cpu_s, 2), "unit": "gradients/s", "cores": 1,
                                "kind": "oracle",
                                "sample": "first %d stamps, FP64 oracle chi^2 + gradient + J^T J, "
                                          "one thread, %.1f s" % (m, cpu_s)}
    print(json.dumps(line), flush=True)


def bench_frames(args):
    """Front end on 512x512 frames: detection (border sky, brightest pixel,
    growth-curve r50, 6 r50 box), offsets, and the cut into a stamp batch."""
    import numpy as np

    import synth

    t = time.time()
    f = synth.make_frames(count=args.count)
    log("generated %d frames (512x512) in %.1f s" % (f.n, time.time() - t))

    import torch

    import paper_1203_0571_amd as shape

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    fr = shape.DeviceFrames.from_host(f, dev)
    sigma = torch.from_numpy(f.sigma).to(dev)
    out = torch.empty(f.n * 128 * 128, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    def step(ev=None):
        if ev:
            ev[0].record()
        d = shape.frame_detect(fr)
        if ev:
            ev[1].record()
        db = shape.frame_cut(fr, d["box"], sigma, out=out)
        if ev:
            ev[2].record()
        return d, db

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        d, db = step(evs[k])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    det_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    cut_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    box = d["box"].cpu().numpy()
    st = d["status"].cpu().numpy()
    frame_bytes = float(f.pixels[0].nbytes)
    # algorithmic bytes of the detection launch: each frame read once, plus
    # the outputs (info 12 B, peak 8 B, box 12 B, status 4 B)
    det_bytes = f.n * (frame_bytes + 36.0)
    achieved = det_bytes / (det_ms * 1e-3) / 1e9
    cut_px = float((box[:, 2].astype(np.float64) ** 2).sum())
    log("frames: %.0f frames/s; detect %.3f ms (%.0f GB/s), offsets+cut %.3f ms, %.0f cut px"
        % (f.n * args.steps / el, det_ms, achieved, cut_ms, cut_px))
    line = {"metric": "frames processed/sec (512x512 frames: detection + 6 r50 cut-outs)",
            "value": round(f.n * args.steps / el, 1), "unit": "frames/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(el / args.steps * 1e3, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "frames512: %d x 512x512 frames, one Sersic galaxy each, seed 0"
                                   % f.n,
                       "detect_ms": round(det_ms, 4), "offsets_cut_ms": round(cut_ms, 4),
                       "mean_side": round(float(box[:, 2].mean()), 3),
                       "nonpositive_flux_frames": int(((st & shape.ST_NONPOSITIVE_FLUX) != 0).sum())},
            "roofline": {"bound": "hbm", "kernel": "frame detect", "achieved": round(achieved, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": counter_traffic(FRAME_TRAFFIC_FILE, FRAME_SOURCES),
                         "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, "
                                         "copy-calibrated)",
                         "launch_ms": round(det_ms, 4), "bytes_per_launch": det_bytes}}
    if not args.no_cpu:
        import oracle
        m = min(1024, f.n)
        t = time.perf_counter()
        ref = [oracle.frame_detect(f.pixels[i].astype(np.float64)) for i in range(m)]
        cpu_s = time.perf_counter() - t
        line["cpu_baseline"] = {"value": round(m / cpu_s, 2), "unit": "frames/s", "cores": 1,
                                "kind": "oracle",
                                "sample": "first %d frames, FP64 oracle detection, one thread, "
                                          "%.1f s" % (m, cpu_s)}
        gb = box[:m]
        gp = d["peak"][:m].cpu().numpy()
        line["parity"] = {"sample": m,
                          "box_equal": float(np.mean([tuple(gb[i].tolist()) == ref[i]["box"]
                                                      for i in range(m)])),
                          "peak_equal": float(np.mean([tuple(gp[i].tolist()) == ref[i]["peak"]
                                                       for i in range(m)]))}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
