"""Autotuner for the work-queue fit: waves per stamp, team threshold,
persistent grid, stamps per cursor pop and the point where the drain pass
takes over.

For a batch it times the whole queue fit (start, graph-replayed steps, drain,
finish) for each candidate on an evenly spaced sample of the batch.  First
round: teams of 1, 2 or 4 waves for stamps at or above a threshold side; the
persistent grid at the resident workgroup count or half of it; the drain once
the active stamps fall to 2%, 8% or 25% of the batch (chunk 8).  Second
round: the best of those with 2, 4, 16 or 32 stamps per pop.  It keeps the
fastest and caches the choice in a JSON file keyed by the device, the free
mask, the storage type and a coarse histogram of the stamp sides.  The cache
lives in $SHAPE_TUNE_CACHE (default ~/.cache/shape/queue_tune.json).
(Waves per SIMD are fixed when the kernels are compiled: four, as the fused
fit, where the sweep's registers fit without spills.)
"""
from __future__ import annotations

import itertools
import json
import os

import torch

from . import DeviceBatch, default_opts, fit_queue, queue_cfg

TEAMS = [dict(team=1, team_min_side=96), dict(team=2, team_min_side=64),
         dict(team=2, team_min_side=96), dict(team=4, team_min_side=96)]
GRID_FRACTIONS = [1.0, 0.5]        # of the resident single-wave workgroups
DRAIN_FRACTIONS = [0.02, 0.08, 0.25]
CHUNKS = [2, 4, 16, 32]            # second round (the first uses the default 8)


def candidates(device, free_mask=0xFF):
    """Every configuration tried: (queue_cfg fields, drain fraction)."""
    cus = torch.cuda.get_device_properties(device).multi_processor_count
    out = []
    for t, g, d in itertools.product(TEAMS, GRID_FRACTIONS, DRAIN_FRACTIONS):
        if free_mask != 0xFF and t["team"] != 1:
            continue
        grid = 0 if g == 1.0 else int(cus * 16 * g / t["team"])
        out.append((dict(t, grid=grid), d))
    return out


def _cache_path():
    return os.environ.get("SHAPE_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "shape", "queue_tune.json")


def _signature(batch: DeviceBatch, opts):
    if batch.sides is None:
        hist = {str(int(batch.side0)): 1.0}
    else:
        s = batch.sides.to("cpu")
        edges = [4, 24, 32, 48, 64, 96, 129]
        counts = torch.histc(s.float(), bins=len(edges) - 1, min=4, max=129)
        tot = max(float(counts.sum()), 1.0)
        hist = {"%d-%d" % (edges[k], edges[k + 1]): round(float(counts[k]) / tot, 2)
                for k in range(len(edges) - 1)}
    dev = torch.cuda.get_device_name(batch.device)
    return json.dumps(dict(dev=dev, mask=int(opts.free_mask),
                           dtype=str(batch.pixels.dtype), hist=hist), sort_keys=True)


def _subset(batch: DeviceBatch, max_stamps: int) -> DeviceBatch:
    n = batch.n
    if n <= max_stamps or batch.offsets is None:
        return batch
    idx = torch.linspace(0, n - 1, max_stamps, device=batch.device).long()
    return DeviceBatch(pixels=batch.pixels, sigma=batch.sigma[idx].contiguous(), side0=batch.side0,
                       offsets=batch.offsets[idx].contiguous(), sides=batch.sides[idx].contiguous(),
                       scale=None if batch.scale is None else batch.scale[idx].contiguous(),
                       model=None if batch.model is None else batch.model[idx].contiguous())


def time_queue(batch: DeviceBatch, rec: torch.Tensor, opts, cfg, drain_frac: float) -> float:
    """Milliseconds for the whole queue fit of batch with configuration cfg."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fit_queue(batch, rec=rec, opts=opts, cfg=cfg, use_graph=True,
              drain_at=int(drain_frac * batch.n))
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def tune_queue(batch: DeviceBatch, rec: torch.Tensor, opts=None, sample: int = 65536,
               use_cache: bool = True, verbose: bool = False):
    """The fastest configuration for this batch: dict(cfg=queue_cfg, drain_frac,
    timings=[dict(cfg, drain_frac, ms), ...])."""
    opts = opts or default_opts()
    key = _signature(batch, opts)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache and "drain_frac" in cache[key]:
            e = cache[key]
            return dict(cfg=queue_cfg(**e["cfg"]), drain_frac=e["drain_frac"], timings=e["timings"])
    sub = _subset(batch, sample)
    sub_rec = rec
    if sub is not batch:
        idx = torch.linspace(0, batch.n - 1, sub.n, device=batch.device).long()
        sub_rec = rec[idx].contiguous()
    timings = []

    def run(c, d):
        cfg = queue_cfg(**c)
        time_queue(sub, sub_rec, opts, cfg, d)           # warm-up
        ms = min(time_queue(sub, sub_rec, opts, cfg, d) for _ in range(2))
        timings.append(dict(cfg=c, drain_frac=d, ms=ms))
        if verbose:
            print("autotune", c, d, "%.3f ms" % ms, flush=True)

    for c, d in candidates(batch.device, opts.free_mask):
        run(c, d)
    first = min(timings, key=lambda t: t["ms"])
    for k in CHUNKS:
        run(dict(first["cfg"], chunk=k), first["drain_frac"])
    best = min(timings, key=lambda t: t["ms"])
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            cache[key] = dict(cfg=best["cfg"], drain_frac=best["drain_frac"], timings=timings)
            tmp = path + ".tmp%d" % os.getpid()
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1)
            os.replace(tmp, path)
        except OSError:
            pass
    return dict(cfg=queue_cfg(**best["cfg"]), drain_frac=best["drain_frac"], timings=timings)
