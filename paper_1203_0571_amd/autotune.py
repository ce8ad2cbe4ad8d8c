"""Autotuner for the work-queue fit: waves per stamp and the team threshold.

For a batch of uneven stamps it times a few queue steps for each candidate
configuration (team of 1, 2 or 4 waves for stamps at or above a threshold
side; persistent grid sized by the device or doubled) on an evenly spaced
sample of the batch, keeps the fastest, and caches the choice in a JSON file
keyed by the device, the free mask, the storage type and a coarse histogram of
the stamp sides.  The cache lives in $SHAPE_TUNE_CACHE (default
~/.cache/shape/queue_tune.json).
"""
from __future__ import annotations

import json
import os

import torch

from . import (DeviceBatch, default_opts, lib, queue_cfg, queue_workspace_bytes, _check, _ptr,
               _stream)

CANDIDATES = [
    dict(team=1, team_min_side=96, grid=0),
    dict(team=2, team_min_side=64, grid=0),
    dict(team=2, team_min_side=96, grid=0),
    dict(team=4, team_min_side=96, grid=0),
    dict(team=4, team_min_side=112, grid=0),
]


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


def time_queue(batch: DeviceBatch, rec: torch.Tensor, opts, cfg, steps: int = 3) -> float:
    """Milliseconds for queue start + `steps` steps with configuration cfg."""
    import ctypes as C
    n, dev = batch.n, batch.device
    nbytes = queue_workspace_bytes(n)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = batch.c_struct()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    _check(lib.shape_queue_start(C.byref(b), C.byref(opts), C.byref(cfg), None, _ptr(rec),
                                 _ptr(ws), nbytes, _stream(dev)), "shape_queue_start")
    for _ in range(steps):
        _check(lib.shape_queue_step(C.byref(b), C.byref(opts), C.byref(cfg), _ptr(ws), nbytes,
                                    _stream(dev)), "shape_queue_step")
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def tune_queue(batch: DeviceBatch, rec: torch.Tensor, opts=None, sample: int = 65536,
               use_cache: bool = True, verbose: bool = False):
    """Return the fastest queue_cfg for this batch (and the timings tried)."""
    opts = opts or default_opts()
    key = _signature(batch, opts)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return queue_cfg(**cache[key]["cfg"]), cache[key]["timings"]
    sub = _subset(batch, sample)
    sub_rec = rec
    if sub is not batch:
        idx = torch.linspace(0, batch.n - 1, sub.n, device=batch.device).long()
        sub_rec = rec[idx].contiguous()
    cands = [c for c in CANDIDATES if opts.free_mask == 0xFF or c["team"] == 1]
    timings = []
    for c in cands:
        cfg = queue_cfg(**c)
        time_queue(sub, sub_rec, opts, cfg, steps=1)           # warm-up
        ms = min(time_queue(sub, sub_rec, opts, cfg) for _ in range(2))
        timings.append(dict(cfg=c, ms=ms))
        if verbose:
            print("autotune", c, "%.3f ms" % ms, flush=True)
    best = min(timings, key=lambda t: t["ms"])
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            cache[key] = dict(cfg=best["cfg"], timings=timings)
            tmp = path + ".tmp%d" % os.getpid()
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1)
            os.replace(tmp, path)
        except OSError:
            pass
    return queue_cfg(**best["cfg"]), timings
