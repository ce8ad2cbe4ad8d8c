"""GPU: the work-queue form of the fit (persistent launch per LM trial,
hipGraph replays, teams of waves for large stamps) against the fused fit and
the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from parity_util import check_fit, compare, oracle_opts_like

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def shape():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1203_0571_amd as shape
    return shape


def _moments(shape, db, o):
    rec0, _, _ = shape.centroid(db, o)
    rec1, _, _ = shape.moments(db, rec0, o)
    return rec1


def _np(d):
    return {k: v.cpu().numpy() for k, v in d.items() if hasattr(v, "cpu")}


@pytest.mark.parametrize("workload", ["sersic64", "sersic64h", "uneven"])
def test_queue_equals_fused_fit(shape, workload):
    """One wave per stamp: the queue runs the fused kernel's LM trials (the
    same lm.hpp arithmetic, split into sweep and decide passes; the drain pass
    runs the fused loop), so the results are bit-identical, with steps only,
    with the drain after a few steps, and with graphs or eager steps."""
    import torch
    b = synth.make(workload, count=1024)
    db = shape.DeviceBatch.from_host(b, "cuda:0")
    o = shape.default_opts()
    rec = _moments(shape, db, o)
    fused = _np(shape.fit_sersic(db, rec=rec, opts=o, want_perr=True))
    for use_graph, drain_at in ((False, 0), (True, 0), (True, 256), (True, 10 ** 6)):
        q = shape.fit_queue(db, rec=rec, opts=o, cfg=shape.queue_cfg(team=1),
                            use_graph=use_graph, want_perr=True, drain_at=drain_at)
        torch.cuda.synchronize()
        qn = _np(q)
        for k in ("p", "chi2", "perr", "iters", "status", "sweeps"):
            np.testing.assert_array_equal(qn[k], fused[k], err_msg="%s graph=%s drain_at=%d"
                                          % (k, use_graph, drain_at))
        assert 1 <= q["steps"] <= o.max_iter_lm
        if not drain_at:
            assert not q["drained"]
        if drain_at >= b.n:
            assert q["drained"] and q["steps"] == 2


@pytest.mark.parametrize("grid,chunk", [(1, 0), (3, 1), (8, 0), (100, 64)])
def test_queue_small_grids(shape, grid, chunk):
    """Persistent grids smaller than the cursor count still drain every cursor
    (a workgroup moves on to the next cursor when its own is empty), at any
    number of stamps per pop."""
    b = synth.make("uneven", count=512)
    db = shape.DeviceBatch.from_host(b, "cuda:0")
    o = shape.default_opts()
    rec = _moments(shape, db, o)
    fused = _np(shape.fit_sersic(db, rec=rec, opts=o))
    q = _np(shape.fit_queue(db, rec=rec, opts=o,
                            cfg=shape.queue_cfg(team=1, grid=grid, chunk=chunk), drain_at=0))
    for k in ("p", "chi2", "iters", "status", "sweeps"):
        np.testing.assert_array_equal(q[k], fused[k], err_msg=k)


def test_graph_replays_match_eager_steps(shape):
    """Replays of the captured step, with eager work and synchronisations in
    between, reproduce the eager steps exactly."""
    import torch
    b = synth.make("uneven", count=256)
    db = shape.DeviceBatch.from_host(b, "cuda:0")
    o = shape.default_opts(max_iter_lm=6)
    rec = _moments(shape, db, o)
    cfg = shape.queue_cfg(team=2, team_min_side=64)
    a = _np(shape.fit_queue(db, rec=rec, opts=o, cfg=cfg, use_graph=False, check_every=0))
    for _ in range(2):
        _ = torch.ones(1000, device="cuda").sum().item()       # eager work in between
        g = _np(shape.fit_queue(db, rec=rec, opts=o, cfg=cfg, use_graph=True, check_every=1,
                                drain_at=0))
        for k in ("p", "chi2", "iters", "status"):
            np.testing.assert_array_equal(g[k], a[k], err_msg=k)
    # the drain pass (teams for the team class) finishes the same fits
    d = _np(shape.fit_queue(db, rec=rec, opts=o, cfg=cfg, use_graph=True, check_every=1,
                            drain_at=10 ** 6))
    for k in ("p", "chi2", "iters", "status"):
        np.testing.assert_array_equal(d[k], a[k], err_msg=k)


@pytest.mark.parametrize("team,min_side", [(1, 96), (2, 64), (4, 96)])
def test_queue_uneven_parity(shape, team, min_side):
    b = synth.make("uneven", count=1024)
    db = shape.DeviceBatch.from_host(b, "cuda:0")
    o = shape.default_opts()
    rec = _moments(shape, db, o)
    q = shape.fit_queue(db, rec=rec, opts=o, cfg=shape.queue_cfg(team=team, team_min_side=min_side),
                        want_perr=True)
    import torch
    torch.cuda.synchronize()
    g = _np(q)
    g["centroid"] = _np({"c": shape.centroid(db, o)[0]})["c"]
    g["moments"] = rec.cpu().numpy()
    g["status"] = np.stack([shape.centroid(db, o)[2].cpu().numpy(), shape.moments(db, shape.centroid(db, o)[0], o)[2].cpu().numpy(), g["status"]], 1)
    ref = oracle.pipeline(b, oracle_opts_like(o, tol_lm=1e-9, max_iter_lm=200))
    r = compare(g, ref, 0xFF, "queue team=%d" % team, batch=b)
    check_fit(r, 0.8)


def test_queue_caps_and_empty(shape):
    import torch
    b = synth.make("plain48", count=64)
    db = shape.DeviceBatch.from_host(b, "cuda:0")
    for cap, drain_at in ((0, 0), (1, 0), (1, 4096), (3, 4096)):
        o = shape.default_opts(max_iter_lm=cap)
        rec = _moments(shape, db, o)
        q = _np(shape.fit_queue(db, rec=rec, opts=o, drain_at=drain_at))
        f = _np(shape.fit_sersic(db, rec=rec, opts=o))
        np.testing.assert_array_equal(q["p"], f["p"])
        np.testing.assert_array_equal(q["status"], f["status"])
    e = shape.DeviceBatch(pixels=torch.zeros(0, device="cuda"), sigma=torch.zeros(0, device="cuda"),
                          side0=16)
    assert shape.fit_queue(e)["p"].shape == (0, 8)


def test_autotuner_picks_a_measured_candidate(shape, tmp_path, monkeypatch):
    from paper_1203_0571_amd import autotune
    monkeypatch.setenv("SHAPE_TUNE_CACHE", str(tmp_path / "tune.json"))
    b = synth.make("uneven", count=2048)
    db = shape.DeviceBatch.from_host(b, "cuda:0")
    o = shape.default_opts()
    rec = _moments(shape, db, o)
    t = autotune.tune_queue(db, rec, o, sample=1024)
    assert len(t["timings"]) == len(autotune.candidates(db.device, o.free_mask)) + \
        len(autotune.CHUNKS)
    best = min(t["timings"], key=lambda x: x["ms"])
    cfg = t["cfg"]
    assert (cfg.team, cfg.team_min_side, cfg.grid, cfg.chunk) == (
        best["cfg"]["team"], best["cfg"]["team_min_side"], best["cfg"]["grid"],
        best["cfg"].get("chunk", 0))
    assert t["drain_frac"] == best["drain_frac"]
    t2 = autotune.tune_queue(db, rec, o, sample=1024)      # served from the cache
    assert (t2["cfg"].team, t2["cfg"].grid, t2["drain_frac"]) == (cfg.team, cfg.grid,
                                                                  t["drain_frac"])
    assert t2["timings"] == t["timings"]
    q = shape.fit_queue(db, rec=rec, opts=o, cfg=cfg, drain_at=int(t["drain_frac"] * db.n))
    f = shape.fit_sersic(db, rec=rec, opts=o)
    conv_q = ((q["status"] & 1) != 0).float().mean().item()
    conv_f = ((f["status"] & 1) != 0).float().mean().item()
    assert abs(conv_q - conv_f) < 0.02
