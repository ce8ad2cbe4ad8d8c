"""GPU parity at the benchmark workloads' full sizes, in the launch
configurations bench.py times; a seeded sample of stamps is recomputed by the
oracle one by one (same bars as the small-size tests)."""
import numpy as np
import pytest

import oracle
import synth
from parity_util import BAR_REL, check_fit, compare, oracle_opts_like

pytestmark = pytest.mark.gpu

SAMPLE = 128


@pytest.fixture(scope="module")
def shape():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1203_0571_amd as shape
    return shape


def _subset(b, idx):
    """The stamps idx of a synth.Batch as a Batch of their own (host)."""
    sides = b.sides[idx]
    sizes = sides.astype(np.int64) ** 2
    offs = np.zeros(len(idx), np.int64)
    np.cumsum(sizes[:-1], out=offs[1:])
    pix = np.concatenate([b.pixels[b.offsets[i]:b.offsets[i] + int(b.sides[i]) ** 2] for i in idx])
    return synth.Batch("sample", pix, offs, sides, b.sigma[idx], b.model[idx], b.truth[idx],
                       None if b.scale is None else b.scale[idx])


def _gpu_pipeline(shape, db, o, queue_cfg=None):
    import torch
    rec0, it0, st0 = shape.centroid(db, o)
    rec1, it1, st1 = shape.moments(db, rec0, o)
    if queue_cfg is None:
        fit = shape.fit_sersic(db, rec=rec1, opts=o, want_perr=True)
    else:
        fit = shape.fit_queue(db, rec=rec1, opts=o, cfg=queue_cfg, use_graph=True, want_perr=True)
    torch.cuda.synchronize()
    out = dict(centroid=rec0, moments=rec1, p=fit["p"], chi2=fit["chi2"], perr=fit["perr"],
               status=torch.stack([st0, st1, fit["status"]], 1),
               iters=torch.stack([it0, it1, fit["iters"]], 1))
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("storage,queue", [("f32", False), ("f16", False), ("f16", True)])
def test_sersic64h_full(shape, storage, queue):
    """262,144 x 64^2 stamps: the bench's three forms (FP32 fused, FP16 fused,
    FP16 work queue with one hipGraph replay per LM iteration)."""
    b = synth.make("sersic64h", storage=storage)
    db = shape.DeviceBatch.from_host(b, "cuda:0")
    o = shape.default_opts()
    g = _gpu_pipeline(shape, db, o, shape.queue_cfg(team=1) if queue else None)
    idx = np.sort(np.random.default_rng(11).choice(b.n, SAMPLE, replace=False))
    sub = _subset(b, idx)
    ref = oracle.pipeline(sub, oracle_opts_like(o, tol_lm=1e-9, max_iter_lm=200))
    r = compare({k: v[idx] for k, v in g.items()}, ref, 0xFF, "sersic64h %s queue=%s" % (storage, queue),
                batch=sub)
    check_fit(r, 0.85)
    assert ((g["status"][:, 2] & shape.ST_CONVERGED) != 0).mean() > 0.85


@pytest.mark.parametrize("queue", [False, True])
def test_plain48_full(shape, queue):
    """100,000 x 48^2 Sersic stamps, 8 parameters, LM cap 30: the bench's two
    forms (fused, and the work queue with one hipGraph replay per LM
    iteration); 48 does not divide 64, so the stages take the any-side
    register layout."""
    b = synth.make("plain48")
    db = shape.DeviceBatch.from_host(b, "cuda:0")
    o = shape.default_opts()
    g = _gpu_pipeline(shape, db, o, shape.queue_cfg(team=1) if queue else None)
    idx = np.sort(np.random.default_rng(16).choice(b.n, SAMPLE, replace=False))
    sub = _subset(b, idx)
    ref = oracle.pipeline(sub, oracle_opts_like(o, tol_lm=1e-9, max_iter_lm=200))
    r = compare({k: v[idx] for k, v in g.items()}, ref, 0xFF, "plain48 queue=%s" % queue, batch=sub)
    assert r["centroid_dxy"] <= 1e-3 and r["moments_dxy"] <= 1e-3 and r["moments_de"] <= 1e-4, r
    check_fit(r, 0.85)
    assert ((g["status"][:, 2] & shape.ST_CONVERGED) != 0).mean() > 0.85


def test_uneven_full(shape):
    """1,000,000 uneven stamps (side 16-128, 20% Moffat): fused fit and the
    work queue with teams of two waves for sides >= 64."""
    b = synth.make("uneven")
    db = shape.DeviceBatch.from_host(b, "cuda:0")
    o = shape.default_opts()
    idx = np.sort(np.random.default_rng(12).choice(b.n, SAMPLE, replace=False))
    sub = _subset(b, idx)
    ref = oracle.pipeline(sub, oracle_opts_like(o, tol_lm=1e-9, max_iter_lm=200))
    for cfg in (None, shape.queue_cfg(team=2, team_min_side=64)):
        g = _gpu_pipeline(shape, db, o, cfg)
        r = compare({k: v[idx] for k, v in g.items()}, ref, 0xFF, "uneven queue=%s" % (cfg is not None),
                    batch=sub)
        check_fit(r, 0.85)


def test_stars32_full(shape):
    """1,048,576 32^2 Moffat stars: centroid, moments and the star estimator."""
    import torch
    b = synth.make("stars32")
    db = shape.DeviceBatch.from_host(b, "cuda:0")
    rec0, _, _ = shape.centroid(db)
    rec1, _, _ = shape.moments(db, rec0)
    out, it, st = shape.star_moments(db, rec1, shape.STAR_MOFFAT, 1e-4, 20)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(13).choice(b.n, 4 * SAMPLE, replace=False))
    ref = oracle.star_pipeline(_subset(b, idx), oracle.MOFFAT, 1e-4, 20)
    g, s = out.cpu().numpy()[idx].astype(np.float64), st.cpu().numpy()[idx].astype(np.uint32)
    assert (s == ref["status"]).mean() >= 0.95
    both = ((s & 1) != 0) & ((ref["status"] & 1) != 0)
    assert both.mean() >= 0.5
    rel = np.abs(g[both][:, :3] / ref["out"][both][:, :3] - 1)
    assert rel.max() <= BAR_REL


def test_frames512_full(shape):
    """4,096 512^2 frames: detection sampled frame by frame, cut-outs exact."""
    import torch
    f = synth.make_frames()
    fr = shape.DeviceFrames.from_host(f, "cuda:0")
    d = shape.frame_detect(fr)
    db = shape.frame_cut(fr, d["box"], torch.from_numpy(f.sigma).cuda())
    torch.cuda.synchronize()
    box, peak = d["box"].cpu().numpy(), d["peak"].cpu().numpy()
    off, stamps = db.offsets.cpu().numpy(), db.pixels.cpu().numpy()
    for i in np.sort(np.random.default_rng(14).choice(f.n, 48, replace=False)):
        r = oracle.frame_detect(f.pixels[i].astype(np.float64))
        assert tuple(peak[i]) == r["peak"] and tuple(box[i]) == r["box"], i
        s = int(box[i, 2])
        np.testing.assert_array_equal(stamps[off[i]:off[i] + s * s].reshape(s, s),
                                      oracle.frame_cut(f.pixels[i], r["box"]))


@pytest.mark.parametrize("linear_init", [1, 0])
def test_plain32x_full(shape, linear_init):
    """262,144 32^2 Gaussian galaxies, 4-parameter fit, profiled and unprofiled."""
    b = synth.make("plain32x")
    db = shape.DeviceBatch.from_host(b, "cuda:0")
    o = shape.default_opts(free_mask=shape.MASK_SIZE, linear_init=linear_init)
    g = _gpu_pipeline(shape, db, o)
    idx = np.sort(np.random.default_rng(15).choice(b.n, SAMPLE, replace=False))
    sub = _subset(b, idx)
    ref = oracle.pipeline(sub, oracle_opts_like(o, tol_lm=1e-9, max_iter_lm=200))
    r = compare({k: v[idx] for k, v in g.items()}, ref, 0xF0, "plain32x li=%d" % linear_init,
                batch=sub)
    check_fit(r, 0.95)
