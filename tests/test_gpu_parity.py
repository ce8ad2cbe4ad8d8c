"""GPU parity: the HIP stages against the FP64 oracle on seeded stamps.

Stages: centroid and moments within |dx|, |dy| <= 1e-3 px and |de| <= 1e-4 on
stamps both sides converge.  Fit: the rule of parity_util (bars on stamps both
sides fit to the interior of the parameter box, chi^2, sigma_p and amplitudes
checked there, every disagreement validated as an equally good minimum of the
oracle's chi^2).  Inputs are the synthetic workloads of the generator (the
paper's simulation recipe, Sec. 4.1)."""
import numpy as np
import pytest

import oracle
import synth
from parity_util import (BAR_E, BAR_REL, BAR_X, check_fit, compare, fit_class, oracle_opts_like,
                         run_gpu, validate_minimum)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def shape():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1203_0571_amd as shape
    return shape


def _check_stages(r):
    assert r["centroid_dxy"] <= BAR_X, r
    assert r["moments_dxy"] <= BAR_X and r["moments_de"] <= BAR_E, r
    assert r["size_rel"] <= 1e-3 and r["size_defined_agree"] >= 0.99, r


def test_gaussian_workload_4_params(shape):
    """1,000 x 32^2 Gaussian galaxies, centroid + moments + (Re, n, I0, sky) fit."""
    b = synth.make("plain32")
    o = shape.default_opts(free_mask=shape.MASK_SIZE)
    g = run_gpu(shape, b, o)
    ref = oracle.pipeline(b, oracle_opts_like(o, tol_lm=1e-9, max_iter_lm=200))
    r = compare(g, ref, 0xF0, "plain32", batch=b)
    assert r["r50_rel"] < 1e-5 and r["sigw_rel"] < 1e-5
    assert r["status0_agree"] > 0.99 and r["status1_agree"] > 0.99
    _check_stages(r)
    check_fit(r, 0.98)
    # the centre and ellipticity are held in the 4-parameter fit
    conv = (g["status"][:, 2] & shape.ST_CONVERGED) != 0
    np.testing.assert_array_equal(g["p"][conv, :4], g["moments"][conv, :4])


def test_unprofiled_4_params(shape):
    """The unprofiled form (linear_init = 0: I0 and sky searched with Re and n
    by the same LM) against the oracle's unprofiled form; it reaches the
    profiled fit's minimum in more trials."""
    b = synth.make("plain32", count=512)
    o = shape.default_opts(free_mask=shape.MASK_SIZE, linear_init=0)
    g = run_gpu(shape, b, o)
    ref = oracle.pipeline(b, oracle_opts_like(o, tol_lm=1e-9, max_iter_lm=200))
    r = compare(g, ref, 0xF0, "plain32 unprofiled", batch=b)
    _check_stages(r)
    check_fit(r, 0.95)
    gp = run_gpu(shape, b, shape.default_opts(free_mask=shape.MASK_SIZE))
    both = ((g["status"][:, 2] & gp["status"][:, 2] & shape.ST_CONVERGED) != 0)
    assert both.mean() > 0.95
    rel = np.abs(g["p"][both, 4:6] / gp["p"][both, 4:6] - 1)
    assert rel.max() <= BAR_REL
    assert g["iters"][both, 2].mean() > gp["iters"][both, 2].mean()


@pytest.mark.parametrize("workload,count", [("plain48", 2048), ("sersic64", 1024)])
def test_sersic_workloads_8_params(shape, workload, count):
    b = synth.make(workload, count=count)
    o = shape.default_opts()
    g = run_gpu(shape, b, o)
    ref = oracle.pipeline(b, oracle_opts_like(o, tol_lm=1e-9, max_iter_lm=200))
    r = compare(g, ref, 0xFF, workload, batch=b)
    _check_stages(r)
    check_fit(r, 0.85)


@pytest.mark.parametrize("side", [16, 32])
def test_row_layout_8_params_small_sides(shape, side):
    """Uniform batches of side 16 and 32 with all eight parameters free take
    the row layout's moment form (the shape columns summed as moments of
    h u2^j per lane column) at 4 and 16 rows per lane: the fit's parity rule
    against the oracle, Sersic galaxies of Re ~ side/8 (Sec. 4.1 recipe)."""
    rng = np.random.default_rng(100 + side)
    stamps, sig = [], []
    for k in range(256):
        c = (side - 1) / 2.0 + rng.uniform(-1.0, 1.0, 2)
        e = np.clip(rng.normal(0.0, 0.25, 2), -0.45, 0.45)
        re = side / 8.0 * np.exp(rng.uniform(-0.3, 0.3))
        p = np.array([c[0], c[1], e[0], e[1], re, rng.uniform(0.5, 4.0), 0.0, 10.0])
        prof = synth.render_sersic(side, np.concatenate([p[:6], [1.0, 0.0]]))[0]
        flux = np.exp(rng.uniform(np.log(2e3), np.log(2e4)))
        img = prof * (flux / prof.sum()) + 10.0
        s_ = float(np.sqrt(img.max() - 10.0) / 8.0 + 1.0)
        stamps.append(img + rng.normal(0.0, s_, img.shape))
        sig.append(s_)
    b = _custom_batch(stamps, sig)
    o = shape.default_opts()
    g = run_gpu(shape, b, o)
    ref = oracle.pipeline(b, oracle_opts_like(o, tol_lm=1e-9, max_iter_lm=200))
    r = compare(g, ref, 0xFF, "sersic%d" % side, batch=b)
    _check_stages(r)
    check_fit(r, 0.8)


def test_fit_from_pixel_centred_start(shape):
    """Fits started with the centre exactly on a pixel centre: the first sweep
    meets R^2 = 0 there (the floor, with the shape columns' factor h set to
    zero) in the row layout's moment form.  Every fit stays finite, and the
    fits agree with the oracle's fits from the same starting points by the
    bars, or end at a validated minimum of the oracle's chi^2."""
    import torch
    b = synth.make("sersic64", count=64)
    p0 = b.truth.astype(np.float64).copy()
    p0[:, :2] = np.round(p0[:, :2])
    db = shape.DeviceBatch.from_host(b, "cuda:0")
    out = shape.fit_sersic(db, p_init=torch.from_numpy(p0.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items() if hasattr(v, "cpu")}
    assert np.isfinite(g["p"]).all() and np.isfinite(g["chi2"]).all()
    assert ((g["status"] & shape.ST_NONFINITE_INPUT) == 0).all()
    pix = b.dequantised_f64()
    o = oracle.opts(tol_lm=1e-9, max_iter_lm=200)
    both = 0
    for s in range(b.n):
        img = pix[b.offsets[s]:b.offsets[s] + 64 * 64].reshape(64, 64)
        ref = oracle.fit(img, float(b.sigma[s]), p0[s].astype(np.float32).astype(np.float64), o=o)
        if not (g["status"][s] & shape.ST_CONVERGED and ref["status"] & oracle.CONVERGED):
            continue
        if (g["status"][s] | ref["status"]) & oracle.AT_BOUND:
            continue
        both += 1
        pg = g["p"][s].astype(np.float64)
        inside = (np.abs(pg[:2] - ref["p"][:2]).max() <= BAR_X and
                  np.abs(pg[2:4] - ref["p"][2:4]).max() <= BAR_E and
                  np.abs(pg[4:6] / ref["p"][4:6] - 1).max() <= BAR_REL)
        if not inside:
            assert validate_minimum(img, float(b.sigma[s]), 0, pg, ref["chi2"],
                                    list(range(8)))[0], s
    assert both >= 56, both


def test_standard_error_stop_only_adds_convergence(shape):
    """The stop on steps below tol_sigma standard errors is an extra way to
    converge: every stamp that converges without it converges with it (the
    trajectories agree until the rule fires), and both meet the bars."""
    b = synth.make("sersic64", count=512)
    o = shape.default_opts()
    o0 = shape.default_opts(tol_sigma=0.0)
    g, g0 = run_gpu(shape, b, o), run_gpu(shape, b, o0)
    ref = oracle.pipeline(b, oracle_opts_like(o, tol_lm=1e-9, max_iter_lm=200))
    for gg, label in ((g, "tol_sigma default"), (g0, "tol_sigma 0")):
        r = compare(gg, ref, 0xFF, label, batch=b)
        _check_stages(r)
        check_fit(r, 0.85)
    c, c0 = (((x["status"][:, 2] & shape.ST_CONVERGED) != 0) for x in (g, g0))
    assert np.all(c[c0])
    assert g["iters"][c0, 2].mean() <= g0["iters"][c0, 2].mean()


def test_fp16_storage(shape):
    """FP16 stamps with a per-stamp scale: the oracle reads the same dequantised pixels."""
    b = synth.make("sersic64h", count=1024)
    o = shape.default_opts()
    g = run_gpu(shape, b, o)
    ref = oracle.pipeline(b, oracle_opts_like(o, tol_lm=1e-9, max_iter_lm=200))
    r = compare(g, ref, 0xFF, "sersic64h", batch=b)
    _check_stages(r)
    check_fit(r, 0.85)


def test_uneven_sizes_and_moffat_stars(shape):
    b = synth.make("uneven", count=1024)
    o = shape.default_opts()
    g = run_gpu(shape, b, o)
    ref = oracle.pipeline(b, oracle_opts_like(o, tol_lm=1e-9, max_iter_lm=200))
    r = compare(g, ref, 0xFF, "uneven", batch=b)
    _check_stages(r)
    check_fit(r, 0.8)
    stars = b.model == 1
    assert ((g["status"][stars, 2] & shape.ST_CONVERGED) != 0).mean() > 0.8


def _custom_batch(stamps, sigmas, sides=None, offsets=None, n_pixels=None):
    pix = np.concatenate([np.asarray(s, np.float32).ravel() for s in stamps])
    sides_a = np.array([s.shape[0] for s in stamps] if sides is None else sides, np.int32)
    if offsets is None:
        offsets = np.concatenate([[0], np.cumsum([s.size for s in stamps])[:-1]]).astype(np.int64)
    b = synth.Batch("custom", pix, np.asarray(offsets, np.int64), sides_a,
                    np.asarray(sigmas, np.float32), np.zeros(len(stamps), np.uint8),
                    np.zeros((len(stamps), 8)), None)
    return b


def test_edge_cases(shape):
    import torch
    rng = np.random.default_rng(7)
    small = synth.render_sersic(4, np.array([1.6, 1.4, 0.1, 0.0, 1.0, 1.0, 500.0, 10.0]))[0] + 10
    small = small + rng.normal(0, 1.0, small.shape)
    big = synth.render_sersic(128, np.array([63.2, 64.1, 0.3, -0.2, 9.0, 1.5, 300.0, 10.0]))[0] + 10
    big = big + rng.normal(0, 2.0, big.shape)
    mid = synth.render_sersic(40, np.array([19.2, 20.1, 0.2, 0.1, 3.0, 2.0, 800.0, 10.0]))[0] + 10
    mid = mid + rng.normal(0, 3.0, mid.shape)
    nan = mid.copy()
    nan[5, 7] = np.nan
    flat = np.full((24, 24), 10.0)
    stamps = [small, big, mid, nan, mid, flat]
    sig = [1.0, 2.0, 3.0, 3.0, -1.0, 1.0]
    b = _custom_batch(stamps, sig)
    g = run_gpu(shape, b)
    ref = oracle.pipeline(b, oracle_opts_like(shape.default_opts(), tol_lm=1e-9, max_iter_lm=200))
    st = g["status"]
    assert st[3, 0] == shape.ST_NONFINITE_INPUT and np.isnan(g["p"][3]).all()
    assert st[4, 0] == shape.ST_BAD_INPUT and st[4, 2] == shape.ST_BAD_INPUT
    assert st[5, 0] & shape.ST_NONPOSITIVE_FLUX
    np.testing.assert_array_equal(st[:, 0], ref["status"][:, 0])
    for s in (1, 2):   # max side and an ordinary ragged stamp
        assert st[s, 2] & shape.ST_CONVERGED and ref["status"][s, 2] & oracle.CONVERGED
        assert np.abs(g["p"][s, :2] - ref["p"][s, :2]).max() <= BAR_X
        assert np.abs(g["p"][s, 2:4] - ref["p"][s, 2:4]).max() <= BAR_E
        assert np.abs(g["p"][s, 4:6] / ref["p"][s, 4:6] - 1).max() <= BAR_REL
    # side out of range and a stamp that overruns the pixel buffer
    b2 = _custom_batch([mid, mid, mid], [3.0, 3.0, 3.0], sides=[3, 200, 40],
                       offsets=[0, 0, 40 * 40 * 2 + 1])
    g2 = run_gpu(shape, b2)
    assert (g2["status"][:, 0] == shape.ST_BAD_INPUT).all()
    assert np.isnan(g2["p"]).all()
    # empty batch
    e = shape.DeviceBatch(pixels=torch.zeros(0, device="cuda"), sigma=torch.zeros(0, device="cuda"),
                          side0=16)
    out = shape.pipeline(e)
    assert out["p"].shape == (0, 8)


def test_two_stamps_per_wave(shape):
    """Batches of 32 x 32 stamps take two stamps per wave in the register-stamp
    centroid and moments: a stamp's results do not depend on its partner (bit
    for bit, against a batch that pairs it differently), a failing stamp
    leaves its partner alone, and an odd count leaves the last stamp without
    one.  Statuses agree with the oracle."""
    rng = np.random.default_rng(11)

    def gal(x, y, e1, e2, re, n, amp):
        img = synth.render_sersic(32, np.array([x, y, e1, e2, re, n, amp, 10.0]))[0] + 10
        return img + rng.normal(0, 2.0, img.shape)

    A = gal(15.3, 16.1, 0.2, -0.1, 3.0, 1.5, 600.0)
    B = gal(14.2, 15.7, -0.3, 0.1, 4.0, 0.8, 400.0)
    C = gal(16.8, 14.9, 0.05, 0.25, 2.5, 2.5, 900.0)
    nan = A.copy()
    nan[3, 9] = np.nan
    flat = np.full((32, 32), 10.0)
    # pairs: (A, nan), (B, A with sigma <= 0), (flat, C), (B, -)
    b1 = _custom_batch([A, nan, B, A, flat, C, B], [2.0, 2.0, 2.0, -1.0, 1.0, 2.0, 2.0])
    b2 = _custom_batch([C, B, A], [2.0, 2.0, 2.0])
    o = shape.default_opts()
    outs = []
    for b in (b1, b2):
        db = shape.DeviceBatch.from_host(b, "cuda:0")
        assert db.side0 == 32 and db.sides is None
        rec0, it0, st0 = shape.centroid(db, o)
        rec1, it1, st1 = shape.moments(db, rec0, o)
        outs.append([x.cpu().numpy() for x in (rec0, it0, st0, rec1, it1, st1)])
    for i1, i2 in ((0, 2), (2, 1), (5, 0), (6, 1)):
        for a, c in zip(outs[0], outs[1]):
            np.testing.assert_array_equal(a[i1], c[i2])
    st0, st1 = outs[0][2], outs[0][5]
    assert st0[1] == shape.ST_NONFINITE_INPUT and st0[3] == shape.ST_BAD_INPUT
    # the moments stage rejects the failed centroid records themselves
    assert st1[1] == shape.ST_BAD_INPUT and st1[3] == shape.ST_BAD_INPUT
    assert st0[4] & shape.ST_NONPOSITIVE_FLUX
    assert np.isnan(outs[0][0][1]).all() and np.isnan(outs[0][3][3]).all()
    ref = oracle.pipeline(b1, oracle_opts_like(o))
    np.testing.assert_array_equal(st0, ref["status"][:, 0])
    good = [0, 2, 5, 6]
    np.testing.assert_array_equal(st1[good + [4]], ref["status"][good + [4], 1])
    assert np.abs(outs[0][3][good, :2] - ref["mom"][good, :2]).max() <= BAR_X
    assert np.abs(outs[0][3][good, 2:4] - ref["mom"][good, 2:4]).max() <= BAR_E


def test_every_side_stages(shape):
    """Centroid and moments on one batch holding every side from 4 to 128
    (two stamps each, mixed in order): every register layout of the any-side
    forms (one wave up to side 64, a team of four above) against the oracle."""
    rng = np.random.default_rng(11)
    stamps, sig = [], []
    for side in range(4, 129):
        for k in range(2):
            re = max(0.6, side / 8.0 * rng.uniform(0.7, 1.3))
            c = (side - 1) / 2.0 + rng.uniform(-0.3, 0.3, 2) * max(1.0, side / 16.0)
            e = rng.uniform(-0.2, 0.2, 2)
            p = np.array([c[0], c[1], e[0], e[1], re, rng.uniform(0.7, 3.0), 400.0, 0.0])
            img = synth.render_sersic(side, p)[0] + 10.0
            stamps.append(img + rng.normal(0, 1.5, img.shape))
            sig.append(1.5)
    order = rng.permutation(len(stamps))
    b = _custom_batch([stamps[i] for i in order], [sig[i] for i in order])
    o = shape.default_opts()
    g = run_gpu(shape, b, o)
    ref = oracle.pipeline(b, oracle_opts_like(o, max_iter_lm=1))
    st_g, st_o = g["status"].astype(np.uint32), ref["status"]
    assert (st_g[:, 0] == st_o[:, 0]).mean() >= 0.99
    assert (st_g[:, 1] == st_o[:, 1]).mean() >= 0.98
    lost = ((st_g[:, 0] | st_o[:, 0]) & oracle.LOST) != 0
    ok0 = ~lost
    assert ok0.mean() > 0.95
    cg, mo = g["centroid"], ref["mom"]
    assert np.abs(cg[ok0, :2] - ref["xy"][ok0]).max() <= BAR_X
    assert np.abs(cg[ok0, 5] / mo[ok0, 5] - 1).max() <= 1e-5      # r50
    assert np.abs(cg[ok0, 4] / mo[ok0, 4] - 1).max() <= 1e-5      # sigma_w
    both = ((st_g[:, 1] & st_o[:, 1]) & oracle.CONVERGED) != 0
    assert both.mean() > 0.9
    mg = g["moments"]
    assert np.abs(mg[both, :2] - mo[both, :2]).max() <= BAR_X
    assert np.abs(mg[both, 2:4] - mo[both, 2:4]).max() <= BAR_E


def test_deterministic(shape):
    b = synth.make("plain48", count=512)
    g1 = run_gpu(shape, b)
    g2 = run_gpu(shape, b)
    for k in ("centroid", "moments", "p", "chi2", "iters", "status"):
        np.testing.assert_array_equal(g1[k], g2[k])


def test_full_size_sampled(shape):
    """The 65,536 x 64^2 workload at full size in one launch per stage; 128
    sampled stamps are recomputed by the oracle one by one."""
    b = synth.make("sersic64")
    o = shape.default_opts()
    g = run_gpu(shape, b, o)
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(b.n, 128, replace=False))
    sub = synth.Batch("sample", np.concatenate([b.pixels[b.offsets[i]:b.offsets[i] + 4096] for i in idx]),
                      np.arange(128, dtype=np.int64) * 4096, b.sides[idx], b.sigma[idx],
                      b.model[idx], b.truth[idx], None)
    ref = oracle.pipeline(sub, oracle_opts_like(o, tol_lm=1e-9, max_iter_lm=200))
    gs = {k: v[idx] for k, v in g.items() if isinstance(v, np.ndarray) and v.shape[:1] == (b.n,)}
    r = compare(gs, ref, 0xFF, "sersic64 full, sampled", batch=sub)
    _check_stages(r)
    check_fit(r, 0.85)
    conv = (g["status"][:, 2] & shape.ST_CONVERGED) != 0
    print("full-size convergence fraction %.4f" % conv.mean())
    assert conv.mean() > 0.85


@pytest.mark.parametrize("workload", ["plain32", "sersic64h"])
def test_register_and_memory_paths_agree(shape, workload):
    """A uniform batch takes the register-stamp centroid/moments and the
    column-per-lane fit sweep; the same stamps with a side array take the
    memory paths and the generic sweep.  Two codings of the same stages: they
    agree within the parity bars, and their statuses agree."""
    import torch
    b = synth.make(workload, count=512)
    o = shape.default_opts(free_mask=shape.MASK_SIZE) if workload == "plain32" else shape.default_opts()
    outs = []
    for uniform in (True, False):
        db = shape.DeviceBatch.from_host(b, "cuda:0", uniform=uniform)
        out = shape.pipeline(db, o)
        torch.cuda.synchronize()
        outs.append({k: v.cpu().numpy() for k, v in out.items() if hasattr(v, "cpu")})
    r, m = outs
    for stage in ("centroid", "moments"):
        k = 0 if stage == "centroid" else 1
        ok = ((r["status"][:, k] & m["status"][:, k] & shape.ST_CONVERGED) != 0)
        assert (r["status"][:, k] == m["status"][:, k]).mean() > 0.99, stage
        assert ok.mean() > 0.85, stage   # the workloads' own converged fractions (~0.9 at 64^2)
        assert np.abs(r[stage][ok, :2] - m[stage][ok, :2]).max() <= BAR_X
        if stage == "moments":
            assert np.abs(r[stage][ok, 2:4] - m[stage][ok, 2:4]).max() <= BAR_E
    both = (fit_class(r["status"][:, 2]) == "interior") & (fit_class(m["status"][:, 2]) == "interior")
    assert both.mean() > 0.85
    mask = 0xF0 if workload == "plain32" else 0xFF
    pr, pm = r["p"].astype(np.float64), m["p"].astype(np.float64)
    ok = (np.abs(pr[:, :2] - pm[:, :2]).max(1) <= BAR_X) & \
         (np.abs(pr[:, 2:4] - pm[:, 2:4]).max(1) <= BAR_E) & \
         (np.abs(pr[:, 4:6] / pm[:, 4:6] - 1).max(1) <= BAR_REL)
    # where the two codings part, each must have ended at a stationary point
    # of the oracle's chi^2 (two minima of a flat valley)
    pix = b.dequantised_f64()
    idx = [k for k in range(8) if (mask >> k) & 1]
    for s in np.flatnonzero(both & ~ok):
        img = pix[b.offsets[s]:b.offsets[s] + b.sides[s] ** 2].reshape(b.sides[s], b.sides[s])
        sig = float(b.sigma[s])
        for pp in (pr[s], pm[s]):
            c = oracle.chi2(img, sig, pp)
            assert validate_minimum(img, sig, 0, pp, c, idx)[0], s
