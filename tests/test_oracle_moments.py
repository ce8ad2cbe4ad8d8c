"""Pins of the oracle's starting estimates, centroid (Sec. 2) and
elliptical-weight KSB iteration (Sec. 3, App. A, App. B).

The App. A polarisability is pinned by its defining property: the first-order
response of the weighted ellipticity to a shear applied to the image with the
weight held fixed.  The App. B-corrected matrix (with g read as g_w) is pinned
by the response of e_obs to the source's own ellipticity at the aligned point,
divided out by (1 - |g|^2) as in eq. newg.  Both are checked by finite
differences on Gaussian images, where pixel sums equal the integrals.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def grid(side):
    j, i = np.meshgrid(np.arange(side, dtype=float), np.arange(side, dtype=float))
    return j, i


def gauss_cov(side, cov, x0, y0, amp=1000.0, sky=0.0, shear=None):
    j, i = grid(side)
    u = np.stack([j - x0, i - y0], -1)
    if shear is not None:
        A = np.array([[1 - shear[0], -shear[1]], [-shear[1], 1 + shear[0]]])
        u = u @ A.T
    q = np.einsum("...i,ij,...j->...", u, np.linalg.inv(cov), u)
    return amp * np.exp(-0.5 * q) + sky


def elliptical_src(side, g, width, x0, y0, amp=1000.0):
    """Gaussian source whose isophotes are |S(g) u| = const."""
    j, i = grid(side)
    u1, u2 = j - x0, i - y0
    v1 = (1 - g[0]) * u1 - g[1] * u2
    v2 = -g[1] * u1 + (1 + g[0]) * u2
    return amp * np.exp(-(v1 * v1 + v2 * v2) / (2 * width * width))


def one_step(img, sky0, sigw, x, y, k=1.0):
    o = oracle.opts(max_iter_centroid=1, k_gain=k)
    xx, yy, _, _ = oracle.centroid(img, sky0, sigw, x, y, o)
    return xx - x, yy - y


@pytest.mark.parametrize("sigma,sigw", [(2.0, 2.0), (2.0, 3.0), (3.0, 2.0), (1.6, 4.0)])
def test_centroid_gain(sigma, sigw):
    """<x>/N = k dx with k = sigma_w^2 / (sigma^2 + sigma_w^2) (Sec. 2)."""
    side = 80
    c = (side - 1) / 2
    dx, dy = 1.37, -0.82
    img = gauss_cov(side, np.eye(2) * sigma ** 2, c + dx, c + dy)
    sx, sy = one_step(img, 0.0, sigw, c, c)
    k = sigw ** 2 / (sigma ** 2 + sigw ** 2)
    assert sx == pytest.approx(k * dx, rel=1e-10)
    assert sy == pytest.approx(k * dy, rel=1e-10)
    if sigma == sigw:
        assert sx / dx == pytest.approx(GOLD["centroid_gain_equal_widths"]["value"], rel=1e-10)


def test_centroid_gain_compact_limit():
    side = 32
    img = np.zeros((side, side))
    img[17, 12] = 500.0          # a point source on a pixel centre
    sx, sy = one_step(img, 0.0, 3.0, 15.0, 19.0)
    assert sx / (12 - 15.0) == pytest.approx(GOLD["centroid_gain_point_source"]["value"], rel=1e-12)
    assert sy / (17 - 19.0) == pytest.approx(1.0, rel=1e-12)


@pytest.mark.parametrize("sigma", [1.5, 2.0, 2.5, 2.9])
def test_centroid_contraction(sigma):
    """With k = 0.75 and 0.5 < k_true < 1 each step cuts the offset by 3 or more."""
    side, sigw = 64, 3.0
    c = (side - 1) / 2
    true = np.array([c + 2.3, c - 1.9])
    img = gauss_cov(side, np.eye(2) * sigma ** 2, *true)
    x, y = c, c
    bound = GOLD["centroid_contraction"]["value"]
    for _ in range(6):
        d0 = math.hypot(x - true[0], y - true[1])
        sx, sy = one_step(img, 0.0, sigw, x, y, k=GOLD["centroid_fixed_gain"]["value"])
        x, y = x + sx, y + sy
        d1 = math.hypot(x - true[0], y - true[1])
        assert d1 <= bound * d0 + 1e-12


def test_centroid_fixed_point_is_symmetry_centre():
    side = 48
    true = (23.87, 21.36)
    img = gauss_cov(side, np.array([[6.0, 1.2], [1.2, 4.0]]), *true, sky=10.0)
    o = oracle.opts(tol_x=1e-12, max_iter_centroid=200)
    x, y, it, st = oracle.centroid(img, 10.0, 2.5, 22.0, 22.0, o)
    assert st & oracle.CONVERGED
    assert abs(x - true[0]) < 1e-9 and abs(y - true[1]) < 1e-9


def test_init_brute_force_growth_curve():
    """Border-mean sky, argmax, and the first crossing of F/2 of the circular
    growth curve, checked against a sort-by-distance brute force."""
    rng = np.random.default_rng(5)
    for trial in range(20):
        side = int(rng.integers(6, 14))
        img = rng.normal(10.0, 1.0, (side, side))
        i0, j0 = rng.integers(1, side - 1, 2)
        img[i0, j0] += 40.0 + 10 * trial
        img[i0 - 1:i0 + 2, j0 - 1:j0 + 2] += 8.0
        got = oracle.init(img)
        border = np.concatenate([img[0], img[-1], img[1:-1, 0], img[1:-1, -1]])
        sky = border.mean()
        assert got["sky0"] == pytest.approx(sky, rel=1e-14)
        assert got["imax"] == int(np.argmax(img))
        bi, bj = divmod(got["imax"], side)
        ii, jj = np.indices((side, side))
        d = np.sqrt((ii - bi) ** 2 + (jj - bj) ** 2).ravel()
        f = (img - sky).ravel()
        F = f.sum()
        radii = np.arange(0, 2 * side)
        cum = np.array([f[d <= r + 1e-12].sum() for r in radii])
        cum[0] = 0.0              # the curve starts from zero flux at radius 0
        r = int(np.argmax(cum >= F / 2))
        r50 = (r - 1) + (F / 2 - cum[r - 1]) / (cum[r] - cum[r - 1])
        assert got["r50"] == pytest.approx(r50, rel=1e-12)
        assert got["sigw"] == pytest.approx(min(max(r50 / math.sqrt(2 * math.log(2)), 1.0), side / 4), rel=1e-12)


def test_weighted_second_moments_closed_form():
    """Gaussian source x elliptical Gaussian weight: N = I0 2 pi sqrt(det C) and
    Q = N C with C = (C_f^-1 + C_w^-1)^-1, C_w^-1 = S(g_w)^T S(g_w) / sigma_w^2."""
    side = 96
    c = (side - 1) / 2
    Cf = np.array([[9.0, 2.5], [2.5, 5.0]])
    img = gauss_cov(side, Cf, c, c, amp=700.0)
    for gw in [(0.0, 0.0), (0.2, -0.3), (-0.4, 0.1)]:
        sigw = 3.3
        S = np.array([[1 - gw[0], -gw[1]], [-gw[1], 1 + gw[0]]])
        C = np.linalg.inv(np.linalg.inv(Cf) + S.T @ S / sigw ** 2)
        N = 700.0 * 2 * math.pi * math.sqrt(np.linalg.det(C))
        t = oracle.ksb_terms(img, 0.0, sigw, c, c, np.array(gw))
        assert t["N"] == pytest.approx(N, rel=1e-10)
        assert t["T"] == pytest.approx(N * (C[0, 0] + C[1, 1]), rel=1e-10)
        e_ref = np.array([C[0, 0] - C[1, 1], 2 * C[0, 1]]) / (C[0, 0] + C[1, 1])
        np.testing.assert_allclose(t["e"], e_ref, atol=1e-11)
        np.testing.assert_allclose(t["S"], [0.0, 0.0], atol=1e-9 * N)


@pytest.mark.parametrize("gw", [(0.0, 0.0), (0.3, -0.2), (-0.1, 0.5)])
@pytest.mark.parametrize("cov", [((9.0, 0.0), (0.0, 9.0)), ((12.0, 3.0), (3.0, 7.0))])
def test_app_a_polarisability_is_shear_response(gw, cov):
    """X^SH - e (x) e^SH (App. A) = d e_obs / d(applied shear), weight fixed."""
    side = 96
    c = (side - 1) / 2
    cov = np.array(cov)
    mk = lambda s: gauss_cov(side, cov, c, c, shear=s)
    t = oracle.ksb_terms(mk(None), 0.0, 5.0, c, c, np.array(gw))
    P = t["X"] - np.outer(t["e"], t["eSH"])
    h = 1e-5
    J = np.zeros((2, 2))
    for k in range(2):
        d = np.zeros(2)
        d[k] = h
        ep = oracle.ksb_terms(mk(d), 0.0, 5.0, c, c, np.array(gw))["e"]
        em = oracle.ksb_terms(mk(-d), 0.0, 5.0, c, c, np.array(gw))["e"]
        J[:, k] = (ep - em) / (2 * h)
    np.testing.assert_allclose(P, J, atol=1e-8)


@pytest.mark.parametrize("g", [(0.3, -0.2), (0.5, 0.1), (0.1, 0.0), (-0.25, 0.55)])
def test_app_b_polarisability_is_source_response(g):
    """(X + dX - e (x) (e^SH + de)) / (1 - |g|^2) = d e_obs / d g_source at the
    aligned point g_source = g_w (App. B with g read as g_w, eq. newg)."""
    side = 128
    c = (side - 1) / 2
    g = np.array(g)
    t = oracle.ksb_terms(elliptical_src(side, g, 5.0, c, c), 0.0, 6.0, c, c, g)
    P = t["X"] + t["dX"] - np.outer(t["e"], t["eSH"] + t["de"])
    h = 1e-5
    J = np.zeros((2, 2))
    for k in range(2):
        d = np.zeros(2)
        d[k] = h
        ep = oracle.ksb_terms(elliptical_src(side, g + d, 5.0, c, c), 0.0, 6.0, c, c, g)["e"]
        em = oracle.ksb_terms(elliptical_src(side, g - d, 5.0, c, c), 0.0, 6.0, c, c, g)["e"]
        J[:, k] = (ep - em) / (2 * h)
    np.testing.assert_allclose(P / (1 - g @ g), J, atol=2e-8)
    # at g_w = 0 the App. B terms vanish (KSB limit)
    t0 = oracle.ksb_terms(elliptical_src(side, g, 5.0, c, c), 0.0, 6.0, c, c, np.zeros(2))
    assert np.abs(t0["dX"]).max() == 0.0 and np.abs(t0["de"]).max() == 0.0


@pytest.mark.parametrize("g", [(0.0, 0.0), (0.3, -0.2), (0.5, 0.3), (-0.6, 0.2), (0.1, -0.65)])
def test_moments_recover_gaussian_shape(g):
    """The iteration's fixed point is the source's own ellipticity and centre."""
    side = 96
    true = (48.31, 46.77)
    img = elliptical_src(side, g, 3.5, *true) + 10.0
    o = oracle.opts(tol_x=1e-11, tol_g=1e-11, max_iter_moments=60)
    out, it, st = oracle.moments(img, 10.0, 4.0, 4.7, 47.0, 47.0, o)
    assert st & oracle.CONVERGED
    np.testing.assert_allclose(out[:2], true, atol=1e-8)
    np.testing.assert_allclose(out[2:4], g, atol=1e-9)


def test_moments_converges_fast_with_app_b():
    """A few iterations from the circular-weight start (Sec. 3 claim of quick convergence)."""
    side = 96
    img = elliptical_src(side, (0.45, -0.3), 3.5, 47.5, 47.5)
    o = oracle.opts(tol_x=1e-9, tol_g=1e-9, max_iter_moments=60)
    out, it, st = oracle.moments(img, 0.0, 4.0, 4.7, 47.5, 47.5, o)
    assert st & oracle.CONVERGED
    assert it <= 15


def _pipeline_on(stamps, sigma=5.0):
    side = stamps[0].shape[0]
    pix = np.concatenate([s.ravel() for s in stamps])
    n = len(stamps)
    b = synth.Batch("custom", pix.astype(np.float64), np.arange(n, dtype=np.int64) * side * side,
                    np.full(n, side, np.int32), np.full(n, sigma, np.float32),
                    np.zeros(n, np.uint8), np.zeros((n, 8)), None)
    return oracle.pipeline(b, oracle.opts(max_iter_lm=0), pixels_f64=pix)


def test_pixel_permutation_invariants():
    """rot90 flips (e1, e2); a transpose flips e1; an x-mirror flips e2; the
    centroid maps with the pixels.  Exact up to summation order."""
    b = synth.make("plain48", count=16)
    W = 48
    base, rot, tr, mir = [], [], [], []
    for s in range(b.n):
        img = b.stamp(s)
        base.append(img)
        rot.append(np.rot90(img, 2))      # 180 deg: e unchanged, centre mirrored
        tr.append(img.T)
        mir.append(img[:, ::-1])
    r0, r_rot, r_tr, r_mir = (_pipeline_on(x) for x in (base, rot, tr, mir))
    ok = (r0["status"][:, 1] & oracle.CONVERGED) != 0
    m0, mr, mt, mm = r0["mom"][ok], r_rot["mom"][ok], r_tr["mom"][ok], r_mir["mom"][ok]
    np.testing.assert_allclose(mr[:, 0], W - 1 - m0[:, 0], atol=1e-9)
    np.testing.assert_allclose(mr[:, 2:4], m0[:, 2:4], atol=1e-9)
    np.testing.assert_allclose(mt[:, 0], m0[:, 1], atol=1e-9)
    np.testing.assert_allclose(mt[:, 2], -m0[:, 2], atol=1e-9)
    np.testing.assert_allclose(mt[:, 3], m0[:, 3], atol=1e-9)
    np.testing.assert_allclose(mm[:, 0], W - 1 - m0[:, 0], atol=1e-9)
    np.testing.assert_allclose(mm[:, 2], m0[:, 2], atol=1e-9)
    np.testing.assert_allclose(mm[:, 3], -m0[:, 3], atol=1e-9)
    assert ok.sum() >= 12


def test_rot90_flips_both_components():
    side = 64
    img = elliptical_src(side, (0.3, 0.2), 3.0, 31.5, 31.5) + 10.0
    a = _pipeline_on([img, np.rot90(img)])
    np.testing.assert_allclose(a["mom"][1, 2:4], -a["mom"][0, 2:4], atol=1e-9)


def test_rotation_45_degrees_swaps_components():
    """Re-rendering at 45 deg rotated parameters maps (e1, e2) -> (-e2, e1)."""
    side = 96
    c = (side - 1) / 2
    e = np.array([0.35, -0.15])
    img1 = elliptical_src(side, e, 4.0, c, c) + 10.0
    img2 = elliptical_src(side, np.array([-e[1], e[0]]), 4.0, c, c) + 10.0
    o = oracle.opts(tol_x=1e-11, tol_g=1e-11, max_iter_moments=60)
    o1, _, _ = oracle.moments(img1, 10.0, 4.0, 4.7, c, c, o)
    o2, _, _ = oracle.moments(img2, 10.0, 4.0, 4.7, c, c, o)
    np.testing.assert_allclose(o2[2:4], [-o1[3], o1[2]], atol=1e-9)


def test_step_halving_keeps_weight_inside_disk():
    side = 96
    g = np.array([0.6, 0.3])           # |g| = 0.67: the undamped iteration leaves the disk
    img = synth.render_sersic(side, np.array([47.5, 47.5, g[0], g[1], 6.0, 1.0, 1000.0, 0.0]))[0]
    o = oracle.opts(tol_x=1e-9, tol_g=1e-9, max_iter_moments=60)
    out, it, st = oracle.moments(img, 0.0, 5.0, 5.9, 47.5, 47.5, o)
    assert st & oracle.CONVERGED
    assert np.hypot(*out[2:4]) < 0.95
    np.testing.assert_allclose(out[2:4], g, atol=2e-3)   # pixelisation of the cusp


def test_status_flags_for_bad_stamps():
    side = 16
    good = np.full((side, side), 10.0)
    good[8, 8] = 100.0
    nan = good.copy()
    nan[3, 4] = np.nan
    flat = np.full((side, side), 10.0)
    a = _pipeline_on([good, nan, flat])
    assert a["status"][1, 0] == oracle.NONFINITE_INPUT
    assert a["status"][2, 0] & oracle.NONPOSITIVE_FLUX
    b = synth.Batch("custom", np.concatenate([good.ravel()] * 2), np.array([0, 0], np.int64),
                    np.array([16, 200], np.int32), np.array([-1.0, 1.0], np.float32),
                    np.zeros(2, np.uint8), np.zeros((2, 8)), None)
    r = oracle.pipeline(b, oracle.opts(), pixels_f64=b.pixels)
    assert (r["status"] == oracle.BAD_INPUT).all()


# --- the fit's starting size (a reading: the paper gives no start for Re) ---

@pytest.mark.parametrize("g,width", [((0.0, 0.0), 2.5), ((0.3, -0.2), 3.0), ((-0.1, 0.45), 4.0)])
def test_size_closed_form_for_gaussian_sources(g, width):
    """For a Gaussian source with isophotes |S(g) u| = const the weighted
    second moment inverts exactly, whatever the weight width: the Gaussian
    integral of exp(-R^2 / 2 s^2) exp(-R^2 / 2 w^2) R^2 gives
    <R^2> = 2 s^2 w^2 / (s^2 + w^2), and the half-light radius of
    exp(-R^2 / 2 s^2) along R / sqrt(1 - |g|^2) is s sqrt(2 ln 2) / sqrt(1 - |g|^2)."""
    side, x0, y0 = 72, 35.3, 36.6
    img = elliptical_src(side, g, width, x0, y0)
    want = width * math.sqrt(2 * math.log(2)) / math.sqrt(1 - g[0] ** 2 - g[1] ** 2)
    for sigw in (2.0, 3.0, 6.0):
        assert oracle.size(img + 10.0, 10.0, sigw, x0, y0, g) == pytest.approx(want, rel=1e-9)


@pytest.mark.parametrize("re,e", [(2.0, (0.0, 0.0)), (3.0, (0.2, -0.1)), (5.5, (-0.35, 0.25))])
def test_size_is_re_for_half_index_sersic(re, e):
    """A Sersic profile of index 1/2 is a Gaussian in the model's elliptical
    radius with half-light radius Re (b(1/2) = ln 2), so the starting size of
    the oracle's own rendering is Re."""
    side = 64
    p = np.array([31.3, 32.6, e[0], e[1], re, 0.5, 50.0, 0.0])
    img = oracle.model(side, p)
    assert oracle.size(img, 0.0, 3.0, p[0], p[1], e) == pytest.approx(re, rel=1e-9)


def test_size_undefined_cases():
    side = 48
    src = elliptical_src(side, (0.1, 0.0), 3.0, 23.5, 24.5)
    # no positive weighted flux
    assert math.isnan(oracle.size(-src, 0.0, 3.0, 23.5, 24.5, (0.1, 0.0)))
    # a flat image: <R^2> under the weight alone is 2 w^2, no finite source size
    assert math.isnan(oracle.size(np.full((side, side), 5.0), 0.0, 3.0, 23.5, 24.5, (0.0, 0.0)))


def test_moments_report_size_at_their_last_step():
    """orc_moments returns the starting size evaluated at the centre and g_w
    of its last step, which for a converged iteration is its output."""
    side = 96
    true, g = (48.31, 46.77), (0.25, -0.15)
    img = elliptical_src(side, g, 3.5, *true) + 10.0
    o = oracle.opts(tol_x=1e-11, tol_g=1e-11, max_iter_moments=60)
    out, it, st = oracle.moments(img, 10.0, 4.0, 4.7, 47.0, 47.0, o)
    assert st & oracle.CONVERGED
    assert out[6] == pytest.approx(oracle.size(img, 10.0, 4.0, out[0], out[1], out[2:4]), rel=1e-9)
    assert out[6] == pytest.approx(3.5 * math.sqrt(2 * math.log(2)) / math.sqrt(1 - 0.25 ** 2 - 0.15 ** 2),
                                   rel=1e-8)
