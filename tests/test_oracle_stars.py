"""Pins of the star-size estimators of Sec. 4.2 (weighted moments r0, r2, r4
with the weight iterated onto the star)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _gauss(side, sigma, c, g=(0.0, 0.0), amp=1.0):
    p = np.array([c[0], c[1], g[0], g[1], sigma * math.sqrt(2 * math.log(2)), 0.5, amp, 0.0])
    return synth.render_sersic(side, p)[0]


@pytest.mark.parametrize("sigma", [2.0, 3.5, 6.0])
def test_gaussian_closed_forms(sigma):
    """With sigma_w = sigma: r0 = pi sigma^2 I0 and r2 = pi sigma^4 I0 (Sec. 4.2.1)."""
    side = 128
    c = (63.3, 64.1)
    img = _gauss(side, sigma, c, amp=700.0)
    r = oracle.star_moments(img, 0.0, c[0], c[1], (0.0, 0.0), oracle.SERSIC, sigma, max_iter=1)
    pi = GOLD["gaussian_star_r0_over_I0_sigma2"]["value"]
    assert r["r0"] == pytest.approx(pi * sigma ** 2 * 700.0, rel=1e-10)
    assert r["r2"] == pytest.approx(GOLD["gaussian_star_r2_over_I0_sigma4"]["value"] * sigma ** 4 * 700.0,
                                    rel=1e-10)
    assert r["size"] == pytest.approx(sigma, rel=1e-10)
    assert r["I0"] == pytest.approx(700.0, rel=1e-10)


@pytest.mark.parametrize("g", [(0.0, 0.0), (0.15, -0.1)])
def test_gaussian_iteration_recovers_sigma(g):
    side = 96
    c = (47.2, 48.6)
    img = _gauss(side, 2.7, c, g=g, amp=300.0) + 10.0
    r = oracle.star_moments(img, 10.0, c[0], c[1], g, oracle.SERSIC, 1.5, tol=1e-12, max_iter=200)
    assert r["status"] & oracle.CONVERGED
    assert r["size"] == pytest.approx(2.7, rel=1e-9)
    assert r["I0"] == pytest.approx(300.0, rel=1e-9)


def _moffat_radial_integrals(I0, rd, beta, rdw):
    """r0, r2, r4 by quadrature of the radial integrals (any rdw)."""
    from scipy import integrate
    f = lambda r, k: I0 * (1 + r * r / rd ** 2) ** -beta * (1 + r * r / rdw ** 2) ** -3 * 2 * math.pi * r ** (2 * k + 1)
    return [integrate.quad(f, 0, np.inf, args=(k,), epsabs=0, epsrel=1e-12, limit=400)[0]
            for k in (0, 1, 2)]


@pytest.mark.parametrize("beta", [3.0, 4.2])
def test_moffat_closed_forms(beta):
    """With rdw = rd: r0 = I0 pi rd^2/(b+2), r2 = I0 pi rd^4/((b+1)(b+2)),
    r4 = 2 I0 pi rd^6/(b(b+1)(b+2)) (Sec. 4.2.2); checked by quadrature, and
    the inversion of these three for (beta, rd, I0)."""
    I0, rd = 50.0, 3.0
    r0, r2, r4 = _moffat_radial_integrals(I0, rd, beta, rd)
    assert r0 == pytest.approx(I0 * math.pi * rd ** 2 / (beta + 2), rel=1e-10)
    assert r2 == pytest.approx(I0 * math.pi * rd ** 4 / ((beta + 1) * (beta + 2)), rel=1e-10)
    assert r4 == pytest.approx(2 * I0 * math.pi * rd ** 6 / (beta * (beta + 1) * (beta + 2)), rel=1e-10)


def test_moffat_iteration_recovers_beta_rd():
    """A well-sampled noiseless Moffat star: the iteration onto rdw = rd recovers
    (beta, rd, I0) up to the pixel-sum error."""
    side = 128
    c = (64.4, 63.7)
    p = np.array([c[0], c[1], 0.0, 0.0, 7.0, 3.5, 400.0, 0.0])
    img = synth.render_moffat(side, p)[0]
    r = oracle.star_moments(img, 0.0, c[0], c[1], (0.0, 0.0), oracle.MOFFAT, 5.0, tol=1e-12, max_iter=200)
    assert r["status"] & oracle.CONVERGED
    assert r["size"] == pytest.approx(7.0, rel=2e-3)     # truncation of the r^4 wing at the edge
    assert r["beta"] == pytest.approx(3.5, rel=5e-3)
    assert r["I0"] == pytest.approx(400.0, rel=5e-3)


def test_moffat_inversion_exact_at_matched_weight():
    """Pixel sums of a wide, well-sampled star at rdw = rd invert exactly."""
    side = 128
    c = (63.5, 63.5)
    beta, rd = 4.0, 4.0
    img = synth.render_moffat(side, np.array([c[0], c[1], 0, 0, rd, beta, 1000.0, 0]))[0]
    r = oracle.star_moments(img, 0.0, c[0], c[1], (0.0, 0.0), oracle.MOFFAT, rd, max_iter=1)
    # the pixel sums approximate the integrals to the midpoint-rule error (~1e-6 here)
    assert r["r0"] == pytest.approx(1000.0 * math.pi * rd ** 2 / (beta + 2), rel=1e-5)
    assert r["beta"] == pytest.approx(beta, rel=1e-4)
    assert r["size"] == pytest.approx(rd, rel=1e-4)


def test_moffat_fixed_beta_inversion_exact_at_matched_weight():
    """Beta fixed at the star's own: the pixel sums at rdw = rd give rd and I0
    through r0 and r2 alone (eqs. mofrditer, mofI0iter with beta known)."""
    side = 128
    c = (63.5, 63.5)
    beta, rd = 4.0, 4.0
    img = synth.render_moffat(side, np.array([c[0], c[1], 0, 0, rd, beta, 1000.0, 0]))[0]
    r = oracle.star_moments(img, 0.0, c[0], c[1], (0.0, 0.0), oracle.MOFFAT_BETA, rd, max_iter=1,
                            beta=beta)
    assert r["beta"] == beta
    assert r["size"] == pytest.approx(rd, rel=1e-5)
    assert r["I0"] == pytest.approx(1000.0, rel=1e-5)


def test_moffat_fixed_beta_iteration_recovers_rd():
    """From a weight twice too wide, the fixed-beta iteration converges to the
    star's rd; with a wrong beta it converges to a different width."""
    side = 128
    c = (64.4, 63.7)
    p = np.array([c[0], c[1], 0.0, 0.0, 5.0, 3.5, 400.0, 0.0])
    img = synth.render_moffat(side, p)[0]
    r = oracle.star_moments(img, 0.0, c[0], c[1], (0.0, 0.0), oracle.MOFFAT_BETA, 10.0, tol=1e-12,
                            max_iter=200, beta=3.5)
    assert r["status"] & oracle.CONVERGED
    assert r["size"] == pytest.approx(5.0, rel=1e-4)
    assert r["I0"] == pytest.approx(400.0, rel=1e-4)
    w = oracle.star_moments(img, 0.0, c[0], c[1], (0.0, 0.0), oracle.MOFFAT_BETA, 10.0, tol=1e-12,
                            max_iter=200, beta=5.0)
    assert w["status"] & oracle.CONVERGED and abs(w["size"] / 5.0 - 1) > 0.05


def test_moffat_fixed_beta_converges_where_free_beta_does_not():
    """On the 32^2 star workload (beta U(2.5, 5)) a noisy fourth moment often
    makes the free-beta estimate undefined (r4 r0 / (2 r2^2) <= 1); with beta
    fixed (the paper's remedy, Sec. 4.2.2) r4 is not needed."""
    b = synth.make("stars32", 512)
    free = oracle.star_pipeline(b, oracle.MOFFAT, 1e-4, 20)
    fixed = oracle.star_pipeline(b, oracle.MOFFAT_BETA, 1e-4, 20, beta=3.75)
    conv = lambda r: ((r["status"] & oracle.CONVERGED) != 0).mean()
    assert conv(free) < 0.8
    assert conv(fixed) > 0.97


@pytest.mark.parametrize("kind", [oracle.SERSIC, oracle.MOFFAT, oracle.MOFFAT_BETA])
def test_batched_chain_matches_per_stamp_calls(kind):
    """orc_star_pipeline is the per-stamp chain init -> centroid -> moments ->
    star estimator, run over a batch."""
    b = synth.make("stars32", 24)
    o = oracle.opts()
    r = oracle.star_pipeline(b, kind, 1e-4, 20, o, threads=2)
    for i in range(b.n):
        img = b.stamp(i)
        ini = oracle.init(img)
        x, y, _, _ = oracle.centroid(img, ini["sky0"], ini["sigw"], ini["imax"] % 32,
                                     ini["imax"] // 32, o)
        mo, _, _ = oracle.moments(img, ini["sky0"], ini["sigw"], ini["r50"], x, y, o)
        # the Moffat of half-light radius r50 with beta = 3 (also the fixed beta here)
        w0 = ini["sigw"] if kind == oracle.SERSIC else ini["r50"] / math.sqrt(math.sqrt(2) - 1)
        s = oracle.star_moments(img, ini["sky0"], mo[0], mo[1], mo[2:4], kind, w0)
        assert s["status"] == r["status"][i]
        assert s["iters"] == r["iters"][i]
        np.testing.assert_array_equal(
            np.array([s["size"], s["beta"], s["I0"], s["r0"], s["r2"], s["r4"]]), r["out"][i])
