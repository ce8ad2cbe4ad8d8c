"""Pins of the oracle's Sersic b(n), incomplete gamma, model and Jacobian.

The half-light definition of b (Sec. 4.1, eq. ser) is checked three
independent ways: scipy's inverse incomplete gamma, closed forms at n = 0.5
and n = 1, and direct radial integration of the profile.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, optimize, special

import oracle
import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


@pytest.mark.parametrize("n", [0.2, 0.35, 0.5, 0.8, 1.0, 1.7, 2.5, 4.0, 6.3, 10.0])
def test_b_matches_scipy(n):
    ref = special.gammaincinv(2 * n, 0.5)
    assert oracle.sersic_b(n) == pytest.approx(ref, rel=1e-12)


def test_b_closed_forms():
    # n = 0.5: P(1, b) = 1 - exp(-b) = 1/2  =>  b = ln 2
    assert oracle.sersic_b(0.5) == pytest.approx(math.log(2.0), rel=1e-14)
    # n = 1: P(2, b) = 1 - exp(-b)(1 + b) = 1/2
    b1 = optimize.brentq(lambda b: 1 - math.exp(-b) * (1 + b) - 0.5, 0.1, 5, xtol=1e-15)
    assert oracle.sersic_b(1.0) == pytest.approx(b1, rel=1e-13)


@pytest.mark.parametrize("n", [0.5, 1.0, 2.5, 4.0, 8.0])
def test_b_half_light_by_integration(n):
    """Flux inside r = Re is half the total (the definition of b)."""
    b = oracle.sersic_b(n)
    f = lambda r: 2 * math.pi * r * math.exp(-b * r ** (1.0 / n))
    inner = integrate.quad(f, 0, 1, epsabs=0, epsrel=1e-13, limit=400)[0]
    outer = integrate.quad(f, 1, np.inf, epsabs=0, epsrel=1e-13, limit=400)[0]
    assert inner / (inner + outer) == pytest.approx(0.5, abs=1e-10)


@pytest.mark.parametrize("a,x", [(0.4, 0.1), (1.0, 0.7), (2.5, 1.0), (2.5, 6.0), (8.0, 7.7),
                                 (20.0, 19.6), (0.7, 3.0), (15.0, 30.0)])
def test_gamma_p_matches_scipy(a, x):
    assert oracle.gamma_p(a, x) == pytest.approx(special.gammainc(a, x), rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("n", [0.3, 0.5, 1.0, 2.0, 4.0, 9.0])
def test_db_dn(n):
    h = 1e-4 * n
    ref = (special.gammaincinv(2 * (n + h), 0.5) - special.gammaincinv(2 * (n - h), 0.5)) / (2 * h)
    assert oracle.sersic_db(n) == pytest.approx(ref, rel=1e-7)


def test_db_dn_asymptotic():
    # Ciotti & Bertin (1999): b = 2n - 1/3 + 4/(405 n) + 46/(25515 n^2) + ...
    for n in [6.0, 8.0, 10.0]:
        deriv = 2 - 4 / (405 * n * n) - 92 / (25515 * n ** 3)
        assert oracle.sersic_db(n) == pytest.approx(deriv, abs=2e-6)


GEOMS = [
    (0.5, (30.3, 29.1, 0.0, 0.0)),
    (0.5, (31.0, 30.6, 0.3, -0.2)),
    (1.0, (30.7, 31.2, -0.25, 0.4)),
    (3.2, (31.4, 30.2, 0.1, 0.15)),
]


@pytest.mark.parametrize("n,geom", GEOMS)
def test_model_matches_generator(n, geom):
    """The oracle's renderer agrees with the stamp generator's (scipy b)."""
    p = np.array([*geom, 4.3, n, 812.0, 10.0])
    ours = oracle.model(64, p)
    ref = synth.render_sersic(64, p)[0] + 10.0
    np.testing.assert_allclose(ours, ref, rtol=1e-12, atol=1e-12)
    pm = np.array([*geom, 2.7, 3.0, 500.0, 10.0])
    ours = oracle.model(64, pm, kind=oracle.MOFFAT)
    ref = synth.render_moffat(64, pm)[0] + 10.0
    np.testing.assert_allclose(ours, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kind", [oracle.SERSIC, oracle.MOFFAT])
@pytest.mark.parametrize("n,geom", GEOMS)
def test_jacobian_matches_finite_differences(kind, n, geom):
    p = np.array([*geom, 4.3, n if kind == oracle.SERSIC else 2.5 + n, 812.0, 10.0])
    side = 64
    _, J = oracle.model(side, p, kind=kind, jac=True)
    for k in range(8):
        h = 1e-6 * max(abs(p[k]), 1.0)
        dp = np.zeros(8)
        dp[k] = h
        fd = (oracle.model(side, p + dp, kind=kind) - oracle.model(side, p - dp, kind=kind)) / (2 * h)
        scale = np.abs(fd).max()
        # the floored cusp pixel (R^2 < 1e-8) never occurs at these centres
        np.testing.assert_allclose(J[..., k], fd, rtol=0, atol=2e-6 * scale + 1e-12,
                                   err_msg="column %d" % k)


@pytest.mark.parametrize("n,re,side,tol", [(0.5, 4.0, 96, 1e-10), (0.5, 2.3, 64, 1e-10),
                                           (1.0, 6.0, 128, 2e-3), (2.0, 4.0, 128, 2e-2)])
@pytest.mark.parametrize("e", [(0.0, 0.0), (0.3, -0.4)])
def test_flux_closed_form(n, re, side, tol, e):
    """Sum over pixels of the point-sampled model = 2 pi n Gamma(2n) b^-2n Re^2 I0,
    independent of the ellipticity (area-preserving R)."""
    c = (side - 1) / 2
    p = np.array([c + 0.21, c - 0.37, e[0], e[1], re, n, 1.0, 0.0])
    m = oracle.model(side, p)
    b = special.gammaincinv(2 * n, 0.5)
    flux = 2 * math.pi * n * special.gamma(2 * n) * b ** (-2 * n) * re ** 2
    assert m.sum() == pytest.approx(flux, rel=tol)


@pytest.mark.parametrize("e", [(0.3, 0.0), (0.0, 0.3), (-0.2, 0.45), (0.6, -0.1)])
def test_ellipse_orientation_and_distortion(e):
    """Unweighted second moments of the n = 0.5 model: (Q11-Q22, 2Q12)/(Q11+Q22)
    is the distortion 2e/(1+|e|^2); e1 > 0 is elongated along x, e2 > 0 along y = x."""
    side = 96
    c = (side - 1) / 2
    p = np.array([c, c, e[0], e[1], 5.0, 0.5, 1.0, 0.0])
    m = oracle.model(side, p)
    j, i = np.meshgrid(np.arange(side) - c, np.arange(side) - c)
    q11, q22, q12 = (m * j * j).sum(), (m * i * i).sum(), (m * i * j).sum()
    chi = np.array([q11 - q22, 2 * q12]) / (q11 + q22)
    ee = np.array(e)
    np.testing.assert_allclose(chi, 2 * ee / (1 + ee @ ee), atol=1e-10)
    if e[1] == 0.0 and e[0] > 0:
        assert q11 > q22


def test_paper_constants_fixture():
    assert GOLD["centroid_fixed_gain"]["value"] == 0.75
    assert GOLD["max_iterations"]["value"] == 20
