"""Pins of the whole-frame front end (Sec. 4.1, the paragraph on the starting
point): brightest pixel, growth-curve r50 about it, and the 6 r50 cut-out."""
import math

import numpy as np
import pytest

import oracle


def _brute(img, max_side=128):
    """The same definition written independently with numpy."""
    H, W = img.shape
    border = np.concatenate([img[0], img[-1], img[1:-1, 0], img[1:-1, -1]])
    sky = border.sum() / border.size
    k = int(np.argmax(img))            # first index among equal maxima
    i0, j0 = divmod(k, W)
    y, x = np.mgrid[0:H, 0:W]
    d2 = (y - i0) ** 2 + (x - j0) ** 2
    ring = np.ceil(np.sqrt(d2)).astype(int)
    f = img - sky
    F = f.sum()
    sums = np.bincount(ring.ravel(), weights=f.ravel())
    sums[1] += sums[0]                 # the peak pixel belongs to the first ring
    C = np.cumsum(sums[1:])            # C[r-1] = flux within radius r
    r50 = min(H, W) / 8.0
    if F > 0:
        r = int(np.argmax(C >= F / 2)) + 1
        lo = C[r - 2] if r >= 2 else 0.0
        r50 = (r - 1) + (F / 2 - lo) / (C[r - 1] - lo)
    side = int(math.floor(6 * r50 + 0.5))
    side = max(4, min(side, max_side, H, W))
    ox = max(min(j0 - side // 2, W - side), 0)
    oy = max(min(i0 - side // 2, H - side), 0)
    return dict(sky=sky, r50=r50, flux=F, peak=(j0, i0), box=(ox, oy, side))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("shape", [(9, 13), (17, 17), (40, 23)])
def test_brute_force_tiny_frames(seed, shape):
    rng = np.random.default_rng(seed)
    img = rng.normal(0.0, 1.0, shape)
    i, j = rng.integers(0, shape[0]), rng.integers(0, shape[1])
    img[i, j] += 30.0
    img += rng.uniform(0, 5) * np.exp(-((np.mgrid[0:shape[0], 0:shape[1]][0] - i) ** 2) / 8.0)
    a = oracle.frame_detect(img)
    b = _brute(img)
    assert a["peak"] == b["peak"]
    assert a["sky"] == pytest.approx(b["sky"], rel=1e-12, abs=1e-12)
    assert a["flux"] == pytest.approx(b["flux"], rel=1e-10, abs=1e-9)
    assert a["r50"] == pytest.approx(b["r50"], rel=1e-10)
    assert a["box"] == b["box"]


def test_point_source_half_light_radius():
    """All flux in one pixel: the curve goes from 0 at radius 0 to F at radius 1,
    so the interpolated crossing is 0.5; side clamps to 4 around the peak."""
    img = np.zeros((64, 80))
    img[10, 20] = 5.0
    r = oracle.frame_detect(img)
    assert r["r50"] == 0.5
    assert r["peak"] == (20, 10)
    assert r["box"] == (18, 8, 4)


@pytest.mark.parametrize("pos,origin", [((10, 10), (0, 0)), ((69, 53), (55, 39)),
                                        ((10, 53), (0, 39)), ((69, 10), (55, 0))])
def test_box_shifted_inside_frame(pos, origin):
    """A flat disk of radius 6 with a brighter centre, 10 px from two edges:
    r50 = 4.23, side 25 > 2 * 10, so the square slides inward to the edge."""
    H, W = 64, 80
    y, x = np.mgrid[0:H, 0:W]
    img = (((x - pos[0]) ** 2 + (y - pos[1]) ** 2) <= 36).astype(float)
    img[pos[1], pos[0]] += 0.5
    r = oracle.frame_detect(img)
    assert r["sky"] == 0.0
    assert r["box"] == origin + (25,)
    assert r["box"] == _brute(img)["box"]


def test_ties_take_lowest_index():
    img = np.zeros((16, 16))
    img[7, 3] = img[5, 9] = img[9, 1] = 2.0
    assert oracle.frame_detect(img)["peak"] == (9, 5)


@pytest.mark.parametrize("sigma", [2.0, 4.0, 8.0])
def test_gaussian_r50(sigma):
    """Noiseless circular Gaussian: r50 = sigma sqrt(2 ln 2) up to pixelisation
    (ring binning and linear interpolation), and side = round(6 r50)."""
    H = W = 256
    y, x = np.mgrid[0:H, 0:W]
    img = 100.0 * np.exp(-((x - 100.3) ** 2 + (y - 130.7) ** 2) / (2 * sigma ** 2)) + 7.0
    r = oracle.frame_detect(img)
    assert r["sky"] == pytest.approx(7.0, abs=1e-9)
    assert r["flux"] == pytest.approx(100.0 * 2 * math.pi * sigma ** 2, rel=1e-6)
    assert r["r50"] == pytest.approx(sigma * math.sqrt(2 * math.log(2)), rel=0.02)
    assert r["box"][2] == int(math.floor(6 * r["r50"] + 0.5))
    assert r["peak"] == (100, 131)


def test_rectangular_frame_and_max_side():
    H, W = 48, 300
    y, x = np.mgrid[0:H, 0:W]
    img = np.exp(-((x - 250.0) ** 2 + (y - 20.0) ** 2) / (2 * 10.0 ** 2))
    r = oracle.frame_detect(img, max_side=128)
    assert r["box"][2] == 48          # min(H, W) bounds the side
    assert r["box"][1] == 0
    r = oracle.frame_detect(img, max_side=32)
    assert r["box"] == (250 - 16, 20 - 16, 32)


def test_nonpositive_flux():
    img = -np.ones((32, 40))
    img[5, 5] = 0.5
    img[0, :] = 10.0                  # bright border: sky above everything inside
    r = oracle.frame_detect(img)
    assert r["status"] & oracle.NONPOSITIVE_FLUX
    assert r["r50"] == 32 / 8.0


def test_nonfinite_frame_gives_no_cutout():
    img = np.ones((16, 16))
    img[3, 4] = np.nan
    r = oracle.frame_detect(img)
    assert r["status"] == oracle.NONFINITE_INPUT
    assert r["box"] == (0, 0, 0)
    assert r["peak"] == (-1, -1)
