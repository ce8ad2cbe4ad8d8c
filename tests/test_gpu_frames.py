"""GPU front end on whole frames (shape_frame_detect / _offsets / _cut)
against the FP64 oracle: brightest pixel, growth-curve r50, the 6 r50 box and
the cut-out pixels."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def shape():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1203_0571_amd as shape
    return shape


def _gpu_detect(shape, pix, max_side=128, scale=None):
    import torch
    fr = shape.DeviceFrames(pixels=torch.from_numpy(np.ascontiguousarray(pix)).cuda(),
                            scale=None if scale is None else torch.from_numpy(scale).cuda())
    d = shape.frame_detect(fr, max_side)
    torch.cuda.synchronize()
    return fr, {k: v.cpu().numpy() for k, v in d.items()}


def _compare(pix_f64, g, max_side=128):
    """Every frame: peak, status and box exact (a box may differ only where
    6 r50 sits within 1e-6 of a rounding boundary); sky, r50 and F close."""
    ambiguous = 0
    for i in range(pix_f64.shape[0]):
        r = oracle.frame_detect(pix_f64[i], max_side)
        assert int(g["status"][i]) == r["status"], i
        assert tuple(g["peak"][i]) == r["peak"], i
        if r["status"] & oracle.NONFINITE_INPUT:
            assert tuple(g["box"][i]) == (0, 0, 0)
            assert np.isnan(g["info"][i]).all()
            continue
        sky, r50, F = (float(v) for v in g["info"][i])
        assert sky == pytest.approx(r["sky"], rel=1e-6, abs=1e-6)
        assert r50 == pytest.approx(r["r50"], rel=1e-6)
        assert F == pytest.approx(r["flux"], rel=1e-6, abs=1e-3)
        x = 6.0 * r["r50"]
        if abs(x - np.floor(x) - 0.5) < 1e-6:
            ambiguous += 1
            continue
        assert tuple(g["box"][i]) == r["box"], (i, tuple(g["box"][i]), r["box"], r["r50"])
    return ambiguous


def test_detect_and_cut_vs_oracle(shape):
    import torch
    f = synth.make_frames(48)
    fr, g = _gpu_detect(shape, f.pixels)
    assert _compare(f.pixels.astype(np.float64), g) == 0
    box = torch.from_numpy(g["box"]).cuda()
    db = shape.frame_cut(fr, box, torch.from_numpy(f.sigma).cuda())
    torch.cuda.synchronize()
    off = db.offsets.cpu().numpy()
    sides = db.sides.cpu().numpy()
    stamps = db.pixels.cpu().numpy()
    np.testing.assert_array_equal(sides, g["box"][:, 2])
    assert off[0] == 0
    np.testing.assert_array_equal(off[1:], np.cumsum(sides.astype(np.int64) ** 2)[:-1])
    for i in range(f.n):
        s = int(sides[i])
        ref = oracle.frame_cut(f.pixels[i], tuple(g["box"][i]))
        np.testing.assert_array_equal(stamps[off[i]:off[i] + s * s].reshape(s, s), ref)


def test_detect_is_deterministic(shape):
    f = synth.make_frames(16)
    _, a = _gpu_detect(shape, f.pixels)
    _, b = _gpu_detect(shape, f.pixels)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


def _edge_frames(H, W, rng):
    """Point sources, sources near every edge and corner, flat frames, a
    non-finite frame and a frame with no positive flux."""
    y, x = np.mgrid[0:H, 0:W]
    out = []
    for (cx, cy, s) in [(0, 0, 0.0), (W - 1, H - 1, 0.0), (W // 2, H // 2, 0.0), (3, H - 4, 2.0),
                        (W - 5, 2, 1.5), (W // 3, H // 2, 4.0), (W - 2, H // 2, 3.0)]:
        if s == 0.0:
            img = np.zeros((H, W))
            img[cy, cx] = 7.0
        else:
            img = 100.0 * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * s * s))
        out.append(img + 3.0 + rng.normal(0, 0.01, (H, W)))
    img = np.full((H, W), 2.0)
    out.append(img)                                  # flat: F = 0
    img = rng.normal(0, 1.0, (H, W))
    img[H // 2, W // 3] = np.nan
    out.append(img)                                  # non-finite
    img = -np.ones((H, W))
    img[0, :] = 50.0
    img[H // 2, W // 2] = 1.0
    out.append(img)                                  # F < 0
    img = np.zeros((H, W))
    img[1, 1] = img[H - 2, W - 2] = 5.0
    out.append(img)                                  # tie: first index wins
    return np.stack(out).astype(np.float32)


@pytest.mark.parametrize("H,W,max_side", [(37, 300, 128), (4, 4, 128), (130, 129, 32),
                                          (512, 64, 128)])
def test_edge_frames(shape, H, W, max_side):
    rng = np.random.default_rng(H * 1000 + W)
    pix = _edge_frames(H, W, rng)
    _, g = _gpu_detect(shape, pix, max_side)
    _compare(pix.astype(np.float64), g, max_side)


def test_f16_frames(shape):
    """FP16 frames with a power-of-two scale: the oracle sees the dequantised values."""
    f = synth.make_frames(8)
    peak = np.abs(f.pixels).reshape(f.n, -1).max(1)
    scale = np.exp2(np.ceil(np.log2(peak / 32768.0))).astype(np.float32)
    q = (f.pixels / scale[:, None, None]).astype(np.float16)
    _, g = _gpu_detect(shape, q, scale=scale)
    deq = q.astype(np.float64) * scale[:, None, None].astype(np.float64)
    _compare(deq, g)


def test_frames_to_fitted_objects(shape):
    """Cut-outs feed the per-object pipeline: fit parity on them as on stamps."""
    import torch
    from parity_util import check_fit, fit_parity
    f = synth.make_frames(32)
    fr, g = _gpu_detect(shape, f.pixels)
    db = shape.frame_cut(fr, torch.from_numpy(g["box"]).cuda(), torch.from_numpy(f.sigma).cuda())
    out = shape.pipeline(db, want_perr=True)
    torch.cuda.synchronize()
    pix = db.pixels.cpu().numpy()
    b = synth.Batch("frames", pix, db.offsets.cpu().numpy(), db.sides.cpu().numpy(), f.sigma,
                    np.zeros(f.n, np.uint8), f.truth, None)
    ref = oracle.pipeline(b, oracle.opts())
    gpu = {k: v.cpu().numpy() for k, v in out.items() if hasattr(v, "cpu")}
    st, failures = fit_parity(gpu, ref, b, 0xFF, "frames")
    print(st)
    r = {"fit_" + k: v for k, v in st.items()}
    r.update(n=st["n"], fit_failures=failures)
    check_fit(r, 0.8)
