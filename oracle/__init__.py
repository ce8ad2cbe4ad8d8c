"""ctypes binding of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the library.  Every routine follows the
passage of Li, Xin & Cui (2012) cited in oracle.c.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

CONVERGED = 0x001
MAX_ITER = 0x002
STALLED = 0x004
SINGULAR = 0x008
NONFINITE_INPUT = 0x010
NONPOSITIVE_FLUX = 0x020
AT_BOUND = 0x040
G_CLAMPED = 0x080
BAD_INPUT = 0x100
LOST = 0x200

SERSIC = 0
MOFFAT = 1
MOFFAT_BETA = 2     # star estimator: Moffat with beta fixed


class Opts(C.Structure):
    _fields_ = [
        ("max_iter_centroid", C.c_int),
        ("max_iter_moments", C.c_int),
        ("max_iter_lm", C.c_int),
        ("k_gain", C.c_double),
        ("tol_x", C.c_double),
        ("tol_g", C.c_double),
        ("gmax", C.c_double),
        ("tol_lm", C.c_double),
        ("lambda0", C.c_double),
        ("chi2_rtol", C.c_double),
        ("n0", C.c_double),
        ("moffat_beta", C.c_double),
        ("free_mask", C.c_uint32),
        ("linear_init", C.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        d = C.POINTER(C.c_double)
        L.orc_default_opts.argtypes = [C.POINTER(Opts)]
        L.orc_sersic_b.restype = C.c_double
        L.orc_sersic_b.argtypes = [C.c_double]
        L.orc_sersic_db.restype = C.c_double
        L.orc_sersic_db.argtypes = [C.c_double]
        L.orc_gamma_p.restype = C.c_double
        L.orc_gamma_p.argtypes = [C.c_double, C.c_double]
        L.orc_model.argtypes = [C.c_int, d, C.c_int, d, d]
        L.orc_init.argtypes = [d, C.c_int, d, C.POINTER(C.c_int), d, d, d, C.POINTER(C.c_uint32)]
        L.orc_centroid.argtypes = [d, C.c_int, C.c_double, C.c_double, C.POINTER(Opts), d, d,
                                   C.POINTER(C.c_int), C.POINTER(C.c_uint32)]
        L.orc_ksb_terms.argtypes = [d, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, d, d]
        L.orc_size.argtypes = [d, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, d]
        L.orc_size.restype = C.c_double
        L.orc_moments.argtypes = [d, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.POINTER(Opts), d, C.POINTER(C.c_int),
                                  C.POINTER(C.c_uint32)]
        L.orc_linear.argtypes = [d, C.c_int, d, C.c_int, d, d]
        L.orc_chi2.restype = C.c_double
        L.orc_chi2.argtypes = [d, C.c_int, C.c_double, d, C.c_int, d, d]
        L.orc_fit.argtypes = [d, C.c_int, C.c_double, C.c_int, d, C.POINTER(Opts), d, d,
                              C.POINTER(C.c_int), C.POINTER(C.c_uint32), d]
        L.orc_star_moments.argtypes = [d, C.c_int, C.c_double, C.c_double, C.c_double, d,
                                       C.c_int, C.c_double, C.c_double, C.c_double, C.c_int, d,
                                       C.POINTER(C.c_int), C.POINTER(C.c_uint32)]
        L.orc_pipeline.restype = C.c_int
        L.orc_pipeline.argtypes = [C.c_int64, d, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.POINTER(Opts), d, d, d, d, d, C.c_void_p, C.c_void_p, C.c_int]
        L.orc_frame_detect.argtypes = [d, C.c_int, C.c_int, C.c_int, d, d, d,
                                       C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_void_p,
                                       C.POINTER(C.c_uint32)]
        L.orc_star_pipeline.restype = C.c_int
        L.orc_star_pipeline.argtypes = [C.c_int64, d, C.c_void_p, C.c_void_p, C.POINTER(Opts),
                                        C.c_int, C.c_double, C.c_double, C.c_int, d, C.c_void_p,
                                        C.c_void_p, C.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def opts(**kw):
    o = Opts()
    lib().orc_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def sersic_b(n):
    return lib().orc_sersic_b(float(n))


def sersic_db(n):
    return lib().orc_sersic_db(float(n))


def gamma_p(a, x):
    return lib().orc_gamma_p(float(a), float(x))


def model(side, p, kind=SERSIC, jac=False):
    p = _f64(p)
    m = np.zeros(side * side)
    J = np.zeros((side * side, 8)) if jac else None
    lib().orc_model(side, _dp(p), kind, _dp(m), _dp(J) if jac else None)
    m = m.reshape(side, side)
    return (m, J.reshape(side, side, 8)) if jac else m


def init(img):
    img = _f64(img)
    side = img.shape[0]
    sky0, r50, flux, sigw = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    imax, st = C.c_int(), C.c_uint32(0)
    lib().orc_init(_dp(img), side, C.byref(sky0), C.byref(imax), C.byref(r50), C.byref(flux),
                   C.byref(sigw), C.byref(st))
    return dict(sky0=sky0.value, imax=imax.value, r50=r50.value, flux=flux.value,
                sigw=sigw.value, status=st.value)


def centroid(img, sky0, sigw, x, y, o=None):
    img = _f64(img)
    o = o or opts()
    xx, yy, it, st = C.c_double(x), C.c_double(y), C.c_int(), C.c_uint32(0)
    lib().orc_centroid(_dp(img), img.shape[0], sky0, sigw, C.byref(o), C.byref(xx), C.byref(yy),
                       C.byref(it), C.byref(st))
    return xx.value, yy.value, it.value, st.value


def ksb_terms(img, sky0, sigw, xc, yc, gw):
    img = _f64(img)
    g = _f64(gw)
    out = np.zeros(20)
    lib().orc_ksb_terms(_dp(img), img.shape[0], sky0, sigw, xc, yc, _dp(g), _dp(out))
    return dict(N=out[0], S=out[1:3].copy(), T=out[3], e=out[4:6].copy(),
                X=out[6:10].reshape(2, 2).copy(), eSH=out[10:12].copy(),
                dX=out[12:16].reshape(2, 2).copy(), de=out[16:18].copy())


def moments(img, sky0, sigw, r50, x, y, o=None):
    img = _f64(img)
    o = o or opts()
    out = np.zeros(7)
    it, st = C.c_int(), C.c_uint32(0)
    lib().orc_moments(_dp(img), img.shape[0], sky0, sigw, r50, x, y, C.byref(o), _dp(out),
                      C.byref(it), C.byref(st))
    return out, it.value, st.value


def size(img, sky0, sigw, x, y, g):
    """orc_size: the fit's starting Re from the weighted second moment."""
    img = _f64(img)
    gg = _f64(np.asarray(g, dtype=np.float64))
    return lib().orc_size(_dp(img), img.shape[0], float(sky0), float(sigw), float(x), float(y),
                          _dp(gg))


def linear(img, p, kind=SERSIC):
    img = _f64(img)
    p = _f64(p)
    a, b = C.c_double(), C.c_double()
    lib().orc_linear(_dp(img), img.shape[0], _dp(p), kind, C.byref(a), C.byref(b))
    return a.value, b.value


def chi2(img, sigma, p, kind=SERSIC, want_grad=False):
    img = _f64(img)
    p = _f64(p)
    g = np.zeros(8)
    jtj = np.zeros(36)
    c = lib().orc_chi2(_dp(img), img.shape[0], float(sigma), _dp(p), kind, _dp(g), _dp(jtj))
    return (c, g, jtj) if want_grad else c


def fit(img, sigma, p_init, kind=SERSIC, o=None):
    img = _f64(img)
    p0 = _f64(p_init)
    o = o or opts()
    out = np.zeros(8)
    perr = np.zeros(8)
    c2, it, st = C.c_double(), C.c_int(), C.c_uint32(0)
    lib().orc_fit(_dp(img), img.shape[0], float(sigma), kind, _dp(p0), C.byref(o), _dp(out),
                  C.byref(c2), C.byref(it), C.byref(st), _dp(perr))
    return dict(p=out, chi2=c2.value, iters=it.value, status=st.value, perr=perr)


def star_moments(img, sky, xc, yc, g, kind, w0, tol=1e-4, max_iter=20, beta=3.0):
    """Sec. 4.2 star estimators; kind SERSIC = Gaussian star, MOFFAT = Moffat,
    MOFFAT_BETA = Moffat with beta fixed at `beta`."""
    img = _f64(img)
    gg = _f64(g)
    out = np.zeros(6)
    it, st = C.c_int(), C.c_uint32(0)
    lib().orc_star_moments(_dp(img), img.shape[0], float(sky), float(xc), float(yc), _dp(gg),
                           int(kind), float(beta), float(w0), float(tol), int(max_iter), _dp(out),
                           C.byref(it), C.byref(st))
    return dict(size=out[0], beta=out[1], I0=out[2], r0=out[3], r2=out[4], r4=out[5],
                iters=it.value, status=st.value)


def pipeline(batch, o=None, threads=0, pixels_f64=None):
    """Run the whole procedure on a synth.Batch (FP16 storage is dequantised)."""
    o = o or opts()
    n = batch.n
    pix = pixels_f64 if pixels_f64 is not None else batch.dequantised_f64()
    pix = _f64(pix)
    offs = np.ascontiguousarray(batch.offsets, np.int64)
    sides = np.ascontiguousarray(batch.sides, np.int32)
    sig = np.ascontiguousarray(batch.sigma, np.float32)
    mdl = np.ascontiguousarray(batch.model, np.uint8)
    xy = np.zeros((n, 2))
    mom = np.zeros((n, 7))
    p = np.zeros((n, 8))
    c2 = np.zeros(n)
    perr = np.zeros((n, 8))
    iters = np.zeros((n, 3), np.int32)
    status = np.zeros((n, 3), np.uint32)
    used = lib().orc_pipeline(n, _dp(pix), offs.ctypes.data, sides.ctypes.data, sig.ctypes.data,
                              mdl.ctypes.data, C.byref(o), _dp(xy), _dp(mom), _dp(p), _dp(c2),
                              _dp(perr), iters.ctypes.data, status.ctypes.data, int(threads))
    return dict(xy=xy, mom=mom, p=p, chi2=c2, perr=perr, iters=iters, status=status,
                threads=used)


def star_pipeline(batch, kind, tol=1e-4, max_iter=20, o=None, threads=0, beta=3.0):
    """Star sizes over a synth.Batch (Sec. 4.2) after the centroid and moments
    stages; out[n, 6] = (size, beta, I0, r0, r2, r4).  kind MOFFAT_BETA fixes
    beta at `beta`."""
    o = o or opts()
    n = batch.n
    pix = _f64(batch.dequantised_f64())
    offs = np.ascontiguousarray(batch.offsets, np.int64)
    sides = np.ascontiguousarray(batch.sides, np.int32)
    out = np.zeros((n, 6))
    iters = np.zeros(n, np.int32)
    status = np.zeros(n, np.uint32)
    used = lib().orc_star_pipeline(n, _dp(pix), offs.ctypes.data, sides.ctypes.data, C.byref(o),
                                   int(kind), float(beta), float(tol), int(max_iter), _dp(out),
                                   iters.ctypes.data, status.ctypes.data, int(threads))
    return dict(out=out, iters=iters, status=status, threads=used)


def frame_detect(img, max_side=128):
    """Front end on one frame: sky, r50, flux, peak (x, y), box (x0, y0, side)."""
    img = _f64(img)
    H, W = img.shape
    sky, r50, flux = C.c_double(), C.c_double(), C.c_double()
    px, py, st = C.c_int(), C.c_int(), C.c_uint32(0)
    box = np.zeros(3, np.int32)
    lib().orc_frame_detect(_dp(img), H, W, int(max_side), C.byref(sky), C.byref(r50),
                           C.byref(flux), C.byref(px), C.byref(py), box.ctypes.data, C.byref(st))
    return dict(sky=sky.value, r50=r50.value, flux=flux.value, peak=(px.value, py.value),
                box=tuple(int(v) for v in box), status=st.value)


def frame_cut(img, box):
    """The cut-out square of a frame as a copy."""
    x0, y0, s = box
    return np.array(img[y0:y0 + s, x0:x0 + s], dtype=np.float64, copy=True)
