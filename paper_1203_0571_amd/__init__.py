"""Batched galaxy/star shape measurement on AMD MI355X (gfx950).

A thin ctypes binding of libshape.so, the C ABI declared in include/shape.h.
The three stages of Li, Xin & Cui (2012) -- centroid (Sec. 2), elliptical-
weight KSB ellipticity (Sec. 3, App. A, B) and the Sersic profile fit
(Sec. 4.1) -- run entirely in the library's HIP kernels; this module only
marshals torch tensors (device memory and the current HIP stream) into the
C calls.  There is no CPU fallback: a missing library raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libshape.so")

OK = 0
EINVAL = -1
EDEVICE = -2
ENOMEM = -3
EUNSUPPORTED = -4

F32 = 0
F16_SCALED = 1
SERSIC = 0
MOFFAT = 1

ST_CONVERGED = 0x001
ST_MAX_ITER = 0x002
ST_STALLED = 0x004
ST_SINGULAR = 0x008
ST_NONFINITE_INPUT = 0x010
ST_NONPOSITIVE_FLUX = 0x020
ST_AT_BOUND = 0x040
ST_G_CLAMPED = 0x080
ST_BAD_INPUT = 0x100
ST_LOST = 0x200

REC_LEN = 8
MASK_ALL = 0xFF
MASK_SIZE = 0xF0


class ShapeBatch(C.Structure):
    _fields_ = [
        ("pixels", C.c_void_p),
        ("offset", C.c_void_p),
        ("side", C.c_void_p),
        ("scale", C.c_void_p),
        ("sigma", C.c_void_p),
        ("model", C.c_void_p),
        ("n", C.c_int64),
        ("n_pixels", C.c_int64),
        ("side0", C.c_int32),
        ("dtype", C.c_int32),
    ]


class ShapeOpts(C.Structure):
    _fields_ = [
        ("max_iter_centroid", C.c_int32),
        ("max_iter_moments", C.c_int32),
        ("max_iter_lm", C.c_int32),
        ("free_mask", C.c_uint32),
        ("k_gain", C.c_double),
        ("tol_x", C.c_double),
        ("tol_g", C.c_double),
        ("gmax", C.c_double),
        ("tol_lm", C.c_double),
        ("lambda0", C.c_double),
        ("chi2_rtol", C.c_double),
        ("n0", C.c_double),
        ("moffat_beta", C.c_double),
        ("linear_init", C.c_int32),
        ("reserved", C.c_int32),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libshape.so is not built (run __graft_entry__.build() or "
                          "python -m paper_1203_0571_amd.build); there is no fallback")
    lib = C.CDLL(LIB_PATH)
    vp, bp, op = C.c_void_p, C.POINTER(ShapeBatch), C.POINTER(ShapeOpts)
    lib.shape_abi_version.restype = C.c_int
    lib.shape_default_opts.argtypes = [op]
    lib.shape_default_opts.restype = C.c_int
    lib.shape_status_string.argtypes = [C.c_int]
    lib.shape_status_string.restype = C.c_char_p
    lib.shape_centroid.argtypes = [bp, op, vp, vp, vp, vp]
    lib.shape_centroid.restype = C.c_int
    lib.shape_moments.argtypes = [bp, op, vp, vp, vp, vp, vp]
    lib.shape_moments.restype = C.c_int
    lib.shape_fit_sersic.argtypes = [bp, op, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.shape_fit_sersic.restype = C.c_int
    return lib


lib = _load()


class ShapeError(RuntimeError):
    pass


def _check(rc, what):
    if rc != OK:
        raise ShapeError("%s failed: %s (%d)" % (what, lib.shape_status_string(rc).decode(), rc))


def default_opts(**overrides) -> ShapeOpts:
    o = ShapeOpts()
    _check(lib.shape_default_opts(C.byref(o)), "shape_default_opts")
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


@dataclass
class DeviceBatch:
    """Stamps resident on one GPU, in the layout the library expects."""
    pixels: torch.Tensor                 # float32, or float16 with `scale`
    sigma: torch.Tensor                  # float32 [n]
    side0: int = 0
    offsets: torch.Tensor | None = None  # int64 [n]
    sides: torch.Tensor | None = None    # int32 [n]
    scale: torch.Tensor | None = None    # float32 [n]
    model: torch.Tensor | None = None    # uint8 [n]

    @property
    def n(self):
        return int(self.sigma.shape[0])

    @property
    def device(self):
        return self.pixels.device

    def c_struct(self) -> ShapeBatch:
        b = ShapeBatch()
        b.pixels = _ptr(self.pixels)
        b.offset = _ptr(self.offsets)
        b.side = _ptr(self.sides)
        b.scale = _ptr(self.scale)
        b.sigma = _ptr(self.sigma)
        b.model = _ptr(self.model)
        b.n = self.n
        b.n_pixels = int(self.pixels.numel())
        b.side0 = int(self.side0)
        b.dtype = F16_SCALED if self.pixels.dtype == torch.float16 else F32
        return b

    @staticmethod
    def from_host(batch, device="cuda", uniform=None):
        """Upload a synth.Batch (numpy) to the GPU."""
        dev = torch.device(device)
        sides = batch.sides
        if uniform is None:
            uniform = batch.n > 0 and bool((sides == sides[0]).all()) and not batch.model.any()
        pix = torch.from_numpy(batch.pixels).to(dev)
        kw = dict(pixels=pix, sigma=torch.from_numpy(batch.sigma).to(dev))
        if batch.scale is not None:
            kw["scale"] = torch.from_numpy(batch.scale).to(dev)
        if uniform:
            kw["side0"] = int(sides[0]) if batch.n else 4
        else:
            kw["offsets"] = torch.from_numpy(batch.offsets).to(dev)
            kw["sides"] = torch.from_numpy(sides).to(dev)
            kw["model"] = torch.from_numpy(batch.model).to(dev)
        return DeviceBatch(**kw)


def _outs(n, device, *shapes_dtypes):
    return [torch.empty(sh, dtype=dt, device=device) for sh, dt in shapes_dtypes]


def centroid(batch: DeviceBatch, opts: ShapeOpts | None = None):
    """shape_centroid: returns (rec [n,8], iters [n], status [n])."""
    opts = opts or default_opts()
    n, dev = batch.n, batch.device
    rec, it, st = _outs(n, dev, ((n, REC_LEN), torch.float32), ((n,), torch.int32),
                        ((n,), torch.int32))
    b = batch.c_struct()
    _check(lib.shape_centroid(C.byref(b), C.byref(opts), _ptr(rec), _ptr(it), _ptr(st),
                              _stream(dev)), "shape_centroid")
    return rec, it, st


def moments(batch: DeviceBatch, rec_in: torch.Tensor, opts: ShapeOpts | None = None):
    """shape_moments: returns (rec [n,8], iters, status)."""
    opts = opts or default_opts()
    n, dev = batch.n, batch.device
    rec, it, st = _outs(n, dev, ((n, REC_LEN), torch.float32), ((n,), torch.int32),
                        ((n,), torch.int32))
    b = batch.c_struct()
    _check(lib.shape_moments(C.byref(b), C.byref(opts), _ptr(rec_in), _ptr(rec), _ptr(it),
                             _ptr(st), _stream(dev)), "shape_moments")
    return rec, it, st


def fit_sersic(batch: DeviceBatch, rec: torch.Tensor | None = None,
               p_init: torch.Tensor | None = None, opts: ShapeOpts | None = None,
               want_perr: bool = False):
    """shape_fit_sersic: returns dict(p, chi2, perr, iters, status, sweeps)."""
    opts = opts or default_opts()
    n, dev = batch.n, batch.device
    p, chi2, it, st, sw = _outs(n, dev, ((n, 8), torch.float32), ((n,), torch.float32),
                                ((n,), torch.int32), ((n,), torch.int32), ((n,), torch.int32))
    perr = torch.empty((n, 8), dtype=torch.float32, device=dev) if want_perr else None
    b = batch.c_struct()
    _check(lib.shape_fit_sersic(C.byref(b), C.byref(opts), _ptr(p_init), _ptr(rec), _ptr(p),
                                _ptr(chi2), _ptr(perr), _ptr(it), _ptr(st), _ptr(sw),
                                _stream(dev)), "shape_fit_sersic")
    return dict(p=p, chi2=chi2, perr=perr, iters=it, status=st, sweeps=sw)


def pipeline(batch: DeviceBatch, opts: ShapeOpts | None = None, want_perr: bool = False):
    """The three stages back to back on the current stream (the plain form)."""
    opts = opts or default_opts()
    rec0, it0, st0 = centroid(batch, opts)
    rec1, it1, st1 = moments(batch, rec0, opts)
    fit = fit_sersic(batch, rec=rec1, opts=opts, want_perr=want_perr)
    return dict(centroid=rec0, moments=rec1, iters=torch.stack([it0, it1, fit["iters"]], 1),
                status=torch.stack([st0, st1, fit["status"]], 1), p=fit["p"], chi2=fit["chi2"],
                perr=fit["perr"], sweeps=fit["sweeps"])
