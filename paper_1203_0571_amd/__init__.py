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
LIB_PATH = os.environ.get("SHAPE_LIB") or os.path.join(_PKG, "libshape.so")

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

REC_LEN = 9
MASK_ALL = 0xFF
MASK_SIZE = 0xF0
STATIC_MAX_STAMPS = 65536   # SHAPE_STATIC_MAX_STAMPS: shape_fit_queue_static's limit


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
        ("tol_sigma", C.c_double),
    ]


class QueueCfg(C.Structure):
    _fields_ = [
        ("team", C.c_int32),
        ("team_min_side", C.c_int32),
        ("grid", C.c_int32),
        ("chunk", C.c_int32),
    ]


class ShapeFrames(C.Structure):
    _fields_ = [
        ("pixels", C.c_void_p),
        ("scale", C.c_void_p),
        ("n", C.c_int64),
        ("height", C.c_int32),
        ("width", C.c_int32),
        ("dtype", C.c_int32),
        ("reserved", C.c_int32),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libshape.so is not built (run __graft_entry__.build() or "
                          "python __graft_entry__.py); there is no fallback")
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
    lib.shape_chi2_fwd.argtypes = [bp, vp, vp, vp]
    lib.shape_chi2_fwd.restype = C.c_int
    lib.shape_chi2_bwd.argtypes = [bp, vp, vp, vp, vp, vp, vp, vp]
    lib.shape_chi2_bwd.restype = C.c_int
    lib.shape_chi2_grad_scale.argtypes = [vp, vp, C.c_int64, vp, vp]
    lib.shape_chi2_grad_scale.restype = C.c_int
    lib.shape_star_moments.argtypes = [bp, C.c_int32, vp, C.c_double, C.c_int32, vp, vp, vp, vp]
    lib.shape_star_moments.restype = C.c_int
    lib.shape_star_moments_beta.argtypes = [bp, C.c_double, vp, C.c_double, C.c_int32, vp, vp, vp,
                                            vp]
    lib.shape_star_moments_beta.restype = C.c_int
    fp = C.POINTER(ShapeFrames)
    lib.shape_frame_detect.argtypes = [fp, C.c_int32, vp, vp, vp, vp, vp]
    lib.shape_frame_offsets.argtypes = [vp, C.c_int64, vp, vp, vp]
    lib.shape_frame_cut.argtypes = [fp, vp, vp, vp, C.c_int64, vp, vp]
    for f in ("shape_frame_detect", "shape_frame_offsets", "shape_frame_cut"):
        getattr(lib, f).restype = C.c_int
    qp = C.POINTER(QueueCfg)
    lib.shape_queue_default_cfg.argtypes = [qp]
    lib.shape_queue_workspace_bytes.argtypes = [C.c_int64, C.POINTER(C.c_size_t)]
    lib.shape_queue_start.argtypes = [bp, op, qp, vp, vp, vp, C.c_size_t, vp]
    lib.shape_queue_step.argtypes = [bp, op, qp, vp, C.c_size_t, vp]
    lib.shape_queue_finish.argtypes = [bp, op, vp, C.c_size_t, vp, vp, vp, vp, vp, vp, vp]
    lib.shape_queue_drain.argtypes = [bp, op, qp, vp, C.c_size_t, vp]
    lib.shape_queue_graph_create.argtypes = [bp, op, qp, vp, C.c_size_t, C.POINTER(C.c_void_p)]
    lib.shape_queue_graph_launch.argtypes = [vp, vp]
    lib.shape_queue_graph_destroy.argtypes = [vp]
    lib.shape_fit_queue_static.argtypes = [bp, op, qp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    for f in ("shape_queue_default_cfg", "shape_queue_workspace_bytes", "shape_queue_start",
              "shape_queue_step", "shape_queue_finish", "shape_queue_graph_create",
              "shape_queue_graph_launch", "shape_queue_graph_destroy", "shape_fit_queue_static",
              "shape_queue_drain"):
        getattr(lib, f).restype = C.c_int
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

    def validate(self):
        """Raise ValueError unless every tensor is contiguous, on the pixels'
        device, and of the dtype and length the library reads (a strided or
        mistyped tensor would make the kernels read past its end)."""
        n, dev = self.n, self.pixels.device
        if self.pixels.dtype not in (torch.float32, torch.float16):
            raise ValueError("pixels must be float32, or float16 with a scale")
        if (self.pixels.dtype == torch.float16) != (self.scale is not None):
            raise ValueError("float16 pixels need a per-stamp scale (and only they)")
        want = [("pixels", self.pixels, self.pixels.dtype, None),
                ("sigma", self.sigma, torch.float32, (n,)),
                ("offsets", self.offsets, torch.int64, (n,)),
                ("sides", self.sides, torch.int32, (n,)),
                ("scale", self.scale, torch.float32, (n,)),
                ("model", self.model, torch.uint8, (n,))]
        for name, t, dt, shp in want:
            if t is None:
                continue
            if t.dtype != dt or t.device != dev or not t.is_contiguous():
                raise ValueError("%s must be a contiguous %s tensor on %s" % (name, dt, dev))
            if shp is not None and tuple(t.shape) != shp:
                raise ValueError("%s must have shape %s" % (name, shp))
        if (self.offsets is None) != (self.sides is None) and self.offsets is not None:
            raise ValueError("offsets need sides")
        if self.sides is None and n and not 4 <= int(self.side0) <= 128:
            raise ValueError("a uniform batch needs side0 in [4, 128]")

    def c_struct(self) -> ShapeBatch:
        self.validate()
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
        """Upload a synth.Batch (numpy) to the GPU.  A batch of one side is
        passed as side0 (no side or offset arrays: the kernels then take
        their uniform-side paths), with the model array only if it has a
        model other than Sersic."""
        dev = torch.device(device)
        sides = batch.sides
        if uniform is None:
            uniform = batch.n > 0 and bool((sides == sides[0]).all())
        pix = torch.from_numpy(batch.pixels).to(dev)
        kw = dict(pixels=pix, sigma=torch.from_numpy(batch.sigma).to(dev))
        if batch.scale is not None:
            kw["scale"] = torch.from_numpy(batch.scale).to(dev)
        if uniform:
            kw["side0"] = int(sides[0]) if batch.n else 4
            if batch.model.any():
                kw["model"] = torch.from_numpy(batch.model).to(dev)
        else:
            kw["offsets"] = torch.from_numpy(batch.offsets).to(dev)
            kw["sides"] = torch.from_numpy(sides).to(dev)
            kw["model"] = torch.from_numpy(batch.model).to(dev)
        return DeviceBatch(**kw)


@dataclass
class DeviceFrames:
    """Equal frames resident on one GPU: pixels [n, H, W] float32, or float16
    with a per-frame scale."""
    pixels: torch.Tensor
    scale: torch.Tensor | None = None

    @property
    def n(self):
        return int(self.pixels.shape[0])

    @property
    def device(self):
        return self.pixels.device

    def c_struct(self) -> ShapeFrames:
        if self.pixels.dim() != 3 or not self.pixels.is_contiguous():
            raise ValueError("frames must be a contiguous [n, H, W] tensor")
        f = ShapeFrames()
        f.pixels = _ptr(self.pixels)
        f.scale = _ptr(self.scale)
        f.n = self.n
        f.height = int(self.pixels.shape[1])
        f.width = int(self.pixels.shape[2])
        f.dtype = F16_SCALED if self.pixels.dtype == torch.float16 else F32
        return f

    @staticmethod
    def from_host(frames, device="cuda"):
        """Upload a synth.Frames (numpy) to the GPU."""
        return DeviceFrames(pixels=torch.from_numpy(frames.pixels).to(torch.device(device)))


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
    rec_in = _rows(rec_in, n, REC_LEN, "rec_in", dev)
    rec, it, st = _outs(n, dev, ((n, REC_LEN), torch.float32), ((n,), torch.int32),
                        ((n,), torch.int32))
    b = batch.c_struct()
    _check(lib.shape_moments(C.byref(b), C.byref(opts), _ptr(rec_in), _ptr(rec), _ptr(it),
                             _ptr(st), _stream(dev)), "shape_moments")
    return rec, it, st


def _rows(t, n, width, name, device):
    """A float32 [n, width] input on the batch's device, contiguous (or None)."""
    if t is None:
        return None
    if t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != (n, width) \
            or t.device != device:
        raise ValueError("%s must be a contiguous float32 [%d, %d] tensor on %s"
                         % (name, n, width, device))
    return t


def fit_sersic(batch: DeviceBatch, rec: torch.Tensor | None = None,
               p_init: torch.Tensor | None = None, opts: ShapeOpts | None = None,
               want_perr: bool = False):
    """shape_fit_sersic: returns dict(p, chi2, perr, iters, status, sweeps)."""
    opts = opts or default_opts()
    n, dev = batch.n, batch.device
    rec = _rows(rec, n, REC_LEN, "rec", dev)
    p_init = _rows(p_init, n, 8, "p_init", dev)
    p, chi2, it, st, sw = _outs(n, dev, ((n, 8), torch.float32), ((n,), torch.float32),
                                ((n,), torch.int32), ((n,), torch.int32), ((n,), torch.int32))
    perr = torch.empty((n, 8), dtype=torch.float32, device=dev) if want_perr else None
    b = batch.c_struct()
    _check(lib.shape_fit_sersic(C.byref(b), C.byref(opts), _ptr(p_init), _ptr(rec), _ptr(p),
                                _ptr(chi2), _ptr(perr), _ptr(it), _ptr(st), _ptr(sw),
                                _stream(dev)), "shape_fit_sersic")
    return dict(p=p, chi2=chi2, perr=perr, iters=it, status=st, sweeps=sw)


def _params(params):
    if params.dtype != torch.float32 or not params.is_contiguous() or params.dim() != 2 \
            or params.shape[1] != 8:
        raise ValueError("params must be a contiguous float32 [n, 8] tensor")
    return params


def chi2_fwd(batch: DeviceBatch, params: torch.Tensor) -> torch.Tensor:
    """shape_chi2_fwd: chi^2 [n] of params [n, 8]."""
    params = _params(params)
    n, dev = batch.n, batch.device
    chi2 = torch.empty(n, dtype=torch.float32, device=dev)
    b = batch.c_struct()
    _check(lib.shape_chi2_fwd(C.byref(b), _ptr(params), _ptr(chi2), _stream(dev)),
           "shape_chi2_fwd")
    return chi2


def chi2_bwd(batch: DeviceBatch, params: torch.Tensor, grad_chi2: torch.Tensor | None = None,
             want_normal: bool = False):
    """shape_chi2_bwd: dict(grad [n,8], chi2 [n], jtj [n,36] and jtr [n,8] if asked)."""
    params = _params(params)
    n, dev = batch.n, batch.device
    if grad_chi2 is not None:
        grad_chi2 = grad_chi2.to(torch.float32).contiguous()
    grad = torch.empty((n, 8), dtype=torch.float32, device=dev)
    chi2 = torch.empty(n, dtype=torch.float32, device=dev)
    jtj = torch.empty((n, 36), dtype=torch.float32, device=dev) if want_normal else None
    jtr = torch.empty((n, 8), dtype=torch.float32, device=dev) if want_normal else None
    b = batch.c_struct()
    _check(lib.shape_chi2_bwd(C.byref(b), _ptr(params), _ptr(grad_chi2), _ptr(chi2), _ptr(grad),
                              _ptr(jtj), _ptr(jtr), _stream(dev)), "shape_chi2_bwd")
    return dict(grad=grad, chi2=chi2, jtj=jtj, jtr=jtr)


def chi2_grad_scale(grad_unit: torch.Tensor, grad_chi2: torch.Tensor | None = None,
                    out: torch.Tensor | None = None) -> torch.Tensor:
    """shape_chi2_grad_scale: grad [n, 8] = grad_chi2 [n] x grad_unit [n, 8]
    (grad_unit taken by chi2_bwd with grad_chi2 = None)."""
    dev = grad_unit.device
    if (grad_unit.dtype != torch.float32 or grad_unit.dim() != 2 or grad_unit.shape[1] != 8
            or not grad_unit.is_contiguous()):
        raise ValueError("grad_unit must be a contiguous float32 [n, 8] tensor")
    n = int(grad_unit.shape[0])
    if grad_chi2 is not None:
        grad_chi2 = grad_chi2.to(device=dev, dtype=torch.float32).contiguous()
        if grad_chi2.numel() != n:
            raise ValueError("grad_chi2 must hold one value per stamp")
    if out is None:
        out = torch.empty_like(grad_unit)
    elif out.shape != grad_unit.shape or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 [n, 8] tensor")
    _check(lib.shape_chi2_grad_scale(_ptr(grad_unit), _ptr(grad_chi2), n, _ptr(out),
                                     _stream(dev)), "shape_chi2_grad_scale")
    return out


class SersicChi2(torch.autograd.Function):
    """chi^2 of the model per stamp, differentiable in the parameters.  When
    the parameters need a gradient, the forward pass is the library's adjoint
    sweep with dL/dchi2 = 1 (chi^2 and the gradient in one sweep) and the
    backward pass only scales that gradient by the upstream dL/dchi2;
    otherwise the forward pass sweeps chi^2 alone."""

    @staticmethod
    def forward(ctx, params, batch):
        p = params.detach().contiguous()
        if ctx.needs_input_grad[0]:
            out = chi2_bwd(batch, p)
            ctx.grad_unit = out["grad"]
            return out["chi2"]
        return chi2_fwd(batch, p)

    @staticmethod
    def backward(ctx, grad_chi2):
        return chi2_grad_scale(ctx.grad_unit, grad_chi2), None


def sersic_chi2(params: torch.Tensor, batch: DeviceBatch) -> torch.Tensor:
    return SersicChi2.apply(params, batch)


def frame_detect(frames: DeviceFrames, max_side: int = 128):
    """shape_frame_detect: dict(info [n,3] = sky, r50, F; peak [n,2]; box [n,3]; status)."""
    n, dev = frames.n, frames.device
    info, peak, box, st = _outs(n, dev, ((n, 3), torch.float32), ((n, 2), torch.int32),
                                ((n, 3), torch.int32), ((n,), torch.int32))
    f = frames.c_struct()
    _check(lib.shape_frame_detect(C.byref(f), int(max_side), _ptr(info), _ptr(peak), _ptr(box),
                                  _ptr(st), _stream(dev)), "shape_frame_detect")
    return dict(info=info, peak=peak, box=box, status=st)


def frame_offsets(box: torch.Tensor):
    """shape_frame_offsets: (offset [n] int64, total [1] int64), on the device."""
    n, dev = int(box.shape[0]), box.device
    off, tot = _outs(n, dev, ((n,), torch.int64), ((1,), torch.int64))
    _check(lib.shape_frame_offsets(_ptr(box), n, _ptr(off), _ptr(tot), _stream(dev)),
           "shape_frame_offsets")
    return off, tot


def frame_cut(frames: DeviceFrames, box: torch.Tensor, sigma: torch.Tensor,
              out: torch.Tensor | None = None) -> DeviceBatch:
    """Cut the boxes out into a DeviceBatch (FP32 stamps); sigma [n] is each
    frame's pixel noise.  Without `out` the total pixel count is read back to
    size the stamps; with `out` (float32, at least n * max_side^2 elements)
    nothing is read back and the batch views all of `out`."""
    n, dev = frames.n, frames.device
    off, tot = frame_offsets(box)
    if out is None:
        total = int(tot.item())
        stamps = torch.empty(max(total, 1), dtype=torch.float32, device=dev)
    else:
        if out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor")
        stamps, total = out, out.numel()
    sides = torch.empty(n, dtype=torch.int32, device=dev)
    f = frames.c_struct()
    _check(lib.shape_frame_cut(C.byref(f), _ptr(box), _ptr(off), _ptr(stamps), stamps.numel(),
                               _ptr(sides), _stream(dev)), "shape_frame_cut")
    return DeviceBatch(pixels=stamps[:total] if total else stamps[:0], sigma=sigma, offsets=off,
                       sides=sides)


STAR_GAUSSIAN = 0
STAR_MOFFAT = 1


def star_moments(batch: DeviceBatch, rec: torch.Tensor, profile: int = STAR_GAUSSIAN,
                 tol: float = 1e-4, max_iter: int = 20):
    """shape_star_moments: returns (out [n,4] = size, beta, I0, r0; iters; status)."""
    n, dev = batch.n, batch.device
    rec = _rows(rec, n, REC_LEN, "rec", dev)
    out, it, st = _outs(n, dev, ((n, 4), torch.float32), ((n,), torch.int32), ((n,), torch.int32))
    b = batch.c_struct()
    _check(lib.shape_star_moments(C.byref(b), int(profile), _ptr(rec), float(tol), int(max_iter),
                                  _ptr(out), _ptr(it), _ptr(st), _stream(dev)),
           "shape_star_moments")
    return out, it, st


def star_moments_beta(batch: DeviceBatch, rec: torch.Tensor, beta: float, tol: float = 1e-4,
                      max_iter: int = 20):
    """shape_star_moments_beta (Moffat, beta fixed): returns (out [n,4] = rd,
    beta, I0, r0; iters; status)."""
    n, dev = batch.n, batch.device
    rec = _rows(rec, n, REC_LEN, "rec", dev)
    out, it, st = _outs(n, dev, ((n, 4), torch.float32), ((n,), torch.int32), ((n,), torch.int32))
    b = batch.c_struct()
    _check(lib.shape_star_moments_beta(C.byref(b), float(beta), _ptr(rec), float(tol),
                                       int(max_iter), _ptr(out), _ptr(it), _ptr(st),
                                       _stream(dev)), "shape_star_moments_beta")
    return out, it, st


def queue_cfg(**overrides) -> QueueCfg:
    c = QueueCfg()
    _check(lib.shape_queue_default_cfg(C.byref(c)), "shape_queue_default_cfg")
    for k, v in overrides.items():
        if not hasattr(c, k):
            raise AttributeError(k)
        setattr(c, k, v)
    return c


def queue_workspace_bytes(n: int) -> int:
    b = C.c_size_t()
    _check(lib.shape_queue_workspace_bytes(int(n), C.byref(b)), "shape_queue_workspace_bytes")
    return int(b.value)


class QueueGraph:
    """A captured queue step (one LM trial for every active stamp)."""

    def __init__(self, batch, opts, cfg, ws):
        self._b = batch.c_struct()   # kept alive: the graph holds the values
        self._o, self._c, self._ws = opts, cfg, ws
        h = C.c_void_p()
        _check(lib.shape_queue_graph_create(C.byref(self._b), C.byref(opts), C.byref(cfg),
                                            _ptr(ws), ws.numel(), C.byref(h)),
               "shape_queue_graph_create")
        self.handle = h

    def launch(self, device):
        _check(lib.shape_queue_graph_launch(self.handle, _stream(device)),
               "shape_queue_graph_launch")

    def close(self):
        if self.handle:
            _check(lib.shape_queue_graph_destroy(self.handle), "shape_queue_graph_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def queue_active(ws: torch.Tensor) -> int:
    """Stamps still iterating after the last step (synchronises the stream)."""
    return int(ws[8:12].view(torch.int32).item())


def fit_queue(batch: DeviceBatch, rec: torch.Tensor | None = None,
              p_init: torch.Tensor | None = None, opts: ShapeOpts | None = None,
              cfg: QueueCfg | None = None, use_graph: bool = True, check_every: int = 2,
              want_perr: bool = False, drain_at: int = 4096):
    """Work-queue fit: shape_queue_start, then one LM trial per step (a hipGraph
    replay when use_graph) until every stamp is done or max_iter_lm steps, then
    shape_queue_finish.  The active count is read every check_every steps;
    once it is at most drain_at (0: never) the remaining stamps are finished
    by shape_queue_drain.  Returns the fit_sersic outputs plus the step count
    and whether the drain ran."""
    opts = opts or default_opts()
    cfg = cfg or queue_cfg()
    n, dev = batch.n, batch.device
    rec = _rows(rec, n, REC_LEN, "rec", dev)
    p_init = _rows(p_init, n, 8, "p_init", dev)
    p, chi2, it, st, sw = _outs(n, dev, ((n, 8), torch.float32), ((n,), torch.float32),
                                ((n,), torch.int32), ((n,), torch.int32), ((n,), torch.int32))
    perr = torch.empty((n, 8), dtype=torch.float32, device=dev) if want_perr else None
    if n == 0:
        return dict(p=p, chi2=chi2, perr=perr, iters=it, status=st, sweeps=sw, steps=0)
    nbytes = queue_workspace_bytes(n)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = batch.c_struct()
    _check(lib.shape_queue_start(C.byref(b), C.byref(opts), C.byref(cfg), _ptr(p_init), _ptr(rec),
                                 _ptr(ws), nbytes, _stream(dev)), "shape_queue_start")
    graph = QueueGraph(batch, opts, cfg, ws) if use_graph else None
    steps = 0
    drained = False
    try:
        while steps < opts.max_iter_lm:
            if graph:
                graph.launch(dev)
            else:
                _check(lib.shape_queue_step(C.byref(b), C.byref(opts), C.byref(cfg), _ptr(ws),
                                            nbytes, _stream(dev)), "shape_queue_step")
            steps += 1
            if check_every and steps % check_every == 0:
                active = queue_active(ws)
                if active == 0:
                    break
                if active <= drain_at:
                    _check(lib.shape_queue_drain(C.byref(b), C.byref(opts), C.byref(cfg),
                                                 _ptr(ws), nbytes, _stream(dev)),
                           "shape_queue_drain")
                    drained = True
                    break
    finally:
        if graph:
            graph.close()
    _check(lib.shape_queue_finish(C.byref(b), C.byref(opts), _ptr(ws), nbytes, _ptr(p),
                                  _ptr(chi2), _ptr(perr), _ptr(it), _ptr(st), _ptr(sw),
                                  _stream(dev)), "shape_queue_finish")
    return dict(p=p, chi2=chi2, perr=perr, iters=it, status=st, sweeps=sw, steps=steps,
                drained=drained)


def fit_queue_static(batch: DeviceBatch, rec: torch.Tensor | None = None,
                     p_init: torch.Tensor | None = None, opts: ShapeOpts | None = None,
                     cfg: QueueCfg | None = None, out: dict | None = None,
                     want_perr: bool = False):
    """shape_fit_queue_static: the work-queue fit in one call on the library's
    static workspace (at most STATIC_MAX_STAMPS stamps).  With `out` (a dict of
    preallocated p, chi2, iters, status and optional perr, sweeps tensors) the
    call allocates nothing on the device."""
    opts = opts or default_opts()
    cfg = cfg or queue_cfg()
    n, dev = batch.n, batch.device
    rec = _rows(rec, n, REC_LEN, "rec", dev)
    p_init = _rows(p_init, n, 8, "p_init", dev)
    if out is None:
        p, chi2, it, st, sw = _outs(n, dev, ((n, 8), torch.float32), ((n,), torch.float32),
                                    ((n,), torch.int32), ((n,), torch.int32), ((n,), torch.int32))
        perr = torch.empty((n, 8), dtype=torch.float32, device=dev) if want_perr else None
        out = dict(p=p, chi2=chi2, perr=perr, iters=it, status=st, sweeps=sw)
    b = batch.c_struct()
    _check(lib.shape_fit_queue_static(C.byref(b), C.byref(opts), C.byref(cfg), _ptr(p_init),
                                      _ptr(rec), _ptr(out["p"]), _ptr(out["chi2"]),
                                      _ptr(out.get("perr")), _ptr(out["iters"]),
                                      _ptr(out["status"]), _ptr(out.get("sweeps")), _stream(dev)),
           "shape_fit_queue_static")
    return out


def pipeline(batch: DeviceBatch, opts: ShapeOpts | None = None, want_perr: bool = False):
    """The three stages back to back on the current stream (the plain form)."""
    opts = opts or default_opts()
    rec0, it0, st0 = centroid(batch, opts)
    rec1, it1, st1 = moments(batch, rec0, opts)
    fit = fit_sersic(batch, rec=rec1, opts=opts, want_perr=want_perr)
    return dict(centroid=rec0, moments=rec1, iters=torch.stack([it0, it1, fit["iters"]], 1),
                status=torch.stack([st0, st1, fit["status"]], 1), p=fit["p"], chi2=fit["chi2"],
                perr=fit["perr"], sweeps=fit["sweeps"])
