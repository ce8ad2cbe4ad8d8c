"""Seeded synthetic postage stamps for the five benchmark workloads.

This module only makes inputs.  It draws per-object truth parameters, renders
them point-sampled at pixel centres, adds sky and i.i.d. Gaussian noise, and
packs the stamps row-major.  It holds none of the measurement arithmetic
(centroiding, weighted moments, profile fitting); both the FP64 oracle and the
HIP library only consume what it produces.

Conventions (shared with the library's public header):
  * pixel (row i, col j) has centre (x, y) = (j, i); stamps are square, side W,
    stored row-major; the stamp centre is ((W-1)/2, (W-1)/2);
  * parameter vector p = (x0, y0, e1, e2, Re, n, I0, sky); for Moffat stars the
    5th and 6th slots hold (rd, beta);
  * u = (x-x0, y-y0), v = S(e) u with S(e) = [[1-e1, -e2], [-e2, 1+e1]],
    D = 1-|e|^2, R^2 = |v|^2 / D (area-preserving, so Re is the circularised
    half-light radius);
  * Sersic (Sec. 4.1, eq. ser): I0 exp(-b(n) (R/Re)^(1/n)), b(n) fixed by
    "Re is the half-light radius", i.e. P(2n, b) = 1/2; here b comes from
    scipy's inverse regularised incomplete gamma function, a third
    implementation independent of both the oracle and the library;
  * Moffat (Sec. 4.2.2, eq. mof): I0 (1 + R^2/rd^2)^(-beta).

Workload recipes (sizes and distributions of the paper's simulations, Sec. 4.1,
as restated for a stamp batch):
  plain32     1,000 x 32^2 FP32, Gaussian galaxies (n = 0.5), sigma U(2,4),
              offset U(+-2), e_i ~ N(0,0.2) re-drawn until |e| < 0.6,
              peak 1000, sky 10, noise sigma 20 (peak S/N 50).
  plain48     100,000 x 48^2 FP32 Sersic: n U(0.5,4), Re log-U(1.5,6),
              e_i ~ N(0,0.25) re-drawn until |e| < 0.7, offset U(+-2),
              flux log-U(1e3,1e5), sky 10, matched-filter S/N log-U(20,200).
  uneven      1,000,000 stamps, side round(exp U(ln16, ln128)); 80% Sersic as
              plain48 with Re = side/8, 20% Moffat beta = 3, FWHM U(2,5),
              e uniform in the disk |e| < 0.1.
  sersic64    65,536 x 64^2 FP32, drawn as plain48.
  sersic64h   262,144 x 64^2 stored FP16 with a per-stamp power-of-two scale.

Randomness: stamps are generated in chunks of CHUNK objects; chunk c uses
numpy.random.default_rng([seed, c]), so any sub-range is reproducible alone and
chunks can be made in parallel.  Within a chunk the draw order is fixed:
(side, type,) x-offset, y-offset, ellipticity (with re-draws), size, index,
flux, S/N, then the pixel noise.
"""
from __future__ import annotations

import math
import os
import sys
from concurrent.futures import ProcessPoolExecutor
from dataclasses import dataclass, field

import numpy as np
from scipy.special import gammaincinv, gamma as gamma_fn

CHUNK = 1024
SKY = 10.0
MOFFAT_BETA = 3.0

SERSIC = 0
MOFFAT = 1


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    side: int | None          # None => uneven sides
    kind: str                 # "gauss32" | "sersic" | "uneven"
    storage: str = "f32"      # "f32" | "f16"
    description: str = ""


WORKLOADS = {
    "plain32": Workload("plain32", 1_000, 32, "gauss32",
                        description="1,000 x 32x32 FP32 elliptical Gaussian galaxies, 4-parameter fit"),
    "plain32x": Workload("plain32x", 262_144, 32, "gauss32",
                         description="262,144 x 32x32 FP32 elliptical Gaussian galaxies drawn as "
                                     "plain32 (its first 1,000 stamps are plain32)"),
    "plain48": Workload("plain48", 100_000, 48, "sersic",
                        description="100,000 x 48x48 FP32 Sersic galaxies, 8-parameter fit"),
    "uneven": Workload("uneven", 1_000_000, None, "uneven",
                       description="1,000,000 stamps, side log-U(16,128), 80% Sersic / 20% Moffat"),
    "sersic64": Workload("sersic64", 65_536, 64, "sersic",
                         description="65,536 x 64x64 FP32 Sersic galaxies"),
    "sersic64h": Workload("sersic64h", 262_144, 64, "sersic", storage="f16",
                          description="262,144 x 64x64 Sersic galaxies, FP16 + per-stamp scale"),
    "stars32": Workload("stars32", 1_048_576, 32, "moffat",
                        description="1,048,576 x 32x32 FP32 Moffat stars, beta U(2.5,5), "
                                    "FWHM U(2,5)"),
}


def sersic_b(n):
    """b(n) with P(2n, b) = 1/2 (half-light normalisation of eq. ser)."""
    return gammaincinv(2.0 * np.asarray(n, dtype=np.float64), 0.5)


def sersic_flux_factor(n, re):
    """Total flux / I0 for the area-normalised elliptical Sersic profile."""
    n = np.asarray(n, dtype=np.float64)
    b = sersic_b(n)
    return 2.0 * math.pi * n * gamma_fn(2.0 * n) * b ** (-2.0 * n) * np.asarray(re) ** 2


def moffat_flux_factor(rd, beta):
    """Total flux / I0 for the area-normalised Moffat profile (beta > 1)."""
    return math.pi * np.asarray(rd) ** 2 / (beta - 1.0)


def _radius2(side, p):
    """Area-normalised elliptical R^2 on a side x side grid for params p[k,8]."""
    coords = np.arange(side, dtype=np.float64)
    x = coords[None, None, :]
    y = coords[None, :, None]
    x0 = p[:, 0][:, None, None]
    y0 = p[:, 1][:, None, None]
    e1 = p[:, 2][:, None, None]
    e2 = p[:, 3][:, None, None]
    ux = x - x0
    uy = y - y0
    vx = (1.0 - e1) * ux - e2 * uy
    vy = -e2 * ux + (1.0 + e1) * uy
    d = 1.0 - e1 * e1 - e2 * e2
    return (vx * vx + vy * vy) / d


def render_sersic(side, p):
    """Noiseless Sersic galaxies without sky, shape [k, side, side], FP64."""
    p = np.asarray(p, dtype=np.float64).reshape(-1, 8)
    r2 = _radius2(side, p)
    re = p[:, 4][:, None, None]
    n = p[:, 5][:, None, None]
    i0 = p[:, 6][:, None, None]
    b = sersic_b(n)
    s = np.sqrt(r2) / re
    return i0 * np.exp(-b * s ** (1.0 / n))


def render_moffat(side, p):
    """Noiseless Moffat stars without sky; p[:,4] = rd, p[:,5] = beta."""
    p = np.asarray(p, dtype=np.float64).reshape(-1, 8)
    r2 = _radius2(side, p)
    rd = p[:, 4][:, None, None]
    beta = p[:, 5][:, None, None]
    i0 = p[:, 6][:, None, None]
    return i0 * (1.0 + r2 / (rd * rd)) ** (-beta)


def _draw_e(rng, k, sd, emax):
    e = rng.normal(0.0, sd, size=(k, 2))
    bad = np.hypot(e[:, 0], e[:, 1]) >= emax
    while bad.any():
        e[bad] = rng.normal(0.0, sd, size=(int(bad.sum()), 2))
        bad = np.hypot(e[:, 0], e[:, 1]) >= emax
    return e


def _loguniform(rng, lo, hi, k):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=k))


@dataclass
class Chunk:
    pixels: np.ndarray        # float32 (or float16) packed stamps
    sides: np.ndarray         # int32 [k]
    sigma: np.ndarray         # float32 [k]
    model: np.ndarray         # uint8 [k]
    truth: np.ndarray         # float64 [k, 8]
    scale: np.ndarray | None = None   # float32 [k] (FP16 storage only)


def _noise_and_pack(rng, side, clean, sigma, storage):
    k = clean.shape[0]
    noisy = clean + SKY + rng.standard_normal(clean.shape) * sigma[:, None, None]
    if storage == "f16":
        peak = np.abs(noisy).reshape(k, -1).max(axis=1)
        # power-of-two scale so that every stored value fits FP16's range
        # with headroom: scale = 2^ceil(log2(max|I| / 32768)).
        scale = np.exp2(np.ceil(np.log2(np.maximum(peak, 1e-30) / 32768.0)))
        q = (noisy / scale[:, None, None]).astype(np.float16)
        return q.reshape(-1), scale.astype(np.float32)
    return noisy.astype(np.float32).reshape(-1), None


def _sersic_chunk(rng, k, side, storage, gauss32):
    c = (side - 1) / 2.0
    p = np.zeros((k, 8))
    p[:, 0] = c + rng.uniform(-2.0, 2.0, k)
    p[:, 1] = c + rng.uniform(-2.0, 2.0, k)
    if gauss32:
        p[:, 2:4] = _draw_e(rng, k, 0.2, 0.6)
        sig = rng.uniform(2.0, 4.0, k)
        p[:, 4] = sig * math.sqrt(2.0 * math.log(2.0))
        p[:, 5] = 0.5
        p[:, 6] = 1000.0
        p[:, 7] = SKY
        clean = render_sersic(side, p)
        sigma = np.full(k, 1000.0 / 50.0)
    else:
        p[:, 2:4] = _draw_e(rng, k, 0.25, 0.7)
        p[:, 4] = _loguniform(rng, 1.5, 6.0, k)
        p[:, 5] = rng.uniform(0.5, 4.0, k)
        flux = _loguniform(rng, 1e3, 1e5, k)
        snr = _loguniform(rng, 20.0, 200.0, k)
        p[:, 6] = flux / sersic_flux_factor(p[:, 5], p[:, 4])
        p[:, 7] = SKY
        clean = render_sersic(side, p)
        sigma = np.sqrt((clean.reshape(k, -1) ** 2).sum(axis=1)) / snr
    sigma32 = sigma.astype(np.float32)
    pix, scale = _noise_and_pack(rng, side, clean, sigma32.astype(np.float64), storage)
    return Chunk(pix, np.full(k, side, np.int32), sigma32, np.zeros(k, np.uint8), p, scale)


def _uneven_chunk(rng, k, storage):
    sides = np.rint(np.exp(rng.uniform(math.log(16.0), math.log(128.0), k))).astype(np.int32)
    star = rng.uniform(0.0, 1.0, k) < 0.2
    p = np.zeros((k, 8))
    c = (sides - 1) / 2.0
    p[:, 0] = c + rng.uniform(-2.0, 2.0, k)
    p[:, 1] = c + rng.uniform(-2.0, 2.0, k)
    eg = _draw_e(rng, k, 0.25, 0.7)
    # stars: uniform in the disk |e| < 0.1
    rad = 0.1 * np.sqrt(rng.uniform(0.0, 1.0, k))
    phi = rng.uniform(0.0, 2.0 * math.pi, k)
    es = np.stack([rad * np.cos(phi), rad * np.sin(phi)], axis=1)
    p[:, 2:4] = np.where(star[:, None], es, eg)
    fwhm = rng.uniform(2.0, 5.0, k)
    rd = fwhm / (2.0 * math.sqrt(2.0 ** (1.0 / MOFFAT_BETA) - 1.0))
    p[:, 4] = np.where(star, rd, sides / 8.0)
    nser = rng.uniform(0.5, 4.0, k)
    p[:, 5] = np.where(star, MOFFAT_BETA, nser)
    flux = _loguniform(rng, 1e3, 1e5, k)
    snr = _loguniform(rng, 20.0, 200.0, k)
    gal_f = sersic_flux_factor(np.where(star, 1.0, p[:, 5]), np.where(star, 1.0, p[:, 4]))
    star_f = moffat_flux_factor(p[:, 4], MOFFAT_BETA)
    p[:, 6] = flux / np.where(star, star_f, gal_f)
    p[:, 7] = SKY
    sigma = np.zeros(k)
    pix_parts, scales = [], np.ones(k, np.float32)
    for idx in range(k):
        s = int(sides[idx])
        pp = p[idx:idx + 1]
        clean = render_moffat(s, pp) if star[idx] else render_sersic(s, pp)
        sigma[idx] = math.sqrt(float((clean ** 2).sum())) / snr[idx]
        pix, sc = _noise_and_pack(rng, s, clean, np.array([np.float32(sigma[idx])], np.float64), storage)
        pix_parts.append(pix)
        if sc is not None:
            scales[idx] = sc[0]
    return Chunk(np.concatenate(pix_parts), sides, sigma.astype(np.float32),
                 star.astype(np.uint8), p, scales if storage == "f16" else None)


def _moffat_chunk(rng, k, side, storage):
    c = (side - 1) / 2.0
    p = np.zeros((k, 8))
    p[:, 0] = c + rng.uniform(-2.0, 2.0, k)
    p[:, 1] = c + rng.uniform(-2.0, 2.0, k)
    rad = 0.1 * np.sqrt(rng.uniform(0.0, 1.0, k))
    phi = rng.uniform(0.0, 2.0 * math.pi, k)
    p[:, 2] = rad * np.cos(phi)
    p[:, 3] = rad * np.sin(phi)
    beta = rng.uniform(2.5, 5.0, k)
    fwhm = rng.uniform(2.0, 5.0, k)
    p[:, 4] = fwhm / (2.0 * np.sqrt(2.0 ** (1.0 / beta) - 1.0))
    p[:, 5] = beta
    flux = _loguniform(rng, 1e4, 1e6, k)
    snr = _loguniform(rng, 50.0, 500.0, k)
    p[:, 6] = flux / moffat_flux_factor(p[:, 4], beta)
    p[:, 7] = SKY
    clean = render_moffat(side, p)
    sigma = (np.sqrt((clean.reshape(k, -1) ** 2).sum(axis=1)) / snr).astype(np.float32)
    pix, scale = _noise_and_pack(rng, side, clean, sigma.astype(np.float64), storage)
    return Chunk(pix, np.full(k, side, np.int32), sigma, np.ones(k, np.uint8), p, scale)


def _make_chunk(args):
    wl_name, seed, cidx, k, storage = args
    wl = WORKLOADS[wl_name]
    rng = np.random.default_rng([seed, cidx])
    if wl.kind == "uneven":
        return _uneven_chunk(rng, k, storage)
    if wl.kind == "moffat":
        return _moffat_chunk(rng, k, wl.side, storage)
    return _sersic_chunk(rng, k, wl.side, storage, wl.kind == "gauss32")


@dataclass
class Batch:
    """A packed batch of stamps (host numpy arrays)."""
    workload: str
    pixels: np.ndarray
    offsets: np.ndarray       # int64 [n] element offset of each stamp
    sides: np.ndarray         # int32 [n]
    sigma: np.ndarray         # float32 [n]
    model: np.ndarray         # uint8 [n] 0 = Sersic, 1 = Moffat
    truth: np.ndarray         # float64 [n, 8]
    scale: np.ndarray | None  # float32 [n] for FP16 storage
    start: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return int(self.sides.shape[0])

    def stamp(self, i):
        o = int(self.offsets[i])
        s = int(self.sides[i])
        a = self.pixels[o:o + s * s].astype(np.float64).reshape(s, s)
        if self.scale is not None:
            a = a * float(self.scale[i])
        return a

    def head(self, m):
        """The first m stamps as a Batch of their own (same storage)."""
        m = min(int(m), self.n)
        end = int(self.offsets[m - 1] + int(self.sides[m - 1]) ** 2) if m else 0
        return Batch(self.workload, self.pixels[:end], self.offsets[:m].copy(), self.sides[:m],
                     self.sigma[:m], self.model[:m], self.truth[:m],
                     None if self.scale is None else self.scale[:m], self.start, dict(self.meta))

    def dequantised_f64(self):
        """All pixels as FP64 (FP16 storage multiplied by its exact scale)."""
        if self.scale is None:
            return self.pixels.astype(np.float64)
        per_px = np.repeat(self.scale.astype(np.float64), self.sides.astype(np.int64) ** 2)
        return self.pixels.astype(np.float64) * per_px


def make(workload, count=None, start=0, seed=0, storage=None, workers=None):
    """Generate stamps [start, start+count) of a workload.

    `start` must be a multiple of CHUNK so chunk streams line up.
    """
    wl = WORKLOADS[workload]
    if count is None:
        count = wl.n - start
    if start % CHUNK:
        raise ValueError("start must be a multiple of %d" % CHUNK)
    if start < 0 or count < 0 or start + count > wl.n:
        raise ValueError("range outside the workload")
    storage = storage or wl.storage
    jobs = []
    c0 = start // CHUNK
    remaining = count
    c = c0
    while remaining > 0:
        k = min(CHUNK, remaining)
        jobs.append((workload, seed, c, k, storage))
        remaining -= k
        c += 1
    if workers is None:
        workers = min(len(jobs), int(os.environ.get("SYNTH_WORKERS", min(16, os.cpu_count() or 1))))
        # never fork workers from a process whose GPU runtime is already up
        tmod = sys.modules.get("torch")
        if tmod is not None and tmod.cuda.is_initialized():
            workers = 1
    if workers > 1 and len(jobs) > 1:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            chunks = list(ex.map(_make_chunk, jobs))
    else:
        chunks = [_make_chunk(j) for j in jobs]
    if not chunks:
        empty32 = np.zeros(0, np.float32)
        return Batch(workload, np.zeros(0, np.float16 if storage == "f16" else np.float32),
                     np.zeros(0, np.int64), np.zeros(0, np.int32), empty32,
                     np.zeros(0, np.uint8), np.zeros((0, 8)), empty32 if storage == "f16" else None, start)
    sides = np.concatenate([ch.sides for ch in chunks])
    sizes = sides.astype(np.int64) ** 2
    offsets = np.zeros(len(sides), np.int64)
    np.cumsum(sizes[:-1], out=offsets[1:])
    scale = np.concatenate([ch.scale for ch in chunks]) if storage == "f16" else None
    return Batch(workload, np.concatenate([ch.pixels for ch in chunks]), offsets, sides,
                 np.concatenate([ch.sigma for ch in chunks]),
                 np.concatenate([ch.model for ch in chunks]),
                 np.concatenate([ch.truth for ch in chunks]), scale, start)


# ---------------------------------------------------------------------------
# Whole frames with one galaxy each (the paper's simulations place each galaxy
# on a 512 x 512 grid and cut a stamp of side 6 r50 around it).
# ---------------------------------------------------------------------------
FRAME_SIDE = 512
FRAME_WINDOW = 128     # the profile is rendered in a 128 x 128 window about its centre
FRAME_CHUNK = 64
FRAMES_N = 4096


@dataclass
class Frames:
    """A stack of equal frames (host numpy arrays)."""
    pixels: np.ndarray        # float32 [n, H, W]
    sigma: np.ndarray         # float32 [n]
    truth: np.ndarray         # float64 [n, 8] (centre in frame pixels)
    start: int = 0

    @property
    def n(self):
        return int(self.pixels.shape[0])

    def head(self, m):
        m = min(int(m), self.n)
        return Frames(self.pixels[:m], self.sigma[:m], self.truth[:m], self.start)


def _frame_chunk(args):
    seed, cidx, k = args
    rng = np.random.default_rng([seed, 0x46524D, cidx])
    H = W = FRAME_SIDE
    p = np.zeros((k, 8))
    p[:, 0] = rng.uniform(128.0, 384.0, k)
    p[:, 1] = rng.uniform(128.0, 384.0, k)
    p[:, 2:4] = _draw_e(rng, k, 0.25, 0.7)
    p[:, 4] = _loguniform(rng, 1.5, 6.0, k)
    p[:, 5] = rng.uniform(0.5, 4.0, k)
    flux = _loguniform(rng, 1e4, 1e6, k)
    snr = _loguniform(rng, 5e3, 5e4, k)
    p[:, 6] = flux / sersic_flux_factor(p[:, 5], p[:, 4])
    p[:, 7] = SKY
    out = np.empty((k, H, W), np.float32)
    sig = np.empty(k, np.float32)
    h = FRAME_WINDOW // 2
    for q in range(k):
        cx, cy = int(p[q, 0]), int(p[q, 1])
        win = p[q:q + 1].copy()
        win[0, 0] -= cx - h
        win[0, 1] -= cy - h
        clean = render_sersic(FRAME_WINDOW, win)[0]
        sig[q] = np.float32(math.sqrt(float((clean ** 2).sum())) / snr[q])
        frame = SKY + rng.standard_normal((H, W)) * float(sig[q])
        frame[cy - h:cy + h, cx - h:cx + h] += clean
        out[q] = frame
    return out, sig, p


def make_frames(count=None, start=0, seed=0, workers=None):
    """Frames [start, start+count) of the 512 x 512 one-galaxy-per-frame set:
    Sersic galaxies as the 48x48 set (n U(0.5,4), Re log-U(1.5,6), e_i N(0,0.25)
    with |e| < 0.7, sky 10), centre U(128,384) on both axes, flux log-U(1e4,1e6),
    S/N log-U(5e3,5e4) (the sum over a whole frame carries the noise of
    all its 262,144 pixels, so the total flux needs a high S/N); the profile is rendered in a 128 x 128 window about
    the centre pixel, noise over the whole frame."""
    count = FRAMES_N - start if count is None else count
    if start % FRAME_CHUNK or start < 0 or count < 0 or start + count > FRAMES_N:
        raise ValueError("range outside the frame set")
    jobs, c, left = [], start // FRAME_CHUNK, count
    while left > 0:
        k = min(FRAME_CHUNK, left)
        jobs.append((seed, c, k))
        left -= k
        c += 1
    if workers is None:
        workers = min(len(jobs), int(os.environ.get("SYNTH_WORKERS", min(16, os.cpu_count() or 1))))
        tmod = sys.modules.get("torch")
        if tmod is not None and tmod.cuda.is_initialized():
            workers = 1
    if workers > 1 and len(jobs) > 1:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            parts = list(ex.map(_frame_chunk, jobs))
    else:
        parts = [_frame_chunk(j) for j in jobs]
    if not parts:
        return Frames(np.zeros((0, FRAME_SIDE, FRAME_SIDE), np.float32), np.zeros(0, np.float32),
                      np.zeros((0, 8)), start)
    return Frames(np.concatenate([a for a, _, _ in parts]), np.concatenate([b for _, b, _ in parts]),
                  np.concatenate([t for _, _, t in parts]), start)
