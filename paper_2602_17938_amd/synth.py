"""Seeded synthetic astronomical frames for the L.A.Cosmic workloads.

This module only draws inputs; it holds none of the method's arithmetic and is
shared by the tests, the benchmark and the CPU reference alike.

Two frame kinds stand in for the paper's workloads (astroscrappy's mock data at
4000 x 6500 and an HST WFPC2 frame; neither is available, so neither is
reproduced):

* ``"ccd"``  -- sky 200 e-, read noise 5 e-, gain 1 e-/ADU, Gaussian stars
  (FWHM 2.5-4 px, peaks 1e3-5e4 e-), cosmic rays (60 % single pixels, 40 %
  straight tracks 2-10 px long at a random angle, amplitude log-uniform
  5e2-2e4 e- per pixel) and hot pixels at +3e3 e-.  Densities are those of a
  512 x 512 frame holding 30 stars, 200 cosmic rays and 100 hot pixels, scaled
  by area.
* ``"cmos"`` -- a CMOS-like frame: sky 50 e-, read noise 1.5 e-, gain
  0.25 e-/ADU, no stars, hot pixels at 0.1 % density with amplitude
  log-uniform 1e3-6e4 ADU, cosmic rays at 2 per 1e4 px; rounded, clipped and
  stored as uint16 ADU, then converted to float32 (exactly).

Draw order (fixed): star centres, FWHMs, peaks, the Poisson sky+star image and
the Gaussian read noise (per 256-row block, each block with its own child
stream so the result does not depend on the thread count), cosmic rays, hot
pixels.  Every frame is ``float32`` row-major h x w in ADU.
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

BLOCK_ROWS = 256

# Method parameters used by every workload.
NITER = 4
SIGCLIP = 4.5
SIGFRAC = 0.3
OBJLIM = 5.0


@dataclass(frozen=True)
class FrameParams:
    gain: float
    readnoise: float
    sigclip: float = SIGCLIP
    sigfrac: float = SIGFRAC
    objlim: float = OBJLIM
    niter: int = NITER


CCD = dict(gain=1.0, readnoise=5.0, sky=200.0)
CMOS = dict(gain=0.25, readnoise=1.5, sky=50.0)


def params_for(kind: str) -> FrameParams:
    k = CCD if kind == "ccd" else CMOS
    return FrameParams(gain=k["gain"], readnoise=k["readnoise"])


def _threads(threads):
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    return max(1, int(threads))


def _noise_image(mean_rows, h, w, sky, readnoise, ss_noise, threads):
    """Poisson(mean) + Normal(0, readnoise) in electrons, block by block."""
    nblk = (h + BLOCK_ROWS - 1) // BLOCK_ROWS
    children = ss_noise.spawn(nblk)
    out = np.empty((h, w), np.float64)

    def work(b):
        r0 = b * BLOCK_ROWS
        r1 = min(h, r0 + BLOCK_ROWS)
        g = np.random.Generator(np.random.PCG64(children[b]))
        lam = mean_rows(r0, r1)
        out[r0:r1] = g.poisson(lam).astype(np.float64)
        out[r0:r1] += g.normal(0.0, readnoise, size=(r1 - r0, w))

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(work, range(nblk)))
    return out


def _star_field(g, h, w, nstars):
    """Star centres, FWHMs and peaks, drawn in that order."""
    cy = g.uniform(0.0, h, size=nstars) if nstars else np.zeros(0)
    cx = g.uniform(0.0, w, size=nstars) if nstars else np.zeros(0)
    fwhm = g.uniform(2.5, 4.0, size=nstars) if nstars else np.zeros(0)
    peak = g.uniform(1e3, 5e4, size=nstars) if nstars else np.zeros(0)
    return cy, cx, fwhm, peak


def _render_stars(h, w, sky, stars):
    """Mean image: sky plus each star's Gaussian sampled at pixel centres."""
    cy, cx, fwhm, peak = stars
    mean = np.full((h, w), sky, np.float64)
    for y0, x0, fw, pk in zip(cy, cx, fwhm, peak):
        sig = fw / 2.3548
        rad = int(math.ceil(6.0 * sig))
        ya, yb = max(0, int(y0) - rad), min(h, int(y0) + rad + 1)
        xa, xb = max(0, int(x0) - rad), min(w, int(x0) + rad + 1)
        if ya >= yb or xa >= xb:
            continue
        yy = (np.arange(ya, yb) + 0.5 - y0)[:, None]
        xx = (np.arange(xa, xb) + 0.5 - x0)[None, :]
        mean[ya:yb, xa:xb] += pk * np.exp(-(yy * yy + xx * xx) / (2.0 * sig * sig))
    return mean


def _cosmic_rays(g, h, w, ncr):
    """Pixel coordinates and per-pixel amplitudes (e-) of ncr cosmic rays."""
    single = g.random(ncr) < 0.6
    y0 = g.uniform(0.0, h, size=ncr)
    x0 = g.uniform(0.0, w, size=ncr)
    length = g.integers(2, 11, size=ncr)
    angle = g.uniform(0.0, math.pi, size=ncr)
    ys, xs = [], []
    for i in range(ncr):
        if single[i]:
            pts = {(int(y0[i]), int(x0[i]))}
        else:
            s = np.arange(length[i])
            py = np.floor(y0[i] + s * math.sin(angle[i]) + 0.5).astype(np.int64)
            px = np.floor(x0[i] + s * math.cos(angle[i]) + 0.5).astype(np.int64)
            pts = set(zip(py.tolist(), px.tolist()))
        for (py, px) in sorted(pts):
            if 0 <= py < h and 0 <= px < w:
                ys.append(py)
                xs.append(px)
    ys = np.asarray(ys, np.int64)
    xs = np.asarray(xs, np.int64)
    amp = np.exp(g.uniform(math.log(5e2), math.log(2e4), size=ys.size))
    return ys, xs, amp


def make_frame(kind: str, h: int, w: int, seed: int, threads=None,
               cr_scale: float = 1.0) -> np.ndarray:
    """One synthetic frame (float32, ADU) of the given kind and shape;
    cr_scale multiplies the cosmic-ray density (1: the workload's)."""
    if kind not in ("ccd", "cmos"):
        raise ValueError("kind must be 'ccd' or 'cmos'")
    threads = _threads(threads)
    ss = np.random.SeedSequence(seed)
    ss_feat, ss_noise = ss.spawn(2)
    g = np.random.Generator(np.random.PCG64(ss_feat))
    area = (h * w) / float(512 * 512)

    if kind == "ccd":
        p = CCD
        nstars = int(round(30 * area))
        stars = _star_field(g, h, w, nstars)
        if nstars:
            mean = _render_stars(h, w, p["sky"], stars)
            rows = lambda a, b: mean[a:b]  # noqa: E731
        else:
            rows = lambda a, b: np.full((b - a, w), p["sky"])  # noqa: E731
        e = _noise_image(rows, h, w, p["sky"], p["readnoise"], ss_noise, threads)
        ncr = int(round(200 * area * cr_scale))
        ys, xs, amp = _cosmic_rays(g, h, w, ncr)
        np.add.at(e, (ys, xs), amp)
        nhot = min(h * w, int(round(100 * area)))
        hot = g.choice(h * w, size=nhot, replace=False)
        e.reshape(-1)[hot] += 3e3
        return (e / p["gain"]).astype(np.float32)

    p = CMOS
    rows = lambda a, b: np.full((b - a, w), p["sky"])  # noqa: E731
    e = _noise_image(rows, h, w, p["sky"], p["readnoise"], ss_noise, threads)
    ncr = int(round(2e-4 * h * w * cr_scale))
    ys, xs, amp = _cosmic_rays(g, h, w, ncr)
    np.add.at(e, (ys, xs), amp)
    adu = e / p["gain"]
    nhot = min(h * w, int(round(1e-3 * h * w)))
    hot = g.choice(h * w, size=nhot, replace=False)
    adu.reshape(-1)[hot] += np.exp(g.uniform(math.log(1e3), math.log(6e4), size=nhot))
    u16 = np.clip(np.rint(adu), 0, 65535).astype(np.uint16)
    return u16.astype(np.float32)


# Named workloads: (kind, h, w, seed).
CONFIGS = {
    "c0": ("ccd", 512, 512, 1),
    "c1": ("ccd", 4096, 4096, 2),
    "c2": ("cmos", 6400, 9600, 3),
}


def config_frame(name: str, threads=None):
    kind, h, w, seed = CONFIGS[name]
    return make_frame(kind, h, w, seed, threads), params_for(kind)


def batch_specs():
    """The 64-frame mixed batch: 32 at 2048^2, 24 at 4096^2 and 8 at
    6400 x 9600 (CMOS), seeds 1000 + i."""
    specs = []
    i = 0
    for kind, h, w, count in (("ccd", 2048, 2048, 32), ("ccd", 4096, 4096, 24),
                              ("cmos", 6400, 9600, 8)):
        for _ in range(count):
            specs.append((kind, h, w, 1000 + i))
            i += 1
    return specs


def serve_pool_specs(per_size: int = 8):
    """Frame pool for the serving stream: per_size frames of each size,
    seeds 2000 + i."""
    specs = []
    i = 0
    for kind, h, w in (("ccd", 2048, 2048), ("ccd", 4096, 4096), ("cmos", 6400, 9600)):
        for _ in range(per_size):
            specs.append((kind, h, w, 2000 + i))
            i += 1
    return specs


def poisson_arrivals(rate_hz: float, n: int, seed: int = 7) -> np.ndarray:
    """Arrival times (s) of a Poisson stream of n requests at rate_hz."""
    g = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(g.exponential(1.0 / rate_hz, size=n))
