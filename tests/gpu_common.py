"""Helpers shared by the GPU tests: device frames, oracle comparison, crops."""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# One iteration of the method reads the previous image within 8 pixels
# (pass A: 4, pass B: 4); four iterations reach 32.
DEP_RADIUS_PER_ITER = 8


def host_threads():
    return max(1, min(16, os.cpu_count() or 1))


def lac():
    from paper_2602_17938_amd import lacosmic
    return lacosmic


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def gpu_run(img_np, p, early_stop=False, niter=None, workspace=None, stream=None,
            full_sp=False):
    L = lac()
    params = L.make_params(p.gain, p.readnoise, p.sigclip, p.sigfrac, p.objlim,
                           p.niter if niter is None else niter, early_stop, full_sp)
    m, c, st = L.run_ex(to_dev(img_np), params, workspace=workspace, stream=stream)
    return m.cpu().numpy(), c.cpu().numpy(), st


def oracle_run(img_np, p, early_stop=False, niter=None, trace=False, nthreads=None):
    import oracle
    return oracle.lacosmic(img_np, p.gain, p.readnoise, p.sigclip, p.sigfrac, p.objlim,
                           p.niter if niter is None else niter, early_stop=early_stop,
                           nthreads=nthreads or host_threads(), trace=trace)


def assert_bits_equal(a, b, what):
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    if a.dtype == np.float32:
        av, bv = a.view(np.uint32), b.view(np.uint32)
    else:
        av, bv = a, b
    bad = np.nonzero(av != bv)
    if bad[0].size:
        idx = tuple(x[:5] for x in bad)
        raise AssertionError("%s: %d elements differ, first at %s: gpu %s oracle %s" %
                             (what, bad[0].size, list(zip(*idx)), a[idx], b[idx]))


def crop_windows(h, w, size, niter):
    """Crop regions (core y0, y1, x0, x1) covering corners, edges and the
    interior, and the oracle input window around each (core + margin,
    clipped to the frame)."""
    m = DEP_RADIUS_PER_ITER * niter + 8
    cy = [0, h // 2 - size // 2, h - size]
    cx = [0, w // 2 - size // 2, w - size]
    out = []
    for y0 in cy:
        for x0 in cx:
            y0 = max(0, y0)
            x0 = max(0, x0)
            y1, x1 = min(h, y0 + size), min(w, x0 + size)
            oy0, ox0 = max(0, y0 - m), max(0, x0 - m)
            oy1, ox1 = min(h, y1 + m), min(w, x1 + m)
            out.append(((y0, y1, x0, x1), (oy0, oy1, ox0, ox1)))
    return out
