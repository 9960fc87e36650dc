"""L.A.Cosmic CPU oracle -- TEST INFRASTRUCTURE ONLY.

ctypes wrapper around ``lacosmic_oracle.cpp``: a plain, slow CPU implementation
of the L.A.Cosmic iteration (dfcosmic paper, Methods: "Algorithm" steps 1-7 and
"Main parameters"), templated on float and double.  Only the tests, the package
smoke check and the benchmark's CPU-baseline leg may import this module; the
product library never does, and shares no code with it.

Functions take and return numpy arrays.  ``build()`` compiles the shared
library with ``g++ -O2 -ffp-contract=off -fno-fast-math -fopenmp``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lacosmic_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=c++17"]

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle library in place and return its path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", *CFLAGS, _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    I = ctypes.c_int
    F = ctypes.c_float
    D = ctypes.c_double
    lib.oracle_lacosmic_f32.argtypes = [P, I64, I64, F, F, F, F, F, I, I, I, I, I, P, P, P, P,
                                        P, P, P, P, P, P, P]
    lib.oracle_lacosmic_f32.restype = I
    lib.oracle_lacosmic_f64.argtypes = [P, I64, I64, D, D, D, D, D, I, I, I, I, I, P, P, P, P,
                                        P, P, P, P, P, P, P]
    lib.oracle_lacosmic_f64.restype = I
    lib.oracle_exact_sum.argtypes = [P, I64]
    lib.oracle_exact_sum.restype = D
    lib.oracle_estimate_gain_f32.argtypes = [P, I64, F, P, P, P, P, P]
    lib.oracle_estimate_gain_f32.restype = I
    lib.oracle_laplacian_f32.argtypes = [P, I64, I64, P]
    lib.oracle_laplacian_f64.argtypes = [P, I64, I64, P]
    lib.oracle_median_f32.argtypes = [P, I64, I64, I, P]
    lib.oracle_median_f64.argtypes = [P, I64, I64, I, P]
    lib.oracle_sep_median_f32.argtypes = [P, I64, I64, I, P]
    lib.oracle_noise_f32.argtypes = [P, I64, I64, F, F, P]
    lib.oracle_dilate3.argtypes = [P, I64, I64, P]
    lib.oracle_masked_median5_f32.argtypes = [P, P, I64, I64, P]
    lib.oracle_masked_median5_f32.restype = I64
    lib.oracle_masked_median5_f64.argtypes = [P, P, I64, I64, P]
    lib.oracle_masked_median5_f64.restype = I64
    lib.oracle_max_threads.restype = I
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _img(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    if a.ndim != 2:
        raise ValueError("expected a 2-D image")
    return a


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def lacosmic(img, gain, readnoise, sigclip=4.5, sigfrac=0.3, objlim=5.0, niter=4,
             early_stop=False, nthreads=1, dtype=np.float32, trace=False, estimate_gain=False,
             sepmed=False):
    """Run the whole method; returns a dict with mask (uint8), clean, n_new,
    iters_run, n_unreplaced, the gain each iteration used (gains: the given
    one, or with estimate_gain=True the estimate of that iteration, gain
    ignored) and, with trace=True, per-iteration s, sp, b1, mask and clean
    stacks (shape niter x h x w).  sepmed=True: the detection medians are the
    separable approximation (row medians, then column medians)."""
    lib = _load()
    dtype = np.dtype(dtype)
    img = _img(img, dtype)
    h, w = img.shape
    mask = np.zeros((h, w), np.uint8)
    clean = np.zeros((h, w), dtype)
    n_new = np.zeros(max(niter, 1), np.int64)
    gains = np.zeros(max(niter, 1), np.float64)
    iters = ctypes.c_int(0)
    unrep = ctypes.c_int64(0)
    tr = {}
    if trace:
        tr = dict(s=np.zeros((niter, h, w), dtype), sp=np.zeros((niter, h, w), dtype),
                  b1=np.zeros((niter, h, w), np.uint8),
                  mask=np.zeros((niter, h, w), np.uint8), clean=np.zeros((niter, h, w), dtype))
    fn = lib.oracle_lacosmic_f32 if dtype == np.float32 else lib.oracle_lacosmic_f64
    if dtype not in (np.float32, np.float64):
        raise ValueError("dtype must be float32 or float64")
    cast = np.float32 if dtype == np.float32 else np.float64
    rc = fn(_ptr(img), h, w, cast(gain), cast(readnoise), cast(sigclip), cast(sigfrac),
            cast(objlim), int(niter), int(bool(early_stop)), int(bool(estimate_gain)),
            int(bool(sepmed)), int(nthreads), _ptr(mask), _ptr(clean), _ptr(tr.get("s")), _ptr(tr.get("sp")),
            _ptr(tr.get("b1")), _ptr(tr.get("mask")), _ptr(tr.get("clean")), _ptr(n_new),
            ctypes.byref(iters), ctypes.byref(unrep), _ptr(gains))
    if rc != 0:
        raise ValueError("oracle rejected its arguments (rc=%d)" % rc)
    out = dict(mask=mask, clean=clean, n_new=n_new[:iters.value].copy(),
               iters_run=iters.value, n_unreplaced=unrep.value,
               gains=gains[:iters.value].copy())
    for k, v in tr.items():
        out["trace_" + k] = v[:iters.value]
    return out


def laplacian(img, dtype=np.float32):
    lib = _load()
    img = _img(img, dtype)
    out = np.zeros_like(img)
    f = lib.oracle_laplacian_f32 if img.dtype == np.float32 else lib.oracle_laplacian_f64
    f(_ptr(img), img.shape[0], img.shape[1], _ptr(out))
    return out


def median(img, k, dtype=np.float32):
    lib = _load()
    img = _img(img, dtype)
    out = np.zeros_like(img)
    f = lib.oracle_median_f32 if img.dtype == np.float32 else lib.oracle_median_f64
    f(_ptr(img), img.shape[0], img.shape[1], int(k), _ptr(out))
    return out


def sep_median(img, k):
    """Separable k x k median of a float32 image: row medians, then column
    medians of those, each clamped on its own grid."""
    lib = _load()
    img = _img(img, np.float32)
    out = np.zeros_like(img)
    lib.oracle_sep_median_f32(_ptr(img), img.shape[0], img.shape[1], int(k), _ptr(out))
    return out


def noise(img, gain, readnoise):
    lib = _load()
    img = _img(img, np.float32)
    out = np.zeros_like(img)
    lib.oracle_noise_f32(_ptr(img), img.shape[0], img.shape[1], np.float32(gain),
                         np.float32(readnoise), _ptr(out))
    return out


def dilate3(b):
    lib = _load()
    b = np.ascontiguousarray(b, dtype=np.uint8)
    out = np.zeros_like(b)
    lib.oracle_dilate3(_ptr(b), b.shape[0], b.shape[1], _ptr(out))
    return out


def masked_median5(img, mask, dtype=np.float32):
    lib = _load()
    img = _img(img, dtype)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    out = np.zeros_like(img)
    f = (lib.oracle_masked_median5_f32 if img.dtype == np.float32
         else lib.oracle_masked_median5_f64)
    kept = f(_ptr(img), _ptr(mask), img.shape[0], img.shape[1], _ptr(out))
    return out, int(kept)


def exact_sum(values):
    """Correctly rounded binary64 sum of the values (Shewchuk's exact partials)."""
    v = np.ascontiguousarray(values, dtype=np.float64).ravel()
    return float(_load().oracle_exact_sum(_ptr(v), v.size))


def estimate_gain(img, readnoise):
    """The gain estimate of a float32 image (used when no gain is supplied):
    dict with gain (1.0 when there is no estimate), valid, rounds (clipping
    rounds applied), kept (values kept), mean and var of the kept values."""
    a = _img(img, np.float32) if np.ndim(img) == 2 else np.ascontiguousarray(img, np.float32)
    g, m, v = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    r, k = ctypes.c_int(), ctypes.c_int64()
    valid = _load().oracle_estimate_gain_f32(_ptr(a), a.size, np.float32(readnoise),
                                             ctypes.byref(g), ctypes.byref(r), ctypes.byref(k),
                                             ctypes.byref(m), ctypes.byref(v))
    return dict(gain=g.value, valid=bool(valid), rounds=r.value, kept=k.value, mean=m.value,
                var=v.value)
