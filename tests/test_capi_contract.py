"""C-ABI contract checks that need no GPU.

The library must load, export every function include/lacosmic.h declares,
and reject bad arguments (EINVAL, EALIAS) before making any HIP call -- so
these calls are made with fake device addresses on a machine without a GPU.
"""

import ctypes
import math
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_PATH = os.path.join(ROOT, "paper_2602_17938_amd", "liblacosmic.so")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB_PATH):
        from paper_2602_17938_amd import build
        build.build()
    from paper_2602_17938_amd import lacosmic
    return lacosmic


def test_exports_every_declared_function(L):
    names = L.header_functions()
    assert len(names) >= 14
    raw = ctypes.CDLL(LIB_PATH)
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing


def test_strerror_covers_every_status(L):
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        s = L.strerror(code)
        assert s and s != "unknown status"
    assert L.strerror(-99) == "unknown status"


IMG = 0x10000000
MASK = 0x20000000
CLEAN = 0x30000000


def _run(L, img=IMG, h=64, w=64, mask=MASK, clean=CLEAN, **kw):
    p = L.make_params(kw.get("gain", 1.0), kw.get("readnoise", 5.0), kw.get("sigclip", 4.5),
                      kw.get("sigfrac", 0.3), kw.get("objlim", 5.0), kw.get("niter", 4))
    if "flags" in kw:
        p.flags = kw["flags"]
    st = L.Stats()
    return L.lib().lacosmic_run_ex(img, h, w, ctypes.byref(p), mask, clean, None, None,
                                   ctypes.byref(st))


@pytest.mark.parametrize("kw", [
    dict(img=None), dict(mask=None), dict(clean=None), dict(h=0), dict(w=0), dict(h=-5),
    dict(w=1 << 25), dict(h=1 << 16, w=1 << 15), dict(h=46341, w=46341), dict(niter=0), dict(niter=-1), dict(niter=1025), dict(gain=0.0),
    dict(gain=-1.0), dict(gain=math.nan), dict(gain=math.inf), dict(readnoise=-0.5),
    dict(readnoise=math.nan), dict(sigclip=0.0), dict(sigclip=math.inf), dict(sigfrac=0.0),
    dict(sigfrac=-0.1), dict(objlim=-1.0), dict(objlim=math.nan), dict(flags=32), dict(flags=1 << 31),
])
def test_invalid_arguments_rejected_without_gpu(L, kw):
    assert _run(L, **kw) == L.EINVAL


@pytest.mark.parametrize("kw", [
    dict(clean=IMG), dict(mask=IMG), dict(clean=IMG + 4 * 64 * 64 - 4),
    dict(mask=IMG + 100), dict(mask=CLEAN + 8), dict(clean=MASK - 4 * 64 * 64 + 1),
])
def test_aliasing_rejected_without_gpu(L, kw):
    assert _run(L, **kw) == L.EALIAS


def test_plain_entry_rejects_same_as_ex(L):
    lib = L.lib()
    assert lib.lacosmic_run(None, 8, 8, 1.0, 5.0, 4.5, 0.3, 5.0, 4, MASK, CLEAN) == L.EINVAL
    assert lib.lacosmic_run(IMG, 8, 8, 0.0, 5.0, 4.5, 0.3, 5.0, 4, MASK, CLEAN) == L.EINVAL
    assert lib.lacosmic_run(IMG, 8, 8, 1.0, 5.0, 4.5, 0.3, 5.0, 4, IMG, CLEAN) == L.EALIAS


def test_workspace_size_and_layout(L):
    assert L.workspace_bytes(0, 10) == 0
    assert L.workspace_bytes(10, -1) == 0
    assert L.workspace_bytes(1 << 16, 1 << 15) == 0  # 2^31 pixels: indices are 32-bit
    for h, w in [(1, 1), (512, 512), (4096, 4096), (6400, 9600)]:
        n = L.workspace_bytes(h, w)
        assert n >= 8 * h * w
        lay = L.workspace_layout(h, w)
        assert lay.total_bytes == n
        assert lay.row_words == (w + 63) // 64
        offs = [lay.s_offset, lay.sp_offset, lay.cand_offset, lay.mask_bits_offset]
        assert all(o % 256 == 0 for o in offs)
        assert lay.sp_offset >= lay.s_offset + 4 * h * w
        assert lay.cand_offset >= lay.sp_offset + 4 * h * w
        assert lay.mask_bits_offset >= lay.cand_offset + 8 * h * lay.row_words
        assert lay.mask_bits_offset + 8 * h * lay.row_words <= n


def test_misaligned_workspace_rejected(L):
    p = L.make_params(1.0, 5.0)
    st = L.Stats()
    rc = L.lib().lacosmic_run_ex(IMG, 64, 64, ctypes.byref(p), MASK, CLEAN, 0x40000010, None,
                                 ctypes.byref(st))
    assert rc == L.EINVAL


def test_stats_layout_matches_header(L):
    # iters_run, n_flagged, n_unreplaced, n_new[16], gain[16], gain_estimated[16]
    # with natural alignment
    assert L.Stats.n_unreplaced.offset == 16
    assert L.Stats.n_new.offset == 24
    assert L.Stats.gain.offset == 24 + 16 * 8
    assert L.Stats.gain_estimated.offset == 24 + 16 * 8 + 16 * 4
    assert ctypes.sizeof(L.Stats) == 24 + 16 * 8 + 16 * 4 + 16


def test_estimated_gain_flag_checks_without_gpu(L):
    # with the flag the gain field is ignored but must be finite and >= 0
    assert _run(L, gain=-1.0, flags=L.F_ESTIMATE_GAIN) == L.EINVAL
    assert _run(L, gain=math.nan, flags=L.F_ESTIMATE_GAIN) == L.EINVAL
    # uint16 input: the input spans 2 bytes per pixel for the alias check
    assert _run(L, clean=IMG + 2 * 64 * 64 - 4, flags=L.F_INPUT_U16) == L.EALIAS
    assert _run(L, clean=IMG + 2 * 64 * 64 + 4, flags=0) == L.EALIAS


def test_tile_shape_table(L):
    shapes = L.tile_shapes()
    assert len(shapes) >= 2
    for th, tw in shapes:
        assert th >= 1 and tw % 64 == 0
    th, tw = ctypes.c_int32(), ctypes.c_int32()
    assert L.lib().lacosmic_get_tile_shape(len(shapes), ctypes.byref(th),
                                           ctypes.byref(tw)) == L.EINVAL
    assert L.lib().lacosmic_get_tile_shape(-1, ctypes.byref(th), ctypes.byref(tw)) == L.EINVAL


def _ptrs(vals):
    arr = (ctypes.c_void_p * len(vals))(*vals)
    return ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))


def _batch(L, n=2, imgs=None, masks=None, cleans=None, hs=None, ws=None, params=None):
    imgs = imgs or [IMG + i * 0x1000000 for i in range(n)]
    masks = masks or [MASK + i * 0x1000000 for i in range(n)]
    cleans = cleans or [CLEAN + i * 0x1000000 for i in range(n)]
    hs = hs or [64] * n
    ws = ws or [64] * n
    params = params or [L.make_params(1.0, 5.0)] * n
    H = (ctypes.c_int64 * n)(*hs)
    W = (ctypes.c_int64 * n)(*ws)
    P = (L.Params * n)(*params)
    return L.lib().lacosmic_run_batch(n, _ptrs(imgs), H, W, P, _ptrs(masks), _ptrs(cleans), None)


def test_batch_argument_checks_without_gpu(L):
    lib = L.lib()
    assert lib.lacosmic_run_batch(-1, None, None, None, None, None, None, None) == L.EINVAL
    assert lib.lacosmic_run_batch(0, None, None, None, None, None, None, None) == L.OK
    assert lib.lacosmic_run_batch(2, None, None, None, None, None, None, None) == L.EINVAL
    assert _batch(L, hs=[64, 0]) == L.EINVAL
    assert _batch(L, params=[L.make_params(1.0, 5.0), L.make_params(1.0, 5.0, niter=3)]) \
        == L.EINVAL
    assert _batch(L, params=[L.make_params(1.0, 5.0), L.make_params(-1.0, 5.0)]) == L.EINVAL
    # frame 1 writes into frame 0's input
    assert _batch(L, cleans=[CLEAN, IMG + 64]) == L.EALIAS
    assert _batch(L, masks=[MASK, MASK + 10]) == L.EALIAS
    assert _batch(L, imgs=[IMG, CLEAN]) == L.EALIAS


def test_server_argument_checks_without_gpu(L):
    lib = L.lib()
    out = ctypes.c_void_p()
    assert lib.lacosmic_server_create(0, 4, ctypes.byref(out)) == L.EINVAL
    assert lib.lacosmic_server_create(1 << 30, 0, ctypes.byref(out)) == L.EINVAL
    assert lib.lacosmic_server_create(1 << 30, 4, None) == L.EINVAL
    t = ctypes.c_uint64()
    p = L.make_params(1.0, 5.0)
    assert lib.lacosmic_server_submit(None, IMG, 0, 8, 8, ctypes.byref(p), ctypes.byref(t)) \
        == L.EINVAL
    assert lib.lacosmic_server_poll(None, 1, None, None, None, None) == L.EINVAL
    assert lib.lacosmic_server_drain(None) == L.EINVAL
    assert lib.lacosmic_server_destroy(None) == L.EINVAL


def test_check_sqrt_argument_checks_without_gpu(L):
    """The square-root self-check accepts only ranges inside [2^-96, +inf]."""
    lib = L.lib()
    n = ctypes.c_uint64(0)
    einval = -1
    assert lib.lacosmic_check_sqrt(0x0F800000, 0x7F800000, None) == einval
    assert lib.lacosmic_check_sqrt(0x3F800000, 0x3F000000, ctypes.byref(n)) == einval  # lo > hi
    assert lib.lacosmic_check_sqrt(0x0F7FFFFF, 0x3F800000, ctypes.byref(n)) == einval  # below 2^-96
    assert lib.lacosmic_check_sqrt(0x3F800000, 0x7F800001, ctypes.byref(n)) == einval  # NaN
    assert lib.lacosmic_check_sqrt(0x3F800000, 0xBF800000, ctypes.byref(n)) == einval  # negative

