"""Python binding of liblacosmic.so (argument marshalling only).

Every step of the method runs in the library's HIP kernels; this module only
checks tensors, allocates outputs with torch (device memory and streams are
PyTorch's role here) and forwards pointers through ctypes.  If the library is
not built, importing this module raises ImportError -- there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblacosmic.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "lacosmic.h")

OK, EINVAL, ENOMEM, EHIP, ENONFINITE, EALIAS, EBUDGET, ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7
F_EARLY_STOP = 1
F_FULL_SP = 2
F_INPUT_U16 = 4
F_ESTIMATE_GAIN = 8
F_SEPMED = 16


class LacosmicError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__("%s: %s (%d)" % (where or "lacosmic", strerror(status), status))


class Params(ctypes.Structure):
    _fields_ = [("gain", ctypes.c_float), ("readnoise", ctypes.c_float),
                ("sigclip", ctypes.c_float), ("sigfrac", ctypes.c_float),
                ("objlim", ctypes.c_float), ("niter", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("iters_run", ctypes.c_int32), ("n_flagged", ctypes.c_int64),
                ("n_unreplaced", ctypes.c_int64), ("n_new", ctypes.c_int64 * 16),
                ("gain", ctypes.c_float * 16), ("gain_estimated", ctypes.c_int8 * 16)]


class WsLayout(ctypes.Structure):
    _fields_ = [("s_offset", ctypes.c_size_t), ("sp_offset", ctypes.c_size_t),
                ("cand_offset", ctypes.c_size_t), ("mask_bits_offset", ctypes.c_size_t),
                ("row_words", ctypes.c_size_t), ("total_bytes", ctypes.c_size_t)]


def _signatures():
    P, I64, I32, U64, F, SZ = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                               ctypes.c_uint64, ctypes.c_float, ctypes.c_size_t)
    PP = ctypes.POINTER(ctypes.c_void_p)
    D = ctypes.POINTER(ctypes.c_double)
    return {
        "lacosmic_run": ([P, I64, I64, F, F, F, F, F, I32, P, P], ctypes.c_int),
        "lacosmic_run_ex": ([P, I64, I64, ctypes.POINTER(Params), P, P, P, P,
                             ctypes.POINTER(Stats)], ctypes.c_int),
        "lacosmic_run_noalloc": ([P, I64, I64, ctypes.POINTER(Params), P, P, P,
                                  ctypes.POINTER(Stats)], ctypes.c_int),
        "lacosmic_workspace_bytes": ([I64, I64], SZ),
        "lacosmic_workspace_layout": ([I64, I64, ctypes.POINTER(WsLayout)], ctypes.c_int),
        "lacosmic_run_batch": ([I32, PP, ctypes.POINTER(I64), ctypes.POINTER(I64),
                                ctypes.POINTER(Params), PP, PP, P], ctypes.c_int),
        "lacosmic_server_create": ([U64, I32, ctypes.POINTER(P)], ctypes.c_int),
        "lacosmic_server_submit": ([P, P, ctypes.c_int, I64, I64, ctypes.POINTER(Params),
                                    ctypes.POINTER(U64)], ctypes.c_int),
        "lacosmic_server_poll": ([P, U64, P, P, D, D], ctypes.c_int),
        "lacosmic_server_drain": ([P], ctypes.c_int),
        "lacosmic_server_destroy": ([P], ctypes.c_int),
        "lacosmic_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "lacosmic_set_tile_shape": ([I32], ctypes.c_int),
        "lacosmic_set_frame_graphs": ([I32], ctypes.c_int),
        "lacosmic_get_tile_shape": ([I32, ctypes.POINTER(I32), ctypes.POINTER(I32)],
                                    ctypes.c_int),
        "lacosmic_batch_pass_ms": ([ctypes.POINTER(ctypes.c_float), I32, P], ctypes.c_int),
        "lacosmic_batch_tile_shape": ([], ctypes.c_int),
        "lacosmic_batch_launch_mode": ([], ctypes.c_int),
        "lacosmic_batch_groups": ([], ctypes.c_int),
        "lacosmic_check_sqrt": ([ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(U64)],
                                ctypes.c_int),
        "lacosmic_shutdown": ([], None),
    }


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblacosmic.so is not built (run paper_2602_17938_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in _signatures().items():
        try:
            fn = getattr(lib, name)
        except AttributeError:
            continue  # calling it raises AttributeError: no silent fallback
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def lib():
    return _lib


def header_functions(path=HEADER):
    """Names of the functions include/lacosmic.h declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lacosmic_[a-z_]+)\s*\(", text)))


def strerror(status: int) -> str:
    return _lib.lacosmic_strerror(int(status)).decode()


def _check(rc, where):
    if rc != OK:
        raise LacosmicError(rc, where)


def _dev_image(img, allow_u16=False):
    if not isinstance(img, torch.Tensor) or not img.is_cuda:
        raise TypeError("img must be a CUDA (HIP) torch tensor")
    ok = (torch.float32, torch.uint16) if allow_u16 else (torch.float32,)
    if img.dtype not in ok or img.dim() != 2 or not img.is_contiguous():
        raise TypeError("img must be a contiguous 2-D %s tensor" %
                        " or ".join(str(d).replace("torch.", "") for d in ok))
    return img


def _typed(params: Params, img) -> Params:
    """params with the input-type flag set as the tensor's dtype says."""
    p = Params.from_buffer_copy(params)
    if img.dtype == torch.uint16:
        p.flags |= F_INPUT_U16
    else:
        p.flags &= ~F_INPUT_U16
    return p


def make_params(gain, readnoise, sigclip=4.5, sigfrac=0.3, objlim=5.0, niter=4,
                early_stop=False, full_sp=False, estimate_gain=False, sepmed=False):
    """Method parameters.  estimate_gain=True: no gain is supplied (gain is
    ignored; pass 0) and each iteration estimates it from the current image.
    sepmed=True: separable detection medians (the comparison variant)."""
    return Params(float(gain), float(readnoise), float(sigclip), float(sigfrac), float(objlim),
                  int(niter), (F_EARLY_STOP if early_stop else 0) | (F_FULL_SP if full_sp else 0)
                  | (F_ESTIMATE_GAIN if estimate_gain else 0) | (F_SEPMED if sepmed else 0))


def run(img, gain, readnoise, sigclip=4.5, sigfrac=0.3, objlim=5.0, niter=4):
    """lacosmic_run: synchronous (library stream), early stop on.  Returns
    (mask u8, clean f32)."""
    img = _dev_image(img)
    h, w = img.shape
    mask = torch.empty((h, w), dtype=torch.uint8, device=img.device)
    clean = torch.empty((h, w), dtype=torch.float32, device=img.device)
    with torch.cuda.device(img.device):
        # the library stream does not wait for torch's: finish pending work first
        torch.cuda.current_stream().synchronize()
        rc = _lib.lacosmic_run(img.data_ptr(), h, w, gain, readnoise, sigclip, sigfrac, objlim,
                               int(niter), mask.data_ptr(), clean.data_ptr())
    _check(rc, "lacosmic_run")
    return mask, clean


def run_ex(img, params: Params, out_mask=None, out_clean=None, workspace=None,
           stream="current", stats=True):
    """lacosmic_run_ex.  img: float32, or uint16 ADU (the input-type flag is
    set from the dtype).  stream: "current" (torch's current stream, the
    default), a torch.cuda.Stream, or None (the library's own stream, which
    makes the call synchronous).  With a torch stream the call is
    asynchronous unless stats=True.  Returns (mask, clean, Stats or None)."""
    img = _dev_image(img, allow_u16=True)
    params = _typed(params, img)
    h, w = img.shape
    if out_mask is None:
        out_mask = torch.empty((h, w), dtype=torch.uint8, device=img.device)
    if out_clean is None:
        out_clean = torch.empty((h, w), dtype=torch.float32, device=img.device)
    ws_ptr = None
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < workspace_bytes(h, w):
            raise ValueError("workspace holds fewer than lacosmic_workspace_bytes(h, w) bytes")
        ws_ptr = workspace.data_ptr()
    st = Stats() if stats else None
    with torch.cuda.device(img.device):
        if stream == "current":
            stream = torch.cuda.current_stream()
        elif stream is None:
            torch.cuda.current_stream().synchronize()
        s_ptr = None if stream is None else stream.cuda_stream
        rc = _lib.lacosmic_run_ex(img.data_ptr(), h, w, ctypes.byref(params), out_mask.data_ptr(),
                                  out_clean.data_ptr(), ws_ptr, s_ptr,
                                  ctypes.byref(st) if st is not None else None)
    _check(rc, "lacosmic_run_ex")
    return out_mask, out_clean, st


def run_noalloc(img, params: Params, out_mask=None, out_clean=None, stream="current",
                stats=True):
    """lacosmic_run_noalloc: as run_ex, with the library's static scratch as
    the workspace (the call allocates nothing itself; outputs the caller does
    not pass are allocated here, by torch, before the call)."""
    img = _dev_image(img, allow_u16=True)
    params = _typed(params, img)
    h, w = img.shape
    if out_mask is None:
        out_mask = torch.empty((h, w), dtype=torch.uint8, device=img.device)
    if out_clean is None:
        out_clean = torch.empty((h, w), dtype=torch.float32, device=img.device)
    st = Stats() if stats else None
    with torch.cuda.device(img.device):
        if stream == "current":
            stream = torch.cuda.current_stream()
        s_ptr = None if stream is None else stream.cuda_stream
        rc = _lib.lacosmic_run_noalloc(img.data_ptr(), h, w, ctypes.byref(params),
                                       out_mask.data_ptr(), out_clean.data_ptr(), s_ptr,
                                       ctypes.byref(st) if st is not None else None)
    _check(rc, "lacosmic_run_noalloc")
    return out_mask, out_clean, st


def workspace_bytes(h, w) -> int:
    return int(_lib.lacosmic_workspace_bytes(int(h), int(w)))


def workspace_layout(h, w) -> WsLayout:
    L = WsLayout()
    _check(_lib.lacosmic_workspace_layout(int(h), int(w), ctypes.byref(L)), "workspace_layout")
    return L


def alloc_workspace(h, w, device="cuda"):
    return torch.empty(workspace_bytes(h, w), dtype=torch.uint8, device=device)


def workspace_planes(ws, h, w):
    """S, S' and the candidate map (uint8 0/1) a caller workspace holds after
    a run (those of the last iteration run), as host numpy arrays."""
    L = workspace_layout(h, w)
    host = ws.cpu().numpy()
    S = host[L.s_offset:L.s_offset + 4 * h * w].view(np.float32).reshape(h, w)
    sp = host[L.sp_offset:L.sp_offset + 4 * h * w].view(np.float32).reshape(h, w)
    nb = h * L.row_words * 8
    words = host[L.cand_offset:L.cand_offset + nb].view(np.uint64).reshape(h, L.row_words)
    bits = np.unpackbits(words.view(np.uint8).reshape(h, -1), axis=1, bitorder="little")
    return S, sp, bits[:, :w].copy()


def run_batch(imgs, params, out_masks=None, out_cleans=None, stream="current"):
    """lacosmic_run_batch over a list of device images; params: one Params
    or a list.  Returns lists of masks and cleans."""
    n = len(imgs)
    imgs = [_dev_image(x, allow_u16=True) for x in imgs]
    if isinstance(params, Params):
        params = [params] * n
    params = [_typed(p, x) for p, x in zip(params, imgs)]
    if out_masks is None:
        out_masks = [torch.empty(x.shape, dtype=torch.uint8, device=x.device) for x in imgs]
    if out_cleans is None:
        out_cleans = [torch.empty(x.shape, dtype=torch.float32, device=x.device) for x in imgs]
    VP = ctypes.c_void_p * n
    I64 = ctypes.c_int64 * n
    PA = Params * n
    a_img = VP(*[x.data_ptr() for x in imgs])
    a_h = I64(*[x.shape[0] for x in imgs])
    a_w = I64(*[x.shape[1] for x in imgs])
    a_p = PA(*params)
    a_m = VP(*[m.data_ptr() for m in out_masks])
    a_c = VP(*[c.data_ptr() for c in out_cleans])
    with torch.cuda.device(imgs[0].device if n else torch.device("cuda")):
        if stream == "current":
            stream = torch.cuda.current_stream()
        elif stream is None:
            torch.cuda.current_stream().synchronize()
        s_ptr = None if stream is None else stream.cuda_stream
        rc = _lib.lacosmic_run_batch(n, ctypes.cast(a_img, ctypes.POINTER(ctypes.c_void_p)),
                                     a_h, a_w, a_p,
                                     ctypes.cast(a_m, ctypes.POINTER(ctypes.c_void_p)),
                                     ctypes.cast(a_c, ctypes.POINTER(ctypes.c_void_p)), s_ptr)
    _check(rc, "lacosmic_run_batch")
    return out_masks, out_cleans


# Passes of one iteration in launch order (lacosmic_batch_pass_ms).
PASS_NAMES = ("GAIN", "US", "A1", "SC", "S1", "SG", "B", "S2", "OUT")


def batch_pass_ms(niter, stream="current", per_iter=False):
    """Per-pass durations (ms) of one eager replay of the last batch's
    kernels: dict pass name -> ms summed over iterations, or with per_iter a
    list of such dicts, one per iteration."""
    if stream == "current":
        stream = torch.cuda.current_stream()
    npass = len(PASS_NAMES)
    buf = (ctypes.c_float * (npass * niter))()
    k = _lib.lacosmic_batch_pass_ms(buf, npass * niter,
                                    None if stream is None else stream.cuda_stream)
    if k < 0:
        raise LacosmicError(k, "batch_pass_ms")
    iters = [dict.fromkeys(PASS_NAMES, 0.0) for _ in range(niter)]
    for i in range(k):
        iters[i // npass][PASS_NAMES[i % npass]] += buf[i]
    if per_iter:
        return iters
    return {n: sum(d[n] for d in iters) for n in PASS_NAMES}


def set_frame_graphs(on: bool):
    _check(_lib.lacosmic_set_frame_graphs(1 if on else 0), "set_frame_graphs")


def set_tile_shape(cfg: int):
    _check(_lib.lacosmic_set_tile_shape(int(cfg)), "set_tile_shape")


def tile_shapes():
    out = []
    i = 0
    while True:
        th, tw = ctypes.c_int32(), ctypes.c_int32()
        if _lib.lacosmic_get_tile_shape(i, ctypes.byref(th), ctypes.byref(tw)) != OK:
            return out
        out.append((th.value, tw.value))
        i += 1


class Server:
    """Continuous-batching server (lacosmic_server_*).  Frames are host numpy
    arrays or CUDA tensors (float32, or uint16 ADU); a device frame must stay
    alive and unchanged until poll has returned its results."""

    def __init__(self, hbm_budget_bytes, max_frames=64):
        h = ctypes.c_void_p()
        _check(_lib.lacosmic_server_create(int(hbm_budget_bytes), int(max_frames),
                                           ctypes.byref(h)), "server_create")
        self._h = h
        self._shapes = {}

    def submit(self, img, params: Params) -> int:
        if isinstance(img, torch.Tensor):
            if not img.is_cuda or img.dim() != 2 or not img.is_contiguous():
                raise TypeError("a tensor frame must be a contiguous 2-D CUDA tensor")
            if img.dtype == torch.uint16:
                u16 = 1
            elif img.dtype == torch.float32:
                u16 = 0
            else:
                raise TypeError("img must be float32 or uint16")
            ptr = ctypes.c_void_p(img.data_ptr())
            shape = tuple(img.shape)
        else:
            if img.dtype == np.uint16:
                u16 = 1
            elif img.dtype == np.float32:
                u16 = 0
            else:
                raise TypeError("img must be float32 or uint16")
            img = np.ascontiguousarray(img)
            ptr = img.ctypes.data_as(ctypes.c_void_p)
            shape = img.shape
        t = ctypes.c_uint64()
        _check(_lib.lacosmic_server_submit(self._h, ptr, u16, shape[0], shape[1],
                                           ctypes.byref(params), ctypes.byref(t)),
               "server_submit")
        self._shapes[t.value] = shape
        return t.value

    def poll(self, ticket, want_outputs=True):
        """None while pending; else (mask, clean, t_submit_ns, t_done_ns)."""
        shape = self._shapes[ticket]
        mask = np.empty(shape, np.uint8) if want_outputs else None
        clean = np.empty(shape, np.float32) if want_outputs else None
        ts, td = ctypes.c_double(), ctypes.c_double()
        rc = _lib.lacosmic_server_poll(
            self._h, ticket, None if mask is None else mask.ctypes.data_as(ctypes.c_void_p),
            None if clean is None else clean.ctypes.data_as(ctypes.c_void_p), ctypes.byref(ts),
            ctypes.byref(td))
        if rc < 0:
            raise LacosmicError(rc, "server_poll")
        if rc == 0:
            return None
        del self._shapes[ticket]
        return mask, clean, ts.value, td.value

    def drain(self):
        _check(_lib.lacosmic_server_drain(self._h), "server_drain")

    def close(self):
        if self._h:
            _check(_lib.lacosmic_server_destroy(self._h), "server_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def shutdown():
    _lib.lacosmic_shutdown()
