"""GPU test of lacosmic_run_noalloc, the entry point for callers that cannot
allocate: through the C ABI, its results equal lacosmic_run_ex's bit for bit
on consecutive calls (the second with a smaller frame, so the static scratch
holds a larger frame's leftovers), and a frame too large for the scratch is
rejected."""

import ctypes

import numpy as np
import pytest

from gpu_common import assert_bits_equal, lac, to_dev

pytestmark = pytest.mark.gpu


def _call(L, d, params, stream=None):
    """lacosmic_run_noalloc straight through ctypes: outputs allocated
    beforehand, stats filled."""
    import torch
    h, w = d.shape
    m = torch.empty((h, w), dtype=torch.uint8, device="cuda")
    c = torch.empty((h, w), dtype=torch.float32, device="cuda")
    p = L._typed(params, d)
    st = L.Stats()
    torch.cuda.synchronize()
    rc = L.lib().lacosmic_run_noalloc(d.data_ptr(), h, w, ctypes.byref(p), m.data_ptr(),
                                      c.data_ptr(), None if stream is None else stream.cuda_stream,
                                      ctypes.byref(st))
    return rc, m, c, st


def _same(L, d, params, what, stream=None):
    rc, m, c, st = _call(L, d, params, stream)
    assert rc == L.OK, (what, L.strerror(rc))
    rm, rcl, rst = L.run_ex(d, params)
    assert_bits_equal(m.cpu().numpy(), rm.cpu().numpy(), what + " mask")
    assert_bits_equal(c.cpu().numpy(), rcl.cpu().numpy(), what + " clean")
    n = rst.iters_run
    assert st.iters_run == n
    assert [st.n_new[k] for k in range(n)] == [rst.n_new[k] for k in range(n)]
    assert st.n_unreplaced == rst.n_unreplaced
    assert [st.gain[k] for k in range(n)] == [rst.gain[k] for k in range(n)]
    return m


def test_noalloc_matches_run_ex_on_consecutive_calls():
    import torch
    from paper_2602_17938_amd import synth
    L = lac()
    pc = synth.params_for("ccd")
    big = synth.make_frame("ccd", 1536, 2048, 91)
    small = synth.make_frame("ccd", 300, 257, 92)
    params = L.make_params(pc.gain, pc.readnoise, pc.sigclip, pc.sigfrac, pc.objlim, pc.niter)
    m1 = _same(L, to_dev(big), params, "first call, 1536x2048")
    assert int(m1.sum()) > 0
    _same(L, to_dev(small), params, "second call, 300x257")
    # a third, on a stream of the caller's, with early stop and the gain estimated
    img, p0 = synth.config_frame("c0")
    est = L.make_params(0.0, p0.readnoise, p0.sigclip, p0.sigfrac, p0.objlim, 6, True,
                        estimate_gain=True)
    s = torch.cuda.Stream()
    _same(L, to_dev(img), est, "third call, 512x512, estimated gain", stream=s)
    # uint16 input
    cm = synth.make_frame("cmos", 640, 700, 93)
    pcm = synth.params_for("cmos")
    pu = L.make_params(pcm.gain, pcm.readnoise, pcm.sigclip, pcm.sigfrac, pcm.objlim, pcm.niter)
    _same(L, torch.from_numpy(cm.astype(np.uint16)).cuda(), pu, "fourth call, uint16")


def test_noalloc_rejects_frames_larger_than_the_scratch():
    import torch
    L = lac()
    h, w = 4096, 4096  # its workspace is about twice the scratch
    assert L.workspace_bytes(h, w) > 128 << 20
    d = torch.zeros((h, w), dtype=torch.float32, device="cuda")
    params = L.make_params(1.0, 5.0)
    rc, _, _, _ = _call(L, d, params)
    assert rc == L.ESCRATCH
    assert L.strerror(rc) == "frame needs more than the static scratch buffer"
