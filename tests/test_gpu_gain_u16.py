"""GPU tests of the gain estimate (no gain supplied: estimated at each
iteration from the current image) and of uint16 ADU input, through the C ABI.

The estimate is exact on both sides (the sums are exact and rounded once, the
rest is the same binary64 expression), so the per-iteration gains must equal
the oracle's binary32 gains exactly, and masks and cleaned images bit for bit.
"""

import numpy as np
import pytest

from gpu_common import assert_bits_equal, lac, oracle_run, to_dev

pytestmark = pytest.mark.gpu

F32 = np.float32


def _params(p, niter=None, early=False, est=True):
    return lac().make_params(0.0 if est else p.gain, p.readnoise, p.sigclip, p.sigfrac,
                             p.objlim, p.niter if niter is None else niter, early,
                             estimate_gain=est)


def _oracle_est(img, p, niter=None, early=False):
    import oracle
    from gpu_common import host_threads
    return oracle.lacosmic(img, 0.0, p.readnoise, p.sigclip, p.sigfrac, p.objlim,
                           p.niter if niter is None else niter, early_stop=early,
                           nthreads=host_threads(), estimate_gain=True)


def _check(img, p, r, m, c, st, what):
    assert_bits_equal(m, r["mask"], what + " mask")
    assert_bits_equal(c, r["clean"], what + " clean")
    k = st.iters_run
    assert k == r["iters_run"], what
    assert [st.n_new[j] for j in range(k)] == list(r["n_new"]), what
    got = [F32(st.gain[j]) for j in range(k)]
    want = [F32(x) for x in r["gains"]]
    assert got == want, (what, got, want)
    assert st.n_unreplaced == r["n_unreplaced"], what


def _frames():
    from paper_2602_17938_amd import synth
    g = np.random.Generator(np.random.PCG64(21))
    out = []
    img, p = synth.config_frame("c0")
    out.append(("c0", img, p))
    cm = synth.make_frame("cmos", 700, 650, 31)
    out.append(("cmos", cm, synth.params_for("cmos")))
    # bias-subtracted frame: values around zero, negative ones included
    b = (g.poisson(30.0, (300, 257)) - 30.0 + g.normal(0, 3.0, (300, 257))).astype(F32)
    b.reshape(-1)[g.choice(b.size, 300, replace=False)] += 2000.0
    out.append(("bias", b, synth.params_for("ccd")))
    # gain 3.7 e-/ADU (estimate far from 1), ragged shape
    e = g.poisson(900.0, (211, 333)) + g.normal(0, 6.0, (211, 333))
    e.reshape(-1)[g.choice(e.size, 150, replace=False)] += 8000.0
    out.append(("gain3.7", (e / 3.7).astype(F32), synth.params_for("ccd")))
    return out


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("idx", range(4))
def test_estimated_gain_matches_oracle(idx, fused, monkeypatch):
    monkeypatch.setenv("LACOSMIC_FUSED_MAX_PX", str(1 << 30) if fused else "0")
    name, img, p = _frames()[idx]
    r = _oracle_est(img, p)
    L = lac()
    m, c, st = L.run_ex(to_dev(img), _params(p))
    _check(img, p, r, m.cpu().numpy(), c.cpu().numpy(), st, name)
    assert all(st.gain_estimated[j] == 1 for j in range(st.iters_run))


def test_estimated_gain_early_stop_and_eager():
    from paper_2602_17938_amd import synth
    L = lac()
    img, p = synth.config_frame("c0")
    r = _oracle_est(img, p, niter=8, early=True)
    assert r["iters_run"] < 8
    L.set_frame_graphs(True)
    try:
        m, c, st = L.run_ex(to_dev(img), _params(p, niter=8, early=True))
    finally:
        L.set_frame_graphs(False)  # the default
    _check(img, p, r, m.cpu().numpy(), c.cpu().numpy(), st, "early stop, graph")
    m2, c2, st2 = L.run_ex(to_dev(img), _params(p, niter=8, early=True))
    _check(img, p, r, m2.cpu().numpy(), c2.cpu().numpy(), st2, "eager")


def test_no_spread_uses_gain_one():
    """A constant frame has no spread: gain 1 for every iteration, reported as
    no estimate, and the result of a run with gain 1."""
    from paper_2602_17938_amd.synth import FrameParams
    L = lac()
    img = np.full((90, 130), 250.0, F32)
    img[40, 60] = 900.0  # one outlier, clipped away: the kept values are constant
    p = FrameParams(gain=1.0, readnoise=5.0)
    m, c, st = L.run_ex(to_dev(img), _params(p))
    assert [st.gain[j] for j in range(p.niter)] == [1.0] * p.niter
    assert [st.gain_estimated[j] for j in range(p.niter)] == [-1] * p.niter
    r = oracle_run(img, p)
    assert_bits_equal(m.cpu().numpy(), r["mask"], "mask")
    assert_bits_equal(c.cpu().numpy(), r["clean"], "clean")


def test_estimated_gain_in_batch_and_server():
    """Frames without a supplied gain mixed with frames with one, in one
    batch and through the server: each equals its lone run (and the oracle)."""
    import torch
    from paper_2602_17938_amd import synth
    L = lac()
    fr = _frames()
    imgs = [fr[0][1], fr[1][1], fr[3][1], synth.make_frame("ccd", 333, 444, 41)]
    ps = [fr[0][2], fr[1][2], fr[3][2], synth.params_for("ccd")]
    est = [True, False, True, False]
    params = [_params(p, est=e) for p, e in zip(ps, est)]
    masks, cleans = L.run_batch([to_dev(x) for x in imgs], params)
    torch.cuda.synchronize()
    for i, (img, q) in enumerate(zip(imgs, params)):
        m, c, _ = L.run_ex(to_dev(img), q)
        assert_bits_equal(masks[i].cpu().numpy(), m.cpu().numpy(), "batch mask %d" % i)
        assert_bits_equal(cleans[i].cpu().numpy(), c.cpu().numpy(), "batch clean %d" % i)
    r = _oracle_est(imgs[2], ps[2])
    assert_bits_equal(masks[2].cpu().numpy(), r["mask"], "batch vs oracle mask")
    with L.Server(2 << 30, 8) as srv:
        tickets = [srv.submit(img, q) for img, q in zip(imgs, params)]
        srv.drain()
        for i, t in enumerate(tickets):
            sm, sc, _, _ = srv.poll(t)
            assert_bits_equal(sm, masks[i].cpu().numpy(), "served mask %d" % i)
            assert_bits_equal(sc, cleans[i].cpu().numpy(), "served clean %d" % i)


def test_uint16_input_single_and_batch():
    """uint16 ADU frames read as uint16 by the first pass: identical to the
    same values passed as float32, alone and in a batch with float32 frames
    (and the oracle on the frame)."""
    import torch
    from paper_2602_17938_amd import synth
    L = lac()
    cm = synth.make_frame("cmos", 800, 1100, 51)
    cm2 = synth.make_frame("cmos", 77, 130, 52)
    ccd = synth.make_frame("ccd", 300, 300, 53)
    pc, pd = synth.params_for("cmos"), synth.params_for("ccd")
    par = L.make_params(pc.gain, pc.readnoise, pc.sigclip, pc.sigfrac, pc.objlim, pc.niter)
    pard = L.make_params(pd.gain, pd.readnoise, pd.sigclip, pd.sigfrac, pd.objlim, pd.niter)
    u = torch.from_numpy(cm.astype(np.uint16)).cuda()
    m16, c16, st16 = L.run_ex(u, par)
    m32, c32, st32 = L.run_ex(to_dev(cm), par)
    assert_bits_equal(m16.cpu().numpy(), m32.cpu().numpy(), "u16 mask")
    assert_bits_equal(c16.cpu().numpy(), c32.cpu().numpy(), "u16 clean")
    r = oracle_run(cm, pc)
    assert_bits_equal(m16.cpu().numpy(), r["mask"], "u16 vs oracle mask")
    assert_bits_equal(c16.cpu().numpy(), r["clean"], "u16 vs oracle clean")
    imgs = [u, to_dev(ccd), torch.from_numpy(cm2.astype(np.uint16)).cuda()]
    masks, cleans = L.run_batch(imgs, [par, pard, par])
    for i, ref in enumerate([cm, ccd, cm2]):
        m, c, _ = L.run_ex(to_dev(ref), [par, pard, par][i])
        assert_bits_equal(masks[i].cpu().numpy(), m.cpu().numpy(), "batch u16 mask %d" % i)
        assert_bits_equal(cleans[i].cpu().numpy(), c.cpu().numpy(), "batch u16 clean %d" % i)
    # estimated gain on a uint16 frame
    mu, cu, stu = L.run_ex(u, _params(pc))
    r = _oracle_est(cm, pc)
    _check(cm, pc, r, mu.cpu().numpy(), cu.cpu().numpy(), stu, "u16 estimated")
