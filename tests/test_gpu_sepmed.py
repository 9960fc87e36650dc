"""GPU tests of the separable-median variant (LACOSMIC_F_SEPMED): every
detection median taken as row medians followed by column medians, the
comparison point the paper discusses.  Bit for bit against the oracle run in
the same mode, on both single-frame paths, in a batch, and on the 4096^2
frame; and it must differ from the classic median's result."""

import numpy as np
import pytest

from gpu_common import assert_bits_equal, host_threads, lac, to_dev

pytestmark = pytest.mark.gpu

F32 = np.float32


def _oracle(img, p, sepmed=True):
    import oracle
    return oracle.lacosmic(img, p.gain, p.readnoise, p.sigclip, p.sigfrac, p.objlim, p.niter,
                           nthreads=host_threads(), sepmed=sepmed)


def _params(p, sepmed=True):
    return lac().make_params(p.gain, p.readnoise, p.sigclip, p.sigfrac, p.objlim, p.niter,
                             sepmed=sepmed)


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("case", ["c0", "edges", "cmos"])
def test_sepmed_matches_oracle(case, fused, monkeypatch):
    from paper_2602_17938_amd import synth
    monkeypatch.setenv("LACOSMIC_FUSED_MAX_PX", str(1 << 30) if fused else "0")
    if case == "c0":
        img, p = synth.config_frame("c0")
    elif case == "edges":
        p = synth.params_for("ccd")
        img = synth.make_frame("ccd", 67, 131, 301)
        img[0, :] += 900.0  # structure along the borders
        img[:, -1] += 700.0
    else:
        p = synth.params_for("cmos")
        img = synth.make_frame("cmos", 333, 290, 302)
    r = _oracle(img, p)
    m, c, st = lac().run_ex(to_dev(img), _params(p))
    assert_bits_equal(m.cpu().numpy(), r["mask"], case + " mask")
    assert_bits_equal(c.cpu().numpy(), r["clean"], case + " clean")
    assert [st.n_new[k] for k in range(p.niter)] == list(r["n_new"])
    if case == "c0":
        full = _oracle(img, p, sepmed=False)
        assert (r["mask"] != full["mask"]).any()


def test_sepmed_in_a_batch_with_classic_frames():
    from paper_2602_17938_amd import synth
    L = lac()
    specs = [("ccd", 512, 512, 311, True), ("ccd", 700, 500, 312, False),
             ("cmos", 400, 380, 313, True), ("ccd", 90, 200, 314, False)]
    imgs = [synth.make_frame(k, h, w, s) for k, h, w, s, _ in specs]
    ps = [synth.params_for(k) for k, _, _, _, _ in specs]
    params = [_params(p, sep) for p, (_, _, _, _, sep) in zip(ps, specs)]
    masks, cleans = L.run_batch([to_dev(x) for x in imgs], params)
    for i, (img, p, q) in enumerate(zip(imgs, ps, params)):
        m, c, _ = L.run_ex(to_dev(img), q)
        assert_bits_equal(masks[i].cpu().numpy(), m.cpu().numpy(), "batch mask %d" % i)
        assert_bits_equal(cleans[i].cpu().numpy(), c.cpu().numpy(), "batch clean %d" % i)
    r = _oracle(imgs[2], ps[2])
    assert_bits_equal(masks[2].cpu().numpy(), r["mask"], "batch vs oracle mask")


def test_sepmed_c1_full_frame():
    from paper_2602_17938_amd import synth
    img, p = synth.config_frame("c1")
    m, c, st = lac().run_ex(to_dev(img), _params(p))
    print("gpu done", flush=True)
    r = _oracle(img, p)
    assert_bits_equal(m.cpu().numpy(), r["mask"], "mask")
    assert_bits_equal(c.cpu().numpy(), r["clean"], "clean")
