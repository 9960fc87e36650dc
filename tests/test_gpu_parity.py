"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Masks, S' planes and candidate maps are compared bit for bit; cleaned images
bit for bit as well (the method only selects existing values there, so the
1e-6 relative tolerance the workload allows is never needed).
"""

import numpy as np
import pytest

from gpu_common import assert_bits_equal, gpu_run, lac, oracle_run, to_dev

pytestmark = pytest.mark.gpu

F32 = np.float32
DEFAULT_TILE_CFG = 1  # 32 x 64, the single-frame path's default (and the benchmarked) shape


@pytest.fixture(scope="module")
def synth():
    from paper_2602_17938_amd import synth
    return synth


def _frame_with_features(h, w, seed):
    """Small frames: Poisson sky with hot pixels, CR pixels and a short track
    at random places, including the borders."""
    g = np.random.Generator(np.random.PCG64(seed))
    img = (g.poisson(200.0, size=(h, w)) + g.normal(0, 5.0, size=(h, w))).astype(F32)
    n = max(1, (h * w) // 40)
    ys = g.integers(0, h, size=n)
    xs = g.integers(0, w, size=n)
    img[ys, xs] += g.uniform(300, 20000, size=n).astype(F32)
    if h > 4 and w > 4:
        img[0, 0] += 5000
        img[h - 1, w - 1] += 4000
        img[h // 2, :min(w, 6)] += 3000
    return img


def test_c0_full_parity(synth, single_path):
    img, p = synth.config_frame("c0")
    r = oracle_run(img, p)
    m, c, st = gpu_run(img, p)
    assert_bits_equal(m, r["mask"], "mask")
    assert_bits_equal(c, r["clean"], "clean")
    assert st.iters_run == p.niter
    assert [st.n_new[k] for k in range(p.niter)] == list(r["n_new"])
    assert st.n_flagged == int(r["mask"].sum())
    assert st.n_unreplaced == r["n_unreplaced"]


def _dense_hot_field(h, w, density, seed):
    """Sky with hot pixels on a given fraction of the pixels: the mask grows
    over the iterations into blocks whose 5x5 windows hold no un-flagged cell."""
    g = np.random.Generator(np.random.PCG64(seed))
    img = (g.poisson(200.0, size=(h, w)) + g.normal(0, 5.0, size=(h, w))).astype(F32)
    hot = g.random((h, w)) < density
    img[hot] += g.uniform(300, 20000, size=int(hot.sum())).astype(F32)
    return img


@pytest.mark.parametrize("density,objlim,sigfrac,niter,early",
                         [(0.9, 5.0, 0.3, 4, False), (0.97, 0.0, 0.05, 6, False),
                          (0.8, 0.0, 0.05, 6, True)])
def test_unreplaced_pixels_counted(density, objlim, sigfrac, niter, early, single_path):
    """Step 7 leaves a flagged pixel whose window has no un-flagged cell
    unchanged; the statistics count those of the final mask, as the oracle
    does.  Dense hot-pixel blocks inside an ordinary frame (edges included)."""
    from paper_2602_17938_amd.synth import FrameParams
    p = FrameParams(gain=1.0, readnoise=5.0, sigclip=4.5, sigfrac=sigfrac, objlim=objlim,
                    niter=niter)
    img = _frame_with_features(150, 230, seed=int(density * 1000) + niter)
    img[0:64, 0:80] = _dense_hot_field(64, 80, density, seed=3)
    img[70:134, 120:200] = _dense_hot_field(64, 80, density, seed=4)
    r = oracle_run(img, p, early_stop=early)
    assert r["n_unreplaced"] > 0
    m, c, st = gpu_run(img, p, early_stop=early)
    assert_bits_equal(m, r["mask"], "mask")
    assert_bits_equal(c, r["clean"], "clean")
    assert st.iters_run == r["iters_run"]
    assert [st.n_new[k] for k in range(st.iters_run)] == list(r["n_new"])
    assert st.n_unreplaced == r["n_unreplaced"]


@pytest.mark.parametrize("full_sp", [True, False])
def test_c0_per_iteration_planes(synth, full_sp):
    """S at every pixel (kept up to date near rewritten pixels after
    iteration 0), S' (whole plane with the full-S' flag, at the candidates
    otherwise) and the candidate map after each iteration, bit for bit."""
    import torch
    L = lac()
    img, p = synth.config_frame("c0")
    r = oracle_run(img, p, trace=True)
    h, w = img.shape
    ws = L.alloc_workspace(h, w)
    for k in range(1, p.niter + 1):
        m, c, st = gpu_run(img, p, niter=k, workspace=ws, full_sp=full_sp)
        torch.cuda.synchronize()
        S, sp, cand = L.workspace_planes(ws, h, w)
        assert_bits_equal(S, r["trace_s"][k - 1], "S iter %d" % k)
        ref = r["trace_sp"][k - 1]
        if full_sp:
            assert_bits_equal(sp, ref, "S' iter %d" % k)
        else:
            at = ref > p.sigclip
            assert at.sum() > 100
            assert_bits_equal(sp[at], ref[at], "S' at candidates iter %d" % k)
        assert_bits_equal(cand, r["trace_b1"][k - 1], "cand iter %d" % k)
        assert_bits_equal(m, r["trace_mask"][k - 1], "mask iter %d" % k)
        assert_bits_equal(c, r["trace_clean"][k - 1], "clean iter %d" % k)


@pytest.mark.parametrize("sigclip,sigfrac,objlim", [(4.5, 0.3, 5.0), (3.0, 1.5, 2.0),
                                                    (4.5, 0.05, 0.0), (6.0, 0.9, 1.0),
                                                    (2.0, 0.5, 8.0)])
def test_parameter_variants(sigclip, sigfrac, objlim, single_path):
    """Thresholds on both sides of each other (sigfrac > 1 puts the growth
    threshold above sigclip), objlim 0 (no rejection) and large; 6
    iterations so the later, incremental iterations have work."""
    from paper_2602_17938_amd.synth import FrameParams, params_for
    base = params_for("ccd")
    p = FrameParams(gain=base.gain, readnoise=base.readnoise, sigclip=sigclip, sigfrac=sigfrac,
                    objlim=objlim, niter=6)
    img = _frame_with_features(300, 260, seed=int(sigclip * 100 + sigfrac * 10 + objlim))
    r = oracle_run(img, p)
    m, c, st = gpu_run(img, p)
    assert_bits_equal(m, r["mask"], "mask")
    assert_bits_equal(c, r["clean"], "clean")
    assert [st.n_new[k] for k in range(p.niter)] == list(r["n_new"])


@pytest.mark.parametrize("gain", [0.3, 1.7, 3.0, 0.5, 2.0, 8.0, 2.0 ** -20])
def test_gain_values(gain):
    """The noise model divides by the gain; for a power-of-two gain the kernels
    multiply by its exact reciprocal instead.  Both forms against the oracle,
    single frame and in one batch with a frame of another gain."""
    from paper_2602_17938_amd.synth import FrameParams
    L = lac()
    p = FrameParams(gain=gain, readnoise=5.0, niter=4)
    img = (_frame_with_features(210, 230, seed=int(1e6 * gain) % 100003) / F32(gain)).astype(F32)
    r = oracle_run(img, p)
    m, c, st = gpu_run(img, p)
    assert_bits_equal(m, r["mask"], "mask gain %g" % gain)
    assert_bits_equal(c, r["clean"], "clean gain %g" % gain)
    assert [st.n_new[k] for k in range(p.niter)] == list(r["n_new"])
    other = FrameParams(gain=1.3 if gain != 1.3 else 0.7, readnoise=2.0, niter=4)
    img2 = (_frame_with_features(90, 140, seed=7) / F32(other.gain)).astype(F32)
    r2 = oracle_run(img2, other)
    params = [L.make_params(q.gain, q.readnoise, q.sigclip, q.sigfrac, q.objlim, q.niter)
              for q in (p, other)]
    masks, cleans = L.run_batch([to_dev(img), to_dev(img2)], params)
    assert_bits_equal(masks[0].cpu().numpy(), r["mask"], "batch mask gain %g" % gain)
    assert_bits_equal(cleans[0].cpu().numpy(), r["clean"], "batch clean gain %g" % gain)
    assert_bits_equal(masks[1].cpu().numpy(), r2["mask"], "batch mask gain %g" % other.gain)
    assert_bits_equal(cleans[1].cpu().numpy(), r2["clean"], "batch clean gain %g" % other.gain)


def test_fast_sqrt_matches_sqrtf_on_its_whole_range():
    """The noise model's square root for variances >= 2^-96 agrees with the
    correctly rounded sqrtf on every binary32 input from 2^-96 to +inf."""
    import ctypes
    n = ctypes.c_uint64(12345)
    assert lac().lib().lacosmic_check_sqrt(0x0F800000, 0x7F800000, ctypes.byref(n)) == 0
    assert n.value == 0


SMALL = [(1, 1), (1, 9), (9, 1), (2, 2), (5, 3), (3, 70), (17, 65), (33, 129), (67, 131),
         (100, 257), (130, 63)]


@pytest.fixture(params=["fused", "sparse"])
def single_path(request, monkeypatch):
    """Small frames run the fused launches by default; the sparse passes are
    forced by setting the fused path's pixel limit to 0."""
    if request.param == "sparse":
        monkeypatch.setenv("LACOSMIC_FUSED_MAX_PX", "0")
    else:
        monkeypatch.setenv("LACOSMIC_FUSED_MAX_PX", str(1 << 30))
    return request.param


@pytest.mark.parametrize("shape", SMALL)
def test_small_and_ragged_shapes(shape, single_path):
    from paper_2602_17938_amd.synth import params_for
    p = params_for("ccd")
    img = _frame_with_features(*shape, seed=shape[0] * 1000 + shape[1])
    r = oracle_run(img, p, trace=True)
    m, c, st = gpu_run(img, p)
    assert_bits_equal(m, r["mask"], "mask %s" % (shape,))
    assert_bits_equal(c, r["clean"], "clean %s" % (shape,))


@pytest.mark.parametrize("shape,scale", [((1024, 1024), 8.0), ((700, 900), 25.0)])
def test_dense_cosmic_rays(shape, scale, single_path):
    """Eight and 25 times the workload's cosmic-ray density: far longer
    candidate, confirmed and replacement lists in every iteration."""
    from paper_2602_17938_amd import synth
    p = synth.params_for("ccd")
    img = synth.make_frame("ccd", *shape, seed=int(scale) + 40, cr_scale=scale)
    r = oracle_run(img, p)
    m, c, st = gpu_run(img, p)
    assert_bits_equal(m, r["mask"], "mask")
    assert_bits_equal(c, r["clean"], "clean")
    assert [st.n_new[k] for k in range(p.niter)] == list(r["n_new"])
    assert st.n_unreplaced == r["n_unreplaced"]


# Row widths around the strip-column geometry of the bit-plane passes: rows of
# up to 64 words are one column (a lane per word), wider rows columns of 62
# words with a one-word halo each side.
WIDE = [(40, 3968), (37, 4032), (33, 4096), (35, 4097), (41, 4160), (29, 7937), (18, 8000)]


def _frame_across_columns(h, w, seed):
    """A feature frame with cosmic-ray hits and short tracks placed across
    the 62- and 64-word column boundaries and the strip boundary rows."""
    img = _frame_with_features(h, w, seed)
    for x in (62 * 64 - 1, 62 * 64, 64 * 64 - 1, 64 * 64, 124 * 64 - 1, 124 * 64, w - 1):
        if x < w:
            for y in (0, 7, 15, 16, h - 1):
                if y < h:
                    img[y, x] += 6000.0
            y = min(h - 1, 16)
            img[y, max(0, x - 2):min(w, x + 3)] += 2500.0  # a track across the boundary
    return img


@pytest.mark.parametrize("shape", WIDE)
def test_wide_rows_at_strip_column_boundaries(shape, single_path):
    from paper_2602_17938_amd.synth import params_for
    p = params_for("ccd")
    img = _frame_across_columns(*shape, seed=shape[0] * 7919 + shape[1])
    r = oracle_run(img, p)
    m, c, st = gpu_run(img, p)
    assert_bits_equal(m, r["mask"], "mask %s" % (shape,))
    assert_bits_equal(c, r["clean"], "clean %s" % (shape,))
    assert [st.n_new[k] for k in range(p.niter)] == list(r["n_new"])


def test_wide_rows_in_a_batch():
    """The same widths batched together (each frame its own column layout in
    one launch) give each frame's lone result."""
    from paper_2602_17938_amd.synth import params_for
    L = lac()
    p = params_for("ccd")
    imgs = [_frame_across_columns(*s, seed=s[0] * 7919 + s[1]) for s in WIDE]
    params = [L.make_params(p.gain, p.readnoise, p.sigclip, p.sigfrac, p.objlim, p.niter)] * len(WIDE)
    masks, cleans = L.run_batch([to_dev(x) for x in imgs], params)
    for i, img in enumerate(imgs):
        r = oracle_run(img, p)
        assert_bits_equal(masks[i].cpu().numpy(), r["mask"], "batch mask %s" % (WIDE[i],))
        assert_bits_equal(cleans[i].cpu().numpy(), r["clean"], "batch clean %s" % (WIDE[i],))


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_tile_shapes_give_identical_results(cfg):
    from paper_2602_17938_amd.synth import params_for
    L = lac()
    p = params_for("ccd")
    img = _frame_with_features(150, 300, seed=77)
    r = oracle_run(img, p)
    L.set_tile_shape(cfg)
    try:
        m, c, _ = gpu_run(img, p)
    finally:
        L.set_tile_shape(DEFAULT_TILE_CFG)  # later tests run the default shape
    assert_bits_equal(m, r["mask"], "mask cfg %d" % cfg)
    assert_bits_equal(c, r["clean"], "clean cfg %d" % cfg)


@pytest.mark.parametrize("case", ["hot_interior", "hot_edge", "hot_corner", "pair", "track45",
                                  "growth", "star", "constant"])
def test_hand_built_frames(case):
    from paper_2602_17938_amd.synth import FrameParams
    p = FrameParams(gain=1.0, readnoise=5.0)
    img = np.full((40, 70), 200.0, F32)
    if case == "hot_interior":
        img[20, 30] = 268.0
        img[10, 10] = 267.0
    elif case == "hot_edge":
        img[0, 30] = 300.0
        img[39, 50] = 1000.0
    elif case == "hot_corner":
        img[0, 0] = 400.0
        img[39, 69] = 336.0
    elif case == "pair":
        img[20, 30] = 5000.0
        img[20, 31] = 7000.0
    elif case == "track45":
        for s in range(7):
            img[10 + s, 20 + s] = 3000.0
    elif case == "growth":
        img[20, 30] = 5000.0
        img[20, 31] = 260.0
    elif case == "star":
        y, x = np.mgrid[0:40, 0:70]
        s = 3.0 / 2.3548
        img = (img + 2e4 * np.exp(-((y - 20) ** 2 + (x - 35) ** 2) / (2 * s * s))).astype(F32)
    r = oracle_run(img, p)
    m, c, _ = gpu_run(img, p)
    assert_bits_equal(m, r["mask"], "mask " + case)
    assert_bits_equal(c, r["clean"], "clean " + case)


def test_step_image_golden():
    from golden_io import read_pipeline
    from paper_2602_17938_amd.synth import FrameParams
    g = read_pipeline("step_pipeline.txt")
    p = FrameParams(gain=g["gain"], readnoise=g["readnoise"], sigclip=g["sigclip"],
                    sigfrac=g["sigfrac"], objlim=g["objlim"], niter=int(g["niter"]))
    m, c, st = gpu_run(g["grids"]["input"].astype(F32), p)
    assert np.array_equal(m, g["grids"]["mask"].astype(np.uint8))
    assert np.array_equal(c, g["grids"]["clean"].astype(F32))
    assert [st.n_new[k] for k in range(4)] == g["n_new"]


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_nonfinite_input_rejected(bad):
    from paper_2602_17938_amd.synth import FrameParams
    L = lac()
    img = np.full((30, 90), 100.0, F32)
    img[29, 89] = bad
    with pytest.raises(L.LacosmicError) as e:
        gpu_run(img, FrameParams(gain=1.0, readnoise=5.0))
    assert e.value.status == L.ENONFINITE
    # the library stays usable afterwards
    img[29, 89] = 100.0
    m, c, _ = gpu_run(img, FrameParams(gain=1.0, readnoise=5.0))
    assert not m.any()


def test_negative_zero_is_canonicalised():
    from paper_2602_17938_amd.synth import FrameParams
    img = np.full((20, 20), -0.0, F32)
    img[5:8, 5:8] = 0.0
    img[10, 10] = 1000.0
    p = FrameParams(gain=1.0, readnoise=1.0)
    r = oracle_run(img, p)
    m, c, _ = gpu_run(img, p)
    assert_bits_equal(m, r["mask"], "mask")
    assert_bits_equal(c, r["clean"], "clean")
    assert not np.signbit(c).any()


def test_values_near_the_binary32_maximum(single_path):
    """Values from 2^125 up (finite, and four times them still below the
    binary32 maximum, so every Laplacian sum stays finite), next to an
    ordinary sky: 4c and the sums are large but exact where the oracle's are,
    and the results are the oracle's."""
    from paper_2602_17938_amd.synth import FrameParams
    g = np.random.Generator(np.random.PCG64(17))
    img = _frame_with_features(300, 260, seed=13)
    blk = (5e37 + g.normal(0, 1e35, size=(120, 90))).astype(F32)
    blk[::17, ::13] += np.float32(1e37)
    img[60:180, 100:190] = blk
    assert float(np.abs(img).max()) < 2.0 ** 126 and float(np.abs(img).max()) >= 2.0 ** 125
    p = FrameParams(gain=1.0, readnoise=5.0)
    r = oracle_run(img, p)
    m, c, _ = gpu_run(img, p)
    assert_bits_equal(m, r["mask"], "mask")
    assert_bits_equal(c, r["clean"], "clean")


def test_early_stop_matches_full_run(synth):
    import torch
    L = lac()
    img, p = synth.config_frame("c0")
    d = to_dev(img)
    m1, c1 = L.run(d, p.gain, p.readnoise, p.sigclip, p.sigfrac, p.objlim, 8)
    params = L.make_params(p.gain, p.readnoise, p.sigclip, p.sigfrac, p.objlim, 8)
    m2, c2, st = L.run_ex(d, params)
    assert torch.equal(m1, m2)
    assert torch.equal(c1.view(torch.int32), c2.view(torch.int32))
    params_es = L.make_params(p.gain, p.readnoise, p.sigclip, p.sigfrac, p.objlim, 8, True)
    _, _, st_es = L.run_ex(d, params_es)
    assert st_es.iters_run < 8
    assert st_es.n_flagged == st.n_flagged


def test_async_stream_and_determinism(synth):
    import torch
    L = lac()
    img, p = synth.config_frame("c0")
    d = to_dev(img)
    params = L.make_params(p.gain, p.readnoise, p.sigclip, p.sigfrac, p.objlim, p.niter)
    s = torch.cuda.Stream()
    outs = []
    for _ in range(3):
        m, c, st = L.run_ex(d, params, stream=s, stats=False)
        s.synchronize()
        outs.append((m.clone(), c.clone()))
    m0, c0, _ = L.run_ex(d, params)
    for m, c in outs:
        assert torch.equal(m, m0)
        assert torch.equal(c.view(torch.int32), c0.view(torch.int32))


def test_inputs_from_pending_default_stream_work(synth):
    """An input produced by torch on its default stream (the legacy null
    stream) right before the call, behind a long queue of work, and outputs
    whose memory pending work still uses: the library stream orders itself
    after that work, so the results are those of the finished input."""
    import torch
    L = lac()
    img, p = synth.config_frame("c0")
    r = oracle_run(img, p)
    params = L.make_params(p.gain, p.readnoise, p.sigclip, p.sigfrac, p.objlim, p.niter)
    host = torch.from_numpy(img)
    for stream in ("current", None):
        torch.cuda.synchronize()
        a = torch.randn(2048, 2048, device="cuda")
        src = torch.zeros(img.shape, dtype=torch.float32, device="cuda")
        for _ in range(20):  # keep the default stream busy
            a = a @ a
            a = a / a.norm()
        d = src + host.cuda(non_blocking=True)  # the input: lands after the queue
        mask = torch.full(img.shape, 7, dtype=torch.uint8, device="cuda")
        clean = torch.full(img.shape, -1.0, dtype=torch.float32, device="cuda")
        assert torch.cuda.current_stream().cuda_stream == 0
        m, c, st = L.run_ex(d, params, mask, clean, stream=stream)
        assert_bits_equal(m.cpu().numpy(), r["mask"], "mask (stream %s)" % stream)
        assert_bits_equal(c.cpu().numpy(), r["clean"], "clean (stream %s)" % stream)
        del a


def test_frame_graph_replays_match_eager_launches(synth):
    """The single-frame path replays one recorded graph per workspace and
    shape: several replays with different inputs, parameters and outputs,
    with other device work and host synchronisation between them, each equal
    to the same call with every kernel launched eagerly."""
    import torch
    L = lac()
    from paper_2602_17938_amd.synth import FrameParams
    img0, p0 = synth.config_frame("c0")
    img1 = _frame_with_features(512, 512, seed=5)
    p1 = FrameParams(gain=0.5, readnoise=3.0, sigclip=4.0, sigfrac=0.4, objlim=3.0)
    cases = [(img0, p0), (img1, p1), (img0, p1), (img1, p0)]
    ref = []
    L.set_frame_graphs(False)
    for img, p in cases:
        m, c, st = gpu_run(img, p)
        ref.append((m, c, [st.n_new[k] for k in range(p.niter)]))
    L.set_frame_graphs(True)
    try:
        for rep in range(3):
            for k, (img, p) in enumerate(cases):
                x = torch.randn(1024, 1024, device="cuda")
                x = (x @ x).sum()  # unrelated device work between replays
                m, c, st = gpu_run(img, p)
                torch.cuda.synchronize()
                assert_bits_equal(m, ref[k][0], "replay %d case %d mask" % (rep, k))
                assert_bits_equal(c, ref[k][1], "replay %d case %d clean" % (rep, k))
                assert [st.n_new[j] for j in range(p.niter)] == ref[k][2]
    finally:
        L.set_frame_graphs(False)  # the default
    r = oracle_run(img1, p1)
    assert_bits_equal(ref[1][0], r["mask"], "eager mask vs oracle")


def test_c1_full_parity(synth):
    img, p = synth.config_frame("c1")
    m, c, st = gpu_run(img, p)
    r = oracle_run(img, p)
    assert_bits_equal(m, r["mask"], "mask")
    assert_bits_equal(c, r["clean"], "clean")
    assert [st.n_new[k] for k in range(p.niter)] == list(r["n_new"])


def test_c2_full_parity(synth):
    """The 6400 x 9600 uint16-ADU CMOS frame: mask and cleaned image bit for bit
    against the oracle on all 61.4 Mpx, with the per-iteration counts."""
    img, p = synth.config_frame("c2")
    m, c, st = gpu_run(img, p)
    print("gpu done", flush=True)
    r = oracle_run(img, p)
    print("oracle done", flush=True)
    assert_bits_equal(m, r["mask"], "mask")
    assert_bits_equal(c, r["clean"], "clean")
    assert [st.n_new[k] for k in range(p.niter)] == list(r["n_new"])
    assert st.n_unreplaced == r["n_unreplaced"]
    assert np.array_equal(c[m == 0], img[m == 0])
