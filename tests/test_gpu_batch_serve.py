"""GPU tests of the batched and serving layers.

Every frame a batch or the server returns must be bit-identical to the same
frame run alone through lacosmic_run_ex (which the parity tests pin to the
oracle), whatever else shares its launches; a sample is also checked against
the oracle directly.
"""

import time

import numpy as np
import pytest

from gpu_common import assert_bits_equal, crop_windows, lac, oracle_run, to_dev

pytestmark = pytest.mark.gpu

F32 = np.float32


def _frame(kind, h, w, seed):
    from paper_2602_17938_amd import synth
    return synth.make_frame(kind, h, w, seed)


def _params(kind, niter=4, early=False):
    from paper_2602_17938_amd import synth
    fp = synth.params_for(kind)
    return lac().make_params(fp.gain, fp.readnoise, fp.sigclip, fp.sigfrac, fp.objlim, niter,
                             early)


def _lone(img, params):
    m, c, _ = lac().run_ex(to_dev(img), params)
    return m.cpu().numpy(), c.cpu().numpy()


MIX = [("ccd", 512, 512, 11), ("ccd", 300, 700, 12), ("cmos", 1000, 257, 13),
       ("ccd", 64, 64, 14), ("ccd", 1, 1, 15), ("cmos", 17, 129, 16), ("ccd", 777, 1025, 17)]


def test_batch_matches_lone_runs_and_oracle():
    L = lac()
    imgs = [_frame(*s) for s in MIX]
    params = [_params(s[0]) for s in MIX]
    masks, cleans = L.run_batch([to_dev(x) for x in imgs], params)
    for i, (img, p) in enumerate(zip(imgs, params)):
        m, c = _lone(img, p)
        assert_bits_equal(masks[i].cpu().numpy(), m, "batch mask frame %d" % i)
        assert_bits_equal(cleans[i].cpu().numpy(), c, "batch clean frame %d" % i)
    assert L.lib().lacosmic_batch_tile_shape() in range(len(L.tile_shapes()))
    from paper_2602_17938_amd.synth import params_for
    for i in (0, 2, 5):
        r = oracle_run(imgs[i], params_for(MIX[i][0]))
        assert_bits_equal(masks[i].cpu().numpy(), r["mask"], "oracle mask frame %d" % i)
        assert_bits_equal(cleans[i].cpu().numpy(), r["clean"], "oracle clean frame %d" % i)


def test_batch_replay_new_buffers_and_order():
    """Second call with the same shapes replays the recorded graph with new
    buffers; a shuffled order records a new one.  Same results each time."""
    L = lac()
    rng = np.random.default_rng(5)
    specs = MIX[:5]
    lone = {}
    for rep in range(3):
        order = list(range(len(specs))) if rep < 2 else list(rng.permutation(len(specs)))
        imgs = [_frame(specs[i][0], specs[i][1], specs[i][2], specs[i][3] + 100 * rep)
                for i in order]
        params = [_params(specs[i][0]) for i in order]
        masks, cleans = L.run_batch([to_dev(x) for x in imgs], params)
        for j, i in enumerate(order):
            key = (rep, i)
            lone[key] = _lone(imgs[j], params[j])
            assert_bits_equal(masks[j].cpu().numpy(), lone[key][0], "rep %d frame %d" % (rep, i))
            assert_bits_equal(cleans[j].cpu().numpy(), lone[key][1], "rep %d frame %d" % (rep, i))


@pytest.mark.parametrize("groups", [2, 3])
def test_batch_frame_groups_match_lone_runs(groups, monkeypatch):
    """Frames split into concurrent groups (pinned, on batch shapes no other
    test uses, so a new plan is built): the plan reports the group count and
    every frame is bit-identical to its lone run."""
    L = lac()
    monkeypatch.setenv("LACOSMIC_BATCH_GROUPS", str(groups))
    specs = [("ccd", 230 + 7 * groups, 310, 40), ("cmos", 400, 190 + groups, 41),
             ("ccd", 96, 96, 42), ("ccd", 600, 520, 43), ("cmos", 33, 77, 44),
             ("ccd", 1, 5, 45), ("ccd", 257, 129, 46)]
    imgs = [_frame(*sp) for sp in specs]
    params = [_params(sp[0]) for sp in specs]
    masks, cleans = L.run_batch([to_dev(x) for x in imgs], params)
    assert L.lib().lacosmic_batch_groups() == groups
    for i, (img, p) in enumerate(zip(imgs, params)):
        m, c = _lone(img, p)
        assert_bits_equal(masks[i].cpu().numpy(), m, "groups %d mask frame %d" % (groups, i))
        assert_bits_equal(cleans[i].cpu().numpy(), c, "groups %d clean frame %d" % (groups, i))


@pytest.mark.parametrize("cfg", [0, 1, 2])
@pytest.mark.parametrize("groups", [1, 3])
def test_batch_persistent_queue_plan(cfg, groups, monkeypatch):
    """The persistent tile-queue launch form, pinned for each tile shape
    (LACOSMIC_BATCH_PLAN=cfg,0,groups on a batch shape no other test uses, so
    a new plan is built): every frame bit-identical to its lone run."""
    L = lac()
    monkeypatch.setenv("LACOSMIC_BATCH_PLAN", "%d,0,%d" % (cfg, groups))
    specs = [("ccd", 260 + 10 * cfg + groups, 330, 60), ("cmos", 420, 170 + 3 * cfg, 61),
             ("ccd", 64, 96 + groups, 62), ("ccd", 700, 515, 63), ("cmos", 31, 70, 64),
             ("ccd", 1, 3, 65), ("ccd", 129, 257, 66)]
    imgs = [_frame(*sp) for sp in specs]
    params = [_params(sp[0]) for sp in specs]
    masks, cleans = L.run_batch([to_dev(x) for x in imgs], params)
    assert L.lib().lacosmic_batch_launch_mode() == 0
    assert L.lib().lacosmic_batch_tile_shape() == cfg
    assert L.lib().lacosmic_batch_groups() == groups
    for i, (img, p) in enumerate(zip(imgs, params)):
        m, c = _lone(img, p)
        assert_bits_equal(masks[i].cpu().numpy(), m, "queue cfg %d mask frame %d" % (cfg, i))
        assert_bits_equal(cleans[i].cpu().numpy(), c, "queue cfg %d clean frame %d" % (cfg, i))


def test_batch_async_calls_on_two_streams():
    """Two asynchronous batches of the same shape on different streams share
    the cached plan (frame table, workspaces): the second waits for the
    first, and each result equals its frames' lone runs."""
    import torch
    L = lac()
    specs = [("ccd", 333, 444, 70), ("cmos", 500, 300, 71), ("ccd", 90, 90, 72)]
    sets = []
    for rep in range(2):
        imgs = [_frame(k, h, w, seed + 10 * rep) for k, h, w, seed in specs]
        sets.append(imgs)
    params = [_params(sp[0]) for sp in specs]
    L.run_batch([to_dev(x) for x in sets[0]], params)  # plan built and tuned
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    dev = [[to_dev(x) for x in imgs] for imgs in sets]
    torch.cuda.synchronize()
    outs = []
    for rep in range(2):
        outs.append(L.run_batch(dev[rep], params, stream=streams[rep]))
    for st in streams:
        st.synchronize()
    for rep in range(2):
        for i, (img, p) in enumerate(zip(sets[rep], params)):
            m, c = _lone(img, p)
            assert_bits_equal(outs[rep][0][i].cpu().numpy(), m, "stream %d mask %d" % (rep, i))
            assert_bits_equal(outs[rep][1][i].cpu().numpy(), c, "stream %d clean %d" % (rep, i))


def test_batch_early_stop_and_async_stream():
    import torch
    L = lac()
    imgs = [_frame(*s) for s in MIX[:4]]
    full = L.run_batch([to_dev(x) for x in imgs], [_params(s[0], niter=6) for s in MIX[:4]])
    s = torch.cuda.Stream()
    es = L.run_batch([to_dev(x) for x in imgs],
                     [_params(sp[0], niter=6, early=True) for sp in MIX[:4]], stream=s)
    s.synchronize()
    for i in range(4):
        assert torch.equal(full[0][i], es[0][i])
        assert torch.equal(full[1][i].view(torch.int32), es[1][i].view(torch.int32))


def test_batch_rejects_nonfinite_frame():
    L = lac()
    a = _frame("ccd", 100, 100, 1)
    b = _frame("ccd", 80, 130, 2)
    b[40, 60] = np.nan
    with pytest.raises(L.LacosmicError) as e:
        L.run_batch([to_dev(a), to_dev(b)], [_params("ccd")] * 2, stream=None)
    assert e.value.status == L.ENONFINITE


def test_full_mixed_batch_workload():
    """The 64-frame mixed batch (32 x 2048^2, 24 x 4096^2, 8 x 6400 x 9600
    CMOS) in one batched call: every frame bit-identical to its lone run;
    one frame of each size checked against the oracle on sampled crops."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from paper_2602_17938_amd import synth
    L = lac()
    specs = synth.batch_specs()
    with ThreadPoolExecutor(4) as ex:
        imgs = list(ex.map(lambda s: synth.make_frame(s[0], s[1], s[2], s[3], threads=4), specs))
    print("generated %d frames" % len(imgs), flush=True)
    params = [_params(s[0]) for s in specs]
    dev = [to_dev(x) for x in imgs]
    masks, cleans = L.run_batch(dev, params)
    torch.cuda.synchronize()
    for i in range(len(specs)):
        m, c, _ = L.run_ex(dev[i], params[i])
        assert torch.equal(masks[i], m), "frame %d mask" % i
        assert torch.equal(cleans[i].view(torch.int32), c.view(torch.int32)), "frame %d" % i
    print("all %d frames identical to lone runs" % len(specs), flush=True)
    for i in (0, 32, 56):
        kind, h, w, _ = specs[i]
        fp = synth.params_for(kind)
        mk, cl = masks[i].cpu().numpy(), cleans[i].cpu().numpy()
        for (y0, y1, x0, x1), (oy0, oy1, ox0, ox1) in crop_windows(h, w, 192, fp.niter)[::4]:
            r = oracle_run(np.ascontiguousarray(imgs[i][oy0:oy1, ox0:ox1]), fp)
            sl = (slice(y0 - oy0, y1 - oy0), slice(x0 - ox0, x1 - ox0))
            assert_bits_equal(mk[y0:y1, x0:x1], r["mask"][sl], "frame %d crop mask" % i)
            assert_bits_equal(cl[y0:y1, x0:x1], r["clean"][sl], "frame %d crop clean" % i)


# ------------------------------------------------------------------ serving
def _serve(frames, params, budget, max_frames=16, arrival_gap=0.0):
    L = lac()
    out = {}
    with L.Server(budget, max_frames) as srv:
        tickets = []
        for img, p in zip(frames, params):
            tickets.append(srv.submit(img, p))
            if arrival_gap:
                time.sleep(arrival_gap)
        t0 = time.time()
        while len(out) < len(tickets):
            for i, t in enumerate(tickets):
                if i in out:
                    continue
                r = srv.poll(t)
                if r is not None:
                    out[i] = r
            assert time.time() - t0 < 120, "server did not finish"
            time.sleep(0.001)
    return [out[i] for i in range(len(frames))]


def test_server_alone_and_in_the_mix():
    from paper_2602_17938_amd import synth
    specs = [("ccd", 512, 512, 21), ("cmos", 640, 960, 22), ("ccd", 1024, 1024, 23),
             ("cmos", 333, 555, 24), ("ccd", 2048, 2048, 25), ("ccd", 96, 200, 26)]
    frames, params, lone = [], [], []
    for kind, h, w, seed in specs:
        img = synth.make_frame(kind, h, w, seed)
        p = _params(kind)
        if kind == "cmos":
            frames.append(img.astype(np.uint16))  # exact: CMOS frames hold uint16 values
        else:
            frames.append(img)
        params.append(p)
        lone.append(_lone(img, p))
    mixed = _serve(frames, params, budget=8 << 30)
    for i, (m, c, ts, td) in enumerate(mixed):
        assert td >= ts
        assert_bits_equal(m, lone[i][0], "served mask %d" % i)
        assert_bits_equal(c, lone[i][1], "served clean %d" % i)
    alone = _serve([frames[2]], [params[2]], budget=8 << 30)
    assert_bits_equal(alone[0][0], mixed[2][0], "alone vs mix mask")
    assert_bits_equal(alone[0][1], mixed[2][1], "alone vs mix clean")


@pytest.mark.parametrize("pinned_mb", [0, 8])
def test_server_pageable_staging(pinned_mb, monkeypatch):
    """The server stages host data in a pinned pool and in pageable memory
    when the pool is full: with no pool, and with a pool that holds the small
    frames but not the large ones, results equal the lone runs (a frame over
    32 MB also takes the multi-threaded host copies)."""
    from paper_2602_17938_amd import synth
    monkeypatch.setenv("LACOSMIC_SERVER_PINNED_MB", str(pinned_mb))
    specs = [("ccd", 300, 200, 51), ("cmos", 1500, 1100, 52), ("ccd", 90, 70, 53),
             ("ccd", 1200, 1300, 54), ("ccd", 3000, 2900, 55)]  # the last: copies split over threads
    frames, params, lone = [], [], []
    for kind, h, w, seed in specs:
        img = synth.make_frame(kind, h, w, seed)
        p = _params(kind)
        frames.append(img.astype(np.uint16) if kind == "cmos" else img)
        params.append(p)
        lone.append(_lone(img, p))
    served = _serve(frames, params, budget=4 << 30)
    for i, (m, c, ts, td) in enumerate(served):
        assert_bits_equal(m, lone[i][0], "pinned %d MB: served mask %d" % (pinned_mb, i))
        assert_bits_equal(c, lone[i][1], "pinned %d MB: served clean %d" % (pinned_mb, i))


def test_server_budget_forces_queueing_and_rejects_oversize():
    from paper_2602_17938_amd import synth
    L = lac()
    frames = [synth.make_frame("ccd", 1024, 1024, 30 + i) for i in range(5)]
    params = [_params("ccd")] * 5
    one = 1024 * 1024 * 40  # room for about one such frame's device state
    res = _serve(frames, params, budget=one, max_frames=8)
    for i, (m, c, ts, td) in enumerate(res):
        lm, lc = _lone(frames[i], params[i])
        assert_bits_equal(m, lm, "queued mask %d" % i)
        assert_bits_equal(c, lc, "queued clean %d" % i)
    # one frame at a time: each finishes after the previous one
    dones = [r[3] for r in res]
    assert dones == sorted(dones)
    with L.Server(one, 4) as srv:
        with pytest.raises(L.LacosmicError) as e:
            srv.submit(synth.make_frame("ccd", 4096, 4096, 1), params[0])
        assert e.value.status == L.EBUDGET


def test_server_full_size_frames_host_and_device():
    """A 4096^2 frame and a 6400 x 9600 CMOS frame (uint16) through the
    server, from host memory and from device memory: each result equals the
    frame's lone run."""
    import torch
    from paper_2602_17938_amd import synth
    specs = [("ccd", 4096, 4096, 81), ("cmos", 6400, 9600, 82)]
    frames, params, lone = [], [], []
    for kind, h, w, seed in specs:
        img = synth.make_frame(kind, h, w, seed)
        p = _params(kind)
        frames.append(img.astype(np.uint16) if kind == "cmos" else img)
        params.append(p)
        lone.append(_lone(img, p))
    print("lone runs done", flush=True)
    dev_frames = [torch.from_numpy(f).cuda() for f in frames]
    torch.cuda.synchronize()
    served = _serve(frames + dev_frames, params + params, budget=16 << 30)
    for i, (m, c, ts, td) in enumerate(served):
        k = i % 2
        src = "host" if i < 2 else "device"
        assert_bits_equal(m, lone[k][0], "%s frame %d mask" % (src, k))
        assert_bits_equal(c, lone[k][1], "%s frame %d clean" % (src, k))


def test_server_reports_nonfinite_frame():
    L = lac()
    good = _frame("ccd", 200, 300, 1)
    bad = good.copy()
    bad[10, 10] = np.inf
    with L.Server(1 << 30, 4) as srv:
        tb = srv.submit(bad, _params("ccd"))
        tg = srv.submit(good, _params("ccd"))
        srv.drain()
        with pytest.raises(L.LacosmicError) as e:
            srv.poll(tb)
        assert e.value.status == L.ENONFINITE
        m, c, _, _ = srv.poll(tg)
    lm, lc = _lone(good, _params("ccd"))
    assert_bits_equal(m, lm, "good frame mask")
    assert_bits_equal(c, lc, "good frame clean")
