#!/usr/bin/env python3
"""Benchmark: full 4-iteration L.A.Cosmic on one MI355X.

Headline workload: the 64-frame mixed batch (32 x 2048^2, 24 x 4096^2 and
8 x 6400 x 9600 CMOS frames stored as uint16 ADU; 1.028 Gpx; niter = 4,
sigclip 4.5, sigfrac 0.3, objlim 5; early stop off) through
lacosmic_run_batch -- one launch per pass over the tiles of a frame group
(the launch form, tile shape and group count the autotuner picked), the
niter loop replayed as a HIP graph.  A step is one batch call over all 64
frames with the inputs already resident in HBM, enqueued on a stream of its
own.  The same frames also go through the single-frame path one at a time
(the "plain" figure, asynchronous on the same stream), a Poisson-arrival
stream swept from 1 frame/s to saturation goes through the serving layer
(p50 / p99 frame latency per rate), the 512^2 frame and variants of the
4096^2 frame (a gain that is not a power of two, eight times the cosmic
rays) run alone on the single-frame path, and the CPU oracle is timed on a
bounded sample on the host cores.

Prints one JSON line.  --gpus N > 1 is not supported: one process drives one
GPU and frames shard across GPUs without any exchange.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mpix/s (full 4-iter L.A.Cosmic) batched vs plain on 1 GPU; p99 frame latency"

# MI355X (gfx950) vector ALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz,
# one 32-bit lane operation per lane per clock (non-packed).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0

# Algorithmic 32-bit lane operations per pixel of pass A1, the dense pass of
# iteration 0 that dominates the run (see the design notes for the
# derivation): selection-network min/max operations from the generated
# networks, the Laplacian, and the correctly rounded square root and division
# sequences: med25 over blocks of 4x2 outputs on 32-row tiles (578 / 8),
# of 2x2 outputs on shorter tiles (308 / 4) + Laplacian edge image (29) +
# noise model (floor on the median's key 1, mul, add, square root 9 -- the
# hardware estimate, two fma residuals, two compares, two selects, two ulp
# steps; valid as the frame's variance cannot fall below 2^-96 -- then / gain
# as one multiplication by its exact reciprocal, the gain of every benchmark
# frame being a power of two) + S (mul, division 11).
def a1_ops_per_pixel(tile_cfg):
    med = 578.0 / 8 if tile_cfg == 1 else 308.0 / 4  # cfg 1: 32 x 64 tiles
    return med + 29 + (1 + 1 + 1 + 9 + 1) + 12
# Algorithmic HBM bytes per pixel of A1: read C, write S and the initial
# cleaned image (4 + 4 + 4 bytes), write the candidate bit plane (1 / 8 byte).
A1_BYTES_PER_PIXEL = 12.0 + 1.0 / 8.0

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "a1_batch64_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2602_17938_amd", "csrc", n)
                  for n in ("lacosmic_tiles.h", "lacosmic_kernels.hip", "lacosmic_small.h",
                            "lacosmic_gain.h", "lacosmic_mem.h", "lacosmic_device.h",
                            "gen_median_net.py")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_sha():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def read_traffic(plan_key):
    """HBM bytes per launch of the dominant kernel (for the batch plan
    plan_key = "cfg,mode,groups") from the committed counter summary, or None
    when that plan was not measured or the kernel sources changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_sources_sha():
        return None
    try:
        return float(vals["plan %s: A1 hbm_bytes_per_launch" % plan_key])
    except (KeyError, ValueError):
        return None


def ensure_built():
    lib = os.path.join(ROOT, "paper_2602_17938_amd", "liblacosmic.so")
    if not os.path.exists(lib):
        from paper_2602_17938_amd import build
        build.build()


def make_batch(threads):
    from concurrent.futures import ThreadPoolExecutor
    from paper_2602_17938_amd import synth
    specs = synth.batch_specs()
    per = max(1, threads // 4)
    with ThreadPoolExecutor(4) as ex:
        imgs = list(ex.map(lambda s: synth.make_frame(s[0], s[1], s[2], s[3], threads=per),
                           specs))
    return specs, imgs


def host_threads():
    """Threads the host lets this process use: the CPUs in its affinity set,
    capped by OMP_NUM_THREADS when that is set (a shared host gives each GPU
    a share of its cores and says so there)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(img, p, threads):
    """The oracle as it stands, timed on the host: one 2048 x 2048 frame of the
    batch with every thread the host gives this process, and a 1024 x 1024
    crop of it with one thread."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    t = time.perf_counter()
    oracle.lacosmic(img, p.gain, p.readnoise, p.sigclip, p.sigfrac, p.objlim, p.niter,
                    nthreads=threads)
    dt = time.perf_counter() - t
    crop = np.ascontiguousarray(img[:1024, :1024])
    t = time.perf_counter()
    oracle.lacosmic(crop, p.gain, p.readnoise, p.sigclip, p.sigfrac, p.objlim, p.niter,
                    nthreads=1)
    dt1 = time.perf_counter() - t
    return {"value": round(img.size / dt / 1e6, 3), "unit": "Mpix/s", "cores": threads,
            "kind": "oracle", "value_1_thread": round(crop.size / dt1 / 1e6, 3),
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": "one 2048x2048 frame of the batch (4.19 Mpx, niter=4) on %d threads, "
                      "%.1f s; its 1024x1024 corner on 1 thread, %.1f s" % (threads, dt, dt1)}


def serve_pool(threads, per_size=8):
    """The serving pool: per_size frames of each of the three sizes (CMOS
    frames as uint16 ADU, the others float32), seeds 2000 + i."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from paper_2602_17938_amd import synth
    specs = synth.serve_pool_specs(per_size=per_size)
    per = max(1, threads // 4)

    def one(sp):
        kind, h, w, s = sp
        img = synth.make_frame(kind, h, w, s, threads=per)
        return (img.astype(np.uint16) if kind == "cmos" else img, kind)

    with ThreadPoolExecutor(4) as ex:
        return list(ex.map(one, specs))


def serve_run(L, pool, n_req, rate, budget, seed=7):
    """Poisson arrivals of frames drawn uniformly from the pool; returns
    latency percentiles and throughput."""
    import numpy as np
    from paper_2602_17938_amd import synth
    rng = np.random.default_rng(seed)
    pick = rng.integers(0, len(pool), size=n_req)
    arrivals = synth.poisson_arrivals(rate, n_req, seed=seed)
    params = {k: L.make_params(synth.params_for(k).gain, synth.params_for(k).readnoise)
              for k in ("ccd", "cmos")}
    lat, pix = [], 0
    with L.Server(budget, 256) as srv:
        t0 = time.perf_counter()
        outstanding = {}
        i = 0
        while i < n_req or outstanding:
            now = time.perf_counter() - t0
            while i < n_req and arrivals[i] <= now:
                img, kind = pool[pick[i]]
                outstanding[srv.submit(img, params[kind])] = img.size
                i += 1
            for t in list(outstanding):
                r = srv.poll(t, want_outputs=False)
                if r is not None:
                    lat.append((r[3] - r[2]) / 1e6)
                    pix += outstanding.pop(t)
            time.sleep(0.0005)
        wall = time.perf_counter() - t0
    lat = np.array(lat)
    return {"rate_hz": rate, "frames": n_req, "p50_ms": round(float(np.percentile(lat, 50)), 2),
            "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "mpix_s": round(pix / wall / 1e6, 1), "wall_s": round(wall, 2)}


def serve_sweep(L, pool, budget, time_budget_s=90.0):
    """Arrival rate 1, 2, 4, ... frames/s (at least 8 frames and 2 s of
    arrivals per rate) until the served throughput stops growing by 10 %
    or the time budget is spent."""
    sweep = []
    rate = 1.0
    t0 = time.perf_counter()
    while True:
        r = serve_run(L, pool, max(8, int(2 * rate)), rate, budget)
        log("serve", r)
        sweep.append(r)
        if len(sweep) > 1 and r["mpix_s"] < 1.1 * sweep[-2]["mpix_s"]:
            break
        if time.perf_counter() - t0 > time_budget_s or rate >= 4096:
            break
        rate *= 2
    return sweep


def per_config(L, synth, args):
    """Single-frame path on each configuration frame (inputs resident in HBM,
    mean over `steps` runs after `warmup`), and the CPU baseline: the oracle
    on the 512^2 frame at 1 thread and at the host share (16 threads at most)."""
    import torch
    import oracle
    oracle.build(force=False)
    threads = host_threads()
    out = {"metric": "Mpix/s per configuration, single-frame path", "unit": "Mpix/s",
           "niter": synth.NITER, "configs": {}}
    for name in ("c0", "c1", "c2"):
        img, fp = synth.config_frame(name, threads=threads)
        d = torch.from_numpy(img).cuda()
        params = L.make_params(fp.gain, fp.readnoise, niter=synth.NITER)
        m = torch.empty(img.shape, dtype=torch.uint8, device="cuda")
        c = torch.empty(img.shape, dtype=torch.float32, device="cuda")
        stream = torch.cuda.Stream()
        row = {"shape": list(img.shape)}
        for mode in ("graph", "eager"):  # the recorded run replayed, or every kernel launched (the default)
            L.set_frame_graphs(mode == "graph")
            torch.cuda.synchronize()
            for _ in range(max(1, args.warmup)):
                L.run_ex(d, params, m, c, stream=stream, stats=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                L.run_ex(d, params, m, c, stream=stream, stats=False)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            row["graph_ms" if mode == "graph" else "ms"] = round(dt * 1e3, 4)
            row["graph_mpix_s" if mode == "graph" else "mpix_s"] = round(img.size / dt / 1e6, 1)
            log("%s %s %s: %.4f ms, %.1f Mpix/s" % (name, img.shape, mode, dt * 1e3,
                                                    img.size / dt / 1e6))
        # the separable-median comparison variant: time, and mask pixels that
        # differ from the classic median's mask
        sp = L.make_params(fp.gain, fp.readnoise, niter=synth.NITER, sepmed=True)
        ms_, cs_ = torch.empty_like(m), torch.empty_like(c)
        for _ in range(max(1, args.warmup)):
            L.run_ex(d, sp, ms_, cs_, stream=stream, stats=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            L.run_ex(d, sp, ms_, cs_, stream=stream, stats=False)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        row["sepmed_ms"] = round(dt * 1e3, 4)
        row["sepmed_mask_px"] = int(ms_.sum().item())
        row["mask_px"] = int(m.sum().item())
        row["sepmed_mask_differ"] = int((ms_ != m).sum().item())
        log("%s sepmed: %.4f ms, %d mask px (classic %d, %d differ)" % (
            name, dt * 1e3, row["sepmed_mask_px"], row["mask_px"], row["sepmed_mask_differ"]))
        del ms_, cs_
        out["configs"][name] = row
        del d, m, c
    img, fp = synth.config_frame("c0")
    oc = {}
    for nt in (1, threads):
        t0 = time.perf_counter()
        oracle.lacosmic(img, fp.gain, fp.readnoise, fp.sigclip, fp.sigfrac, fp.objlim, fp.niter,
                        nthreads=nt)
        dt = time.perf_counter() - t0
        oc["threads_%d" % nt] = round(img.size / dt / 1e6, 3)
    out["cpu_baseline_c0"] = {"kind": "oracle", "mpix_s": oc}
    log("oracle c0: %s" % oc)
    return out


def workload_variants(L, synth, stream, threads, reps=20):
    """The 4096^2 frame through the single-frame path beside two variants the
    headline workload does not exercise: a gain that is not a power of two
    (the noise model divides instead of multiplying by an exact reciprocal)
    and eight times the cosmic-ray density (the sparse passes scale with the
    number of flagged pixels).  Inputs resident in HBM; mean of `reps` runs."""
    import torch
    fp = synth.params_for("ccd")
    base = synth.make_frame("ccd", 4096, 4096, 2, threads)
    dense = synth.make_frame("ccd", 4096, 4096, 2, threads, cr_scale=8.0)
    rows = {}
    for name, img, gain in (("c1", base, fp.gain), ("c1_gain_1.7", base, 1.7),
                            ("c1_cosmic_rays_x8", dense, fp.gain)):
        d = torch.from_numpy(img).cuda()
        prm = L.make_params(gain, fp.readnoise, niter=synth.NITER)
        m = torch.empty(img.shape, dtype=torch.uint8, device="cuda")
        c = torch.empty(img.shape, dtype=torch.float32, device="cuda")
        for _ in range(3):
            L.run_ex(d, prm, m, c, stream=stream, stats=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            L.run_ex(d, prm, m, c, stream=stream, stats=False)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        rows[name] = {"gain": gain, "ms": round(dt * 1e3, 4),
                      "mpix_s": round(img.size / dt / 1e6, 1), "mask_px": int(m.sum().item())}
        log("variant %s: %.4f ms, %.1f Mpix/s, %d mask px" % (name, dt * 1e3, img.size / dt / 1e6,
                                                            rows[name]["mask_px"]))
        del d, m, c
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--serve-one", action="store_true",
                    help="one serving rate (16 frames/s) instead of the sweep to saturation")
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--configs", action="store_true",
                    help="only the per-configuration table: the single-frame path on the "
                         "512^2, 4096^2 and 6400x9600 frames and the oracle on the 512^2 "
                         "frame at 1 and all host threads (one JSON line)")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="first copy this many GiB device-to-device (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: frames are independent and shard across GPUs "
              "without exchange; run one process per GPU instead.", file=sys.stderr)
        sys.exit(2)

    ensure_built()
    import numpy as np
    import torch
    from paper_2602_17938_amd import lacosmic as L
    from paper_2602_17938_amd import synth

    if args.calibrate_copy_gib > 0:
        # a fill kernel that writes N bytes, then a device copy kernel that
        # reads N bytes and writes N bytes
        n = int(args.calibrate_copy_gib * (1 << 30)) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read, %d bytes written" % (4 * n, 4 * n))
        del src, dst
        torch.cuda.empty_cache()

    if args.configs:
        print(json.dumps(per_config(L, synth, args)), flush=True)
        return

    threads = host_threads()
    t = time.perf_counter()
    specs, imgs = make_batch(threads)
    npx = sum(x.size for x in imgs)
    log("generated %d frames, %.1f Mpx, in %.1f s" % (len(imgs), npx / 1e6,
                                                     time.perf_counter() - t))
    dev = [torch.from_numpy(x).cuda() for x in imgs]
    params = [L.make_params(synth.params_for(s[0]).gain, synth.params_for(s[0]).readnoise,
                            niter=synth.NITER) for s in specs]
    masks = [torch.empty(x.shape, dtype=torch.uint8, device="cuda") for x in dev]
    cleans = [torch.empty(x.shape, dtype=torch.float32, device="cuda") for x in dev]
    torch.cuda.synchronize()

    # every call is enqueued on this stream (asynchronous: no host round trip
    # per step); the first call times the candidate plans and records the graph
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        L.run_batch(dev, params, masks, cleans, stream=stream)
    torch.cuda.synchronize()
    cfg = L.lib().lacosmic_batch_tile_shape()
    mode = L.lib().lacosmic_batch_launch_mode()
    groups = L.lib().lacosmic_batch_groups()
    log("batch tile shape: %s, launch mode %s, %d frame groups" %
        (L.tile_shapes()[cfg], ("queue", "grid")[mode], groups))

    # timed region: K batch calls (graph replays) on that stream, bracketed
    # by device synchronisation, with HIP events on the stream between steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        L.run_batch(dev, params, masks, cleans, stream=stream)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed / args.steps * 1e3
    step_ms = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps))
    gpu_ms_step = sum(step_ms) / args.steps
    median_ms = step_ms[len(step_ms) // 2] if len(step_ms) % 2 else \
        0.5 * (step_ms[len(step_ms) // 2 - 1] + step_ms[len(step_ms) // 2])
    value = npx * args.steps / elapsed / 1e6
    # per-pass durations: the same kernels replayed eagerly with events
    pass_ms = dict.fromkeys(L.PASS_NAMES, 0.0)
    iter_ms = [0.0] * synth.NITER
    for _ in range(args.steps):
        per_iter = L.batch_pass_ms(synth.NITER, stream=stream, per_iter=True)
        for i, d in enumerate(per_iter):
            for k, v in d.items():
                pass_ms[k] += v
                iter_ms[i] += v
    for i, d in enumerate(per_iter):
        log("iteration %d (last replay), ms: %s" % (i, {k: round(v, 3) for k, v in d.items()}))
    log("batched: %.2f ms/step (%.2f ms on the GPU), %.1f Mpix/s; passes (ms/step): %s; "
        "iterations (ms/step): %s" %
        (ms_step, gpu_ms_step, value, {k: round(v / args.steps, 3) for k, v in pass_ms.items()},
         [round(v / args.steps, 3) for v in iter_ms]))

    # the plain single-frame path on the same frames, one at a time, enqueued
    # on the same stream without waiting in between
    plain = None
    if not args.no_plain:
        L.set_tile_shape(cfg)
        for i in range(len(dev)):
            L.run_ex(dev[i], params[i], masks[i], cleans[i], stream=stream, stats=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for i in range(len(dev)):
                L.run_ex(dev[i], params[i], masks[i], cleans[i], stream=stream, stats=False)
        torch.cuda.synchronize()
        plain = npx * args.steps / (time.perf_counter() - t0) / 1e6
        log("plain: %.1f Mpix/s" % plain)

    # the 512 x 512 frame alone through the single-frame path (small frames
    # run one fused launch per iteration)
    img0, fp0 = synth.config_frame("c0", threads=threads)
    d0 = torch.from_numpy(img0).cuda()
    p0 = L.make_params(fp0.gain, fp0.readnoise, niter=synth.NITER)
    m0 = torch.empty(img0.shape, dtype=torch.uint8, device="cuda")
    c0 = torch.empty(img0.shape, dtype=torch.float32, device="cuda")
    for _ in range(5):
        L.run_ex(d0, p0, m0, c0, stream=stream, stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(50):
        L.run_ex(d0, p0, m0, c0, stream=stream, stats=False)
    torch.cuda.synchronize()
    c0_ms = (time.perf_counter() - t0) / 50 * 1e3
    log("512x512 single frame: %.4f ms" % c0_ms)
    del d0, m0, c0
    variants = workload_variants(L, synth, stream, threads)

    # roofline of the dominant kernel, A1 (iteration 0; one launch per frame
    # group, each over about 1 / groups of the pixels): per-launch averages
    dom = max(pass_ms, key=lambda k: pass_ms[k])
    step_s = pass_ms["A1"] / 1e3 / args.steps  # all A1 launches of one step
    ops_px = a1_ops_per_pixel(cfg)
    achieved = ops_px * npx / step_s / 1e12
    traffic = read_traffic("%d,%d,%d" % (cfg, mode, groups))
    roofline = {"kernel": "A1", "bound": "alu", "achieved": round(achieved, 2),
                "peak": round(VALU_PEAK_TOPS, 2), "unit": "TOP/s",
                "frac": round(achieved / VALU_PEAK_TOPS, 4),
                "traffic": traffic,
                "algorithmic_bytes": round(A1_BYTES_PER_PIXEL * npx / groups),
                "ops_per_pixel": ops_px, "launches_per_step": groups,
                "launch_ms": round(step_s * 1e3 / groups, 4),
                "hbm_gbs_algorithmic": round(A1_BYTES_PER_PIXEL * npx / step_s / 1e9, 1),
                "share_of_step": round(pass_ms["A1"] / max(sum(pass_ms.values()), 1e-9), 3),
                "largest_pass": dom}

    out = {"metric": METRIC, "value": round(value, 1), "unit": "Mpix/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
           "gpu_ms_per_step": round(gpu_ms_step, 3), "median_gpu_ms_per_step": round(median_ms, 3),
           "median_mpix_s": round(npx / median_ms / 1e3, 1),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "64 mixed frames (32 x 2048^2, 24 x 4096^2, 8 x 6400x9600 "
                                  "uint16-ADU CMOS), niter=4 full, batched (autotuned tile "
                                  "shape, launch form and frame groups) + graph",
                      "frames": len(imgs), "megapixels": round(npx / 1e6, 1),
                      "niter": synth.NITER, "tile_shape": list(L.tile_shapes()[cfg]),
                      "launch": ("persistent queue", "grid")[mode], "frame_groups": groups},
           "plain_mpix_s": round(plain, 1) if plain else None,
           "small_frame": {"workload": "512x512, niter=4, single-frame path (fused launches)",
                           "ms": round(c0_ms, 4), "mpix_s": round(img0.size / c0_ms / 1e3, 1)},
           "workload_variants": variants,
           "batched_vs_plain": round(value / plain, 3) if plain else None,
           "pass_ms_per_step": {k: round(v / args.steps, 3) for k, v in pass_ms.items()},
           "iteration_ms_per_step": [round(v / args.steps, 3) for v in iter_ms],
           "roofline": roofline}

    del dev, masks, cleans
    L.shutdown()
    torch.cuda.empty_cache()

    if not args.no_serve:
        budget = int(args.serve_budget_gb * (1 << 30))
        t = time.perf_counter()
        pool = serve_pool(threads)
        log("serving pool: %d frames in %.1f s" % (len(pool), time.perf_counter() - t))
        if args.serve_one:
            out["serving"] = serve_run(L, pool, 32, 16.0, budget)
            log("serve", out["serving"])
        else:
            sweep = serve_sweep(L, pool, budget)
            best = max(sweep, key=lambda r: r["mpix_s"])
            out["serving"] = {"pool": "8 frames each of 2048^2, 4096^2 and 6400x9600 (uint16)",
                              "budget_gb": args.serve_budget_gb,
                              "latency": "submit (host frame) to completed device-to-host copy",
                              "sweep": sweep, "saturation_mpix_s": best["mpix_s"],
                              "saturation_rate_hz": best["rate_hz"]}
        del pool

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(imgs[0], synth.params_for("ccd"), threads)
        log("cpu baseline", out["cpu_baseline"])

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
