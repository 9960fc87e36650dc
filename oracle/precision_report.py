#!/usr/bin/env python3
"""Binary32 against binary64: the oracle run in both precisions on the
512^2, 4096^2 and 6400x9600 workload frames (niter = 4, the workload's
parameters), and per output the disagreement of the binary32 result with
the binary64 one: mask pixels that differ, the maximum and 99th-percentile
relative error of the cleaned image (relative to max(|x|, 1)), and the
largest and 99th-percentile absolute difference of S' over every pixel in
the first iteration (where both runs start from the same image).

Only the oracle runs here (test infrastructure); the GPU path is bit-identical
to the binary32 oracle, so these are its errors too.  Prints a markdown table;
--out writes it to a file.

    python oracle/precision_report.py --threads 6 --out profiles/oracle_fp64_vs_fp32.md
"""

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2602_17938_amd import synth  # noqa: E402


def report(name, threads):
    img, p = synth.config_frame(name, threads=threads)
    t = time.perf_counter()
    a = oracle.lacosmic(img, p.gain, p.readnoise, p.sigclip, p.sigfrac, p.objlim, p.niter,
                        nthreads=threads, trace=False)
    d = oracle.lacosmic(img.astype(np.float64), p.gain, p.readnoise, p.sigclip, p.sigfrac,
                        p.objlim, p.niter, nthreads=threads, dtype=np.float64, trace=False)
    dt = time.perf_counter() - t
    mdiff = int((a["mask"] != d["mask"]).sum())
    rel = np.abs(a["clean"].astype(np.float64) - d["clean"]) / np.maximum(np.abs(d["clean"]), 1.0)
    row = dict(name=name, shape="%dx%d" % img.shape, flagged32=int(a["mask"].sum()),
               flagged64=int(d["mask"].sum()), mask_diff=mdiff, rel_max=float(rel.max()),
               rel_p99=float(np.percentile(rel, 99)), n_new32=list(map(int, a["n_new"])),
               n_new64=list(map(int, d["n_new"])), seconds=dt)
    del a, d
    # S' of the first iteration in both precisions (one iteration, traced)
    a1 = oracle.lacosmic(img, p.gain, p.readnoise, p.sigclip, p.sigfrac, p.objlim, 1,
                         nthreads=threads, trace=True)
    d1 = oracle.lacosmic(img.astype(np.float64), p.gain, p.readnoise, p.sigclip, p.sigfrac,
                         p.objlim, 1, nthreads=threads, dtype=np.float64, trace=True)
    diff = np.abs(a1["trace_sp"][0].astype(np.float64) - d1["trace_sp"][0])
    row["sp_max_abs"] = float(diff.max())
    row["sp_p99_abs"] = float(np.percentile(diff, 99))
    return row


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", default="c0,c1,c2")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    oracle.build(force=False)
    rows = []
    for name in args.configs.split(","):
        r = report(name, args.threads)
        print(r, file=sys.stderr, flush=True)
        rows.append(r)
    lines = ["# Oracle: binary32 against binary64",
             "",
             "Command: `python oracle/precision_report.py --threads %d --out "
             "profiles/oracle_fp64_vs_fp32.md`.  The GPU path is "
             "bit-identical to the binary32 oracle, so these are its errors against a "
             "binary64 evaluation of the same steps." % args.threads,
             "",
             "| Frame | Shape | Mask px (f32 / f64) | Mask px that differ | Clean max rel err "
             "| Clean p99 rel err | S' max abs diff (it 1) | S' p99 abs diff (it 1) "
             "| New px per iteration f32 / f64 |",
             "|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append("| %s | %s | %d / %d | %d | %.3g | %.3g | %.3g | %.3g | %s / %s |" % (
            r["name"], r["shape"], r["flagged32"], r["flagged64"], r["mask_diff"], r["rel_max"],
            r["rel_p99"], r["sp_max_abs"], r["sp_p99_abs"], r["n_new32"], r["n_new64"]))
    text = "\n".join(lines) + "\n"
    print(text)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)


if __name__ == "__main__":
    main()
