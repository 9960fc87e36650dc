"""The selection networks the kernels use, checked where they are generated:
the 0-1 principle over every 0-1 input for med9 and med25, random inputs with
ties for med49, the shared 2x2- and 4x2-block med25, sort25 and its 13-rank
prefix; and the algorithmic operation count the benchmark prices A1 with
against the sizes of the networks A1 runs."""

import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GEN = os.path.join(ROOT, "paper_2602_17938_amd", "csrc", "gen_median_net.py")


def test_generated_networks_pass_their_checks(tmp_path):
    out = tmp_path / "median_net.gen.h"
    r = subprocess.run([sys.executable, GEN, str(out), "--check"], capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "(checked)" in r.stdout
    assert out.stat().st_size > 0


def test_bench_a1_op_count_follows_the_networks():
    spec = importlib.util.spec_from_file_location("gen_median_net", GEN)
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    n42, o42 = gen.block_median_net(5, 4, 2)
    n22, o22 = gen.block_median_net(5, 2, 2)
    assert (len(o42), len(o22)) == (8, 4)
    sys.path.insert(0, ROOT)
    import bench
    pointwise = 29 + 13 + 12  # Laplacian, noise model, S (the fast forms)
    assert bench.a1_ops_per_pixel(1) == len(n42.ops) / 8 + pointwise  # 32-row tiles
    assert bench.a1_ops_per_pixel(0) == len(n22.ops) / 4 + pointwise  # 16-row tiles
