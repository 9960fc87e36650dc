"""The selection networks the kernels use, checked where they are generated:
the 0-1 principle over every 0-1 input for med9 and med25, random inputs with
ties for med49, the shared 2x2-block med25, sort25 and its 13-rank prefix."""

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
