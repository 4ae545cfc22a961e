"""Host-side checks of bench.py: the one-GPU refusal, and the algorithmic
work, bound and peak it prices each kernel kind with (the roofline figures
of the JSON line rest on them)."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in out["error"]


def test_kernel_work_per_sample():
    n, m, k_tot = 16384, 256, 17195
    st = {"k_tot": k_tot}
    # sweep: the row products of every diagonal tile plus the per-variable cost
    w, bound, peak = bench.kernel_work("sweep", st, n, m, 1)
    assert w == 64 * m * (m - 1) + bench.C_PHI * n and bound == "alu" and peak == bench.PEAK_FP64_VALU
    # ragged last tile
    w, _, _ = bench.kernel_work("sweep", st, 1000, 256, 1)
    assert w == 3 * 256 * 255 + 232 * 231 + bench.C_PHI * 1000
    # low-rank products: 2 m K_tot per sample, three BF16 products in the precision form
    for kind in ("delta", "zproj"):
        w, bound, peak = bench.kernel_work(kind, st, n, m, 1)
        assert w == 3 * 2.0 * m * k_tot and bound == "mfma" and peak == bench.PEAK_BF16_MFMA
    w, bound, peak = bench.kernel_work("delta", st, n, m, 0)
    assert w == 2.0 * m * k_tot and bound == "mfma" and peak == bench.PEAK_FP64_VALU
    w, bound, peak = bench.kernel_work("zproj", st, n, m, 0)
    assert w == 2.0 * m * k_tot and bound == "alu" and peak == bench.PEAK_FP64_VALU


def test_traffic_table_keys():
    kinds = {"sweep", "delta", "zproj"}
    for (cfg, kind, prec), e in bench.TRAFFIC.items():
        assert cfg in (1, 2, 3, 4) and kind in kinds and prec in (0, 1)
        assert e["bytes_per_launch"] > 0 and len(e["digest"]) == 16
