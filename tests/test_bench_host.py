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


def test_sweep_row_flops_are_the_triangles():
    # every tile contributes m_i (m_i - 1) flops of row products; rows inside
    # 16-row blocks on the vector ALU, earlier blocks on matrix cores
    mf, va = bench.sweep_row_flops(16384, 256)
    assert mf + va == 64 * 256 * 255 and va == 64 * 16 * 16 * 15
    mf, va = bench.sweep_row_flops(1000, 256)  # ragged last tile of 232 rows (14 blocks of 16 and one of 8)
    assert mf + va == 3 * 256 * 255 + 232 * 231 and va == 3 * 16 * 240 + 14 * 240 + 8 * 7


def test_kernel_work_per_sample():
    n, m, k_tot = 16384, 256, 17195
    st = {"k_tot": k_tot}
    w = bench.kernel_work("sweep", st, n, m, 1)
    assert w["rows"] == 64 * m * (m - 1)
    assert w["bytes"] == 8 * n + 24 * 64
    # low-rank products: 2 m K_tot per sample, three BF16 products executed in the precision form
    for kind in ("delta", "zproj"):
        w = bench.kernel_work(kind, st, n, m, 1)
        assert w["bf16_mfma"] == 3 * 2.0 * m * k_tot and w["alg"] == 2.0 * m * k_tot
        assert w["bytes"] == 4 * (k_tot + n)
    w = bench.kernel_work("delta", st, n, m, 0)
    assert w["fp64_mfma"] == 2.0 * m * k_tot and w["fp64_valu"] == 0.0
    w = bench.kernel_work("zproj", st, n, m, 0)
    assert w["fp64_valu"] == 2.0 * m * k_tot and w["fp64_mfma"] == 0.0


def test_time_bound_takes_the_slowest_resource():
    # FP64 products and vector operations add on the SIMD issue: 1 s + (2 + 1) s
    w = {"fp64_mfma": 78.6e12, "bf16_mfma": 0.0, "fp64_valu": 2 * 78.6e12, "fp32_valu": 157.3e12, "bytes": 8e12}
    t, b = bench.time_bound(w)
    assert b == "alu" and abs(t - 4.0) < 1e-12
    # the FP64 products the larger part: named after the matrix cores
    w = {"fp64_mfma": 3 * 78.6e12, "bf16_mfma": 0.0, "fp64_valu": 78.6e12, "fp32_valu": 0.0, "bytes": 8e12}
    t, b = bench.time_bound(w)
    assert b == "mfma" and abs(t - 4.0) < 1e-12
    # BF16 products run beside HBM transfers: the slower of the two
    w = {"fp64_mfma": 0.0, "bf16_mfma": 2.5e15, "fp64_valu": 0.0, "fp32_valu": 0.0, "bytes": 16e12}
    t, b = bench.time_bound(w)
    assert b == "hbm" and abs(t - 2.0) < 1e-12
    w = {"fp64_mfma": 0.0, "bf16_mfma": 7.5e15, "fp64_valu": 0.0, "fp32_valu": 0.0, "bytes": 16e12}
    t, b = bench.time_bound(w)
    assert b == "mfma" and abs(t - 3.0) < 1e-12


def test_log_gap_over_se():
    import math
    # P = 1.1 e^-500 against 1.0 e^-500 with relative error 0.2: (0.1) / 0.2
    g = bench.log_gap_over_se({"log_p": math.log(1.1) - 500}, {"log_p": -500.0, "rel_err": 0.2})
    assert abs(g - 0.5) < 1e-12


def test_traffic_table_keys():
    kinds = {"sweep", "delta", "zproj"}
    for (cfg, kind, prec), e in bench.TRAFFIC.items():
        assert cfg in (1, 2, 3, 4) and kind in kinds and prec in (0, 1)
        assert e["bytes_per_launch"] > 0 and len(e["digest"]) == 16


def test_ratio_note_sums_the_lower_bounds():
    roof = {"kinds": {"sweep": {"lower_bound_ms": 0.2, "frac": 0.4}, "delta": {"lower_bound_ms": 0.05, "frac": 0.2},
                      "zproj": {"lower_bound_ms": 0.05, "frac": 0.1}}}
    fp64 = {"roofline": {"kinds": {"sweep": {"lower_bound_ms": 0.4, "frac": 0.3},
                                   "delta": {"lower_bound_ms": 0.35, "frac": 0.2},
                                   "zproj": {"lower_bound_ms": 0.35, "frac": 0.2}}}}
    r = bench.ratio_note(roof, fp64)
    assert abs(r["ratio_at_resource_bounds"] - 1.1 / 0.3) < 1e-12
    assert r["fp64_form_frac"]["sweep"] == 0.3 and r["precision_form_frac"]["zproj"] == 0.1
    assert bench.ratio_note(roof, None) is None


def test_kernel_digest_follows_device_options_not_paths(monkeypatch):
    from paper_2003_11183_amd import build
    d0 = bench.kernel_digest()
    # include paths differ between machines: not part of the digest
    monkeypatch.setattr(build, "DEVICE", build.DEVICE + ["-I/somewhere/else"])
    assert bench.kernel_digest() == d0
    # a device option of a kernel file is
    monkeypatch.setattr(build, "FILE_FLAGS", dict(build.FILE_FLAGS, **{"kernels.hip": []}))
    assert bench.kernel_digest() != d0
