"""Benchmark: QMC sample-dimensions per second of the TLR estimator on one GPU.

Default workload: the Student-t problem at n = 16,384.

- 128 x 128 regular grid on the unit square, exponential covariance with range 0.3, nu = 7.
- Tile m = 256, off-diagonal tiles truncated at 1e-5, a = -inf, b ~ U(0, 4).
- N = 40,000 lattice points x 10 random shifts.

One step is one full estimate (mvt_prob): lattice, chi radii, low-rank limit updates, diagonal-tile sweeps and
the per-shift reductions. It runs in the workload's precision form (BF16x3 MFMA low-rank updates, FP64
elsewhere); the plain FP64 form is timed on the same problem and reported beside it. The factor is built once
before timing, since the paper also times the integration only.

Inputs are synthetic and seeded. The factor, limits and shifts are on the device when the timed region starts.
Prints one JSON line. --gpus N > 1 is refused: this build runs on one GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QMC sample·dims/sec at n=16384 (FP64 vs BF16-MFMA); p50/p99 latency per prob"
PEAK_FP64_VALU = 78.6e12    # 256 CU x 2.4 GHz x 64 lanes x 2 flops (FMA)
PEAK_BF16_MFMA = 2.5e15     # dense
# FP64 operations per variable of the sweep beyond the row products (Phi, log,
# Phi^-1, lattice point, bookkeeping).
C_PHI = 150


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--precision", type=int, default=-1, help="-1 = the workload's own form")
    ap.add_argument("--no-fp64-form", action="store_true", help="skip timing the FP64 form beside it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=1536)
    ap.add_argument("--serve", type=int, default=100, metavar="COUNT",
                    help="requests of the mixed-dimension serving stream to replay (0 = skip)")
    ap.add_argument("--serve-fp64", type=int, default=12, metavar="COUNT",
                    help="of those, how many also run one at a time through the plain FP64 path")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--no-reorder-study", action="store_true",
                    help="skip the ordering study on the n = 4,096 MVN workload")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (scale for HBM byte counters)")
    return ap.parse_args()


def kernel_work(kind: str, st: dict, n: int, m: int, precision: int) -> tuple[float, str, float]:
    """Algorithmic work per sample of all launches of one kernel kind, its
    bound and the peak of that bound: the precision form's low-rank products
    run on BF16 matrix cores, the FP64 form's limit update on FP64 matrix
    cores and its projection on the FP64 vector ALU (both 78.6 TFLOP/s)."""
    if kind == "sweep":
        tri = sum(min(m, n - i * m) * (min(m, n - i * m) - 1) for i in range((n + m - 1) // m))
        return tri + C_PHI * n, "alu", PEAK_FP64_VALU
    if kind in ("delta", "zproj"):
        f = 2.0 * m * st["k_tot"]
        if precision == 1:
            return 3 * f, "mfma", PEAK_BF16_MFMA
        return f, ("mfma" if kind == "delta" else "alu"), PEAK_FP64_VALU
    return float("nan"), "alu", PEAK_FP64_VALU


def time_form(T, ctx, F, c, precision, steps, warmup):
    N, M, nu = c["N"], c["M"], c["nu"]

    def step(profile=False):
        return T.probability(ctx, F, c["a"], c["b"], N, M, c["seed_shift"], nu=nu, precision=precision,
                             profile=profile)

    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    lat, results = [], []
    t_start = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        results.append(step(profile=True))
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    return elapsed, lat, results


# HBM bytes per launch of a kernel (FETCH_SIZE x fetch scale + WRITE_SIZE x
# write scale, both scaled by what the counters read for a plain 1 GiB copy),
# from the rocprofv3 runs summarised under profiles/.  A figure is reported
# only while the kernel sources and the build script (its device flags) still
# have the digest it was measured on.
TRAFFIC = {
    (3, "sweep", 1): {"bytes_per_launch": 1.933e9, "digest": "d03600bba52cbdef"},
    (3, "delta", 1): {"bytes_per_launch": 4.352e8, "digest": "d03600bba52cbdef"},
    (3, "zproj", 1): {"bytes_per_launch": 4.30e8, "digest": "d03600bba52cbdef"},
    (3, "sweep", 0): {"bytes_per_launch": 3.856e9, "digest": "d03600bba52cbdef"},
    (3, "delta", 0): {"bytes_per_launch": 1.304e9, "digest": "d03600bba52cbdef"},
    (3, "zproj", 0): {"bytes_per_launch": 2.414e9, "digest": "d03600bba52cbdef"},
}
KERNEL_SOURCES = tuple(os.path.join("csrc", f) for f in (
    "kernels.hip", "kernels_mfma.hip", "kernels_lr64.hip", "device_math.hpp", "special_tables.hpp",
    "internal.hpp")) + ("build.py",)


def kernel_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2003_11183_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def roofline_of(T, results, st, c, precision, steps):
    """Roofline of the kernel kind with the largest busy time.  achieved =
    algorithmic work per launch / average launch duration (HIP events on the
    launch's stream); launches on the two worker streams overlap, so the
    chip-level rate (all launches' work / union of their intervals) is
    reported beside it."""
    n, m, samples = c["n"], c["m"], c["N"] * c["M"]
    ks = {k: sum(r["kernel_seconds"][k] for r in results) for k in T.KERNEL_NAMES}
    kb = {k: sum(r["kernel_busy_seconds"][k] for r in results) for k in T.KERNEL_NAMES}
    kl = {k: sum(r["kernel_launches"][k] for r in results) for k in T.KERNEL_NAMES}
    dom = max(kb, key=kb.get)
    work, bound, peak = kernel_work(dom, st, n, m, precision)
    launches = max(kl[dom], 1)
    per_launch = work * samples * steps / launches
    avg = ks[dom] / launches
    achieved = per_launch / avg
    chip = work * samples * steps / kb[dom]
    tr = TRAFFIC.get((c["id"], dom, precision))
    traffic = tr["bytes_per_launch"] if tr and tr["digest"] == kernel_digest() else None
    # the same figures for every kernel kind of the step (HBM rate from the
    # measured traffic where it is current)
    kinds = {}
    for k in ("sweep", "delta", "zproj"):
        if kl[k] == 0 or ks[k] <= 0:
            continue
        w_k, b_k, p_k = kernel_work(k, st, n, m, precision)
        pl = w_k * samples * steps / kl[k]
        av = ks[k] / kl[k]
        t_k = TRAFFIC.get((c["id"], k, precision))
        tb = t_k["bytes_per_launch"] if t_k and t_k["digest"] == kernel_digest() else None
        kinds[k] = {"bound": b_k, "achieved": pl / av / 1e12, "peak": p_k / 1e12, "frac": pl / av / p_k,
                    "avg_launch_ms": 1e3 * av, "traffic": tb,
                    "hbm_tb_per_s": (tb / av / 1e12) if tb else None}
    return {"bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic, "traffic_unit": "bytes/launch",
            "kernel": dom, "work_per_launch_tflop": per_launch / 1e12, "avg_launch_ms": 1e3 * avg,
            "achieved_chip": chip / 1e12, "frac_chip": chip / peak,
            "busy_ms_per_step": {k: 1e3 * v / steps for k, v in kb.items()},
            "launch_ms_sum_per_step": {k: 1e3 * v / steps for k, v in ks.items()},
            "launches_per_step": {k: kl[k] // steps for k in kl},
            "kinds": kinds}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(sharding across GPUs is designed, not built)"}))
        sys.exit(2)
    import torch
    if args.copy_calibration > 0:
        copy_calibration(torch, args.copy_calibration)
        return

    import synth
    from paper_2003_11183_amd import tlrqmc as T

    c = synth.config(args.config)
    n, m, N, M, nu = c["n"], c["m"], c["N"], c["M"], c["nu"]
    precision = c["precision"] if args.precision < 0 else args.precision
    ctx = T.Context(0)
    t0 = time.perf_counter()
    cov = {"xy": c["xy"], "beta": c["beta"]}
    perm = T.block_reorder(cov, c["a"], c["b"], m) if c["reorder"] else None
    F = T.Factor.build(ctx, cov, n, m, c["tol"], c["cap"], perm=perm)
    setup_s = time.perf_counter() - t0
    st = F.stats()
    torch.cuda.empty_cache()

    elapsed, lat, results = time_form(T, ctx, F, c, precision, args.steps, args.warmup)
    ms_per_step = 1e3 * elapsed / args.steps
    value = N * M * n / (elapsed / args.steps)
    roof = roofline_of(T, results, st, c, precision, args.steps)
    dev_s = float(np.mean([r["seconds"] for r in results]))

    fp64 = None
    if precision != 0 and not args.no_fp64_form:
        e64, lat64, res64 = time_form(T, ctx, F, c, 0, max(2, args.steps // 2), 1)
        s64 = max(2, args.steps // 2)
        r64 = res64[-1]
        fp64 = {"value": N * M * n / (e64 / s64), "ms_per_step": 1e3 * e64 / s64, "log_p": r64["log_p"],
                "std_err": r64["std_err"], "rel_err": r64["rel_err"],
                "roofline": roofline_of(T, res64, st, c, 0, s64)}

    cpu = None if args.no_cpu_baseline else cpu_baseline(F, c, args.cpu_samples)
    F.free()
    torch.cuda.empty_cache()
    serve = serving(T, ctx, args.serve, args.serve_fp64, args.serve_budget_gib) if args.serve > 0 else None
    study = None if args.no_reorder_study else reorder_study(T, ctx)
    client = None if args.no_reorder_study else skewnormal_client(T, ctx)
    r0 = results[-1]
    lat_ms = [1e3 * x for x in lat]
    out = {
        "metric": METRIC, "value": value, "unit": "sample·dims/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == 0 else "f64+bf16",
        "data": "synthetic (seeded grid, limits and shifts)",
        "config": {"workload": f"{c['name']}: {c['g']}x{c['g']} grid, range {c['beta']}, "
                               f"{'MVT nu ' + str(nu) if nu else 'MVN'}, m {m}, tol {c['tol']}, "
                               f"cap {c['cap']}, reorder {c['reorder']}, N {N} x {M} shifts, "
                               f"{'FP64' if precision == 0 else 'BF16x3-MFMA low-rank / FP64 sweep'}",
                   "n": n, "m": m, "samples": N, "shifts": M, "precision": precision,
                   "k_tot": st["k_tot"], "k_max": st["k_max"], "cap_hits": st["cap_hits"],
                   "factor_mb": st["device_bytes"] / 2 ** 20, "setup_s": setup_s,
                   "setup_phases_s": st["setup_seconds"], "host_tiles": st["host_tiles"]},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "estimate": {"log_p": r0["log_p"], "std_err": r0["std_err"], "rel_err": r0["rel_err"]},
        "value_device_only": N * M * n / dev_s,
        "fp64_form": fp64,
        "ratio_vs_fp64_form": (value / fp64["value"]) if fp64 else None,
        "roofline": roof,
        "cpu_baseline": cpu,
        "serving": serve,
        "reorder_study": study,
        "skewnormal_client": client,
    }
    print(json.dumps(out), flush=True)


def serving(T, ctx, count: int, count_fp64: int, budget_gib: float):
    """Replay the first `count` requests of the mixed-dimension stream at their
    Poisson arrival times through the request server (continuous batching,
    footprint admission; BF16x3-MFMA low-rank form).  Latency = done - submit.
    The first `count_fp64` requests then also run one at a time through the
    plain FP64 single-request path (factor + mvn_prob/mvt_prob)."""
    import synth
    reqs = synth.serving_stream(count=count)
    S = T.Server(ctx, int(budget_gib * 2 ** 30))
    t0 = time.perf_counter()
    tickets = []
    for q in reqs:
        delay = q["arrival"] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append(S.submit({"xy": q["xy"], "beta": q["beta"]}, q["a"], q["b"], q["N"], q["M"], q["seed_shift"],
                                nu=q["nu"], m=q["m"], tol=1e-5, precision=1))
    out = [S.result(t, timeout_s=600) for t in tickets]
    st = S.stats()
    S.close()
    info = [o["info"] for o in out]
    lat = np.array([i["t_done"] - i["t_submit"] for i in info])
    setup = np.array([i["t_ready"] - i["t_admit"] for i in info])
    queue = np.array([i["t_admit"] - i["t_submit"] for i in info])
    run = np.array([i["t_done"] - i["t_start"] for i in info])
    span = max(i["t_done"] for i in info) - min(i["t_submit"] for i in info)
    work = float(sum(q["N"] * q["M"] * q["n"] for q in reqs))
    res = {"requests": count, "rate_per_s": 20.0, "budget_gib": budget_gib,
           "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)), "p99": 1e3 * float(np.percentile(lat, 99)),
                          "mean": 1e3 * float(lat.mean())},
           "phase_ms_mean": {"queue": 1e3 * float(queue.mean()), "setup": 1e3 * float(setup.mean()),
                             "run": 1e3 * float(run.mean())},
           "run_ms": {"p50": 1e3 * float(np.percentile(run, 50)), "p99": 1e3 * float(np.percentile(run, 99))},
           "throughput": work / span, "unit": "sample·dims/s", "makespan_s": span,
           "server": {k: st[k] for k in ("steps", "launches", "slot_steps", "max_active_slots",
                                         "peak_reserved_bytes", "arena_peak_bytes")},
           "n_mix": {str(g * g): sum(1 for q in reqs if q["g"] == g) for g in (32, 64, 96, 128)}}
    if count_fp64 > 0:
        import torch
        lat64, work64 = [], 0.0
        t1 = time.perf_counter()
        for q in reqs[:count_fp64]:
            ts = time.perf_counter()
            F = T.Factor.build(ctx, {"xy": q["xy"], "beta": q["beta"]}, q["n"], q["m"], 1e-5, 0)
            T.probability(ctx, F, q["a"], q["b"], q["N"], q["M"], q["seed_shift"], nu=q["nu"], precision=0)
            F.free()
            lat64.append(time.perf_counter() - ts)
            work64 += q["N"] * q["M"] * q["n"]
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        res["fp64_one_at_a_time"] = {"requests": count_fp64, "latency_ms_mean": 1e3 * float(np.mean(lat64)),
                                     "throughput": work64 / el, "unit": "sample·dims/s"}
    return res


def reorder_study(T, ctx, cid: int = 2):
    """Orderings on one workload (n = 4,096 MVN, m = 64, rank cap 32): the
    geometric order, block reordering, and block reordering during the
    Cholesky factorization.  Setup seconds and the estimate's relative error
    at the workload's N x M (the same lattice and shifts for all three)."""
    import synth
    c = synth.config(cid)
    cov = {"xy": c["xy"], "beta": c["beta"]}
    out = {"workload": c["name"], "n": c["n"], "m": c["m"], "samples": c["N"], "shifts": c["M"]}
    for name in ("geometric", "block", "block_during_cholesky"):
        t0 = time.perf_counter()
        if name == "block_during_cholesky":
            F = T.Factor.build_reordered(ctx, cov, c["a"], c["b"], c["m"], c["tol"], c["cap"])
        else:
            perm = T.block_reorder(cov, c["a"], c["b"], c["m"]) if name == "block" else None
            F = T.Factor.build(ctx, cov, c["n"], c["m"], c["tol"], c["cap"], perm=perm)
        setup = time.perf_counter() - t0
        r = T.probability(ctx, F, c["a"], c["b"], c["N"], c["M"], c["seed_shift"], nu=c["nu"], precision=0)
        out[name] = {"setup_s": setup, "log_p": r["log_p"], "rel_err": r["rel_err"], "k_tot": F.stats()["k_tot"],
                     "estimate_ms": 1e3 * r["seconds"]}
        F.free()
    return out


def skewnormal_client(T, ctx, g: int = 128):
    """One skew-normal log-likelihood evaluation (Eq. 6) at n = g^2 on a grid
    of unit distance 1/15 with sigma1 = sigma2 = 1, beta1 = beta2 = 0.3, the
    model drawn once from SplitMix64 normals; N = 10^4 x 10 samples in the
    precision form, tile 128; both orderings."""
    import synth
    n = g * g
    xy = synth.grid_xy(g) * ((g - 1) / 15.0)
    x = synth.workloads._normals(705, n, 0)
    y = synth.workloads._normals(805, n, 0)
    prm = dict(xi=0.2, sigma1=1.0, beta1=0.3, sigma2=1.0, beta2=0.3)
    # the draw z = xi + A x + B |y| on the device through torch (input generation only)
    import torch
    dev = torch.device("cuda:0")
    X = torch.tensor(xy, dtype=torch.float64, device=dev)
    d = torch.cdist(X, X)
    A = torch.linalg.cholesky(torch.exp(-d / prm["beta1"]))
    B = torch.exp(-d / prm["beta2"])
    z = (prm["xi"] + A @ torch.tensor(x, device=dev) + B @ torch.tensor(np.abs(y), device=dev)).cpu().numpy()
    del X, d, A, B
    torch.cuda.empty_cache()
    out = {"n": n, "samples": 10000, "shifts": 10, "m": 128}
    for name, order in (("geometric", 0), ("block_during_cholesky", 2)):
        t0 = time.perf_counter()
        r = T.skewnormal_loglik(ctx, xy, z, N=10000, M=10, seed=7, m=128, order=order, precision=1, **prm)
        out[name] = {"seconds": time.perf_counter() - t0, "phases_s": r["seconds"], "loglik": r["loglik"],
                     "log_prob": r["log_prob"], "rel_err": r["log_prob_rel_err"]}
    return out


def copy_calibration(torch, mib: int):
    """A plain device-to-device copy of known size: what the HBM byte counters read for it scales theirs."""
    n = mib * 2 ** 20 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 3}}), flush=True)


def cpu_baseline(F, c, S: int):
    """The oracle (dense SOV on the expanded factor) on the host, S points of shift 0."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    perm, diag, ranks, U, V = F.export()
    fac = (diag, ranks, U, V)
    ap, bp = c["a"][perm], c["b"][perm]
    t0 = time.perf_counter()
    lat = oracle.api.Lattice(c["n"], c["M"], c["seed_shift"])
    oracle.sample_logp(fac, ap, bp, c["nu"], c["seed_shift"], c["M"], 0, np.arange(1, S + 1), lat)
    t = time.perf_counter() - t0
    return {"value": S * c["n"] / t, "unit": "sample·dims/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{S} lattice points of shift 0 of the same workload (dense SOV over the expanded "
                      f"factor, numpy/scipy), {t:.1f} s"}


if __name__ == "__main__":
    main()
