"""GPU parity at the workloads' full sizes, in the launch configuration of bench.py.

The factor is the library's own (tlr_factor, block reordering where the
workload has it); the estimate is the whole N x M run of mvn_prob / mvt_prob
with the chunking and worker streams the bench uses.  The oracle cannot redo
a whole run at these sizes, so it recomputes sampled samples one by one on
the exported factor: the first and last samples of the first and last
shifts, a middle one, and the samples on both sides of the boundary between
the two worker-stream chunks.  FP64 form: 1e-10 relative per sample.
Precision form (BF16x3 low-rank updates, FP32 special functions): 1e-3
relative per sample, and the two forms' estimates within a tenth of the
standard error.
"""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL_PREC = 1e-3


@pytest.fixture(scope="module")
def T():
    from paper_2003_11183_amd import tlrqmc
    return tlrqmc


@pytest.fixture(scope="module")
def ctx(T):
    return T.Context(0)


def sample_points(N, M):
    """(shift, k) pairs: ends of the first and last shifts, a middle sample,
    and the two sides of the boundary between the two chunks."""
    count = N * M
    chunk = -(-((count + 1) // 2) // 256) * 256  # the library's split over two streams
    g = chunk
    pts = {(0, 1), (0, N), (M - 1, 1), (M - 1, N), (M // 2, N // 2 + 1)}
    for gg in (g - 1, g):
        pts.add((gg // N, gg % N + 1))
    return sorted(pts)


def oracle_logp(T, F, a, b, nu, seed, M, pts):
    perm, diag, ranks, U, V = F.export()
    fac = (diag, ranks, U, V)
    ap, bp = np.asarray(a)[perm], np.asarray(b)[perm]
    lat = oracle.api.Lattice(len(a), M, seed)
    out = {}
    by_shift = {}
    for s, k in pts:
        by_shift.setdefault(s, []).append(k)
    for s, ks in by_shift.items():
        lp = oracle.sample_logp(fac, ap, bp, nu, seed, M, s, np.array(ks), lat)
        for k, v in zip(ks, lp):
            out[(s, k)] = v
    return out


def scaled_err(got, ref):
    if np.isneginf(ref):
        return 0.0 if np.isneginf(got) else np.inf
    return abs(got - ref) / max(1.0, abs(ref))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("cid", [2, 3, 4])
def test_full_size_sampled_against_oracle(T, ctx, cid):
    c = synth.config(cid)
    n, m, N, M, nu = c["n"], c["m"], c["N"], c["M"], c["nu"]
    print(f"config {cid}: n={n} m={m} N={N} M={M} nu={nu}", flush=True)
    cov = {"xy": c["xy"], "beta": c["beta"]}
    perm = T.block_reorder(cov, c["a"], c["b"], m) if c["reorder"] else None
    F = T.Factor.build(ctx, cov, n, m, c["tol"], c["cap"], perm=perm)
    res = {p: T.probability(ctx, F, c["a"], c["b"], N, M, c["seed_shift"], nu=nu, precision=p, return_logp=True)
           for p in (0, 1)}
    assert res[0]["chunks"] == 2 and res[1]["chunks"] == 2
    pts = sample_points(N, M)
    ref = oracle_logp(T, F, c["a"], c["b"], nu, c["seed_shift"], M, pts)
    F.free()
    for s, k in pts:
        r = ref[(s, k)]
        e64 = scaled_err(res[0]["logp"][s, k - 1], r)
        e32 = scaled_err(res[1]["logp"][s, k - 1], r)
        print(f"  sample (shift {s}, k {k}): oracle {r:.12g}  fp64 err {e64:.2e}  precision err {e32:.2e}",
              flush=True)
        assert e64 <= TOL64
        assert e32 <= TOL_PREC
    # the two forms' estimates agree within a tenth of the standard error
    d = abs(np.expm1(res[1]["log_p"] - res[0]["log_p"]))
    print(f"  log P: fp64 {res[0]['log_p']:.10f}  precision {res[1]['log_p']:.10f}  rel SE {res[0]['rel_err']:.3g}",
          flush=True)
    assert d <= 0.1 * res[0]["rel_err"]
