"""Per-kernel timing of profiled calls (the launch-marked events).

A profiled call reports, per kernel kind, the number of launches, the sum of
their durations and the union of their intervals.  The counts follow from
the factor's tiles and the chunking; profiling changes no result; the
context's event pool is reused by the next profiled call.
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    from paper_2003_11183_amd import tlrqmc
    return tlrqmc


@pytest.fixture(scope="module")
def ctx(T):
    return T.Context(0)


def expected_launches(ranks, r, chunks):
    krow = [int(ranks[i, :i].sum()) for i in range(r)]
    kcol = [int(ranks[i + 1:, i].sum()) for i in range(r)]
    return {
        "init": chunks,
        "delta": chunks * sum(1 for j in range(1, r) if krow[j] > 0),
        "sweep": chunks * r,
        "zproj": chunks * sum(1 for j in range(r - 1) if kcol[j] > 0),
        "reduce": 1,
    }


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("N", [3000, 70000])
def test_profiled_calls_count_every_launch_and_change_nothing(T, ctx, precision, N):
    n, m, M = 900, 64, 2
    diag, ranks, U, V = synth.random_tlr_factor(n, m, seed=77, rank_mean=4.0, rank_max=16)
    r = (n + m - 1) // m
    # one block row and one block column with no low-rank tiles: their
    # low-rank launches are skipped
    ranks = np.array(ranks, dtype=np.int32)
    ranks[3, :3] = 0
    ranks[13:, 12] = 0
    F = T.Factor.from_tiles(ctx, n, m, diag, ranks, U, V)
    b = np.linspace(0.2, 2.0, n)
    a = np.full(n, -np.inf)
    plain = T.probability(ctx, F, a, b, N, M, 5, nu=4.0, precision=precision)
    runs = [T.probability(ctx, F, a, b, N, M, 5, nu=4.0, precision=precision, profile=True) for _ in range(2)]
    for res in runs:
        # profiling changes no result
        assert list(res["log_p_shift"]) == list(plain["log_p_shift"])
        assert res["log_p"] == plain["log_p"]
        # N = 70,000 x 2 shifts is above the two-stream threshold
        assert res["chunks"] == (2 if N * M >= 131072 else 1)
        want = expected_launches(ranks, r, res["chunks"])
        assert res["kernel_launches"] == want
        for k in want:
            total, busy = res["kernel_seconds"][k], res["kernel_busy_seconds"][k]
            assert total > 0.0 and 0.0 < busy <= total * (1 + 1e-6) + 1e-9, (k, total, busy)
            # every launch lies inside the call's own timed region
            assert busy <= res["seconds"] * (1 + 1e-3) + 1e-6, (k, busy, res["seconds"])
    # the second profiled call took its events from the pool the first returned
    assert runs[0]["kernel_launches"] == runs[1]["kernel_launches"]
    # an unprofiled call reports no kernel times
    assert all(v == 0 for v in plain["kernel_launches"].values())
