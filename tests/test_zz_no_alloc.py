"""The no-allocation estimator entry point (tlrqmc_prob_noalloc) on the GPU.

It must return what mvn_prob / mvt_prob return on the same arguments, bit
for bit (same kernels and per-sample arithmetic, chunks sized to its fixed
scratch array), on consecutive calls whose inputs shrink, without calling
the context's allocator, and refuse a problem that does not fit its scratch
before doing any device work.
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_11183_amd import tlrqmc
    return tlrqmc


@pytest.fixture(scope="module")
def ctx(T):
    return T.Context(0)


def factor(T, ctx, n, m, seed):
    return T.Factor.from_tiles(ctx, n, m, *synth.random_tlr_factor(n, m, seed=seed))


def limits(n, seed, two_sided=False):
    b = 0.5 + 2.0 * synth.uniform01(seed, n, 0)
    a = b - 2.5 if two_sided else np.full(n, -np.inf)
    return a, b


def same(x, y):
    assert x["log_p"] == y["log_p"]
    assert x["std_err"] == y["std_err"]
    assert np.array_equal(x["log_p_shift"], y["log_p_shift"])
    assert x["n_dead"] == y["n_dead"]


def allocations():
    import torch
    return torch.cuda.memory_stats(0).get("allocation.all.allocated", 0)


CASES = [
    # n, m, N, M, nu, precision, two_sided: each later call smaller than the one before it
    (1500, 128, 40000, 8, 7.0, 1, False),
    (700, 64, 3000, 6, 0.0, 0, True),
    (300, 64, 1000, 4, 5.0, 0, False),
]


def test_noalloc_matches_the_allocating_entry_points_on_shrinking_calls(T, ctx):
    import torch
    refs, facs = [], []
    for i, (n, m, N, M, nu, prec, two) in enumerate(CASES):
        F = factor(T, ctx, n, m, 40 + i)
        a, b = limits(n, 50 + i, two)
        refs.append(T.probability(ctx, F, a, b, N, M, 11 + i, nu=nu, precision=prec))
        facs.append((F, a, b))
    torch.cuda.synchronize()
    before = allocations()
    got = []
    for (n, m, N, M, nu, prec, two), (F, a, b), i in zip(CASES, facs, range(len(CASES))):
        got.append(T.probability_noalloc(ctx, F, a, b, N, M, 11 + i, nu=nu, precision=prec))
    assert allocations() == before, "the no-allocation entry point called the allocator"
    for g, r in zip(got, refs):
        assert g["status"] == r["status"]
        same(g, r)
    # the first case runs in several chunks of the scratch
    assert got[0]["chunks"] >= 2
    # and once more, the large case again after the small ones
    again = T.probability_noalloc(ctx, facs[0][0], facs[0][1], facs[0][2], CASES[0][2], CASES[0][3], 11,
                                  nu=CASES[0][4], precision=CASES[0][5])
    same(again, refs[0])
    for F, _, _ in facs:
        F.free()


def test_noalloc_refuses_what_does_not_fit(T, ctx):
    n, m = 300, 64
    F = factor(T, ctx, n, m, 60)
    a, b = limits(n, 61)
    try:
        # 4e7 samples need 320 MB of per-sample log P alone: more than the scratch
        with pytest.raises(T.TLRQMCError) as e:
            T.probability_noalloc(ctx, F, a, b, 4_000_000, 10, 1)
        assert e.value.status == T.ENOMEM and "no-allocation scratch" in str(e.value)
        # the entry point still works after the refusal
        r = T.probability_noalloc(ctx, F, a, b, 500, 4, 2)
        same(r, T.probability(ctx, F, a, b, 500, 4, 2))
    finally:
        F.free()
