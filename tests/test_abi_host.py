"""CPU tests of the C ABI: exported symbols and the host-side setup logic.

No compute runs on a device here.  The geometric order and the block
reordering are host code in the library and are compared with the oracle's
independent implementation of the same definitions.
"""

import ctypes
import math
import os
import re

import numpy as np
import pytest

import synth
from oracle import factor as OF
from oracle import reorder as OR

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tlrqmc.h")


def _lib():
    from paper_2003_11183_amd import tlrqmc
    return tlrqmc


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("alloc", "free")))


def test_library_exports_every_declared_function():
    t = _lib()
    names = declared_functions()
    assert len(names) >= 12
    lib = ctypes.CDLL(t.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []
    assert set(names) <= set(t.SIGNATURES)


def test_context_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    t = _lib()
    h = ctypes.c_void_p()
    st = t.lib().tlrqmc_ctx_create(0, None, None, ctypes.byref(h))
    assert st == t.EDEVICE
    assert b"device" in t.lib().tlrqmc_last_error()


@pytest.mark.parametrize("g", [4, 16, 33, 64])
def test_geometric_order_matches_oracle(g):
    t = _lib()
    xy = synth.grid_xy(g)
    assert np.array_equal(t.geometric_order(xy), OF.morton_order(xy))


def test_geometric_order_scattered_points():
    t = _lib()
    rng = np.random.default_rng(5)
    xy = rng.random((500, 2)) * [3.0, 0.5] + [1.0, -2.0]
    assert np.array_equal(t.geometric_order(xy), OF.morton_order(xy))


def _near_tie_ok(perm_lib, perm_or, S, a, b, m):
    """Blocks of both orders sorted by score; differences only among near ties."""
    n = len(a)
    def scores(perm):
        out = []
        for q in range(n // m):
            blk = perm[q * m:(q + 1) * m]
            out.append(OR.univariate_conditioning(S[np.ix_(blk, blk)], a[blk], b[blk])[1])
        return np.array(out)
    s1, s2 = scores(perm_lib), scores(perm_or)
    return np.allclose(np.sort(s1), np.sort(s2), rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("g,m,beta,seed", [(16, 16, 0.1, 1), (24, 32, 0.3, 2), (32, 64, 0.1, 3)])
def test_block_reorder_matches_oracle(g, m, beta, seed):
    t = _lib()
    xy = synth.grid_xy(g)
    n = g * g
    b = synth.upper_limits_uniform(n, seed)
    a = np.full(n, -np.inf)
    S = OF.exp_cov(xy, beta)
    base = OF.morton_order(xy)
    mine = t.block_reorder({"xy": xy, "beta": beta}, a, b, m)
    ref = OR.block_reorder(S, a, b, m, base)
    if not np.array_equal(mine, ref):
        assert sorted(mine.tolist()) == list(range(n))
        assert _near_tie_ok(mine, ref, S, a, b, m)


def test_block_reorder_two_sided_and_dense_sigma():
    t = _lib()
    rng = np.random.default_rng(9)
    n, m = 96, 12
    xy = rng.random((n, 2))
    S = OF.exp_cov(xy, 0.2)
    a = np.where(rng.random(n) < 0.5, -np.inf, rng.uniform(-2, 0, n))
    b = rng.uniform(0.2, 2.5, n)
    mine = t.block_reorder({"sigma": S}, a, b, m)
    ref = OR.block_reorder(S, a, b, m, np.arange(n))
    assert np.array_equal(mine, ref) or _near_tie_ok(mine, ref, S, a, b, m)


def test_block_reorder_ragged_last_block_stays_last():
    t = _lib()
    xy = synth.grid_xy(10)
    n, m = 100, 16
    b = synth.upper_limits_uniform(n, 4)
    perm = t.block_reorder({"xy": xy, "beta": 0.2}, np.full(n, -np.inf), b, m)
    base = OF.morton_order(xy)
    assert set(perm[96:].tolist()) == set(base[96:].tolist())


def test_invalid_arguments_raise():
    t = _lib()
    xy = synth.grid_xy(4)
    with pytest.raises(t.TLRQMCError) as e:
        t.block_reorder({"xy": xy, "beta": 0.1}, np.full(16, np.nan), np.ones(16), 4)
    assert e.value.status == t.EINVAL
    with pytest.raises(t.TLRQMCError):
        t.block_reorder({"xy": xy, "beta": -1.0}, np.zeros(16), np.ones(16), 4)
    with pytest.raises(t.TLRQMCError):
        t.block_reorder({"xy": xy, "beta": 0.1}, np.zeros(16), np.ones(16), 0)
