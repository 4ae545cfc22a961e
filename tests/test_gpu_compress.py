"""Device compression of the off-diagonal tiles (Section 3.3) against the
oracle's truncated SVD of the same dense factor: every tile's error
||L_ij - U V^T||_2 stays within the tolerance, ranks agree with the exact
SVD's to within one (a singular value within rounding of the tolerance may
fall either way), and V has orthonormal columns.

Cases: ragged last tile row (n = 2025, m = 128), a 512-wide tile with a
ragged row count (seven rows per lane in the QR kernel), and a tolerance so
small that some tiles need more QR steps than the device kernels hold:
those are compressed on the host, and the factor says how many.  Degenerate
cases: a one-row last tile, a tolerance above every tile's norm (all ranks
zero), and tiles of 64 and of 512 with a short last row of tiles.
"""

import numpy as np
import pytest

import synth
from oracle import factor as OF

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    from paper_2003_11183_amd import tlrqmc
    return tlrqmc


@pytest.fixture(scope="module")
def ctx(T):
    return T.Context(0)


def check_factor(T, ctx, g, beta, m, tol, cap=0, xy=None):
    xy = synth.grid_xy(g) if xy is None else xy
    n = len(xy)
    F = T.Factor.build(ctx, {"xy": xy, "beta": beta}, n, m, tol, cap)
    st = F.stats()
    perm, diag, ranks, U, V = F.export()
    F.free()
    L = np.linalg.cholesky(OF.exp_cov(xy, beta, perm))
    ref = OF.tlr_from_dense(L, m, tol, cap)
    sz = OF.tile_sizes(n, m)
    off = np.concatenate([[0], np.cumsum(sz)])
    worst = 0.0
    for i in range(len(sz)):
        assert np.allclose(np.tril(diag[i]), L[off[i]:off[i + 1], off[i]:off[i + 1]], rtol=0, atol=1e-12)
        for j in range(i):
            Tij = L[off[i]:off[i + 1], off[j]:off[j + 1]]
            k = int(ranks[i, j])
            assert U[(i, j)].shape == (sz[i], k) and V[(i, j)].shape == (sz[j], k)
            err = np.linalg.norm(Tij - U[(i, j)] @ V[(i, j)].T, 2)
            worst = max(worst, err / tol)
            if cap == 0 or k < cap:
                assert err <= tol * 1.01 + 1e-12, (i, j, k, err)
                assert abs(k - int(ref[1][i, j])) <= 1, (i, j, k, int(ref[1][i, j]))
            else:
                assert k == cap
            if k:
                assert np.allclose(V[(i, j)].T @ V[(i, j)], np.eye(k), rtol=0, atol=1e-9)
    print(f"n={n} m={m} tol={tol:g}: host tiles {st['host_tiles']} of {len(sz) * (len(sz) - 1) // 2}, "
          f"k_tot {st['k_tot']}, worst error / tol {worst:.3f}", flush=True)
    return st


def test_device_compression_ragged(T, ctx):
    st = check_factor(T, ctx, 45, 0.1, 128, 1e-5)
    assert st["host_tiles"] == 0


def test_device_compression_512_wide_tiles(T, ctx):
    # one 388 x 512 tile (seven rows per lane), about 80 QR steps
    st = check_factor(T, ctx, 30, 0.05, 512, 1e-2)
    assert st["n"] == 900 and st["host_tiles"] == 0


def test_device_compression_deep_tiles_go_to_host(T, ctx):
    st = check_factor(T, ctx, 32, 0.1, 256, 1e-9)
    assert 0 < st["host_tiles"] < 6


def test_device_compression_rank_cap(T, ctx):
    st = check_factor(T, ctx, 45, 0.1, 128, 1e-5, cap=8)
    assert st["cap_hits"] > 0 and st["host_tiles"] == 0


def test_device_compression_is_reproducible(T, ctx):
    xy = synth.grid_xy(40)
    sums = []
    for _ in range(2):
        F = T.Factor.build(ctx, {"xy": xy, "beta": 0.1}, 1600, 128, 1e-5)
        sums.append(F.stats()["checksum"])
        F.free()
    assert sums[0] == sums[1]


def test_device_compression_one_row_tile(T, ctx):
    # n = 129, m = 128: the only off-diagonal tile is 1 x 128
    st = check_factor(T, ctx, 0, 0.1, 128, 1e-5, xy=synth.grid_xy(12)[:129])
    assert st["r"] == 2 and st["host_tiles"] == 0


def test_device_compression_all_ranks_zero(T, ctx):
    # tolerance above every tile's norm: every off-diagonal tile has rank 0
    st = check_factor(T, ctx, 32, 0.1, 128, 10.0)
    assert st["k_tot"] == 0 and st["host_tiles"] == 0


@pytest.mark.parametrize("m", [64, 512])
def test_device_compression_short_last_tile_row(T, ctx, m):
    # n = 600: last tile row of 24 rows (m = 64) or 88 rows (m = 512)
    st = check_factor(T, ctx, 0, 0.3, m, 1e-3, xy=synth.grid_xy(25)[:600])
    assert st["host_tiles"] == 0
