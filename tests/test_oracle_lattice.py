"""Pins of the oracle's lattice: published constants and exact arithmetic."""

import os
from decimal import Decimal, getcontext

import numpy as np

from oracle import lattice


def _read(path):
    rows = []
    with open(path) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_splitmix64_published_outputs(golden_dir):
    for row in _read(os.path.join(golden_dir, "splitmix64.txt")):
        state = int(row[0])
        want = [int(h, 16) for h in row[1:]]
        assert lattice.splitmix64(state, len(want)) == want


def test_generators_match_fips_sqrt_fractions(golden_dir):
    rows = _read(os.path.join(golden_dir, "sqrt_prime_fractions.txt"))
    A = lattice.generators(len(rows))
    for c, (p, h) in enumerate(rows):
        assert lattice.primes(c + 1)[-1] == int(p)
        assert int(A[c]) == int(h, 16)


def test_generators_match_decimal_sqrt():
    getcontext().prec = 80
    ps = lattice.primes(300)
    A = lattice.generators(300)
    for c in list(range(0, 300, 7)) + [299]:
        r = Decimal(ps[c]).sqrt()
        frac = r - int(r)
        assert int(A[c]) == int(frac * (Decimal(2) ** 64))


def test_prime_count_known_values():
    ps = lattice.primes(10000)
    assert ps[:10] == [2, 3, 5, 7, 11, 13, 17, 19, 23, 29]
    assert ps[-1] == 104729          # the 10,000th prime


def test_points_exact_against_big_integers():
    A = lattice.generators(50)
    D = lattice.shifts(99, 3, 50)
    ks = np.array([1, 2, 3, 1000, 123456789, 2 ** 40 + 17], dtype=np.uint64)
    W = lattice.points(A, D[2], ks)
    for ci in (0, 1, 17, 49):
        for j, k in enumerate(ks):
            Wi = (int(k) * int(A[ci]) + int(D[2, ci])) % (1 << 64)
            want = ((Wi >> 12) + 0.5) / 2.0 ** 52
            assert W[ci, j] == want
            assert 2.0 ** -53 <= W[ci, j] <= 1 - 2.0 ** -53
    # w * 2^52 - 1/2 is an integer: the points are exact doubles
    t = W * 2.0 ** 52 - 0.5
    assert np.all(t == np.floor(t))


def test_shift_table_is_one_stream():
    D = lattice.shifts(7, 4, 5)
    flat = lattice.splitmix64(7, 20)
    assert [int(x) for x in D.ravel()] == flat


def test_lattice_equidistribution():
    # frac(k alpha) with irrational alpha is equidistributed: the mean of
    # N points is 1/2 + O(log N / N), far inside 1e-3 at N = 20000.
    A = lattice.generators(10)
    D = np.zeros((1, 10), dtype=np.uint64)
    W = lattice.points(A, D[0], np.arange(1, 20001))
    assert np.all(np.abs(W.mean(axis=1) - 0.5) < 1e-3)
    assert np.all(np.abs((W ** 2).mean(axis=1) - 1.0 / 3.0) < 1e-3)
