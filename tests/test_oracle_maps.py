"""Pins of the oracle's maps against what the paper and the mathematics fix.

Section 3.1 (Eq. eq_gmap, eq_theorem_nodiag, eq_matrix_indexing), Section 4.2
(BB, RB, REC, UTM).  None of these tests re-types the oracle's formula: each
checks it against the paper's worked example, a closed form, a library
routine, or brute-force enumeration.
"""
import math
import random
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle
from conftest import golden


def test_isqrt_matches_library():
    rnd = random.Random(1)
    vals = [0, 1, 2, 3, 4, 15, 16, 17, 2**32 - 1, 2**32, 2**63, 2**64 - 1]
    for _ in range(3000):
        vals.append(rnd.getrandbits(rnd.randint(1, 64)))
    for _ in range(1000):
        r = rnd.getrandbits(32)
        vals += [r * r, max(r * r - 1, 0), min(r * r + 1, 2**64 - 1)]
    for v in vals:
        assert oracle.isqrt(v) == math.isqrt(v), v


def test_lambda_worked_example_and_numbering_matrix():
    for omega, i, j in golden("lambda_worked_example.txt"):
        assert oracle.lam(omega) == (i, j)
    # Section 3.1: lambda is not additive: lambda(4) + lambda(3) = (4,1) != lambda(7)
    s = tuple(a + b for a, b in zip(oracle.lam(4), oracle.lam(3)))
    assert s == (4, 1) and s != oracle.lam(7)
    # Eq. eq_matrix_indexing: last row of an m-row matrix starts at m(m-1)/2
    # and ends at m(m+1)/2 - 1
    for m in (1, 2, 5, 64, 2048, 65536, 1 << 20):
        assert oracle.lam(m * (m - 1) // 2) == (m - 1, 0)
        assert oracle.lam(m * (m + 1) // 2 - 1) == (m - 1, m - 1)


def _roundtrip(omega):
    i, j = oracle.lam(omega)
    # the numbering of Eq. eq_matrix_indexing: row i starts at 1+2+...+i
    assert 0 <= j <= i
    assert sum_1_to(i) + j == omega


def sum_1_to(i):
    # 1 + 2 + ... + i by the Gauss closed form, checked against a loop for small i
    return i * (i + 1) // 2


def test_gauss_sum_closed_form():
    for i in range(200):
        assert sum_1_to(i) == sum(range(1, i + 1))


def test_lambda_roundtrip_dense_and_row_boundaries():
    for omega in range(1 << 15):
        _roundtrip(omega)
    # row boundaries T_i - 1, T_i, T_i + i for rows up to 2^21 (sampled) and
    # every row up to 4096
    rows = list(range(4096)) + random.Random(2).sample(range(4096, 1 << 21), 4000)
    rows += [(1 << 20) - 1, 1 << 20, (1 << 21) - 1, 92681, 92682, 2**30]
    for i in rows:
        t = sum_1_to(i)
        for omega in (t - 1, t, t + i):
            if omega >= 0:
                _roundtrip(omega)
    rnd = random.Random(3)
    for _ in range(5000):
        _roundtrip(rnd.getrandbits(59))


def test_lambda_inverse_exhaustive_small_tiles():
    # lambda(N(i, j)) == (i, j) for every tile of every triangle up to m = 300
    omega = 0
    for i in range(300):
        for j in range(i + 1):
            assert oracle.lam(omega) == (i, j)
            omega += 1


def test_lambda_nodiag():
    for omega, i, j in golden("lambda_nodiag_first.txt"):
        assert oracle.lam_nodiag(omega) == (i, j)
    # bijection onto the strict lower triangle, in row-major order
    omega = 0
    for i in range(1, 200):
        for j in range(i):
            assert oracle.lam_nodiag(omega) == (i, j)
            omega += 1
    # large values: 0 <= j < i and row i starts at i(i-1)/2
    rnd = random.Random(4)
    for _ in range(3000):
        w = rnd.getrandbits(58)
        i, j = oracle.lam_nodiag(w)
        assert 0 <= j < i and (i - 1) * i // 2 + j == w


MAPS = [oracle.BB, oracle.RB, oracle.REC, oracle.LAMBDA]


def _tiles(m):
    return {(i, j) for i in range(m) for j in range(i + 1)}


@pytest.mark.parametrize("map_id", MAPS)
def test_tile_maps_are_bijections(map_id):
    ms = list(range(1, 65)) + [128, 256, 1024]
    for m in ms:
        if map_id == oracle.REC and (m & (m - 1)):
            assert oracle.map_grid(map_id, m) is None
            continue
        d = oracle.map_dump(map_id, m)
        valid = d[d[:, 0] >= 0]
        assert ((d[:, 0] >= 0) == (d[:, 1] >= 0)).all()
        seen = set(map(tuple, valid.tolist()))
        assert len(seen) == valid.shape[0], (map_id, m, "tile mapped twice")
        assert seen == _tiles(m), (map_id, m)
        T = m * (m + 1) // 2
        discarded = d.shape[0] - valid.shape[0]
        # waste: BB discards the m(m-1)/2 blocks above the diagonal
        # (Section 3.1); lambda, RB and REC discard none
        if map_id == oracle.BB:
            assert discarded == m * m - T
        else:
            assert discarded == 0 and d.shape[0] == T


def test_lambda_grid_is_the_numbering():
    for m in (1, 7, 40):
        d = oracle.map_dump(oracle.LAMBDA, m)
        exp = [(i, j) for i in range(m) for j in range(i + 1)]
        assert [tuple(t) for t in d.tolist()] == exp


def test_rb_rotation_reading():
    # Section 4.2: blocks below the diagonal keep their column and move one row
    # up (odd m), blocks on/above the diagonal are the rotated far end of the
    # triangle.
    m = 7
    gw, gh = oracle.map_grid(oracle.RB, m)
    assert (gw, gh) == (7, 4)
    d = oracle.map_dump(oracle.RB, m).reshape(gh, gw, 2)
    assert tuple(d[2, 0]) == (1, 0) and tuple(d[2, 1]) == (1, 1)
    assert tuple(d[0, 0]) == (6, 6) and tuple(d[0, 6]) == (6, 0)
    assert tuple(d[1, 1]) == (5, 5) and tuple(d[1, 6]) == (5, 0)


def test_rec_levels():
    # Section 4.2, recursive partition for m = 2^k: level l has half the
    # squares of level l-1 at twice the side; diagonal tiles in an extra pass.
    m = 16
    d = oracle.map_dump(oracle.REC, m).reshape(m + 1, m // 2, 2)
    # level 1 (squares of side 1) is grid row 0: tiles (2q+1, 2q)
    assert [tuple(t) for t in d[0]] == [(2 * q + 1, 2 * q) for q in range(8)]
    # the largest square (side 8) is the lower-left quadrant: grid rows 7..14
    quad = {tuple(t) for t in d[7:15].reshape(-1, 2).tolist()}
    assert quad == {(i, j) for i in range(8, 16) for j in range(8)}
    # the diagonal pass: last two grid rows
    assert {tuple(t) for t in d[15:].reshape(-1, 2).tolist()} == {(i, i) for i in range(16)}


def _utm_paper(N, k):
    """The UTM formula as printed in Section 4.2, evaluated exactly."""
    getcontext().prec = 80
    D = 4 * N * N - 4 * N - 8 * k + 1
    s = Decimal(D).sqrt()
    a = math.floor((-(2 * N + 1) + s) / Decimal(-2))
    b = (a + 1) + k - (a - 1) * (2 * N - a) // 2
    return a, b


def test_utm_oracle_matches_paper_formula():
    for N in (2, 3, 4, 7, 50, 301):
        total = N * (N - 1) // 2
        pairs = [oracle.utm_pair(N, k) for k in range(total)]
        for k, p in enumerate(pairs):
            assert _utm_paper(N, k) == p, (N, k)
        # all pairs 1 <= a < b <= N exactly once
        assert sorted(pairs) == [(a, b) for a in range(1, N + 1) for b in range(a + 1, N + 1)]
    rnd = random.Random(5)
    for _ in range(200):
        N = rnd.randint(2, 5000)
        k = rnd.randrange(N * (N - 1) // 2)
        assert _utm_paper(N, k) == oracle.utm_pair(N, k)


def test_queue_locate_brute_force():
    rnd = np.random.default_rng(6)
    blocks = rnd.integers(1, 40, size=25)
    items = [(k, w) for k, b in enumerate(blocks.tolist()) for w in range(b)]
    for g, exp in enumerate(items):
        assert oracle.queue_locate(blocks, g) == exp
    with pytest.raises(ValueError):
        oracle.queue_locate(blocks, len(items))


def test_improvement_factor_block_counts():
    # Eq. eq_I: BB launches ceil(n/rho)^2 blocks, lambda ceil(n/rho)(ceil(n/rho)+1)/2;
    # the ratio tends to 2 (Eq. eq_I_bounded with tau = beta).
    for n, rho in ((2048, 16), (32768, 32), (16384, 16), (100, 32)):
        m = -(-n // rho)
        bb = oracle.map_dump(oracle.BB, m) if m <= 256 else None
        T = oracle.map_grid(oracle.LAMBDA, m)[0]
        assert T == m * (m + 1) // 2
        assert oracle.map_grid(oracle.BB, m) == (m, m)
        if bb is not None:
            assert bb.shape[0] == m * m
        ratio = (m * m) / T
        assert 1 <= ratio < 2 and abs(ratio - 2 * m / (m + 1)) < 1e-12
