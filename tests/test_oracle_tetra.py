"""Pins of the oracle's tetrahedral block map (Section 6) and of its
triangle counts (a triplet kernel over the tetrahedron): tetrahedral numbers
as binomial coefficients, the numbering enumerated by brute force, the
paper's closed-form root of the cubic, the 3-D bounding box, and triangle
counts against the trace identity of the cube of the adjacency matrix on
lattice points where every binary32 decision is exact."""
import math

import numpy as np

import oracle


def test_tet_is_binomial():
    for k in list(range(0, 200)) + [2**20, 2**21 + 5, 1_000_000]:
        assert oracle.tet(k) == math.comb(k + 2, 3)


def test_lambda3_is_the_layer_row_column_numbering():
    """Blocks numbered layer by layer (k), each layer's triangle row by row
    (j), each row by column (i): the enumeration and lambda3 agree."""
    w = 0
    for k in range(40):
        for j in range(k + 1):
            for i in range(j + 1):
                assert oracle.lam3(w) == (i, j, k), w
                w += 1
    assert w == oracle.tet(40)


def test_lambda3_layer_matches_the_cubic_root():
    """Section 6: the layer is the integer part of the real root x of
    x^3 + 3x^2 + 2x - 6 omega = 0 (Cardano form, omega >= 1; at omega = 0
    the printed form takes the root of a negative number)."""
    for w in list(range(1, 20000)) + [10**6 + 7, 123456789]:
        s = math.sqrt(729.0 * w * w - 3.0)
        c = (s + 27.0 * w) ** (1.0 / 3.0)
        x = c / 3.0 ** (2.0 / 3.0) + 1.0 / (3.0 ** (1.0 / 3.0) * c) - 1.0
        k = oracle.lam3(w)[2]
        assert k <= x + 1e-6 and x < k + 1, (w, x, k)
        assert x ** 3 + 3 * x ** 2 + 2 * x == np.float64(6 * w) or \
            abs(x ** 3 + 3 * x ** 2 + 2 * x - 6 * w) <= 1e-6 * 6 * w


def test_lambda3_large_round_trip():
    rng = np.random.default_rng(3)
    for w in rng.integers(0, 2**62, 2000).tolist() + [2**32 - 1, 2**32, 2**40 + 11]:
        i, j, k = oracle.lam3(w)
        assert 0 <= i <= j <= k
        assert oracle.tet(k) + j * (j + 1) // 2 + i == w
        assert oracle.tet(k + 1) > w


def test_bb3_keeps_exactly_the_tetrahedron():
    for m in (1, 2, 3, 7, 16):
        d = oracle.bb3_dump(m)
        kept = d[d[:, 0] >= 0]
        assert len(kept) == oracle.tet(m)
        assert len({tuple(t) for t in kept.tolist()}) == len(kept)
        assert ((kept[:, 0] <= kept[:, 1]) & (kept[:, 1] <= kept[:, 2])).all()
        assert len(d) == m ** 3   # m^3 - Tet(m) blocks are discarded


def _lattice(n, seed):
    """Coordinates k / 64 (k < 64): squared distances are exact multiples of
    2^-12, so with r2 = q / 4096 the binary32 test is the integer test
    sum (dk)^2 < q."""
    rng = np.random.default_rng(seed)
    K = rng.integers(0, 64, (n, 3)).astype(np.int64)
    P = np.zeros((n, 4), dtype=np.float32)
    P[:, :3] = K / 64.0
    return P, K


def test_triangles_equal_trace_identity_on_lattice():
    n, q = 300, 300
    P, K = _lattice(n, 5)
    counts, total = oracle.triangles(P, q / 4096.0)
    d2 = ((K[:, None, :] - K[None, :, :]) ** 2).sum(-1)
    A = (d2 < q).astype(np.int64)
    np.fill_diagonal(A, 0)
    A3 = A @ A @ A
    assert (counts == np.diag(A3) // 2).all()
    assert total == np.trace(A3) // 6
    assert total > 50
    ties = (d2 == q)
    np.fill_diagonal(ties, False)
    assert ties.any()                  # pairs at exactly r are present and are not neighbours


def test_triangles_one_equals_full():
    rng = np.random.default_rng(8)
    P = np.zeros((400, 4), dtype=np.float32)
    P[:, :3] = rng.random((400, 3), dtype=np.float32)
    r2 = np.float32(0.02)
    counts, total = oracle.triangles(P, r2)
    assert counts.sum() == 3 * total and total > 0
    for v in (0, 1, 200, 399):
        assert oracle.triangles_one(P, r2, v) == counts[v]
