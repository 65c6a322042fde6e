"""Pins of the oracle's kernel bodies: closed forms, library routines,
textbook Life patterns and an independent formulation.

Integer body (the dummy-kernel role, Section 4.1), single-precision a*X + Y^T,
Game of Life B3/S23 on a lower-triangular domain (cellular automata on
triangular domains, Section 1), Euclidean distance map (Section 5, EDM test).
"""
import numpy as np
import pytest
from scipy.spatial.distance import pdist, squareform

import oracle


# --------------------------------------------------------------------------
# integer body
# --------------------------------------------------------------------------

def _c0(A, B, fill=0x5A5A5A5A):
    n = A.shape[0]
    out = np.full((n, n), fill, dtype=np.uint32).view(np.int32)
    return oracle.c0(A, B, out).view(np.uint32)


def test_c0_closed_forms():
    n = 90
    idx = np.arange(n, dtype=np.uint64)
    ij = (idx[:, None] * idx[None, :]) & 0xFFFFFFFF
    low = np.tril(np.ones((n, n), dtype=bool))
    # A = all ones, B = 0: (A xor B) + ij = 2^32 - 1 + ij = ij - 1 (mod 2^32).
    # The other precedence, A xor (B + ij), would give ~ij.
    C = _c0(np.full(n, 0xFFFFFFFF, np.uint32), np.zeros(n, np.uint32))
    assert (C[low] == ((ij + 0xFFFFFFFF) & 0xFFFFFFFF)[low]).all()
    # A[i] = i, B = 0: i + i*j = i (j + 1); a swapped operand (A[j]) gives j (i + 1)
    C = _c0(idx.astype(np.uint32), np.zeros(n, np.uint32))
    assert (C[low] == (idx[:, None] * (idx[None, :] + 1))[low]).all()
    # A and B the same constant: the xor vanishes
    k = np.full(n, 0x9E3779B9, np.uint32)
    C = _c0(k, k.copy())
    assert (C[low] == ij[low]).all()
    r = np.random.default_rng(0).integers(0, 2**32, n, dtype=np.uint32)
    # upper triangle untouched, diagonal written
    C = _c0(r, r[::-1].copy())
    assert (C[~low] == 0x5A5A5A5A).all()
    assert (np.diag(C) == ((r ^ r[::-1]).astype(np.uint64) + idx * idx) % 2**32).all()


def test_c0_row_range():
    rng = np.random.default_rng(1)
    A = rng.integers(0, 2**32, 50, dtype=np.uint32)
    B = rng.integers(0, 2**32, 50, dtype=np.uint32)
    full = _c0(A, B)
    part = np.zeros((10, 50), dtype=np.int32)
    oracle.c0(A, B, part, 20, 30)
    low = np.tril(np.ones((50, 50), dtype=bool))[20:30]
    assert (part.view(np.uint32)[low] == full[20:30][low]).all()


# --------------------------------------------------------------------------
# single-precision body
# --------------------------------------------------------------------------

def _c1(a, X, Y):
    out = np.full(X.shape, np.nan, dtype=np.float32)
    return oracle.c1(a, X, Y, out)


def test_c1_matches_numpy_float32():
    rng = np.random.default_rng(2)
    n = 131
    X = (rng.random((n, n), dtype=np.float32) * 2 - 1).astype(np.float32)
    Y = (rng.random((n, n), dtype=np.float32) * 2 - 1).astype(np.float32)
    a = np.float32(1.25)
    C = _c1(a, X, Y)
    low = np.tril(np.ones((n, n), dtype=bool))
    # numpy float32 ufuncs: one rounding for the product, one for the sum
    ref = np.multiply(a, X, dtype=np.float32)
    ref = np.add(ref, Y.T, dtype=np.float32)
    assert (C.view(np.uint32)[low] == ref.view(np.uint32)[low]).all()
    assert np.isnan(C[~low]).all()
    # a value where fused and unfused results differ: a*x + y with the exact
    # product not representable (checks there is no contraction)
    x = np.float32(1 + 2**-12)
    y = np.float32(-(1 + 2**-11))
    X1 = np.array([[x]], dtype=np.float32)
    Y1 = np.array([[y]], dtype=np.float32)
    a1 = np.float32(1 + 2**-12)
    got = _c1(a1, X1, Y1)[0, 0]
    unfused = np.float32(np.float32(a1 * x) + y)
    fused = np.float32(np.float64(a1) * np.float64(x) + np.float64(y))
    assert unfused != fused and got == unfused


def test_c1_special_cases():
    rng = np.random.default_rng(3)
    n = 77
    X = rng.standard_normal((n, n)).astype(np.float32)
    Y = rng.standard_normal((n, n)).astype(np.float32)
    low = np.tril(np.ones((n, n), dtype=bool))
    assert (_c1(np.float32(0), X, Y)[low] == Y.T[low]).all()
    assert (_c1(np.float32(1), X, np.zeros_like(Y))[low] == X[low]).all()


# --------------------------------------------------------------------------
# Game of Life on the lower triangle
# --------------------------------------------------------------------------

def _place(n, cells, r0, c0):
    g = np.zeros((n, n), dtype=np.uint8)
    for r, c in cells:
        g[r0 + r, c0 + c] = 1
    return g


BLOCK = [(0, 0), (0, 1), (1, 0), (1, 1)]                 # still life
BLINKER_H = [(1, 0), (1, 1), (1, 2)]                     # period 2
BLINKER_V = [(0, 1), (1, 1), (2, 1)]
GLIDER = [(0, 1), (1, 2), (2, 0), (2, 1), (2, 2)]        # moves (+1, +1) per 4 gens


def test_life_textbook_patterns():
    n = 64
    g = _place(n, BLOCK, 40, 10)
    assert (oracle.gol(g, n, 7) == g).all()
    g = _place(n, BLINKER_H, 40, 10)
    assert (oracle.gol(g, n, 1) == _place(n, BLINKER_V, 40, 10)).all()
    assert (oracle.gol(g, n, 2) == g).all()
    g = _place(n, GLIDER, 30, 5)
    assert (oracle.gol(g, n, 4) == _place(n, GLIDER, 31, 6)).all()
    assert (oracle.gol(g, n, 20) == _place(n, GLIDER, 35, 10)).all()
    assert not oracle.gol(np.zeros((n, n), np.uint8), n, 5).any()


def test_life_domain_boundaries():
    n = 40
    # a horizontal blinker whose right cell is above the diagonal: that cell
    # is outside the domain (dead), the two remaining cells die of isolation
    g = _place(n, BLINKER_H, 19, 19)      # cells (20,19) (20,20) (20,21)
    assert (oracle.gol(g, n, 1) == 0).all()
    # at the bottom edge row n is outside the domain: a vertical pair on the
    # last two rows dies (no third cell below), a vertical blinker ending on
    # the last row still flips to horizontal
    g = _place(n, [(0, 1), (1, 1)], n - 2, 9)
    out = oracle.gol(g, n, 1)
    assert out.sum() == 0
    g = _place(n, BLINKER_V, n - 3, 9)
    out = oracle.gol(g, n, 1)
    assert (out == _place(n, [(1, 0), (1, 1), (1, 2)], n - 3, 9)).all()
    # a glider walking into the diagonal never creates cells above it
    g = _place(n, [(0, 1), (1, 2), (2, 0), (2, 1), (2, 2)], 10, 2)
    for s in range(1, 30):
        out = oracle.gol(g, n, s)
        assert not np.triu(out, 1).any()


def _life_numpy(g, steps):
    """Independent formulation: zero-padded shifted sums + lower mask."""
    n = g.shape[0]
    low = np.tril(np.ones((n, n), dtype=bool))
    cur = np.where(low, g, 0).astype(np.int32)
    for _ in range(steps):
        p = np.pad(cur, 1)
        cnt = sum(p[1 + dr:1 + dr + n, 1 + dc:1 + dc + n]
                  for dr in (-1, 0, 1) for dc in (-1, 0, 1) if dr or dc)
        cur = (((cnt == 3) | ((cur == 1) & (cnt == 2))) & low).astype(np.int32)
    return cur.astype(np.uint8)


@pytest.mark.parametrize("n,steps", [(1, 3), (2, 5), (37, 13), (160, 40)])
def test_life_matches_independent_formulation(n, steps):
    rng = np.random.default_rng(n)
    g = np.tril((rng.random((n, n)) < 0.3).astype(np.uint8))
    assert (oracle.gol(g, n, steps) == _life_numpy(g, steps)).all()


def test_life_upper_input_ignored_and_composition():
    n = 90
    rng = np.random.default_rng(7)
    g = np.tril((rng.random((n, n)) < 0.3).astype(np.uint8))
    noisy = g | np.triu((rng.random((n, n)) < 0.5).astype(np.uint8), 1)
    assert (oracle.gol(noisy, n, 9) == oracle.gol(g, n, 9)).all()
    # run(a) then run(b) == run(a + b)
    mid = oracle.gol(g, n, 11)
    assert (oracle.gol(mid, n, 14) == oracle.gol(g, n, 25)).all()


def test_life_window_light_cone():
    n, steps = 150, 12
    rng = np.random.default_rng(8)
    g = np.tril((rng.random((n, n)) < 0.3).astype(np.uint8))
    full = oracle.gol(g, n, steps)
    for (r, c) in [(100, 40), (149, 3), (80, 80), (60, 55), (12, 0)]:
        r0, c0 = r - steps, c - steps
        w = oracle.gol(g, n, steps, r0, c0, 2 * steps + 1, 2 * steps + 1)
        assert w[steps, steps] == full[r, c]


# --------------------------------------------------------------------------
# Euclidean distance map
# --------------------------------------------------------------------------

def test_edm_matches_scipy_pdist():
    rng = np.random.default_rng(9)
    for n, d in ((2, 1), (17, 4), (130, 33), (257, 128)):
        X = rng.random((n, d), dtype=np.float32)
        got = oracle.edm_condensed(X)
        D = squareform(pdist(X.astype(np.float64)))
        exp = D[np.tril_indices(n, -1)]   # row-major strict lower: (i, j), j < i
        np.testing.assert_allclose(got, exp, rtol=1e-13, atol=0)


def test_edm_integer_lattice_and_duplicates():
    X = np.zeros((4, 128), dtype=np.float32)
    X[1, 0], X[1, 1] = 3, 4          # |x1 - x0| = 5
    X[2, 5], X[2, 70] = 5, 12        # |x2 - x0| = 13
    X[3] = X[1]                      # exact duplicate of x1
    got = oracle.edm_condensed(X)
    # order: (1,0) (2,0) (2,1) (3,0) (3,1) (3,2)
    exp = [5.0, 13.0, np.sqrt(9 + 16 + 25 + 144), 5.0, 0.0, np.sqrt(9 + 16 + 25 + 144)]
    assert got.tolist() == exp


def test_edm_rows_subset():
    rng = np.random.default_rng(10)
    X = rng.random((60, 16), dtype=np.float32)
    full = oracle.edm_condensed(X)
    rows = [59, 3, 0, 30]
    parts = oracle.edm_rows(X, rows)
    for r, p in zip(rows, parts):
        assert (p == full[r * (r - 1) // 2: r * (r - 1) // 2 + r]).all()
