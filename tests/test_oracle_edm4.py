"""Pins of the oracle's four-feature distance map (the global-memory test of
Section 5, formula of the EDM paragraph of Section 5): SciPy's binary64
distances within the derived binary32 error bound, exact Pythagorean
quadruples (each feature slot distinct), the fixed summation order, and row
ranges.
"""
import numpy as np
from scipy.spatial.distance import pdist, squareform

import oracle

U32 = 2.0 ** -24


def test_edm4_within_binary32_bound_of_scipy():
    """Differences, squares, three additions and the square root each round
    once (relative u = 2^-24): |d32 - d| <= (1/2 (1 + 2 + 3) + 1) u d = 4u d
    to first order, so 4.5u with margin; the diagonal is exactly 0."""
    rng = np.random.default_rng(11)
    P = rng.random((300, 4), dtype=np.float32)
    P[7] = P[3]                      # exact duplicate
    got = oracle.edm4(P)
    ref = squareform(pdist(P.astype(np.float64)))
    low = np.tril(np.ones_like(ref, dtype=bool))
    err = np.abs(got[low].astype(np.float64) - ref[low])
    assert (err <= 4.5 * U32 * ref[low]).all(), err.max()
    assert (np.diag(got) == 0).all() and got[7, 3] == 0
    assert not got[~low].any()       # cells j > i untouched (fresh zeros)


def test_edm4_pythagorean_quadruples_exact():
    """Small integers: every step is exact, so d is the integer root.  The
    offsets put a different value in each feature slot, so a dropped, doubled
    or swapped feature changes the result."""
    base = np.array([3.0, 5.0, 11.0, 2.0], dtype=np.float32)
    offs = [((1, 2, 2, 0), 3), ((2, 3, 6, 0), 7), ((1, 4, 8, 0), 9), ((2, 4, 5, 6), 9),
            ((0, 0, 0, 5), 5), ((6, 2, 3, 0), 7), ((1, 1, 1, 1), 2), ((0, 2, 3, 6), 7)]
    P = np.stack([base] + [base + np.array(o, dtype=np.float32) for o, _ in offs])
    got = oracle.edm4(P)
    for k, (_, d) in enumerate(offs, start=1):
        assert got[k, 0] == np.float32(d), (k, got[k, 0], d)
    # (2,4,5,6) vs (1,1,1,1): diff (1,3,4,5) -> sqrt(51), correctly rounded
    assert got[7, 4] == np.float32(np.sqrt(np.float64(51)))


def test_edm4_summation_order_left_to_right():
    """dx = 1, dy = dz = dw = 2^-12: squares 1 and three times 2^-24 (exact).
    Left to right each addition ties back to 1 (round half to even), so d = 1;
    summing the small squares first would give 1 + 2^-23 after the root."""
    t = np.float32(2.0 ** -12)
    P = np.array([[0, 0, 0, 0], [1, t, t, t]], dtype=np.float32)
    got = oracle.edm4(P)
    assert got[1, 0] == np.float32(1.0)
    other = np.sqrt(np.float32(np.float32(3 * 2.0 ** -24) + np.float32(1.0)))
    assert other != np.float32(1.0)  # the order is observable


def test_edm4_row_range():
    rng = np.random.default_rng(5)
    P = rng.random((100, 4), dtype=np.float32)
    full = oracle.edm4(P)
    part = oracle.edm4(P, r0=40, r1=71)
    assert (part == full[40:71]).all()
