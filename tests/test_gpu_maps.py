"""GPU parity of the maps: the device map must equal the oracle's map block
for block (tile maps) or thread for thread (UTM), and the device lambda must
be exact at every row boundary of the 32-bit range (Eq. eq_gmap)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import dev, host, note

pytestmark = pytest.mark.gpu

def _tm():
    from paper_1609_01490_amd import trimap
    return trimap


TILE_MAPS = ["bb", "rb", "rec", "lambda"]


@pytest.mark.parametrize("map_name", TILE_MAPS)
@pytest.mark.parametrize("tile", [8, 16, 32, 64])
def test_tile_map_dump_equals_oracle(map_name, tile):
    tm = _tm()
    for n in (1, 7, 8, 9, 100, 255, 256, 257, 1000, 2048, 4100):
        for diag in (True, False):
            ne = n if diag else n - 1
            m = -(-ne // tile)
            if map_name == "rec" and (m & (m - 1)):
                with pytest.raises(tm.TrimapError):
                    tm.Plan(n, tile, map_name, include_diag=diag)
                continue
            p = tm.Plan(n, tile, map_name, include_diag=diag)
            if p.info.grid_blocks == 0:
                continue
            note("map dump", map_name, tile, n, diag)
            got = host(p.dump())
            exp = oracle.map_dump(oracle.MAP_NAMES[map_name], m)
            assert got.shape == exp.shape
            assert (got == exp).all(), (map_name, tile, n, diag)


@pytest.mark.parametrize("flags", [8, 16, 17, 9])
def test_lambda_dispatch_orders_are_permutations(flags):
    tm = _tm()
    for n in (1, 100, 257, 2048, 5000):
        p = tm.Plan(n, 16, "lambda", flags=flags)
        note("order dump", flags, n)
        got = host(p.dump())
        exp = oracle.map_dump(oracle.LAMBDA, p.info.m)
        assert sorted(map(tuple, got.tolist())) == sorted(map(tuple, exp.tolist()))
        if flags == 8:       # reverse
            assert (got == exp[::-1]).all()
        if flags == 16:      # front, back, front + 1, back - 1, ...
            T = exp.shape[0]
            order = [(L // 2) if L % 2 == 0 else T - 1 - L // 2 for L in range(T)]
            assert (got == exp[order]).all()


@pytest.mark.parametrize("tile", [16, 32])
def test_lambda_xcd_swizzle_is_a_permutation(tile):
    tm = _tm()
    for n in (100, 257, 2048, 32768):
        p = tm.Plan(n, tile, "lambda", flags=tm.FLAG_XCD_SWIZZLE)
        note("swizzle dump", tile, n)
        got = host(p.dump())
        m = p.info.m
        exp = oracle.map_dump(oracle.LAMBDA, m)
        # same set of tiles, each once
        assert sorted(map(tuple, got.tolist())) == sorted(map(tuple, exp.tolist()))
        # XCD x (blocks b = x mod 8) walks a contiguous range of omega
        T = p.info.tiles
        omega = (got[:, 0] * (got[:, 0] + 1)) // 2 + got[:, 1]
        for x in range(8):
            w = omega[x::8]
            assert (np.diff(w) == 1).all()


def test_utm_dump_equals_oracle():
    tm = _tm()
    for n in (1, 2, 3, 10, 64, 100, 301):
        for diag in (True, False):
            p = tm.Plan(n, 32, "utm", include_diag=diag)
            if p.info.elements == 0:
                continue
            note("utm dump", n, diag)
            got = host(p.dump())
            N = n + 1 if diag else n
            exp = []
            for k in range(p.info.elements):
                a, b = oracle.utm_pair(N, k)
                exp.append((n - a, n + 1 - b) if diag else (n - a, n - b))
            assert (got == np.array(exp)).all(), (n, diag)


def _boundary_omegas():
    rows = np.arange(0, 92683, dtype=np.uint64)       # every row with T_i < 2^32
    T = rows * (rows + 1) // 2
    w = np.concatenate([T, T + rows, np.maximum(T, 1) - 1])
    rng = np.random.default_rng(11)
    w = np.concatenate([w, rng.integers(0, 2**32, 200000, dtype=np.uint64),
                        np.array([2**32 - 1, 2**32, 2**32 + 7, 2**40 + 3, 2**59 - 1],
                                 dtype=np.uint64),
                        rng.integers(2**32, 2**59, 2000, dtype=np.uint64)])
    return np.unique(w)


@pytest.mark.parametrize("flags", [0, 2, 4, 64])
def test_lambda_exact_at_row_boundaries(flags):
    tm = _tm()
    w = _boundary_omegas()
    note("lambda eval", flags, w.size)
    got = host(tm.lambda_eval(dev(w.view(np.int64)), True, flags))
    # oracle: integer square root (exact); checked row by row
    i = got[:, 0].astype(np.uint64)
    j = got[:, 1].astype(np.uint64)
    assert (got[:, 1] >= 0).all() and (j <= i).all()
    assert ((i * (i + 1) // 2 + j) == w).all()
    sample = np.random.default_rng(12).choice(w.size, 3000, replace=False)
    for s in sample:
        assert oracle.lam(int(w[s])) == tuple(got[s])


def test_lambda_nodiag_eval():
    tm = _tm()
    w = _boundary_omegas()[:300000]
    note("lambda nodiag eval", w.size)
    got = host(tm.lambda_eval(dev(w.view(np.int64)), False, 0))
    for s in np.random.default_rng(13).choice(w.size, 3000, replace=False):
        assert oracle.lam_nodiag(int(w[s])) == tuple(got[s])
    i = got[:, 0].astype(np.uint64)
    j = got[:, 1].astype(np.uint64)
    assert (j < i).all() and (((i - 1) * i // 2 + j) == w).all()


@pytest.mark.parametrize("base", [0, 2, 64])
def test_lambda_epsilon_variants_study(base):
    """The paper's inexact rows (TRI_FLAG_SQRT_EPS: +1e-4, no integer
    correction) with each FP32 square root.  Below T_1000 they are exact:
    there 1/4 + 2 omega is exact in FP32, the root is off by a few units in
    the last place (<= 2e-4) and the row boundaries are 2/(2i + 1) >= 1e-3
    apart from the nearest integer, so the epsilon only repairs roots that
    fall just short of an exact integer.  Higher up the gap shrinks below
    epsilon and the rounding of 2 omega grows, and they go wrong, though
    never by more than one row.  The corrected variants (test above) are
    exact everywhere."""
    tm = _tm()
    w = _boundary_omegas()
    w = w[w < 2**32]
    note("lambda eps eval", base, w.size)
    got = host(tm.lambda_eval(dev(w.view(np.int64)), True, base | tm.FLAG_SQRT_EPS))
    i = got[:, 0].astype(np.int64)
    wi = w.astype(np.int64)
    # the true row from the exact integer relation T_i <= w < T_{i+1}
    t = np.floor((np.sqrt(8.0 * w.astype(np.float64) + 1.0) - 1.0) / 2.0).astype(np.int64)
    t -= (t * (t + 1) // 2 > wi).astype(np.int64)
    t += ((t + 1) * (t + 2) // 2 <= wi).astype(np.int64)
    assert (np.abs(i - t) <= 1).all()
    small = wi < 1000 * 1001 // 2
    assert (i[small] == t[small]).all()
    wrong = w[i != t]
    note("eps variant", base, "wrong", wrong.size, "of", w.size,
         "first", int(wrong.min()) if wrong.size else None)
    assert wrong.size > 0


@pytest.mark.parametrize("map_name,flags", [("bb", 0), ("rb", 0), ("rec", 0), ("utm", 0),
                                            ("lambda", 0), ("lambda", 1), ("lambda", 2),
                                            ("lambda", 64), ("lambda", 4), ("lambda", 128),
                                            ("lambda", 130), ("lambda", 192), ("lambda", 16)])
@pytest.mark.parametrize("tile", [8, 16, 32, 64])
def test_dummy_kernel_reaches_every_sum(map_name, flags, tile):
    """Cells of the domain reach exactly the sums i + j in 0..2n-2 (with the
    diagonal) or 1..2n-3 (without); only a reached target is stored.  For
    lambda every root of the square-root study, with the correction and in
    the paper's epsilon form (exact at these sizes: below T_1000)."""
    import torch
    tm = _tm()
    for n, diag in ((1, True), (5, True), (100, True), (257, False), (300, True), (513, False)):
        m = -(-(n if diag else n - 1) // tile)
        if map_name == "rec" and m and (m & (m - 1)):
            continue
        p = tm.Plan(n, tile, map_name, include_diag=diag, flags=flags)
        lo, hi = (0, 2 * n - 2) if diag else (1, 2 * n - 3)
        for target in sorted({-1, 0, 1, lo, hi, hi + 1, n - 1, (lo + hi) // 2, 2 * n + 5}):
            note("dummy", map_name, flags, tile, n, diag, target)
            sink = torch.full((1,), -123, dtype=torch.int32, device="cuda")
            p.dummy(target, sink)
            exp = target if (lo <= target <= hi and n > (0 if diag else 1)) else -123
            assert int(host(sink)[0]) == exp, (map_name, tile, n, diag, target)


@pytest.mark.parametrize("n,tile,flags", [(65537, 8, 0), (65537, 8, 1), (50000, 8, 2)])
def test_lambda_two_dimensional_grid_dump(n, tile, flags):
    """More than 2^24 tiles: lambda is launched on a 2-D grid of 2^16-block
    rows (32-bit map path without flags, the general path with them); every
    block within T maps to lambda(L) and the surplus blocks are discarded."""
    tm = _tm()
    p = tm.Plan(n, tile, "lambda", flags=flags)
    assert p.info.tiles > 2 ** 24 and p.info.grid_y > 1
    note("lambda 2-D dump", n, tile, flags, p.info.tiles)
    got = host(p.dump())
    T = p.info.tiles
    L = np.arange(T, dtype=np.int64)
    if flags & tm.FLAG_XCD_SWIZZLE:
        # the swizzle permutes the grid blocks: the kept tiles are all of them
        kept = got[got[:, 0] >= 0]
        assert kept.shape[0] == T
        w = kept[:, 0] * (kept[:, 0] + 1) // 2 + kept[:, 1]
        assert (np.sort(w) == L).all()
        return
    i, j = got[:T, 0], got[:T, 1]
    assert ((j >= 0) & (j <= i)).all()
    assert (i * (i + 1) // 2 + j == L).all()
    assert (got[T:] == -1).all()
    for s in np.random.default_rng(1).choice(T, 2000, replace=False):
        assert oracle.lam(int(s)) == (int(i[s]), int(j[s]))
