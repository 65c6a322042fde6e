"""GPU parity of the triangular Game of Life against the oracle: bit-exact
final grid, cells above the diagonal untouched whatever they hold, every tile
map and tile size, ragged sizes, odd and even step counts, and the full
16384 x 16384, 100-step case checked on light-cone windows."""
import numpy as np
import pytest

import oracle
from gpu_helpers import dev, host, note, padded_ld
from paper_1609_01490_amd import inputs

pytestmark = pytest.mark.gpu

MAPS = ["bb", "rb", "rec", "lambda", "utm"]


def _tm():
    from paper_1609_01490_amd import trimap
    return trimap


def _run(tm, p, g, steps, garbage_seed=None):
    """Run on device; the upper triangle of both buffers holds garbage that
    must be ignored and left untouched."""
    n, ld = g.shape
    cur = g.copy()
    nxt = np.zeros_like(g)
    if garbage_seed is not None:
        rng = np.random.default_rng(garbage_seed)
        up = np.triu(np.ones((n, ld), dtype=bool), 1)
        cur[up] = rng.integers(0, 256, up.sum(), dtype=np.uint8)
        nxt[up] = rng.integers(0, 256, up.sum(), dtype=np.uint8)
    up_cur, up_nxt = cur.copy(), nxt.copy()
    dc, dn = dev(cur), dev(nxt)
    p.stencil(dc, dn, steps, ld=ld)
    res = host(dc if steps % 2 == 0 else dn)
    other = host(dn if steps % 2 == 0 else dc)
    up = np.triu(np.ones((n, ld), dtype=bool), 1)
    assert (res[up] == (up_cur if steps % 2 == 0 else up_nxt)[up]).all(), "upper triangle written"
    assert (other[up] == (up_nxt if steps % 2 == 0 else up_cur)[up]).all(), "upper triangle written"
    return res


@pytest.mark.parametrize("map_name", MAPS)
@pytest.mark.parametrize("tile,multiple", [(8, 4), (16, 4), (32, 4), (64, 4), (64, 16)])
def test_life_bit_exact(map_name, tile, multiple):
    """One generation per launch; rows padded to 4 bytes, and for tile 64
    also to 16 (the bit-sliced one-generation kernel with 16-byte rows)."""
    tm = _tm()
    for n in (1, 2, 5, 33, 100, 257) + ((1000,) if multiple == 16 else ()):
        m = -(-n // tile)
        if map_name == "rec" and (m & (m - 1)):
            continue
        ld = padded_ld(n, multiple)
        g = inputs.life(n, 0.3, seed=3000 + n, ld=ld)
        p = tm.Plan(n, tile, map_name)
        for steps in (1, 2, 7):
            note("life", map_name, tile, n, steps)
            got = _run(tm, p, g, steps, garbage_seed=n + steps)
            exp = oracle.gol(g, n, steps)
            low = np.tril(np.ones((n, n), dtype=bool))
            assert (got[:, :n][low] == exp[low]).all(), (map_name, tile, n, steps)


def test_life_long_run_and_composition():
    tm = _tm()
    n = 300
    ld = padded_ld(n)
    g = inputs.life(n, 0.3, seed=77, ld=ld)
    p = tm.Plan(n, 32, "lambda")
    note("life long", n)
    got = _run(tm, p, g, 60)
    exp = oracle.gol(g, n, 60)
    low = np.tril(np.ones((n, n), dtype=bool))
    assert (got[:, :n][low] == exp[low]).all()
    half = _run(tm, p, g, 30)
    again = _run(tm, p, half, 30)
    assert (again == got).all()


def test_life_textbook_glider_on_device():
    tm = _tm()
    n = 128
    g = np.zeros((n, n), dtype=np.uint8)
    for r, c in [(0, 1), (1, 2), (2, 0), (2, 1), (2, 2)]:
        g[60 + r, 10 + c] = 1
    p = tm.Plan(n, 16, "lambda")
    note("glider")
    got = _run(tm, p, g, 8)
    exp = np.zeros_like(g)
    for r, c in [(0, 1), (1, 2), (2, 0), (2, 1), (2, 2)]:
        exp[62 + r, 12 + c] = 1
    assert (got == exp).all()


def test_life_errors():
    import torch
    tm = _tm()
    x = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    y = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    with pytest.raises(tm.TrimapError):  # UTM has no tile for temporal blocking
        tm.Plan(64, 16, "utm", flags=tm.FLAG_LIFE_TEMPORAL).stencil(x, y, 1)
    with pytest.raises(tm.TrimapError):
        tm.Plan(64, 16, "lambda").stencil(x, y, 1, ld=63)
    with pytest.raises(tm.TrimapError):
        tm.Plan(64, 16, "lambda").stencil(x, x, 1)


@pytest.mark.slow
@pytest.mark.parametrize("map_name,tile,flags", [("lambda", 32, 0), ("bb", 32, 0), ("utm", 16, 0),
                                                 ("lambda", 64, 0x12301), ("bb", 64, 0x10300),
                                                 ("lambda", 64, 0x301)])
def test_life_full_size_windows(map_name, tile, flags):
    """n = 16384, density 0.3, 100 steps, one generation per launch (tile 64
    with 16-byte rows: the bit-sliced strips, one tile per wave or with
    0x10000 neighbouring tiles in pairs).  The oracle recomputes 64 x 64
    cell blocks from their light cones (the initial state within 100
    cells): at the diagonal, the bottom edge, the left edge, a corner and
    inside."""
    import torch
    tm = _tm()
    n, steps = 16384, 100
    g = inputs.life(n, 0.3)
    note("life full", map_name, tile, flags, n, steps)
    cur = dev(g)
    nxt = torch.zeros_like(cur)
    p = tm.Plan(n, tile, map_name, flags=flags)
    p.stencil(cur, nxt, steps)
    res = cur if steps % 2 == 0 else nxt
    torch.cuda.synchronize()
    blocks = [(8000, 7970), (n - 64, 5000), (9000, 0), (n - 64, n - 64), (12000, 3000),
              (64, 0), (5000, 4990)]
    for (r, c) in blocks:
        h = w = 64
        win = oracle.gol(g, n, steps, r - steps, c - steps, h + 2 * steps, w + 2 * steps)
        exp = win[steps:steps + h, steps:steps + w]
        got = res[r:r + h, c:c + w].cpu().numpy()
        rr = np.arange(r, r + h)[:, None]
        cc = np.arange(c, c + w)[None, :]
        dom = cc <= rr
        assert (got[dom] == exp[dom]).all(), (r, c)
        assert not got[~dom].any(), (r, c)
    del cur, nxt
    torch.cuda.empty_cache()


@pytest.mark.parametrize("map_name,tile,multiple", [("lambda", 32, 4), ("utm", 32, 4),
                                                    ("lambda", 64, 16), ("bb", 64, 16)])
def test_life_graph_mode_matches_eager_and_replays(map_name, tile, multiple):
    """use_graph builds the generations into a hipGraph once per (buffers,
    steps) and replays it; every replay, with eager work in between, equals
    the eager launches and the oracle (tile 64 with 16-byte rows: the
    bit-sliced one-generation kernel in the graph)."""
    import torch
    tm = _tm()
    n, steps = 200, 6
    ld = padded_ld(n, multiple)
    g = inputs.life(n, 0.3, seed=5, ld=ld)
    p = tm.Plan(n, tile, map_name)
    eager = _run(tm, p, g, steps)
    cur, nxt = dev(g), torch.zeros((n, ld), dtype=torch.uint8, device="cuda")
    state = g.copy()
    low = np.tril(np.ones((n, n), dtype=bool))
    for rep in range(3):
        note("life graph replay", rep)
        p.stencil(cur, nxt, steps, ld=ld, use_graph=True)   # even steps: result in cur
        torch.cuda.synchronize()
        _ = torch.ones(100, device="cuda").sum().item()
        got = host(cur)[:, :n]
        state = np.pad(oracle.gol(state, n, steps), ((0, 0), (0, ld - n)))
        assert (got[low] == state[:, :n][low]).all(), rep
        if rep == 0:
            assert (got[low] == eager[:, :n][low]).all()


@pytest.mark.parametrize("map_name,flags", [("lambda", 0), ("lambda", 17), ("lambda", 0x2000),
                                            ("lambda", 0x1001), ("bb", 0), ("rb", 0), ("rec", 0),
                                            ("lambda", 0x10000), ("lambda", 0x12000),
                                            ("lambda", 0x12011), ("bb", 0x10000), ("rb", 0x10000),
                                            ("rec", 0x10000)])
@pytest.mark.parametrize("strip", [0, 2, 3, 5])
@pytest.mark.parametrize("temporal", [False, True])
def test_life_strips_bit_exact(map_name, flags, strip, temporal):
    """Tile 64 with 16-byte rows in strips of 1, 4, 8 and 32 tiles per
    workgroup (each wave its own tiles, or with 0x10000 neighbouring pairs
    of tiles as one 64 x 128 window): one generation per launch (eager and
    in a graph) and the temporal kernel, bit-exact against the oracle,
    upper triangle untouched."""
    import torch
    tm = _tm()
    fl = flags | tm.FLAG_STRIP(strip) | (tm.FLAG_LIFE_TEMPORAL if temporal else 0)
    for n in (1, 33, 200, 700, 1500):
        m = -(-n // 64)
        if map_name == "rec" and (m & (m - 1)):
            continue
        ld = padded_ld(n, 16)
        g = inputs.life(n, 0.3, seed=7000 + n + strip, ld=ld)
        p = tm.Plan(n, 64, map_name, flags=fl)
        low = np.tril(np.ones((n, n), dtype=bool))
        for steps in (1, 2, 5, 20):
            note("life strips", map_name, flags, strip, temporal, n, steps)
            got = _run(tm, p, g, steps, garbage_seed=n * 7 + steps)
            exp = oracle.gol(g, n, steps)
            assert (got[:, :n][low] == exp[low]).all(), (map_name, fl, n, steps)
        if not temporal and n == 700:
            cur, nxt = dev(g), torch.zeros((n, ld), dtype=torch.uint8, device="cuda")
            for rep in range(2):
                note("life strips graph", map_name, flags, strip, rep)
                p.stencil(cur, nxt, 4, ld=ld, use_graph=True)
                torch.cuda.synchronize()
                _ = torch.ones(100, device="cuda").sum().item()
            exp = oracle.gol(g, n, 8)
            assert (host(cur)[:, :n][low] == exp[low]).all()


@pytest.mark.parametrize("map_name", ["lambda", "bb", "rb"])
@pytest.mark.parametrize("tile", [16, 32, 64])
def test_life_temporal_blocking_bit_exact(map_name, tile):
    """Up to four generations per launch from a tile staged with a 4-cell
    halo: bit-exact against the oracle, upper triangle untouched, result in
    the buffer the one-step path uses (parity of the step count)."""
    tm = _tm()
    for n in (1, 5, 33, 100, 257):
        ld = padded_ld(n)
        g = inputs.life(n, 0.3, seed=6000 + n, ld=ld)
        p = tm.Plan(n, tile, map_name, flags=tm.FLAG_LIFE_TEMPORAL)
        for steps in (1, 2, 3, 4, 5, 7, 12):
            note("life temporal", map_name, tile, n, steps)
            got = _run(tm, p, g, steps, garbage_seed=n * 31 + steps)
            exp = oracle.gol(g, n, steps)
            low = np.tril(np.ones((n, n), dtype=bool))
            assert (got[:, :n][low] == exp[low]).all(), (map_name, tile, n, steps)


@pytest.mark.slow
def test_life_temporal_full_size_windows():
    import torch
    tm = _tm()
    n, steps = 16384, 100
    g = inputs.life(n, 0.3)
    note("life temporal full", n, steps)
    cur = dev(g)
    nxt = torch.zeros_like(cur)
    p = tm.Plan(n, 64, "lambda", flags=tm.FLAG_LIFE_TEMPORAL | tm.FLAG_XCD_SWIZZLE)
    p.stencil(cur, nxt, steps)
    torch.cuda.synchronize()
    for (r, c) in [(8000, 7970), (n - 64, 5000), (9000, 0), (n - 64, n - 64), (64, 0)]:
        win = oracle.gol(g, n, steps, r - steps, c - steps, 64 + 2 * steps, 64 + 2 * steps)
        exp = win[steps:steps + 64, steps:steps + 64]
        got = cur[r:r + 64, c:c + 64].cpu().numpy()
        dom = np.arange(c, c + 64)[None, :] <= np.arange(r, r + 64)[:, None]
        assert (got[dom] == exp[dom]).all(), (r, c)
        assert not got[~dom].any(), (r, c)


def _gol_whole(g, n, steps, bands=16):
    """The oracle's final grid of the whole domain, computed in row bands
    (each from its light cone: the band plus `steps` rows and columns
    around it) on a thread pool; the oracle's C loop runs without the GIL."""
    import concurrent.futures as cf
    h = -(-n // bands)

    def band(r):
        hh = min(h, n - r)
        w = min(n, r + hh)  # columns j <= i < r + hh
        win = oracle.gol(g, n, steps, r - steps, -steps, hh + 2 * steps, w + 2 * steps)
        return r, win[steps:steps + hh, steps:steps + w]

    out = np.zeros((n, n), dtype=np.uint8)
    with cf.ThreadPoolExecutor(16) as ex:
        for r, blk in ex.map(band, range(0, n, h)):
            out[r:r + blk.shape[0], :blk.shape[1]] = blk
            print(f"[life whole grid] rows {r}..{r + blk.shape[0]} from the oracle", flush=True)
    return out


_WHOLE = {}


@pytest.mark.slow
@pytest.mark.parametrize("flags", [0x21, 0x31, 0x12421, 0x12431])
def test_life_temporal_full_size_whole_grid(flags):
    """The benchmarked launches (n = 16384, density 0.3, 100 generations,
    lambda tile 64, temporal blocking: the bit-sliced kernels, one tile per
    workgroup with the XCD swizzle and pairs order, or in aligned strips of
    8 with neighbouring tiles moved in pairs): the whole final grid, bit
    for bit, against the oracle's (computed once for all of them)."""
    import torch
    tm = _tm()
    n, steps = 16384, 100
    g = inputs.life(n, 0.3)
    note("life temporal whole grid", n, steps, flags)
    cur = dev(g)
    nxt = torch.zeros_like(cur)
    p = tm.Plan(n, 64, "lambda", flags=flags)
    p.stencil(cur, nxt, steps)
    torch.cuda.synchronize()
    got = cur.cpu().numpy()
    del cur, nxt
    torch.cuda.empty_cache()
    if "exp" not in _WHOLE:
        _WHOLE["exp"] = _gol_whole(g, n, steps)
    exp = _WHOLE["exp"]
    bad = np.argwhere(got != exp)
    assert bad.shape[0] == 0, (bad.shape[0], bad[:4].tolist())


@pytest.mark.parametrize("steps", [1, 4, 7, 15, 16, 32])
@pytest.mark.parametrize("multiple", [4, 16])
@pytest.mark.parametrize("n", [181 * 64 + 3, 33 * 64 + 5])
def test_life_bit_sliced_whole_grid(steps, multiple, n):
    """Grids with a ragged last tile row: n = 181 * 64 + 3 (>= 16384 tiles:
    the bit-sliced one-wave kernel for either row padding) and
    n = 33 * 64 + 5 (595 tiles: bit-sliced with 16-byte rows, byte-sliced
    otherwise), the leading dimension padded to a multiple of 4 (rows moved
    byte by byte, up to 4 generations per launch) or of 16 (16-byte row
    loads and stores, up to 16 generations per launch: 15 steps are one
    launch of 15, 32 steps two of 16): the whole final
    grid against the oracle's, and nothing written above the diagonal or in
    the padding."""
    import torch
    tm = _tm()
    ld = padded_ld(n, multiple)
    g = inputs.life(n, 0.3, seed=900 + steps, ld=ld)
    g[:, n:] = 0
    p = tm.Plan(n, 64, "lambda", flags=tm.FLAG_LIFE_TEMPORAL | tm.FLAG_XCD_SWIZZLE)
    assert p.info.tiles >= 512
    note("life bit-sliced whole grid", n, ld, steps)
    cur = dev(g)
    nxt = torch.zeros_like(cur)
    p.stencil(cur, nxt, steps, ld=ld)
    res = (cur if steps % 2 == 0 else nxt).cpu().numpy()
    exp = _gol_whole(g, n, steps)
    bad = np.argwhere(res[:, :n] != exp)
    assert bad.shape[0] == 0, (bad.shape[0], bad[:4].tolist())
    assert not res[:, n:].any()
