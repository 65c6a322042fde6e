"""GPU parity of the triangular elementwise kernels against the oracle:
bit-exact on every cell of the domain, cells above the diagonal untouched,
for every map and tile size, ragged sizes, aligned (16-byte vector) and
unaligned (scalar) leading dimensions, and at full size (n = 32768 fp32)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import dev, host, note, padded_ld
from paper_1609_01490_amd import inputs

pytestmark = pytest.mark.gpu

MAPS = ["bb", "rb", "rec", "utm", "lambda"]
SIZES = [1, 2, 3, 17, 64, 100, 257, 300, 1024]


def _tm():
    from paper_1609_01490_amd import trimap
    return trimap


def _plan_or_none(tm, n, tile, map_name):
    m = -(-n // tile)
    if map_name == "rec" and (m & (m - 1)):
        return None
    return tm.Plan(n, tile, map_name)


def _low(n, ld):
    r = np.arange(n)[:, None]
    c = np.arange(ld)[None, :]
    return c <= r


@pytest.mark.parametrize("map_name", MAPS)
@pytest.mark.parametrize("tile", [8, 16, 32, 64, 128])
def test_xormul_i32_bit_exact(map_name, tile):
    tm = _tm()
    for n in SIZES:
        for ld in sorted({n, padded_ld(n), padded_ld(n) + 4}):
            p = _plan_or_none(tm, n, tile, map_name)
            if p is None:
                continue
            A, B, C0 = inputs.int_elementwise(n, seed=1000 + n, ld=ld)
            exp = C0.copy()
            oracle.c0(A, B, exp)
            note("xormul", map_name, tile, n, ld)
            c = dev(C0)
            p.elementwise(tm.OP_XORMUL_I32, dev(A), dev(B), c, ld=ld)
            got = host(c)
            assert (got.view(np.uint32) == exp.view(np.uint32)).all(), (map_name, tile, n, ld)


@pytest.mark.parametrize("map_name", MAPS)
@pytest.mark.parametrize("tile", [8, 16, 32, 64, 128])
def test_axpyt_f32_bit_exact(map_name, tile):
    tm = _tm()
    for n in SIZES:
        for ld in sorted({n, padded_ld(n)}):
            p = _plan_or_none(tm, n, tile, map_name)
            if p is None:
                continue
            a, X, Y, C0 = inputs.f32_elementwise(n, seed=2000 + n, ld=ld)
            exp = C0.copy()
            oracle.c1(a, X, Y, exp, n=n)
            note("axpyt", map_name, tile, n, ld)
            c = dev(C0)
            p.elementwise(tm.OP_AXPYT_F32, dev(X), dev(Y), c, ld=ld, a=float(a))
            got = host(c)
            assert (got.view(np.uint32) == exp.view(np.uint32)).all(), (map_name, tile, n, ld)


@pytest.mark.parametrize("map_name", ["bb", "rb", "rec", "lambda"])
@pytest.mark.parametrize("tile", [16, 32])
@pytest.mark.parametrize("strip,flags", [(0, 0), (2, 0), (4, 0), (5, 0), (4, 16), (4, 1),
                                         (4, 0x1000), (3, 0x1001), (2, 0x2000), (3, 0x2010),
                                         (5, 0x2001), (2, 0x8000), (4, 0x8000), (5, 0x8010),
                                         (3, 0x8001), (3, 0x9000)])
def test_axpyt_f32_strips_bit_exact(map_name, tile, strip, flags):
    """Workgroups of four waves walking strips of 1, 4, 16 and 32 tiles (each
    wave every fourth tile, its next tile's loads in flight), in row order
    or aligned to tile rows (column-major 0x1000, row-major 0x2000), over
    two-row bands (0x8000: at tile 16 a wave moves 2 x 2 blocks of tiles)
    and under the lambda orders: bit-exact at ragged n with 16-byte rows,
    the upper part untouched."""
    if map_name != "lambda" and flags & ~0x8000:
        pytest.skip("orders and column-major strips are lambda flags")
    tm = _tm()
    for n in (1, 17, 100, 257, 300, 1024, 1500):
        ld = padded_ld(n)
        m = -(-n // tile)
        if map_name == "rec" and (m & (m - 1)):
            continue
        p = tm.Plan(n, tile, map_name, flags=flags | tm.FLAG_STRIP(strip))
        a, X, Y, C0 = inputs.f32_elementwise(n, seed=2500 + n + tile, ld=ld)
        exp = C0.copy()
        oracle.c1(a, X, Y, exp, n=n)
        note("axpyt strips", map_name, tile, strip, flags, n, ld)
        c = dev(C0)
        p.elementwise(tm.OP_AXPYT_F32, dev(X), dev(Y), c, ld=ld, a=float(a))
        got = host(c)
        assert (got.view(np.uint32) == exp.view(np.uint32)).all(), (map_name, tile, strip, flags, n)


def test_band_strips_need_four_tiles():
    """Two-row band strips need strips of at least 4 tiles in the
    elementwise kernels; the distance map and the stencil refuse them."""
    import torch
    tm = _tm()
    n = 64
    a, X, Y, C0 = inputs.f32_elementwise(n, seed=7, ld=n)
    c = dev(C0)
    p = tm.Plan(n, 16, "lambda", flags=tm.FLAG_STRIP_BAND | tm.FLAG_STRIP(1))
    with pytest.raises(tm.TrimapError):
        p.elementwise(tm.OP_AXPYT_F32, dev(X), dev(Y), c, ld=n, a=float(a))
    pts = torch.rand((n, 4), device="cuda")
    out = torch.empty(n * (n - 1) // 2, device="cuda")
    with pytest.raises(tm.TrimapError):
        tm.Plan(n, 16, "lambda", include_diag=False,
                flags=tm.FLAG_STRIP_BAND | tm.FLAG_STRIP(2)).edm(pts, out, mode=tm.EDM_FP32)
    g = torch.zeros((n, n), dtype=torch.uint8, device="cuda")
    with pytest.raises(tm.TrimapError):
        tm.Plan(n, 16, "lambda", flags=tm.FLAG_STRIP_BAND | tm.FLAG_STRIP(2)).stencil(g, g.clone(), 1)


def test_empty_domain_is_a_no_op():
    import torch
    tm = _tm()
    p = tm.Plan(0, 16, "lambda")
    c = torch.zeros(4, device="cuda")
    p.elementwise(tm.OP_AXPYT_F32, c, c, c, ld=1, a=1.0)
    assert host(c).sum() == 0


def test_argument_errors():
    import torch
    tm = _tm()
    p = tm.Plan(64, 16, "lambda")
    x = torch.zeros((64, 64), device="cuda")
    with pytest.raises(tm.TrimapError) as e:
        p.elementwise(tm.OP_AXPYT_F32, x, x, x, ld=63, a=1.0)
    assert e.value.status == tm.E_INVAL
    with pytest.raises(tm.TrimapError) as e:
        p.elementwise(7, x, x, x, ld=64)
    assert e.value.status == tm.E_INVAL
    q = tm.Plan(64, 16, "lambda", include_diag=False)
    with pytest.raises(tm.TrimapError) as e:
        q.elementwise(tm.OP_AXPYT_F32, x, x, x, ld=64, a=1.0)
    assert e.value.status == tm.E_UNSUPPORTED


@pytest.fixture(scope="module")
def full_inputs():
    import torch
    n = 32768
    a, X, Y, _ = inputs.f32_elementwise(n, with_fill=False)
    note("axpyt full inputs", n)
    xd, yd = dev(X), dev(Y)
    yield n, a, X, Y, xd, yd
    del xd, yd
    torch.cuda.empty_cache()


@pytest.mark.slow
@pytest.mark.parametrize("map_name,tile,flags", [("lambda", 128, 16), ("lambda", 64, 16),
                                                 ("bb", 128, 0), ("lambda", 32, 0), ("bb", 32, 0),
                                                 ("lambda", 16, 0), ("lambda", 16, 0x500),
                                                 ("lambda", 32, 0x500), ("bb", 16, 0x500),
                                                 ("lambda", 16, 0x511), ("lambda", 32, 0x601),
                                                 ("lambda", 16, 0x2300), ("lambda", 32, 0x2410),
                                                 ("lambda", 16, 0x8510), ("lambda", 16, 0x8500),
                                                 ("bb", 16, 0x8500), ("lambda", 32, 0x8310)])
def test_axpyt_full_size_sampled_rows(full_inputs, map_name, tile, flags):
    """n = 32768 (12 GiB of operands), the configuration the benchmark times
    (lambda, tile 128, pairs order) and its neighbours; 64 sampled rows plus
    the first and last rows are checked bit for bit against the oracle, and
    the upper part of those rows is untouched."""
    import torch
    tm = _tm()
    n, a, X, Y, xd, yd = full_inputs
    note("axpyt full", map_name, tile, flags, n)
    fill = np.float32(-7.5)
    c = torch.full((n, n), float(fill), dtype=torch.float32, device="cuda")
    p = tm.Plan(n, tile, map_name, flags=flags)
    p.elementwise(tm.OP_AXPYT_F32, xd, yd, c, ld=n, a=float(a))
    torch.cuda.synchronize()
    rows = np.concatenate([[0, 1, n - 1], np.random.default_rng(14).choice(n, 64, replace=False)])
    for r in rows.tolist():
        got = c[r].cpu().numpy()
        exp = np.empty((1, n), dtype=np.float32)
        oracle.c1(a, X, Y, exp, r0=r, r1=r + 1)
        assert (got[: r + 1].view(np.uint32) == exp[0, : r + 1].view(np.uint32)).all(), r
        assert (got[r + 1:] == fill).all(), r
    # the upper triangle as a whole is untouched
    upper = torch.ones((1024, 1024), dtype=torch.bool, device="cuda").triu(1)
    for r0 in (0, 16384, n - 1024):
        blk = c[r0:r0 + 1024, r0:r0 + 1024]
        assert bool((blk[upper] == float(fill)).all())
    del c
    torch.cuda.empty_cache()


@pytest.mark.slow
@pytest.mark.parametrize("which", ["t128_pairs", "tuned"])
def test_axpyt_full_size_whole_triangle(full_inputs, which):
    """At n = 32768: the launch the benchmark timed before tile-16/32 strips
    existed (lambda, tile 128, pairs order) and the lambda launch the
    autotuner picks now (what the benchmark times): every cell of the lower
    triangle bit for bit against the oracle, which computes 1024-row bands
    on a thread pool (its C loop runs without the GIL); every cell above
    the diagonal keeps its pre-fill."""
    import concurrent.futures as cf
    import torch
    tm = _tm()
    n, a, X, Y, xd, yd = full_inputs
    if which == "tuned":
        tm.tune_cache_clear()
        _, table = tm.autotune(tm.TUNE_ELEMENTWISE_F32, n, 0, reps=3, use_cache=False)
        best = min((c for c in table if c["map"] == "lambda"), key=lambda c: c["ms"])
        tile, flags = best["tile"], best["flags"]
    else:
        tile, flags = 128, tm.FLAG_ORDER_PAIRS
    note("axpyt whole triangle", n, tile, flags)
    fill = np.float32(-7.5)
    c = torch.full((n, n), float(fill), dtype=torch.float32, device="cuda")
    tm.Plan(n, tile, "lambda", flags=flags).elementwise(tm.OP_AXPYT_F32, xd, yd, c, ld=n, a=float(a))
    torch.cuda.synchronize()
    got = c.cpu().numpy()
    del c
    torch.cuda.empty_cache()

    def band(r0):
        r1 = min(n, r0 + 1024)
        exp = np.empty((r1 - r0, n), dtype=np.float32)
        oracle.c1(a, X, Y, exp, r0=r0, r1=r1)
        low = np.arange(n)[None, :] <= np.arange(r0, r1)[:, None]
        g = got[r0:r1]
        bad = int((g.view(np.uint32)[low] != exp.view(np.uint32)[low]).sum())
        return bad, int((g[~low] != fill).sum())

    with cf.ThreadPoolExecutor(16) as ex:
        res = list(ex.map(band, range(0, n, 1024)))
    print(f"[axpyt whole triangle] tile {tile} flags {flags}: {len(res)} bands checked", flush=True)
    assert sum(r[0] for r in res) == 0, [r[0] for r in res]
    assert sum(r[1] for r in res) == 0, [r[1] for r in res]


def test_stream_add_probe_is_exact():
    import torch
    tm = _tm()
    a = torch.rand(1 << 20, device="cuda")
    b = torch.rand(1 << 20, device="cuda")
    c = torch.empty_like(a)
    note("stream add")
    tm.stream_add(c, a, b)
    assert torch.equal(c, a + b)
    with pytest.raises(tm.TrimapError):
        tm.stream_add(c[:5], a[:5], b[:5])


@pytest.mark.parametrize("unroll,threads,nt,wg", [(1, 256, True, 0), (4, 512, False, 0),
                                                  (8, 1024, True, 64), (2, 64, False, 3)])
def test_stream_probe_mixes_are_exact(unroll, threads, nt, wg):
    """Every mix of the bandwidth probe computes what it states (c = a + b,
    c = a, c filled with the target -1), over a count that is not a multiple
    of a chunk, with and without the persistent grid; the read probe writes
    nothing."""
    import torch
    tm = _tm()
    cnt = (1 << 18) + 4 * 37
    a = torch.rand(cnt, device="cuda")
    b = torch.rand(cnt, device="cuda")
    c = torch.full((cnt,), 7.0, device="cuda")
    note("stream probe", unroll, threads, nt, wg)
    tm.stream_probe(tm.PROBE_READ, c, a, None, unroll=unroll, threads=threads, nontemporal=nt,
                    workgroups=wg)
    assert bool((c == 7.0).all())
    tm.stream_probe(tm.PROBE_ADD, c, a, b, unroll=unroll, threads=threads, nontemporal=nt,
                    workgroups=wg)
    assert torch.equal(c, a + b)
    tm.stream_probe(tm.PROBE_COPY, c, b, None, unroll=unroll, threads=threads, nontemporal=nt,
                    workgroups=wg)
    assert torch.equal(c, b)
    tm.stream_probe(tm.PROBE_FILL, c, None, None, unroll=unroll, threads=threads,
                    nontemporal=nt, workgroups=wg)
    assert bool((c == -1.0).all())
    with pytest.raises(tm.TrimapError):
        tm.stream_probe(tm.PROBE_ADD, c, a, b, unroll=3)
