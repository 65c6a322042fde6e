"""GPU parity of the four-feature distance map (TRI_OP_EDM4_F32, the
global-memory distance test of Section 5) against the oracle: bit-exact on
every cell j <= i (the operation is one binary32 expression with a fixed
order and a correctly rounded root), cells above the diagonal untouched, for
all five maps and every tile size, ragged sizes, vector and scalar leading
dimensions, and sampled rows at the full size n = 32768."""
import numpy as np
import pytest

import oracle
from gpu_helpers import dev, host, note, padded_ld
from paper_1609_01490_amd import inputs

pytestmark = pytest.mark.gpu

MAPS = ["bb", "rb", "rec", "utm", "lambda"]
SIZES = [1, 2, 3, 17, 64, 100, 257, 300]


def _tm():
    from paper_1609_01490_amd import trimap
    return trimap


def _garbage(n, ld, seed):
    return np.random.default_rng(seed).integers(0, 2 ** 32, (n, ld), dtype=np.uint32).view(
        np.float32)


@pytest.mark.parametrize("map_name", MAPS)
@pytest.mark.parametrize("tile", [8, 16, 32, 64])
def test_edm4_bit_exact(map_name, tile):
    tm = _tm()
    for n in SIZES:
        m = -(-n // tile)
        if map_name == "rec" and (m & (m - 1)):
            continue
        P = inputs.points4(n, seed=4000 + n)
        P[n // 2] = P[0]                           # an exact duplicate pair
        p = tm.Plan(n, tile, map_name)
        for ld in sorted({n, padded_ld(n), padded_ld(n) + 4}):
            C0 = _garbage(n, ld, n * 7 + ld)
            exp = C0.copy()
            oracle.edm4(P, exp)
            note("edm4", map_name, tile, n, ld)
            c = dev(C0)
            p.elementwise(tm.OP_EDM4_F32, dev(P), None, c, ld=ld)
            got = host(c)
            assert (got.view(np.uint32) == exp.view(np.uint32)).all(), (map_name, tile, n, ld)


def test_edm4_rejects_unaligned_points():
    import torch
    tm = _tm()
    p = tm.Plan(8, 8, "lambda")
    P = torch.zeros(8 * 4 + 1, device="cuda")
    c = torch.zeros((8, 8), device="cuda")
    with pytest.raises(tm.TrimapError):
        p.elementwise(tm.OP_EDM4_F32, P[1:], None, c, ld=8)


@pytest.mark.slow
@pytest.mark.parametrize("map_name,tile,flags", [("lambda", 128, 16), ("lambda", 64, 0),
                                                 ("bb", 64, 0), ("rb", 64, 0), ("utm", 64, 0)])
def test_edm4_full_size_sampled_rows(map_name, tile, flags):
    """n = 32768, the launch the benchmark times: whole rows sampled at the
    start, the end, tile borders and at random, bit-exact; upper cells of the
    sampled rows keep their pre-fill."""
    import torch
    tm = _tm()
    n = 32768
    P = inputs.points4(n)
    note("edm4 full", map_name, tile, flags, n)
    c = torch.full((n, n), -1.0, device="cuda")
    tm.Plan(n, tile, map_name, flags=flags).elementwise(tm.OP_EDM4_F32, dev(P), None, c, ld=n)
    rng = np.random.default_rng(9)
    rows = sorted({0, 1, 63, 64, 65, n // 2, n - 65, n - 2, n - 1,
                   *rng.integers(0, n, 24).tolist()})
    for r in rows:
        exp = oracle.edm4(P, r0=r, r1=r + 1)[0]
        got = c[r].cpu().numpy()
        assert (got[:r + 1].view(np.uint32) == exp[:r + 1].view(np.uint32)).all(), r
        assert (got[r + 1:] == -1.0).all(), r
    del c
    torch.cuda.empty_cache()


@pytest.mark.slow
def test_edm4_full_size_whole_triangle():
    """The fastest launch of the four-feature benchmark (n = 32768, lambda,
    tile 128, pairs order): every cell of the triangle bit for bit against
    the oracle (1024-row bands on a thread pool), every cell above the
    diagonal keeps its pre-fill."""
    import concurrent.futures as cf
    import torch
    tm = _tm()
    n = 32768
    P = inputs.points4(n)
    note("edm4 whole triangle", n)
    c = torch.full((n, n), -1.0, device="cuda")
    tm.Plan(n, 128, "lambda", flags=tm.FLAG_ORDER_PAIRS).elementwise(
        tm.OP_EDM4_F32, dev(P), None, c, ld=n)
    torch.cuda.synchronize()
    got = c.cpu().numpy()
    del c
    torch.cuda.empty_cache()

    def band(r0):
        r1 = min(n, r0 + 1024)
        exp = oracle.edm4(P, r0=r0, r1=r1)
        low = np.arange(n)[None, :] <= np.arange(r0, r1)[:, None]
        g = got[r0:r1]
        return (int((g.view(np.uint32)[low] != exp.view(np.uint32)[low]).sum()),
                int((g[~low] != -1.0).sum()))

    with cf.ThreadPoolExecutor(16) as ex:
        res = list(ex.map(band, range(0, n, 1024)))
    print(f"[edm4 whole triangle] {len(res)} bands checked", flush=True)
    assert sum(r[0] for r in res) == 0, [r[0] for r in res]
    assert sum(r[1] for r in res) == 0, [r[1] for r in res]
