"""GPU parity of the Euclidean distance map against the FP64 oracle.

FP32 direct mode: each distance is a sum of d rounded squares of rounded
differences, accumulated with fused multiply-adds, then a correctly rounded
square root.  Relative error of the squared distance <= (d + 2) u with
u = 2^-24 (standard bound for a sum of non-negative terms), so the distance
itself is within (d + 2) u / 2 + u.  The test asserts that bound."""
import numpy as np
import pytest

import oracle
from gpu_helpers import dev, host, note
from paper_1609_01490_amd import inputs

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _tm():
    from paper_1609_01490_amd import trimap
    return trimap


def _fp32_bound(d):
    return (d + 2) * U / 2 + U


def _check_rows(X, out_host, rows, tol, dup_rows=()):
    exp = oracle.edm_rows(X, rows)
    worst = 0.0
    for r, e in zip(rows, exp):
        g = out_host[r * (r - 1) // 2: r * (r - 1) // 2 + r].astype(np.float64)
        nz = e > 0
        rel = np.abs(g[nz] - e[nz]) / e[nz]
        if rel.size:
            worst = max(worst, float(rel.max()))
        assert (g[~nz] <= 1e-6).all()
    assert worst <= tol, worst
    return worst


@pytest.mark.parametrize("map_name", ["bb", "rb", "rec", "lambda"])
@pytest.mark.parametrize("tile", [16, 32, 64, 128])
def test_edm_fp32_small(map_name, tile):
    import torch
    tm = _tm()
    for n in (2, 3, 50, 257, 700):
        for d in (1, 4, 33, 128):
            m = -(-(n - 1) // tile)
            if map_name == "rec" and (m & (m - 1)):
                continue
            X, _ = inputs.points(n, d, dup_frac=0.02, seed=4000 + n + d)
            p = tm.Plan(n, tile, map_name, include_diag=False)
            note("edm fp32", map_name, tile, n, d)
            out = torch.full((n * (n - 1) // 2,), -1.0, dtype=torch.float32, device="cuda")
            p.edm(dev(X), out, mode=tm.EDM_FP32)
            got = host(out)
            _check_rows(X, got, list(range(n)), _fp32_bound(d))


@pytest.mark.parametrize("tile", [32, 64, 128])
def test_edm_fp32_padded_rows(tile):
    """Coordinates with a leading dimension above d: a multiple of 4 (the
    16-byte staging of tiles 64 and 128), and not (the scalar staging)."""
    import torch
    tm = _tm()
    n, d = 300, 32
    for ldx in (32, 36, 37, 40):
        X, _ = inputs.points(n, d, dup_frac=0.02, seed=4500 + ldx)
        W = np.full((n, ldx), np.nan, dtype=np.float32)
        W[:, :d] = X
        xd = dev(W)[:, :d]
        assert xd.stride(0) == ldx
        note("edm fp32 padded", tile, ldx)
        out = torch.full((n * (n - 1) // 2,), -1.0, dtype=torch.float32, device="cuda")
        tm.Plan(n, tile, "lambda", include_diag=False).edm(xd, out, mode=tm.EDM_FP32)
        _check_rows(X, host(out), list(range(n)), _fp32_bound(d))


@pytest.mark.slow
@pytest.mark.parametrize("tile", [64, 128])
def test_edm_fp32_full_size_sampled_rows(tile):
    import torch
    tm = _tm()
    n, d = 65536, 128
    X, pairs = inputs.points(n, d)
    p = tm.Plan(n, tile, "lambda", include_diag=False)
    note("edm fp32 full", n, d, tile)
    out = torch.empty((n * (n - 1) // 2,), dtype=torch.float32, device="cuda")
    p.edm(dev(X), out, mode=tm.EDM_FP32)
    torch.cuda.synchronize()
    rng = np.random.default_rng(15)
    rows = sorted(set([1, 2, n - 1] + rng.choice(n, 24, replace=False).tolist()
                      + pairs[:8].max(axis=1).tolist()))
    for r in rows:
        g = out[r * (r - 1) // 2: r * (r - 1) // 2 + r].cpu().numpy()
        e = oracle.edm_rows(X, [r])[0]
        nz = e > 0
        rel = np.abs(g[nz].astype(np.float64) - e[nz]) / e[nz]
        assert rel.max() <= _fp32_bound(d), (r, rel.max())
    del out
    torch.cuda.empty_cache()


# --------------------------------------------------------------------------
# MFMA modes.  The distance map target is a maximum relative error of 1e-3
# against FP64: split BF16 (hi.hi + hi.lo + lo.hi, 16 significant bits per
# operand) is held to it.  Single BF16 rounds each centred coordinate to
# 8 significant bits (relative error <= 2^-8), so its distance error is
# absolute: |d_gpu - d| <= 2^-8 (|x~_i| + |x~_j|) plus FP32 accumulation;
# it is held to twice that.  Near-duplicates below the fix-up threshold are
# recomputed in FP32 and held to the FP32 bound.
# --------------------------------------------------------------------------

MFMA_TOL = {1: 1e-3}


def _check_rows_bf16(X, out_host, rows):
    Xc = X.astype(np.float64) - X.astype(np.float64).mean(axis=0)
    nrm = np.sqrt((Xc ** 2).sum(axis=1))
    exp = oracle.edm_rows(X, rows)
    for r, e in zip(rows, exp):
        g = out_host[r * (r - 1) // 2: r * (r - 1) // 2 + r].astype(np.float64)
        bound = 2.0 ** -7 * (nrm[r] + nrm[:r])
        assert (np.abs(g - e) <= bound).all(), r


def _edm_mfma(tm, p, X, mode, thr=1e-2):
    import torch
    n = X.shape[0]
    ws = torch.empty(p.edm_workspace_size(X.shape[1], mode), dtype=torch.uint8, device="cuda")
    out = torch.full((n * (n - 1) // 2,), -1.0, dtype=torch.float32, device="cuda")
    p.edm(dev(X), out, mode=mode, fixup_thr=thr, ws=ws)
    return out


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("map_name", ["bb", "lambda", "rb", "rec"])
def test_edm_mfma_small(mode, map_name):
    """Whole rows of every n against the FP64 oracle.  REC needs m (tiles
    per side) a power of two: n = 2..129 (m = 1), 130 and 257 (m = 2), 513
    (m = 4), 1025 (m = 8); the other maps also take n = 700 (m = 6)."""
    tm = _tm()
    for n in (2, 3, 50, 129, 130, 257, 513, 700, 1025):
        m = -(-(n - 1) // 128)
        if map_name == "rec" and (m & (m - 1)):
            continue
        if map_name != "rec" and n in (513, 1025):
            continue
        for d in (1, 4, 33, 128):
            X, pairs = inputs.points(n, d, dup_frac=0.02, seed=5000 + n + d)
            p = tm.Plan(n, 128, map_name, include_diag=False)
            note("edm mfma", mode, map_name, n, d)
            got = host(_edm_mfma(tm, p, X, mode))
            assert (got >= 0).all()
            if mode == 1:
                _check_rows(X, got, list(range(n)), MFMA_TOL[mode])
            else:
                _check_rows_bf16(X, got, list(range(n)))
            # near-duplicates go through the FP32 recompute
            exp = oracle.edm_rows(X, [int(max(a, b)) for a, b in pairs])
            for (a, b), e in zip(pairs.tolist(), exp):
                i, j = max(a, b), min(a, b)
                g = float(got[i * (i - 1) // 2 + j])
                if e[j] > 0 and e[j] ** 2 < 1e-2:
                    assert abs(g - e[j]) / e[j] <= _fp32_bound(d)


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("map_name,flags", [("lambda", 0), ("lambda", 1 | 16), ("lambda", 8),
                                            ("lambda", 0x1000), ("lambda", 0x1000 | 1),
                                            ("lambda", 0x1000 | 1 | 8), ("lambda", 0x2000),
                                            ("lambda", 0x2000 | 1 | 16),
                                            ("bb", 0), ("rb", 0), ("rec", 0)])
@pytest.mark.parametrize("strip", [1, 2, 5])
def test_edm_mfma_strips(mode, map_name, flags, strip):
    """Workgroups walking strips of 2, 4 and 32 consecutive tiles (row
    operands reloaded at each change of tile row, the carry of block 3 passed
    along the strip), in omega order or aligned to tile rows (column-major
    0x1000, row-major 0x2000): whole rows
    against the FP64 oracle at n where strips cross tile rows and end past the
    last tile.  REC at m = 8 and 16."""
    tm = _tm()
    cases = ((1025, 128), (2049, 33)) if map_name == "rec" else ((900, 128), (1500, 4), (2100, 40))
    for n, d in cases:
        X, pairs = inputs.points(n, d, dup_frac=0.02, seed=5100 + n + d + strip)
        p = tm.Plan(n, 128, map_name, include_diag=False, flags=flags | tm.FLAG_STRIP(strip))
        note("edm mfma strips", mode, map_name, flags, strip, n, d)
        got = host(_edm_mfma(tm, p, X, mode))
        assert (got >= 0).all()
        if mode == 1:
            _check_rows(X, got, list(range(n)), MFMA_TOL[mode])
        else:
            _check_rows_bf16(X, got, list(range(n)))
        # and identical to one tile per workgroup (same arithmetic per tile)
        q = tm.Plan(n, 128, map_name, include_diag=False, flags=flags | tm.FLAG_STRIP(0))
        one = host(_edm_mfma(tm, q, X, mode))
        assert (got.view(np.uint32) == one.view(np.uint32)).all()


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("map_name,flags", [("lambda", 0x1400), ("lambda", 0x1001), ("lambda", 0x2501),
                                            ("lambda", 0x0300), ("lambda", 0x0100), ("bb", 0x0400),
                                            ("rb", 0x0400), ("rec", 0x0300)])
def test_edm_pipe_kernel(mode, map_name, flags):
    """The pipelined kernel (TRI_FLAG_EDM_PIPE: one workgroup per CU, two
    tiles' column operands in LDS, each tile's stores inside the next
    tile's products): whole rows against the FP64 oracle, and bit for bit
    the line kernel's result, at n where strips start and end mid-row, the
    last tile row is ragged and d takes all three k-step counts."""
    tm = _tm()
    cases = ((1025, 128), (2049, 33)) if map_name == "rec" else ((900, 128), (1500, 4), (2100, 40),
                                                                  (1300, 64))
    for n, d in cases:
        X, _ = inputs.points(n, d, dup_frac=0.02, seed=5400 + n + d)
        p = tm.Plan(n, 128, map_name, include_diag=False, flags=flags | tm.FLAG_EDM_PIPE)
        note("edm pipe", mode, map_name, flags, n, d)
        got = host(_edm_mfma(tm, p, X, mode))
        assert (got >= 0).all()
        if mode == 1:
            _check_rows(X, got, list(range(n)), MFMA_TOL[mode])
        else:
            _check_rows_bf16(X, got, list(range(n)))
        q = tm.Plan(n, 128, map_name, include_diag=False, flags=flags)
        ref = host(_edm_mfma(tm, q, X, mode))
        assert (got.view(np.uint32) == ref.view(np.uint32)).all()


@pytest.mark.parametrize("mode", [1, 2])
def test_edm_mfma_beyond_128_dims(mode):
    """d above 128: the chunked kernel (row-major planes, 64 dimensions per
    LDS chunk)."""
    tm = _tm()
    for n, d in ((300, 129), (700, 200)):
        X, _ = inputs.points(n, d, dup_frac=0.02, seed=5300 + n + d)
        p = tm.Plan(n, 128, "lambda", include_diag=False)
        note("edm mfma wide", mode, n, d)
        got = host(_edm_mfma(tm, p, X, mode))
        if mode == 1:
            _check_rows(X, got, list(range(n)), MFMA_TOL[mode])
        else:
            _check_rows_bf16(X, got, list(range(n)))


def test_edm_mfma_exact_duplicates_are_zero():
    tm = _tm()
    n, d = 300, 64
    X, _ = inputs.points(n, d, dup_frac=0.0, seed=9)
    X[17] = X[250]
    X[299] = X[0]
    p = tm.Plan(n, 128, "lambda", include_diag=False)
    for mode in (1, 2):
        note("edm dup", mode)
        got = host(_edm_mfma(tm, p, X, mode))
        assert got[250 * 249 // 2 + 17] == 0.0
        assert got[299 * 298 // 2 + 0] == 0.0


def test_edm_mfma_argument_errors():
    import torch
    tm = _tm()
    p = tm.Plan(100, 64, "lambda", include_diag=False)
    with pytest.raises(tm.TrimapError) as e:
        p.edm_workspace_size(16, tm.EDM_BF16X3)
    assert e.value.status == tm.E_UNSUPPORTED
    q = tm.Plan(100, 128, "lambda", include_diag=False)
    x = torch.zeros((100, 16), device="cuda")
    out = torch.zeros(4950, device="cuda")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(tm.TrimapError) as e:
        q.edm(x, out, mode=tm.EDM_BF16X3, ws=small)
    assert e.value.status == tm.E_NOMEM


@pytest.mark.slow
@pytest.mark.parametrize("flags", [0, 1, 8, 16, 17])
def test_edm_bf16x3_full_size_sampled_rows(flags):
    """n = 65536, d = 128 with 1 % near-duplicates: 24 random rows plus the
    rows of 64 duplicate pairs, against the FP64 oracle; max relative error
    reported and held to 1e-3.  Flags: the lambda variants the autotuner
    times (plain, XCD swizzle, reverse, pairs, swizzle + pairs)."""
    import torch
    tm = _tm()
    n, d = 65536, 128
    X, pairs = inputs.points(n, d)
    p = tm.Plan(n, 128, "lambda", include_diag=False, flags=flags)
    note("edm bf16x3 full", n, d, flags)
    out = _edm_mfma(tm, p, X, tm.EDM_BF16X3)
    torch.cuda.synchronize()
    rng = np.random.default_rng(16)
    rows = sorted(set([1, 2, n - 1] + rng.choice(n, 24, replace=False).tolist()
                      + pairs[:64].max(axis=1).tolist()))
    worst = 0.0
    for r in rows:
        g = out[r * (r - 1) // 2: r * (r - 1) // 2 + r].cpu().numpy().astype(np.float64)
        e = oracle.edm_rows(X, [r])[0]
        nz = e > 0
        worst = max(worst, float((np.abs(g[nz] - e[nz]) / e[nz]).max()))
    print(f"[edm bf16x3 n={n} d={d}] max relative error {worst:.3e} over {len(rows)} rows",
          flush=True)
    assert worst <= 1e-3
    del out
    torch.cuda.empty_cache()


@pytest.mark.slow
def test_edm_bf16x3_4096_sampled_rows():
    """The distance-map workload's own accuracy check: n = 65536, d = 128
    with 1 % near-duplicates (jitter 1e-4), BF16X3 on the matrix cores with
    the FP32 recompute below d^2 = 1e-2; 4096 seeded random rows plus the
    row of every near-duplicate pair (all 655), whole rows, against the FP64
    oracle.  Max relative error printed and held to 1e-3; the near pairs
    themselves to the FP32 direct bound."""
    import concurrent.futures as cf
    import torch
    tm = _tm()
    n, d = 65536, 128
    X, pairs = inputs.points(n, d)
    p = tm.Plan(n, 128, "lambda", include_diag=False, flags=tm.FLAG_XCD_SWIZZLE)
    note("edm bf16x3 4096 rows", n, d)
    out = _edm_mfma(tm, p, X, tm.EDM_BF16X3)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4096)
    rows = sorted(set(rng.choice(np.arange(1, n), 4096, replace=False).tolist())
                  | set(pairs.max(axis=1).tolist()))
    chunks = [rows[k::16] for k in range(16)]
    with cf.ThreadPoolExecutor(8) as ex:  # the oracle's C loop runs without the GIL
        exp = dict(zip([r for c in chunks for r in c],
                       [e for es in ex.map(lambda c: oracle.edm_rows(X, c), chunks) for e in es]))
    worst, worst_near = 0.0, 0.0
    near = {}
    for a, b in pairs.tolist():
        near.setdefault(max(a, b), []).append(min(a, b))
    rels = []
    for k, r in enumerate(rows):
        g = out[r * (r - 1) // 2: r * (r - 1) // 2 + r].cpu().numpy().astype(np.float64)
        e = exp[r]
        nz = e > 0
        rel = np.abs(g[nz] - e[nz]) / e[nz]
        rels.append(rel.astype(np.float32))
        worst = max(worst, float(rel.max()))
        for j in near.get(r, ()):
            if e[j] > 0 and e[j] ** 2 < 1e-2:
                worst_near = max(worst_near, abs(g[j] - e[j]) / e[j])
        if k % 1024 == 0:
            print(f"[edm 4096 rows] {k}/{len(rows)} rows checked", flush=True)
    allrel = np.concatenate(rels)
    p999 = float(np.percentile(allrel, 99.9))
    print(f"[edm bf16x3 n={n} d={d}] max relative error {worst:.3e}, p99.9 {p999:.3e} over "
          f"{len(rows)} rows ({allrel.size} pairs; {len(near)} near-duplicate pairs: "
          f"{worst_near:.3e})", flush=True)
    assert worst <= 1e-3
    assert worst_near <= _fp32_bound(d)
    del out
    torch.cuda.empty_cache()



@pytest.mark.slow
@pytest.mark.parametrize("mode", [1, 2])
def test_edm_mfma_rec_full_size_sampled_rows(mode):
    """REC (m = 512 tiles per side, a power of two) at n = 65536, d = 128:
    the map the autotuner times among the MFMA candidates.  Whole sampled
    rows (first, last, 24 seeded random, 16 near-duplicate rows) against the
    FP64 oracle: BF16X3 within 1e-3, single BF16 within its absolute
    bound."""
    import torch
    tm = _tm()
    n, d = 65536, 128
    X, pairs = inputs.points(n, d)
    p = tm.Plan(n, 128, "rec", include_diag=False)
    note("edm rec full", mode, n, d)
    out = _edm_mfma(tm, p, X, mode)
    torch.cuda.synchronize()
    rng = np.random.default_rng(17)
    rows = sorted(set([1, 2, n - 1] + rng.choice(n, 24, replace=False).tolist()
                      + pairs[:16].max(axis=1).tolist()))
    sub = {r: out[r * (r - 1) // 2: r * (r - 1) // 2 + r].cpu().numpy() for r in rows}
    if mode == 1:
        for r, e in zip(rows, oracle.edm_rows(X, rows)):
            g = sub[r].astype(np.float64)
            nz = e > 0
            assert (np.abs(g[nz] - e[nz]) / e[nz]).max() <= 1e-3, r
    else:
        Xc = X.astype(np.float64) - X.astype(np.float64).mean(axis=0)
        nrm = np.sqrt((Xc ** 2).sum(axis=1))
        for r, e in zip(rows, oracle.edm_rows(X, rows)):
            g = sub[r].astype(np.float64)
            assert (np.abs(g - e) <= 2.0 ** -7 * (nrm[r] + nrm[:r])).all(), r
    del out
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def plain_edm():
    """The one-tile-per-workgroup full-size output of the last mode asked
    for, shared by the strip-order cases and freed after the module."""
    cache = {}
    yield cache
    cache.clear()
    import torch
    torch.cuda.empty_cache()


@pytest.mark.slow
@pytest.mark.parametrize("mode,flags", [(1, 0x1400), (1, 0x1401), (1, 0x1500), (1, 0x1501),
                                        (1, 0x1600), (1, 0x1601), (1, 0x5400), (1, 0x5500),
                                        (1, 0x5600), (2, 0x1500), (2, 0x1601)])
def test_edm_mfma_full_size_strip_orders(mode, flags, plain_edm):
    """n = 65536, d = 128 in the launch configurations the autotuner times
    for the distance map: lambda in column-major strips of 8, 16 and 32
    tiles aligned to tile rows, with and without the XCD swizzle, and the
    one-wave-per-SIMD kernel.  The whole output is bit-identical to one
    tile per workgroup (each tile's arithmetic is the same; only the order
    and the carried stores differ), and sampled whole rows (first, last, 8
    seeded random, 8 near-duplicate rows) meet the mode's bound against the
    FP64 oracle."""
    import torch
    tm = _tm()
    n, d = 65536, 128
    X, pairs = inputs.points(n, d)
    if plain_edm.get("mode") != mode:
        plain_edm.clear()
        torch.cuda.empty_cache()
        note("edm full plain", mode, n, d)
        plain_edm["mode"] = mode
        plain_edm["out"] = _edm_mfma(tm, tm.Plan(n, 128, "lambda", include_diag=False), X, mode)
    p = tm.Plan(n, 128, "lambda", include_diag=False, flags=flags)
    note("edm full strips", mode, hex(flags), n, d)
    out = _edm_mfma(tm, p, X, mode)
    torch.cuda.synchronize()
    assert torch.equal(out.view(torch.int32), plain_edm["out"].view(torch.int32))
    rng = np.random.default_rng(18 + flags)
    rows = sorted(set([1, n - 1] + rng.choice(np.arange(1, n), 8, replace=False).tolist()
                      + pairs[:8].max(axis=1).tolist()))
    sub = np.concatenate([out[r * (r - 1) // 2: r * (r - 1) // 2 + r].cpu().numpy()
                          for r in rows])
    offs = np.cumsum([0] + rows[:-1])
    view = {r: sub[o:o + r] for r, o in zip(rows, offs)}
    exp = oracle.edm_rows(X, rows)
    if mode == 1:
        for r, e in zip(rows, exp):
            g = view[r].astype(np.float64)
            nz = e > 0
            assert (np.abs(g[nz] - e[nz]) / e[nz]).max() <= 1e-3, r
    else:
        Xc = X.astype(np.float64) - X.astype(np.float64).mean(axis=0)
        nrm = np.sqrt((Xc ** 2).sum(axis=1))
        for r, e in zip(rows, exp):
            g = view[r].astype(np.float64)
            assert (np.abs(g - e) <= 2.0 ** -7 * (nrm[r] + nrm[:r])).all(), r
    del out
    torch.cuda.empty_cache()
