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
@pytest.mark.parametrize("tile", [16, 32, 64])
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


@pytest.mark.slow
def test_edm_fp32_full_size_sampled_rows():
    import torch
    tm = _tm()
    n, d = 65536, 128
    X, pairs = inputs.points(n, d)
    p = tm.Plan(n, 64, "lambda", include_diag=False)
    note("edm fp32 full", n, d)
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
