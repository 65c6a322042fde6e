"""The allocation-free distance map (tri_edm_noalloc) against tri_edm with a
caller workspace: same kernels, so the outputs must be identical bit for
bit, and both within the FP64 oracle's tolerance on sampled rows.  Two calls
in a row on the library's one scratch array, the second smaller (what the
first left in the scratch must not leak into the second)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import dev, host, note
from paper_1609_01490_amd import inputs

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
TOL = {0: None, 1: 1e-3, 2: None}


def _tm():
    from paper_1609_01490_amd import trimap
    return trimap


def _with_workspace(tm, p, xd, n, mode):
    import torch
    ws = torch.empty(max(1, p.edm_workspace_size(xd.shape[1], mode)), dtype=torch.uint8,
                     device="cuda")
    out = torch.full((n * (n - 1) // 2,), -1.0, dtype=torch.float32, device="cuda")
    p.edm(xd, out, mode=mode, ws=ws)
    return host(out)


def _check_sampled_rows(X, got, mode, seed):
    n, d = X.shape
    rng = np.random.default_rng(seed)
    rows = sorted(set([1, n - 1] + rng.choice(np.arange(1, n), 12, replace=False).tolist()))
    exp = oracle.edm_rows(X, rows)
    Xc = X.astype(np.float64) - X.astype(np.float64).mean(axis=0)
    nrm = np.sqrt((Xc ** 2).sum(axis=1))
    for r, e in zip(rows, exp):
        g = got[r * (r - 1) // 2: r * (r - 1) // 2 + r].astype(np.float64)
        if mode == 2:
            # single BF16: absolute bound 2^-7 (|x~_i| + |x~_j|)
            assert (np.abs(g - e) <= 2.0 ** -7 * (nrm[r] + nrm[:r])).all(), r
            continue
        tol = TOL[mode] if mode == 1 else (d + 2) * U / 2 + U
        nz = e > 0
        assert (np.abs(g[nz] - e[nz]) / e[nz] <= tol).all(), r


@pytest.mark.parametrize("mode", [1, 2, 0])
def test_noalloc_matches_workspace_entry_point(mode):
    import torch
    tm = _tm()
    for k, (n, d) in enumerate(((3000, 128), (1100, 40))):
        X, _ = inputs.points(n, d, dup_frac=0.01, seed=7100 + 10 * mode + k)
        p = tm.Plan(n, 128, "lambda", include_diag=False,
                    flags=tm.FLAG_XCD_SWIZZLE | tm.FLAG_ORDER_PAIRS)
        xd = dev(X)
        note("edm noalloc", mode, n, d)
        out = torch.full((n * (n - 1) // 2,), -1.0, dtype=torch.float32, device="cuda")
        p.edm_noalloc(xd, out, mode=mode)
        got = host(out)
        ref = _with_workspace(tm, p, xd, n, mode)
        assert (got.view(np.uint32) == ref.view(np.uint32)).all(), (mode, n, d)
        _check_sampled_rows(X, got, mode, seed=k)


def test_noalloc_rejects_beyond_scratch():
    import torch
    tm = _tm()
    n, d = 40000, 128
    p = tm.Plan(n, 128, "lambda", include_diag=False)
    assert p.edm_workspace_size(d, tm.EDM_BF16X3) > tm.EDM_NOALLOC_SCRATCH_BYTES
    x = torch.zeros((n, d), dtype=torch.float32, device="cuda")
    out = torch.full((n * (n - 1) // 2,), -1.0, dtype=torch.float32, device="cuda")
    note("edm noalloc too large", n, d)
    with pytest.raises(tm.TrimapError) as e:
        p.edm_noalloc(x, out, mode=tm.EDM_BF16X3)
    assert e.value.status == tm.E_RANGE
    torch.cuda.synchronize()
    assert bool((out[:1000] == -1.0).all()) and bool((out[-1000:] == -1.0).all())
