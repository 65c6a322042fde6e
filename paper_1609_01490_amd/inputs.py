"""Seeded synthetic inputs for the triangular-domain workloads.

This module only draws random data (numpy PCG64); it holds none of the
method's arithmetic.  The same arrays feed the HIP path and the CPU oracle.
Large arrays are filled in fixed chunks, each from its own child of the
array's SeedSequence, so the result depends only on (seed, shape), not on the
number of threads used to fill it.

Workloads (sizes of the defaults):
  * int32 elementwise: n = 2048, A and B uint32, C pre-filled with random bits.
  * fp32 elementwise:  n = 32768, X and Y uniform [-1, 1), a = 1.25.
  * Game of Life:      n = 16384 uint8, lower triangle Bernoulli(0.3), upper 0.
  * distance map:      n = 65536 points in d = 128, uniform [0, 1), 1 % of the
                       rows replaced by near-duplicates (copy + U[-1e-4, 1e-4)).
  * four-feature distances: n = 32768 points (x, y, z, w) uniform in [0, 1)^4.
  * collision detection: n = 131072 spheres, centres uniform in the unit
                       box (3-D, or 1-D on x), radii uniform in [0, r_max)
                       with r_max set for about 4 overlaps per sphere.
  * triangles (tetrahedral domain): n = 8192 points uniform in the unit
                       cube, neighbour radius for about 8 neighbours each.
  * batched:           512 instances, n log-uniform in [64, 8192]; even
                       instance index = distance map (d = 32), odd = Life
                       (density 0.3, 20 steps).
"""
from __future__ import annotations

import concurrent.futures as _cf
import os

import numpy as np

BASE_SEED = 160901490
_CHUNK = 1 << 24  # elements per independently seeded chunk


def seed_for(workload: int) -> int:
    return BASE_SEED + workload


def _streams(seed: int, count: int) -> list[np.random.SeedSequence]:
    return np.random.SeedSequence(seed).spawn(count)


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunked(out: np.ndarray, ss: np.random.SeedSequence, fill) -> np.ndarray:
    flat = out.reshape(-1)
    nchunks = max(1, -(-flat.size // _CHUNK))
    kids = ss.spawn(nchunks)

    def job(c):
        lo = c * _CHUNK
        hi = min(flat.size, lo + _CHUNK)
        fill(np.random.Generator(np.random.PCG64(kids[c])), flat[lo:hi])

    if nchunks == 1:
        job(0)
    else:
        with _cf.ThreadPoolExecutor(_workers()) as ex:
            list(ex.map(job, range(nchunks)))
    return out


def uniform_f32(shape, ss: np.random.SeedSequence, lo: float, hi: float) -> np.ndarray:
    """float32 uniform on [lo, hi): lo + (hi - lo) * U[0, 1) in float32."""
    out = np.empty(shape, dtype=np.float32)
    span, base = np.float32(hi - lo), np.float32(lo)

    def fill(g, a):
        g.random(out=a, dtype=np.float32)
        if span != 1:
            a *= span
        if base != 0:
            a += base

    return _chunked(out, ss, fill)


def random_bits(shape, ss: np.random.SeedSequence, dtype) -> np.ndarray:
    out = np.empty(shape, dtype=dtype)
    v = out.view(np.uint32) if np.dtype(dtype).itemsize == 4 else out.view(np.uint8)

    def fill(g, a):
        a[...] = g.integers(0, np.iinfo(a.dtype).max, size=a.shape, dtype=a.dtype,
                            endpoint=True)

    _chunked(v, ss, fill)
    return out


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def int_elementwise(n: int = 2048, seed: int | None = None, ld: int | None = None):
    """A, B uint32[n]; C0 int32[n, ld] pre-filled with random bits."""
    seed = seed_for(0) if seed is None else seed
    ld = n if ld is None else ld
    sa, sb, sc = _streams(seed, 3)
    A = random_bits((n,), sa, np.uint32)
    B = random_bits((n,), sb, np.uint32)
    C0 = random_bits((n, ld), sc, np.int32)
    return A, B, C0


def f32_elementwise(n: int = 32768, seed: int | None = None, ld: int | None = None,
                    with_fill: bool = True):
    """X, Y float32[n, ld] uniform [-1, 1); a = 1.25; C0 random bits (or None)."""
    seed = seed_for(1) if seed is None else seed
    ld = n if ld is None else ld
    sx, sy, sc = _streams(seed, 3)
    X = uniform_f32((n, ld), sx, -1.0, 1.0)
    Y = uniform_f32((n, ld), sy, -1.0, 1.0)
    C0 = random_bits((n, ld), sc, np.float32) if with_fill else None
    return np.float32(1.25), X, Y, C0


def life(n: int = 16384, density: float = 0.3, seed: int | None = None, ld: int | None = None):
    """uint8[n, ld]: lower-triangle cells alive with probability `density`,
    cells above the diagonal and in the padding 0."""
    seed = seed_for(2) if seed is None else seed
    ld = n if ld is None else ld
    (ss,) = _streams(seed, 1)
    u = uniform_f32((n, ld), ss, 0.0, 1.0)
    g = (u < np.float32(density)).astype(np.uint8)
    del u
    g[:, n:] = 0
    # upper triangle dead: zero cells with column > row
    rows = np.arange(n)[:, None]
    for r0 in range(0, n, 4096):
        blk = g[r0:r0 + 4096, :n]
        blk[np.arange(n)[None, :] > rows[r0:r0 + 4096]] = 0
    return g


def points(n: int = 65536, d: int = 128, dup_frac: float = 0.01, jitter: float = 1e-4,
           seed: int | None = None):
    """X float32[n, d] uniform [0, 1) with round(dup_frac*n) near-duplicate
    rows: each target row p is a copy of a non-target source row q plus a
    per-coordinate jitter U[-jitter, jitter).  Returns (X, pairs) with pairs
    an int64[k, 2] array of (p, q)."""
    seed = seed_for(3) if seed is None else seed
    sx, sd = _streams(seed, 2)
    X = uniform_f32((n, d), sx, 0.0, 1.0)
    g = np.random.Generator(np.random.PCG64(sd))
    k = int(round(dup_frac * n))
    if k == 0 or n < 2:
        return X, np.zeros((0, 2), dtype=np.int64)
    k = min(k, n // 2)
    perm = g.permutation(n)
    targets = np.sort(perm[:k])
    sources = perm[k:2 * k]
    jit = g.random((k, d), dtype=np.float32) * np.float32(2 * jitter) - np.float32(jitter)
    X[targets] = X[sources] + jit
    return X, np.stack([targets, sources], axis=1).astype(np.int64)


def points4(n: int = 32768, seed: int | None = None) -> np.ndarray:
    """P float32[n, 4]: points (x, y, z, w) uniform in the unit box [0, 1)^4
    (the four-feature distance test)."""
    seed = seed_for(5) if seed is None else seed
    (sp,) = _streams(seed, 1)
    return uniform_f32((n, 4), sp, 0.0, 1.0)


def spheres(n: int = 131072, dim: int = 3, mean_degree: float = 4.0,
            seed: int | None = None) -> np.ndarray:
    """S float32[n, 4] = (x, y, z, r): centres uniform in the unit box (in
    dim = 1 only x is drawn, y = z = 0) and radii uniform in [0, r_max).
    r_max sets the expected number of overlaps per sphere to about
    mean_degree, away from the box walls: two radii uniform in [0, R) have
    E[(r_a + r_b)^k] = R^k E[(u + v)^k], which is 1 for k = 1 and 3/2 for
    k = 3, so the pair probability is 2 R in 1-D and (4/3) pi (3/2) R^3 =
    2 pi R^3 in 3-D."""
    assert dim in (1, 3)
    seed = seed_for(6 if dim == 3 else 7) if seed is None else seed
    sc, sr = _streams(seed, 2)
    S = np.zeros((n, 4), dtype=np.float32)
    pairs_per = max(n - 1, 1)
    if dim == 3:
        S[:, :3] = uniform_f32((n, 3), sc, 0.0, 1.0)
        r_max = (mean_degree / (2.0 * np.pi * pairs_per)) ** (1.0 / 3.0)
    else:
        S[:, 0] = uniform_f32((n,), sc, 0.0, 1.0)
        r_max = mean_degree / (2.0 * pairs_per)
    S[:, 3] = uniform_f32((n,), sr, 0.0, float(r_max))
    return S


def points3(n: int = 8192, mean_degree: float = 8.0, seed: int | None = None):
    """P float32[n, 4] = (x, y, z, 0), points uniform in the unit cube, and
    the squared radius r2 (float32) that gives about mean_degree neighbours
    per point away from the walls: (n - 1) (4/3) pi r^3 = mean_degree."""
    seed = seed_for(8) if seed is None else seed
    (sp,) = _streams(seed, 1)
    P = np.zeros((n, 4), dtype=np.float32)
    P[:, :3] = uniform_f32((n, 3), sp, 0.0, 1.0)
    r = (3.0 * mean_degree / (4.0 * np.pi * max(n - 1, 1))) ** (1.0 / 3.0)
    return P, np.float32(r * r)


def batch_instances(count: int = 512, n_lo: int = 64, n_hi: int = 8192,
                    seed: int | None = None):
    """List of (kind, n) with kind 'edm' for even index and 'life' for odd,
    n = round(exp(U(ln n_lo, ln n_hi))) clamped to [n_lo, n_hi]."""
    seed = seed_for(4) if seed is None else seed
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    u = g.random(count)
    ns = np.rint(np.exp(np.log(n_lo) + u * (np.log(n_hi) - np.log(n_lo)))).astype(np.int64)
    ns = np.clip(ns, n_lo, n_hi)
    return [("edm" if k % 2 == 0 else "life", int(ns[k])) for k in range(count)]
