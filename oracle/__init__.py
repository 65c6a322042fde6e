"""CPU oracle for the triangular-domain hot path (arXiv 1609.01490).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the package entry module's
``smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import this
package.  The product path (``paper_1609_01490_amd``) never imports it and
shares no code with it.

The arithmetic lives in ``trimap_oracle.c`` (plain C, built with gcc); this
module only builds that file and marshals numpy arrays to it.  Every function
cites the passage of the paper it follows in the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "trimap_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# a prebuilt oracle library to load instead (the sanitizer test builds one)
_LIB_OVERRIDE = os.environ.get("TRIMAP_ORACLE_LIB")

BB, RB, REC, UTM, LAMBDA = 0, 1, 2, 3, 4
MAP_NAMES = {"bb": BB, "rb": RB, "rec": REC, "utm": UTM, "lambda": LAMBDA}


def build(force: bool = True, out: str | None = None, extra_flags=()) -> str:
    """Compile the oracle with gcc (no HIP, no shared headers); `out` and
    `extra_flags` build a variant elsewhere (e.g. with sanitizers)."""
    if out is not None:
        subprocess.check_call(
            ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
             *extra_flags, "-o", out, _SRC, "-lm"])
        return out
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = f"{_LIB}.tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_lib_lock = threading.Lock()


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    with _lib_lock:
        return _load()


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            build(force=False)
            L = ctypes.CDLL(_LIB)
        i64, u64, vp = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
        p64 = ctypes.POINTER(ctypes.c_int64)
        L.orc_isqrt.restype = u64
        L.orc_isqrt.argtypes = [u64]
        L.orc_lambda.argtypes = [u64, p64, p64]
        L.orc_lambda_nodiag.argtypes = [u64, p64, p64]
        L.orc_map_grid.restype = ctypes.c_int
        L.orc_map_grid.argtypes = [ctypes.c_int, i64, p64, p64]
        L.orc_map_tile.argtypes = [ctypes.c_int, i64, i64, i64, p64, p64]
        L.orc_map_dump.restype = i64
        L.orc_map_dump.argtypes = [ctypes.c_int, i64, vp]
        L.orc_utm_pair.restype = ctypes.c_int
        L.orc_utm_pair.argtypes = [i64, i64, p64, p64]
        L.orc_c0.argtypes = [i64, vp, vp, i64, i64, vp, i64]
        L.orc_c1.argtypes = [i64, ctypes.c_float, vp, vp, i64, i64, i64, vp, i64]
        L.orc_gol.restype = ctypes.c_int
        L.orc_gol.argtypes = [i64, vp, i64, i64, i64, i64, i64, ctypes.c_int, vp, i64]
        L.orc_edm_rows.argtypes = [i64, i64, vp, i64, vp, i64, vp]
        L.orc_edm4.argtypes = [i64, vp, i64, i64, vp, i64]
        L.orc_collide.argtypes = [i64, ctypes.c_int, vp, vp]
        L.orc_tet.restype = u64
        L.orc_tet.argtypes = [u64]
        L.orc_lambda3.argtypes = [u64, p64, p64, p64]
        L.orc_bb3_dump.restype = i64
        L.orc_bb3_dump.argtypes = [i64, vp]
        L.orc_triangles.argtypes = [i64, vp, ctypes.c_float, vp, ctypes.POINTER(u64)]
        L.orc_triangles_one.restype = ctypes.c_int32
        L.orc_triangles_one.argtypes = [i64, vp, ctypes.c_float, i64, vp]
        L.orc_collide_one.restype = ctypes.c_int32
        L.orc_collide_one.argtypes = [i64, ctypes.c_int, vp, i64]
        L.orc_queue_locate.restype = ctypes.c_int
        L.orc_queue_locate.argtypes = [i64, vp, i64, p64, p64]
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def isqrt(x: int) -> int:
    return int(lib().orc_isqrt(x))


def lam(omega: int) -> tuple[int, int]:
    """lambda(omega), diagonal included (Eq. eq_gmap)."""
    i, j = ctypes.c_int64(), ctypes.c_int64()
    lib().orc_lambda(omega, ctypes.byref(i), ctypes.byref(j))
    return i.value, j.value


def lam_nodiag(omega: int) -> tuple[int, int]:
    """lambda(omega), diagonal excluded (Eq. eq_theorem_nodiag, column read
    as omega - i(i-1)/2)."""
    i, j = ctypes.c_int64(), ctypes.c_int64()
    lib().orc_lambda_nodiag(omega, ctypes.byref(i), ctypes.byref(j))
    return i.value, j.value


def map_grid(map_id: int, m: int) -> tuple[int, int] | None:
    gw, gh = ctypes.c_int64(), ctypes.c_int64()
    if lib().orc_map_grid(map_id, m, ctypes.byref(gw), ctypes.byref(gh)):
        return None
    return gw.value, gh.value


def map_dump(map_id: int, m: int) -> np.ndarray:
    """(blocks, 2) int64 array: tile of every grid block (row-major), -1 if
    the block is discarded."""
    g = map_grid(map_id, m)
    if g is None:
        raise ValueError("map does not apply to this tile count")
    out = np.empty((g[0] * g[1], 2), dtype=np.int64)
    lib().orc_map_dump(map_id, m, _ptr(out))
    return out


def utm_pair(N: int, k: int) -> tuple[int, int]:
    a, b = ctypes.c_int64(), ctypes.c_int64()
    if lib().orc_utm_pair(N, k, ctypes.byref(a), ctypes.byref(b)):
        raise ValueError("k out of range")
    return a.value, b.value


def c0(A: np.ndarray, B: np.ndarray, out: np.ndarray, r0: int = 0, r1: int | None = None):
    """Integer body into out (rows r0..r1-1; int32, C-contiguous rows)."""
    n = A.shape[0]
    r1 = n if r1 is None else r1
    assert A.dtype == np.uint32 and B.dtype == np.uint32 and out.dtype == np.int32
    assert out.shape[0] >= r1 - r0 and out.strides[1] == 4
    lib().orc_c0(n, _ptr(A), _ptr(B), r0, r1, _ptr(out), out.strides[0] // 4)
    return out


def c1(a: float, X: np.ndarray, Y: np.ndarray, out: np.ndarray, r0: int = 0,
       r1: int | None = None, n: int | None = None):
    """Single-precision body a*X + Y^T into out (rows r0..r1-1)."""
    n = X.shape[0] if n is None else n
    r1 = n if r1 is None else r1
    assert X.dtype == np.float32 and Y.dtype == np.float32 and out.dtype == np.float32
    assert X.strides == Y.strides and X.strides[1] == 4 and out.strides[1] == 4
    lib().orc_c1(n, float(a), _ptr(X), _ptr(Y), X.strides[0] // 4, r0, r1, _ptr(out),
                 out.strides[0] // 4)
    return out


def edm4(P: np.ndarray, out: np.ndarray | None = None, r0: int = 0,
         r1: int | None = None) -> np.ndarray:
    """Four-feature binary32 distances |P_i - P_j| for rows r0..r1-1, j <= i
    (cells j > i of out untouched; a new out starts at zero)."""
    n = P.shape[0]
    r1 = n if r1 is None else min(r1, n)
    P = np.ascontiguousarray(P, dtype=np.float32)
    assert P.shape == (n, 4)
    if out is None:
        out = np.zeros((r1 - r0, n), dtype=np.float32)
    assert out.dtype == np.float32 and out.strides[1] == 4 and out.shape[0] >= r1 - r0
    lib().orc_edm4(n, _ptr(P), r0, r1, _ptr(out), out.strides[0] // 4)
    return out


def collide(S: np.ndarray, dim: int) -> np.ndarray:
    """Per-sphere overlap counts (int32[n]) for spheres S = (x, y, z, r)."""
    S = np.ascontiguousarray(S, dtype=np.float32)
    assert S.ndim == 2 and S.shape[1] == 4 and dim in (1, 3)
    out = np.zeros(S.shape[0], dtype=np.int32)
    lib().orc_collide(S.shape[0], dim, _ptr(S), _ptr(out))
    return out


def collide_one(S: np.ndarray, dim: int, k: int) -> int:
    """Overlap count of sphere k alone."""
    S = np.ascontiguousarray(S, dtype=np.float32)
    return int(lib().orc_collide_one(S.shape[0], dim, _ptr(S), int(k)))


def tet(k: int) -> int:
    """Tetrahedral number k(k+1)(k+2)/6."""
    return int(lib().orc_tet(k))


def lam3(omega: int) -> tuple[int, int, int]:
    """Tetrahedral lambda(omega) = (i, j, k), i <= j <= k."""
    i, j, k = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    lib().orc_lambda3(omega, ctypes.byref(i), ctypes.byref(j), ctypes.byref(k))
    return i.value, j.value, k.value


def bb3_dump(m: int) -> np.ndarray:
    """(i, j, k) per block of the m^3 bounding-box grid, -1 if discarded."""
    out = np.empty((m * m * m, 3), dtype=np.int64)
    lib().orc_bb3_dump(m, _ptr(out))
    return out


def triangles(P: np.ndarray, r2: float) -> tuple[np.ndarray, int]:
    """Per-point triangle counts of the neighbour graph, and the total."""
    P = np.ascontiguousarray(P, dtype=np.float32)
    assert P.ndim == 2 and P.shape[1] == 4
    counts = np.zeros(P.shape[0], dtype=np.int32)
    tot = ctypes.c_uint64()
    lib().orc_triangles(P.shape[0], _ptr(P), float(np.float32(r2)), _ptr(counts),
                        ctypes.byref(tot))
    return counts, tot.value


def triangles_one(P: np.ndarray, r2: float, v: int) -> int:
    """Triangle count of vertex v alone."""
    P = np.ascontiguousarray(P, dtype=np.float32)
    nb = np.empty(P.shape[0], dtype=np.int64)
    return int(lib().orc_triangles_one(P.shape[0], _ptr(P), float(np.float32(r2)), int(v),
                                       _ptr(nb)))


def gol(grid: np.ndarray, n: int, steps: int, r0: int = 0, c0_: int = 0,
        h: int | None = None, w: int | None = None) -> np.ndarray:
    """Triangular Game of Life B3/S23 on a window (whole domain by default)."""
    h = n if h is None else h
    w = n if w is None else w
    assert grid.dtype == np.uint8 and grid.strides[1] == 1
    out = np.zeros((h, w), dtype=np.uint8)
    rc = lib().orc_gol(n, _ptr(grid), grid.strides[0], r0, c0_, h, w, steps, _ptr(out), w)
    if rc:
        raise MemoryError("oracle gol")
    return out


def edm_rows(X: np.ndarray, rows) -> list[np.ndarray]:
    """FP64 distances d(r, 0..r-1) for each requested row r."""
    assert X.dtype == np.float32 and X.strides[1] == 4
    n, d = X.shape
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    total = int(rows.sum())
    out = np.empty(total, dtype=np.float64)
    lib().orc_edm_rows(n, d, _ptr(X), X.strides[0] // 4, _ptr(rows), rows.shape[0], _ptr(out))
    res, o = [], 0
    for r in rows.tolist():
        res.append(out[o:o + r])
        o += r
    return res


def edm_condensed(X: np.ndarray) -> np.ndarray:
    """Full condensed strict lower triangle, entry (i, j) at i(i-1)/2 + j."""
    n = X.shape[0]
    return np.concatenate(edm_rows(X, np.arange(n))) if n > 1 else np.zeros(0)


def queue_locate(blocks: np.ndarray, g: int) -> tuple[int, int]:
    blocks = np.ascontiguousarray(blocks, dtype=np.int64)
    k, w = ctypes.c_int64(), ctypes.c_int64()
    if lib().orc_queue_locate(blocks.shape[0], _ptr(blocks), g, ctypes.byref(k), ctypes.byref(w)):
        raise ValueError("g past the last item")
    return k.value, w.value
