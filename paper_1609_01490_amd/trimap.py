"""Python binding of libtrimap.so: argument marshalling only.

Every step of the triangular-domain path runs in the HIP library; this module
turns torch tensors into device pointers, picks the current HIP stream, and
turns a non-zero tri_status into an exception.  PyTorch provides device
memory and streams, nothing else.  There is no fallback: if the library is
missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtrimap.so")

BB, RB, REC, UTM, LAMBDA = 0, 1, 2, 3, 4
MAPS = {"bb": BB, "rb": RB, "rec": REC, "utm": UTM, "lambda": LAMBDA}
MAP_NAMES = {v: k for k, v in MAPS.items()}

FLAG_XCD_SWIZZLE, FLAG_SQRT_RSQ, FLAG_SQRT_F64 = 1, 2, 4
FLAG_ORDER_REVERSE, FLAG_ORDER_PAIRS, FLAG_LIFE_TEMPORAL = 8, 16, 32
FLAG_SQRT_NEWTON, FLAG_SQRT_EPS = 64, 128
FLAG_STRIP_MASK = 0xF00


def FLAG_STRIP(k: int) -> int:
    """Plan flag: strips of 2^k consecutive tiles per workgroup (k = 0..5)."""
    return (k + 1) << 8


FLAG_STRIP_COLS = 0x1000  # lambda strips aligned to tile rows, taken column by column
FLAG_STRIP_ALIGN = 0x2000  # lambda strips aligned to tile rows, taken row by row
FLAG_STRIP_BAND = 0x8000  # elementwise strips over two-row bands (2 x 2 tile blocks)
FLAG_LIFE_WIDE = 0x10000  # bit-sliced Life strips: neighbouring tiles moved in pairs
FLAG_EDM_PIPE = 0x4000  # distance map: the pipelined matrix-core kernel
OP_XORMUL_I32, OP_AXPYT_F32, OP_EDM4_F32 = 0, 1, 2
EDM_FP32, EDM_BF16X3, EDM_BF16 = 0, 1, 2
EDM_NOALLOC_SCRATCH_BYTES = 16 << 20
KIND_EDM, KIND_LIFE = 0, 1
TUNE_ELEMENTWISE_F32, TUNE_ELEMENTWISE_I32, TUNE_LIFE, TUNE_EDM_FP32, TUNE_EDM_BF16X3 = range(5)
BATCH_GRAPH, BATCH_STREAM, BATCH_PER_INSTANCE = 0, 1, 2

OK, E_INVAL, E_RANGE, E_NOMEM, E_HIP, E_UNSUPPORTED = range(6)


class TrimapError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{status_str(status)}: {msg}")
        self.status = status


class TrimapArgError(TrimapError, ValueError):
    """A tensor argument the binding refuses before any device pointer is
    passed on: wrong device, dtype or layout, or a buffer smaller than the
    extent the call touches (the C side sees bare pointers and cannot check
    extents).  Status TRI_E_INVAL."""

    def __init__(self, msg: str):
        super().__init__(E_INVAL, msg)


class tri_plan_info(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "n", "tile", "m", "tiles", "grid_x", "grid_y", "grid_blocks", "wasted_blocks",
        "elements", "dump_entries")] + [
        ("map", ctypes.c_int32), ("include_diag", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32)]


class tri_batch_info(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in (
        "count", "life_instances", "edm_tile", "life_tile", "life_steps",
        "persistent_workgroups", "graph_nodes", "reserved")] + [
        ("items_generation0", ctypes.c_int64), ("items_per_later_generation", ctypes.c_int64)]


class tri_tune_choice(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("map", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("ms", ctypes.c_float)]


def _load() -> ctypes.CDLL:
    # torch owns the device memory and the streams handed to the library, so
    # the library must resolve libamdhip64.so.7 to the HIP runtime torch has
    # loaded (same soname): import torch before the library is opened.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1609_01490_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    i64, u32, vp, i32 = ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int
    st = ctypes.c_int
    L.tri_map_plan.restype = st
    L.tri_map_plan.argtypes = [ctypes.POINTER(vp), i64, i32, i32, i32, u32]
    L.tri_plan_destroy.restype = st
    L.tri_plan_destroy.argtypes = [vp]
    L.tri_plan_query.restype = st
    L.tri_plan_query.argtypes = [vp, ctypes.POINTER(tri_plan_info)]
    L.tri_map_dump.restype = st
    L.tri_map_dump.argtypes = [vp, vp, vp]
    L.tri_lambda_eval.restype = st
    L.tri_lambda_eval.argtypes = [vp, i64, i32, u32, vp, vp]
    L.tri_launch_elementwise.restype = st
    L.tri_launch_elementwise.argtypes = [vp, i32, vp, vp, vp, i64, ctypes.c_float, vp]
    L.tri_launch_stencil.restype = st
    L.tri_launch_stencil.argtypes = [vp, vp, vp, i64, i32, i32, vp]
    L.tri_edm_workspace_size.restype = st
    L.tri_edm_workspace_size.argtypes = [vp, i64, i32, ctypes.POINTER(ctypes.c_size_t)]
    L.tri_edm.restype = st
    L.tri_edm.argtypes = [vp, vp, i64, i64, vp, i32, ctypes.c_float, vp, ctypes.c_size_t, vp]
    L.tri_edm_noalloc.restype = st
    L.tri_edm_noalloc.argtypes = [vp, vp, i64, i64, vp, i32, ctypes.c_float, vp]
    L.tri_tet_plan.restype = st
    L.tri_tet_plan.argtypes = [ctypes.POINTER(vp), i64, i32, i32, i32, u32]
    L.tri_tet_destroy.restype = st
    L.tri_tet_destroy.argtypes = [vp]
    L.tri_tet_query.restype = st
    L.tri_tet_query.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_int64)]
    L.tri_tet_dump.restype = st
    L.tri_tet_dump.argtypes = [vp, vp, vp]
    L.tri_lambda3_eval.restype = st
    L.tri_lambda3_eval.argtypes = [vp, i64, u32, vp, vp]
    L.tri_triangles.restype = st
    L.tri_triangles.argtypes = [vp, vp, ctypes.c_float, vp, vp, vp]
    L.tri_tet_dummy.restype = st
    L.tri_tet_dummy.argtypes = [vp, i32, vp, vp]
    L.tri_launch_dummy.restype = st
    L.tri_launch_dummy.argtypes = [vp, i32, vp, vp]
    L.tri_collide.restype = st
    L.tri_collide.argtypes = [vp, vp, i32, vp, vp]
    L.tri_batch_plan.restype = st
    L.tri_batch_plan.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, vp, vp, vp, i32, i32, i32, u32]
    L.tri_batch_bind.restype = st
    L.tri_batch_bind.argtypes = [vp, vp, vp, vp]
    L.tri_batch_launch.restype = st
    L.tri_batch_launch.argtypes = [vp, i32, vp]
    L.tri_batch_query.restype = st
    L.tri_batch_query.argtypes = [vp, ctypes.POINTER(tri_batch_info)]
    L.tri_batch_autotune.restype = st
    L.tri_batch_autotune.argtypes = [ctypes.c_int32, vp, vp, vp, i32, vp, vp, vp, i32, vp,
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_float)]
    L.tri_batch_destroy.restype = st
    L.tri_batch_destroy.argtypes = [vp]
    L.tri_autotune.restype = st
    L.tri_autotune.argtypes = [i32, i64, i64, i32, i32, vp, ctypes.POINTER(tri_tune_choice),
                               ctypes.POINTER(tri_tune_choice), ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_int32)]
    L.tri_tune_cache_save.restype = st
    L.tri_tune_cache_save.argtypes = [ctypes.c_char_p]
    L.tri_tune_cache_load.restype = st
    L.tri_tune_cache_load.argtypes = [ctypes.c_char_p]
    L.tri_tune_cache_clear.restype = st
    L.tri_tune_cache_clear.argtypes = []
    L.tri_stream_add.restype = st
    L.tri_stream_add.argtypes = [vp, vp, vp, i64, vp]
    L.tri_stream_probe.restype = st
    L.tri_stream_probe.argtypes = [i32, i32, i32, i32, i64, vp, vp, vp, i64, vp]
    L.tri_status_str.restype = ctypes.c_char_p
    L.tri_status_str.argtypes = [st]
    L.tri_last_error.restype = ctypes.c_char_p
    L.tri_last_error.argtypes = []
    return L


lib = _load()


def status_str(status: int) -> str:
    return lib.tri_status_str(status).decode()


def _check(status: int):
    if status != OK:
        raise TrimapError(status, lib.tri_last_error().decode())


def _stream(stream=None) -> int | None:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dptr(t) -> int:
    if t is None:
        return None
    if not t.is_cuda:
        raise TrimapArgError("expected a device tensor")
    return t.data_ptr()


def _span(t) -> int:
    """Bytes of t's allocation from t.data_ptr() to its end."""
    return t.untyped_storage().nbytes() - t.storage_offset() * t.element_size()


def _arg(t, name: str, dtypes, elems: int, optional: bool = False):
    """Device pointer of t after checking that it is a device tensor of one of
    `dtypes` (torch dtype names), with unit stride in its last dimension, and
    that its allocation holds at least `elems` elements from its first one."""
    if t is None:
        if optional:
            return None
        raise TrimapArgError(f"{name}: a tensor is required")
    if not t.is_cuda:
        raise TrimapArgError(f"{name}: expected a device tensor")
    if str(t.dtype).replace("torch.", "") not in dtypes:
        raise TrimapArgError(f"{name}: dtype {t.dtype} not in {sorted(dtypes)}")
    if t.dim() > 0 and t.numel() > 1 and t.stride(-1) != 1:
        raise TrimapArgError(f"{name}: the last dimension must have stride 1")
    if elems > 0 and _span(t) < elems * t.element_size():
        raise TrimapArgError(f"{name}: {elems} elements needed from its first one, the "
                             f"allocation holds {_span(t) // t.element_size()}")
    return t.data_ptr()


def _rows_ld(t, ld):
    """Row pitch of a 2-D grid argument (its stride unless given)."""
    if ld is None:
        ld = t.stride(0) if t.dim() == 2 else t.shape[-1]
    return int(ld)


F32 = {"float32"}
I32 = {"int32", "uint32"}
U8 = {"uint8"}


@dataclass
class PlanInfo:
    n: int
    tile: int
    m: int
    tiles: int
    grid_x: int
    grid_y: int
    grid_blocks: int
    wasted_blocks: int
    elements: int
    dump_entries: int
    map: int
    include_diag: int
    flags: int


class Plan:
    """A tile space of a triangular domain under one map (tri_map_plan)."""

    def __init__(self, n: int, tile: int = 32, map: int | str = LAMBDA,
                 include_diag: bool = True, flags: int = 0):
        if isinstance(map, str):
            map = MAPS[map]
        h = ctypes.c_void_p()
        _check(lib.tri_map_plan(ctypes.byref(h), int(n), int(tile), int(map),
                                1 if include_diag else 0, int(flags)))
        self._h = h
        info = tri_plan_info()
        _check(lib.tri_plan_query(h, ctypes.byref(info)))
        self.info = PlanInfo(**{f: getattr(info, f) for f in PlanInfo.__dataclass_fields__})

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            lib.tri_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __repr__(self):
        i = self.info
        return (f"Plan(n={i.n}, tile={i.tile}, map={MAP_NAMES[i.map]}, diag={i.include_diag}, "
                f"m={i.m}, tiles={i.tiles}, grid={i.grid_x}x{i.grid_y})")

    # -- test hooks -------------------------------------------------------
    def dump(self, stream=None):
        import torch
        out = torch.empty((self.info.dump_entries, 2), dtype=torch.int64, device="cuda")
        if self.info.dump_entries:
            _check(lib.tri_map_dump(self._h, _dptr(out), _stream(stream)))
        return out

    # -- kernels ----------------------------------------------------------
    def elementwise(self, op: int, x, y, c, ld: int | None = None, a: float = 0.0,
                    stream=None):
        n = self.info.n
        ld = _rows_ld(c, ld)
        grid = n * max(ld, n)  # an n x ld matrix (ld < n is refused by the library)
        if op == OP_XORMUL_I32:
            px, py = _arg(x, "A", I32, n), _arg(y, "B", I32, n)
            pc = _arg(c, "C", I32, grid)
        elif op == OP_AXPYT_F32:
            for t, nm in ((x, "X"), (y, "Y")):
                if t is not None and t.dim() == 2 and t.stride(0) != ld:
                    raise TrimapArgError(f"{nm}: row pitch {t.stride(0)} differs from ld {ld}")
            px, py, pc = _arg(x, "X", F32, grid), _arg(y, "Y", F32, grid), _arg(c, "C", F32, grid)
        elif op == OP_EDM4_F32:
            px, py = _arg(x, "P", F32, 4 * n), _arg(y, "y", F32, 0, optional=True)
            pc = _arg(c, "C", F32, grid)
        else:
            px, py, pc = _dptr(x), _dptr(y), _dptr(c)  # the library refuses the op
        _check(lib.tri_launch_elementwise(self._h, int(op), px, py, pc, int(ld), float(a),
                                          _stream(stream)))

    def stencil(self, cur, nxt, steps: int, ld: int | None = None, use_graph: bool = False,
                stream=None):
        n = self.info.n
        ld = _rows_ld(cur, ld)
        if nxt is not None and cur is not None and nxt.dim() == 2 and cur.dim() == 2 and \
                nxt.stride(0) != cur.stride(0):
            raise TrimapArgError("cur and nxt must have the same row pitch")
        grid = n * max(ld, n)
        _check(lib.tri_launch_stencil(self._h, _arg(cur, "cur", U8, grid),
                                      _arg(nxt, "nxt", U8, grid), int(ld), int(steps),
                                      1 if use_graph else 0, _stream(stream)))

    def edm_workspace_size(self, d: int, mode: int) -> int:
        b = ctypes.c_size_t()
        _check(lib.tri_edm_workspace_size(self._h, int(d), int(mode), ctypes.byref(b)))
        return b.value

    def edm(self, x, out, mode: int = EDM_FP32, fixup_thr: float = 1e-2, ws=None,
            stream=None):
        n = self.info.n
        if x is None or x.dim() != 2:
            raise TrimapArgError("x: an n x d matrix is required")
        d, ldx = x.shape[1], x.stride(0)
        if x.shape[0] != n:
            raise TrimapArgError(f"x: {x.shape[0]} rows for a plan of n = {n}")
        px = _arg(x, "x", F32, (n - 1) * ldx + d if n else 0)
        po = _arg(out, "out", F32, n * (n - 1) // 2)
        wsb = 0 if ws is None else min(ws.numel() * ws.element_size(), _span(ws))
        pw = _arg(ws, "ws", {"uint8", "int8", "float32", "int32", "int64", "float64"}, 0,
                  optional=True)
        _check(lib.tri_edm(self._h, px, int(d), int(ldx), po, int(mode), float(fixup_thr), pw,
                           int(wsb), _stream(stream)))

    def edm_noalloc(self, x, out, mode: int = EDM_FP32, fixup_thr: float = 1e-2, stream=None):
        """tri_edm_noalloc: the distance map with the library's own scratch
        (no workspace argument, nothing allocated)."""
        n = self.info.n
        if x is None or x.dim() != 2:
            raise TrimapArgError("x: an n x d matrix is required")
        d, ldx = x.shape[1], x.stride(0)
        if x.shape[0] != n:
            raise TrimapArgError(f"x: {x.shape[0]} rows for a plan of n = {n}")
        px = _arg(x, "x", F32, (n - 1) * ldx + d if n else 0)
        po = _arg(out, "out", F32, n * (n - 1) // 2)
        _check(lib.tri_edm_noalloc(self._h, px, int(d), int(ldx), po, int(mode),
                                   float(fixup_thr), _stream(stream)))

    def dummy(self, target: int, sink, stream=None):
        """The square-root study's dummy kernel (tri_launch_dummy)."""
        _check(lib.tri_launch_dummy(self._h, int(target), _arg(sink, "sink", I32, 1),
                                    _stream(stream)))

    def collide(self, spheres, counts, dim: int = 3, stream=None):
        """Per-sphere overlap counts (tri_collide); spheres is a float32
        device tensor n x 4 (x, y, z, r), counts an int32 device tensor."""
        n = self.info.n
        _check(lib.tri_collide(self._h, _arg(spheres, "spheres", F32, 4 * n), int(dim),
                               _arg(counts, "counts", I32, n), _stream(stream)))


class TetPlan:
    """A tile space of a tetrahedral domain (tri_tet_plan): BB or lambda."""

    def __init__(self, n: int, tile: int = 16, map: int | str = LAMBDA, strict: bool = True,
                 flags: int = 0):
        if isinstance(map, str):
            map = MAPS[map]
        h = ctypes.c_void_p()
        _check(lib.tri_tet_plan(ctypes.byref(h), int(n), int(tile), int(map),
                                1 if strict else 0, int(flags)))
        self._h = h
        t, g, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.tri_tet_query(h, ctypes.byref(t), ctypes.byref(g), ctypes.byref(c)))
        self.n, self.tile, self.map, self.strict = int(n), int(tile), int(map), bool(strict)
        self.tiles, self.grid_blocks, self.cells = t.value, g.value, c.value

    def close(self):
        if self._h is not None and self._h.value:
            lib.tri_tet_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dump(self, stream=None):
        """(i, j, k) per grid block, -1 for discarded blocks (int64 [blocks, 3])."""
        import torch
        out = torch.empty((max(self.grid_blocks, 0), 3), dtype=torch.int64, device="cuda")
        if self.grid_blocks:
            _check(lib.tri_tet_dump(self._h, _dptr(out), _stream(stream)))
        return out

    def triangles(self, points, r2: float, counts, total, stream=None):
        """Triangle counts of the neighbour graph (tri_triangles)."""
        n = self.n
        _check(lib.tri_triangles(self._h, _arg(points, "points", F32, 4 * n), float(r2),
                                 _arg(counts, "counts", I32, n),
                                 _arg(total, "total", {"int64", "uint64"}, 1), _stream(stream)))

    def dummy(self, target: int, sink, stream=None):
        _check(lib.tri_tet_dummy(self._h, int(target), _arg(sink, "sink", I32, 1),
                                 _stream(stream)))


def lambda3_eval(omega, flags: int = 0, stream=None):
    """Device tetrahedral lambda(omega) -> int64 [count, 3] = (i, j, k)."""
    import torch
    out = torch.empty((omega.numel(), 3), dtype=torch.int64, device=omega.device)
    if not omega.is_contiguous():
        raise TrimapArgError("omega: a contiguous tensor is required")
    _check(lib.tri_lambda3_eval(_arg(omega, "omega", {"int64", "uint64"}, omega.numel()),
                                int(omega.numel()), int(flags), _dptr(out), _stream(stream)))
    return out


def lambda_eval(omega, include_diag: bool = True, flags: int = 0, stream=None):
    """Device lambda(omega) for a uint64/int64 device tensor of omegas."""
    import torch
    out = torch.empty((omega.numel(), 2), dtype=torch.int64, device=omega.device)
    if not omega.is_contiguous():
        raise TrimapArgError("omega: a contiguous tensor is required")
    _check(lib.tri_lambda_eval(_arg(omega, "omega", {"int64", "uint64"}, omega.numel()),
                               int(omega.numel()), 1 if include_diag else 0, int(flags),
                               _dptr(out), _stream(stream)))
    return out


class Batch:
    """Uneven triangular domains in one persistent launch per generation
    (tri_batch_plan / tri_batch_bind / tri_batch_launch).

    kinds: KIND_EDM or KIND_LIFE per instance; ns: sides; ds: dimensions
    (distance maps).  bind() takes per-instance device tensors: distance map
    (x, out), Life (grid holding generation 0, the other grid)."""

    def __init__(self, kinds, ns, ds, edm_tile: int = 32, life_tile: int = 32,
                 life_steps: int = 20, flags: int = 0):
        import numpy as np
        self.kinds = np.ascontiguousarray(kinds, dtype=np.int32)
        self.ns = np.ascontiguousarray(ns, dtype=np.int64)
        self.ds = np.ascontiguousarray(ds, dtype=np.int64)
        h = ctypes.c_void_p()
        _check(lib.tri_batch_plan(ctypes.byref(h), int(self.kinds.size),
                                  self.kinds.ctypes.data, self.ns.ctypes.data,
                                  self.ds.ctypes.data, int(edm_tile), int(life_tile),
                                  int(life_steps), int(flags)))
        self._h = h
        self._keep = None

    @property
    def info(self) -> dict:
        """tri_batch_query now (binding picks the kernel, its workgroups and,
        for the bit-sliced Life kernel, fewer graph nodes)."""
        info = tri_batch_info()
        _check(lib.tri_batch_query(self._h, ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in tri_batch_info._fields_}

    def bind(self, a_list, b_list):
        import numpy as np
        n = self.kinds.size
        if len(a_list) != n or len(b_list) != n:
            raise TrimapArgError(f"bind: {n} instances, {len(a_list)} / {len(b_list)} buffers")
        A, B, ld = _batch_buffers(self.kinds, self.ns, self.ds, a_list, b_list)
        _check(lib.tri_batch_bind(self._h, A, B, ld.ctypes.data))
        self._keep = (list(a_list), list(b_list))  # the buffers must outlive the plan's use

    def launch(self, how: int = BATCH_GRAPH, stream=None):
        _check(lib.tri_batch_launch(self._h, int(how), _stream(stream)))

    def close(self):
        if self._h is not None and self._h.value:
            lib.tri_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(workload: int, n: int, d: int = 0, reps: int = 3, use_cache: bool = True,
             stream=None):
    """Time the tile/map candidates (tri_autotune); returns (best, all) with
    each choice a dict(tile, map, flags, ms)."""
    best = tri_tune_choice()
    cap = 256
    arr = (tri_tune_choice * cap)()
    cnt = ctypes.c_int32()
    _check(lib.tri_autotune(int(workload), int(n), int(d), int(reps), 1 if use_cache else 0,
                            _stream(stream), ctypes.byref(best), arr, cap, ctypes.byref(cnt)))
    conv = lambda c: {"tile": c.tile, "map": MAP_NAMES.get(c.map, c.map), "flags": c.flags,
                      "ms": c.ms}
    return conv(best), [conv(arr[k]) for k in range(cnt.value)]


def tune_cache_save(path: str):
    _check(lib.tri_tune_cache_save(path.encode()))


def tune_cache_load(path: str):
    _check(lib.tri_tune_cache_load(path.encode()))


def tune_cache_clear():
    _check(lib.tri_tune_cache_clear())


def batch_autotune(kinds, ns, ds, life_steps, a_list, b_list, reps: int = 2, stream=None):
    """Fastest (edm_tile, life_tile, flags, ms) for a batch
    (tri_batch_autotune).  Runs the batch on the given buffers (Life grids
    advance)."""
    import numpy as np
    kinds = np.ascontiguousarray(kinds, dtype=np.int32)
    ns = np.ascontiguousarray(ns, dtype=np.int64)
    ds = np.ascontiguousarray(ds, dtype=np.int64)
    n = kinds.size
    if len(a_list) != n or len(b_list) != n:
        raise TrimapArgError(f"batch_autotune: {n} instances, {len(a_list)} / {len(b_list)} "
                             "buffers")
    A, B, ld = _batch_buffers(kinds, ns, ds, a_list, b_list)
    te, tl, fl, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_uint32(), ctypes.c_float()
    _check(lib.tri_batch_autotune(n, kinds.ctypes.data, ns.ctypes.data, ds.ctypes.data,
                                  int(life_steps), A, B, ld.ctypes.data, int(reps),
                                  _stream(stream), ctypes.byref(te), ctypes.byref(tl),
                                  ctypes.byref(fl), ctypes.byref(ms)))
    return te.value, tl.value, fl.value, ms.value


def _batch_buffers(kinds, ns, ds, a_list, b_list):
    """Checked device pointers and row pitches of a batch's buffers: a
    distance map k takes x (n_k x d_k FP32 rows of pitch >= d_k) and its
    condensed output (n_k (n_k - 1) / 2 FP32); a Life instance two uint8
    grids of n_k rows of one pitch."""
    import numpy as np
    A, B, lds = [], [], []
    for k, (a, b) in enumerate(zip(a_list, b_list)):
        n, kind = int(ns[k]), int(kinds[k])
        if kind == KIND_EDM:
            d = int(ds[k])
            if a is None or a.dim() != 2 or a.shape[1] < d:
                raise TrimapArgError(f"instance {k}: x must be an n x d matrix")
            ld = a.stride(0)
            A.append(_arg(a, f"x[{k}]", F32, (n - 1) * ld + d if n else 0))
            B.append(_arg(b, f"out[{k}]", F32, n * (n - 1) // 2))
        else:
            ld = _rows_ld(a, None)
            if b is not None and b.dim() == 2 and a.dim() == 2 and b.stride(0) != a.stride(0):
                raise TrimapArgError(f"instance {k}: both Life grids need one row pitch")
            A.append(_arg(a, f"grid_a[{k}]", U8, n * max(ld, n)))
            B.append(_arg(b, f"grid_b[{k}]", U8, n * max(ld, n)))
        lds.append(ld)
    m = len(A)
    return ((ctypes.c_void_p * m)(*A), (ctypes.c_void_p * m)(*B),
            np.ascontiguousarray(lds, dtype=np.int64))


def stream_add(c, a, b, stream=None):
    """c = a + b with the library's streaming probe kernel (tri_stream_add)."""
    cnt = c.numel()
    for t, nm in ((c, "c"), (a, "a"), (b, "b")):
        if not t.is_contiguous():
            raise TrimapArgError(f"{nm}: a contiguous tensor is required")
    _check(lib.tri_stream_add(_arg(c, "c", F32, cnt), _arg(a, "a", F32, cnt),
                              _arg(b, "b", F32, cnt), int(cnt), _stream(stream)))


PROBE_READ, PROBE_ADD, PROBE_FILL, PROBE_COPY = range(4)


def stream_probe(kind: int, c, a=None, b=None, count: int | None = None, unroll: int = 4,
                 threads: int = 256, nontemporal: bool = True, workgroups: int = 0,
                 stream=None):
    """One launch of the bandwidth probe (tri_stream_probe) over `count`
    floats (default: all of a, or of c for the fill)."""
    src = c if kind == PROBE_FILL else a
    cnt = src.numel() if count is None else int(count)
    for t, nm in ((c, "c"), (a, "a"), (b, "b")):
        if t is not None and not t.is_contiguous():
            raise TrimapArgError(f"{nm}: a contiguous tensor is required")
    _check(lib.tri_stream_probe(int(kind), int(unroll), int(threads), 1 if nontemporal else 0,
                                int(workgroups), _arg(c, "c", F32, cnt),
                                _arg(a, "a", F32, cnt, optional=kind == PROBE_FILL),
                                _arg(b, "b", F32, cnt, optional=kind != PROBE_ADD),
                                cnt, _stream(stream)))
