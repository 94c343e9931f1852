"""CPU FP64 oracle for the hierarchical 2D FMM (complex log kernel).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It is a plain, slow,
step-by-step implementation written from the paper (Luo & Duraiswami,
arXiv:1204.3105, Secs. 2-6) plus the Greengard-Rokhlin 1987 operators the
paper cites but omits.  It shares no code with the GPU library.

The C source is ``fmm_oracle.c``; this module is argument marshalling only.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

QUAD, SEPT, TRI = 0, 1, 2
TILINGS = {"quad": QUAD, "sept": SEPT, "tri": TRI}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
            "-fopenmp", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Geom(C.Structure):
    """Tree geometry: tiling, leaf level L, origin (ox, oy) and scale.

    quadtree: origin = lower-left corner of the root square, size = side.
    septree: origin = centre of leaf hexagon 0, size = leaf circumradius r.
    triangle-quadtree: origin = root centroid, size = leaf circumradius r.
    """
    _fields_ = [("tiling", C.c_int32), ("L", C.c_int32), ("ox", C.c_double),
                ("oy", C.c_double), ("size", C.c_double)]

    def __repr__(self):
        return "Geom(tiling=%d, L=%d, ox=%r, oy=%r, size=%r)" % (
            self.tiling, self.L, self.ox, self.oy, self.size)


def geom(tiling, L, ox, oy, size) -> Geom:
    if isinstance(tiling, str):
        tiling = TILINGS[tiling]
    return Geom(int(tiling), int(L), float(ox), float(oy), float(size))


_lib = None

_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)
_I32 = C.POINTER(C.c_int32)
_G = C.POINTER(Geom)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        L.orc_cell_index.restype = C.c_int64
        L.orc_cell_index.argtypes = [_G, C.c_double, C.c_double, C.c_int32]
        L.orc_cell_index_many.argtypes = [_G, _D, _D, C.c_int64, C.c_int32, _I64]
        L.orc_cell_center.argtypes = [_G, C.c_int64, C.c_int32, _D, _D]
        L.orc_cell_center_many.argtypes = [_G, _I64, C.c_int64, C.c_int32, _D, _D]
        L.orc_sept_center_polar.argtypes = [_G, C.c_int64, C.c_int32, _D, _D]
        L.orc_center_units.argtypes = [_G, C.c_int64, C.c_int32, _I64, _I64]
        L.orc_parent.restype = C.c_int64
        L.orc_parent.argtypes = [C.c_int32, C.c_int64]
        L.orc_neighbors.restype = C.c_int32
        L.orc_neighbors.argtypes = [_G, C.c_int64, C.c_int32, _I64]
        L.orc_e4.restype = C.c_int32
        L.orc_e4.argtypes = [_G, C.c_int64, C.c_int32, _I64]
        L.orc_e4_many.argtypes = [_G, _I64, C.c_int64, C.c_int32, _I64, _I32]
        L.orc_neighbors_many.argtypes = [_G, _I64, C.c_int64, C.c_int32, _I64, _I32]
        L.orc_gbt_add.restype = C.c_int64
        L.orc_gbt_add.argtypes = [C.c_int64, C.c_int64]
        L.orc_tq_adjacent.restype = C.c_int32
        L.orc_tq_adjacent.argtypes = [C.c_int64, C.c_int32, C.c_int32, _I64]
        L.orc_tq_is_up.restype = C.c_int32
        L.orc_tq_is_up.argtypes = [C.c_int64, C.c_int32]
        L.orc_op_p2m.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_int64, _D, _D, _D, _D]
        L.orc_op_m2m.argtypes = [C.c_int32, _D, C.c_double, C.c_double, _D]
        L.orc_op_m2l.argtypes = [C.c_int32, _D, C.c_double, C.c_double, C.c_double, C.c_double, _D]
        L.orc_op_l2l.argtypes = [C.c_int32, _D, C.c_double, C.c_double, _D]
        L.orc_op_l2p.argtypes = [C.c_int32, _D, C.c_double, C.c_double, C.c_int64, _D, _D, _D]
        L.orc_op_mpole_eval.argtypes = [C.c_int32, _D, C.c_double, C.c_double, C.c_int64, _D, _D, _D]
        L.orc_max_threads.restype = C.c_int32
        L.orc_direct_principal.argtypes = [C.c_int64, _D, _D, _D, C.c_int64, _D, _D, _D, C.c_int32]
        L.orc_direct_branch_aware.restype = C.c_int32
        L.orc_direct_branch_aware.argtypes = [_G, C.c_int64, _D, _D, _D, C.c_int64, _D, _D, _D,
                                              C.c_int32]
        L.orc_fmm.restype = C.c_int32
        L.orc_fmm.argtypes = [_G, C.c_int32, C.c_int64, _D, _D, _D, C.c_int64, _D, _D, _D,
                              C.c_int32, _D]
        L.orc_fmm_field.restype = C.c_int32
        L.orc_fmm_field.argtypes = [_G, C.c_int32, C.c_int64, _D, _D, _D, C.c_int64, _D, _D, _D, _D,
                                    C.c_int32, _D]
        L.orc_direct_field.argtypes = [C.c_int64, _D, _D, _D, C.c_int64, _D, _D, _D, C.c_int32]
        L.orc_upward_level.restype = C.c_int64
        L.orc_upward_level.argtypes = [_G, C.c_int32, C.c_int64, _D, _D, _D, C.c_int32, _I64, _D]
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _pd(a):
    return a.ctypes.data_as(_D)


def _pi64(a):
    return a.ctypes.data_as(_I64)


def _pi32(a):
    return a.ctypes.data_as(_I32)


def _cplx_out(buf):
    return buf[0::2] + 1j * buf[1::2]


# ---------------------------------------------------------------- addressing
def cell_index(g: Geom, x, y, level: int) -> np.ndarray:
    """CellIndex(x, y, l) for every point; -1 for a point outside the root."""
    x, y = _d(x), _d(y)
    out = np.empty(len(x), dtype=np.int64)
    lib().orc_cell_index_many(C.byref(g), _pd(x), _pd(y), len(x), int(level), _pi64(out))
    return out


def cell_center(g: Geom, keys, level: int):
    keys = np.ascontiguousarray(np.atleast_1d(keys), dtype=np.int64)
    cx = np.empty(len(keys))
    cy = np.empty(len(keys))
    lib().orc_cell_center_many(C.byref(g), _pi64(keys), len(keys), int(level), _pd(cx), _pd(cy))
    return cx, cy


def sept_center_polar(g: Geom, key: int, level: int):
    cx, cy = C.c_double(), C.c_double()
    lib().orc_sept_center_polar(C.byref(g), int(key), int(level), C.byref(cx), C.byref(cy))
    return cx.value, cy.value


def center_units(g: Geom, key: int, level: int):
    """Integer coordinates of a centre: quadtree (ix, iy), septree lattice
    (b, c) in leaf units, triangle-quadtree (U, V) in units of
    (sqrt(3)/2 r, r/2)."""
    a, b = C.c_int64(), C.c_int64()
    lib().orc_center_units(C.byref(g), int(key), int(level), C.byref(a), C.byref(b))
    return a.value, b.value


def neighbors(g: Geom, key: int, level: int) -> list:
    out = np.empty(16, dtype=np.int64)
    n = lib().orc_neighbors(C.byref(g), int(key), int(level), _pi64(out))
    return sorted(int(v) for v in out[:n])


def e4(g: Geom, key: int, level: int) -> list:
    out = np.empty(64, dtype=np.int64)
    n = lib().orc_e4(C.byref(g), int(key), int(level), _pi64(out))
    return sorted(int(v) for v in out[:n])


def e4_many(g: Geom, keys, level: int):
    """E4 lists of many cells: (out[n, 64], counts[n]) in generation order."""
    keys = np.ascontiguousarray(keys, dtype=np.int64)
    out = np.full((len(keys), 64), -1, dtype=np.int64)
    cnt = np.empty(len(keys), dtype=np.int32)
    lib().orc_e4_many(C.byref(g), _pi64(keys), len(keys), int(level), _pi64(out), _pi32(cnt))
    return out, cnt


def neighbors_many(g: Geom, keys, level: int):
    keys = np.ascontiguousarray(keys, dtype=np.int64)
    out = np.full((len(keys), 16), -1, dtype=np.int64)
    cnt = np.empty(len(keys), dtype=np.int32)
    lib().orc_neighbors_many(C.byref(g), _pi64(keys), len(keys), int(level), _pi64(out),
                             _pi32(cnt))
    return out, cnt


def gbt_add(a: int, b: int) -> int:
    """GBT sum of two base-7 indices given as integers (value, not numeral)."""
    return int(lib().orc_gbt_add(int(a), int(b)))


def tq_adjacent(key: int, level: int, direction: int):
    """adjacentNeighbor (direction 0 = L, 1 = R, 2 = V); None if absent."""
    out = C.c_int64()
    ok = lib().orc_tq_adjacent(int(key), int(level), int(direction), C.byref(out))
    return out.value if ok else None


def tq_is_up(key: int, level: int) -> int:
    return int(lib().orc_tq_is_up(int(key), int(level)))


def parent(tiling: int, key: int) -> int:
    return int(lib().orc_parent(int(tiling), int(key)))


# ---------------------------------------------------------------- operators
def _coef(a, p):
    a = np.asarray(a, dtype=np.complex128)
    buf = np.zeros(2 * (p + 1))
    buf[0::2] = a.real
    buf[1::2] = a.imag
    return buf


def p2m(p, c, x, y, u):
    x, y, u = _d(x), _d(y), _d(u)
    buf = np.zeros(2 * (p + 1))
    lib().orc_op_p2m(p, c.real, c.imag, len(x), _pd(x), _pd(y), _pd(u), _pd(buf))
    return _cplx_out(buf)


def m2m(p, a, z0):
    ab = _coef(a, p)
    out = np.zeros(2 * (p + 1))
    lib().orc_op_m2m(p, _pd(ab), z0.real, z0.imag, _pd(out))
    return _cplx_out(out)


def m2l(p, a, c_src, c_tgt):
    ab = _coef(a, p)
    out = np.zeros(2 * (p + 1))
    lib().orc_op_m2l(p, _pd(ab), c_src.real, c_src.imag, c_tgt.real, c_tgt.imag, _pd(out))
    return _cplx_out(out)


def l2l(p, b, w):
    bb = _coef(b, p)
    out = np.zeros(2 * (p + 1))
    lib().orc_op_l2l(p, _pd(bb), w.real, w.imag, _pd(out))
    return _cplx_out(out)


def l2p(p, b, c, x, y):
    bb = _coef(b, p)
    x, y = _d(x), _d(y)
    out = np.zeros(2 * len(x))
    lib().orc_op_l2p(p, _pd(bb), c.real, c.imag, len(x), _pd(x), _pd(y), _pd(out))
    return _cplx_out(out)


def mpole_eval(p, a, c, x, y):
    ab = _coef(a, p)
    x, y = _d(x), _d(y)
    out = np.zeros(2 * len(x))
    lib().orc_op_mpole_eval(p, _pd(ab), c.real, c.imag, len(x), _pd(x), _pd(y), _pd(out))
    return _cplx_out(out)


# ---------------------------------------------------------------- sums
def direct_principal(xs, ys, u, xt, yt, nthreads=0) -> np.ndarray:
    """D1: sum_i u_i Log(y_j - x_i), principal branch, coincident pairs skipped."""
    xs, ys, u, xt, yt = map(_d, (xs, ys, u, xt, yt))
    out = np.zeros(2 * len(xt))
    lib().orc_direct_principal(len(xs), _pd(xs), _pd(ys), _pd(u), len(xt), _pd(xt), _pd(yt),
                               _pd(out), int(nthreads))
    return _cplx_out(out)


def direct_branch_aware(g: Geom, xs, ys, u, xt, yt, nthreads=0) -> np.ndarray:
    """D2: the exact sum with the FMM's branch of the logarithm on this tree."""
    xs, ys, u, xt, yt = map(_d, (xs, ys, u, xt, yt))
    out = np.zeros(2 * len(xt))
    rc = lib().orc_direct_branch_aware(C.byref(g), len(xs), _pd(xs), _pd(ys), _pd(u), len(xt),
                                       _pd(xt), _pd(yt), _pd(out), int(nthreads))
    if rc:
        raise ValueError("point outside the root (rc=%d)" % rc)
    return _cplx_out(out)


def fmm(g: Geom, p: int, xs, ys, u, xt, yt, nthreads=0, times=None) -> np.ndarray:
    """Full FP64 FMM on the given tree; complex potential in target order.

    ``times`` (optional list) receives the stage wall times: keys+tree,
    P2M+M2M, M2L, L2L, L2P+P2P, total (seconds)."""
    xs, ys, u, xt, yt = map(_d, (xs, ys, u, xt, yt))
    out = np.zeros(2 * len(xt))
    tbuf = np.zeros(6)
    rc = lib().orc_fmm(C.byref(g), int(p), len(xs), _pd(xs), _pd(ys), _pd(u), len(xt), _pd(xt),
                       _pd(yt), _pd(out), int(nthreads), _pd(tbuf))
    if rc == 2:
        raise ValueError("point outside the root")
    if rc:
        raise ValueError("bad arguments (rc=%d)" % rc)
    if times is not None:
        times[:] = list(tbuf)
    return _cplx_out(out)


def fmm_field(g: Geom, p: int, xs, ys, u, xt, yt, nthreads=0):
    """Full FP64 FMM returning (Phi, Phi') in target order; Phi' is the
    derivative in y (the local expansion's derivative plus the near sum of
    u_i / (y - x_i))."""
    xs, ys, u, xt, yt = map(_d, (xs, ys, u, xt, yt))
    out = np.zeros(2 * len(xt))
    fld = np.zeros(2 * len(xt))
    rc = lib().orc_fmm_field(C.byref(g), int(p), len(xs), _pd(xs), _pd(ys), _pd(u), len(xt), _pd(xt),
                             _pd(yt), _pd(out), _pd(fld), int(nthreads), None)
    if rc == 2:
        raise ValueError("point outside the root")
    if rc:
        raise ValueError("bad arguments (rc=%d)" % rc)
    return _cplx_out(out), _cplx_out(fld)


def direct_field(xs, ys, u, xt, yt, nthreads=0) -> np.ndarray:
    """sum_i u_i / (y_j - x_i), coincident pairs skipped."""
    xs, ys, u, xt, yt = map(_d, (xs, ys, u, xt, yt))
    out = np.zeros(2 * len(xt))
    lib().orc_direct_field(len(xs), _pd(xs), _pd(ys), _pd(u), len(xt), _pd(xt), _pd(yt), _pd(out),
                           int(nthreads))
    return _cplx_out(out)


def upward_level(g: Geom, p: int, xs, ys, u, level: int):
    """(keys, multipole coefficients[n, p+1]) of the source cells at a level."""
    xs, ys, u = map(_d, (xs, ys, u))
    n = lib().orc_upward_level(C.byref(g), int(p), len(xs), _pd(xs), _pd(ys), _pd(u), int(level),
                               None, None)
    if n < 0:
        raise ValueError("bad level or point outside the root")
    keys = np.empty(n, dtype=np.int64)
    coef = np.empty(2 * n * (p + 1))
    lib().orc_upward_level(C.byref(g), int(p), len(xs), _pd(xs), _pd(ys), _pd(u), int(level),
                           _pi64(keys), _pd(coef))
    return keys, _cplx_out(coef).reshape(n, p + 1)


def max_threads() -> int:
    return int(lib().orc_max_threads())
