"""Python binding of libfmm2d.so (the C ABI in include/fmm2d.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  Inputs may be numpy arrays (host; the call is synchronous) or
torch CUDA tensors (device; work is ordered on torch's current stream).
There is no fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm2d.so")

QUADTREE, SEPTREE, TRIQUADTREE = 0, 1, 2
TILINGS = {"quad": QUADTREE, "quadtree": QUADTREE, "sept": SEPTREE, "septree": SEPTREE,
           "tri": TRIQUADTREE, "triquadtree": TRIQUADTREE, "triangle": TRIQUADTREE}
PREC = {"auto": 0, "fp64": 1, "mixed": 2}
PREC_NAMES = {0: "auto", 1: "fp64", 2: "mixed"}
STATUS = {0: "OK", 1: "INVALID", 2: "DOMAIN", 3: "NOMEM", 4: "DEVICE", 5: "BUSY"}


class FMMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Options(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("leaf_size", C.c_int32), ("lmax", C.c_int32),
                ("p", C.c_int32), ("precision", C.c_int32), ("has_geometry", C.c_int32),
                ("geometry", C.c_double * 3), ("stream", C.c_void_p),
                ("device_pointers", C.c_int32), ("depth_rule", C.c_int32), ("near_stream", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("tiling", C.c_int32), ("lmax", C.c_int32), ("p", C.c_int32),
                ("precision", C.c_int32), ("geometry", C.c_double * 3), ("n_src", C.c_int64),
                ("n_tgt", C.c_int64), ("targets_are_sources", C.c_int32),
                ("e4_width", C.c_int32), ("n_cells", C.c_int64 * 32),
                ("n_m2l_pairs", C.c_int64), ("n_near_pairs", C.c_int64),
                ("device_bytes", C.c_int64), ("plan_ms", C.c_double), ("eval_ms", C.c_double),
                ("stage_ms", C.c_double * 8)]


class ServerOptions(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("hbm_budget_bytes", C.c_int64),
                ("max_inflight", C.c_int32), ("leaf_size", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("tiling", C.c_int32), ("precision", C.c_int32), ("eps", C.c_double),
                ("n_src", C.c_int64), ("n_tgt", C.c_int64), ("src", C.c_void_p),
                ("tgt", C.c_void_p), ("u", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("p", C.c_int32), ("lmax", C.c_int32),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_start", C.c_double),
                ("t_end", C.c_double)]


EXPORTED = ["fmm_options_default", "fmm_plan", "fmm_eval", "fmm_plan_info_get",
            "fmm_plan_export_points", "fmm_plan_export_level", "fmm_plan_destroy",
            "fmm_last_error", "fmm_order_for_eps", "fmm_server_create", "fmm_submit",
            "fmm_poll", "fmm_server_drain", "fmm_server_destroy", "fmm_direct",
            "fmm_eval_field", "fmm_direct_noalloc", "fmm_probe_pair_rate"]

_lib = None


def lib():
    """Load libfmm2d.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfmm2d.so is not built (run __graft_entry__.build()): %s" % LIB_PATH)
    # PyTorch ships its own HIP runtime under the same soname.  Loading torch
    # first makes the library bind to that runtime, so device pointers and
    # streams from torch are valid here; loading ours first would put a second
    # HIP runtime into the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    D = C.POINTER(C.c_double)
    I64 = C.POINTER(C.c_int64)
    I32 = C.POINTER(C.c_int32)
    L.fmm_options_default.argtypes = [C.POINTER(Options)]
    L.fmm_options_default.restype = C.c_int
    L.fmm_plan.argtypes = [C.c_int, P, C.c_int64, P, C.c_int64, C.c_double, C.POINTER(Options),
                           C.POINTER(P)]
    L.fmm_plan.restype = C.c_int
    L.fmm_eval.argtypes = [P, P, P]
    L.fmm_eval_field.argtypes = [P, P, P, P]
    L.fmm_eval_field.restype = C.c_int
    L.fmm_eval.restype = C.c_int
    L.fmm_plan_info_get.argtypes = [P, C.POINTER(PlanInfo)]
    L.fmm_plan_info_get.restype = C.c_int
    L.fmm_plan_export_points.argtypes = [P, I64, I64, I64, I64]
    L.fmm_plan_export_points.restype = C.c_int
    L.fmm_plan_export_level.argtypes = [P, C.c_int32, I64, I32, I64, I64, I64, I64]
    L.fmm_plan_export_level.restype = C.c_int
    L.fmm_plan_destroy.argtypes = [P]
    L.fmm_plan_destroy.restype = None
    L.fmm_last_error.argtypes = []
    L.fmm_last_error.restype = C.c_char_p
    L.fmm_order_for_eps.argtypes = [C.c_int, C.c_double]
    L.fmm_order_for_eps.restype = C.c_int32
    L.fmm_direct.argtypes = [P, C.c_int64, P, C.c_int64, P, P, C.POINTER(Options)]
    L.fmm_direct.restype = C.c_int
    L.fmm_direct_noalloc.argtypes = [P, C.c_int64, P, C.c_int64, P, P, P]
    L.fmm_direct_noalloc.restype = C.c_int
    L.fmm_probe_pair_rate.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_double)]
    L.fmm_probe_pair_rate.restype = C.c_int
    L.fmm_server_create.argtypes = [C.POINTER(ServerOptions), C.POINTER(P)]
    L.fmm_server_create.restype = C.c_int
    L.fmm_submit.argtypes = [P, C.POINTER(Request), C.POINTER(C.c_uint64)]
    L.fmm_submit.restype = C.c_int
    L.fmm_poll.argtypes = [P, C.c_uint64, D, C.POINTER(Result)]
    L.fmm_poll.restype = C.c_int
    L.fmm_server_drain.argtypes = [P]
    L.fmm_server_drain.restype = C.c_int
    L.fmm_server_destroy.argtypes = [P]
    L.fmm_server_destroy.restype = C.c_int
    _lib = L
    return L


def _check(st: int):
    if st != 0:
        raise FMMError(st, lib().fmm_last_error().decode())


def _tiling(t) -> int:
    return TILINGS[t] if isinstance(t, str) else int(t)


def order_for_eps(tiling, eps: float) -> int:
    return int(lib().fmm_order_for_eps(_tiling(tiling), float(eps)))


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _points_host(x, y=None) -> np.ndarray:
    """(x, y) arrays or an (n, 2) / complex array -> contiguous complex128."""
    if y is not None:
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        out = np.empty(2 * len(x))
        out[0::2] = x
        out[1::2] = y
        return out
    a = np.asarray(x)
    if np.iscomplexobj(a):
        return np.ascontiguousarray(a, dtype=np.complex128).view(np.float64).reshape(-1).copy()
    return np.ascontiguousarray(a, dtype=np.float64).reshape(-1)


DEPTH = {"mean": 0, "cost": 1}
NEAR_STREAM = {"side": 0, "own": 1}


class Plan:
    """A solve plan: tree, keys, lists and device buffers for one point set.

    Host mode: Plan("quad", xs, ys, xt, yt, eps) with numpy arrays.
    Device mode: Plan("quad", src=tensor, tgt=tensor, eps=...) with torch CUDA
    tensors of dtype complex128 (or float64 of shape (n, 2)); tgt may be the
    same tensor object as src.
    """

    def __init__(self, tiling, xs=None, ys=None, xt=None, yt=None, eps=1e-6, *, src=None, tgt=None,
                 leaf_size=64, lmax=-1, p=-1, precision="auto", geometry=None, stream=None, depth="mean",
                 near_stream="side"):
        L = lib()
        self._plan = C.c_void_p()
        opt = Options()
        _check(L.fmm_options_default(C.byref(opt)))
        opt.leaf_size = int(leaf_size)
        opt.lmax = int(lmax)
        opt.p = int(p)
        opt.precision = PREC[precision] if isinstance(precision, str) else int(precision)
        opt.depth_rule = DEPTH[depth] if isinstance(depth, str) else int(depth)
        opt.near_stream = NEAR_STREAM[near_stream] if isinstance(near_stream, str) else int(near_stream)
        if geometry is not None:
            opt.has_geometry = 1
            for k in range(3):
                opt.geometry[k] = float(geometry[k])
        self.device = src is not None and _is_torch(src) and src.is_cuda
        if self.device:
            import torch
            self._src = src.contiguous()
            self._tgt = self._src if (tgt is None or tgt is src) else tgt.contiguous()
            for t in (self._src, self._tgt):
                if t.dtype not in (torch.complex128, torch.float64):
                    raise TypeError("device points must be complex128 or float64 (n, 2)")
            n_src = self._src.numel() if self._src.dtype == torch.complex128 else self._src.numel() // 2
            n_tgt = self._tgt.numel() if self._tgt.dtype == torch.complex128 else self._tgt.numel() // 2
            opt.device_pointers = 1
            st = stream if stream is not None else torch.cuda.current_stream()
            opt.stream = C.c_void_p(st.cuda_stream)
            self._stream = st
            sp = C.c_void_p(self._src.data_ptr())
            tp = sp if self._tgt is self._src else C.c_void_p(self._tgt.data_ptr())
        else:
            if src is not None:
                s = _points_host(src)
                t = s if (tgt is None or tgt is src) else _points_host(tgt)
            else:
                s = _points_host(xs, ys)
                same = xt is None or (xt is xs and yt is ys)
                t = s if same else _points_host(xt, yt)
            self._src, self._tgt = s, t
            n_src, n_tgt = len(s) // 2, len(t) // 2
            sp = C.c_void_p(s.ctypes.data) if n_src else None
            tp = sp if t is s else (C.c_void_p(t.ctypes.data) if n_tgt else None)
        self.n_src, self.n_tgt = int(n_src), int(n_tgt)
        _check(L.fmm_plan(_tiling(tiling), sp, self.n_src, tp, self.n_tgt, float(eps),
                          C.byref(opt), C.byref(self._plan)))
        if self.device:
            # The plan copied what it needs; drop the references.
            self._src = self._tgt = None

    # -------------------------------------------------------------- solve
    def eval(self, u, out=None):
        """Phi for strengths u.  Host: returns complex128 ndarray.  Device:
        returns (or fills) a complex128 CUDA tensor."""
        L = lib()
        if self.device:
            import torch
            u = u.contiguous()
            if u.dtype != torch.float64 or not u.is_cuda or u.numel() != self.n_src:
                raise TypeError("u must be a float64 CUDA tensor of n_src elements")
            if out is None:
                out = torch.empty(self.n_tgt, dtype=torch.complex128, device=u.device)
            _check(L.fmm_eval(self._plan, C.c_void_p(u.data_ptr()), C.c_void_p(out.data_ptr())))
            return out
        u = np.ascontiguousarray(u, dtype=np.float64)
        if len(u) != self.n_src:
            raise ValueError("u must have n_src elements")
        res = np.empty(self.n_tgt, dtype=np.complex128) if out is None else out
        _check(L.fmm_eval(self._plan, C.c_void_p(u.ctypes.data) if self.n_src else None,
                          C.c_void_p(res.ctypes.data) if self.n_tgt else None))
        return res

    def eval_field(self, u, out=None, field_out=None):
        """(Phi, Phi') for strengths u; Phi'(y) = sum u_i / (y - x_i).  Host:
        complex128 ndarrays.  Device: complex128 CUDA tensors (or fills the
        given ones)."""
        L = lib()
        if self.device:
            import torch
            u = u.contiguous()
            if u.dtype != torch.float64 or not u.is_cuda or u.numel() != self.n_src:
                raise TypeError("u must be a float64 CUDA tensor of n_src elements")
            if out is None:
                out = torch.empty(self.n_tgt, dtype=torch.complex128, device=u.device)
            if field_out is None:
                field_out = torch.empty(self.n_tgt, dtype=torch.complex128, device=u.device)
            _check(L.fmm_eval_field(self._plan, C.c_void_p(u.data_ptr()), C.c_void_p(out.data_ptr()),
                                    C.c_void_p(field_out.data_ptr())))
            return out, field_out
        u = np.ascontiguousarray(u, dtype=np.float64)
        if len(u) != self.n_src:
            raise ValueError("u must have n_src elements")
        res = np.empty(self.n_tgt, dtype=np.complex128) if out is None else out
        fld = np.empty(self.n_tgt, dtype=np.complex128) if field_out is None else field_out
        _check(L.fmm_eval_field(self._plan, C.c_void_p(u.ctypes.data) if self.n_src else None,
                                C.c_void_p(res.ctypes.data) if self.n_tgt else None,
                                C.c_void_p(fld.ctypes.data) if self.n_tgt else None))
        return res, fld

    # -------------------------------------------------------------- info
    def info(self) -> dict:
        inf = PlanInfo()
        _check(lib().fmm_plan_info_get(self._plan, C.byref(inf)))
        return {
            "tiling": inf.tiling, "lmax": inf.lmax, "p": inf.p,
            "precision": PREC_NAMES.get(inf.precision, inf.precision),
            "geometry": tuple(inf.geometry), "n_src": inf.n_src, "n_tgt": inf.n_tgt,
            "targets_are_sources": bool(inf.targets_are_sources), "e4_width": inf.e4_width,
            "n_cells": list(inf.n_cells[: inf.lmax + 1]), "n_m2l_pairs": inf.n_m2l_pairs,
            "n_near_pairs": inf.n_near_pairs, "device_bytes": inf.device_bytes,
            "plan_ms": inf.plan_ms, "eval_ms": inf.eval_ms, "stage_ms": list(inf.stage_ms[:5]),
        }

    def export_points(self):
        sk = np.empty(self.n_src, dtype=np.int64)
        tk = np.empty(self.n_tgt, dtype=np.int64)
        sp = np.empty(self.n_src, dtype=np.int64)
        tp = np.empty(self.n_tgt, dtype=np.int64)
        P64 = C.POINTER(C.c_int64)
        _check(lib().fmm_plan_export_points(self._plan, sk.ctypes.data_as(P64),
                                            tk.ctypes.data_as(P64), sp.ctypes.data_as(P64),
                                            tp.ctypes.data_as(P64)))
        return {"src_keys": sk, "tgt_keys": tk, "src_perm": sp, "tgt_perm": tp}

    def export_level(self, level: int) -> dict:
        inf = self.info()
        n = inf["n_cells"][level]
        w = inf["e4_width"]
        keys = np.empty(n, dtype=np.int64)
        occ = np.empty(n, dtype=np.int32)
        sr = np.empty(2 * n, dtype=np.int64)
        tr = np.empty(2 * n, dtype=np.int64)
        e4 = np.empty(n * w, dtype=np.int64)
        near = np.empty(n * 13, dtype=np.int64)
        P64 = C.POINTER(C.c_int64)
        _check(lib().fmm_plan_export_level(self._plan, int(level), keys.ctypes.data_as(P64),
                                           occ.ctypes.data_as(C.POINTER(C.c_int32)),
                                           sr.ctypes.data_as(P64), tr.ctypes.data_as(P64),
                                           e4.ctypes.data_as(P64), near.ctypes.data_as(P64)))
        return {"keys": keys, "occupancy": occ, "src_range": sr.reshape(n, 2),
                "tgt_range": tr.reshape(n, 2), "e4": e4.reshape(n, w),
                "near": near.reshape(n, 13) if level == inf["lmax"] else None}

    def close(self):
        if getattr(self, "_plan", None) and self._plan.value:
            lib().fmm_plan_destroy(self._plan)
            self._plan = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def solve(tiling, xs, ys, u, xt=None, yt=None, eps=1e-6, **kw):
    """One-shot host solve: plan + eval + destroy."""
    with Plan(tiling, xs, ys, xt, yt, eps, **kw) as p:
        return p.eval(u)


def direct(xs, ys, u, xt=None, yt=None, *, src=None, tgt=None, out=None, stream=None):
    """Direct sum of u_i Log(y_j - x_i) on the GPU (fmm_direct in the C ABI).

    Host mode: direct(xs, ys, u, xt, yt) with numpy arrays (targets default
    to the sources) returns a complex128 ndarray.  Device mode:
    direct(None, None, u, src=tensor, tgt=tensor) with complex128 CUDA
    tensors returns (or fills) a complex128 CUDA tensor, ordered on `stream`
    (default: torch's current stream)."""
    L = lib()
    opt = Options()
    _check(L.fmm_options_default(C.byref(opt)))
    if src is not None and _is_torch(src) and src.is_cuda:
        import torch
        s = src.contiguous()
        t = s if (tgt is None or tgt is src) else tgt.contiguous()
        for a in (s, t):
            if a.dtype != torch.complex128:
                raise TypeError("device points must be complex128")
        u = u.contiguous()
        if u.dtype != torch.float64 or not u.is_cuda or u.numel() != s.numel():
            raise TypeError("u must be a float64 CUDA tensor of n_src elements")
        if out is None:
            out = torch.empty(t.numel(), dtype=torch.complex128, device=s.device)
        opt.device_pointers = 1
        st = stream if stream is not None else torch.cuda.current_stream()
        opt.stream = C.c_void_p(st.cuda_stream)
        _check(L.fmm_direct(C.c_void_p(s.data_ptr()), s.numel(), C.c_void_p(t.data_ptr()), t.numel(),
                            C.c_void_p(u.data_ptr()), C.c_void_p(out.data_ptr()), C.byref(opt)))
        return out
    s = _points_host(src) if src is not None else _points_host(xs, ys)
    if tgt is not None:
        t = _points_host(tgt)
    elif xt is not None:
        t = _points_host(xt, yt)
    else:
        t = s
    u = np.ascontiguousarray(u, dtype=np.float64)
    ns, nt = len(s) // 2, len(t) // 2
    if len(u) != ns:
        raise ValueError("u must have n_src elements")
    res = np.empty(nt, dtype=np.complex128) if out is None else out
    _check(L.fmm_direct(C.c_void_p(s.ctypes.data) if ns else None, ns,
                        C.c_void_p(t.ctypes.data) if nt else None, nt,
                        C.c_void_p(u.ctypes.data) if ns else None,
                        C.c_void_p(res.ctypes.data) if nt else None, C.byref(opt)))
    return res


def direct_noalloc(src, tgt, u, out, stream=None):
    """fmm_direct_noalloc: the direct sum of `direct` with device tensors
    only, writing into the caller's `out` (complex128, one per target) and
    taking its partial sums from the library's fixed device scratch instead
    of allocating.  Ordered on `stream` (default: torch's current stream);
    returns `out`."""
    import torch
    L = lib()
    for a in (src, tgt):
        if not (_is_torch(a) and a.is_cuda and a.dtype == torch.complex128 and a.is_contiguous()):
            raise TypeError("points must be contiguous complex128 CUDA tensors")
    if not (u.is_cuda and u.dtype == torch.float64 and u.is_contiguous() and u.numel() == src.numel()):
        raise TypeError("u must be a contiguous float64 CUDA tensor of n_src elements")
    if not (out.is_cuda and out.dtype == torch.complex128 and out.is_contiguous() and out.numel() == tgt.numel()):
        raise TypeError("out must be a contiguous complex128 CUDA tensor of n_tgt elements")
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(L.fmm_direct_noalloc(C.c_void_p(src.data_ptr()), src.numel(), C.c_void_p(tgt.data_ptr()),
                                tgt.numel(), C.c_void_p(u.data_ptr()), C.c_void_p(out.data_ptr()),
                                C.c_void_p(st.cuda_stream)))
    return out


def probe_pair_rate(rounds: int = 2000, blocks: int = 0) -> float:
    """fmm_probe_pair_rate: FP64 pair evaluations per second that the near
    field's pair function reaches with its operands in registers (the
    near-field kernel's ceiling on this chip)."""
    L = lib()
    r = C.c_double(0.0)
    _check(L.fmm_probe_pair_rate(int(rounds), int(blocks), C.byref(r)))
    return float(r.value)


class Server:
    """Continuous-batching solve server (fmm_server_* in the C ABI).

    submit() copies the inputs and returns a ticket; poll() returns None while
    the request is queued or running, else (phi, result) where result holds
    the status, p, lmax and the submit / admit / start / end timestamps
    (seconds, steady clock)."""

    def __init__(self, hbm_budget_bytes: int = 8 << 30, max_inflight: int = 64, leaf_size: int = 64):
        L = lib()
        o = ServerOptions()
        o.struct_size = C.sizeof(ServerOptions)
        o.hbm_budget_bytes = int(hbm_budget_bytes)
        o.max_inflight = int(max_inflight)
        o.leaf_size = int(leaf_size)
        self._s = C.c_void_p()
        _check(L.fmm_server_create(C.byref(o), C.byref(self._s)))
        self._n = {}

    def submit(self, tiling, xs, ys, u, eps=1e-6, precision="auto", xt=None, yt=None) -> int:
        src = _points_host(xs, ys)
        tgt = None if xt is None else _points_host(xt, yt)
        u = np.ascontiguousarray(u, dtype=np.float64)
        r = Request()
        r.tiling = _tiling(tiling)
        r.precision = PREC[precision] if isinstance(precision, str) else int(precision)
        r.eps = float(eps)
        r.n_src = len(src) // 2
        r.n_tgt = r.n_src if tgt is None else len(tgt) // 2
        r.src = src.ctypes.data if r.n_src else None
        r.tgt = None if tgt is None else (tgt.ctypes.data if r.n_tgt else None)
        r.u = u.ctypes.data if r.n_src else None
        t = C.c_uint64()
        _check(lib().fmm_submit(self._s, C.byref(r), C.byref(t)))
        self._n[t.value] = r.n_tgt
        return t.value

    def poll(self, ticket: int, want_phi: bool = True):
        """None while the request is queued or running; then (phi, result),
        phi None when want_phi is false (the result is still consumed)."""
        n = self._n[ticket]
        phi = np.empty(n, dtype=np.complex128) if want_phi else None
        res = Result()
        st = lib().fmm_poll(self._s, C.c_uint64(ticket),
                            phi.ctypes.data_as(C.POINTER(C.c_double)) if (n and want_phi) else None,
                            C.byref(res))
        if st == 5:
            return None
        del self._n[ticket]
        out = {"status": STATUS.get(res.status, res.status), "p": res.p, "lmax": res.lmax,
               "t_submit": res.t_submit, "t_admit": res.t_admit, "t_start": res.t_start,
               "t_end": res.t_end}
        return (phi if st == 0 else None), out

    def drain(self):
        _check(lib().fmm_server_drain(self._s))

    def close(self):
        if getattr(self, "_s", None) and self._s.value:
            lib().fmm_server_destroy(self._s)
            self._s = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
