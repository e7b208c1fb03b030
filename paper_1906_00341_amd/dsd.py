"""Thin ctypes binding of libdsd (include/dsd.h): argument marshalling only.

Every computation runs in the HIP library; this module only converts numpy
arrays / torch tensors to pointers and status codes to exceptions.  There is
no CPU fallback: a missing library or GPU raises.

Names follow the C ABI: ``build_csr``, ``clique_degrees``, ``clique_core``,
``core_app``, ``core_exact``, ``batch_run`` and the ``Server`` class
(``dsd_server_*``).
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdsd.so")

DSD_MEM_HOST = 0
DSD_MEM_DEVICE = 1

STATUS = {0: "DSD_OK", -1: "DSD_EINVAL", -2: "DSD_ENOMEM", -3: "DSD_EDEVICE",
          -4: "DSD_EOVERFLOW", -5: "DSD_EUNSUPPORTED", -6: "DSD_EBUSY", -7: "DSD_ETIMEDOUT",
          -8: "DSD_ECANCELED"}
DSD_EBUSY, DSD_ETIMEDOUT, DSD_ECANCELED = -6, -7, -8

OP_DEGREES, OP_CORE, OP_APP, OP_EXACT, OP_PEEL = 0, 1, 2, 3, 4
OPS = {"degrees": OP_DEGREES, "core": OP_CORE, "app": OP_APP, "exact": OP_EXACT, "peel": OP_PEEL}

EXPORTS = ["dsd_build_csr", "dsd_graph_info", "dsd_graph_free", "dsd_clique_degrees", "dsd_clique_degrees_noalloc",
           "dsd_autotune", "dsd_tune_load",
           "dsd_clique_core", "dsd_core_app", "dsd_peel_app", "dsd_core_exact", "dsd_core_exact_query",
           "dsd_pattern_degrees", "dsd_pattern_core",
           "dsd_last_stats", "dsd_set_kernel_timing", "dsd_release_cache",
           "dsd_batch_run", "dsd_server_create", "dsd_server_submit", "dsd_server_wait",
           "dsd_server_cancel", "dsd_server_destroy", "dsd_status_str", "dsd_last_error"]


class DsdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Rational(C.Structure):
    _fields_ = [("num", C.c_uint64), ("den", C.c_uint64)]


class TuneResult(C.Structure):
    _fields_ = [("cls", C.c_int32), ("roots", C.c_int32), ("cap_default", C.c_int32), ("cap_best", C.c_int32),
                ("ms_default", C.c_double), ("ms_best", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Stats(C.Structure):
    _fields_ = [("t_orient_ms", C.c_double), ("t_enum_ms", C.c_double), ("t_peel_ms", C.c_double),
                ("t_locate_ms", C.c_double), ("t_exact_ms", C.c_double), ("t_total_ms", C.c_double),
                ("num_cliques", C.c_uint64), ("peel_rounds", C.c_uint64), ("peel_levels", C.c_uint64),
                ("flow_calls", C.c_uint64), ("flow_nodes_max", C.c_uint64),
                ("located_vertices", C.c_uint64),
                ("k3_ms", C.c_double), ("k4_ms", C.c_double),
                ("k3_launches", C.c_uint64), ("k4_launches", C.c_uint64),
                ("n", C.c_uint64), ("m", C.c_uint64), ("w2", C.c_uint64), ("s2", C.c_uint64),
                ("t_flow_build_ms", C.c_double), ("t_flow_ms", C.c_double),
                ("k4_main_ms", C.c_double), ("k4_main_launches", C.c_uint64),
                ("k4_main_pairs", C.c_uint64), ("k4_main_nbrs", C.c_uint64),
                ("flow_gpu_calls", C.c_uint64), ("k4_main_kind", C.c_uint64),
                ("t_flow_setup_ms", C.c_double), ("flow_gpu_networks", C.c_uint64),
                ("k4_tail_ms", C.c_double), ("k4_tail_launches", C.c_uint64), ("k4_tail_pairs", C.c_uint64),
                ("k4_tail_vertices", C.c_uint64), ("k4_tail_grid_ms", C.c_double),
                ("k4_tail_grid_rounds", C.c_uint64), ("k4_tail_grid_pairs", C.c_uint64),
                ("locate_rho1_num", C.c_uint64), ("locate_rho1_den", C.c_uint64), ("locate_k1", C.c_uint64),
                ("locate_rho2_num", C.c_uint64), ("locate_rho2_den", C.c_uint64), ("locate_k2", C.c_uint64),
                ("locate_components", C.c_uint64), ("k4_main_entries", C.c_uint64),
                ("k4_main2_ms", C.c_double), ("k4_main2_launches", C.c_uint64),
                ("k4_main2_words", C.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Result(C.Structure):
    """dsd_result: the scalar outcome of one graph of a batch or one served request."""
    _fields_ = [("status", C.c_int), ("h", C.c_int32), ("op", C.c_int32),
                ("num_cliques", C.c_uint64), ("kmax", C.c_uint64), ("density", Rational),
                ("members", C.c_uint64), ("peel_rounds", C.c_uint64), ("t_ms", C.c_double)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "density"}
        d["density"] = Fraction(self.density.num, self.density.den or 1)
        return d


_NOT_WRITTEN = -999
_lib = None


def load(path: str = LIB_PATH):
    """Load libdsd.so (built by paper_1906_00341_amd/build.py); raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"libdsd.so not built at {path}; run paper_1906_00341_amd/build.py")
    # torch provides device memory and streams; loading it first makes libdsd
    # bind to the same HIP runtime (both carry the soname libamdhip64.so.7)
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover
        pass
    lib = C.CDLL(path)
    P, I32, I64, I = C.c_void_p, C.c_int32, C.c_int64, C.c_int
    lib.dsd_build_csr.argtypes = [I32, I64, P, P, I, P, C.POINTER(P)]
    lib.dsd_graph_info.argtypes = [P, C.POINTER(I32), C.POINTER(I64)]
    lib.dsd_graph_free.argtypes = [P]
    lib.dsd_release_cache.argtypes = []
    lib.dsd_clique_degrees.argtypes = [P, I, I, P, C.POINTER(C.c_uint64)]
    lib.dsd_clique_degrees_noalloc.argtypes = [P, I, I, P, C.POINTER(C.c_uint64)]
    lib.dsd_autotune.argtypes = [P, I, C.c_char_p, I32, C.POINTER(TuneResult), C.POINTER(I32)]
    lib.dsd_tune_load.argtypes = [C.c_char_p]
    lib.dsd_clique_core.argtypes = [P, I, I, P, C.POINTER(C.c_uint64)]
    lib.dsd_core_app.argtypes = [P, I, I, P, C.POINTER(C.c_uint64), C.POINTER(Rational)]
    lib.dsd_peel_app.argtypes = [P, I, I, P, C.POINTER(Rational), C.POINTER(I64), C.POINTER(I64)]
    lib.dsd_core_exact.argtypes = [P, I, I, P, C.POINTER(Rational)]
    lib.dsd_core_exact_query.argtypes = [P, I, I32, P, I, P, C.POINTER(Rational)]
    lib.dsd_pattern_degrees.argtypes = [P, I, I, I, P, C.POINTER(C.c_uint64)]
    lib.dsd_pattern_core.argtypes = [P, I, I, I, P, C.POINTER(C.c_uint64)]
    lib.dsd_last_stats.argtypes = [P, C.POINTER(Stats)]
    lib.dsd_batch_run.argtypes = [I32, C.POINTER(P), C.POINTER(I), I, I, C.POINTER(P), C.POINTER(Result)]
    lib.dsd_server_create.argtypes = [C.c_size_t, I, C.POINTER(P)]
    lib.dsd_server_submit.argtypes = [P, P, I, I, I, P, C.POINTER(C.c_uint64)]
    lib.dsd_server_wait.argtypes = [P, C.c_uint64, I64, C.POINTER(Result)]
    lib.dsd_server_cancel.argtypes = [P, C.c_uint64]
    lib.dsd_server_destroy.argtypes = [P]
    lib.dsd_status_str.argtypes = [I]
    lib.dsd_status_str.restype = C.c_char_p
    lib.dsd_last_error.restype = C.c_char_p
    for f in EXPORTS[:-2]:
        getattr(lib, f).restype = I
    _lib = lib
    atexit.register(_release_at_exit)
    return lib


# Handles and servers still alive when the interpreter exits are released
# here, from an atexit hook: it runs while the HIP runtime is still up,
# before the interpreter clears modules and before the C library runs the
# runtime's own exit handlers.  A finalizer that ran later would call into a
# runtime that is already gone.
_live_graphs = weakref.WeakSet()
_live_servers = weakref.WeakSet()
_exiting = False


def _release_at_exit():
    global _exiting
    if _lib is None or _exiting:
        return
    for s in list(_live_servers):
        s.close()
    for g in list(_live_graphs):
        g.free()
    _lib.dsd_release_cache()
    _exiting = True


def _check(rc: int):
    if rc != 0:
        raise DsdError(rc, (_lib.dsd_last_error() or b"").decode())


def _ptr(a):
    """(pointer, mem flag, keepalive) for a numpy array or a torch tensor."""
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be contiguous")
        return a.ctypes.data, DSD_MEM_HOST, a
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(a, torch.Tensor):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr(), (DSD_MEM_DEVICE if a.is_cuda else DSD_MEM_HOST), a
    raise TypeError(f"unsupported buffer type {type(a)}")


class Graph:
    """A device-resident graph handle (dsd_graph)."""

    def __init__(self, handle):
        self._h = handle
        _live_graphs.add(self)

    @property
    def handle(self):
        return self._h

    def info(self):
        n, m = C.c_int32(), C.c_int64()
        _check(_lib.dsd_graph_info(self._h, C.byref(n), C.byref(m)))
        return int(n.value), int(m.value)

    def free(self):
        if self._h is not None and _lib is not None and not _exiting:
            _lib.dsd_graph_free(self._h)
        self._h = None

    def __del__(self):
        self.free()

    def stats(self) -> dict:
        s = Stats()
        _check(_lib.dsd_last_stats(self._h, C.byref(s)))
        return s.as_dict()

    def set_kernel_timing(self, on: bool):
        """dsd_set_kernel_timing: HIP events around every launch of the peel's main kernel."""
        _check(_lib.dsd_set_kernel_timing(self._h, 1 if on else 0))


def build_csr(n: int, src, dst, stream=None) -> Graph:
    """dsd_build_csr: src/dst int32 numpy arrays (host) or torch int32 tensors (host or device)."""
    lib = load()
    if isinstance(src, np.ndarray):
        src = np.ascontiguousarray(src, dtype=np.int32)
    if isinstance(dst, np.ndarray):
        dst = np.ascontiguousarray(dst, dtype=np.int32)
    ps, ms, ks = _ptr(src)
    pd, md, kd = _ptr(dst)
    if ms != md:
        raise ValueError("src and dst must live in the same memory")
    if len(src) != len(dst):
        raise ValueError("src and dst differ in length")
    h = C.c_void_p()
    _check(lib.dsd_build_csr(int(n), int(len(src)), ps, pd, ms, stream, C.byref(h)))
    del ks, kd
    return Graph(h)


def _out_u64(g: Graph, out):
    n, _ = g.info()
    if out is None:
        out = np.zeros(max(n, 1), dtype=np.uint64)
    p, mem, keep = _ptr(out)
    return out, p, mem


def clique_degrees(g: Graph, h: int, out=None):
    """dsd_clique_degrees -> (deg[n], mu)."""
    out, p, mem = _out_u64(g, out)
    mu = C.c_uint64()
    _check(_lib.dsd_clique_degrees(g.handle, int(h), mem, p, C.byref(mu)))
    n, _ = g.info()
    return out[:n] if isinstance(out, np.ndarray) else out, int(mu.value)


def clique_degrees_noalloc(g: Graph, h: int, out=None):
    """dsd_clique_degrees_noalloc -> (deg[n], mu): the same results with no
    device allocation (a fixed scratch array inside the library)."""
    out, p, mem = _out_u64(g, out)
    mu = C.c_uint64()
    _check(_lib.dsd_clique_degrees_noalloc(g.handle, int(h), mem, p, C.byref(mu)))
    n, _ = g.info()
    return out[:n] if isinstance(out, np.ndarray) else out, int(mu.value)


def autotune(g: Graph, h: int, path=None):
    """dsd_autotune -> one dict per measured class of the enumeration's
    roots (class, roots, default and chosen grid caps, their launch times);
    the chosen caps go to the library's table and, with path, to that JSON
    file."""
    cap = 8
    res = (TuneResult * cap)()
    cnt = C.c_int32()
    p = None if path is None else os.fsencode(path)
    _check(load().dsd_autotune(g.handle, int(h), p, cap, res, C.byref(cnt)))
    return [res[i].as_dict() for i in range(min(cnt.value, cap))]


def tune_load(path=None):
    """dsd_tune_load: the enumeration's grid caps from a JSON file written by
    autotune (None: back to the built-in caps)."""
    _check(load().dsd_tune_load(None if path is None else os.fsencode(path)))


def release_cache():
    """dsd_release_cache: free the device memory that freed handles left for reuse."""
    _check(_lib.dsd_release_cache())


def clique_core(g: Graph, h: int, out=None):
    """dsd_clique_core -> (core[n], kmax)."""
    out, p, mem = _out_u64(g, out)
    km = C.c_uint64()
    _check(_lib.dsd_clique_core(g.handle, int(h), mem, p, C.byref(km)))
    n, _ = g.info()
    return out[:n] if isinstance(out, np.ndarray) else out, int(km.value)


def _out_u8(g: Graph, out):
    n, _ = g.info()
    if out is None:
        out = np.zeros(max(n, 1), dtype=np.uint8)
    p, mem, keep = _ptr(out)
    return out, p, mem, n


def core_app(g: Graph, h: int, out=None):
    """dsd_core_app -> (member[n] uint8, kmax, density Fraction)."""
    out, p, mem, n = _out_u8(g, out)
    km, r = C.c_uint64(), Rational()
    _check(_lib.dsd_core_app(g.handle, int(h), mem, p, C.byref(km), C.byref(r)))
    return (out[:n] if isinstance(out, np.ndarray) else out), int(km.value), Fraction(r.num, r.den)


def peel_app(g: Graph, h: int, out=None):
    """dsd_peel_app -> (member[n] uint8, density Fraction, rounds, best_round)."""
    out, p, mem, n = _out_u8(g, out)
    r, rounds, best = Rational(), C.c_int64(), C.c_int64()
    _check(_lib.dsd_peel_app(g.handle, int(h), mem, p, C.byref(r), C.byref(rounds), C.byref(best)))
    return ((out[:n] if isinstance(out, np.ndarray) else out), Fraction(r.num, r.den),
            int(rounds.value), int(best.value))


def core_exact(g: Graph, h: int, out=None):
    """dsd_core_exact -> (member[n] uint8, rho_opt Fraction)."""
    out, p, mem, n = _out_u8(g, out)
    r = Rational()
    _check(_lib.dsd_core_exact(g.handle, int(h), mem, p, C.byref(r)))
    return (out[:n] if isinstance(out, np.ndarray) else out), Fraction(r.num, r.den)


def core_exact_query(g: Graph, h: int, q, out=None):
    """dsd_core_exact_query -> (member[n] uint8, density Fraction): the densest
    subgraph containing every vertex of q."""
    q = np.ascontiguousarray(np.atleast_1d(q), dtype=np.int32)
    out, p, mem, n = _out_u8(g, out)
    r = Rational()
    _check(_lib.dsd_core_exact_query(g.handle, int(h), int(q.size), q.ctypes.data_as(C.c_void_p), mem, p,
                                     C.byref(r)))
    return (out[:n] if isinstance(out, np.ndarray) else out), Fraction(r.num, r.den)


PATTERN_STAR, PATTERN_LOOP4 = 1, 2


def pattern_degrees(g: Graph, pattern: int, x: int, out=None):
    """dsd_pattern_degrees -> (deg[n], instances)."""
    out, p, mem = _out_u64(g, out)
    cnt = C.c_uint64()
    _check(_lib.dsd_pattern_degrees(g.handle, int(pattern), int(x), mem, p, C.byref(cnt)))
    n, _ = g.info()
    return out[:n] if isinstance(out, np.ndarray) else out, int(cnt.value)


def pattern_core(g: Graph, pattern: int, x: int, out=None):
    """dsd_pattern_core -> (core[n], kmax)."""
    out, p, mem = _out_u64(g, out)
    km = C.c_uint64()
    _check(_lib.dsd_pattern_core(g.handle, int(pattern), int(x), mem, p, C.byref(km)))
    n, _ = g.info()
    return out[:n] if isinstance(out, np.ndarray) else out, int(km.value)


def status_str(s: int) -> str:
    return load().dsd_status_str(int(s)).decode()


def _op(op) -> int:
    return OPS[op] if isinstance(op, str) else int(op)


def batch_run(graphs, hs, op, outs=None, out_mem=None):
    """dsd_batch_run -> list of result dicts (one per graph, each with its own
    ``status``).  outs: None or a list (entries None, numpy arrays or torch
    tensors of n_i entries: uint64 for degrees/core, uint8 for app/exact/peel; all
    in the same memory).  Raises DsdError for argument errors."""
    lib = load()
    cnt = len(graphs)
    if isinstance(hs, int):
        hs = [hs] * cnt
    arr_g = (C.c_void_p * cnt)(*[g.handle for g in graphs])
    arr_h = (C.c_int * cnt)(*[int(x) for x in hs])
    res = (Result * cnt)()
    for r in res:
        r.status = _NOT_WRITTEN
    keep, arr_o, mem = [], None, DSD_MEM_HOST
    if outs is not None:
        ptrs = []
        for o in outs:
            if o is None:
                ptrs.append(None)
                continue
            p, m, k = _ptr(o)
            ptrs.append(p)
            keep.append(k)
            mem = m
        arr_o = (C.c_void_p * cnt)(*ptrs)
    if out_mem is not None:
        mem = out_mem
    rc = lib.dsd_batch_run(cnt, arr_g, arr_h, _op(op), mem, arr_o, res)
    if cnt and res[0].status == _NOT_WRITTEN:
        _check(rc)
    return [r.as_dict() for r in res]


class Server:
    """dsd_server_*: queued requests served in batches by a worker thread."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int):
        lib = load()
        self._s = C.c_void_p()
        _check(lib.dsd_server_create(int(hbm_budget_bytes), int(max_slots), C.byref(self._s)))
        self._keep = {}
        _live_servers.add(self)

    def submit(self, g: Graph, h: int, op, out=None) -> int:
        p, mem, k = (None, DSD_MEM_HOST, None) if out is None else _ptr(out)
        t = C.c_uint64()
        _check(_lib.dsd_server_submit(self._s, g.handle, int(h), _op(op), mem, p, C.byref(t)))
        self._keep[int(t.value)] = (g, k)
        return int(t.value)

    def wait(self, ticket: int, timeout_us: int = -1):
        """(status, result dict or None): status 0, DSD_ETIMEDOUT or DSD_ECANCELED."""
        r = Result()
        rc = _lib.dsd_server_wait(self._s, int(ticket), int(timeout_us), C.byref(r))
        if rc == DSD_ETIMEDOUT:
            return rc, None
        self._keep.pop(int(ticket), None)
        if rc == DSD_ECANCELED:
            return rc, None
        _check(rc)
        return 0, r.as_dict()

    def cancel(self, ticket: int) -> int:
        rc = _lib.dsd_server_cancel(self._s, int(ticket))
        if rc not in (0, DSD_EBUSY):
            _check(rc)
        return rc

    def close(self):
        if self._s is not None and _lib is not None and not _exiting:
            _lib.dsd_server_destroy(self._s)
        self._s = None
        self._keep.clear()

    def __del__(self):
        self.close()
