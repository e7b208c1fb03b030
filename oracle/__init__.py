"""CPU oracle for the k-clique-core densest-subgraph path (Python side).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It wraps the
plain single-threaded C library in ``oracle.c`` (built with gcc by
``oracle/buildlib.py``) and shares no code with the GPU library.  For the
benchmark's secondary CPU line only, ``omp_enum.c`` runs the same clique
listing on OpenMP threads (``clique_degrees_omp``, checked against
``Graph.clique_degrees``).

All counts are exact integers and all densities are ``fractions.Fraction``.
"""
from __future__ import annotations

import ctypes as C
import os
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    from . import buildlib as _b
    return _b.build(force=force)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = C.CDLL(_LIB_PATH)
    P = C.c_void_p
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
    u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
    u64 = C.POINTER(C.c_uint64)
    i64 = C.POINTER(C.c_int64)
    lib.orc_graph_new.restype = P
    lib.orc_graph_new.argtypes = [C.c_int32, C.c_int64, i32p, i32p]
    lib.orc_graph_free.argtypes = [P]
    lib.orc_graph_n.restype = C.c_int32
    lib.orc_graph_n.argtypes = [P]
    lib.orc_graph_m.restype = C.c_int64
    lib.orc_graph_m.argtypes = [P]
    lib.orc_graph_adjacency.argtypes = [P, i64p, i32p]
    lib.orc_clique_degrees.argtypes = [P, C.c_int, u64p, u64]
    lib.orc_clique_degree_of.argtypes = [P, C.c_int, C.c_int32, u64]
    lib.orc_core_decomposition.argtypes = [P, C.c_int, u64p, u64]
    lib.orc_level_table.argtypes = [P, C.c_int, u64p, u64p, u64p, u64p, i64]
    lib.orc_inc_app.argtypes = [P, C.c_int, u8p, u64, u64, u64]
    lib.orc_core_app.argtypes = [P, C.c_int, C.c_int, C.c_int64, u8p, u64, u64, u64, i64]
    lib.orc_peel_app.argtypes = [P, C.c_int, C.c_int, u8p, u64, u64, i64, i64]
    lib.orc_locate.argtypes = [P, C.c_int, u64p, u64, u64, u64, u64, u64, u64, i32p, i64]
    lib.orc_exact.argtypes = [P, C.c_int, C.c_int, u8p, u64, u64, i64]
    lib.orc_denser_than.argtypes = [P, C.c_int, C.c_uint64, C.c_uint64, u8p]
    lib.orc_pattern_degrees.argtypes = [P, C.c_int, C.c_int, u64p, u64]
    lib.orc_pattern_core.argtypes = [P, C.c_int, C.c_int, u64p, u64]
    lib.orc_exact_query.argtypes = [P, C.c_int, C.c_int32, i32p, u8p, u64, u64, i64]
    for f in ("orc_clique_degrees", "orc_clique_degree_of", "orc_core_decomposition",
              "orc_level_table", "orc_inc_app", "orc_core_app", "orc_peel_app", "orc_locate",
              "orc_exact", "orc_denser_than", "orc_exact_query", "orc_pattern_degrees", "orc_pattern_core"):
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise OracleError(f"{what}: status {rc}")
    return rc


class Graph:
    """A simple undirected graph built by the oracle from raw vertex pairs."""

    def __init__(self, n: int, src, dst):
        lib = _load()
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        if src.shape != dst.shape:
            raise ValueError("src and dst differ in length")
        p = lib.orc_graph_new(int(n), int(src.size), src, dst)
        if not p:
            raise ValueError("vertex id out of range or negative n")
        self._p = C.c_void_p(p)
        self.n = int(lib.orc_graph_n(self._p))
        self.m = int(lib.orc_graph_m(self._p))

    def __del__(self):
        p = getattr(self, "_p", None)
        if p is not None and _lib is not None:
            _lib.orc_graph_free(p)
            self._p = None

    def adjacency(self):
        off = np.zeros(self.n + 1, dtype=np.int64)
        adj = np.zeros(max(1, 2 * self.m), dtype=np.int32)
        _lib.orc_graph_adjacency(self._p, off, adj)
        return off, adj[: 2 * self.m]

    # -- Definition 3 ---------------------------------------------------
    def clique_degrees(self, h: int):
        deg = np.zeros(max(1, self.n), dtype=np.uint64)
        mu = C.c_uint64()
        _check(_lib.orc_clique_degrees(self._p, h, deg, C.byref(mu)), "clique_degrees")
        return deg[: self.n], int(mu.value)

    def clique_degree_of(self, h: int, v: int) -> int:
        out = C.c_uint64()
        _check(_lib.orc_clique_degree_of(self._p, h, int(v), C.byref(out)), "clique_degree_of")
        return int(out.value)

    # -- Alg. 3 ---------------------------------------------------------
    def core_decomposition(self, h: int):
        core = np.zeros(max(1, self.n), dtype=np.uint64)
        kmax = C.c_uint64()
        _check(_lib.orc_core_decomposition(self._p, h, core, C.byref(kmax)), "core_decomposition")
        return core[: self.n], int(kmax.value)

    def level_table(self, h: int, core):
        core = np.ascontiguousarray(core, dtype=np.uint64)
        if core.size == 0:
            core = np.zeros(1, np.uint64)
        lv = np.zeros(self.n + 2, dtype=np.uint64)
        rs = np.zeros(self.n + 2, dtype=np.uint64)
        rm = np.zeros(self.n + 2, dtype=np.uint64)
        nl = C.c_int64()
        _check(_lib.orc_level_table(self._p, h, core, lv, rs, rm, C.byref(nl)), "level_table")
        k = nl.value
        return lv[:k], rs[:k], rm[:k]

    # -- Alg. 5 / Alg. 6 ------------------------------------------------
    def inc_app(self, h: int):
        mem = np.zeros(max(1, self.n), dtype=np.uint8)
        kmax, a, b = C.c_uint64(), C.c_uint64(), C.c_uint64()
        _check(_lib.orc_inc_app(self._p, h, mem, C.byref(kmax), C.byref(a), C.byref(b)), "inc_app")
        return mem[: self.n].astype(bool), int(kmax.value), Fraction(int(a.value), int(b.value))

    def core_app(self, h: int, literal: bool = False, w0: int = 0):
        mem = np.zeros(max(1, self.n), dtype=np.uint8)
        kmax, a, b = C.c_uint64(), C.c_uint64(), C.c_uint64()
        it = C.c_int64()
        _check(_lib.orc_core_app(self._p, h, int(bool(literal)), int(w0), mem, C.byref(kmax),
                                 C.byref(a), C.byref(b), C.byref(it)), "core_app")
        return (mem[: self.n].astype(bool), int(kmax.value),
                Fraction(int(a.value), int(b.value)), int(it.value))

    # -- Alg. 2 ---------------------------------------------------------
    def peel_app(self, h: int, rounds: bool = True):
        """PeelApp.  rounds=True: every minimum-degree vertex leaves in the
        same step; False: one vertex (smallest id) per step.  Returns
        (member, density, steps, best_step)."""
        mem = np.zeros(max(1, self.n), dtype=np.uint8)
        a, b = C.c_uint64(), C.c_uint64()
        st, bs = C.c_int64(), C.c_int64()
        _check(_lib.orc_peel_app(self._p, h, int(bool(rounds)), mem, C.byref(a), C.byref(b),
                                 C.byref(st), C.byref(bs)), "peel_app")
        return (mem[: self.n].astype(bool), Fraction(int(a.value), int(b.value)),
                int(st.value), int(bs.value))

    # -- special patterns (1 = x-star, 2 = 4-loop) -------------------------
    def pattern_degrees(self, pattern: int, x: int = 0):
        deg = np.zeros(max(1, self.n), dtype=np.uint64)
        cnt = C.c_uint64()
        _check(_lib.orc_pattern_degrees(self._p, int(pattern), int(x), deg, C.byref(cnt)), "pattern_degrees")
        return deg[: self.n], int(cnt.value)

    def pattern_core(self, pattern: int, x: int = 0):
        core = np.zeros(max(1, self.n), dtype=np.uint64)
        km = C.c_uint64()
        _check(_lib.orc_pattern_core(self._p, int(pattern), int(x), core, C.byref(km)), "pattern_core")
        return core[: self.n], int(km.value)

    # -- Pruning1/2 -----------------------------------------------------
    def locate(self, h: int, core):
        core = np.ascontiguousarray(core, dtype=np.uint64)
        if core.size == 0:
            core = np.zeros(1, np.uint64)
        lab = np.zeros(max(1, self.n), dtype=np.int32)
        r1n, r1d, k1, r2n, r2d, k2 = (C.c_uint64() for _ in range(6))
        nc = C.c_int64()
        _check(_lib.orc_locate(self._p, h, core, C.byref(r1n), C.byref(r1d), C.byref(k1),
                               C.byref(r2n), C.byref(r2d), C.byref(k2), lab, C.byref(nc)), "locate")
        return dict(rho1=Fraction(int(r1n.value), int(r1d.value)), k1=int(k1.value),
                    rho2=Fraction(int(r2n.value), int(r2d.value)), k2=int(k2.value),
                    label=lab[: self.n], ncomp=int(nc.value))

    # -- Alg. 1 / Alg. 4 -------------------------------------------------
    def exact(self, h: int, route: str = "core"):
        mem = np.zeros(max(1, self.n), dtype=np.uint8)
        a, b = C.c_uint64(), C.c_uint64()
        calls = C.c_int64()
        r = {"whole": 0, "core": 1}[route]
        _check(_lib.orc_exact(self._p, h, r, mem, C.byref(a), C.byref(b), C.byref(calls)), "exact")
        return mem[: self.n].astype(bool), Fraction(int(a.value), int(b.value)), int(calls.value)

    def exact_query(self, h: int, q):
        """Densest subgraph containing every vertex of q -> (member, density, flow calls)."""
        q = np.ascontiguousarray(np.atleast_1d(q), dtype=np.int32)
        mem = np.zeros(max(1, self.n), dtype=np.uint8)
        a, b = C.c_uint64(), C.c_uint64()
        calls = C.c_int64()
        _check(_lib.orc_exact_query(self._p, h, int(q.size), q, mem, C.byref(a), C.byref(b), C.byref(calls)),
               "exact_query")
        return mem[: self.n].astype(bool), Fraction(int(a.value), int(b.value)), int(calls.value)

    def denser_than(self, h: int, alpha: Fraction):
        mem = np.zeros(max(1, self.n), dtype=np.uint8)
        rc = _check(_lib.orc_denser_than(self._p, h, alpha.numerator, alpha.denominator, mem),
                    "denser_than")
        return bool(rc), mem[: self.n].astype(bool)


def graph(n, src, dst) -> Graph:
    return Graph(n, src, dst)


_omp = None


def clique_degrees_omp(g: Graph, h: int):
    """The benchmark's secondary CPU line: the same listing as
    ``Graph.clique_degrees`` (each h-clique once, from its smallest-id
    member) with the roots spread over OpenMP threads (``oracle/omp_enum.c``).
    Returns (deg, mu, threads)."""
    global _omp
    if _omp is None:
        path = os.path.join(_HERE, "liboracle_omp.so")
        if not os.path.exists(path):
            build(force=True)
        lib = C.CDLL(path)
        lib.omp_clique_degrees.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                           C.POINTER(C.c_uint64)]
        lib.omp_clique_degrees.restype = C.c_int
        _omp = lib
    off, adj = g.adjacency()
    off = np.ascontiguousarray(off, dtype=np.int64)
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    deg = np.zeros(max(1, g.n), dtype=np.uint64)
    mu = C.c_uint64()
    nt = _omp.omp_clique_degrees(g.n, off.ctypes.data, adj.ctypes.data, int(h), deg.ctypes.data, C.byref(mu))
    if nt < 0:
        raise OracleError("omp_clique_degrees failed")
    return deg[: g.n], int(mu.value), nt
