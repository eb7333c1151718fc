"""CPU oracle for the population graph-coloring hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark may import this package; the product path never
does.  It shares no code with the HIP kernels.

``oracle.c`` holds the search algorithms (plain C, built with gcc);
``scorer.py`` the FP64 numpy reference of the offspring scorer;
``invnet.py`` the FP64 reference of the paper's colour-invariant network;
``brute.py`` exhaustive solvers for tiny graphs used as pins;
``diversity.py`` the partition distance, spacing update and nearest
neighbours of the population (plain Python); ``reduce.py`` the step from k to
k - 1 colours of the decreasing-k driver.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

NSTATS = 8
D_TENURE = 0x80000001
D_INIT = 0x80000002
D_GPXFILL = 0x80000003
D_SELECT = 0x80000006
D_GPXTIE = 0x80000007
D_GREEDY = 0x80000008
TT_CAP = 32757


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, OpenMP, no intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unused-function", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _TabuParams(C.Structure):
    _fields_ = [("k", C.c_int32), ("max_iters", C.c_int32), ("ten_num", C.c_int32),
                ("ten_den", C.c_int32), ("ten_rand", C.c_int32), ("check", C.c_int32),
                ("seed", C.c_uint64)]


class _WvcpParams(C.Structure):
    _fields_ = [("k", C.c_int32), ("iters_per_round", C.c_int32), ("rounds", C.c_int32),
                ("ten_rand", C.c_int32), ("frz_num", C.c_int32), ("frz_den", C.c_int32),
                ("shift", C.c_int32), ("check", C.c_int32), ("seed", C.c_uint64)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB)
            P = C.c_void_p
            L.orc_last_error.restype = C.c_char_p
            L.orc_philox.argtypes = [C.c_uint32] * 4 + [C.c_uint64, P]
            L.orc_uniform.restype = C.c_uint32
            L.orc_uniform.argtypes = [C.c_uint32, C.c_uint32]
            L.orc_conflicts.restype = C.c_int64
            L.orc_conflicts.argtypes = [C.c_int32, P, P, P]
            L.orc_wscore.restype = C.c_int64
            L.orc_wscore.argtypes = [C.c_int32, P, C.c_int32, P]
            L.orc_init_random.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                          C.c_int32, P]
            L.orc_greedy_init.restype = C.c_int32
            L.orc_greedy_init.argtypes = [C.c_int32, P, P, P, C.c_uint64, C.c_int32, P]
            L.orc_tabucol.restype = C.c_int
            L.orc_tabucol.argtypes = [C.c_int32, P, P, P, C.c_int32, P, P, P, P, P, P,
                                      C.c_int32]
            L.orc_tabucol_batch.restype = C.c_int
            L.orc_tabucol_batch.argtypes = [C.c_int32, P, P, P, C.c_int32, P, P, P, P, P, P,
                                            C.c_int32]
            L.orc_wvcp_tabu.restype = C.c_int
            L.orc_wvcp_tabu.argtypes = [C.c_int32, P, P, P, P, C.c_int32, P, P, P, P, P,
                                        C.c_int32, P]
            L.orc_wvcp_batch.restype = C.c_int
            L.orc_wvcp_batch.argtypes = [C.c_int32, P, P, P, P, C.c_int32, P, P, P, P, P,
                                         C.c_int32]
            L.orc_gpx.argtypes = [C.c_int32, C.c_int32, P, P, C.c_uint32, C.c_uint64, P]
            L.orc_gpx_batch.argtypes = [C.c_int32, C.c_int32, P, P, C.c_int32, C.c_int32,
                                        C.c_uint32, C.c_uint64, P]
            L.orc_select.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                     C.c_uint32, P]
            L.orc_random_pairs.argtypes = [C.c_int32, C.c_uint64, C.c_uint32, P]
            _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _csr(g):
    return (np.ascontiguousarray(g.row_ptr, dtype=np.int32),
            np.ascontiguousarray(g.col_idx, dtype=np.int32))


# --------------------------------------------------------------------------
def philox(c0: int, c1: int, c2: int, c3: int, seed: int) -> tuple:
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(c0 & 0xffffffff, c1 & 0xffffffff, c2 & 0xffffffff, c3 & 0xffffffff,
                     seed & 0xffffffffffffffff, _p(out))
    return tuple(int(x) for x in out)


def uniform(x: int, K: int) -> int:
    return int(lib().orc_uniform(x, K))


def conflicts(g, colors: np.ndarray) -> int:
    rp, ci = _csr(g)
    col = np.ascontiguousarray(colors, dtype=np.int16)
    return int(lib().orc_conflicts(g.n, _p(rp), _p(ci), _p(col)))


def wscore(weights: np.ndarray, k: int, colors: np.ndarray) -> int:
    w = np.ascontiguousarray(weights, dtype=np.int32)
    col = np.ascontiguousarray(colors, dtype=np.int16)
    return int(lib().orc_wscore(w.shape[0], _p(w), k, _p(col)))


def init_random(n: int, k: int, pop: int, seed: int, ind_base: int = 0) -> np.ndarray:
    out = np.zeros((pop, n), dtype=np.int16)
    lib().orc_init_random(n, k, pop, seed, ind_base, _p(out))
    return out


def greedy_init(g, seed: int, ind: int) -> tuple[np.ndarray, int]:
    rp, ci = _csr(g)
    w = np.ascontiguousarray(g.weights, dtype=np.int32)
    out = np.zeros(g.n, dtype=np.int16)
    used = lib().orc_greedy_init(g.n, _p(rp), _p(ci), _p(w), seed, ind, _p(out))
    return out, int(used)


def tabucol(g, colors: np.ndarray, k: int, iters: int, seed: int, ind: int,
            ten_num: int = 6, ten_den: int = 10, ten_rand: int = 10,
            check: bool = False, trace_cap: int = 0) -> dict:
    """One TabuCol run; returns best colouring, f_best, iterations, stats, hash."""
    rp, ci = _csr(g)
    col = np.ascontiguousarray(colors, dtype=np.int16).copy()
    prm = _TabuParams(k, iters, ten_num, ten_den, ten_rand, int(check), seed)
    fb = C.c_int32()
    it = C.c_int32()
    st = np.zeros(NSTATS, dtype=np.int64)
    h = C.c_uint64()
    trace = np.zeros((max(trace_cap, 1), 2), dtype=np.int32)
    rc = lib().orc_tabucol(g.n, _p(rp), _p(ci), C.byref(prm), ind, _p(col), C.byref(fb),
                           C.byref(it), _p(st), C.byref(h), _p(trace) if trace_cap else None,
                           trace_cap)
    if rc != 0:
        raise AssertionError(lib().orc_last_error().decode())
    return {"colors": col, "f_best": fb.value, "iters": it.value, "stats": st,
            "hash": h.value, "trace": trace[:min(trace_cap, it.value)] if trace_cap else None}


def tabucol_batch(g, colors: np.ndarray, ind_ids, k: int, iters: int, seed: int,
                  ten_num: int = 6, ten_den: int = 10, ten_rand: int = 10,
                  nthreads: int | None = None) -> dict:
    rp, ci = _csr(g)
    col = np.ascontiguousarray(colors, dtype=np.int16).copy()
    ids = np.ascontiguousarray(ind_ids, dtype=np.int32)
    cnt = ids.shape[0]
    assert col.shape == (cnt, g.n)
    prm = _TabuParams(k, iters, ten_num, ten_den, ten_rand, 0, seed)
    fb = np.zeros(cnt, dtype=np.int32)
    it = np.zeros(cnt, dtype=np.int32)
    st = np.zeros((cnt, NSTATS), dtype=np.int64)
    hs = np.zeros(cnt, dtype=np.uint64)
    nt = nthreads or os.cpu_count() or 1
    rc = lib().orc_tabucol_batch(g.n, _p(rp), _p(ci), C.byref(prm), cnt, _p(ids), _p(col),
                                 _p(fb), _p(it), _p(st), _p(hs), nt)
    if rc != 0:
        raise AssertionError(lib().orc_last_error().decode())
    return {"colors": col, "f_best": fb, "iters": it, "stats": st, "hash": hs}


def wvcp_tabu(g, colors: np.ndarray, k: int, iters_per_round: int, rounds: int, seed: int,
              ind: int, ten_rand: int = 10, frz_num: int = 2, frz_den: int = 10,
              shift: int = 10, check: bool = False, trace_cap: int = 0) -> dict:
    rp, ci = _csr(g)
    w = np.ascontiguousarray(g.weights, dtype=np.int32)
    col = np.ascontiguousarray(colors, dtype=np.int16).copy()
    prm = _WvcpParams(k, iters_per_round, rounds, ten_rand, frz_num, frz_den, shift,
                      int(check), seed)
    bl = C.c_int32()
    st = np.zeros(NSTATS, dtype=np.int64)
    h = C.c_uint64()
    trace = np.zeros((max(trace_cap, 1), 2), dtype=np.int64)
    rlog = np.zeros((max(rounds, 1), 3), dtype=np.int64)
    rc = lib().orc_wvcp_tabu(g.n, _p(rp), _p(ci), _p(w), C.byref(prm), ind, _p(col),
                             C.byref(bl), _p(st), C.byref(h),
                             _p(trace) if trace_cap else None, trace_cap, _p(rlog))
    if rc != 0:
        raise AssertionError(lib().orc_last_error().decode())
    return {"colors": col, "best_legal": bl.value, "stats": st, "hash": h.value,
            "trace": trace[:trace_cap] if trace_cap else None, "rounds": rlog[:rounds]}


def wvcp_batch(g, colors: np.ndarray, ind_ids, k: int, iters_per_round: int, rounds: int,
               seed: int, ten_rand: int = 10, frz_num: int = 2, frz_den: int = 10,
               shift: int = 10, nthreads: int | None = None) -> dict:
    rp, ci = _csr(g)
    w = np.ascontiguousarray(g.weights, dtype=np.int32)
    col = np.ascontiguousarray(colors, dtype=np.int16).copy()
    ids = np.ascontiguousarray(ind_ids, dtype=np.int32)
    cnt = ids.shape[0]
    prm = _WvcpParams(k, iters_per_round, rounds, ten_rand, frz_num, frz_den, shift, 0, seed)
    bl = np.zeros(cnt, dtype=np.int32)
    st = np.zeros((cnt, NSTATS), dtype=np.int64)
    hs = np.zeros(cnt, dtype=np.uint64)
    nt = nthreads or os.cpu_count() or 1
    rc = lib().orc_wvcp_batch(g.n, _p(rp), _p(ci), _p(w), C.byref(prm), cnt, _p(ids),
                              _p(col), _p(bl), _p(st), _p(hs), nt)
    if rc != 0:
        raise AssertionError(lib().orc_last_error().decode())
    return {"colors": col, "best_legal": bl, "stats": st, "hash": hs}


def gpx(k: int, A: np.ndarray, B: np.ndarray, child: int, seed: int) -> np.ndarray:
    a = np.ascontiguousarray(A, dtype=np.int16)
    b = np.ascontiguousarray(B, dtype=np.int16)
    out = np.zeros_like(a)
    lib().orc_gpx(a.shape[0], k, _p(a), _p(b), child, seed, _p(out))
    return out


def gpx_batch(k: int, parents: np.ndarray, pairs: np.ndarray, per_pair: int,
              child_base: int, seed: int) -> np.ndarray:
    par = np.ascontiguousarray(parents, dtype=np.int16)
    pr = np.ascontiguousarray(pairs, dtype=np.int32)
    npairs = pr.shape[0]
    out = np.zeros((npairs * per_pair, par.shape[1]), dtype=np.int16)
    lib().orc_gpx_batch(par.shape[1], k, _p(par), _p(pr), npairs, per_pair, child_base, seed,
                        _p(out))
    return out


def select(scores: np.ndarray, keep: int, mode: int, seed: int = 0, gen: int = 0) -> np.ndarray:
    s = np.ascontiguousarray(scores, dtype=np.float32)
    out = np.zeros(max(keep, 1), dtype=np.int32)
    lib().orc_select(_p(s), s.shape[0], keep, mode, seed, gen, _p(out))
    return out[:keep]


def random_pairs(pop: int, seed: int, gen: int) -> np.ndarray:
    out = np.zeros((max(pop, 1), 2), dtype=np.int32)
    lib().orc_random_pairs(pop, seed, gen, _p(out))
    return out[:pop]
