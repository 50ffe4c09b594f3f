"""Reference oracle for HP-MOCD (arXiv 2506.01752): ctypes binding of ``oracle.c``.

Test infrastructure only: the tests, the smoke check and the benchmark's CPU-baseline leg
load it; the product path never does. It shares no code with the HIP library.

Every function mirrors one step of the paper's method (section 4, Alg. 1-3); the C source
states the reading taken wherever the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TAG_INIT, TAG_SEL, TAG_XOV, TAG_MUT = 0, 1, 2, 3
GATE_X = 0xFFFFFFFF


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (-O2 -ffp-contract=off, OpenMP over individuals)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("pop_size", C.c_int32), ("generations", C.c_int32),
                ("crossover_p", C.c_double), ("mutation_p", C.c_double),
                ("parents_per_child", C.c_int32), ("seed", C.c_uint64)]


class _View(C.Structure):
    _fields_ = [("g", C.c_int32), ("pop_size", C.c_int32), ("n_nodes", C.c_int32),
                ("labels", C.POINTER(C.c_int32)),
                ("A", C.POINTER(C.c_int64)), ("S", C.POINTER(C.c_int64)),
                ("f1", C.POINTER(C.c_double)), ("f2", C.POINTER(C.c_double)),
                ("rank", C.POINTER(C.c_int32)), ("crowd", C.POINTER(C.c_double))]


_CB = C.CFUNCTYPE(None, C.POINTER(_View), C.c_void_p)
_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB)
        i32p, i64p, f64p = C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_double)
        lib.or_philox.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                  C.POINTER(C.c_uint32)]
        lib.or_pick.argtypes = [C.c_uint32, C.c_uint32]
        lib.or_pick.restype = C.c_uint32
        lib.or_thr.argtypes = [C.c_double]
        lib.or_thr.restype = C.c_uint64
        lib.or_eval.argtypes = [C.c_int32, i32p, i32p, i32p, i64p, i64p, f64p, f64p]
        lib.or_eval_batch.argtypes = [C.c_int32, i32p, i32p, i32p, C.c_int32, i64p, i64p, f64p,
                                      f64p]
        lib.or_init_individual.argtypes = [C.c_int32, i32p, i32p, C.c_uint64, C.c_int32, i32p]
        lib.or_crossover.argtypes = [C.c_int32, C.c_int32, i32p, C.c_int32, C.c_uint64,
                                     C.c_uint32, C.c_uint32, i32p]
        lib.or_neighbour_plurality.argtypes = [C.c_int32, i32p, i32p, i32p, C.c_int32,
                                               C.c_uint64, C.c_uint32, C.c_uint32]
        lib.or_neighbour_plurality.restype = C.c_int32
        lib.or_mutate.argtypes = [C.c_int32, i32p, i32p, i32p, C.c_double, C.c_uint64,
                                  C.c_uint32, C.c_uint32, i32p]
        lib.or_tournament.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                      C.c_int32]
        lib.or_tournament.restype = C.c_int32
        lib.or_gate.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_double, C.c_int32]
        lib.or_gate.restype = C.c_int32
        lib.or_offspring.argtypes = [C.c_int32, i32p, i32p, i32p, C.c_int32, C.c_int32,
                                     C.c_double, C.c_double, C.c_uint64, C.c_uint32,
                                     C.c_uint32, i32p, i32p, i32p]
        lib.or_rank.argtypes = [C.c_int32, i64p, i64p, i32p]
        lib.or_crowding.argtypes = [C.c_int32, i32p, i64p, i64p, f64p, f64p, f64p]
        lib.or_order.argtypes = [C.c_int32, i32p, f64p, i32p]
        lib.or_run.argtypes = [C.c_int32, i32p, i32p, C.POINTER(_Params), C.c_int32, _CB,
                               C.c_void_p, i32p, i32p, i64p, i64p, f64p, f64p, i32p]
        lib.or_run.restype = C.c_int
        _lib = lib
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def philox(seed: int, x: int, ind: int, gen: int, tag: int) -> np.ndarray:
    """Philox4x32-10 block for counter (x, ind, gen, tag) under key = seed (64-bit)."""
    out = (C.c_uint32 * 4)()
    _L().or_philox(seed, x & 0xFFFFFFFF, ind, gen, tag, out)
    return np.array(list(out), dtype=np.uint32)


def pick(r: int, k: int) -> int:
    return int(_L().or_pick(r, k))


def thr(p: float) -> int:
    return int(_L().or_thr(p))


def evaluate(row_ptr, col, labels):
    """(A, S, f1, f2) of one partition (section 4.1, eq. "objectives")."""
    rp, cl, lb = _i32(row_ptr), _i32(col), _i32(labels)
    A, S = C.c_int64(), C.c_int64()
    f1, f2 = C.c_double(), C.c_double()
    _L().or_eval(len(rp) - 1, _p(rp, C.c_int32), _p(cl, C.c_int32), _p(lb, C.c_int32),
                 C.byref(A), C.byref(S), C.byref(f1), C.byref(f2))
    return A.value, S.value, f1.value, f2.value


def evaluate_batch(row_ptr, col, labels):
    """evaluate() of every row of labels (k x n) against one copy of the graph."""
    rp, cl, lb = _i32(row_ptr), _i32(col), _i32(labels)
    k = lb.shape[0]
    A = np.empty(k, dtype=np.int64)
    S = np.empty(k, dtype=np.int64)
    f1 = np.empty(k, dtype=np.float64)
    f2 = np.empty(k, dtype=np.float64)
    _L().or_eval_batch(len(rp) - 1, _p(rp, C.c_int32), _p(cl, C.c_int32), _p(lb, C.c_int32), k,
                       _p(A, C.c_int64), _p(S, C.c_int64), _p(f1, C.c_double), _p(f2, C.c_double))
    return A, S, f1, f2


def init_individual(row_ptr, col, seed: int, i: int) -> np.ndarray:
    rp, cl = _i32(row_ptr), _i32(col)
    out = np.empty(len(rp) - 1, dtype=np.int32)
    _L().or_init_individual(len(rp) - 1, _p(rp, C.c_int32), _p(cl, C.c_int32), seed, i,
                            _p(out, C.c_int32))
    return out


def crossover(parents, gate_copy: int, seed: int, gen: int, j: int) -> np.ndarray:
    """Alg. 2 for offspring j of generation gen; gate_copy < 0 means the majority vote."""
    par = _i32(parents)
    es, n = par.shape
    out = np.empty(n, dtype=np.int32)
    _L().or_crossover(n, es, _p(par, C.c_int32), gate_copy, seed, gen, j, _p(out, C.c_int32))
    return out


def neighbour_plurality(row_ptr, col, child, v: int, seed: int, gen: int, j: int) -> int:
    rp, cl, ch = _i32(row_ptr), _i32(col), _i32(child)
    return int(_L().or_neighbour_plurality(len(rp) - 1, _p(rp, C.c_int32), _p(cl, C.c_int32),
                                           _p(ch, C.c_int32), v, seed, gen, j))


def mutate(row_ptr, col, child, mutation_p: float, seed: int, gen: int, j: int) -> np.ndarray:
    rp, cl, ch = _i32(row_ptr), _i32(col), _i32(child)
    out = np.empty(len(rp) - 1, dtype=np.int32)
    _L().or_mutate(len(rp) - 1, _p(rp, C.c_int32), _p(cl, C.c_int32), _p(ch, C.c_int32),
                   mutation_p, seed, gen, j, _p(out, C.c_int32))
    return out


def tournament(seed: int, gen: int, j: int, k: int, pop_size: int) -> int:
    """Winner position of parent slot k of offspring j (Alg. 1 TournamentSelection, k = 2)
    in a population already in crowded-comparison order."""
    return int(_L().or_tournament(seed, gen, j, k, pop_size))


def gate(seed: int, gen: int, j: int, crossover_p: float, parents_per_child: int) -> int:
    """Crossover gate of offspring j (Alg. 2): -1 = ensemble crossover, else the copied
    parent slot."""
    return int(_L().or_gate(seed, gen, j, crossover_p, parents_per_child))


def offspring(row_ptr, col, pop, parents_per_child: int, crossover_p: float,
              mutation_p: float, seed: int, gen: int, j: int):
    """Offspring j of generation gen from the rows of ``pop`` (N_p x n, crowded order):
    tournaments, gate, crossover, mutation. Returns (child, parent positions, gate)."""
    rp, cl, P = _i32(row_ptr), _i32(col), _i32(pop)
    np_, n = P.shape
    child = np.empty(n, dtype=np.int32)
    pos = np.empty(parents_per_child, dtype=np.int32)
    g = C.c_int32()
    _L().or_offspring(n, _p(rp, C.c_int32), _p(cl, C.c_int32), _p(P, C.c_int32), np_,
                      parents_per_child, crossover_p, mutation_p, seed, gen, j,
                      _p(child, C.c_int32), _p(pos, C.c_int32), C.byref(g))
    return child, pos, g.value


def rank(k1, k2) -> np.ndarray:
    a = np.ascontiguousarray(k1, dtype=np.int64)
    b = np.ascontiguousarray(k2, dtype=np.int64)
    out = np.empty(len(a), dtype=np.int32)
    _L().or_rank(len(a), _p(a, C.c_int64), _p(b, C.c_int64), _p(out, C.c_int32))
    return out


def crowding(rank_, k1, k2, f1, f2) -> np.ndarray:
    r = _i32(rank_)
    a = np.ascontiguousarray(k1, dtype=np.int64)
    b = np.ascontiguousarray(k2, dtype=np.int64)
    x = np.ascontiguousarray(f1, dtype=np.float64)
    y = np.ascontiguousarray(f2, dtype=np.float64)
    out = np.empty(len(a), dtype=np.float64)
    _L().or_crowding(len(a), _p(r, C.c_int32), _p(a, C.c_int64), _p(b, C.c_int64),
                     _p(x, C.c_double), _p(y, C.c_double), _p(out, C.c_double))
    return out


def order(rank_, crowd) -> np.ndarray:
    r = _i32(rank_)
    c = np.ascontiguousarray(crowd, dtype=np.float64)
    out = np.empty(len(r), dtype=np.int32)
    _L().or_order(len(r), _p(r, C.c_int32), _p(c, C.c_double), _p(out, C.c_int32))
    return out


@dataclass
class Front:
    labels: np.ndarray      # (k, n) int32, rank-1 members of P^(T) in crowded order
    A: np.ndarray
    S: np.ndarray
    f1: np.ndarray
    f2: np.ndarray
    selected: int


@dataclass
class State:
    g: int
    labels: np.ndarray
    A: np.ndarray
    S: np.ndarray
    f1: np.ndarray
    f2: np.ndarray
    rank: np.ndarray | None
    crowd: np.ndarray | None


def run(row_ptr, col, pop_size=100, generations=100, crossover_p=0.9, mutation_p=0.1,
        parents_per_child=4, seed=0, threads=1, on_generation=None, copy_labels=True):
    """Alg. 1 end to end. ``on_generation(State)`` is called after generation 0 (init) and
    after the environmental selection of every generation."""
    rp, cl = _i32(row_ptr), _i32(col)
    n = len(rp) - 1
    prm = _Params(pop_size, generations, crossover_p, mutation_p, parents_per_child, seed)
    lab = np.empty((pop_size, n), dtype=np.int32)
    A = np.empty(pop_size, dtype=np.int64)
    S = np.empty(pop_size, dtype=np.int64)
    f1 = np.empty(pop_size, dtype=np.float64)
    f2 = np.empty(pop_size, dtype=np.float64)
    k = C.c_int32()
    sel = C.c_int32()

    def _cb(vp, _user):
        v = vp.contents
        np_, nn = v.pop_size, v.n_nodes
        labels = np.ctypeslib.as_array(v.labels, shape=(np_, nn))
        st = State(
            g=v.g,
            labels=labels.copy() if copy_labels else labels,
            A=np.ctypeslib.as_array(v.A, shape=(np_,)).copy(),
            S=np.ctypeslib.as_array(v.S, shape=(np_,)).copy(),
            f1=np.ctypeslib.as_array(v.f1, shape=(np_,)).copy(),
            f2=np.ctypeslib.as_array(v.f2, shape=(np_,)).copy(),
            rank=(np.ctypeslib.as_array(v.rank, shape=(np_,)).copy() if v.rank else None),
            crowd=(np.ctypeslib.as_array(v.crowd, shape=(np_,)).copy() if v.crowd else None),
        )
        on_generation(st)

    cb = _CB(_cb) if on_generation is not None else _CB()
    rc = _L().or_run(n, _p(rp, C.c_int32), _p(cl, C.c_int32), C.byref(prm), threads, cb, None,
                     C.byref(k), _p(lab, C.c_int32), _p(A, C.c_int64), _p(S, C.c_int64),
                     _p(f1, C.c_double), _p(f2, C.c_double), C.byref(sel))
    if rc != 0:
        raise ValueError("oracle run rejected its arguments")
    kk = k.value
    return Front(lab[:kk].copy(), A[:kk].copy(), S[:kk].copy(), f1[:kk].copy(), f2[:kk].copy(),
                 sel.value)
