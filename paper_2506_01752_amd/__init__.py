"""MI355X (gfx950) implementation of the HP-MOCD community search (arXiv 2506.01752).

A thin ctypes binding of ``libhpmocd.so`` (C ABI declared in ``include/hpmocd.h``). Every
step of the method runs in the library's HIP kernels; this module only marshals arguments.
PyTorch supplies the device workspace and the stream. There is no CPU fallback: when the
library is missing, importing ``lib()`` raises.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhpmocd.so")

OK = 0
ERR = {
    -1: "ERR_ARG", -2: "ERR_CSR_ASYM", -3: "ERR_SELF_LOOP", -4: "ERR_DUP_EDGE",
    -5: "ERR_RANGE", -6: "ERR_EMPTY", -7: "ERR_TOO_LARGE", -8: "ERR_WORKSPACE",
    -9: "ERR_HIP", -10: "ERR_BUDGET", -11: "ERR_NOMEM", -12: "ERR_CANCELLED",
    -13: "ERR_TIMEOUT", -14: "ERR_SCRATCH",
}
ERR_ARG = -1
ERR_RANGE = -5
ERR_BUDGET = -10
ERR_CANCELLED = -12
ERR_TIMEOUT = -13
ERR_SCRATCH = -14
NOALLOC_SCRATCH_BYTES = 64 << 20
MAX_POP = 512
MAX_PARENTS = 8
NO_GRAPH = 1
TIME_KERNELS = 2
TRACE_NO_LABELS = 4
AUTOTUNE = 8
SERVER_FIFO = 1
REQ_QUEUED, REQ_RUNNING, REQ_DONE = 0, 1, 2

# every entry point that include/hpmocd.h declares
EXPORTS = [
    "hpmocd_graph_create", "hpmocd_graph_destroy", "hpmocd_graph_info",
    "hpmocd_workspace_size", "hpmocd_run", "hpmocd_run_ex", "hpmocd_run_traced",
    "hpmocd_front_free",
    "hpmocd_eval_workspace_size", "hpmocd_eval", "hpmocd_strerror",
    "hpmocd_batch_workspace_size", "hpmocd_run_batch",
    "hpmocd_server_arena_overhead", "hpmocd_server_create", "hpmocd_server_submit",
    "hpmocd_server_poll", "hpmocd_server_wait", "hpmocd_server_cancel",
    "hpmocd_server_stats_get", "hpmocd_server_destroy",
    "hpmocd_run_to", "hpmocd_resume", "hpmocd_snapshot_free",
    "hpmocd_eval_noalloc", "hpmocd_graph_hash",
]


class HpmocdError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {ERR.get(status, status)} ({_strerror(status)})")


class Params(C.Structure):
    _fields_ = [("pop_size", C.c_int32), ("generations", C.c_int32),
                ("crossover_p", C.c_double), ("mutation_p", C.c_double),
                ("parents_per_child", C.c_int32), ("seed", C.c_uint64)]


class _Front(C.Structure):
    _fields_ = [("n_solutions", C.c_int32), ("n_nodes", C.c_int32),
                ("labels", C.POINTER(C.c_int32)), ("intra_arcs", C.POINTER(C.c_int64)),
                ("sum_deg_sq", C.POINTER(C.c_int64)), ("f1", C.POINTER(C.c_double)),
                ("f2", C.POINTER(C.c_double)), ("selected", C.c_int32)]


class _View(C.Structure):
    _fields_ = [("g", C.c_int32), ("pop_size", C.c_int32), ("n_nodes", C.c_int32),
                ("labels", C.POINTER(C.c_int32)),
                ("A", C.POINTER(C.c_int64)), ("S", C.POINTER(C.c_int64)),
                ("f1", C.POINTER(C.c_double)), ("f2", C.POINTER(C.c_double)),
                ("rank", C.POINTER(C.c_int32)), ("crowd", C.POINTER(C.c_double))]


class Profile(C.Structure):
    _fields_ = [("total_ms", C.c_double), ("loop_ms", C.c_double),
                ("fitness_ms", C.c_double), ("sweep_ms", C.c_double),
                ("variation_ms", C.c_double), ("select_ms", C.c_double),
                ("fitness_launches", C.c_int64), ("individual_evals", C.c_int64),
                ("tune_fit_target_waves", C.c_int32), ("tune_xo_target_blocks", C.c_int32),
                ("tune_mut_target_items", C.c_int32), ("tune_hist_min_log2", C.c_int32),
                ("tune_hist_rbits", C.c_int32), ("tune_hist_narrow", C.c_int32),
                ("tune_probe_ms", C.c_double), ("crossover_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}




class _Snapshot(C.Structure):
    _fields_ = [("g", C.c_int32), ("pop_size", C.c_int32), ("n_nodes", C.c_int32),
                ("labels", C.POINTER(C.c_int32)), ("A", C.POINTER(C.c_int64)),
                ("S", C.POINTER(C.c_int64)), ("params", Params), ("graph_hash", C.c_uint64)]


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_active", C.c_int32),
                ("parents_per_child", C.c_int32), ("flags", C.c_int32),
                ("host_stage_bytes", C.c_size_t)]


class RequestInfo(C.Structure):
    _fields_ = [("submit_s", C.c_double), ("admit_s", C.c_double), ("done_s", C.c_double),
                ("device_bytes", C.c_int64), ("steps", C.c_int32), ("max_mix", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("cancelled", C.c_int64), ("peak_active", C.c_int32),
                ("peak_bytes", C.c_int64), ("busy_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_TRACE = C.CFUNCTYPE(None, C.POINTER(_View), C.c_void_p)
_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        i32p, i64p, f64p, vp = (C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                C.POINTER(C.c_double), C.c_void_p)
        L.hpmocd_graph_create.argtypes = [C.c_int32, i32p, i32p, C.POINTER(vp)]
        L.hpmocd_graph_destroy.argtypes = [vp]
        L.hpmocd_graph_destroy.restype = None
        L.hpmocd_graph_info.argtypes = [vp, i32p, i64p, i32p]
        L.hpmocd_graph_hash.argtypes = [vp, C.POINTER(C.c_uint64)]
        L.hpmocd_workspace_size.argtypes = [vp, C.POINTER(Params), C.POINTER(C.c_size_t)]
        L.hpmocd_run.argtypes = [vp, C.POINTER(Params), vp, C.c_size_t, vp,
                                 C.POINTER(C.POINTER(_Front))]
        L.hpmocd_run_ex.argtypes = [vp, C.POINTER(Params), vp, C.c_size_t, vp, C.c_int,
                                    C.POINTER(Profile), _TRACE, vp,
                                    C.POINTER(C.POINTER(_Front))]
        L.hpmocd_run_traced.argtypes = [vp, C.POINTER(Params), vp, C.c_size_t, vp, _TRACE, vp,
                                        C.POINTER(C.POINTER(_Front))]
        L.hpmocd_front_free.argtypes = [C.POINTER(_Front)]
        L.hpmocd_front_free.restype = None
        L.hpmocd_eval_workspace_size.argtypes = [vp, C.c_int32, C.POINTER(C.c_size_t)]
        L.hpmocd_eval.argtypes = [vp, vp, C.c_int32, vp, C.c_size_t, vp, i64p, i64p, f64p, f64p,
                                  f64p]
        L.hpmocd_eval_noalloc.argtypes = [vp, vp, C.c_int32, vp, i64p, i64p, f64p, f64p]
        L.hpmocd_batch_workspace_size.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(Params),
                                                  C.c_int, C.POINTER(C.c_size_t)]
        L.hpmocd_run_batch.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(Params), vp,
                                       C.c_size_t, vp, C.c_int, C.POINTER(Profile),
                                       C.POINTER(C.POINTER(_Front))]
        L.hpmocd_server_arena_overhead.argtypes = [C.c_int32]
        L.hpmocd_server_create.argtypes = [C.POINTER(ServerConfig), vp, C.c_size_t, vp,
                                           C.POINTER(vp)]
        L.hpmocd_server_submit.argtypes = [vp, C.c_int32, i32p, i32p, C.POINTER(Params), i64p,
                                           C.POINTER(C.c_size_t)]
        L.hpmocd_server_poll.argtypes = [vp, C.c_int64, i32p]
        L.hpmocd_server_wait.argtypes = [vp, C.c_int64, C.c_double,
                                         C.POINTER(C.POINTER(_Front)), C.POINTER(RequestInfo)]
        L.hpmocd_server_cancel.argtypes = [vp, C.c_int64]
        L.hpmocd_server_stats_get.argtypes = [vp, C.POINTER(ServerStats)]
        L.hpmocd_server_destroy.argtypes = [vp]
        L.hpmocd_server_destroy.restype = None
        L.hpmocd_run_to.argtypes = [vp, C.POINTER(Params), C.c_int32, vp, C.c_size_t, vp,
                                    C.POINTER(C.POINTER(_Snapshot))]
        L.hpmocd_resume.argtypes = [vp, C.POINTER(Params), C.POINTER(_Snapshot), vp, C.c_size_t,
                                    vp, C.POINTER(C.POINTER(_Front))]
        L.hpmocd_snapshot_free.argtypes = [C.POINTER(_Snapshot)]
        L.hpmocd_snapshot_free.restype = None
        L.hpmocd_strerror.argtypes = [C.c_int]
        L.hpmocd_strerror.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("hpmocd_graph_destroy", "hpmocd_front_free", "hpmocd_strerror",
                            "hpmocd_server_destroy", "hpmocd_server_arena_overhead",
                            "hpmocd_snapshot_free"):
                getattr(L, name).restype = C.c_int
        L.hpmocd_server_arena_overhead.restype = C.c_size_t
        _lib = L
    return _lib


def _strerror(status: int) -> str:
    try:
        return lib().hpmocd_strerror(status).decode()
    except Exception:  # pragma: no cover - only used for messages
        return "?"


def _check(status: int, what: str):
    if status != OK:
        raise HpmocdError(status, what)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def graph_create_status(n: int, row_ptr, col) -> int:
    """Runs hpmocd_graph_create and returns its status (destroying the graph on success).
    Validation happens before any device call, so this also works without a GPU."""
    rp, cl = _i32(row_ptr), _i32(col)
    h = C.c_void_p()
    st = lib().hpmocd_graph_create(n, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                                   cl.ctypes.data_as(C.POINTER(C.c_int32)) if cl.size else None,
                                   C.byref(h))
    if st == OK:
        lib().hpmocd_graph_destroy(h)
    return st


class Graph:
    """Device-resident simple undirected graph (hpmocd_graph)."""

    def __init__(self, row_ptr, col):
        rp, cl = _i32(row_ptr), _i32(col)
        self._h = C.c_void_p()
        _check(lib().hpmocd_graph_create(len(rp) - 1, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                                         cl.ctypes.data_as(C.POINTER(C.c_int32)),
                                         C.byref(self._h)), "hpmocd_graph_create")
        n, arcs, md = C.c_int32(), C.c_int64(), C.c_int32()
        _check(lib().hpmocd_graph_info(self._h, C.byref(n), C.byref(arcs), C.byref(md)),
               "hpmocd_graph_info")
        self.n, self.arcs, self.max_deg = n.value, arcs.value, md.value
        h = C.c_uint64()
        _check(lib().hpmocd_graph_hash(self._h, C.byref(h)), "hpmocd_graph_hash")
        self.hash = h.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().hpmocd_graph_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Front:
    labels: np.ndarray   # (k, n) int32
    A: np.ndarray        # intra arcs, int64
    S: np.ndarray        # sum of squared community degrees, int64
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


def make_params(pop_size=100, generations=100, crossover_p=0.9, mutation_p=0.1,
                parents_per_child=4, seed=0) -> Params:
    return Params(pop_size, generations, crossover_p, mutation_p, parents_per_child, seed)


def workspace_size(graph: Graph, params: Params) -> int:
    b = C.c_size_t()
    _check(lib().hpmocd_workspace_size(graph.handle, C.byref(params), C.byref(b)),
           "hpmocd_workspace_size")
    return b.value


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _free_front(ptr):
    try:
        lib().hpmocd_front_free(ptr)
    except Exception:  # pragma: no cover - interpreter shutdown
        pass


def _front_from(ptr) -> Front:
    """The library's front as numpy arrays. The label matrix (k x n int32, hundreds of MB on
    large graphs) is not copied: the array views the library's memory, which is released
    when the array (and every view of it) is gone."""
    f = ptr.contents
    k, n = f.n_solutions, f.n_nodes
    buf = (C.c_int32 * (k * n)).from_address(C.addressof(f.labels.contents))
    labels = np.frombuffer(buf, dtype=np.int32).reshape(k, n)
    weakref.finalize(buf, _free_front, ptr)
    return Front(labels,
                 np.ctypeslib.as_array(f.intra_arcs, shape=(k,)).copy(),
                 np.ctypeslib.as_array(f.sum_deg_sq, shape=(k,)).copy(),
                 np.ctypeslib.as_array(f.f1, shape=(k,)).copy(),
                 np.ctypeslib.as_array(f.f2, shape=(k,)).copy(), f.selected)


def run(graph: Graph, params: Params | None = None, *, stream=None, workspace=None, flags=0,
        profile: bool = False, on_generation=None, **kw):
    """hpmocd_run / hpmocd_run_ex. Returns the Front, or (Front, profile dict) when
    profile=True. ``on_generation(State)`` traces every generation (tests only)."""
    import torch
    if params is None:
        params = make_params(**kw)
    nbytes = workspace_size(graph, params)
    ws = workspace if workspace is not None else torch.empty(nbytes, dtype=torch.uint8,
                                                             device="cuda")
    assert ws.numel() >= nbytes and ws.is_cuda
    prof = Profile()
    out = C.POINTER(_Front)()
    cb = _TRACE()
    if on_generation is not None:
        def _cb(vp, _u):
            v = vp.contents
            np_, nn = v.pop_size, v.n_nodes
            on_generation(State(
                v.g,
                np.ctypeslib.as_array(v.labels, shape=(np_, nn)).copy() if v.labels else None,
                np.ctypeslib.as_array(v.A, shape=(np_,)).copy(),
                np.ctypeslib.as_array(v.S, shape=(np_,)).copy(),
                np.ctypeslib.as_array(v.f1, shape=(np_,)).copy(),
                np.ctypeslib.as_array(v.f2, shape=(np_,)).copy(),
                np.ctypeslib.as_array(v.rank, shape=(np_,)).copy() if v.rank else None,
                np.ctypeslib.as_array(v.crowd, shape=(np_,)).copy() if v.crowd else None))
        cb = _TRACE(_cb)
    if on_generation is not None and not flags and not profile:
        st = lib().hpmocd_run_traced(graph.handle, C.byref(params), C.c_void_p(ws.data_ptr()),
                                     nbytes, _stream_handle(stream), cb, None, C.byref(out))
        _check(st, "hpmocd_run_traced")
    else:
        st = lib().hpmocd_run_ex(graph.handle, C.byref(params), C.c_void_p(ws.data_ptr()),
                                 nbytes, _stream_handle(stream), flags,
                                 C.byref(prof) if profile else None, cb, None, C.byref(out))
        _check(st, "hpmocd_run_ex")
    front = _front_from(out)
    return (front, prof.as_dict()) if profile else front


@dataclass
class Snapshot:
    g: int               # generations completed
    labels: np.ndarray   # (pop, n) int32, selection order
    A: np.ndarray
    S: np.ndarray
    params: Params | None = None   # the run's parameters (checked on resume)
    graph_hash: int = 0            # fingerprint of the run's graph (checked on resume)


def run_to(graph: Graph, params: Params | None = None, *, stop_gen: int, stream=None,
           workspace=None, **kw) -> Snapshot:
    """hpmocd_run_to: the population after generation stop_gen (checkpoint)."""
    import torch
    if params is None:
        params = make_params(**kw)
    nbytes = workspace_size(graph, params)
    ws = workspace if workspace is not None else torch.empty(nbytes, dtype=torch.uint8,
                                                             device="cuda")
    out = C.POINTER(_Snapshot)()
    _check(lib().hpmocd_run_to(graph.handle, C.byref(params), stop_gen,
                               C.c_void_p(ws.data_ptr()), nbytes, _stream_handle(stream),
                               C.byref(out)), "hpmocd_run_to")
    sn = out.contents
    res = Snapshot(sn.g, np.ctypeslib.as_array(sn.labels, shape=(sn.pop_size, sn.n_nodes)).copy(),
                   np.ctypeslib.as_array(sn.A, shape=(sn.pop_size,)).copy(),
                   np.ctypeslib.as_array(sn.S, shape=(sn.pop_size,)).copy(),
                   Params(*[getattr(sn.params, f) for f, _ in Params._fields_]),
                   int(sn.graph_hash))
    lib().hpmocd_snapshot_free(out)
    return res


def resume(graph: Graph, snapshot: Snapshot, params: Params | None = None, *, stream=None,
           workspace=None, **kw) -> Front:
    """hpmocd_resume: continue a run from a snapshot to params.generations."""
    import torch
    if params is None:
        params = make_params(**kw)
    labels = np.ascontiguousarray(snapshot.labels, dtype=np.int32)
    A = np.ascontiguousarray(snapshot.A, dtype=np.int64)
    S = np.ascontiguousarray(snapshot.S, dtype=np.int64)
    sn = _Snapshot(snapshot.g, labels.shape[0], labels.shape[1],
                   labels.ctypes.data_as(C.POINTER(C.c_int32)),
                   A.ctypes.data_as(C.POINTER(C.c_int64)), S.ctypes.data_as(C.POINTER(C.c_int64)),
                   snapshot.params if snapshot.params is not None else Params(),
                   snapshot.graph_hash)
    nbytes = workspace_size(graph, params)
    ws = workspace if workspace is not None else torch.empty(nbytes, dtype=torch.uint8,
                                                             device="cuda")
    out = C.POINTER(_Front)()
    _check(lib().hpmocd_resume(graph.handle, C.byref(params), C.byref(sn),
                               C.c_void_p(ws.data_ptr()), nbytes, _stream_handle(stream),
                               C.byref(out)), "hpmocd_resume")
    return _front_from(out)


def run_batch(graphs, params, *, stream=None, workspace=None, flags=0, profile=False):
    """hpmocd_run_batch: one run per graph (params: one Params, or one per graph), all
    advanced together. Returns the list of fronts, or (fronts, profile dict)."""
    import torch
    count = len(graphs)
    if isinstance(params, Params):
        params = [params] * count
    assert len(params) == count
    handles = (C.c_void_p * count)(*[g.handle.value for g in graphs])
    parr = (Params * count)(*params)
    b = C.c_size_t()
    _check(lib().hpmocd_batch_workspace_size(handles, count, parr, flags, C.byref(b)),
           "hpmocd_batch_workspace_size")
    ws = workspace if workspace is not None else torch.empty(b.value, dtype=torch.uint8,
                                                             device="cuda")
    assert ws.numel() >= b.value and ws.is_cuda
    prof = Profile()
    outs = (C.POINTER(_Front) * count)()
    _check(lib().hpmocd_run_batch(handles, count, parr, C.c_void_p(ws.data_ptr()), b.value,
                                  _stream_handle(stream), flags,
                                  C.byref(prof) if profile else None, outs),
           "hpmocd_run_batch")
    fronts = [_front_from(outs[i]) for i in range(count)]
    return (fronts, prof.as_dict()) if profile else fronts


def batch_workspace_size(graphs, params, flags=0) -> int:
    count = len(graphs)
    if isinstance(params, Params):
        params = [params] * count
    handles = (C.c_void_p * count)(*[g.handle.value for g in graphs])
    parr = (Params * count)(*params)
    b = C.c_size_t()
    _check(lib().hpmocd_batch_workspace_size(handles, count, parr, flags, C.byref(b)),
           "hpmocd_batch_workspace_size")
    return b.value


def evaluate(graph: Graph, labels, *, stream=None, timing=False):
    """hpmocd_eval: objectives of n_ind partitions given as a CUDA int32 tensor (n_ind, n)."""
    import torch
    assert labels.is_cuda and labels.dtype == torch.int32 and labels.is_contiguous()
    n_ind = labels.shape[0]
    assert labels.shape[1] == graph.n
    b = C.c_size_t()
    _check(lib().hpmocd_eval_workspace_size(graph.handle, n_ind, C.byref(b)),
           "hpmocd_eval_workspace_size")
    ws = torch.empty(b.value, dtype=torch.uint8, device="cuda")
    A = np.empty(n_ind, dtype=np.int64)
    S = np.empty(n_ind, dtype=np.int64)
    f1 = np.empty(n_ind, dtype=np.float64)
    f2 = np.empty(n_ind, dtype=np.float64)
    ms = C.c_double()
    _check(lib().hpmocd_eval(graph.handle, C.c_void_p(labels.data_ptr()), n_ind,
                             C.c_void_p(ws.data_ptr()), b.value, _stream_handle(stream),
                             A.ctypes.data_as(C.POINTER(C.c_int64)),
                             S.ctypes.data_as(C.POINTER(C.c_int64)),
                             f1.ctypes.data_as(C.POINTER(C.c_double)),
                             f2.ctypes.data_as(C.POINTER(C.c_double)), C.byref(ms)),
           "hpmocd_eval")
    return (A, S, f1, f2, ms.value) if timing else (A, S, f1, f2)


def evaluate_noalloc(graph: Graph, labels, *, stream=None):
    """hpmocd_eval_noalloc: hpmocd_eval with the library's fixed device scratch (no
    workspace, no device allocation); labels as for evaluate()."""
    import torch
    assert labels.is_cuda and labels.dtype == torch.int32 and labels.is_contiguous()
    n_ind = labels.shape[0]
    assert labels.shape[1] == graph.n
    A = np.empty(n_ind, dtype=np.int64)
    S = np.empty(n_ind, dtype=np.int64)
    f1 = np.empty(n_ind, dtype=np.float64)
    f2 = np.empty(n_ind, dtype=np.float64)
    _check(lib().hpmocd_eval_noalloc(graph.handle, C.c_void_p(labels.data_ptr()), n_ind,
                                     _stream_handle(stream),
                                     A.ctypes.data_as(C.POINTER(C.c_int64)),
                                     S.ctypes.data_as(C.POINTER(C.c_int64)),
                                     f1.ctypes.data_as(C.POINTER(C.c_double)),
                                     f2.ctypes.data_as(C.POINTER(C.c_double))),
           "hpmocd_eval_noalloc")
    return A, S, f1, f2


class Server:
    """hpmocd_server_*: continuous-batching service on the current device. The arena (device
    memory: table overhead + hbm_budget bytes) and the stream come from torch and are kept
    alive by this object. submit() returns a ticket at once; wait() blocks until the front
    is on the host (the GIL is released meanwhile)."""

    def __init__(self, hbm_budget: int, max_active: int = 256, parents_per_child: int = 4,
                 fifo: bool = False, stream=None, host_stage_bytes: int = 0):
        import torch
        self._h = C.c_void_p()
        over = lib().hpmocd_server_arena_overhead(max_active)
        self.arena = torch.empty(over + hbm_budget, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        cfg = ServerConfig(hbm_budget, max_active, parents_per_child, SERVER_FIFO if fifo else 0,
                           host_stage_bytes)
        _check(lib().hpmocd_server_create(C.byref(cfg), C.c_void_p(self.arena.data_ptr()),
                                          self.arena.numel(), C.c_void_p(self.stream.cuda_stream),
                                          C.byref(self._h)), "hpmocd_server_create")

    def submit(self, row_ptr, col, params: Params | None = None, **kw):
        """Queues one run; returns (ticket, device bytes it will hold)."""
        if params is None:
            params = make_params(**kw)
        rp, cl = _i32(row_ptr), _i32(col)
        t, b = C.c_int64(), C.c_size_t()
        _check(lib().hpmocd_server_submit(self._h, len(rp) - 1,
                                          rp.ctypes.data_as(C.POINTER(C.c_int32)),
                                          cl.ctypes.data_as(C.POINTER(C.c_int32)),
                                          C.byref(params), C.byref(t), C.byref(b)),
               "hpmocd_server_submit")
        return t.value, b.value

    def poll(self, ticket: int) -> int:
        st = C.c_int32()
        _check(lib().hpmocd_server_poll(self._h, ticket, C.byref(st)), "hpmocd_server_poll")
        return st.value

    def wait(self, ticket: int, timeout: float = -1.0):
        """(Front, info dict); raises HpmocdError (ERR_TIMEOUT, ERR_CANCELLED, ...)."""
        out = C.POINTER(_Front)()
        info = RequestInfo()
        _check(lib().hpmocd_server_wait(self._h, ticket, float(timeout), C.byref(out),
                                        C.byref(info)), "hpmocd_server_wait")
        return _front_from(out), info.as_dict()

    def cancel(self, ticket: int):
        _check(lib().hpmocd_server_cancel(self._h, ticket), "hpmocd_server_cancel")

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().hpmocd_server_stats_get(self._h, C.byref(st)), "hpmocd_server_stats_get")
        return st.as_dict()

    def close(self):
        if self._h:
            lib().hpmocd_server_destroy(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
