"""The C-ABI library on the CPU: it loads, exports every entry point its header declares,
and its graph validation rejects what section 2.1 excludes before any device call."""
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2506_01752_amd as hp
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_entry_points():
    text = open(os.path.join(ROOT, "include", "hpmocd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hpmocd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    declared = header_entry_points()
    assert "hpmocd_run" in declared and "hpmocd_graph_create" in declared
    out = subprocess.run(["nm", "-D", "--defined-only", hp.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\b(hpmocd_[a-z_]+)\b", out))
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    assert sorted(hp.EXPORTS) == declared
    lib = hp.lib()
    for s in declared:
        assert hasattr(lib, s)


def test_strerror_names_every_status():
    for code, name in hp.ERR.items():
        msg = hp.lib().hpmocd_strerror(code).decode()
        assert msg and msg != "unknown status", (code, name)
    assert hp.lib().hpmocd_strerror(0).decode() == "ok"


def _csr(n, arcs):
    arcs = sorted(arcs)
    rp = np.zeros(n + 1, dtype=np.int32)
    for u, _ in arcs:
        rp[u + 1] += 1
    rp = np.cumsum(rp).astype(np.int32)
    col = np.array([v for _, v in arcs], dtype=np.int32)
    return rp, col


def test_validation_codes():
    # asymmetric: arc 0->1 without 1->0 (node 0's in-degree differs from its degree)
    rp, col = _csr(3, [(0, 1), (1, 2), (2, 1)])
    assert hp.graph_create_status(3, rp, col) == -2
    # asymmetric with every in-degree equal to the degree: a directed 3-cycle
    rp, col = _csr(3, [(0, 1), (1, 2), (2, 0)])
    assert hp.graph_create_status(3, rp, col) == -2
    # self-loop
    rp, col = _csr(2, [(0, 0), (0, 1), (1, 0)])
    assert hp.graph_create_status(2, rp, col) == -3
    # duplicate edge
    rp, col = _csr(2, [(0, 1), (0, 1), (1, 0), (1, 0)])
    assert hp.graph_create_status(2, rp, col) == -4
    # column out of range, negative column, non-monotone row_ptr, row_ptr[0] != 0
    rp, col = _csr(2, [(0, 1), (1, 0)])
    assert hp.graph_create_status(2, rp, np.array([5, 0], dtype=np.int32)) == -5
    assert hp.graph_create_status(2, rp, np.array([-1, 0], dtype=np.int32)) == -5
    assert hp.graph_create_status(2, np.array([0, 2, 1], dtype=np.int32),
                                  np.array([1, 0], dtype=np.int32)) == -5
    assert hp.graph_create_status(2, np.array([1, 1, 2], dtype=np.int32),
                                  np.array([1, 0], dtype=np.int32)) == -5
    # no edge (f1 = 0/0)
    assert hp.graph_create_status(3, np.zeros(4, dtype=np.int32), np.zeros(0, dtype=np.int32)) == -6
    # (2m)^2 > 2^53: the largest exact arc count is 94,906,265
    assert hp.graph_create_status(1, np.array([0, 94906266], dtype=np.int32),
                                  np.zeros(2, dtype=np.int32)) == -7
    # bad arguments
    assert hp.graph_create_status(0, np.zeros(1, dtype=np.int32), np.zeros(1, dtype=np.int32)) == -1


def test_valid_graphs_pass_validation():
    """A valid graph gets past validation: without a GPU the first device call fails
    (ERR_HIP); with one the graph is created."""
    for g in [synth.fig1_graph(), synth.appendix_graph(), synth.star(7),
              synth.with_isolated(synth.path(5), 3)]:
        st = hp.graph_create_status(g.n, g.row_ptr, g.col)
        assert st in (0, -9), st
    # unsorted adjacency is accepted (the library sorts it)
    g = synth.fig3_graph()
    col = g.col.copy()
    for v in range(g.n):
        col[g.row_ptr[v]:g.row_ptr[v + 1]] = col[g.row_ptr[v]:g.row_ptr[v + 1]][::-1]
    assert hp.graph_create_status(g.n, g.row_ptr, col) in (0, -9)


def test_symmetry_check_on_random_graphs():
    """Random simple graphs pass; the same graphs with one arc moved to another target
    (in-degrees then differ) or with two arcs' targets swapped between two sources (every
    in-degree and degree unchanged) are rejected as asymmetric."""
    rng = np.random.default_rng(5)
    for trial in range(20):
        n = int(rng.integers(5, 60))
        pairs = {(int(a), int(b)) for a, b in rng.integers(0, n, (3 * n, 2)) if a != b}
        arcs = sorted(pairs | {(b, a) for a, b in pairs})
        rp, col = _csr(n, arcs)
        assert hp.graph_create_status(n, rp, col) in (0, -9), trial
        out = {v: {b for a, b in arcs if a == v} for v in range(n)}
        # one arc v->u moved to v->w (w not yet a neighbour of v)
        v = next(x for x in range(n) if out[x] and len(out[x]) < n - 1)
        u = min(out[v])
        w = next(x for x in range(n) if x != v and x not in out[v])
        moved = sorted((a, b) if (a, b) != (v, u) else (v, w) for a, b in arcs)
        rp2, col2 = _csr(n, moved)
        assert hp.graph_create_status(n, rp2, col2) == -2, trial
        # two sources swap a target each: v->x, y->z become v->z, y->x
        cand = [(a, b, c, d) for a, b in arcs for c, d in arcs
                if a < c and b != d and d not in out[a] and b not in out[c] and d != a and b != c]
        if not cand:
            continue
        a, b, c, d = cand[int(rng.integers(len(cand)))]
        swapped = sorted({(x, y) for x, y in arcs if (x, y) not in ((a, b), (c, d))} | {(a, d), (c, b)})
        rp3, col3 = _csr(n, swapped)
        assert hp.graph_create_status(n, rp3, col3) == -2, trial


def test_no_cpu_fallback_when_library_missing(tmp_path, monkeypatch):
    monkeypatch.setattr(hp, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(hp, "_lib", None)
    with pytest.raises(RuntimeError):
        hp.lib()


def test_server_config_checks_before_any_device_call():
    """hpmocd_server_create rejects bad configurations before touching a device."""
    import ctypes as C
    L = hp.lib()
    over = L.hpmocd_server_arena_overhead(16)
    assert over > 0 and over % 256 == 0
    assert L.hpmocd_server_arena_overhead(4096) > over
    h = C.c_void_p()
    fake = C.c_void_p(1 << 20)  # never dereferenced: every case fails validation first

    def create(budget, max_active, es, flags, arena):
        cfg = hp.ServerConfig(budget, max_active, es, flags)
        return L.hpmocd_server_create(C.byref(cfg), fake, arena, None, C.byref(h))

    assert create(1 << 20, 0, 4, 0, over + (1 << 20)) == -1        # no slot
    assert create(1 << 20, 4097, 4, 0, over + (1 << 20)) == -1     # above the slot limit
    assert create(1 << 20, 16, 9, 0, over + (1 << 20)) == -1       # E_S above 8
    assert create(1 << 20, 16, 4, 2, over + (1 << 20)) == -1       # unknown flag
    assert create(1 << 20, 16, 4, 0, over + (1 << 20) - 1) == -8   # arena below budget
    assert create(0, 16, 4, 0, over + (1 << 20)) == -8             # empty budget
    assert L.hpmocd_server_submit(None, 1, None, None, None, None, None) == -1
    assert L.hpmocd_server_poll(None, 1, None) == -1
    assert L.hpmocd_server_wait(None, 1, 0.0, None, None) == -1
    assert L.hpmocd_server_cancel(None, 1) == -1
    L.hpmocd_server_destroy(None)


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N (N > 1) exits with a message instead of running (one-GPU build)."""
    import json
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]
