"""The allocation-free fitness entry point (hpmocd_eval_noalloc) through the C ABI: the same
results as hpmocd_eval, bit for bit, on consecutive calls that share the library's fixed
device scratch (a larger call, then a smaller one, then the plain-histogram path over what
the binned one left behind), and its errors."""
import ctypes as C
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_01752_amd as m
    m.lib()
    return m


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def _labels(g, k, seed):
    """k partitions: half drawn from a few communities, half self-or-neighbour rows"""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(k):
        if i % 2:
            rows.append(rng.integers(0, max(1, g.n // 50), size=g.n) * 7 % g.n)
        else:
            lab = np.arange(g.n)
            for v in range(0, g.n, 3):
                d = g.row_ptr[v + 1] - g.row_ptr[v]
                if d:
                    lab[v] = g.col[g.row_ptr[v] + rng.integers(0, d)]
            rows.append(lab)
    return np.ascontiguousarray(np.stack(rows), dtype=np.int32)


def _same(a, b):
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(bits(a[2]), bits(b[2])) and np.array_equal(bits(a[3]), bits(b[3]))


def test_noalloc_equals_eval_on_consecutive_calls(hp):
    import torch
    stream = torch.cuda.Stream()
    big = synth.planted_partition(20000, 12, 120, 0.3, 20, 400, seed=3)
    small = synth.gnp(300, 0.03, seed=5)
    cases = [(big, 100, 1), (big, 37, 2), (small, 9, 3), (small, 64, 4)]
    graphs = {}
    for g, k, seed in cases:
        say(f"noalloc: n={g.n} m={g.m} n_ind={k} seed={seed}")
        if id(g) not in graphs:
            graphs[id(g)] = hp.Graph(g.row_ptr, g.col)
        dg = graphs[id(g)]
        lab = _labels(g, k, seed)
        dl = torch.from_numpy(lab).cuda()
        ref = hp.evaluate(dg, dl, stream=stream)
        got = hp.evaluate_noalloc(dg, dl, stream=stream)
        _same(got, ref)
        # and against the oracle on a sample of rows
        for i in (0, k // 2, k - 1):
            A, S, f1, f2 = oracle.evaluate(g.row_ptr, g.col, lab[i])
            assert (got[0][i], got[1][i]) == (A, S)
            assert bits([got[2][i], got[3][i]]).tolist() == bits([f1, f2]).tolist()
    torch.cuda.synchronize()


def test_noalloc_errors(hp):
    import torch
    g = synth.planted_partition(20000, 12, 120, 0.3, 20, 400, seed=3)
    dg = hp.Graph(g.row_ptr, g.col)
    # 20,000 nodes x 512 partitions needs more than the fixed scratch
    need = C.c_size_t()
    assert hp.lib().hpmocd_eval_workspace_size(dg.handle, 512, C.byref(need)) == 0
    assert need.value > hp.NOALLOC_SCRATCH_BYTES
    lab = torch.zeros((512, g.n), dtype=torch.int32, device="cuda")
    say("noalloc: oversize call")
    with pytest.raises(hp.HpmocdError) as e:
        hp.evaluate_noalloc(dg, lab)
    assert e.value.status == hp.ERR_SCRATCH
    say("noalloc: label out of range")
    bad = torch.zeros((3, g.n), dtype=torch.int32, device="cuda")
    bad[1, 17] = g.n
    with pytest.raises(hp.HpmocdError) as e:
        hp.evaluate_noalloc(dg, bad)
    assert e.value.status == hp.ERR_RANGE
    # a good call after the errors still matches hpmocd_eval
    lab = torch.from_numpy(_labels(g, 5, 9)).cuda()
    _same(hp.evaluate_noalloc(dg, lab), hp.evaluate(dg, lab))
    torch.cuda.synchronize()
