"""Checkpoint / resume: a run stopped after generation k and resumed from its snapshot gives
the uninterrupted run's front bit for bit; the snapshot is the traced population."""
import numpy as np
import pytest

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


def same(a, b):
    bits = lambda x: np.ascontiguousarray(x, dtype=np.float64).view(np.uint64)
    return (np.array_equal(a.labels, b.labels) and np.array_equal(a.A, b.A)
            and np.array_equal(a.S, b.S) and np.array_equal(bits(a.f1), bits(b.f1))
            and np.array_equal(bits(a.f2), bits(b.f2)) and a.selected == b.selected)


@pytest.mark.parametrize("gname,k", [("small_1k", 0), ("small_1k", 7), ("small_1k", 12),
                                     ("mid_40k", 5), ("hub", 3)])
def test_resume_equals_uninterrupted(hp, gname, k):
    import torch
    s = torch.cuda.Stream()
    if gname == "hub":  # degree classes up to the large-node path
        rng = np.random.default_rng(1)
        edges = [(0, i) for i in range(1, 3001)] + [tuple(e) for e in rng.integers(1, 3001, (5000, 2))]
        g = synth.csr_from_edges(3001, edges)
    else:
        g = {"small_1k": synth.small_1k, "mid_40k": lambda: synth.mid_40k(0.5)}[gname]()
    dg = hp.Graph(g.row_ptr, g.col)
    p = hp.make_params(pop_size=48, generations=12, mutation_p=0.3, seed=17)
    states = []
    full = hp.run(dg, p, stream=s, on_generation=states.append)
    snap = hp.run_to(dg, p, stop_gen=k, stream=s)
    assert snap.g == k
    st = states[k]
    assert np.array_equal(snap.labels, st.labels)
    assert np.array_equal(snap.A, st.A) and np.array_equal(snap.S, st.S)
    resumed = hp.resume(dg, snap, p, stream=s)
    assert same(resumed, full), f"{gname}: resumed after {k} differs"
    plain = hp.run(dg, p, stream=s)
    assert same(plain, full)


def test_snapshot_of_a_wide_population(hp):
    """pop 300: the snapshot's 300 label rows leave the device through the extraction kernel
    in three tiles of up to 128 rows (the last one partial). They equal the traced population,
    resuming from them (which re-evaluates them) gives the uninterrupted front, and that
    front is the oracle's."""
    import torch

    import oracle
    s = torch.cuda.Stream()
    g = synth.small_1k()
    dg = hp.Graph(g.row_ptr, g.col)
    p = hp.make_params(pop_size=300, generations=5, seed=23)
    states = []
    full = hp.run(dg, p, stream=s, on_generation=states.append)
    snap = hp.run_to(dg, p, stop_gen=3, stream=s)
    assert snap.labels.shape == (300, g.n)
    assert np.array_equal(snap.labels, states[3].labels)
    assert same(hp.resume(dg, snap, p, stream=s), full)
    ref = oracle.run(g.row_ptr, g.col, pop_size=300, generations=5, seed=23, threads=4)
    assert same(full, ref)


def test_resume_rejects_bad_snapshots(hp):
    g = synth.small_1k()
    dg = hp.Graph(g.row_ptr, g.col)
    p = hp.make_params(pop_size=16, generations=4, seed=1)
    snap = hp.run_to(dg, p, stop_gen=2)
    bad = hp.Snapshot(snap.g, snap.labels.copy(), snap.A, snap.S)
    bad.labels[3, 5] = g.n  # label outside [0, n)
    with pytest.raises(hp.HpmocdError):
        hp.resume(dg, bad, p)
    with pytest.raises(hp.HpmocdError):
        hp.resume(dg, hp.Snapshot(9, snap.labels, snap.A, snap.S), p)  # g > T
    with pytest.raises(hp.HpmocdError):
        hp.run_to(dg, p, stop_gen=5)  # beyond T
    assert snap.graph_hash == dg.hash and snap.params.seed == 1
    # another seed, crossover or mutation rate, ensemble size: not this run's snapshot
    for kw in (dict(seed=2), dict(crossover_p=0.8), dict(mutation_p=0.2),
               dict(parents_per_child=3)):
        with pytest.raises(hp.HpmocdError) as e:
            hp.resume(dg, snap, hp.make_params(**dict(dict(pop_size=16, generations=4, seed=1),
                                                      **kw)))
        assert e.value.status == hp.ERR_ARG, kw
    # another graph with the same number of nodes
    other = synth.small_1k(seed=1)
    assert other.n == g.n
    dg2 = hp.Graph(other.row_ptr, other.col)
    assert dg2.hash != dg.hash
    with pytest.raises(hp.HpmocdError) as e:
        hp.resume(dg2, snap, p)
    assert e.value.status == hp.ERR_ARG
    # objectives that do not belong to the labels (re-evaluated on the device)
    for which in ("A", "S"):
        stale = hp.Snapshot(snap.g, snap.labels, snap.A.copy(), snap.S.copy(), snap.params,
                            snap.graph_hash)
        getattr(stale, which)[7] += 2
        with pytest.raises(hp.HpmocdError) as e:
            hp.resume(dg, stale, p)
        assert e.value.status == hp.ERR_ARG, which
    # a snapshot without its fingerprint (e.g. built by hand) is refused
    with pytest.raises(hp.HpmocdError):
        hp.resume(dg, hp.Snapshot(snap.g, snap.labels, snap.A, snap.S), p)


def test_resume_to_more_generations(hp):
    """The generation count may grow on resume: a run stopped at k of T and resumed to T' > T
    equals the uninterrupted run of T' generations."""
    import torch
    s = torch.cuda.Stream()
    g = synth.small_1k()
    dg = hp.Graph(g.row_ptr, g.col)
    p6 = hp.make_params(pop_size=24, generations=6, seed=3)
    p11 = hp.make_params(pop_size=24, generations=11, seed=3)
    snap = hp.run_to(dg, p6, stop_gen=6, stream=s)
    assert same(hp.resume(dg, snap, p11, stream=s), hp.run(dg, p11, stream=s))
