"""Batched form (many graphs, each with its own population, advanced by shared launches):
every run's front equals its single-run front and the oracle's, bit for bit, whatever the
mix, the per-run parameters and the launch shapes the autotuner picks."""
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


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def same(a, b):
    return (a.labels.shape == b.labels.shape and np.array_equal(a.labels, b.labels)
            and np.array_equal(a.A, b.A) and np.array_equal(a.S, b.S)
            and np.array_equal(bits(a.f1), bits(b.f1)) and np.array_equal(bits(a.f2), bits(b.f2))
            and a.selected == b.selected)


def small_batch(count, seed=0, nmax=6000):
    out = []
    for p in synth.batch_params(count, seed=seed):
        p = dict(p, n=min(p["n"], nmax))
        out.append(synth.batch_graph(p))
    return out


def test_batch_matches_single_runs_and_oracle(hp):
    import torch
    s = torch.cuda.Stream()
    graphs = small_batch(10) + [synth.fig1_graph(), synth.star(30), synth.small_1k()]
    print(f"batch of {len(graphs)}: n = {[g.n for g in graphs]}", flush=True)
    rng = np.random.default_rng(3)
    params = []
    for i, g in enumerate(graphs):
        params.append(hp.make_params(pop_size=int(rng.choice([8, 33, 64, 100])), generations=9,
                                     crossover_p=float(rng.choice([0.8, 0.9, 1.0])),
                                     mutation_p=float(rng.choice([0.1, 0.2, 0.5])),
                                     parents_per_child=4, seed=int(rng.integers(0, 2**40))))
    dgs = [hp.Graph(g.row_ptr, g.col) for g in graphs]
    fronts = hp.run_batch(dgs, params, stream=s)
    for i, (g, dg, p) in enumerate(zip(graphs, dgs, params)):
        single = hp.run(dg, p, stream=s)
        assert same(fronts[i], single), f"graph {i}: batched front differs from its single run"
        ref = oracle.run(g.row_ptr, g.col, pop_size=p.pop_size, generations=p.generations,
                         crossover_p=p.crossover_p, mutation_p=p.mutation_p,
                         parents_per_child=p.parents_per_child, seed=p.seed, threads=4)
        assert same(fronts[i], ref), f"graph {i}: batched front differs from the oracle"


def test_batch_autotuned_and_plain_launches_agree(hp):
    import torch
    s = torch.cuda.Stream()
    graphs = small_batch(16, seed=1, nmax=20000)
    dgs = [hp.Graph(g.row_ptr, g.col) for g in graphs]
    p = hp.make_params(pop_size=64, generations=6, seed=5)
    a = hp.run_batch(dgs, p, stream=s)
    b, prof = hp.run_batch(dgs, p, stream=s, flags=hp.AUTOTUNE, profile=True)
    c = hp.run_batch(dgs, p, stream=s, flags=hp.NO_GRAPH)
    d = hp.run_batch(dgs, p, stream=s, flags=hp.TIME_KERNELS, profile=True)[0]
    print("tuned", {k: v for k, v in prof.items() if k.startswith("tune")}, flush=True)
    assert prof["tune_probe_ms"] > 0
    for i in range(len(graphs)):
        assert same(a[i], b[i]) and same(a[i], c[i]) and same(a[i], d[i]), i
    for i in (0, 7, 15):
        g = graphs[i]
        ref = oracle.run(g.row_ptr, g.col, pop_size=64, generations=6, seed=5, threads=4)
        assert same(a[i], ref), i


def test_batch_of_one_is_a_run(hp):
    import torch
    s = torch.cuda.Stream()
    g = synth.mid_40k(0.3)
    dg = hp.Graph(g.row_ptr, g.col)
    p = hp.make_params(pop_size=100, generations=5)
    assert same(hp.run_batch([dg], p, stream=s)[0], hp.run(dg, p, stream=s))


def test_batch_rejects_mixed_generations(hp):
    g = synth.fig1_graph()
    dg = hp.Graph(g.row_ptr, g.col)
    with pytest.raises(hp.HpmocdError):
        hp.run_batch([dg, dg], [hp.make_params(generations=3), hp.make_params(generations=4)])


def test_batch_largest_benchmark_graphs_full_run_against_oracle(hp):
    """The batched benchmark's own graphs at full size: its three largest graphs (|V| about
    48,000-49,000) and its three smallest, pop 64, 100 generations, autotuned launch shapes
    as in the benchmark: every front equals the oracle's bit for bit."""
    import os

    import torch
    s = torch.cuda.Stream()
    ps = synth.batch_params(256, seed=0)
    by_n = sorted(range(len(ps)), key=lambda i: ps[i]["n"])
    pick = by_n[-3:] + by_n[:3]
    graphs = [synth.batch_graph(ps[i]) for i in pick]
    print(f"benchmark graphs {pick}: n = {[g.n for g in graphs]}", flush=True)
    dgs = [hp.Graph(g.row_ptr, g.col) for g in graphs]
    p = hp.make_params(pop_size=64, generations=100, crossover_p=0.9, mutation_p=0.1,
                       parents_per_child=4, seed=0)
    fronts = hp.run_batch(dgs, p, stream=s, flags=hp.AUTOTUNE)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    for i, g in zip(pick, graphs):
        ref = oracle.run(g.row_ptr, g.col, pop_size=64, generations=100, crossover_p=0.9,
                         mutation_p=0.1, parents_per_child=4, seed=0, threads=threads)
        print(f"  graph {i} (n={g.n}, m={g.m}): front {len(ref.A)}", flush=True)
        assert same(fronts[pick.index(i)], ref), f"benchmark graph {i} differs from the oracle"


def test_batch_many_fronts_through_one_pipelined_copy(hp):
    """Thirty-two fronts of |V| = 40,000 at pop 16 (up to 2.5 MB of labels each, tens of MB
    together): the batch copies them to the host in one pipelined pass, the pieces of many
    fronts (and their small objective arrays) sharing page-locked chunks and crossing chunk
    boundaries; each single run copies its front on its own. Every front must agree."""
    import torch
    s = torch.cuda.Stream()
    graphs = [synth.batch_graph(dict(p, n=40000, mean_deg=8.0))
              for p in synth.batch_params(32, seed=7)]
    dgs = [hp.Graph(g.row_ptr, g.col) for g in graphs]
    p = hp.make_params(pop_size=16, generations=3, seed=11)
    fronts = hp.run_batch(dgs, p, stream=s)
    total = sum(f.labels.nbytes for f in fronts)
    print(f"{len(fronts)} fronts, {total / 2**20:.1f} MiB of labels", flush=True)
    assert total > (8 << 20)  # more than one page-locked chunk
    for i, dg in enumerate(dgs):
        assert same(fronts[i], hp.run(dg, p, stream=s)), f"front {i} differs from its single run"
    g = graphs[5]
    ref = oracle.run(g.row_ptr, g.col, pop_size=16, generations=3, seed=11, threads=4)
    assert same(fronts[5], ref)


def test_batch_with_an_item_over_the_resident_binning_cap(hp):
    """One item of |V| = 300,000 at pop 40 has over a thousand (chunk, individual group)
    binning units, more than the binning kernel's resident workgroups, which then walk
    several units each; beside it, items small enough for one unit per workgroup. Every
    front equals its single run (whose histogram plan differs: a graph alone gets narrower
    tiles) and the large item's front equals the oracle's."""
    import torch
    s = torch.cuda.Stream()
    big = synth.planted_partition(300000, 12, 500, 0.4, 50, 2000, seed=3)
    graphs = [big, synth.small_1k(), synth.fig1_graph(),
              synth.batch_graph(dict(synth.batch_params(1, seed=4)[0], n=20000))]
    dgs = [hp.Graph(g.row_ptr, g.col) for g in graphs]
    p = hp.make_params(pop_size=40, generations=3, crossover_p=0.9, mutation_p=0.2,
                       parents_per_child=4, seed=17)
    print(f"batch n = {[g.n for g in graphs]}, pop 40", flush=True)
    fronts = hp.run_batch(dgs, p, stream=s)
    for i, dg in enumerate(dgs):
        assert same(fronts[i], hp.run(dg, p, stream=s)), f"front {i} differs from its single run"
    ref = oracle.run(big.row_ptr, big.col, pop_size=40, generations=3, crossover_p=0.9,
                     mutation_p=0.2, parents_per_child=4, seed=17, threads=8)
    assert same(fronts[0], ref)
