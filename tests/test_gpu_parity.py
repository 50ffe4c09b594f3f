"""GPU path vs the CPU oracle, through the C ABI: bit-exact labels, integer counts and
binary64 objectives (and, per generation, ranks and crowding distances)."""
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


@pytest.fixture(scope="module")
def stream(hp):
    import torch
    return torch.cuda.Stream()


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def assert_front_equal(got, ref):
    assert got.labels.shape == ref.labels.shape, (got.labels.shape, ref.labels.shape)
    assert np.array_equal(got.labels, ref.labels)
    assert np.array_equal(got.A, ref.A)
    assert np.array_equal(got.S, ref.S)
    assert np.array_equal(bits(got.f1), bits(ref.f1))
    assert np.array_equal(bits(got.f2), bits(ref.f2))
    assert got.selected == ref.selected


def assert_states_equal(gs, os_):
    assert len(gs) == len(os_)
    for a, b in zip(gs, os_):
        assert a.g == b.g
        assert np.array_equal(a.labels, b.labels), f"labels differ at generation {a.g}"
        assert np.array_equal(a.A, b.A) and np.array_equal(a.S, b.S), a.g
        assert np.array_equal(bits(a.f1), bits(b.f1)) and np.array_equal(bits(a.f2), bits(b.f2))
        if b.rank is None:
            assert a.rank is None
        else:
            assert np.array_equal(a.rank, b.rank), a.g
            assert np.array_equal(bits(a.crowd), bits(b.crowd)), a.g


# ---------------------------------------------------------------------------------------
# fitness kernel alone
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("gname", ["fig1", "appendix", "small_1k", "isolated", "star70",
                                   "mid_40k"])
@pytest.mark.parametrize("n_ind", [1, 3, 64, 100, 129, 300])
def test_eval_matches_oracle(hp, stream, gname, n_ind):
    """Small problems use the plain histogram, |V| = 40,000 with 27 or more individuals the
    binned one (both for ragged individual counts)."""
    import torch
    g = {"fig1": synth.fig1_graph, "appendix": synth.appendix_graph, "small_1k": synth.small_1k,
         "isolated": lambda: synth.with_isolated(synth.gnp(90, 0.08, 1), 13),
         "star70": lambda: synth.star(70), "mid_40k": lambda: synth.mid_40k(0.5)}[gname]()
    say(f"eval {gname} n={g.n} n_ind={n_ind}")
    rng = np.random.default_rng(n_ind)
    labs = []
    for i in range(n_ind):
        k = int(rng.integers(1, g.n + 1))
        labs.append(rng.integers(0, k, size=g.n))
    labs = np.stack(labs).astype(np.int32)
    labs[0] = g.membership if g.membership is not None else labs[0]
    dg = hp.Graph(g.row_ptr, g.col)
    t = torch.from_numpy(labs).cuda()
    A, S, f1, f2 = hp.evaluate(dg, t, stream=stream)
    for i in range(n_ind):
        ra, rs, r1, r2 = oracle.evaluate(g.row_ptr, g.col, labs[i])
        assert (A[i], S[i]) == (ra, rs), i
        assert bits([f1[i]])[0] == bits([r1])[0] and bits([f2[i]])[0] == bits([r2])[0]


def test_eval_community_indices_1m(hp, stream):
    """|V| = 1,000,000, 16 partitions: 8 labelled by planted-community indices 0..k-1 (a narrow
    label range, spread by the evaluation's interleaved histogram tiles) and 8 by node ids,
    each with 10% of its nodes relabelled at random; every objective equals the oracle's."""
    import torch
    g = synth.large_1m()
    rng = np.random.default_rng(23)
    memb = g.membership.astype(np.int64)
    k = int(memb.max()) + 1
    rows = []
    for i in range(16):
        lab = memb.copy() if i < 8 else rng.permutation(g.n)[memb]
        hi = k if i < 8 else g.n
        flip = rng.random(g.n) < 0.1
        lab[flip] = rng.integers(0, hi, int(flip.sum()))
        rows.append(lab)
    labs = np.stack(rows).astype(np.int32)
    say(f"eval large_1m n_ind=16, {k} communities")
    A, S, f1, f2 = hp.evaluate(hp.Graph(g.row_ptr, g.col), torch.from_numpy(labs).cuda(),
                               stream=stream)
    for i in range(16):
        ra, rs, r1, r2 = oracle.evaluate(g.row_ptr, g.col, labs[i])
        assert (A[i], S[i]) == (ra, rs), i
        assert bits([f1[i]])[0] == bits([r1])[0] and bits([f2[i]])[0] == bits([r2])[0]


@pytest.mark.parametrize("bad", [-1, 1000, 2**31 - 1])
def test_eval_out_of_range_label_is_an_error(hp, stream, bad):
    """A label outside [0, n) is reported as ERR_RANGE (the kernel that reads the labels
    replaces it by 0 before any label-indexed access); valid labels evaluated afterwards on the
    same graph are unaffected."""
    import torch
    g = synth.small_1k()
    say(f"eval out-of-range label {bad}")
    dg = hp.Graph(g.row_ptr, g.col)
    labs = np.zeros((3, g.n), dtype=np.int32)
    labs[1, 17] = bad
    with pytest.raises(hp.HpmocdError) as e:
        hp.evaluate(dg, torch.from_numpy(labs).cuda(), stream=stream)
    assert e.value.status == hp.ERR_RANGE
    ok = np.stack([g.membership, np.arange(g.n)]).astype(np.int32)
    A, S, f1, f2 = hp.evaluate(dg, torch.from_numpy(ok).cuda(), stream=stream)
    for i in range(2):
        assert (A[i], S[i]) == oracle.evaluate(g.row_ptr, g.col, ok[i])[:2]


# ---------------------------------------------------------------------------------------
# whole runs, traced every generation
# ---------------------------------------------------------------------------------------
def traced_pair(hp, stream, g, threads=1, **kw):
    gs, os_ = [], []
    dg = hp.Graph(g.row_ptr, g.col)
    got = hp.run(dg, stream=stream, on_generation=gs.append, **kw)
    ref = oracle.run(g.row_ptr, g.col, threads=threads, on_generation=os_.append, **kw)
    return got, ref, gs, os_


@pytest.mark.parametrize("gname", ["fig1", "fig3", "appendix", "star", "path", "k12",
                                   "isolated", "two_cliques"])
def test_run_small_graphs_every_generation(hp, stream, gname):
    g = {"fig1": synth.fig1_graph, "fig3": synth.fig3_graph, "appendix": synth.appendix_graph,
         "star": lambda: synth.star(40), "path": lambda: synth.path(33),
         "k12": lambda: synth.complete(12),
         "isolated": lambda: synth.with_isolated(synth.fig1_graph(), 7),
         "two_cliques": lambda: synth.two_cliques(9, 40)}[gname]()
    say(f"run {gname} n={g.n}")
    got, ref, gs, os_ = traced_pair(hp, stream, g, pop_size=24, generations=15, seed=3)
    assert_states_equal(gs, os_)
    assert_front_equal(got, ref)


@pytest.mark.parametrize("pop,es,cp,mp,T", [(1, 4, 0.9, 0.1, 3), (2, 1, 0.9, 0.1, 4),
                                            (3, 2, 1.0, 1.0, 4), (100, 3, 0.0, 0.5, 3),
                                            (17, 8, 1.0, 0.0, 5), (64, 4, 0.8, 0.2, 0),
                                            (130, 5, 0.7, 0.3, 3), (512, 4, 0.9, 0.1, 2)])
def test_run_parameter_edges(hp, stream, pop, es, cp, mp, T):
    g = synth.small_1k(seed=2)
    say(f"params pop={pop} es={es} cp={cp} mp={mp} T={T}")
    got, ref, gs, os_ = traced_pair(hp, stream, g, threads=4, pop_size=pop, generations=T,
                                    crossover_p=cp, mutation_p=mp, parents_per_child=es,
                                    seed=11)
    assert_states_equal(gs, os_)
    assert_front_equal(got, ref)


def test_run_1k_full_every_generation(hp, stream):
    """|V| = 1,000 planted partition, pop 100, 100 generations: every generation."""
    g = synth.small_1k()
    say("run small_1k pop100 T100 traced")
    got, ref, gs, os_ = traced_pair(hp, stream, g, threads=4, **synth.GA_DEFAULT)
    assert_states_equal(gs, os_)
    assert_front_equal(got, ref)


def test_graph_replay_equals_plain_launches(hp, stream):
    g = synth.small_1k(seed=5)
    dg = hp.Graph(g.row_ptr, g.col)
    kw = dict(pop_size=50, generations=9, seed=9)
    say("graph replay vs plain")
    a = hp.run(dg, stream=stream, **kw)                       # hipGraph replay of the loop
    b = hp.run(dg, stream=stream, flags=hp.NO_GRAPH, **kw)    # one launch per kernel
    c = hp.run(dg, stream=stream, flags=hp.TIME_KERNELS, profile=True, **kw)[0]
    ref = oracle.run(g.row_ptr, g.col, **kw)
    for x in (a, b, c):
        assert_front_equal(x, ref)


def test_high_degree_mutation_paths(hp, stream):
    """Every mutation work class: degrees up to 16 and 32 (one item per lane), 33-64,
    65-128, 129-256, 257-512 (one item per wave, cross-lane sort), 513-2048 (LDS sort) and
    above 2048 (exact scan)."""
    rng = np.random.default_rng(0)
    n = 5001
    edges = [(0, i) for i in range(1, 5001)]                      # degree 5000
    for hub, deg in [(1, 1500), (2, 700), (3, 300), (4, 200), (5, 100), (6, 50), (7, 20)]:
        nb = rng.choice(np.arange(8, n), size=deg, replace=False)
        edges += [(hub, int(u)) for u in nb]
    extra = rng.integers(8, n, size=(6000, 2))
    g = synth.csr_from_edges(n, np.concatenate([np.array(edges), extra]))
    deg = np.diff(g.row_ptr)
    say(f"hubs n={g.n} degrees={sorted(deg)[-8:]}")
    # pop 100 at M_P 1.0 fills every per-wave gather batch several times over (up to 25
    # mutations per slice), pop 20 leaves them partly empty
    for mp, seed, pop in [(0.6, 5, 20), (1.0, 6, 20), (1.0, 7, 100), (0.3, 8, 100)]:
        got, ref, gs, os_ = traced_pair(hp, stream, g, threads=4, pop_size=pop, generations=3,
                                        mutation_p=mp, seed=seed)
        assert_states_equal(gs, os_)
        assert_front_equal(got, ref)


@pytest.mark.parametrize("mu", [0.1, 0.7])
def test_run_40k_traced(hp, stream, mu):
    """|V| = 40,000 planted partition (the paper's mid scale), pop 100, first generations."""
    g = synth.mid_40k(mu)
    say(f"run mid_40k mu={mu}")
    kw = dict(synth.GA_DEFAULT, generations=4)
    got, ref, gs, os_ = traced_pair(hp, stream, g, threads=8, **kw)
    assert_states_equal(gs, os_)
    assert_front_equal(got, ref)


def test_deterministic_repeat(hp, stream):
    g = synth.small_1k(seed=7)
    dg = hp.Graph(g.row_ptr, g.col)
    a = hp.run(dg, stream=stream, pop_size=40, generations=12, seed=1)
    b = hp.run(dg, stream=stream, pop_size=40, generations=12, seed=1)
    assert_front_equal(a, b)


def test_single_edge_and_many_components(hp, stream):
    """Smallest graph (one edge) and a forest of small components with isolated nodes."""
    k2 = synth.csr_from_edges(2, [(0, 1)])
    rng = np.random.default_rng(4)
    edges = []
    for c in range(30):  # 30 small trees of 2-6 nodes, then 40 isolated nodes
        base = 6 * c
        size = int(rng.integers(2, 7))
        edges += [(base + i, base + int(rng.integers(0, i))) for i in range(1, size)]
    forest = synth.csr_from_edges(220, edges)
    for name, g in [("k2", k2), ("forest", forest)]:
        say(f"run {name} n={g.n} m={g.m}")
        got, ref, gs, os_ = traced_pair(hp, stream, g, pop_size=12, generations=6, seed=8,
                                        mutation_p=0.5)
        assert_states_equal(gs, os_)
        assert_front_equal(got, ref)


@pytest.mark.parametrize("pop", [16, 17])
def test_binned_histogram_small_population_1m(hp, stream, pop):
    """|V| = 1,000,000 with 16 and 17 individuals (one and two 16-column histogram groups,
    row strides 16 and 32): every generation against the oracle."""
    g = synth.large_1m()
    say(f"run large_1m pop={pop}")
    got, ref, gs, os_ = traced_pair(hp, stream, g, threads=8, pop_size=pop, generations=2,
                                    seed=21)
    assert_states_equal(gs, os_)
    assert_front_equal(got, ref)


def test_random_sweep_against_oracle(hp, stream):
    """Seeded random graphs (random, two-level planted, stars with isolated nodes) and random
    parameters; every front bit-exact against the oracle."""
    rng = np.random.default_rng(2024)
    for case in range(40):
        kind = case % 3
        if kind == 0:
            g = synth.gnp(int(rng.integers(2, 300)), float(rng.uniform(0.01, 0.3)), case)
        elif kind == 1:
            g = synth.planted_partition(int(rng.integers(50, 600)), float(rng.uniform(3, 12)), 40,
                                        float(rng.uniform(0.05, 0.6)), 5, 60, seed=case)
        else:
            g = synth.with_isolated(synth.star(int(rng.integers(3, 80))), int(rng.integers(0, 9)))
        if g.m == 0:
            continue
        kw = dict(pop_size=int(rng.integers(1, 70)), generations=int(rng.integers(0, 7)),
                  crossover_p=float(rng.choice([0.0, 0.5, 0.9, 1.0])),
                  mutation_p=float(rng.choice([0.0, 0.05, 0.3, 1.0])),
                  parents_per_child=int(rng.integers(1, 9)), seed=int(rng.integers(0, 2**62)))
        say(f"case {case}: n={g.n} m={g.m} {kw}")
        got = hp.run(hp.Graph(g.row_ptr, g.col), stream=stream, **kw)
        ref = oracle.run(g.row_ptr, g.col, threads=4, **kw)
        assert_front_equal(got, ref)


def test_random_hub_graphs_against_oracle(hp, stream):
    """Seeded random graphs with hubs in every per-wave and LDS mutation class (degrees up to
    ~2600) under random populations and rates, so that the per-wave gather batches run full,
    partial and split over 1, 2 or 4 slices; every front bit-exact against the oracle."""
    rng = np.random.default_rng(77)
    for case in range(12):
        n = int(rng.integers(800, 4000))
        edges = []
        for h in range(int(rng.integers(2, 7))):
            deg = int(min(n - 10, rng.choice([40, 90, 200, 400, 900, 1500, 2600])))
            nb = rng.choice(np.arange(10, n), size=deg, replace=False)
            edges += [(h, int(u)) for u in nb]
        extra = rng.integers(10, n, size=(int(rng.integers(n, 4 * n)), 2))
        g = synth.csr_from_edges(n, np.concatenate([np.array(edges), extra]))
        kw = dict(pop_size=int(rng.choice([7, 33, 100, 160])), generations=int(rng.integers(1, 4)),
                  crossover_p=float(rng.choice([0.5, 0.9])),
                  mutation_p=float(rng.choice([0.05, 0.2, 0.5, 1.0])),
                  parents_per_child=int(rng.integers(2, 6)), seed=int(rng.integers(0, 2**62)))
        say(f"hub case {case}: n={g.n} m={g.m} max_deg={int(np.diff(g.row_ptr).max())} {kw}")
        got = hp.run(hp.Graph(g.row_ptr, g.col), stream=stream, **kw)
        ref = oracle.run(g.row_ptr, g.col, threads=4, **kw)
        assert_front_equal(got, ref)
