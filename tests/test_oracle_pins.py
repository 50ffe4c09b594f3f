"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU needed).

Each test checks one oracle function against something other than itself: closed forms of
the paper's graphs, exhaustive enumeration of every partition, the modularity identity over
the adjacency matrix, the paper's worked crossover/mutation example, rocRAND's independent
Philox, and brute-force non-dominated ranks.
"""
import json
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import synth
from tests import bruteforce as bf

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_closed_forms.json")))


def F(s):
    return Fraction(s)


# ------------------------------------------------------------------------------------------
# evaluation (section 4.1, eq. objectives)
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("name,maker", [("fig1", synth.fig1_graph), ("fig3", synth.fig3_graph),
                                        ("appendix", synth.appendix_graph)])
def test_eval_paper_graphs_closed_form(oracle_lib, name, maker):
    g = maker()
    gold = GOLD[name]
    assert g.m == gold["m"]
    A, S, f1, f2 = oracle_lib.evaluate(g.row_ptr, g.col, g.membership)
    nat = gold["natural"]
    assert (A, S) == (nat["A"], nat["S"])
    assert f1 == float(F(nat["f1"])) and f2 == float(F(nat["f2"]))
    # modularity of the drawn partition = 1 - f1 - f2 (selection criterion, eq. Q(C))
    assert F(nat["Q"]) == 1 - F(nat["f1"]) - F(nat["f2"])
    # all-in-one and all-singleton partitions
    one = np.zeros(g.n, dtype=np.int32)
    A1, S1, f11, f21 = oracle_lib.evaluate(g.row_ptr, g.col, one)
    assert (A1, S1, f11, f21) == (2 * g.m, (2 * g.m) ** 2, 0.0, 1.0)
    sing = np.arange(g.n, dtype=np.int32)
    As, Ss, f1s, f2s = oracle_lib.evaluate(g.row_ptr, g.col, sing)
    assert As == 0 and f1s == 1.0 and f2s == float(F(gold["singleton_f2"]))


@pytest.mark.parametrize("a,b", [(3, 3), (4, 7), (10, 2), (12, 12)])
def test_eval_two_cliques_closed_form(oracle_lib, a, b):
    g = synth.two_cliques(a, b)
    m = a * (a - 1) // 2 + b * (b - 1) // 2 + 1
    assert g.m == m
    labels = np.array([0] * a + [a] * b, dtype=np.int32)
    A, S, f1, f2 = oracle_lib.evaluate(g.row_ptr, g.col, labels)
    # natural split: every edge but the bridge is internal; community degree sums are
    # a(a-1)+1 and b(b-1)+1
    assert A == 2 * (m - 1)
    assert S == (a * (a - 1) + 1) ** 2 + (b * (b - 1) + 1) ** 2
    assert f1 == float(Fraction(1, m))
    assert f2 == float(Fraction(S, (2 * m) ** 2))


def test_eval_is_label_value_agnostic(oracle_lib):
    """Relabelling communities (any injective map into [0, n)) leaves A and S unchanged."""
    g = synth.gnp(60, 0.1, seed=3)
    rng = np.random.default_rng(0)
    lab = rng.integers(0, 7, size=g.n).astype(np.int32)
    perm = rng.permutation(g.n).astype(np.int32)
    assert oracle_lib.evaluate(g.row_ptr, g.col, lab) == \
        oracle_lib.evaluate(g.row_ptr, g.col, perm[lab])


@pytest.mark.parametrize("seed", range(6))
def test_modularity_identity_integers(oracle_lib, seed):
    """Newman modularity (eq. modularity) over the adjacency matrix, in integers:
    sum_ij (2m A_ij - k_i k_j) [c_i = c_j] = 2m A - S, and Q = (1 - f1) - f2 within 4 ulp."""
    rng = np.random.default_rng(seed)
    g = synth.gnp(int(rng.integers(5, 70)), float(rng.uniform(0.05, 0.5)), seed=seed)
    if g.m == 0:
        pytest.skip("empty draw")
    Amat = bf.adjacency(g)
    k = Amat.sum(1)
    for _ in range(5):
        lab = rng.integers(0, int(rng.integers(1, g.n + 1)), size=g.n).astype(np.int32)
        same = lab[:, None] == lab[None, :]
        lhs = int(((2 * g.m) * Amat - np.outer(k, k))[same].sum())
        A, S, f1, f2 = oracle_lib.evaluate(g.row_ptr, g.col, lab)
        assert lhs == 2 * g.m * A - S
        Qbf = float(Fraction(lhs, (2 * g.m) ** 2))
        assert abs(Qbf - ((1.0 - f1) - f2)) <= 4 * np.spacing(1.0)


def test_eval_invariants_random(oracle_lib):
    rng = np.random.default_rng(1)
    g = synth.small_1k()
    deg = g.deg
    for _ in range(10):
        lab = rng.integers(0, g.n, size=g.n).astype(np.int32)
        A, S, f1, f2 = oracle_lib.evaluate(g.row_ptr, g.col, lab)
        ncomm = len(np.unique(lab))
        assert A % 2 == 0 and 0 <= A <= 2 * g.m
        assert (2 * g.m) ** 2 // ncomm <= S <= (2 * g.m) ** 2
        # S from a histogram built a different way
        D = np.bincount(lab, weights=deg, minlength=g.n).astype(np.int64)
        assert D.sum() == 2 * g.m and int((D * D).sum()) == S


# ------------------------------------------------------------------------------------------
# exhaustive Pareto fronts (section 2.2 definitions of dominance, PF)
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("name,maker,bell", [("appendix", synth.appendix_graph, 4140),
                                             ("fig1", synth.fig1_graph, 115975)])
def test_bruteforce_front_and_oracle_eval(oracle_lib, name, maker, bell):
    g = maker()
    parts = bf.all_partitions(g.n)
    assert len(parts) == bell
    A, S = bf.objectives_bruteforce(g, parts)
    m2 = 2 * g.m
    front = bf.pareto_points(np.stack([m2 - A, S], axis=1))
    gold = GOLD[name]
    if "front" in gold:
        want = [(F(a), F(b)) for a, b in gold["front"]]
        got = [(Fraction(int(k1), m2), Fraction(int(k2), m2 * m2)) for k1, k2 in front]
        assert got == want
    else:
        assert len(front) == gold["front_size"]
    nat = gold["natural"]
    assert (m2 - nat["A"], nat["S"]) in front
    # the oracle's evaluation agrees with the pair-sum definition on a sample of partitions
    rng = np.random.default_rng(0)
    for idx in rng.choice(len(parts), size=300, replace=False):
        lab = parts[idx].astype(np.int32)
        a, s, f1, f2 = oracle_lib.evaluate(g.row_ptr, g.col, lab)
        assert (a, s) == (int(A[idx]), int(S[idx]))


@pytest.mark.parametrize("maker", [synth.appendix_graph, synth.fig1_graph, synth.fig3_graph])
def test_oracle_run_front_is_valid_on_small_graphs(oracle_lib, maker):
    """Whole runs on graphs small enough to enumerate: every returned (A, S) is the exact
    value of its partition, returned points are mutually non-dominated, and none of them
    strictly dominates a point of the true front."""
    g = maker()
    parts = bf.all_partitions(g.n) if g.n <= 10 else None
    fr = oracle_lib.run(g.row_ptr, g.col, pop_size=20, generations=30, seed=7)
    m2 = 2 * g.m
    for i in range(len(fr.A)):
        A2, S2 = bf.objectives_bruteforce(g, fr.labels[i:i + 1])
        assert (int(A2[0]), int(S2[0])) == (int(fr.A[i]), int(fr.S[i]))
        assert 0 <= fr.labels[i].min() and fr.labels[i].max() < g.n
    k1 = m2 - fr.A
    k2 = fr.S
    assert (bf.ranks_by_peeling(k1, k2) == 1).all()
    if parts is not None:
        A, S = bf.objectives_bruteforce(g, parts)
        true_front = bf.pareto_points(np.stack([m2 - A, S], axis=1))
        for a1, a2 in zip(k1, k2):
            for t1, t2 in true_front:
                assert not (a1 <= t1 and a2 <= t2 and (a1 < t1 or a2 < t2))
    q = (1.0 - fr.f1) - fr.f2
    assert fr.selected == int(np.argmax(q))       # Alg. 3: first maximum wins


# ------------------------------------------------------------------------------------------
# crossover and mutation: the appendix worked example (Alg. 2, section 4.3)
# ------------------------------------------------------------------------------------------
def test_appendix_worked_example(oracle_lib):
    g = synth.appendix_graph()
    ex = GOLD["appendix"]["example"]
    B, G = 0, 7                                # any two label values in [0, n)

    def row(s):
        return np.array([B if ch == "B" else G for ch in s], dtype=np.int32)

    parents = np.stack([row(ex["parent1"]), row(ex["parent2"]), row(ex["parent3"])])
    child = oracle_lib.crossover(parents, -1, seed=0, gen=1, j=0)
    assert (child == row(ex["child"])).all()
    v = ex["mutated_node"] - 1
    new_label = oracle_lib.neighbour_plurality(g.row_ptr, g.col, child, v, seed=0, gen=1, j=0)
    mutated = child.copy()
    mutated[v] = new_label
    assert (mutated == row(ex["mutated"])).all()
    for key, lab in [("parent1", parents[0]), ("parent2", parents[1]), ("parent3", parents[2]),
                     ("child", child), ("mutated", mutated)]:
        A, S, f1, f2 = oracle_lib.evaluate(g.row_ptr, g.col, lab)
        w1, w2 = ex["objectives"][key]
        assert Fraction(2 * g.m - A, 2 * g.m) == F(w1)
        assert Fraction(S, (2 * g.m) ** 2) == F(w2)
        assert bf.frac_objectives(g, lab) == (F(w1), F(w2))
    # mutation with probability 1 applies the neighbour plurality to every node at once
    # (synchronously): on the example's offspring every node's neighbourhood is unanimous
    # or has a strict majority except nodes 4 and 5
    full = oracle_lib.mutate(g.row_ptr, g.col, child, 1.0, seed=0, gen=1, j=0)
    for u in [0, 1, 2, 5, 6, 7]:
        nb = child[g.col[g.row_ptr[u]:g.row_ptr[u + 1]]]
        vals, cnt = np.unique(nb, return_counts=True)
        assert full[u] == vals[np.argmax(cnt)]


def test_crossover_copy_gate(oracle_lib):
    rng = np.random.default_rng(5)
    parents = rng.integers(0, 50, size=(4, 50)).astype(np.int32)
    for k in range(4):
        assert (oracle_lib.crossover(parents, k, 0, 3, 2) == parents[k]).all()


def test_crossover_tie_break_is_valid_and_uniform(oracle_lib):
    """Ties (eq. arg_max) are broken uniformly over the tied labels: with parents carrying
    labels {a, a, b, b} at every node, the child takes a or b with frequency 1/2 each."""
    n = 4000
    a, b = 3, 11
    parents = np.array([[a] * n, [b] * n, [a] * n, [b] * n], dtype=np.int32)
    child = oracle_lib.crossover(parents, -1, seed=42, gen=5, j=9)
    assert set(np.unique(child)) <= {a, b}
    frac = np.count_nonzero(child == a) / n
    assert abs(frac - 0.5) < 4 * np.sqrt(0.25 / n)
    # four distinct labels: each chosen about a quarter of the time
    parents = np.array([[1] * n, [2] * n, [3] * n, [4] * n], dtype=np.int32)
    child = oracle_lib.crossover(parents, -1, seed=1, gen=2, j=3)
    cnt = np.bincount(child, minlength=5)[1:]
    chi2 = ((cnt - n / 4) ** 2 / (n / 4)).sum()
    assert chi2 < 16.3                          # 3 dof, p ~ 0.001


def test_mutation_rate_and_validity(oracle_lib):
    g = synth.small_1k()
    rng = np.random.default_rng(2)
    C = rng.integers(0, 30, size=g.n).astype(np.int32)
    out = oracle_lib.mutate(g.row_ptr, g.col, C, 0.25, seed=3, gen=4, j=5)
    changed_or_picked = 0
    for v in range(g.n):
        nb = C[g.col[g.row_ptr[v]:g.row_ptr[v + 1]]]
        if out[v] != C[v]:
            vals, cnt = np.unique(nb, return_counts=True)
            assert out[v] in vals[cnt == cnt.max()]
            changed_or_picked += 1
    assert 0 < changed_or_picked < g.n * 0.25 + 4 * np.sqrt(g.n)
    assert (oracle_lib.mutate(g.row_ptr, g.col, C, 0.0, 3, 4, 5) == C).all()


# ------------------------------------------------------------------------------------------
# Philox4x32-10 against rocRAND's implementation (an independent library routine)
# ------------------------------------------------------------------------------------------
def test_philox_matches_rocrand(oracle_lib, tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "kat")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "rocrand_philox_kat.cpp")])
    rng = np.random.default_rng(0)
    # rocRAND reaches counter words (x, ind) through a 64-bit skip-ahead of 4 (x + 2^32 ind)
    # outputs, so ind stays below 2^30 here; gen and tag are its 64-bit subsequence
    cases = [(0, 0, 0, 0, 0), (2**64 - 1, 2**32 - 1, 2**30 - 1, 2**32 - 1, 3)]
    for _ in range(200):
        cases.append((int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2)),
                      int(rng.integers(0, 2**32)), int(rng.integers(0, 2**30)),
                      int(rng.integers(0, 2**32)), int(rng.integers(0, 4))))
    inp = "\n".join(" ".join(map(str, c)) for c in cases) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [list(map(int, line.split())) for line in out.strip().splitlines()]
    for c, r in zip(cases, ref):
        assert list(oracle_lib.philox(*c)) == r, c


def test_pick_and_threshold(oracle_lib):
    assert oracle_lib.pick(0, 7) == 0
    assert oracle_lib.pick(2**32 - 1, 7) == 6
    assert oracle_lib.pick(2**31, 10) == 5
    assert oracle_lib.thr(0.0) == 0 and oracle_lib.thr(1.0) == 2**32
    assert oracle_lib.thr(0.5) == 2**31 and oracle_lib.thr(0.1) == 429496729


# ------------------------------------------------------------------------------------------
# initialisation (reading: own id or a uniform neighbour; parity unpinned by the paper)
# ------------------------------------------------------------------------------------------
def test_init_support_and_uniformity(oracle_lib):
    g = synth.star(9)
    cnt = np.zeros(9, dtype=np.int64)
    for i in range(4000):
        lab = oracle_lib.init_individual(g.row_ptr, g.col, 0, i)
        cnt[lab[0]] += 1
        for v in range(1, 9):
            assert lab[v] in (v, 0)
    chi2 = ((cnt - 4000 / 9) ** 2 / (4000 / 9)).sum()
    assert chi2 < 26.1                         # 8 dof, p ~ 0.001
    g = synth.small_1k()
    lab = oracle_lib.init_individual(g.row_ptr, g.col, 5, 3)
    for v in range(g.n):
        assert lab[v] == v or lab[v] in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]


# ------------------------------------------------------------------------------------------
# non-dominated sort, crowding and order (NSGA-II routines of Alg. 1)
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(8))
def test_rank_matches_peeling(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 120))
    hi = int(rng.choice([3, 10, 1000]))          # small ranges give many duplicates
    k1 = rng.integers(0, hi, size=n)
    k2 = rng.integers(0, hi, size=n)
    assert (oracle_lib.rank(k1, k2) == bf.ranks_by_peeling(k1, k2)).all()


def test_crowding_hand_cases(oracle_lib):
    inf = np.inf
    # one front of four points on 2m = 4: f1 = k1/4, f2 = k2/16
    k1 = np.array([0, 1, 2, 4]); k2 = np.array([16, 8, 4, 0])
    r = oracle_lib.rank(k1, k2)
    assert (r == 1).all()
    cd = oracle_lib.crowding(r, k1, k2, k1 / 4, k2 / 16)
    # f1 pass adds (0.5-0)/1 and (1-0.25)/1 to members 1 and 2; the f2 pass (sorted 3,2,1,0)
    # adds (0.5-0)/1 to member 2 and (1-0.25)/1 to member 1
    assert list(cd) == [inf, 1.25, 1.25, inf]
    assert list(oracle_lib.order(r, cd)) == [0, 3, 1, 2]
    # fronts of size <= 2 get +inf; a duplicated point keeps its own entry
    k1 = np.array([0, 0, 3, 1]); k2 = np.array([5, 5, 9, 9])
    r = oracle_lib.rank(k1, k2)
    assert list(r) == [1, 1, 3, 2]
    cd = oracle_lib.crowding(r, k1, k2, k1 / 8.0, k2 / 64.0)
    assert list(cd) == [inf, inf, inf, inf]
    # zero range in one objective adds nothing for it; ends are still +inf
    k1 = np.array([2, 2, 2]); k2 = np.array([1, 1, 1])
    r = oracle_lib.rank(k1, k2)
    cd = oracle_lib.crowding(r, k1, k2, k1 / 4.0, k2 / 16.0)
    assert list(cd) == [inf, 0.0, inf]
    # five points, unequal spacing: f1 = (0, 1, 3, 4, 8)/8, f2 = (8, 6, 5, 2, 0)/8
    k1 = np.array([0, 1, 3, 4, 8]); k2 = np.array([8, 6, 5, 2, 0])
    r = oracle_lib.rank(k1, k2)
    cd = oracle_lib.crowding(r, k1, k2, k1 / 8.0, k2 / 8.0)
    # member 1: (3-0)/8 + (8-5)/8 = 0.75; member 2: (4-1)/8 + (6-2)/8 = 0.875;
    # member 3: (8-3)/8 + (5-0)/8 = 1.25
    assert list(cd) == [inf, 0.75, 0.875, 1.25, inf]
    assert list(oracle_lib.order(r, cd)) == [0, 4, 3, 2, 1]


def test_order_tie_rules(oracle_lib):
    rank_ = np.array([2, 1, 1, 2, 1])
    crowd = np.array([np.inf, 0.5, np.inf, np.inf, np.inf])
    assert list(oracle_lib.order(rank_, crowd)) == [2, 4, 1, 0, 3]


# ------------------------------------------------------------------------------------------
# whole runs: determinism, thread invariance, elitism
# ------------------------------------------------------------------------------------------
def test_run_deterministic_and_thread_invariant(oracle_lib):
    g = synth.small_1k()
    a = oracle_lib.run(g.row_ptr, g.col, pop_size=16, generations=8, seed=3)
    b = oracle_lib.run(g.row_ptr, g.col, pop_size=16, generations=8, seed=3, threads=4)
    assert (a.labels == b.labels).all() and (a.A == b.A).all() and (a.S == b.S).all()
    c = oracle_lib.run(g.row_ptr, g.col, pop_size=16, generations=8, seed=4)
    assert not (len(c.A) == len(a.A) and (c.labels == a.labels).all())


def test_run_elitism_and_trace(oracle_lib):
    g = synth.small_1k()
    states = []
    oracle_lib.run(g.row_ptr, g.col, pop_size=24, generations=12, seed=1,
                   on_generation=states.append)
    assert [s.g for s in states] == list(range(13))
    m2 = 2 * g.m
    for s in states:
        for i in range(len(s.A)):
            A, S, _, _ = oracle_lib.evaluate(g.row_ptr, g.col, s.labels[i])
            assert (A, S) == (s.A[i], s.S[i])
    for prev, cur in zip(states, states[1:]):
        k1c, k2c = m2 - cur.A, cur.S
        if (bf.ranks_by_peeling(k1c, k2c) == 1).sum() < len(cur.A):
            for a1, a2 in zip(m2 - prev.A, prev.S):
                assert ((k1c <= a1) & (k2c <= a2)).any()
        # rank/crowd reported for generation g are those of P^(g-1) after reordering
        assert cur.rank is not None and (np.diff(cur.rank) >= 0).all()


def test_run_edge_cases(oracle_lib):
    g = synth.appendix_graph()
    for np_, T in [(1, 0), (1, 3), (2, 5), (3, 4)]:
        fr = oracle_lib.run(g.row_ptr, g.col, pop_size=np_, generations=T, seed=0)
        assert 1 <= len(fr.A) <= np_
    for es in [1, 2, 3, 8]:
        oracle_lib.run(g.row_ptr, g.col, pop_size=6, generations=3, parents_per_child=es)
    for cp, mp in [(0.0, 0.0), (1.0, 1.0), (0.0, 1.0), (1.0, 0.0)]:
        oracle_lib.run(g.row_ptr, g.col, pop_size=6, generations=3, crossover_p=cp,
                       mutation_p=mp)
    gi = synth.with_isolated(synth.fig1_graph(), 5)
    fr = oracle_lib.run(gi.row_ptr, gi.col, pop_size=8, generations=4)
    deg = np.diff(gi.row_ptr)
    for row in fr.labels:     # isolated nodes are never mutated: they keep their init label
        assert (row[deg == 0] == np.flatnonzero(deg == 0)).all()


# ------------------------------------------------------------------------------------------
# tournament selection (Alg. 1 TournamentSelection, k = 2) and the crossover gate (Alg. 2,
# section 4.3.1)
# ------------------------------------------------------------------------------------------
def _chi2(cnt, p):
    e = p * cnt.sum()
    return float(((cnt - e) ** 2 / e).sum())


@pytest.mark.parametrize("N,crit", [(2, 10.83), (7, 22.46), (100, 148.2), (130, 184.4)])
def test_tournament_winner_law(oracle_lib, N, crit):
    """A binary tournament with replacement over a population in crowded order, the better
    (lower) position winning, picks position q with probability ((N-q)^2 - (N-q-1)^2) / N^2
    = (2(N-q) - 1) / N^2. The reversed rule (higher position wins) has law (2q + 1) / N^2 and
    a single uniform contestant 1 / N; both must fail the same chi-square test (p = 0.001)."""
    draws = 60 * N if N > 10 else 20000
    cnt = np.zeros(N, dtype=np.int64)
    for t in range(draws):
        g, j, k = 1 + t % 97, t // 97, t % 5
        q = oracle_lib.tournament(seed=11, gen=g, j=j, k=k, pop_size=N)
        assert 0 <= q < N
        cnt[q] += 1
    q = np.arange(N)
    law = (2 * (N - q) - 1) / N**2
    assert abs(law.sum() - 1) < 1e-12
    assert _chi2(cnt, law) < crit
    assert _chi2(cnt, (2 * q + 1) / N**2) > 10 * crit        # higher position winning
    assert _chi2(cnt, np.full(N, 1.0 / N)) > 2 * crit         # no comparison at all


def test_tournament_edges_and_slot_independence(oracle_lib):
    assert all(oracle_lib.tournament(3, g, j, k, 1) == 0
               for g in range(3) for j in range(5) for k in range(8))
    # the E_S slots of one offspring are independent tournaments: the joint law of slot 0
    # and slot 1 winning in the top half factorises (2 x 2 contingency chi-square, 1 dof)
    N, tab = 50, np.zeros((2, 2), dtype=np.int64)
    for j in range(8000):
        a = oracle_lib.tournament(5, 3, j, 0, N) < N // 2
        b = oracle_lib.tournament(5, 3, j, 1, N) < N // 2
        tab[int(a), int(b)] += 1
    e = np.outer(tab.sum(1), tab.sum(0)) / tab.sum()
    assert float(((tab - e) ** 2 / e).sum()) < 10.83


@pytest.mark.parametrize("cp,es", [(0.9, 4), (0.5, 3), (0.2, 8), (0.8, 1)])
def test_crossover_gate_frequency(oracle_lib, cp, es):
    """Alg. 2 crosses over when its uniform draw x satisfies x <= C_P (probability C_P) and
    otherwise copies one parent, each of the E_S with probability 1 / E_S. An inverted gate
    (crossover with probability 1 - C_P) must fail the binomial bound."""
    n = 40000
    gates = np.array([oracle_lib.gate(seed=2, gen=1 + j % 50, j=j // 50, crossover_p=cp,
                                      parents_per_child=es) for j in range(n)])
    assert ((gates >= -1) & (gates < es)).all()
    frac = np.count_nonzero(gates == -1) / n
    sd = np.sqrt(cp * (1 - cp) / n)
    assert abs(frac - cp) < 5 * sd
    assert abs(frac - (1 - cp)) > 5 * sd or cp == 0.5
    copies = np.bincount(gates[gates >= 0], minlength=es)
    if es > 1:
        crit = {3: 13.82, 4: 16.27, 8: 24.32}[es]
        assert _chi2(copies, np.full(es, 1.0 / es)) < crit
    assert all(oracle_lib.gate(2, 1, j, 0.0, es) >= 0 for j in range(500))
    assert all(oracle_lib.gate(2, 1, j, 1.0, es) == -1 for j in range(500))


def test_run_copies_only_without_crossover_and_mutation(oracle_lib):
    """With C_P = 0 and M_P = 0 every offspring is a copy of a parent, so every row of every
    P(g) is a row of the initial population P(0)."""
    g = synth.small_1k()
    states = []
    oracle_lib.run(g.row_ptr, g.col, pop_size=16, generations=8, crossover_p=0.0,
                   mutation_p=0.0, seed=4, on_generation=states.append)
    rows0 = {r.tobytes() for r in states[0].labels}
    assert len(rows0) > 1
    for s in states[1:]:
        for r in s.labels:
            assert r.tobytes() in rows0


def _reordered_previous(oracle_lib, g, prev, cur):
    """P(g-1) of a trace reordered by its own rank and crowding (Alg. 1 SortByRankAndDistance),
    checked against the rank / crowding the run reports at generation g."""
    m2 = 2 * g.m
    k1, k2 = m2 - prev.A, prev.S
    r = oracle_lib.rank(k1, k2)
    cd = oracle_lib.crowding(r, k1, k2, prev.f1, prev.f2)
    o = oracle_lib.order(r, cd)
    assert (r[o] == cur.rank).all()
    assert (cd[o].view(np.uint64) == cur.crowd.view(np.uint64)).all()
    return prev.labels[o]


@pytest.mark.parametrize("es", [1, 3, 4])
def test_run_crossover_only_children_are_parent_pluralities(oracle_lib, es):
    """With C_P = 1 and M_P = 0 every offspring is the ensemble crossover of its E_S
    tournament winners: at every node the child's label has the maximal multiplicity among
    the parents' labels there (eq. arg_max), and the next population consists of members
    of the previous one and of these children only."""
    g = synth.small_1k()
    states = []
    Np = 12
    kw = dict(crossover_p=1.0, mutation_p=0.0, parents_per_child=es, seed=9)
    oracle_lib.run(g.row_ptr, g.col, pop_size=Np, generations=5, on_generation=states.append,
                   **kw)
    for prev, cur in zip(states, states[1:]):
        P = _reordered_previous(oracle_lib, g, prev, cur)
        kids = set()
        for j in range(Np):
            child, pos, gate = oracle_lib.offspring(g.row_ptr, g.col, P, es, 1.0, 0.0, 9,
                                                    cur.g, j)
            assert gate == -1 and ((pos >= 0) & (pos < Np)).all()
            par = P[pos]                                   # (es, n)
            mult = (par[:, None, :] == par[None, :, :]).sum(1)   # multiplicity of each label
            assert (((par == child[None, :]).sum(0)) == mult.max(0)).all()
            if es == 1:
                assert (child == par[0]).all()
            kids.add(child.tobytes())
        allowed = kids | {r.tobytes() for r in P}
        for r in cur.labels:
            assert r.tobytes() in allowed


def test_run_copy_gate_children_are_their_parents(oracle_lib):
    """With C_P = 0 the gate copies parent slot pick(w1, E_S); with M_P = 0 the offspring is
    that parent's row unchanged."""
    g = synth.appendix_graph()
    rng = np.random.default_rng(3)
    P = rng.integers(0, g.n, size=(9, g.n)).astype(np.int32)
    for j in range(40):
        child, pos, gate = oracle_lib.offspring(g.row_ptr, g.col, P, 4, 0.0, 0.0, 1, 2, j)
        assert 0 <= gate < 4
        assert (child == P[pos[gate]]).all()
