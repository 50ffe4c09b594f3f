"""Partition-agreement measures (reporting tools): pinned to closed forms, brute force and,
where scikit-learn is importable, to its implementations."""
import itertools

import numpy as np
import pytest

from paper_2506_01752_amd import quality as q


def test_identical_up_to_renaming():
    a = np.array([0, 0, 1, 1, 2, 2, 2])
    b = np.array([7, 7, 3, 3, 9, 9, 9])
    assert q.nmi(a, b) == pytest.approx(1.0)
    assert q.ami(a, b) == pytest.approx(1.0)
    assert q.ari(a, b) == pytest.approx(1.0)
    assert q.pair_f1(a, b) == pytest.approx(1.0)


def test_single_community_and_singletons():
    n = 10
    one = np.zeros(n, dtype=int)
    single = np.arange(n)
    assert q.nmi(one, one) == 1.0
    # one side carries no information
    assert q.nmi(one, single) == pytest.approx(0.0)
    # F1: all pairs positive vs none: precision undefined -> 0 true positives
    assert q.pair_f1(single, one) == 0.0
    assert q.ari(one, single) == pytest.approx(0.0)


def test_closed_form_pairs():
    # found {0,1,2},{3,4}; truth {0,1},{2,3,4}: TP pairs = {01} + {34} = 2
    found = np.array([0, 0, 0, 1, 1])
    truth = np.array([0, 0, 1, 1, 1])
    pos_f, pos_t = 3 + 1, 1 + 3
    assert q.pair_f1(found, truth) == pytest.approx(2 * 2 / (pos_f + pos_t))
    # Rand-index pieces by hand: sum_ij C(n_ij,2) = 2, a = 4, b = 4, C(5,2) = 10
    exp = 4 * 4 / 10
    assert q.ari(found, truth) == pytest.approx((2 - exp) / (4 - exp))


def test_nmi_by_definition_small():
    a = np.array([0, 0, 1, 1])
    b = np.array([0, 1, 0, 1])
    assert q.nmi(a, b) == pytest.approx(0.0, abs=1e-12)   # independent
    a = np.array([0, 0, 0, 1])
    b = np.array([0, 0, 1, 1])
    # MI by hand: p = [[1/2, 1/4], [0, 1/4]], marginals a (3/4, 1/4), b (1/2, 1/2)
    mi = 0.5 * np.log(0.5 / (0.75 * 0.5)) + 0.25 * np.log(0.25 / (0.75 * 0.5)) + \
        0.25 * np.log(0.25 / (0.25 * 0.5))
    ha = -(0.75 * np.log(0.75) + 0.25 * np.log(0.25))
    hb = np.log(2)
    assert q.nmi(a, b) == pytest.approx(mi / (0.5 * (ha + hb)))


def test_against_sklearn_random():
    metrics = pytest.importorskip("sklearn.metrics")
    rng = np.random.default_rng(0)
    for _ in range(20):
        n = int(rng.integers(2, 400))
        a = rng.integers(0, int(rng.integers(1, 30)), size=n)
        b = rng.integers(0, int(rng.integers(1, 30)), size=n)
        assert q.nmi(a, b) == pytest.approx(metrics.normalized_mutual_info_score(a, b), abs=1e-9)
        assert q.ari(a, b) == pytest.approx(metrics.adjusted_rand_score(a, b), abs=1e-9)
        assert q.ami(a, b) == pytest.approx(
            metrics.adjusted_mutual_info_score(a, b, average_method="max"), abs=1e-9)


def test_modularity_matches_fig1_closed_form():
    # Fig. 1 graph, natural split: f1 = 1/21, f2 = 1/2, Q = 19/42
    assert q.modularity(1 / 21, 1 / 2) == pytest.approx(19 / 42)


def _mi(a, b):
    c = q._contingency(a, b)
    n = c.sum()
    ra, rb = c.sum(1), c.sum(0)
    return sum(c[i, j] / n * np.log(c[i, j] * n / (ra[i] * rb[j]))
               for i in range(c.shape[0]) for j in range(c.shape[1]) if c[i, j] > 0)


@pytest.mark.parametrize("a,b", [([0, 0, 0, 1, 1, 2, 2], [0, 1, 1, 1, 2, 2, 2]),
                                 ([0, 0, 1, 1, 1, 1], [0, 1, 0, 1, 0, 2]),
                                 ([0, 1, 2, 3, 0, 1], [5, 5, 5, 6, 6, 6])])
def test_ami_expectation_by_brute_force(a, b):
    """E[MI] is the mean MI over every relabelling of b's items (all n! orders), so AMI follows
    from the definition of section 5 with no library in the loop."""
    a, b = np.array(a), np.array(b)
    perms = itertools.permutations(range(len(b)))
    emi = float(np.mean([_mi(a, b[list(p)]) for p in perms]))
    c = q._contingency(a, b)
    assert q._expected_mi(c.sum(1), c.sum(0), c.sum()) == pytest.approx(emi, rel=1e-12)
    n = len(a)
    h = lambda x: -sum(k / n * np.log(k / n) for k in np.unique(x, return_counts=True)[1])
    want = (_mi(a, b) - emi) / (max(h(a), h(b)) - emi)
    assert q.ami(a, b) == pytest.approx(want, rel=1e-10)


def test_ami_is_zero_on_average_for_independent_partitions():
    rng = np.random.default_rng(3)
    vals = [q.ami(rng.integers(0, 6, size=60), rng.integers(0, 4, size=60)) for _ in range(300)]
    assert abs(np.mean(vals)) < 0.01
    assert q.ami(np.zeros(9, dtype=int), np.zeros(9, dtype=int)) == 1.0
    assert q.ami(np.arange(9), np.arange(9)[::-1]) == 1.0

