"""Served form (continuous batching): every request's front equals its plain single-run front
bit for bit, whatever shares the device with it (requests of different sizes, populations,
generation counts and arrival times), under slot and device-byte limits, in FIFO mode, and
with cancellations."""
import threading
import time

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


def mixed_requests(count, seed, nmax=8000):
    rng = np.random.default_rng(seed)
    reqs = []
    for i, p in enumerate(synth.batch_params(count, seed=seed)):
        g = synth.batch_graph(dict(p, n=min(p["n"], nmax)))
        reqs.append((g, dict(pop_size=int(rng.choice([8, 33, 64, 100])),
                             generations=int(rng.integers(0, 14)),
                             crossover_p=float(rng.choice([0.8, 0.9, 1.0])),
                             mutation_p=float(rng.choice([0.1, 0.3])),
                             parents_per_child=4, seed=int(rng.integers(0, 2**40)))))
    return reqs


def alone(hp, g, kw, stream):
    return hp.run(hp.Graph(g.row_ptr, g.col), stream=stream, **kw)


@pytest.mark.parametrize("stage", [0, 300_000, 1])
def test_server_mix_equals_alone(hp, stage):
    """stage: page-locked host staging per in-flight step (0: the default, ample; 300 KB:
    small graphs and fronts staged, larger ones copied from and to pageable memory; 1: none,
    every copy pageable and every front extracted when its step completes)."""
    import torch
    reqs = mixed_requests(14, seed=4) + [(synth.fig1_graph(), dict(pop_size=16, generations=5,
                                                                    seed=3)),
                                         (synth.star(50), dict(pop_size=20, generations=7,
                                                               seed=2))]
    print(f"{len(reqs)} requests, n = {[g.n for g, _ in reqs]}", flush=True)
    srv = hp.Server(hbm_budget=2 << 30, max_active=64, host_stage_bytes=stage)
    tickets = []
    rng = np.random.default_rng(0)
    for g, kw in reqs:  # staggered arrivals: requests join runs already in progress
        tickets.append(srv.submit(g.row_ptr, g.col, **kw)[0])
        time.sleep(float(rng.uniform(0, 0.004)))
    results = [srv.wait(t, timeout=120) for t in tickets]
    st = srv.stats()
    srv.close()
    print("stats", st, "mix", [r[1]["max_mix"] for r in results], flush=True)
    assert st["completed"] == len(reqs) and st["cancelled"] == 0
    assert max(r[1]["max_mix"] for r in results) > 1  # the requests did share the device
    s = torch.cuda.Stream()
    for i, ((g, kw), (front, info)) in enumerate(zip(reqs, results)):
        assert same(front, alone(hp, g, kw, s)), f"request {i}: served front differs from alone"
        assert info["submit_s"] <= info["admit_s"] <= info["done_s"]
        assert info["steps"] == max(kw["generations"], 1)  # init shares a step with gen 1
    for i in (0, 5, len(reqs) - 1):
        g, kw = reqs[i]
        ref = oracle.run(g.row_ptr, g.col, threads=4, **kw)
        assert same(results[i][0], ref), i


def test_server_budget_and_slots(hp):
    import torch
    reqs = mixed_requests(8, seed=7, nmax=20000)
    srv0 = hp.Server(hbm_budget=1 << 30, max_active=4)
    sizes = []
    for g, kw in reqs[:1]:
        t, b = srv0.submit(g.row_ptr, g.col, **kw)
        sizes.append(b)
        srv0.wait(t)
    srv0.close()
    # budget: about two typical requests at a time; at most three slots
    budget = int(2.2 * max(1, sizes[0]))
    srv = hp.Server(hbm_budget=budget, max_active=3)
    tickets, nbytes = [], []
    for g, kw in reqs:
        try:
            t, b = srv.submit(g.row_ptr, g.col, **kw)
        except hp.HpmocdError as e:
            assert e.status == hp.ERR_BUDGET
            continue
        tickets.append((t, g, kw))
        nbytes.append(b)
    res = [(srv.wait(t, timeout=120), g, kw) for t, g, kw in tickets]
    st = srv.stats()
    srv.close()
    print("budget", budget, "bytes", nbytes, "stats", st, flush=True)
    assert st["peak_bytes"] <= budget
    assert st["peak_active"] <= 3
    s = torch.cuda.Stream()
    for (front, info), g, kw in res:
        assert info["max_mix"] <= 3
        assert same(front, alone(hp, g, kw, s))


def test_server_fifo_mode_one_at_a_time(hp):
    reqs = mixed_requests(5, seed=9)
    srv = hp.Server(hbm_budget=1 << 30, max_active=16, fifo=True)
    tickets = [srv.submit(g.row_ptr, g.col, **kw)[0] for g, kw in reqs]
    res = [srv.wait(t, timeout=120) for t in tickets]
    srv.close()
    import torch
    s = torch.cuda.Stream()
    for (front, info), (g, kw) in zip(res, reqs):
        assert info["max_mix"] == 1
        assert same(front, alone(hp, g, kw, s))
    # arrival order is completion order in FIFO mode
    done = [info["done_s"] for _, info in res]
    assert done == sorted(done)


def test_server_threads_cancel_and_errors(hp):
    import torch
    reqs = mixed_requests(10, seed=11)
    for i, (g, kw) in enumerate(reqs):
        # the two requests cancelled below cannot finish first
        kw["generations"] = 10**6 if i in (0, 9) else 12
    srv = hp.Server(hbm_budget=1 << 30, max_active=4)
    tickets = [None] * len(reqs)

    def submit(i):
        g, kw = reqs[i]
        tickets[i] = srv.submit(g.row_ptr, g.col, **kw)[0]

    th = [threading.Thread(target=submit, args=(i,)) for i in range(len(reqs))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    srv.cancel(tickets[9])
    srv.cancel(tickets[0])
    # parameter and graph errors come back from submit, before anything is queued
    g0 = reqs[0][0]
    with pytest.raises(hp.HpmocdError):
        srv.submit(g0.row_ptr, g0.col, parents_per_child=3)  # server-wide E_S is 4
    with pytest.raises(hp.HpmocdError):
        srv.submit(np.array([0, 1, 1]), np.array([1]))  # asymmetric
    with pytest.raises(hp.HpmocdError):
        srv.submit(g0.row_ptr, g0.col, pop_size=513)  # above the largest population
    s = torch.cuda.Stream()
    for i, t in enumerate(tickets):
        if i in (0, 9):
            with pytest.raises(hp.HpmocdError) as e:
                srv.wait(t, timeout=120)
            assert e.value.status == hp.ERR_CANCELLED
            continue
        front, _ = srv.wait(t, timeout=120)
        g, kw = reqs[i]
        assert same(front, alone(hp, g, kw, s)), i
    st = srv.stats()
    srv.close()
    assert st["cancelled"] == 2


def test_server_budget_rejection_and_timeout(hp):
    g = synth.small_1k()
    srv = hp.Server(hbm_budget=1 << 20, max_active=2)  # 1 MiB: a 1k-node pop-100 run is larger
    with pytest.raises(hp.HpmocdError) as e:
        srv.submit(g.row_ptr, g.col, pop_size=100, generations=5)
    assert e.value.status == hp.ERR_BUDGET
    t, b = srv.submit(synth.fig1_graph().row_ptr, synth.fig1_graph().col, pop_size=8,
                      generations=10**6)
    with pytest.raises(hp.HpmocdError) as e:
        srv.wait(t, timeout=0.001)
    assert e.value.status == hp.ERR_TIMEOUT
    srv.cancel(t)
    with pytest.raises(hp.HpmocdError) as e:
        srv.wait(t, timeout=120)
    assert e.value.status == hp.ERR_CANCELLED
    srv.close()


def test_server_many_small_requests_wide_tables(hp):
    """300 tiny requests with up to 512 resident (item tables of hundreds of entries, requests
    finishing in almost every step); each front equals its run alone."""
    import torch
    rng = np.random.default_rng(12)
    reqs = []
    for i in range(300):
        g = synth.gnp(int(rng.integers(5, 60)), 0.15, 1000 + i)
        if g.m == 0:
            continue
        reqs.append((g, dict(pop_size=int(rng.integers(1, 40)), generations=int(rng.integers(0, 9)),
                             seed=int(rng.integers(0, 2**32)))))
    srv = hp.Server(hbm_budget=1 << 30, max_active=512)
    tickets = [srv.submit(g.row_ptr, g.col, **kw)[0] for g, kw in reqs]
    res = [srv.wait(t, timeout=120) for t in tickets]
    st = srv.stats()
    srv.close()
    print("stats", st, flush=True)
    assert st["completed"] == len(reqs) and st["peak_active"] > 64
    s = torch.cuda.Stream()
    for i in range(0, len(reqs), 7):
        g, kw = reqs[i]
        assert same(res[i][0], alone(hp, g, kw, s)), i


def test_server_two_waiters_on_one_ticket(hp):
    """Two threads wait on one ticket: one receives the front, the other ERR_ARG (the ticket
    was consumed), and so does any later call with it."""
    import torch
    g = synth.small_1k()
    kw = dict(pop_size=32, generations=6, seed=5)
    srv = hp.Server(hbm_budget=1 << 30, max_active=4)
    t, _ = srv.submit(g.row_ptr, g.col, **kw)
    got = [None, None]

    def waiter(i):
        try:
            got[i] = ("front", srv.wait(t, timeout=120)[0])
        except hp.HpmocdError as e:
            got[i] = ("error", e.status)

    th = [threading.Thread(target=waiter, args=(i,)) for i in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    kinds = sorted(k for k, _ in got)
    assert kinds == ["error", "front"], got
    err = [v for k, v in got if k == "error"][0]
    front = [v for k, v in got if k == "front"][0]
    assert err == hp.ERR_ARG
    with pytest.raises(hp.HpmocdError) as e:
        srv.poll(t)
    assert e.value.status == hp.ERR_ARG
    srv.close()
    assert same(front, alone(hp, g, kw, torch.cuda.Stream()))
