"""Benchmark of the HP-MOCD hot path on one MI355X.

One step = one whole run of the method (initialisation, T generations of tournament ->
crossover -> mutation -> fitness -> environmental selection, front extraction) on a
synthetic planted-partition graph already resident in HBM, through the production entry
point (hpmocd_run: the generation loop replayed from a hipGraph). The timed region is K such
runs: ms_per_step is their wall time, gens_per_s comes from HIP events around their
generation loops. The reported value is the fitness throughput in edge-evaluations per
second (one undirected edge tested for one individual; one individual evaluation = m
edge-evaluations) over the fitness kernels' own device time, which a second pass of K runs
in the same process measures with HIP events the library records around every fitness
launch (kernels launched one by one); that pass also gives the per-kernel-group breakdown
and the roofline figures.

Prints one JSON line. ``--gpus N`` with N > 1 is refused: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fitness edge-evals/s & gens/s at 1M nodes; batched runs/s + p50/p99 latency"
HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, AMD public specification

WORKLOADS = {
    "planted_partition_1M": ("large_1m", {}),
    "planted_partition_40k_mu0.3": ("mid_40k", {"mu": 0.3}),
    "planted_partition_1k": ("small_1k", {}),
}


def per_individual_bytes(n: int, m2: int) -> int:
    """Algorithmic bytes of one individual evaluation: the CSR (row_ptr, col) and the
    individual's label row, B_ind = 4(n+1) + 4*2m + 4n."""
    return 4 * (n + 1) + 4 * m2 + 4 * n


def population_floor_bytes(n: int, m2: int, pop: int) -> int:
    """Compulsory bytes of evaluating a whole population in one pass: the CSR once and every
    label row once."""
    return 4 * (n + 1) + 4 * m2 + 4 * n * pop


def measured_counter(workload: str, pop: int, key: str = "fitness_step_traffic_bytes"):
    """A figure of the committed rocprofv3 counter summary (HBM bytes of one fitness step, or
    the fitness kernels' L2 hit rate), or None when there is none for this workload or the
    kernels changed since it was taken."""
    import hashlib
    import re
    if workload != "planted_partition_1M" or pop != 100:
        return None
    path = os.path.join(ROOT, "profiles", "traffic_fitness_planted_1M_pop100.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"kernels.hip sha256 prefix when measured: ([0-9a-f]+)", text)
    m_val = re.search(re.escape(key) + r": ([0-9.]+)", text)
    src = open(os.path.join(ROOT, "paper_2506_01752_amd", "csrc", "kernels.hip"), "rb").read()
    if not m_sha or not m_val or hashlib.sha256(src).hexdigest()[:16] != m_sha.group(1):
        return None
    v = m_val.group(1)
    return float(v) if "." in v else int(v)


def measured_traffic(workload: str, pop: int):
    return measured_counter(workload, pop)


def phase_rates(workload: str, pop: int, ms: dict):
    """Per phase of a generation: counter bytes (committed summary, None when stale or
    absent), duration and the physical rate against the HBM peak."""
    gb = {"crossover": measured_counter(workload, pop, "crossover_traffic_GB"),
          "mutation": measured_counter(workload, pop, "mutation_traffic_GB"),
          "fitness step": measured_counter(workload, pop)}
    out = {}
    for k, t in ms.items():
        b = gb.get(k)
        b = int(round(b * 1e9)) if (b is not None and k != "fitness step") else b
        out[k] = {"ms": t, "traffic_bytes": b,
                  "GBps": (b / (t / 1e3) / 1e9) if (b and t > 0) else None,
                  "frac_physical": (b / (t / 1e3) / 1e9 / HBM_PEAK_GBPS) if (b and t > 0) else None}
    return out


def copy_ceiling_gbps(mib: int = 1024, reps: int = 5) -> float:
    """Achievable HBM bandwidth on this device: a plain device-to-device copy of mib MiB
    (bytes read + bytes written per second, best of reps)."""
    import torch
    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = 0.0
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = max(best, 2 * a.numel() / (e0.elapsed_time(e1) / 1e3) / 1e9)
    del a, b
    return best


def cpu_baseline(g, seed: int, target_s: float = 15.0):
    """The oracle's evaluation, single-threaded, on a bounded sample of the same workload: up
    to 100 rows of the initial population, evaluated repeatedly for about target_s seconds."""
    import numpy as np

    import oracle
    oracle.build()
    first = oracle.init_individual(g.row_ptr, g.col, seed, 0)[None, :]
    t0 = time.perf_counter()
    oracle.evaluate_batch(g.row_ptr, g.col, first)         # upper bound of one evaluation
    single = max(time.perf_counter() - t0, 1e-6)
    k = int(min(100, max(1, target_s / (4 * single))))
    labs = np.stack([oracle.init_individual(g.row_ptr, g.col, seed, i) for i in range(k)])
    t0 = time.perf_counter()
    oracle.evaluate_batch(g.row_ptr, g.col, labs)          # calibration pass
    reps = max(1, int(round(target_s / max(time.perf_counter() - t0, 1e-6))))
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.evaluate_batch(g.row_ptr, g.col, labs)
    dt = time.perf_counter() - t0
    return {"value": reps * k * g.m / dt, "unit": "edge-evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} initial-population rows of the same graph evaluated {reps} times "
                      f"({reps * k} individual evaluations), serial C oracle, {dt:.2f} s"}


def host_cpu():
    """The host CPU as the OS reports it: model name (every distinct /proc/cpuinfo entry,
    plus family / model / stepping numbers), logical CPUs, the CPUs this process may run on,
    and the OpenMP thread count the environment grants."""
    info = {"model_names": [], "family_model_stepping": None, "logical_cpus": os.cpu_count(),
            "cpus_available": None, "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}
    try:
        info["cpus_available"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    fam = mod = step = None
    try:
        for line in open("/proc/cpuinfo"):
            key, _, val = line.partition(":")
            key, val = key.strip(), val.strip()
            if key == "model name" and val not in info["model_names"]:
                info["model_names"].append(val)
            elif key == "cpu family" and fam is None:
                fam = val
            elif key == "model" and mod is None:
                mod = val
            elif key == "stepping" and step is None:
                step = val
    except OSError:
        pass
    if fam is not None:
        info["family_model_stepping"] = f"{fam}/{mod}/{step}"
    return info


def cpu_generation(g, kw, threads: int):
    """Context beside cpu_baseline: one whole oracle generation (tournament, crossover,
    mutation, evaluation, selection), as the difference of a one-generation run and a
    zero-generation run, with OpenMP over individuals on `threads` threads."""
    import oracle
    oracle.build()

    def timed(T):
        t0 = time.perf_counter()
        oracle.run(g.row_ptr, g.col, **dict(kw, generations=T), threads=threads)
        return time.perf_counter() - t0
    t0 = timed(0)
    t1 = timed(1)
    return max(t1 - t0, 1e-9)


def bench_batched(args):
    """Batched form: many independent runs (each graph with its own pop-64 population) in one
    batched call vs the same runs one after another; results must be identical."""
    import numpy as np
    import torch

    import paper_2506_01752_amd as hp
    import synth

    t0 = time.perf_counter()
    specs = synth.batch_params(args.batched, seed=0)
    graphs = [synth.batch_graph(p) for p in specs]
    print(f"# {len(graphs)} graphs built in {time.perf_counter() - t0:.1f} s, total n = "
          f"{sum(g.n for g in graphs)}, total m = {sum(g.m for g in graphs)}",
          file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    dgs = [hp.Graph(g.row_ptr, g.col) for g in graphs]
    params = hp.make_params(pop_size=64, generations=args.generations, crossover_p=0.9,
                            mutation_p=0.1, parents_per_child=4, seed=0)
    ws = torch.empty(hp.batch_workspace_size(dgs, params, hp.AUTOTUNE), dtype=torch.uint8,
                     device="cuda")
    # warm-up (also builds the kernels' code objects)
    hp.run_batch(dgs[:2], params, stream=stream, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fronts_b, prof = hp.run_batch(dgs, params, stream=stream, workspace=ws, flags=hp.AUTOTUNE,
                                  profile=True)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    print(f"# batched {t_batch:.3f} s (autotune probes {prof['tune_probe_ms']:.1f} ms)",
          file=sys.stderr, flush=True)
    if args.no_sequential:   # the batched call alone (for a kernel trace of its loop)
        print(json.dumps({"metric": "batched runs/s (pop 64, 100 generations per run)",
                          "value": len(dgs) / t_batch, "unit": "runs/s", "n_gpus": 1,
                          "batched_loop_ms": prof["loop_ms"],
                          "autotune_probe_ms": prof["tune_probe_ms"]}), flush=True)
        return
    single_ws = torch.empty(max(hp.workspace_size(d, params) for d in dgs), dtype=torch.uint8,
                            device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fronts_s = [hp.run(d, params, stream=stream, workspace=single_ws) for d in dgs]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    identical = all(
        np.array_equal(a.labels, b.labels) and np.array_equal(a.A, b.A)
        and np.array_equal(a.S, b.S) and a.selected == b.selected
        for a, b in zip(fronts_b, fronts_s))
    out = {
        "metric": "batched runs/s (pop 64, 100 generations per run)",
        "value": len(dgs) / t_batch, "unit": "runs/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": t_batch * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"batch_{len(dgs)}_planted_partition",
                   "n_total": sum(g.n for g in graphs), "m_total": sum(g.m for g in graphs),
                   "pop_size": 64, "generations": args.generations},
        "sequential_runs_per_s": len(dgs) / t_seq,
        "speedup_vs_sequential": t_seq / t_batch,
        "identical_to_sequential": identical,
        "batched_loop_ms": prof["loop_ms"], "autotune_probe_ms": prof["tune_probe_ms"],
        "tuning": {k: prof[k] for k in prof if k.startswith("tune_") and k != "tune_probe_ms"},
    }
    print(json.dumps(out), flush=True)


def bench_paper_workload(args):
    """End-to-end wall time (graph creation from host CSR, the run, the front back on the host)
    on a synthetic stand-in for the paper's LFR graph of 20,000 nodes, whose runtime the paper
    reports for its own CPU implementation (hardware not stated)."""
    import numpy as np
    import torch

    import paper_2506_01752_amd as hp
    import synth

    g = synth.planted_partition(20000, 20, 50, 0.3, 20, 100, seed=0)
    params = hp.make_params(pop_size=100, generations=100, crossover_p=0.8, mutation_p=0.2,
                            parents_per_child=4, seed=0)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    hp.run(hp.Graph(g.row_ptr, g.col), params, stream=stream)   # warm-up
    walls = []
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        front = hp.run(hp.Graph(g.row_ptr, g.col), params, stream=stream)
        walls.append(time.perf_counter() - t0)
    paper_s = 148.36
    print(json.dumps({
        "metric": "end-to-end seconds per run (paper's LFR 20k setting)",
        "value": float(np.median(walls)), "unit": "s", "n_gpus": 1, "steps": len(walls),
        "higher_is_better": False, "data": "synthetic",
        "config": {"workload": "planted_partition_20k_mu0.3_paper_setting", "n": g.n, "m": g.m,
                   "pop_size": 100, "generations": 100, "crossover_p": 0.8, "mutation_p": 0.2,
                   "parents_per_child": 4},
        "front_size": int(front.labels.shape[0]),
        "paper_runtime_s": paper_s, "paper_hardware": "not stated (CPU, multi-threaded Rust)",
        "ratio_paper_over_this": paper_s / float(np.median(walls)),
    }), flush=True)


def bench_eval(args):
    """hpmocd_eval alone: the objectives of 100 partitions of the |V| = 1M graph handed in by
    the caller, once labelled by node ids (each planted community by one random member) and
    once by community indices 0..k-1, 10% of the nodes of each partition relabelled at random.
    Device time of the evaluation kernels (the library's events), median of 5 after 2."""
    import numpy as np
    import torch

    import paper_2506_01752_amd as hp
    import synth

    g = synth.large_1m()
    rng = np.random.default_rng(0)
    memb = g.membership.astype(np.int64)
    k = int(memb.max()) + 1
    perm = rng.permutation(g.n)
    rep = np.zeros(k, dtype=np.int64)
    rep[memb[perm]] = perm              # one random member per community
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    dg = hp.Graph(g.row_ptr, g.col)
    out = {}
    for name, base, hi in [("node_ids", rep[memb], g.n), ("community_indices", memb, k)]:
        labs = np.empty((100, g.n), dtype=np.int32)
        for i in range(100):
            lab = base.copy()
            flip = rng.random(g.n) < 0.1
            lab[flip] = rng.integers(0, hi, int(flip.sum()))
            labs[i] = lab
        t = torch.from_numpy(labs).cuda()
        ms = [hp.evaluate(dg, t, stream=stream, timing=True)[4] for _ in range(7)][2:]
        med = float(np.median(ms))
        out[name] = {"kernel_ms": med, "edge_evals_per_s": 100 * g.m / (med * 1e-3)}
        print(f"# {name}: {med:.3f} ms", file=sys.stderr, flush=True)
    print(json.dumps({
        "metric": "fitness evaluation of given partitions (hpmocd_eval), edge-evals/s",
        "value": out["community_indices"]["edge_evals_per_s"], "unit": "edge-evals/s",
        "n_gpus": 1, "higher_is_better": True, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "planted_partition_1M", "n": g.n, "m": g.m, "partitions": 100,
                   "communities": k},
        "detail": out}), flush=True)


def bench_quality(args):
    """Not a speed figure: how well the selected solution (Alg. 3) recovers the planted
    communities, against the best partition of the initial population."""
    import numpy as np
    import torch

    import paper_2506_01752_amd as hp
    from paper_2506_01752_amd import quality as q
    import synth

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()

    def one(g, seed):
        dg = hp.Graph(g.row_ptr, g.col)
        init = {}

        def cb(st):
            if st.g == 0:
                init["labels"] = st.labels
        front = hp.run(dg, stream=stream, on_generation=cb,
                       **dict(synth.GA_DEFAULT, seed=seed))
        sel = front.labels[front.selected]
        best0 = max(q.nmi(row, g.membership) for row in init["labels"])
        return {"nmi": q.nmi(sel, g.membership), "ami": q.ami(sel, g.membership),
                "ari": q.ari(sel, g.membership),
                "pair_f1": q.pair_f1(sel, g.membership),
                "q": q.modularity(front.f1[front.selected], front.f2[front.selected]),
                "front_size": int(front.labels.shape[0]),
                "front_best_nmi": max(q.nmi(r, g.membership) for r in front.labels),
                "communities_found": int(len(np.unique(sel))),
                "communities_planted": int(len(np.unique(g.membership))),
                "init_best_nmi": best0}

    out = {"small_1k_mu0.3": [], "mid_40k": {}}
    g1 = synth.small_1k()
    for seed in range(5):
        out["small_1k_mu0.3"].append(one(g1, seed))
        print(f"# 1k seed {seed}: {out['small_1k_mu0.3'][-1]}", file=sys.stderr, flush=True)
    for mu in (0.1, 0.3, 0.5, 0.7):
        g = synth.mid_40k(mu)
        out["mid_40k"][f"mu{mu}"] = dict(one(g, 0), realised_mu=g.info["realised_mu"])
        print(f"# 40k mu {mu}: {out['mid_40k'][f'mu{mu}']}", file=sys.stderr, flush=True)
    nm = [r["nmi"] for r in out["small_1k_mu0.3"]]
    print(json.dumps({"metric": "solution quality (NMI of the selected solution vs planted)",
                      "value": float(np.mean(nm)), "unit": "NMI", "n_gpus": 1,
                      "higher_is_better": True, "data": "synthetic",
                      "config": {"workload": "quality_1k_and_40k_mu_sweep"},
                      "nmi_1k_std_over_seeds": float(np.std(nm)), "detail": out}), flush=True)


def _request_graph(p):
    import synth
    g = synth.batch_graph(p)
    return g.row_ptr, g.col


def bench_served(args):
    """Served form: a Poisson stream of community-detection requests against the
    continuous-batching server, at about 0.5x and 0.9x of its measured capacity, and the
    same streams against the plain FIFO server (one resident request at a time). Every
    request's front must be identical in both."""
    import multiprocessing as mp

    import numpy as np

    import synth

    count = args.served
    specs = synth.request_stream(count, rate=1.0, seed=0)   # arrival times at rate 1
    t0 = time.perf_counter()
    # graphs are built in worker processes before this process touches the device
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        graphs = pool.map(_request_graph, specs, chunksize=4)
    n_tot = sum(len(rp) - 1 for rp, _ in graphs)
    m_tot = sum(len(c) // 2 for _, c in graphs)
    print(f"# {count} request graphs built in {time.perf_counter() - t0:.1f} s: total n = "
          f"{n_tot}, total m = {m_tot}", file=sys.stderr, flush=True)

    import torch

    import paper_2506_01752_amd as hp
    torch.cuda.set_device(0)
    params = hp.make_params(pop_size=100, generations=args.generations, crossover_p=0.9,
                            mutation_p=0.1, parents_per_child=4, seed=0)
    budget = int(args.hbm_budget_gb * (1 << 30))
    unit = np.array([s["arrival"] for s in specs])

    def serve(fifo, rate):
        """rate None: every request at t = 0 (capacity). Returns (fronts, per-request
        latency s, makespan s, stats)."""
        srv = hp.Server(hbm_budget=budget, max_active=args.max_active, fifo=fifo,
                        host_stage_bytes=args.host_stage_mb << 20)
        t_create = time.monotonic()
        arrivals = np.zeros(count) if rate is None else unit / rate
        tickets = [None] * count
        start = time.monotonic() + 0.05
        nthreads = 4

        def submitter(k):
            for i in range(k, count, nthreads):
                delay = start + arrivals[i] - time.monotonic()
                if delay > 0:
                    time.sleep(delay)
                rp, col = graphs[i]
                tickets[i] = srv.submit(rp, col, params)[0]

        import threading
        th = [threading.Thread(target=submitter, args=(k,)) for k in range(nthreads)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        fronts, lat, done = [], np.zeros(count), np.zeros(count)
        base = start - t_create  # arrival i at server-clock time base + arrivals[i]
        for i in range(count):
            f, info = srv.wait(tickets[i])
            fronts.append(f)
            done[i] = info["done_s"]
            lat[i] = info["done_s"] - (base + arrivals[i])
        st = srv.stats()
        srv.close()
        return fronts, lat, float(done.max() - base), st

    def summary(lat, makespan, st):
        return {"runs_per_s": count / makespan, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "makespan_s": makespan,
                "peak_active": st["peak_active"], "peak_gb": st["peak_bytes"] / 2**30,
                "steps": st["steps"]}

    # warm-up: code objects, first allocations
    srv = hp.Server(hbm_budget=1 << 30, max_active=4)
    rp, col = graphs[0]
    srv.wait(srv.submit(rp, col, hp.make_params(pop_size=100, generations=2))[0])
    srv.close()

    out = {}
    ref_fronts, lat, mk, st = serve(False, None)
    cap = count / mk
    out["capacity"] = summary(lat, mk, st)
    print(f"# capacity (all at t=0): {cap:.2f} runs/s", file=sys.stderr, flush=True)
    if args.served_capacity_only:   # one pass (for a kernel trace of the served loop)
        print(json.dumps({"metric": "served capacity runs/s", "value": cap, "unit": "runs/s",
                          "n_gpus": 1, "detail": out}), flush=True)
        return
    _, lat, mk, st = serve(True, None)
    out["fifo_capacity"] = summary(lat, mk, st)
    print(f"# FIFO capacity: {count / mk:.2f} runs/s", file=sys.stderr, flush=True)
    identical = True
    for frac in (0.5, 0.9):
        rate = frac * cap
        for fifo in (False, True):
            fr, lat, mk, st = serve(fifo, rate)
            key = f"{'fifo' if fifo else 'served'}_{frac}x"
            out[key] = dict(summary(lat, mk, st), arrival_rate=rate)
            identical = identical and all(
                np.array_equal(a.labels, b.labels) and np.array_equal(a.A, b.A)
                and np.array_equal(a.S, b.S) and a.selected == b.selected
                for a, b in zip(fr, ref_fronts))
            print(f"# {key}: {out[key]}", file=sys.stderr, flush=True)
    # a few requests against the plain single-run entry point
    stream = torch.cuda.Stream()
    for i in range(0, count, max(1, count // 4)):
        rp, col = graphs[i]
        f = hp.run(hp.Graph(rp, col), params, stream=stream)
        identical = identical and np.array_equal(f.labels, ref_fronts[i].labels) and \
            np.array_equal(f.A, ref_fronts[i].A) and np.array_equal(f.S, ref_fronts[i].S)
    s9 = out["served_0.9x"]
    line = {
        "metric": "served runs/s + p50/p99 latency (pop 100, 100 generations per request)",
        "value": s9["runs_per_s"], "unit": "runs/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": s9["makespan_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"served_{count}_poisson_planted_partition", "n_total": n_tot,
                   "m_total": m_tot, "pop_size": 100, "generations": args.generations,
                   "max_active": args.max_active, "hbm_budget_gb": args.hbm_budget_gb},
        "p50_ms": s9["p50_ms"], "p99_ms": s9["p99_ms"],
        "identical_to_alone": bool(identical),
        "detail": out,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="planted_partition_1M", choices=sorted(WORKLOADS))
    ap.add_argument("--generations", type=int, default=100)
    ap.add_argument("--pop", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched", type=int, default=0, metavar="COUNT",
                    help="batched form instead: COUNT planted-partition graphs (|V| log-uniform "
                         "in [500, 50000]), pop 64, in one batched run vs COUNT sequential runs")
    ap.add_argument("--served", type=int, default=0, metavar="COUNT",
                    help="served form instead: COUNT requests (|V| log-uniform in [1000, 200000], "
                         "pop 100, 100 generations) arriving as a Poisson stream, continuous "
                         "batching vs plain FIFO")
    ap.add_argument("--quality", action="store_true",
                    help="solution-quality sanity instead: agreement of the selected solution "
                         "with the planted partition at |V| = 1,000 (5 seeds) and |V| = 40,000 "
                         "(mu sweep)")
    ap.add_argument("--paper-workload", action="store_true",
                    help="the paper's LFR setting (n 20,000, mean degree 20, max 50, communities "
                         "20-100, mu 0.3; pop 100, 100 generations, C_P 0.8, M_P 0.2, E_S 4) end "
                         "to end, next to the paper's reported runtime")
    ap.add_argument("--no-sequential", action="store_true",
                    help="with --batched: time the batched call only (no sequential baseline)")
    ap.add_argument("--served-capacity-only", action="store_true",
                    help="with --served: run the capacity pass only (all requests at t = 0)")
    ap.add_argument("--eval", action="store_true",
                    help="fitness evaluation alone instead: 100 given partitions of the 1M "
                         "graph, labelled by node ids and by community indices")
    ap.add_argument("--max-active", type=int, default=64)
    ap.add_argument("--hbm-budget-gb", type=float, default=200.0)
    ap.add_argument("--host-stage-mb", type=int, default=0,
                    help="with --served: page-locked host staging per in-flight step (0: the "
                         "library default)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (calibrates "
                         "the memory-traffic counters) and exit")
    args = ap.parse_args()
    if args.copy_probe_mib:
        import torch
        a = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel()}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.batched:
        return bench_batched(args)
    if args.served:
        return bench_served(args)
    if args.quality:
        return bench_quality(args)
    if args.paper_workload:
        return bench_paper_workload(args)
    if args.eval:
        return bench_eval(args)

    import torch

    import paper_2506_01752_amd as hp
    import synth

    maker, extra = WORKLOADS[args.workload]
    g = getattr(synth, maker)(**extra)
    kw = dict(synth.GA_DEFAULT, pop_size=args.pop, generations=args.generations)
    params = hp.make_params(**kw)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    dg = hp.Graph(g.row_ptr, g.col)
    ws = torch.empty(hp.workspace_size(dg, params), dtype=torch.uint8, device="cuda")
    print(f"# workload {args.workload}: n={g.n} m={g.m} pop={args.pop} T={args.generations}",
          file=sys.stderr, flush=True)

    # the production path: hpmocd_run with its generation loop replayed from a hipGraph
    for _ in range(args.warmup):
        hp.run(dg, params, stream=stream, workspace=ws, profile=True)
    torch.cuda.synchronize()
    loops = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, prof = hp.run(dg, params, stream=stream, workspace=ws, profile=True)
        loops.append(prof["loop_ms"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"# timed {args.steps} hipGraph-replayed runs in {wall:.3f} s", file=sys.stderr,
          flush=True)

    # the kernel-timing pass: the same runs with events around every kernel group
    hp.run(dg, params, stream=stream, workspace=ws, flags=hp.TIME_KERNELS, profile=True)
    torch.cuda.synchronize()
    profs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, prof = hp.run(dg, params, stream=stream, workspace=ws, flags=hp.TIME_KERNELS,
                         profile=True)
        profs.append(prof)
    torch.cuda.synchronize()
    wall_k = time.perf_counter() - t0
    print(f"# kernel-timing pass: {args.steps} runs in {wall_k:.3f} s", file=sys.stderr,
          flush=True)

    T, pop = args.generations, args.pop
    launches = sum(p["fitness_launches"] for p in profs)
    fit_ms = sum(p["fitness_ms"] for p in profs)
    sweep_ms = sum(p["sweep_ms"] for p in profs)
    loop_ms = sum(p["loop_ms"] for p in profs)
    evals = sum(p["individual_evals"] for p in profs)
    edge_evals = evals * g.m
    value = edge_evals / ((fit_ms + sweep_ms) / 1e3)
    eval_ms = (fit_ms + sweep_ms) / launches      # one whole-population evaluation
    bytes_launch = pop * per_individual_bytes(g.n, 2 * g.m)
    floor_launch = population_floor_bytes(g.n, 2 * g.m, pop)
    achieved = bytes_launch / (eval_ms / 1e3) / 1e9
    traffic = measured_traffic(args.workload, pop)
    copy_gbps = copy_ceiling_gbps()
    var_gen = sum(p["variation_ms"] for p in profs) / max(1, T * args.steps)
    xo_gen = sum(p["crossover_ms"] for p in profs) / max(1, T * args.steps)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "edge-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "m": g.m,
                   "mean_deg": g.info.get("mean_deg"), "mu": g.info.get("mu"),
                   "max_deg": g.info.get("realised_max_deg"), "pop_size": pop,
                   "generations": T, "crossover_p": kw["crossover_p"],
                   "mutation_p": kw["mutation_p"], "parents_per_child": kw["parents_per_child"],
                   "seed": kw["seed"], "graph_seed": 0},
        "gens_per_s": T * args.steps / (sum(loops) / 1e3) if T else None,
        "timed_path": "hpmocd_run, generation loop replayed from a hipGraph (production)",
        "kernel_timing_pass": {
            "what": "the same runs launched kernel by kernel with HIP events around every "
                    "kernel group (HPMOCD_TIME_KERNELS): value, the breakdown below, roofline",
            "ms_per_step": wall_k * 1e3 / args.steps,
            "gens_per_s": T * args.steps / (loop_ms / 1e3) if T else None},
        "end_to_end_edge_evals_per_s": edge_evals / wall if wall > 0 else None,
        "fitness_ms_per_population": eval_ms,
        "histogram_clear_ms_per_population": sweep_ms / launches,
        "variation_ms_per_gen": var_gen,
        "crossover_ms_per_gen": xo_gen,
        "mutation_ms_per_gen": var_gen - xo_gen,
        "select_ms_per_gen": sum(p["select_ms"] for p in profs) / max(1, T * args.steps),
        # the other phases of a generation against the same committed counter summary: HBM
        # bytes the counters saw each phase move, over its kernel-timing-pass duration
        "generation_phases": phase_rates(args.workload, pop, {
            "crossover": xo_gen, "mutation": var_gen - xo_gen, "fitness step": eval_ms}),
        "population_floor_GBps": population_floor_bytes(g.n, 2 * g.m, pop) / (eval_ms / 1e3) / 1e9,
        "roofline": {"bound": "hbm", "kernel": "fitness step (k_bin, then k_fitness beside k_hist)",
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic,
                     "bytes_per_launch": bytes_launch, "ms_per_launch": eval_ms,
                     # the same duration against the bytes the counters saw move (L2 misses
                     # to the memory fabric) and against the compulsory bytes of one
                     # population pass (CSR once + every label row once)
                     "frac_physical": (traffic / (eval_ms / 1e3) / 1e9 / HBM_PEAK_GBPS
                                       if traffic else None),
                     "floor_bytes_per_launch": floor_launch,
                     "frac_floor": floor_launch / (eval_ms / 1e3) / 1e9 / HBM_PEAK_GBPS,
                     "l2_hit_rate": measured_counter(args.workload, pop, "fitness_l2_hit_rate"),
                     "copy_ceiling_GBps": copy_gbps, "frac_of_copy": achieved / copy_gbps},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, kw["seed"])
        host = host_cpu()
        avail = host["cpus_available"] or host["logical_cpus"] or 1
        # OpenMP threads: the environment's grant (a one-GPU job's share of the host), else
        # every CPU this process may run on
        threads = int(host["omp_num_threads_env"] or avail)
        threads = max(1, min(threads, avail))
        out["cpu_oracle_generation"] = {
            "seconds_per_generation": cpu_generation(g, kw, threads), "threads": threads,
            "seconds_per_generation_1_thread": cpu_generation(g, kw, 1),
            "threads_reason": "OMP_NUM_THREADS of the environment (the host share granted to a "
                              "one-GPU job), capped by the CPUs this process may use",
            "host": host, "kind": "oracle"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
