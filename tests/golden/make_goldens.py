"""Writes the per-generation oracle digests of the full-size workloads (calls only the oracle
and the input generator). Run from the repository root:

    python tests/golden/make_goldens.py [small_1k|mid_40k|large_1m ...] [--threads N]

Outputs tests/golden/digests_<workload>.json. The |V| = 1,000,000 run hashes objectives only
(labels of 100 million cells per generation are left out) plus the final front in full.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from tests.digest import front_digest, state_digest  # noqa: E402

WORKLOADS = {
    "small_1k": [("mu0.3", lambda: synth.small_1k(), True)],
    "mid_40k": [(f"mu{mu}", (lambda mu=mu: synth.mid_40k(mu)), True) for mu in (0.1, 0.3, 0.5, 0.7)],
    "large_1m": [("mu0.4", lambda: synth.large_1m(), False)],
}


def run_one(g, with_labels, threads):
    digests = []

    def cb(st):
        digests.append(state_digest(st.labels, st.A, st.S, st.f1, st.f2, st.rank, st.crowd,
                                    with_labels=with_labels))
        print(f"  g={st.g} {digests[-1]}", flush=True)

    fr = oracle.run(g.row_ptr, g.col, threads=threads, on_generation=cb,
                    copy_labels=with_labels, **synth.GA_DEFAULT)
    return {"graph": g.info, "ga": synth.GA_DEFAULT, "with_labels": with_labels,
            "generations": digests,
            "front": {"k": int(len(fr.A)), "selected": int(fr.selected),
                      "digest": front_digest(fr.labels, fr.A, fr.S, fr.f1, fr.f2, fr.selected),
                      "A": [int(x) for x in fr.A], "S": [int(x) for x in fr.S]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="*", default=list(WORKLOADS))
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    for w in args.workloads:
        out = {}
        for tag, make, with_labels in WORKLOADS[w]:
            t = time.time()
            g = make()
            print(f"{w} {tag}: n={g.n} m={g.m}", flush=True)
            out[tag] = run_one(g, with_labels, args.threads)
            print(f"{w} {tag}: {time.time() - t:.1f} s", flush=True)
        path = os.path.join(ROOT, "tests", "golden", f"digests_{w}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print("wrote", path)


if __name__ == "__main__":
    main()
