"""GPU path vs the oracle at the benchmark's full sizes, through stored per-generation oracle
digests (tests/golden/digests_*.json, written by tests/golden/make_goldens.py from the oracle
alone):

* |V| = 1,000 and |V| = 40,000 (mu 0.1, 0.3, 0.5, 0.7), pop 100, 100 generations: labels,
  objectives, ranks and crowding of every generation;
* |V| = 1,000,000, pop 100, 100 generations: objectives, ranks and crowding of every
  generation, and the final front in full (labels included), both from a traced run and from
  the plain hipGraph-replayed run that bench.py times.
"""
import json
import os
import sys

import pytest

import synth
from tests.digest import front_digest, state_digest

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def load(w):
    path = os.path.join(HERE, "golden", f"digests_{w}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return json.load(open(path))


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


def check(hp, g, gold, with_labels):
    import torch
    stream = torch.cuda.Stream()
    dg = hp.Graph(g.row_ptr, g.col)
    got = []

    def cb(st):
        got.append(state_digest(st.labels, st.A, st.S, st.f1, st.f2, st.rank, st.crowd,
                                with_labels=with_labels))

    flags = 0 if with_labels else hp.TRACE_NO_LABELS
    fr = hp.run(dg, stream=stream, flags=flags, on_generation=cb, **synth.GA_DEFAULT)
    want = gold["generations"]
    assert len(got) == len(want)
    for gen, (a, b) in enumerate(zip(got, want)):
        assert a == b, f"first mismatch at generation {gen}"
    fd = front_digest(fr.labels, fr.A, fr.S, fr.f1, fr.f2, fr.selected)
    assert fd == gold["front"]["digest"]
    # the plain run (generation loop replayed from a hipGraph) gives the same front
    fr2 = hp.run(dg, stream=stream, **synth.GA_DEFAULT)
    assert front_digest(fr2.labels, fr2.A, fr2.S, fr2.f1, fr2.f2, fr2.selected) == fd


def test_small_1k_every_generation(hp):
    gold = load("small_1k")["mu0.3"]
    say("small_1k full run")
    check(hp, synth.small_1k(), gold, True)


@pytest.mark.parametrize("mu", [0.1, 0.3, 0.5, 0.7])
def test_mid_40k_every_generation(hp, mu):
    gold = load("mid_40k")[f"mu{mu}"]
    say(f"mid_40k mu={mu} full run")
    check(hp, synth.mid_40k(mu), gold, True)


def test_large_1m_every_generation(hp):
    gold = load("large_1m")["mu0.4"]
    say("large_1m full run")
    g = synth.large_1m()
    assert g.m == gold["graph"]["m"]
    check(hp, g, gold, False)
