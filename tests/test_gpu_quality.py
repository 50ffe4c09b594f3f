"""Solution-quality sanity (not parity): the selected solution of a run recovers most of the
planted communities, better than the best initial partition, and less so as the mixing
parameter grows. Values are deterministic (fixed seeds); the bounds leave a margin."""
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


def selected_nmi(hp, g, seed=0, with_init=False):
    import torch
    from paper_2506_01752_amd import quality as q
    init = {}

    def cb(st):
        if st.g == 0:
            init["labels"] = st.labels
    front = hp.run(hp.Graph(g.row_ptr, g.col), stream=torch.cuda.Stream(),
                   on_generation=cb if with_init else None, **dict(synth.GA_DEFAULT, seed=seed))
    nmi = q.nmi(front.labels[front.selected], g.membership)
    best0 = max(q.nmi(r, g.membership) for r in init["labels"]) if with_init else None
    return nmi, best0


def test_quality_1k_beats_initial_population(hp):
    g = synth.small_1k()
    nmi, best0 = selected_nmi(hp, g, with_init=True)
    print(f"1k mu 0.3: selected NMI {nmi:.3f}, best initial {best0:.3f}", flush=True)
    assert nmi >= 0.7
    assert nmi > best0 + 0.1


def test_quality_40k_mu_sweep(hp):
    res = {}
    for mu in (0.1, 0.7):
        res[mu], _ = selected_nmi(hp, synth.mid_40k(mu))
        print(f"40k mu {mu}: selected NMI {res[mu]:.3f}", flush=True)
    assert res[0.1] >= 0.9
    assert res[0.7] < res[0.1]
