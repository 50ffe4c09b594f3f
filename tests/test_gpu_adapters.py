"""detect() on a networkx graph runs the same device path as Graph + run on its CSR."""
import networkx as nx
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_01752_amd as m
    m.lib()
    return m


def test_detect_networkx_equals_csr_run(hp):
    import torch
    from paper_2506_01752_amd import adapters as ad
    G = nx.relabel_nodes(nx.karate_club_graph(), {i: f"m{i}" for i in range(34)})
    s = torch.cuda.Stream()
    front, coms, conv = ad.detect(G, stream=s, pop_size=40, generations=30, seed=7)
    ref = hp.run(hp.Graph(conv.row_ptr, conv.col), stream=s, pop_size=40, generations=30, seed=7)
    assert np.array_equal(front.labels, ref.labels) and front.selected == ref.selected
    assert sorted(set().union(*coms)) == sorted(G.nodes())
    assert sum(len(c) for c in coms) == 34
    print("communities:", [len(c) for c in coms], flush=True)
