"""Structure recovery on the 20-node binary workload (Sec. VI): the sampler's
best graph scores at least as well as the generating graph, and priors on the
edges it got wrong reduce its mistakes."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1210_5128_amd import accuracy as A
from paper_1210_5128_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bnos():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_5128_amd import bnos as b
    return b


def test_best_graph_beats_the_generating_graph_and_priors_fix_mistakes(bnos):
    w = datagen.WORKLOADS["roc20"]
    net, _ = datagen.make(w)
    n = w.n
    true = net.true_parent_masks()
    t = bnos.build_score_table(net.data, net.arities, w.K)
    g, s = A.learn_best_graph(t, 2000, 16, seed=5)
    t.free()
    true_score = sum(oracle.local_score(net.data, net.arities, i, int(true[i])) for i in range(n))
    learned_score = sum(oracle.local_score(net.data, net.arities, i, int(g[i])) for i in range(n))
    assert abs(s - learned_score) <= 1e-5 * abs(learned_score)
    assert learned_score >= true_score - 1e-9 * abs(true_score)
    r0 = A.edge_rates(g, true, n)
    R = A.injected_prior(true, g, n, 0.8, 0.1, 1.0, seed=1)
    tp = bnos.build_score_table(net.data, net.arities, w.K, prior=R, prior_mode=1)
    g2, _ = A.learn_best_graph(tp, 2000, 16, seed=5)
    tp.free()
    r2 = A.edge_rates(g2, true, n)
    # the priors recover missed edges; the edges around them may re-orient, so
    # only the total number of mistakes has to fall (measured: TPR 0.667 -> 0.833,
    # mistakes 12 -> 8)
    assert r2.tpr > r0.tpr
    assert r2.fn + r2.fp < r0.fn + r0.fp
