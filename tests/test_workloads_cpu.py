"""The seeded input generators (no model arithmetic): the directed
scale-free graph of the parameter-recovery study and its workload."""
import numpy as np

from paper_2604_01342_amd import workloads as W


def test_scale_free_digraph_structure():
    rng = np.random.default_rng(5)
    M = 2000
    e = W.scale_free_digraph(rng, M)
    assert e.ndim == 2 and e.shape[1] == 2
    assert e.min() >= 0 and e.max() < M
    assert np.all(e[:, 0] != e[:, 1])                       # no self-loops
    assert len({(int(v), int(w)) for v, w in e}) == e.shape[0]  # distinct edges
    # every node joins with an edge; a step adds a node with probability
    # a + c = 0.46, so about 2.2 edges per node (fewer after merging repeats)
    assert 1.5 * M < e.shape[0] < 2.3 * M
    indeg = np.bincount(e[:, 1], minlength=M)
    outdeg = np.bincount(e[:, 0], minlength=M)
    assert np.all(indeg + outdeg > 0)
    # preferential attachment on in-degree: a heavy tail far above the median
    assert indeg.max() > 20 * max(1.0, float(np.median(indeg)))


def test_recovery_workload():
    w = W.make_recovery(20, 5000)
    assert w.n == 5000 and w.M == 20 and w.T == w.t[-1]
    assert np.all(np.diff(w.t) >= 0) and w.m.min() >= 0 and w.m.max() < 20
    assert np.all(np.diag(w.alpha) > 0)                     # self-excitation
    rho = max(abs(np.linalg.eigvals(w.alpha.astype(np.float64))))
    assert abs(rho - 0.5) < 1e-4
    assert np.allclose(w.mu, 0.001) and w.beta[0] == 1.0
