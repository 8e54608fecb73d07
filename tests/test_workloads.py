"""Seeded synthetic inputs: deterministic, simple, d-regular."""
import numpy as np
import pytest

from workloads import random_angles, random_regular_graph, workload


@pytest.mark.parametrize("n,seed", [(10, 0), (60, 1), (244, 0), (1000, 0)])
def test_random_regular_graph(n, seed):
    e1 = random_regular_graph(n, 3, seed)
    assert e1 == random_regular_graph(n, 3, seed)
    assert len(e1) == 3 * n // 2
    assert len(set(e1)) == len(e1)
    deg = np.zeros(n, int)
    for u, v in e1:
        assert 0 <= u < v < n
        deg[u] += 1
        deg[v] += 1
    assert np.all(deg == 3)


def test_angles_and_workloads():
    g, b = random_angles(3, 7)
    assert g.shape == b.shape == (3,)
    assert np.all((0 <= g) & (g <= np.pi)) and np.all((0 <= b) & (b <= np.pi))
    w = workload("p3_n244")
    assert w.p == 3 and len(w.edges) == 366 and w.dtype == "c64"
    w1 = workload("p1_n10")
    assert list(w1.gamma) == [0.4] and list(w1.beta) == [0.3] and len(w1.edges) == 15
