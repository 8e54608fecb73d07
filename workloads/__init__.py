"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module holds no arithmetic of the simulation method: it only draws graphs
and angle vectors.  Both the oracle (``oracle/``) and the GPU path
(``paper_2106_15740_amd``) receive their inputs from here, so that the two
never share code beyond the inputs themselves.

The paper benchmarks on random 3-regular graphs (Results section, the five
seeded random 3-regular graphs) whose edge lists are not published; the
generator below stands in for them.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

Edge = Tuple[int, int]


def random_regular_graph(n: int, d: int, seed: int) -> List[Edge]:
    """Uniform-ish random simple d-regular graph on vertices 0..n-1.

    Configuration (pairing) model with rejection: every vertex gets d stubs,
    the stubs are shuffled and paired; a pairing with a self-loop or a repeated
    edge is rejected and redrawn.  The result is a sorted list of (u, v) with
    u < v.  Deterministic for a given (n, d, seed).
    """
    if n <= d or (n * d) % 2:
        raise ValueError(f"no simple {d}-regular graph on {n} vertices")
    rng = np.random.default_rng(seed)
    stubs = np.repeat(np.arange(n, dtype=np.int64), d)
    for _ in range(10_000):
        perm = rng.permutation(stubs)
        a, b = perm[0::2], perm[1::2]
        if np.any(a == b):
            continue
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        keys = lo * n + hi
        if np.unique(keys).size != keys.size:
            continue
        order = np.lexsort((hi, lo))
        return [(int(lo[i]), int(hi[i])) for i in order]
    raise RuntimeError("pairing model did not produce a simple graph")


def random_angles(p: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """gamma_l, beta_l ~ U(0, pi) for l = 1..p (float64), seeded."""
    rng = np.random.default_rng(seed)
    g = rng.uniform(0.0, np.pi, size=p)
    b = rng.uniform(0.0, np.pi, size=p)
    return g.astype(np.float64), b.astype(np.float64)


def bfs_subgraph(n: int, edges: Sequence[Edge], k: int, root: int = 0) -> Tuple[int, List[Edge]]:
    """First k vertices in BFS order from ``root`` (neighbours visited in
    increasing id), relabelled 0..k-1 in that order, with their induced edges."""
    adj = [[] for _ in range(n)]
    for u, v in edges:
        adj[u].append(v)
        adj[v].append(u)
    for a in adj:
        a.sort()
    seen = {root: 0}
    order = [root]
    dq = deque([root])
    while dq and len(order) < k:
        u = dq.popleft()
        for w in adj[u]:
            if w not in seen and len(order) < k:
                seen[w] = len(order)
                order.append(w)
                dq.append(w)
    sub = sorted(
        (min(seen[u], seen[v]), max(seen[u], seen[v]))
        for u, v in edges
        if u in seen and v in seen
    )
    return len(order), sub


def triangle_counts(n: int, edges: Sequence[Edge]) -> List[int]:
    """Number of triangles through each edge (graph bookkeeping, used by tests
    that evaluate published closed forms)."""
    nb = [set() for _ in range(n)]
    for u, v in edges:
        nb[u].add(v)
        nb[v].add(u)
    return [len(nb[u] & nb[v]) for u, v in edges]


@dataclass
class Workload:
    """One benchmark configuration: graph, depth, angles and run options."""

    name: str
    n: int
    edges: List[Edge]
    p: int
    gamma: np.ndarray
    beta: np.ndarray
    dtype: str            # "c64" or "c128"
    order: str            # "min_degree" or "min_fill"
    notes: str = ""
    extra: dict = field(default_factory=dict)


def workload(name: str, graph_seed: int = 0, param_seed: int = 1) -> Workload:
    """The five configurations the energy path is exercised on.

    ``p1_n10``   QAOA p=1, 3-regular N=10 (15 edges), gamma=0.4, beta=0.3, c128.
    ``p2_n60``   p=2, 3-regular N=60, angles ~ U(0, pi), c64, min-fill.
    ``p3_n244``  p=3, 3-regular N=244 (366 edges), c64, min-fill.
    ``p4_n100``  p=4, 3-regular N=100, c64 forward + adjoint.
    ``p5_n1000`` p=5, 3-regular N=1000 (1500 edges), c64, min-degree.
    """
    table = {
        "p1_n10": (10, 1, "c128", "min_degree"),
        "p2_n60": (60, 2, "c64", "min_fill"),
        "p3_n244": (244, 3, "c64", "min_fill"),
        "p4_n100": (100, 4, "c64", "min_fill"),
        "p5_n1000": (1000, 5, "c64", "min_degree"),
    }
    if name not in table:
        raise KeyError(name)
    n, p, dt, order = table[name]
    edges = random_regular_graph(n, 3, graph_seed)
    if name == "p1_n10":
        g, b = np.array([0.4]), np.array([0.3])
    else:
        g, b = random_angles(p, param_seed + 1000 * p)
    return Workload(name, n, edges, p, g, b, dt, order)
