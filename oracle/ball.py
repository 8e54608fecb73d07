"""Per-edge state-vector oracle on the radius-p ball (test infrastructure only).

The energy is a sum of two-qubit terms, and every gate outside the backward
light cone of Z_j Z_k cancels against its conjugate (Section II, the
light-cone remark attributed to Farhi et al.).  At depth p only qubits within
graph distance p of {j, k} take part, and only the ZZ gates of edges with an
endpoint within distance p-1.  The depth-p circuit on that subgraph therefore
gives the exact <Z_j Z_k> of the full graph, with as many qubits as the ball
holds.  This is checked against the full state vector in the tests.
"""
from __future__ import annotations

from collections import deque
from typing import Sequence, Tuple

import numpy as np

from . import statevector as sv

Edge = Tuple[int, int]


def ball(n: int, edges: Sequence[Edge], p: int, j: int, k: int):
    """Vertices at distance <= p from {j, k} (relabelled 0..m-1, j -> 0,
    k -> 1) and the edges with an endpoint at distance <= p-1."""
    adj = [[] for _ in range(n)]
    for u, w in edges:
        adj[u].append(w)
        adj[w].append(u)
    dist = {j: 0, k: 0}
    dq = deque([j, k])
    while dq:
        u = dq.popleft()
        if dist[u] == p:
            continue
        for w in adj[u]:
            if w not in dist:
                dist[w] = dist[u] + 1
                dq.append(w)
    verts = [j, k] + sorted(v for v in dist if v not in (j, k))
    lab = {v: i for i, v in enumerate(verts)}
    sub = [(lab[u], lab[w]) for u, w in edges
           if u in dist and w in dist and min(dist[u], dist[w]) <= p - 1]
    return len(verts), sub


def zz_edge(n: int, edges: Sequence[Edge], gamma, beta, j: int, k: int) -> complex:
    """<gamma beta| Z_j Z_k |gamma beta> from the radius-p ball state vector."""
    p = len(gamma)
    m, sub = ball(n, edges, p, j, k)
    psi = sv.qaoa_state(m, sub, gamma, beta)
    prob = psi.conj() * psi
    return complex(np.sum(prob * sv.zz_values(m, 0, 1)))


def ball_size(n: int, edges: Sequence[Edge], p: int, j: int, k: int) -> int:
    return ball(n, edges, p, j, k)[0]
