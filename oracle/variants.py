"""The four tensor networks the paper compares (test infrastructure only).

Section IV and the figures of Section V compare the single amplitude
<0...0|gamma beta> computed from networks built four ways:

* default: the circuit with each ZZ phase decomposed as CNOT, a Z rotation on
  the target and CNOT, and each mixer as H, a Z rotation and H; every gate is a
  full tensor that gives each qubit it touches a fresh index;
* diagonal: the same circuit, but a gate that acts diagonally on a qubit keeps
  that qubit's index (Section IV.B): the Z rotations become rank-1 tensors on
  the current index and CNOT keeps its control index (a rank-3 tensor);
* ZZ: one two-qubit ZZ(gamma) gate per edge and one X rotation per qubit
  (Section IV.A), all as full tensors;
* diagonal + ZZ: the ZZ phase as a rank-2 tensor on the two current indices.

Conventions as in statevector.py: U_C = exp(-i gamma C) (an edge contributes
exp(-i gamma) when its bits differ), U_B = exp(-i beta X), cost before mixer,
layer 1 first, |0> and H on every qubit at the start, <0| at the end, so every
variant gives exactly the state-vector amplitude.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from . import tn

Edge = Tuple[int, int]
VARIANTS = ("default", "diagonal", "zz", "diagonal_zz")


def network(n: int, edges: Sequence[Edge], gamma, beta, variant: str):
    """[(tensor, [index ids])] of <0...0|gamma beta> and the index count."""
    diag = variant in ("diagonal", "diagonal_zz")
    zz = variant in ("zz", "diagonal_zz")
    h = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
    zero = np.array([1, 0], dtype=complex)
    ts: List = []
    nid = [0]

    def fresh():
        nid[0] += 1
        return nid[0] - 1

    cur = [fresh() for _ in range(n)]
    for q in range(n):
        ts.append((zero, [cur[q]]))

    def one(q, m, keeps):
        """one-qubit gate with matrix m (m[out, in]); diagonal ones may keep the index"""
        if keeps:
            ts.append((np.diag(m).copy(), [cur[q]]))
        else:
            w = fresh()
            ts.append((m.T.copy(), [cur[q], w]))  # tensor[in, out]
            cur[q] = w

    for q in range(n):
        one(q, h, False)
    p = len(gamma)
    for l in range(p):
        g, b = gamma[l], beta[l]
        ph = np.array([[1, np.exp(-1j * g)], [np.exp(-1j * g), 1]])  # phase by (bit u, bit w)
        for u, w in edges:
            if zz:
                if diag:
                    ts.append((ph.copy(), [cur[u], cur[w]]))
                else:
                    t = np.zeros((2, 2, 2, 2), dtype=complex)  # [u_in, w_in, u_out, w_out]
                    for a in range(2):
                        for c in range(2):
                            t[a, c, a, c] = ph[a, c]
                    nu, nw = fresh(), fresh()
                    ts.append((t, [cur[u], cur[w], nu, nw]))
                    cur[u], cur[w] = nu, nw
            else:
                for step in range(3):
                    if step == 1:
                        one(w, np.diag([1, np.exp(-1j * g)]), diag)  # the target now holds x_u xor x_w
                        continue
                    if diag:  # CNOT keeps the control's index
                        t = np.zeros((2, 2, 2), dtype=complex)  # [control, t_in, t_out]
                        for a in range(2):
                            for c in range(2):
                                t[a, c, c ^ a] = 1
                        nw = fresh()
                        ts.append((t, [cur[u], cur[w], nw]))
                        cur[w] = nw
                    else:
                        t = np.zeros((2, 2, 2, 2), dtype=complex)  # [c_in, t_in, c_out, t_out]
                        for a in range(2):
                            for c in range(2):
                                t[a, c, a, c ^ a] = 1
                        nu, nw = fresh(), fresh()
                        ts.append((t, [cur[u], cur[w], nu, nw]))
                        cur[u], cur[w] = nu, nw
        for q in range(n):
            if zz:
                one(q, np.array([[np.cos(b), -1j * np.sin(b)], [-1j * np.sin(b), np.cos(b)]]), False)
            else:
                one(q, h, False)
                one(q, np.diag([np.exp(-1j * b), np.exp(1j * b)]), diag)
                one(q, h, False)
    for q in range(n):
        ts.append((zero, [cur[q]]))
    return ts, nid[0]


def amplitude(n: int, edges: Sequence[Edge], gamma, beta, variant: str) -> complex:
    """<0...0|gamma beta> by contracting the variant's network."""
    ts, _ = network(n, edges, gamma, beta, variant)
    order, _ = tn.min_fill_order(ts)
    return tn.contract(ts, order)


def elimination_cost(n: int, edges: Sequence[Edge], p: int, variant: str, order: Sequence[int]) -> Tuple[int, float]:
    """(width, sum over eliminated indices of 2^|union|) of eliminating the
    variant's network in `order` (Section III.B, symbolically): eliminating v
    replaces every tensor that carries v by one tensor on the union of their
    indices without v; the width is the largest such result, and the work of
    the step is 2^|union| (one product term per assignment of the union).
    Index ids as network() numbers them."""
    ts, nidx = network(n, edges, [0.1] * p, [0.2] * p, variant)
    if sorted(order) != list(range(nidx)):
        raise ValueError("order is not a permutation of the network's indices")
    live = [set(ix) for _, ix in ts]
    width, ops = 0, 0.0
    for v in order:
        touching = [t for t in live if v in t]
        live = [t for t in live if v not in t]
        union = set().union(*touching)
        ops += 2.0 ** len(union)
        rest = union - {v}
        width = max(width, len(rest))
        if rest:
            live.append(rest)
    return width, ops


def counts(n: int, edges: Sequence[Edge], p: int, variant: str) -> Tuple[int, int]:
    """(indices, tensors) of the variant's network."""
    ts, nidx = network(n, edges, [0.1] * p, [0.2] * p, variant)
    return nidx, len(ts)
