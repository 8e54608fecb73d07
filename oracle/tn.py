"""Independent CPU tensor-network oracle for one edge term (test infrastructure only).

Steps, in the paper's order:

1. The circuit as a gate list: for layer l = 1..p the ZZ phase gate of every
   edge, then the mixer of every qubit (Section II; the circuit figure and the
   ZZ-merge equation give this gate set).
2. Light cone by pruning: walking the list backwards, a gate is dropped when it
   commutes with the observable and with every gate kept after it (the
   light-cone remark of Section II).  ZZ gates commute with each other and
   with Z_j Z_k; a mixer on q commutes with a ZZ gate unless the gate touches q.
3. Tensor network (Sections III.A and IV): the ket gets |+> = (1,1)/sqrt2 per
   qubit; a mixer creates a new wire index and the 2x2 tensor exp(-i beta X);
   the ZZ gate is diagonal, so it enters as a rank-2 tensor on the two current
   wire indices with no new index (the diagonal-gate rule, eq. example).  The
   bra is the complex conjugate network.  The identity between ket and bra and
   the observable Z_j Z_k are diagonal too, so each qubit's last ket index and
   last bra index are one index, carrying the vector (1, -1) for j and k.
4. Contraction (eq. tn and the bucket procedure of Section III.B): pick an index,
   multiply every tensor that has it (numpy einsum over their union), sum the
   index away, repeat.  The elimination order is this module's own greedy
   minimum-fill order.

ZZ convention (reading of Section II): U_C(gamma) = exp(-i gamma C) with
C = 1/2 sum (1 - Z Z), so one edge contributes exp(-i gamma (1 - z_u z_w)/2):
1 when the two bits agree and exp(-i gamma) when they differ.  This equals the
paper's rank-2 tensor [[rho, conj rho], [conj rho, rho]] with rho = exp(i gamma/2),
times the global phase exp(-i gamma/2).
"""
from __future__ import annotations

import string
from typing import Dict, List, Sequence, Tuple

import numpy as np

Edge = Tuple[int, int]
_LETTERS = string.ascii_letters


def circuit(n: int, edges: Sequence[Edge], p: int):
    """Gate list of the depth-p ansatz: ('zz', l, (u, w)) and ('x', l, (q,))."""
    gates = []
    for l in range(p):
        gates += [("zz", l, (u, w)) for u, w in edges]
        gates += [("x", l, (q,)) for q in range(n)]
    return gates


def prune(gates, j: int, k: int):
    """Keep only gates that fail to commute past the observable Z_j Z_k and all
    later kept gates; returns the kept gates in circuit order."""
    zz_later = set()          # qubits touched by a kept ZZ gate later in the circuit
    x_later = set()           # qubits with a kept mixer later in the circuit
    kept = []
    for g in reversed(gates):
        kind, _, qs = g
        if kind == "x":
            q = qs[0]
            if q in zz_later or q in (j, k):
                kept.append(g)
                x_later.add(q)
        else:
            if qs[0] in x_later or qs[1] in x_later:
                kept.append(g)
                zz_later.update(qs)
    kept.reverse()
    return kept


def zz_tensor(g: float) -> np.ndarray:
    e = np.exp(-1j * g)
    return np.array([[1.0, e], [e, 1.0]], dtype=np.complex128)


def mixer_tensor(b: float) -> np.ndarray:
    c, s = np.cos(b), np.sin(b)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def network(n: int, edges: Sequence[Edge], gamma, beta, j: int, k: int, dtype=np.complex128):
    """Tensors (array, [index ids]) of <gamma beta| Z_j Z_k |gamma beta>.
    The tensors are built in complex128 and stored as `dtype` (complex64 only
    for timing the oracle at the GPU path's precision)."""
    p = len(gamma)
    kept = prune(circuit(n, edges, p), j, k)
    qubits = sorted({q for _, _, qs in kept for q in qs} | {j, k})
    nid = [0]

    def new():
        nid[0] += 1
        return nid[0] - 1

    plus = np.full(2, 2 ** -0.5, dtype=np.complex128)
    tensors = []
    sides = []
    for conj in (False, True):
        cur = {}
        side = []
        for q in qubits:
            cur[q] = new()
            side.append((plus, [cur[q]]))
        for kind, l, qs in kept:
            if kind == "zz":
                t = zz_tensor(gamma[l])
                side.append((t.conj() if conj else t, [cur[qs[0]], cur[qs[1]]]))
            else:
                q = qs[0]
                m = mixer_tensor(beta[l])
                nw = new()
                side.append((m.conj() if conj else m, [nw, cur[q]]))
                cur[q] = nw
        sides.append((side, cur))
    (ket, kcur), (bra, bcur) = sides
    rename = {bcur[q]: kcur[q] for q in qubits}
    tensors = ket + [(a, [rename.get(i, i) for i in ix]) for a, ix in bra]
    zvec = np.array([1.0, -1.0], dtype=np.complex128)
    tensors += [(zvec, [kcur[j]]), (zvec, [kcur[k]])]
    return [(a.astype(dtype), ix) for a, ix in tensors]


def min_fill_order(tensors) -> Tuple[List[int], int]:
    """Greedy order on the interaction graph (indices adjacent when they share a
    tensor): repeatedly take the index whose elimination adds the fewest new
    edges among its neighbours (ties: fewer neighbours, then larger id).
    Returns the order and the contraction width (largest neighbourhood)."""
    adj: Dict[int, set] = {}
    for _, ix in tensors:
        for a in ix:
            adj.setdefault(a, set())
            for b in ix:
                if a != b:
                    adj[a].add(b)

    def fill(v):
        nb = list(adj[v])
        f = 0
        for i in range(len(nb)):
            ai = adj[nb[i]]
            for t in range(i + 1, len(nb)):
                if nb[t] not in ai:
                    f += 1
        return f

    score = {v: fill(v) for v in adj}
    order = []
    width = 0
    while adj:
        v = min(adj, key=lambda x: (score[x], len(adj[x]), -x))
        nb = adj.pop(v)
        width = max(width, len(nb))
        for a in nb:
            adj[a].discard(v)
            adj[a].update(b for b in nb if b != a)
        touched = set(nb)
        for a in nb:
            touched |= adj[a]
        for a in touched:
            score[a] = fill(a)
        order.append(v)
    return order, width


def contract(tensors, order: Sequence[int]) -> complex:
    """Bucket elimination: for each index in order, einsum the tensors that hold
    it over their union and sum the index out; the result is the product of the
    remaining scalars."""
    pool = [(np.asarray(a), list(ix)) for a, ix in tensors]
    for v in order:
        bucket = [t for t in pool if v in t[1]]
        pool = [t for t in pool if v not in t[1]]
        union = sorted({i for _, ix in bucket for i in ix})
        letter = {i: _LETTERS[n] for n, i in enumerate(union)}
        out = [i for i in union if i != v]
        spec = ",".join("".join(letter[i] for i in ix) for _, ix in bucket)
        spec += "->" + "".join(letter[i] for i in out)
        res = np.einsum(spec, *[a for a, _ in bucket], optimize=False)
        pool.append((res, out))
    val = 1.0 + 0.0j
    for a, ix in pool:
        assert not ix
        val *= complex(a)
    return val


def zz_edge(n: int, edges: Sequence[Edge], gamma, beta, j: int, k: int, dtype=np.complex128) -> complex:
    """<gamma beta| Z_j Z_k |gamma beta> by tensor-network contraction."""
    t = network(n, edges, gamma, beta, j, k, dtype)
    order, _ = min_fill_order(t)
    return contract(t, order)


def energy(n: int, edges: Sequence[Edge], gamma, beta) -> float:
    """E = sum over edges of (1 - Re <Z_j Z_k>) / 2 (Section II cost)."""
    return float(sum(0.5 * (1.0 - zz_edge(n, edges, gamma, beta, j, k).real) for j, k in edges))
