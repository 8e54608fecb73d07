"""Complex128 state-vector oracle for QAOA-MaxCut (test infrastructure only).

Definitions followed (Section II of the paper, eq. qaoa1 and the MaxCut cost):

* cost   C = 1/2 sum_{(j,k) in E} (1 - Z_j Z_k): the number of cut edges;
* state  |gamma beta> = U_B(beta_p) U_C(gamma_p) ... U_B(beta_1) U_C(gamma_1) |+>^N
  with U_C(gamma) = exp(-i gamma C) (the paper's U_C with its I - ZZ sum) and
  U_B(beta) = exp(-i beta sum_q X_q); layer 1 acts first and within a layer the
  cost unitary acts before the mixer, as in the paper's circuit figure;
* energy E = <gamma beta| C |gamma beta> and the per-edge <Z_j Z_k>.

Basis convention: qubit q is bit q of the basis-state integer x, and index value
0 is |0>, the +1 eigenstate of Z (the paper's tensor for |0> is (1, 0)), so
z_q(x) = 1 - 2 x_q.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np

Edge = Tuple[int, int]

MAX_QUBITS = 24


def _bits(n: int) -> np.ndarray:
    x = np.arange(1 << n, dtype=np.int64)
    return np.stack([(x >> q) & 1 for q in range(n)]) if n else np.zeros((0, 1), np.int64)


def cut_values(n: int, edges: Sequence[Edge]) -> np.ndarray:
    """cut(x) = number of edges (j,k) with x_j != x_k, i.e. the diagonal of C."""
    b = _bits(n)
    c = np.zeros(1 << n, dtype=np.float64)
    for j, k in edges:
        c += (b[j] ^ b[k]).astype(np.float64)
    return c


def zz_values(n: int, j: int, k: int) -> np.ndarray:
    """Diagonal of Z_j Z_k: z_j(x) z_k(x)."""
    b = _bits(n)
    return ((1 - 2 * b[j]) * (1 - 2 * b[k])).astype(np.float64)


def apply_cost(psi: np.ndarray, cut: np.ndarray, gamma: float) -> np.ndarray:
    """U_C(gamma) = exp(-i gamma C): C is diagonal, so a phase per basis state."""
    return psi * np.exp(-1j * gamma * cut)


def apply_mixer(psi: np.ndarray, n: int, beta: float) -> np.ndarray:
    """U_B(beta) = prod_q exp(-i beta X_q); exp(-i beta X) = cos(beta) I - i sin(beta) X."""
    c, s = np.cos(beta), np.sin(beta)
    out = psi.copy()
    for q in range(n):
        v = out.reshape(1 << (n - 1 - q), 2, 1 << q)
        a = v[:, 0, :].copy()
        b = v[:, 1, :].copy()
        v[:, 0, :] = c * a - 1j * s * b
        v[:, 1, :] = -1j * s * a + c * b
    return out


def apply_x_sum(psi: np.ndarray, n: int) -> np.ndarray:
    """(sum_q X_q) psi: the generator of U_B."""
    out = np.zeros_like(psi)
    for q in range(n):
        v = psi.reshape(1 << (n - 1 - q), 2, 1 << q)
        o = out.reshape(1 << (n - 1 - q), 2, 1 << q)
        o[:, 0, :] += v[:, 1, :]
        o[:, 1, :] += v[:, 0, :]
    return out


def qaoa_state(n: int, edges: Sequence[Edge], gamma: Sequence[float], beta: Sequence[float]) -> np.ndarray:
    """|gamma beta>_p as a length-2^n complex128 vector (eq. qaoa1)."""
    if n > MAX_QUBITS:
        raise ValueError(f"state vector limited to {MAX_QUBITS} qubits")
    if len(gamma) != len(beta):
        raise ValueError("gamma and beta must have the same length p")
    cut = cut_values(n, edges)
    psi = np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)
    for g, b in zip(gamma, beta):
        psi = apply_cost(psi, cut, float(g))
        psi = apply_mixer(psi, n, float(b))
    return psi


def amplitude(n: int, edges: Sequence[Edge], gamma, beta, x: int = 0) -> complex:
    """<x|gamma beta>, by default <0...0|gamma beta>: the single amplitude the
    paper simulates with its tensor networks (Section V), read off the state
    vector."""
    return complex(qaoa_state(n, edges, gamma, beta)[x])


def zz_expectations(n: int, edges: Sequence[Edge], gamma, beta) -> np.ndarray:
    """<gamma beta| Z_j Z_k |gamma beta> for every edge, complex128 (imaginary
    part kept so callers can check that it vanishes)."""
    psi = qaoa_state(n, edges, gamma, beta)
    prob = psi.conj() * psi
    return np.array([np.sum(prob * zz_values(n, j, k)) for j, k in edges], dtype=np.complex128)


def energy(n: int, edges: Sequence[Edge], gamma, beta) -> float:
    """E = <gamma beta| C |gamma beta> (expected cut size)."""
    psi = qaoa_state(n, edges, gamma, beta)
    cut = cut_values(n, edges)
    return float(np.real(np.vdot(psi, cut * psi)))


def energy_grad_adjoint(n: int, edges: Sequence[Edge], gamma, beta,
                        obs_edges: Sequence[Edge] | None = None) -> Tuple[float, np.ndarray, np.ndarray]:
    """E and its exact gradient by the adjoint-state method.

    ``obs_edges`` (default: all edges) selects the edges whose cut terms form
    the measured operator, so a single edge's term and its gradient can be
    taken while the state is still prepared on the whole graph.

    With psi_f = V U(theta) psi_pre, U(theta) = exp(-i theta G) and E = <psi_f|C|psi_f>,
    dE/dtheta = 2 Re < V^dagger C psi_f | (-i G) | U(theta) psi_pre >.  Both the
    state and the co-state lambda = C psi_f are walked back through the layers
    with the inverse gates.  G is the cut diagonal for gamma_l and sum_q X_q for
    beta_l.
    """
    p = len(gamma)
    cut = cut_values(n, edges)
    obs = cut if obs_edges is None else cut_values(n, obs_edges)
    phi = qaoa_state(n, edges, gamma, beta)
    lam = obs * phi
    e = float(np.real(np.vdot(phi, lam)))
    dg = np.zeros(p)
    db = np.zeros(p)
    for l in range(p - 1, -1, -1):
        db[l] = 2.0 * np.real(np.vdot(lam, -1j * apply_x_sum(phi, n)))
        phi = apply_mixer(phi, n, -float(beta[l]))
        lam = apply_mixer(lam, n, -float(beta[l]))
        dg[l] = 2.0 * np.real(np.vdot(lam, -1j * cut * phi))
        phi = apply_cost(phi, cut, -float(gamma[l]))
        lam = apply_cost(lam, cut, -float(gamma[l]))
    return e, dg, db


def energy_grad_fd(fn, gamma, beta, h: float = 1e-4) -> Tuple[np.ndarray, np.ndarray]:
    """Central finite differences (f(x+h) - f(x-h)) / 2h of a scalar function
    fn(gamma, beta), complex128/float64 arithmetic."""
    gamma = np.asarray(gamma, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    dg = np.zeros_like(gamma)
    db = np.zeros_like(beta)
    for l in range(gamma.size):
        gp, gm = gamma.copy(), gamma.copy()
        gp[l] += h
        gm[l] -= h
        dg[l] = (fn(gp, beta) - fn(gm, beta)) / (2 * h)
        bp, bm = beta.copy(), beta.copy()
        bp[l] += h
        bm[l] -= h
        db[l] = (fn(gamma, bp) - fn(gamma, bm)) / (2 * h)
    return dg, db
