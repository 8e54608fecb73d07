"""Pins of the CPU oracle against results fixed by mathematics, not by the oracle.

Each test names what pins it: dense matrix exponentials of the Hamiltonians
(scipy), the published p=1 closed form (Wang et al., PRA 97, 022304), exact
special values (gamma = 0, beta = 0), symmetries of the ansatz, analytic
derivatives, and agreement of three independent routes (full state vector,
radius-p ball state vector, tensor network).  The last tests plant mistakes in
the oracle and check that the pins catch them.
"""
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import ball, statevector as sv, tn
from workloads import bfs_subgraph, random_regular_graph, triangle_counts

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- helpers
def random_graph(n, m, seed):
    rng = np.random.default_rng(seed)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    idx = rng.choice(len(pairs), size=m, replace=False)
    return sorted(pairs[i] for i in idx)


def closed_form_p1(d, e, f, g, b):
    """Wang et al. 2018, Theorem 1 (p = 1 edge term of MaxCut QAOA)."""
    return (0.5 + 0.25 * np.sin(4 * b) * np.sin(g) * (np.cos(g) ** d + np.cos(g) ** e)
            - 0.25 * np.sin(2 * b) ** 2 * np.cos(g) ** (d + e - 2 * f) * (1 - np.cos(2 * g) ** f))


def degrees(n, edges):
    deg = [0] * n
    for u, v in edges:
        deg[u] += 1
        deg[v] += 1
    return deg


def dense_energy(n, edges, gamma, beta):
    """<C> from dense 2^n x 2^n Hamiltonians and scipy.linalg.expm."""
    I2 = np.eye(2)
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    Z = np.diag([1.0, -1.0])

    def op(single, q):
        m = np.array([[1.0]])
        for r in range(n - 1, -1, -1):          # bit q of the index is qubit q
            m = np.kron(m, single if r == q else I2)
        return m

    C = sum(0.5 * (np.eye(1 << n) - op(Z, j) @ op(Z, k)) for j, k in edges)
    B = sum(op(X, q) for q in range(n))
    psi = np.full(1 << n, 2 ** (-n / 2), dtype=complex)
    for g, b in zip(gamma, beta):
        psi = scipy.linalg.expm(-1j * g * C) @ psi
        psi = scipy.linalg.expm(-1j * b * B) @ psi
    zz = [np.vdot(psi, op(Z, j) @ op(Z, k) @ psi) for j, k in edges]
    return np.real(np.vdot(psi, C @ psi)), np.array(zz)


# --------------------------------------------------------------------------- state vector
@pytest.mark.parametrize("n,m,p,seed", [(3, 3, 1, 0), (4, 6, 2, 1), (5, 6, 3, 2), (6, 9, 2, 3)])
def test_statevector_matches_dense_expm(n, m, p, seed):
    edges = random_graph(n, m, seed)
    rng = np.random.default_rng(seed)
    g, b = rng.uniform(-np.pi, np.pi, p), rng.uniform(-np.pi, np.pi, p)
    e_ref, zz_ref = dense_energy(n, edges, g, b)
    assert abs(sv.energy(n, edges, g, b) - e_ref) < 1e-12
    np.testing.assert_allclose(sv.zz_expectations(n, edges, g, b), zz_ref, atol=1e-12)


def test_golden_closed_form_transcription():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "p1_closed_form.txt")) if l[0] != "#"]
    for d, e, f, val in rows:
        assert abs(closed_form_p1(int(d), int(e), int(f), 0.4, 0.3) - float(val)) < 1e-14


@pytest.mark.parametrize("seed", range(5))
def test_statevector_p1_closed_form_regular(seed):
    n = 10
    edges = random_regular_graph(n, 3, seed)
    tri = triangle_counts(n, edges)
    for g, b in [(0.4, 0.3), (1.1, -0.7), (2.5, 2.9)]:
        zz = sv.zz_expectations(n, edges, [g], [b])
        for (u, v), z, f in zip(edges, zz, tri):
            assert abs(0.5 * (1 - z.real) - closed_form_p1(2, 2, f, g, b)) < 1e-13


def test_statevector_p1_closed_form_irregular():
    for seed, (n, m) in enumerate([(8, 12), (9, 15), (7, 14)]):
        edges = random_graph(n, m, 10 + seed)
        deg, tri = degrees(n, edges), triangle_counts(n, edges)
        zz = sv.zz_expectations(n, edges, [0.7], [0.45])
        for (u, v), z, f in zip(edges, zz, tri):
            want = closed_form_p1(deg[u] - 1, deg[v] - 1, f, 0.7, 0.45)
            assert abs(0.5 * (1 - z.real) - want) < 1e-13


def test_k4_and_single_edge_values():
    k4 = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    # every K4 edge has d = e = 2 and f = 2 triangles
    assert abs(sv.energy(4, k4, [0.4], [0.3]) - 6 * closed_form_p1(2, 2, 2, 0.4, 0.3)) < 1e-13
    assert abs(sv.energy(2, [(0, 1)], [0.4], [0.3]) - 0.681476557912114) < 1e-14


def test_zero_angles_give_half_the_edges():
    edges = random_regular_graph(10, 3, 0)
    rng = np.random.default_rng(0)
    for p in (1, 2, 3):
        g, b = rng.uniform(0, np.pi, p), rng.uniform(0, np.pi, p)
        assert abs(sv.energy(10, edges, np.zeros(p), b) - 7.5) < 1e-12
        assert abs(sv.energy(10, edges, g, np.zeros(p)) - 7.5) < 1e-12


def test_depth_reductions():
    n, edges = 10, random_regular_graph(10, 3, 1)
    rng = np.random.default_rng(2)
    g, b = rng.uniform(0, np.pi, 3), rng.uniform(0, np.pi, 3)
    b0 = b.copy()
    b0[-1] = 0.0
    assert abs(sv.energy(n, edges, g, b0) - sv.energy(n, edges, g[:2], b[:2])) < 1e-12
    g0 = g.copy()
    g0[0] = 0.0
    assert abs(sv.energy(n, edges, g0, b) - sv.energy(n, edges, g[1:], b[1:])) < 1e-12


def test_symmetries_and_convention_detector():
    n, edges = 10, random_regular_graph(10, 3, 3)
    rng = np.random.default_rng(3)
    g, b = rng.uniform(0, np.pi, 2), rng.uniform(0, np.pi, 2)
    e = sv.energy(n, edges, g, b)
    assert abs(sv.energy(n, edges, g, b + np.array([np.pi / 2, 0])) - e) < 1e-12
    assert abs(sv.energy(n, edges, -g, -b) - e) < 1e-12
    assert abs(sv.energy(n, edges, g + np.array([0, 2 * np.pi]), b) - e) < 1e-12
    # with U_C = exp(-i gamma C) a shift of gamma by pi is NOT a symmetry on a
    # 3-regular graph (it would be if the gate were exp(i gamma ZZ))
    assert abs(sv.energy(n, edges, g + np.array([np.pi, 0]), b) - e) > 1e-3


def test_bounds_and_realness():
    n, edges = 12, random_regular_graph(12, 3, 4)
    rng = np.random.default_rng(4)
    for p in (1, 2, 3):
        g, b = rng.uniform(0, np.pi, p), rng.uniform(0, np.pi, p)
        zz = sv.zz_expectations(n, edges, g, b)
        assert np.max(np.abs(zz.imag)) < 1e-14
        assert np.all(np.abs(zz.real) <= 1 + 1e-14)
        e = sv.energy(n, edges, g, b)
        assert -1e-12 <= e <= len(edges) + 1e-12
        assert abs(e - np.sum(0.5 * (1 - zz.real))) < 1e-12


# --------------------------------------------------------------------------- gradients
def test_adjoint_gradient_vs_fd():
    n, edges = 10, random_regular_graph(10, 3, 5)
    rng = np.random.default_rng(5)
    for p in (1, 2, 3):
        g, b = rng.uniform(0, np.pi, p), rng.uniform(0, np.pi, p)
        e, dg, db = sv.energy_grad_adjoint(n, edges, g, b)
        assert abs(e - sv.energy(n, edges, g, b)) < 1e-12
        fg, fb = sv.energy_grad_fd(lambda G, B: sv.energy(n, edges, G, B), g, b, h=1e-4)
        np.testing.assert_allclose(dg, fg, atol=2e-6)
        np.testing.assert_allclose(db, fb, atol=2e-6)


def test_adjoint_gradient_p1_analytic():
    """Triangle-free edge of a 3-regular graph at p=1: <C_uv> = 1/2 +
    1/2 sin4b sin g cos^2 g, so d/dg = 1/2 sin4b (cos^3 g - 2 sin^2 g cos g)
    and d/db = 2 cos4b sin g cos^2 g."""
    n = 10
    edges = random_regular_graph(n, 3, 0)
    tri = triangle_counts(n, edges)
    j, k = next(e for e, f in zip(edges, tri) if f == 0)
    for g, b in [(0.4, 0.3), (1.3, 0.9)]:
        _, dg, db = sv.energy_grad_adjoint(n, edges, [g], [b], obs_edges=[(j, k)])
        assert abs(dg[0] - 0.5 * np.sin(4 * b) * (np.cos(g) ** 3 - 2 * np.sin(g) ** 2 * np.cos(g))) < 1e-12
        assert abs(db[0] - 2 * np.cos(4 * b) * np.sin(g) * np.cos(g) ** 2) < 1e-12


# --------------------------------------------------------------------------- ball and tensor network
@pytest.mark.parametrize("p", [1, 2, 3])
def test_ball_matches_full_statevector(p):
    n = 14
    edges = random_regular_graph(n, 3, 6 + p)
    rng = np.random.default_rng(p)
    g, b = rng.uniform(0, np.pi, p), rng.uniform(0, np.pi, p)
    zz = sv.zz_expectations(n, edges, g, b)
    for (j, k), z in zip(edges, zz):
        assert abs(ball.zz_edge(n, edges, g, b, j, k) - z) < 1e-12


@pytest.mark.parametrize("p", [1, 2, 3])
def test_tn_matches_statevector_regular(p):
    n = 12
    edges = random_regular_graph(n, 3, 20 + p)
    rng = np.random.default_rng(20 + p)
    g, b = rng.uniform(0, np.pi, p), rng.uniform(0, np.pi, p)
    zz = sv.zz_expectations(n, edges, g, b)
    got = np.array([tn.zz_edge(n, edges, g, b, j, k) for j, k in edges])
    np.testing.assert_allclose(got, zz, atol=1e-12)


def test_tn_matches_statevector_irregular_and_k4():
    k4 = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    for n, edges, p in [(4, k4, 2), (9, random_graph(9, 16, 7), 2), (7, random_graph(7, 10, 8), 3),
                        (2, [(0, 1)], 3)]:
        rng = np.random.default_rng(n + p)
        g, b = rng.uniform(0, np.pi, p), rng.uniform(0, np.pi, p)
        zz = sv.zz_expectations(n, edges, g, b)
        got = np.array([tn.zz_edge(n, edges, g, b, j, k) for j, k in edges])
        np.testing.assert_allclose(got, zz, atol=1e-12)


def test_tn_light_cone_is_the_distance_rule():
    """The pruned gate list keeps the mixer of layer l on q iff dist(q) <= p - l
    and the ZZ of layer l on (u,w) iff min dist <= p - l (l = 1..p)."""
    n, p = 60, 3
    edges = random_regular_graph(n, 3, 0)
    ball_n, _ = ball.ball(n, edges, p, *edges[0])
    kept = tn.prune(tn.circuit(n, edges, p), *edges[0])
    qubits = {q for _, _, qs in kept for q in qs}
    assert len(qubits) == ball_n
    j, k = edges[0]
    adj = {v: set() for v in range(n)}
    for u, w in edges:
        adj[u].add(w)
        adj[w].add(u)
    dist = {j: 0, k: 0}
    frontier = [j, k]
    while frontier:
        nxt = []
        for u in frontier:
            for w in adj[u]:
                if w not in dist:
                    dist[w] = dist[u] + 1
                    nxt.append(w)
        frontier = nxt
    for kind, l, qs in kept:
        if kind == "x":
            assert dist[qs[0]] <= p - (l + 1)
        else:
            assert min(dist[qs[0]], dist[qs[1]]) <= p - (l + 1)
    n_x = sum(max(0, p - dist[q]) for q in dist)
    assert sum(1 for g in kept if g[0] == "x") == n_x


def test_diagonal_rule_example_and_zz_golden():
    """eq. example: sum_jk U_ij D_jk psi_k with D = diag(alpha) equals
    sum_j U_ij alpha_j psi_j; and the oracle's ZZ tensor against the paper's
    rank-2 form (golden file), under U_C = exp(-i gamma C): the paper's angle is
    gamma/2 and a global phase exp(-i gamma/2) is dropped."""
    rng = np.random.default_rng(0)
    U = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    alpha = rng.normal(size=2) + 1j * rng.normal(size=2)
    psi = rng.normal(size=2) + 1j * rng.normal(size=2)
    close = rng.normal(size=2) + 1j * rng.normal(size=2)
    full = tn.contract([(close, [0]), (U, [0, 1]), (np.diag(alpha), [1, 2]), (psi, [2])], [2, 1, 0])
    diag = tn.contract([(close, [0]), (U, [0, 1]), (alpha, [1]), (psi, [1])], [1, 0])
    assert abs(full - diag) < 1e-13
    rows = [l.split() for l in open(os.path.join(GOLDEN, "zz_gate_section4b.txt")) if l[0] != "#"]
    for g in (0.4, 1.7, -2.2):
        rho = np.exp(1j * g / 2)
        paper = np.zeros((2, 2), complex)
        for bits, sign, ent in rows:
            xi, xj = int(bits[0]), int(bits[1])
            assert np.isclose(np.exp(1j * int(sign) * g / 2), rho if ent == "rho" else rho.conjugate())
            paper[xi, xj] = rho if ent == "rho" else rho.conjugate()
        np.testing.assert_allclose(tn.zz_tensor(g), np.exp(-1j * g / 2) * paper, atol=1e-15)


def test_tn_order_independence_and_width():
    n, edges = 40, random_regular_graph(40, 3, 9)
    rng = np.random.default_rng(9)
    g, b = rng.uniform(0, np.pi, 2), rng.uniform(0, np.pi, 2)
    j, k = edges[3]
    t = tn.network(n, edges, g, b, j, k)
    order, width = tn.min_fill_order(t)
    a = tn.contract(t, order)
    idx = sorted({i for _, ix in t for i in ix})
    bwd = tn.contract(t, idx[::-1])
    assert abs(a - bwd) < 1e-12
    assert abs(a - ball.zz_edge(n, edges, g, b, j, k)) < 1e-12
    assert width >= 2


# --------------------------------------------------------------------------- planted mistakes
def test_pins_catch_planted_mistakes(monkeypatch):
    """Each planted mistake in the oracle must break at least one pin above."""
    n = 10
    edges = random_regular_graph(n, 3, 0)
    tri = triangle_counts(n, edges)

    def closed_form_ok():
        zz = sv.zz_expectations(n, edges, [0.4], [0.3])
        return all(abs(0.5 * (1 - z.real) - closed_form_p1(2, 2, f, 0.4, 0.3)) < 1e-10
                   for z, f in zip(zz, tri))

    assert closed_form_ok()
    orig_mixer, orig_cost = sv.apply_mixer, sv.apply_cost
    # wrong sign of the mixer exponent
    monkeypatch.setattr(sv, "apply_mixer", lambda psi, n_, b: orig_mixer(psi, n_, -b))
    assert not closed_form_ok()
    monkeypatch.setattr(sv, "apply_mixer", orig_mixer)
    # the paper's literal exp(i gamma ZZ) angle (twice the convention's)
    monkeypatch.setattr(sv, "apply_cost", lambda psi, c, g: orig_cost(psi, c, 2 * g))
    assert not closed_form_ok()
    monkeypatch.setattr(sv, "apply_cost", orig_cost)
    # tensor network: a transposed/conjugated ZZ tensor in the ket
    orig_zz = tn.zz_tensor
    monkeypatch.setattr(tn, "zz_tensor", lambda g: orig_zz(-g))
    z_bad = tn.zz_edge(n, edges, [0.4, 1.0], [0.3, 0.2], *edges[0])
    monkeypatch.setattr(tn, "zz_tensor", orig_zz)
    z_ok = sv.zz_expectations(n, edges, [0.4, 1.0], [0.3, 0.2])[0]
    assert abs(z_bad - z_ok) > 1e-3
    # light cone that drops the first-layer ZZ gates
    orig_prune = tn.prune
    monkeypatch.setattr(tn, "prune", lambda gates, j, k: [g for g in orig_prune(gates, j, k)
                                                          if not (g[0] == "zz" and g[1] == 0)])
    z_bad = tn.zz_edge(n, edges, [0.4, 1.0], [0.3, 0.2], *edges[0])
    assert abs(z_bad - z_ok) > 1e-3


def test_subgraph_helper():
    n, edges = 100, random_regular_graph(100, 3, 0)
    m, sub = bfs_subgraph(n, edges, 16)
    assert m == 16
    assert all(0 <= u < v < 16 for u, v in sub)
    assert len(set(sub)) == len(sub)


def test_amplitude_closed_forms():
    """<0...0|gamma beta> from the state vector: at gamma = 0 every cost layer
    is the identity and exp(-i beta X)|+> = exp(-i beta)|+>, so the amplitude
    is 2^(-N/2) exp(-i N sum beta); at beta = 0 the mixers vanish and the
    all-zero string cuts nothing, so it is 2^(-N/2); and the amplitudes of all
    basis states have unit total weight."""
    n, edges = 8, random_regular_graph(8, 3, 2)
    b = [0.3, -0.7]
    a = sv.amplitude(n, edges, [0.0, 0.0], b)
    assert abs(a - 2 ** (-n / 2) * np.exp(-1j * n * sum(b))) < 1e-14
    assert abs(sv.amplitude(n, edges, [0.9, 0.4], [0.0, 0.0]) - 2 ** (-n / 2)) < 1e-14
    g = [0.9, 0.4]
    tot = sum(abs(sv.amplitude(n, edges, g, b, x)) ** 2 for x in range(1 << n))
    assert abs(tot - 1) < 1e-12


@pytest.mark.parametrize("variant", ["default", "diagonal", "zz", "diagonal_zz"])
def test_variant_networks_give_the_amplitude(variant):
    """Each of the paper's four network constructions contracts to the
    state-vector amplitude <0...0|gamma beta> (so the constructions, whose
    sizes the cost model compares, are the same computation)."""
    from oracle import variants

    for n, seed, p in ((4, 0, 1), (6, 1, 2)):
        edges = random_regular_graph(n, 3, seed) if n % 2 == 0 else [(0, 1)]
        rng = np.random.default_rng(seed + 7)
        g, b = rng.uniform(0, np.pi, p), rng.uniform(0, np.pi, p)
        assert abs(variants.amplitude(n, edges, g, b, variant) - sv.amplitude(n, edges, g, b)) < 1e-12


def test_variant_network_sizes_closed_form():
    """Index and tensor counts of the four constructions: 2N + p(5|E| + 3N)
    indices for the default circuit, 2N + p(2|E| + 2N) with the diagonal
    simplification, 2N + p(2|E| + N) for ZZ gates and 2N + pN for diagonal +
    ZZ; tensors 3N + p(3|E| + 3N), 3N + p(3|E| + 3N), 3N + p(|E| + N) twice."""
    from oracle import variants

    n, edges = 8, random_regular_graph(8, 3, 4)
    m = len(edges)
    for p in (1, 2, 3):
        assert variants.counts(n, edges, p, "default") == (2 * n + p * (5 * m + 3 * n), 3 * n + p * (3 * m + 3 * n))
        assert variants.counts(n, edges, p, "diagonal") == (2 * n + p * (2 * m + 2 * n), 3 * n + p * (3 * m + 3 * n))
        assert variants.counts(n, edges, p, "zz") == (2 * n + p * (2 * m + n), 3 * n + p * (m + n))
        assert variants.counts(n, edges, p, "diagonal_zz") == (2 * n + p * n, 3 * n + p * (m + n))


def test_full_size_golden_files_match_the_oracle():
    """The stored full-size expected values (tests/golden/make_full_size.py)
    are the oracle's: a few entries recomputed here, the radius-3 tree-like
    edges of the p = 3 file share one value (their light cones are isomorphic
    trees), and every stored <ZZ> is real and within [-1, 1]."""
    import os

    from oracle import tn
    from workloads import workload

    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

    def rows(name):
        with open(os.path.join(golden, f"full_size_{name}.txt")) as fh:
            return [l.split() for l in fh if not l.startswith("#")]

    for name, picks in (("p3_n244", (0, 101, 365)), ("p4_n100", (7,)), ("p5_n1000", (3,))):
        w = workload(name)
        r = rows(name)
        assert len(r) == len(w.edges)
        for i in picks:
            z = tn.zz_edge(w.n, w.edges, w.gamma, w.beta, *w.edges[i])
            assert abs(z - (float(r[i][4]) + 1j * float(r[i][5]))) < 1e-12
        vals = np.array([float(x[4]) for x in r])
        assert np.all(np.abs(vals) <= 1) and max(abs(float(x[5])) for x in r) < 1e-12
    r = rows("p3_n244")
    w = workload("p3_n244")
    gates = tn.circuit(w.n, w.edges, w.p)
    nq = [len({q for _, _, qs in tn.prune(gates, j, k) for q in qs} | {j, k}) for j, k in w.edges]
    tree = [i for i, q in enumerate(nq) if q == 2 * (2 ** (w.p + 1) - 1)]  # 30 distinct qubits: a tree
    assert len(tree) > 10
    vals = np.array([float(r[i][4]) for i in tree])
    assert np.ptp(vals) < 1e-12
