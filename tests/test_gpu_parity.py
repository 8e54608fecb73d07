"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances: complex128 energies within 1e-10 relative and per-edge <ZZ>
within 1e-10 absolute (|<ZZ>| <= 1 and may be ~0, so absolute); complex64 (FP32
accumulate) within 1e-5 relative / absolute.  Gradients: against the oracle's
exact adjoint-state gradient 1e-9 (c128) / 1e-4 (c64); against central
differences with h = 1e-4 within 1e-6 (truncation ~h^2 E'''/6).
"""
import numpy as np
import pytest

from oracle import ball, statevector as sv, tn
from workloads import bfs_subgraph, random_regular_graph, triangle_counts, workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def make(n, edges, p, dtype, order, g, b, **tune):
    from paper_2106_15740_amd import QaoaNet

    print(f"[case] n={n} m={len(edges)} p={p} {dtype} {order} {tune}", flush=True)
    net = QaoaNet(n, edges, p, dtype=dtype, order=order, device=0)
    if tune:
        net.set_tuning(**tune)
    net.set_params(g, b)
    return net


MODES = ["plain", "batched"]


def lowest_recompute_budget(net):
    """The lowest of a few shares of the largest cone's working set (above
    the pinned leaf tables) that the planner meets by recomputation."""
    from paper_2106_15740_amd import QtnError

    full = net.info()
    for f in (0.9, 0.95, 0.98, 0.99, 0.999):
        budget = full["pinned_bytes"] + int(f * full["max_cone_dynamic"])
        try:
            net.set_memory_budget(budget)
        except QtnError:
            continue
        net.set_memory_budget(0)
        return budget
    raise AssertionError("no budget below the largest cone is met")


@pytest.mark.parametrize("mode", MODES)
def test_config1_c128_vs_statevector(mode):
    w = workload("p1_n10")
    net = make(w.n, w.edges, w.p, "c128", "min_degree", w.gamma, w.beta)
    zz_dev = net.zz_buffer()
    e = net.energy(mode, zz_out=zz_dev)
    zz_ref = sv.zz_expectations(w.n, w.edges, w.gamma, w.beta)
    e_ref = sv.energy(w.n, w.edges, w.gamma, w.beta)
    assert abs(e - e_ref) <= 1e-10 * abs(e_ref)
    np.testing.assert_allclose(zz_dev.cpu().numpy(), zz_ref, atol=1e-10)
    np.testing.assert_allclose(net.edge_results(), zz_ref, atol=1e-10)
    e2, dg, db = net.energy_grad(mode)
    _, dg_ref, db_ref = sv.energy_grad_adjoint(w.n, w.edges, w.gamma, w.beta)
    assert abs(e2 - e_ref) <= 1e-10 * abs(e_ref)
    np.testing.assert_allclose(dg, dg_ref, atol=1e-9)
    np.testing.assert_allclose(db, db_ref, atol=1e-9)


@pytest.mark.parametrize("mode", MODES)
def test_config2_c64_vs_ball_statevector(mode):
    w = workload("p2_n60")
    net = make(w.n, w.edges, w.p, "c64", "min_fill", w.gamma, w.beta)
    e = net.energy(mode)
    zz = net.edge_results()
    ref = np.array([ball.zz_edge(w.n, w.edges, w.gamma, w.beta, j, k) for j, k in w.edges])
    np.testing.assert_allclose(zz, ref, atol=1e-5)
    e_ref = float(np.sum(0.5 * (1 - ref.real)))
    assert abs(e - e_ref) <= 1e-5 * abs(e_ref)
    assert np.max(np.abs(zz.imag)) < 1e-5


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_small_graphs_energy_and_gradient(mode, dtype):
    """Regular, irregular, triangle-rich and tiny graphs, p = 1..3, against the
    full state vector (N <= 12) and its adjoint-state gradient."""
    k4 = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    cases = [(4, k4, 2), (2, [(0, 1)], 3), (12, random_regular_graph(12, 3, 3), 3),
             (9, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0), (0, 5), (5, 6), (6, 7), (2, 8), (8, 1)], 2),
             (7, [(0, 1), (2, 3)], 2)]
    tol_e, tol_g = (1e-10, 1e-9) if dtype == "c128" else (1e-5, 1e-4)
    for n, edges, p in cases:
        rng = np.random.default_rng(n * 10 + p)
        g, b = rng.uniform(0, np.pi, p), rng.uniform(0, np.pi, p)
        for order in ("min_degree", "min_fill"):
            net = make(n, edges, p, dtype, order, g, b)
            e, dg, db = net.energy_grad(mode)
            e_ref, dg_ref, db_ref = sv.energy_grad_adjoint(n, edges, g, b)
            assert abs(e - e_ref) <= tol_e * max(1.0, abs(e_ref)), (n, p, order)
            np.testing.assert_allclose(dg, dg_ref, atol=tol_g * max(1.0, np.abs(dg_ref).max()))
            np.testing.assert_allclose(db, db_ref, atol=tol_g * max(1.0, np.abs(db_ref).max()))
            zz = net.edge_results()
            np.testing.assert_allclose(zz, sv.zz_expectations(n, edges, g, b), atol=tol_e)


def test_special_values_and_empty_graph():
    from paper_2106_15740_amd import QaoaNet

    w = workload("p2_n60")
    net = make(w.n, w.edges, w.p, "c64", "min_fill", [0.0, 0.0], w.beta)
    for mode in MODES:
        assert abs(net.energy(mode) - len(w.edges) / 2) < 1e-5 * len(w.edges)
    net = QaoaNet(6, [], 2, dtype="c64", device=0)
    net.set_params([0.3, 0.2], [0.1, 0.4])
    for mode in MODES:
        e, dg, db = net.energy_grad(mode)
        assert e == 0.0 and np.all(dg == 0) and np.all(db == 0)


@pytest.mark.parametrize("order", ["min_fill", "min_degree"])
def test_config3_p3_n244_batched_vs_tn_oracle(order):
    w = workload("p3_n244")
    net = make(w.n, w.edges, w.p, "c64", order, w.gamma, w.beta)
    e_b, dg_b, db_b = net.energy_grad("batched")
    zz = net.edge_results()
    ref = np.array([tn.zz_edge(w.n, w.edges, w.gamma, w.beta, j, k) for j, k in w.edges])
    np.testing.assert_allclose(zz, ref, atol=1e-5)
    e_ref = float(np.sum(0.5 * (1 - ref.real)))
    assert abs(e_b - e_ref) <= 1e-5 * e_ref
    e_p, dg_p, db_p = net.energy_grad("plain")
    assert abs(e_p - e_b) <= 1e-5 * e_ref
    np.testing.assert_allclose(dg_p, dg_b, rtol=1e-4, atol=1e-3)
    np.testing.assert_allclose(db_p, db_b, rtol=1e-4, atol=1e-3)


def test_config3_tree_like_edges_share_one_value():
    w = workload("p3_n244")
    net = make(w.n, w.edges, w.p, "c128", "min_fill", w.gamma, w.beta)
    net.energy("batched")
    zz = net.edge_results()
    st = net.cone_stats()
    tree = st["n_qubits"] == 30
    assert tree.sum() > 10
    assert np.ptp(zz[tree].real) < 1e-12
    ref = tn.zz_edge(w.n, w.edges, w.gamma, w.beta, *w.edges[int(np.argmax(tree))])
    assert abs(zz[tree][0] - ref) < 1e-10


def test_config4_gradient_subgraph_statevector():
    """p = 4 gradient on the N=16 BFS subgraph of the N=100 graph against the
    state-vector adjoint gradient, c64 and c128."""
    w = workload("p4_n100")
    n, edges = bfs_subgraph(w.n, w.edges, 16)
    e_ref, dg_ref, db_ref = sv.energy_grad_adjoint(n, edges, w.gamma, w.beta)
    for dtype, tol in (("c128", 1e-9), ("c64", 1e-4)):
        for mode in MODES:
            net = make(n, edges, w.p, dtype, "min_fill", w.gamma, w.beta)
            e, dg, db = net.energy_grad(mode)
            assert abs(e - e_ref) <= (1e-10 if dtype == "c128" else 1e-5) * abs(e_ref)
            np.testing.assert_allclose(dg, dg_ref, atol=tol * max(1, np.abs(dg_ref).max()))
            np.testing.assert_allclose(db, db_ref, atol=tol * max(1, np.abs(db_ref).max()))


def test_config4_gradient_vs_finite_differences():
    """p = 4, N = 100: c64 adjoint gradient against central differences of the
    c128 energy (h = 1e-4) computed through the library."""
    w = workload("p4_n100")
    net64 = make(w.n, w.edges, w.p, "c64", "min_fill", w.gamma, w.beta)
    e, dg, db = net64.energy_grad("batched")
    net128 = make(w.n, w.edges, w.p, "c128", "min_fill", w.gamma, w.beta)

    def f(g, b):
        net128.set_params(g, b)
        return net128.energy("batched")

    e128 = f(w.gamma, w.beta)
    assert abs(e - e128) <= 1e-5 * abs(e128)
    fg, fb = sv.energy_grad_fd(f, w.gamma, w.beta, h=1e-4)
    net128.set_params(w.gamma, w.beta)
    _, dg128, db128 = net128.energy_grad("batched")
    np.testing.assert_allclose(dg128, fg, atol=1e-6 * max(1, np.abs(fg).max()) + 2e-6)
    np.testing.assert_allclose(db128, fb, atol=1e-6 * max(1, np.abs(fb).max()) + 2e-6)
    np.testing.assert_allclose(dg, dg128, atol=1e-4 * max(1, np.abs(dg128).max()))
    np.testing.assert_allclose(db, db128, atol=1e-4 * max(1, np.abs(db128).max()))


def test_config4_sampled_edges_vs_tn_oracle():
    w = workload("p4_n100")
    net = make(w.n, w.edges, w.p, "c128", "min_fill", w.gamma, w.beta)
    net.energy("batched")
    zz = net.edge_results()
    for e in (0, 77):
        ref = tn.zz_edge(w.n, w.edges, w.gamma, w.beta, *w.edges[e])
        assert abs(zz[e] - ref) < 1e-10


def test_autograd_function():
    from paper_2106_15740_amd import qaoa_energy

    w = workload("p1_n10")
    net = make(w.n, w.edges, 2, "c128", "min_degree", [0.4, 0.2], [0.3, 0.1])
    g = torch.tensor([0.4, 0.2], dtype=torch.float64, requires_grad=True)
    b = torch.tensor([0.3, 0.1], dtype=torch.float64, requires_grad=True)
    e = qaoa_energy(g, b, net)
    (2.0 * e).backward()
    e_ref, dg_ref, db_ref = sv.energy_grad_adjoint(w.n, w.edges, [0.4, 0.2], [0.3, 0.1])
    assert abs(e.item() - e_ref) < 1e-10 * e_ref
    np.testing.assert_allclose(g.grad.numpy(), 2 * dg_ref, atol=1e-9)
    np.testing.assert_allclose(b.grad.numpy(), 2 * db_ref, atol=1e-9)
    # angles on the GPU: energy and gradients stay on the GPU
    g = torch.tensor([0.4, 0.2], dtype=torch.float64, device="cuda:0", requires_grad=True)
    b = torch.tensor([0.3, 0.1], dtype=torch.float64, device="cuda:0", requires_grad=True)
    e = qaoa_energy(g, b, net)
    assert e.device == g.device
    (3.0 * e).backward()
    assert g.grad.device == g.device and b.grad.device == b.device
    np.testing.assert_allclose(g.grad.cpu().numpy(), 3 * dg_ref, atol=1e-9)
    np.testing.assert_allclose(b.grad.cpu().numpy(), 3 * db_ref, atol=1e-9)


def test_graph_replay_and_param_refresh():
    """The batched sweep is a captured hipGraph: replays with new angles and
    with the program's own work in between must all match the oracle."""
    w = workload("p2_n60")
    net = make(w.n, w.edges, w.p, "c64", "min_fill", w.gamma, w.beta)
    rng = np.random.default_rng(5)
    for it in range(4):
        g, b = rng.uniform(0, np.pi, 2), rng.uniform(0, np.pi, 2)
        net.set_params(g, b)
        e = net.energy_grad("batched")[0]
        x = torch.randn(1 << 16, device="cuda").sum().item()  # unrelated eager work between replays
        ref = sum(0.5 * (1 - ball.zz_edge(w.n, w.edges, g, b, j, k).real) for j, k in w.edges[:: 9])
        zz = net.edge_results()[:: 9]
        assert abs(sum(0.5 * (1 - zz.real)) - ref) < 1e-4, (it, x)
        assert np.isfinite(e)


def test_forced_split_buckets_and_atomics():
    """Force every bucket wider than 4 union bits through the multi-workgroup
    tile items, with partial sums spilled to atomics."""
    w = workload("p3_n244")
    edges = w.edges[:40]
    n = w.n
    ref = np.array([tn.zz_edge(n, edges, w.gamma, w.beta, j, k) for j, k in edges])
    for tune in (dict(seq_max_bits=4, loop_cap=1, tile_blocks=2), dict(seq_max_bits=6, loop_cap=0, lane_cap=3)):
        net = make(n, edges, w.p, "c128", "min_fill", w.gamma, w.beta, **tune)
        for mode in MODES:
            e, dg, db = net.energy_grad(mode)
            np.testing.assert_allclose(net.edge_results(), ref, atol=1e-10)
            if mode == "plain":
                dgp, dbp = dg, db
        np.testing.assert_allclose(dg, dgp, atol=1e-10)
        np.testing.assert_allclose(db, dbp, atol=1e-10)


@pytest.mark.parametrize("lds_kb,lds_threads", [(0, 256), (16, 256), (64, 256), (64, 64), (64, 512)])
def test_lds_resident_and_global_sweeps_agree(lds_kb, lds_threads):
    """The batched sweep keeps a cone in an LDS window when its program fits
    (lds_kb), run by 1 to 8 wavefronts; every window size and workgroup must
    give the oracle's values."""
    w = workload("p3_n244")
    edges = w.edges[:60]
    ref = np.array([tn.zz_edge(w.n, edges, w.gamma, w.beta, j, k) for j, k in edges])
    net = make(w.n, edges, w.p, "c128", "min_fill", w.gamma, w.beta, lds_kb=lds_kb, lds_threads=lds_threads)
    e, dg, db = net.energy_grad("batched")
    np.testing.assert_allclose(net.edge_results(), ref, atol=1e-10)
    e2, dg2, db2 = net.energy_grad("plain")
    assert abs(e - e2) < 1e-10 * abs(e)
    np.testing.assert_allclose(dg, dg2, atol=1e-9)
    np.testing.assert_allclose(db, db2, atol=1e-9)


@pytest.mark.parametrize("mode", MODES)
def test_checkpointed_adjoint_under_memory_budget(mode):
    """Under a workspace budget the cones share their dynamic regions
    (admission in queue order) and, below one cone's own region, the adjoint
    sweep recomputes dropped bucket outputs; energy, gradient and edge terms
    must still match the state vector (p = 3 on a 12-vertex 3-regular graph,
    min-fill order, width 15, LDS-resident programs off)."""
    n, edges = 12, random_regular_graph(12, 3, 3)
    rng = np.random.default_rng(3)
    g, b = rng.uniform(0, np.pi, 3), rng.uniform(0, np.pi, 3)
    e_ref, dg_ref, db_ref = sv.energy_grad_adjoint(n, edges, g, b)
    zz_ref = sv.zz_expectations(n, edges, g, b)
    net = make(n, edges, 3, "c128", "min_fill", g, b, lds_kb=0)
    full = net.info()
    budgets = [max(int(0.5 * full["arena_keep_all"]), full["pinned_bytes"] + full["max_cone_dynamic"]),
               lowest_recompute_budget(net)]
    for k, budget in enumerate(budgets):
        net.set_memory_budget(budget)
        info = net.info()
        assert info["ws_grad"] <= budget + (1 << 16)
        assert (info["n_recomputed"] > 0) == (k == 1)
        print(f"[case] budget {budget} recomputed {info['n_recomputed']}", flush=True)
        for _ in range(2):
            e, dg, db = net.energy_grad(mode)
            assert abs(e - e_ref) <= 1e-10 * abs(e_ref)
            np.testing.assert_allclose(dg, dg_ref, atol=1e-9)
            np.testing.assert_allclose(db, db_ref, atol=1e-9)
        np.testing.assert_allclose(net.edge_results(), zz_ref, atol=1e-10)


@pytest.mark.parametrize("case", ["p3_edges", "p4_wide", "p4_wide_budget"])
def test_one_workgroup_fifo_sweep_matches_plain(case):
    """grid = 1: a single persistent workgroup takes the queue's items in
    order, so no item ever waits and the queue's order alone must be a valid
    schedule (every dependency earlier in the queue).  Its energy, gradient and
    edge terms must equal the plain per-op loop's (complex128, 1e-12), also for
    split buckets with atomics (p = 4, seq_max_bits 9) and under a memory
    budget whose cones share regions; a second run agrees to rounding."""
    w = workload("p3_n244" if case == "p3_edges" else "p4_n100")
    edges = w.edges[:100] if case == "p3_edges" else w.edges
    tune = dict(lds_kb=0) if case == "p3_edges" else dict(lds_kb=0, seq_max_bits=9, lane_cap=6, tile_blocks=64)
    net = make(w.n, edges, w.p, "c128", "min_degree", w.gamma, w.beta, **tune)
    if case == "p4_wide_budget":
        full = net.info()
        net.set_memory_budget(lowest_recompute_budget(net))
        assert net.info()["n_recomputed"] > 0
    e_p, dg_p, db_p = net.energy_grad("plain")
    zz_p = net.edge_results()
    net.set_tuning(grid=1)
    runs = []
    for _ in range(2):
        e, dg, db = net.energy_grad("batched")
        runs.append((e, dg, db, net.edge_results()))
    e, dg, db, zz = runs[0]
    assert abs(e - e_p) <= 1e-12 * abs(e_p)
    np.testing.assert_allclose(dg, dg_p, rtol=0, atol=1e-12 * max(1, np.abs(dg_p).max()))
    np.testing.assert_allclose(db, db_p, rtol=0, atol=1e-12 * max(1, np.abs(db_p).max()))
    np.testing.assert_allclose(zz, zz_p, rtol=0, atol=1e-12)
    np.testing.assert_allclose(runs[1][3], zz, rtol=0, atol=1e-13)
    e_f = net.energy("batched")
    assert abs(e_f - e_p) <= 1e-12 * abs(e_p)


@pytest.mark.parametrize("dtype,tol", [("c64", 1e-5), ("c128", 1e-10)])
def test_wide_executor_plain_and_batched(dtype, tol):
    """Buckets wider than seq_max_bits run in the wide-op executor (its own
    launches in the plain loop; tiles inside the persistent sweep, with fewer
    outputs per thread).  A low seq_max_bits sends most buckets of p = 4 light
    cones there, with reductions over lanes, loops and blocks; the gradient
    with one adjoint pass per input matches the fused adjoint's, the
    LDS-tiled adjoint's (fuse_adjoint = 2) and the outer-product adjoint's
    (fuse_adjoint = 3)."""
    w = workload("p4_n100")
    net = make(w.n, w.edges, w.p, dtype, "min_fill", w.gamma, w.beta, seq_max_bits=9, lane_cap=6, tile_blocks=64)
    net_sep = make(w.n, w.edges, w.p, dtype, "min_fill", w.gamma, w.beta, seq_max_bits=9, lane_cap=6, tile_blocks=64,
                   fuse_adjoint=0, lane_low=0)
    _, dg_s, db_s = net_sep.energy_grad("batched")
    del net_sep
    net_tile = make(w.n, w.edges, w.p, dtype, "min_fill", w.gamma, w.beta, seq_max_bits=9, lane_cap=6,
                    tile_blocks=64, fuse_adjoint=2)
    _, dg_t, db_t = net_tile.energy_grad("batched")
    _, dg_tp, db_tp = net_tile.energy_grad("plain")
    del net_tile
    net_outer = make(w.n, w.edges, w.p, dtype, "min_fill", w.gamma, w.beta, seq_max_bits=9, lane_cap=6,
                     tile_blocks=64, fuse_adjoint=3)
    _, dg_o, db_o = net_outer.energy_grad("batched")
    _, dg_op, db_op = net_outer.energy_grad("plain")
    del net_outer
    ref = np.array([tn.zz_edge(w.n, w.edges, w.gamma, w.beta, j, k) for j, k in w.edges[:3]])
    e_p, dg_p, db_p = net.energy_grad("plain")
    zz_p = net.edge_results()
    e_b, dg_b, db_b = net.energy_grad("batched")
    zz_b = net.edge_results()
    np.testing.assert_allclose(zz_p[:3], ref, atol=tol)
    np.testing.assert_allclose(zz_b[:3], ref, atol=tol)
    np.testing.assert_allclose(zz_b, zz_p, atol=tol)
    assert abs(e_b - e_p) <= tol * abs(e_p)
    gt = 1e-4 if dtype == "c64" else 1e-9
    np.testing.assert_allclose(dg_b, dg_p, atol=gt * max(1, np.abs(dg_p).max()))
    np.testing.assert_allclose(db_b, db_p, atol=gt * max(1, np.abs(db_p).max()))
    np.testing.assert_allclose(dg_b, dg_s, atol=gt * max(1, np.abs(dg_s).max()))
    np.testing.assert_allclose(db_b, db_s, atol=gt * max(1, np.abs(db_s).max()))
    for dg_x, db_x in ((dg_t, db_t), (dg_tp, db_tp), (dg_o, db_o), (dg_op, db_op)):
        np.testing.assert_allclose(dg_x, dg_s, atol=gt * max(1, np.abs(dg_s).max()))
        np.testing.assert_allclose(db_x, db_s, atol=gt * max(1, np.abs(db_s).max()))


@pytest.mark.parametrize("dtype,tol", [("c64", 1e-4), ("c128", 1e-9)])
@pytest.mark.parametrize("lane_low", [0, 1])
def test_fused_adjoint_gradient_vs_statevector(dtype, tol, lane_low):
    """Buckets wider than seq_max_bits compute all input adjoints in one pass
    (fuse_adjoint = 1; 2 also sums the other buckets tile by tile in LDS; 3
    sums outer-product buckets in register slots, complex64 only) or one pass
    per input (0).  All, with either lane policy, plain and batched, give the
    state-vector adjoint gradient of the p = 4, N = 16 BFS subgraph; each
    fused plan has fewer ops."""
    w = workload("p4_n100")
    n, edges = bfs_subgraph(w.n, w.edges, 16)
    e_ref, dg_ref, db_ref = sv.energy_grad_adjoint(n, edges, w.gamma, w.beta)
    n_ops = {}
    for fuse in (0, 1, 2, 3):
        net = make(n, edges, w.p, dtype, "min_fill", w.gamma, w.beta, seq_max_bits=7, merge_bits=0, threads=64,
                   lane_cap=6, tile_blocks=64, lane_low=lane_low, fuse_adjoint=fuse)
        n_ops[fuse] = net.info()["n_ops_grad"]
        for mode in MODES:
            e, dg, db = net.energy_grad(mode)
            assert abs(e - e_ref) <= (1e-10 if dtype == "c128" else 1e-5) * abs(e_ref), (fuse, mode)
            np.testing.assert_allclose(dg, dg_ref, atol=tol * max(1, np.abs(dg_ref).max()))
            np.testing.assert_allclose(db, db_ref, atol=tol * max(1, np.abs(db_ref).max()))
    assert n_ops[2] < n_ops[1] < n_ops[0]
    if dtype == "c64":
        assert n_ops[3] < n_ops[1]


def test_optimisation_driver_reaches_the_p1_optimum():
    """Adam over the library's energy and adjoint gradient on config 1 (p = 1)
    climbs to the maximum of the oracle's energy landscape (dense grid over
    gamma, beta of the state vector), and the final point's energy matches the
    state vector there."""
    from paper_2106_15740_amd import maximize_cut

    w = workload("p1_n10")
    net = make(w.n, w.edges, 1, "c128", "min_degree", [0.1], [0.1])
    res = maximize_cut(net, [0.1], [0.1], steps=150, lr=0.05)
    assert res.history[-1] > res.history[0] + 1.0
    e_ref = sv.energy(w.n, w.edges, res.gamma, res.beta)
    assert abs(res.energy - e_ref) <= 1e-10 * abs(e_ref)
    # the landscape's maximum on a grid (one period in beta, half a period in gamma)
    gs, bs = np.linspace(0, np.pi, 61), np.linspace(0, np.pi / 2, 31)
    best = max(sv.energy(w.n, w.edges, [g], [b]) for g in gs for b in bs)
    assert res.energy >= best - 1e-3


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_single_amplitude_vs_statevector(mode, dtype):
    """<0...0|gamma beta> of whole graphs (the paper's benchmark network)
    against the state vector, p = 1..3, and its derivative from the adjoint
    sweep against central differences of the state-vector amplitude."""
    from paper_2106_15740_amd import QaoaAmplitude

    tol = 1e-12 if dtype == "c128" else 1e-6  # |amplitude| ~ 2^(-N/2)
    for n, seed, p in ((10, 0, 1), (12, 1, 2), (14, 2, 3)):
        edges = random_regular_graph(n, 3, seed)
        rng = np.random.default_rng(seed + 40)
        g, b = rng.uniform(0, np.pi, p), rng.uniform(0, np.pi, p)
        print(f"[case] amplitude n={n} p={p} {dtype} {mode}", flush=True)
        net = QaoaAmplitude(n, edges, p, dtype=dtype, order="min_fill", device=0)
        net.set_params(g, b)
        ref = sv.amplitude(n, edges, g, b)
        assert abs(net.amplitude(mode) - ref) <= tol
        a, dg, db = net.amplitude_grad(mode)
        assert abs(a - ref) <= tol
        h = 1e-5
        for l in range(p):
            for arr, d in ((g, dg), (b, db)):
                arr[l] += h
                up = sv.amplitude(n, edges, g, b)
                arr[l] -= 2 * h
                dn = sv.amplitude(n, edges, g, b)
                arr[l] += h
                fd = (up - dn) / (2 * h)
                assert abs(d[l] - fd) <= (1e-8 if dtype == "c128" else 1e-5), (l, d[l], fd)


def test_sweep_timing_is_opt_in():
    """Batched sweeps record their timing events only while sweep timing is
    on; the results do not depend on it."""
    w = workload("p3_n244")
    edges = w.edges[:24]
    net = make(w.n, edges, w.p, "c64", "min_fill", w.gamma, w.beta)
    e0, dg0, db0 = net.energy_grad("batched")
    net.kernel_time(reset=True)
    for _ in range(3):
        net.energy_grad("batched")
    assert net.kernel_time(reset=True) == (0.0, 0)
    net.set_sweep_timing(True)
    for _ in range(3):
        e1, dg1, db1 = net.energy_grad("batched")
    ms, cnt = net.kernel_time(reset=True)
    net.set_sweep_timing(False)
    assert cnt == 3 and ms > 0
    assert e1 == e0
    # (leaf gradients meet in atomics, so their order of addition may differ)
    np.testing.assert_allclose(dg1, dg0, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(db1, db0, rtol=1e-12, atol=1e-12)
