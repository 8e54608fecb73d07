"""GPU parity at the benchmarked sizes, against expected values the CPU
oracle wrote (tests/golden/make_full_size.py: oracle.tn in complex128 for
every edge term, central differences h = 1e-4 for its derivatives;
oracle.statevector for the amplitude).

Tolerances (complex64 with FP32 accumulation): per-edge <Z_j Z_k> within 1e-5
absolute (|<ZZ>| <= 1 and may be ~0); E within 1e-5 relative; each edge's
derivatives d<ZZ>/d(gamma_l, beta_l) within 1e-4 of that edge's largest
derivative (the central-difference truncation, ~h^2/6 |f'''| ~ 1e-9, is far
below); dE/dtheta within 1e-4 of its largest component.  The imaginary parts
of <ZZ> and of its derivatives vanish mathematically and are held to the same
bounds.
"""
import os

import numpy as np
import pytest

from workloads import random_angles, random_regular_graph, workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def load_edges(name):
    """(zz [m] complex, dzz {edge: [2p] real}) from full_size_<name>.txt."""
    zz, dzz = [], {}
    with open(os.path.join(GOLDEN, f"full_size_{name}.txt")) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            f = line.split()
            i = int(f[0])
            assert i == len(zz)
            zz.append(float(f[4]) + 1j * float(f[5]))
            if len(f) > 6:
                dzz[i] = np.array([float(x) for x in f[6:]])
    return np.array(zz), dzz


def load_amplitude(n, p):
    vals = {}
    with open(os.path.join(GOLDEN, f"amplitude_n{n}_p{p}.txt")) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            k, re, im = line.split()
            vals[k] = float(re) + 1j * float(im)
    return vals


def net_for(name, order, repeats=0, dtype="c64", **tune):
    from paper_2106_15740_amd import QaoaNet

    w = workload(name)
    print(f"[case] {name} {dtype} {order} repeats={repeats} {tune}", flush=True)
    net = QaoaNet(w.n, w.edges, w.p, dtype=dtype, order=order, device=0, repeats=repeats)
    if tune:
        net.set_tuning(**tune)
    net.set_params(w.gamma, w.beta)
    return w, net


def check_against_golden(name, net, mode="batched", width_report=False):
    """Energy, gradient and every edge term of one sweep against the oracle's
    values; returns the largest <ZZ> error per contraction width."""
    zz_ref, dzz_ref = load_edges(name)
    e, dg, db = net.energy_grad(mode)
    zz, dzz = net.edge_results(with_grad=True)
    assert zz.shape == zz_ref.shape
    err = np.abs(zz - zz_ref)
    assert err.max() <= 1e-5, (name, mode, int(err.argmax()), err.max())
    assert np.abs(zz.imag).max() <= 1e-5
    e_ref = float(np.sum(0.5 * (1.0 - zz_ref.real)))
    assert abs(e - e_ref) <= 1e-5 * abs(e_ref), (name, mode, e, e_ref)
    for i, d_ref in dzz_ref.items():
        scale = np.abs(d_ref).max()
        np.testing.assert_allclose(dzz[i].real, d_ref, rtol=0, atol=1e-4 * scale, err_msg=f"{name} edge {i}")
        assert np.abs(dzz[i].imag).max() <= 1e-4 * scale
    if len(dzz_ref) == len(zz_ref):  # every edge has oracle derivatives: the whole gradient too
        p = net.p
        grad_ref = -0.5 * np.sum(np.array([dzz_ref[i] for i in range(len(zz_ref))]), axis=0)
        scale = np.abs(grad_ref).max()
        np.testing.assert_allclose(dg, grad_ref[:p], rtol=0, atol=1e-4 * scale)
        np.testing.assert_allclose(db, grad_ref[p:], rtol=0, atol=1e-4 * scale)
    per_width = {}
    if width_report:
        width = net.cone_stats()["width"]
        for wv in sorted(set(width.tolist())):
            per_width[wv] = float(err[width == wv].max())
        print(f"[{name}] max |<ZZ> - oracle| by width: {per_width}", flush=True)
    return per_width


@pytest.mark.parametrize("order,mode", [("min_fill", "batched"), ("min_fill", "plain"), ("min_degree", "batched")])
def test_p3_n244_every_edge_and_gradient_vs_oracle(order, mode):
    """The headline workload (p = 3, N = 244, 366 edges) in the benchmark's
    order (10 randomized greedy repeats): every edge term and every edge's
    derivatives against the oracle, and E, dE/dgamma, dE/dbeta."""
    _, net = net_for("p3_n244", order, repeats=10)
    check_against_golden("p3_n244", net, mode, width_report=True)


def test_p3_n244_autotuned_plan_vs_oracle():
    """The tile shapes the benchmark times come from the autotuner: its choice
    passes the same comparison."""
    _, net = net_for("p3_n244", "min_fill", repeats=10)
    tuned = net.autotune(with_grad=True)
    print(f"[tuned] {tuned}", flush=True)
    check_against_golden("p3_n244", net, "batched")
    check_against_golden("p3_n244", net, "plain")


def test_p4_n100_band_autotuned_and_cached_plan_vs_oracle(tmp_path):
    """The global and per-band autotuners (tunecache.tuned) pick the tiles of
    the p = 4 workload and store them under (architecture, dtype, plan
    signature); a second net of the same plan takes them from the cache.  Both
    plans pass the full comparison with the oracle."""
    from paper_2106_15740_amd import tunecache

    path = str(tmp_path / "tune.json")
    _, net = net_for("p4_n100", "min_fill")
    e = tunecache.tuned(net, with_grad=True, path=path)
    print(f"[tuned] {e}", flush=True)
    assert e["source"] == "search" and e["stored"]
    check_against_golden("p4_n100", net, "batched")
    _, net2 = net_for("p4_n100", "min_fill")
    e2 = tunecache.tuned(net2, with_grad=True, path=path, search=False)
    assert e2["source"] == "cache" and e2["key"] == e["key"]
    assert net2.tuning() == net.tuning() and net2.band_tuning() == net.band_tuning()
    check_against_golden("p4_n100", net2, "batched")


def test_p4_n100_every_edge_vs_oracle():
    """p = 4, N = 100 (150 edges, widths up to 22): every edge term and, for
    one edge per oracle width, its derivatives."""
    _, net = net_for("p4_n100", "min_fill")
    check_against_golden("p4_n100", net, "batched", width_report=True)


def test_p5_n1000_every_edge_vs_oracle_and_symmetries():
    """p = 5, N = 1000 (1500 edges) at full size, in the launch configuration
    the benchmark times (min-degree randomized greedy with 10 repeats, widths
    up to 26; seq_max_bits 16, tile_blocks 128, par_bits 21; fused adjoints):
    every edge term against the oracle at 1e-5, derivatives of one edge per
    oracle width, the energy, and two symmetries of the whole energy: beta_1 +
    pi/2 and (gamma, beta) -> (-gamma, -beta), under which the gradient flips
    sign."""
    w, net = net_for("p5_n1000", "min_degree", repeats=10, seq_max_bits=16, tile_blocks=128, par_bits=21)
    assert net.cone_stats()["width"].max() >= 26
    check_against_golden("p5_n1000", net, "batched", width_report=True)
    e, dg, db = net.energy_grad("batched")
    shift = np.zeros(w.p)
    shift[0] = np.pi / 2
    net.set_params(w.gamma, w.beta + shift)
    assert abs(net.energy("batched") - e) <= 1e-5 * abs(e)
    net.set_params(-w.gamma, -w.beta)
    e2, dg2, db2 = net.energy_grad("batched")
    assert abs(e2 - e) <= 1e-5 * abs(e)
    scale = max(np.abs(dg).max(), np.abs(db).max())
    np.testing.assert_allclose(dg2, -dg, rtol=0, atol=1e-4 * scale)
    np.testing.assert_allclose(db2, -db, rtol=0, atol=1e-4 * scale)


@pytest.mark.parametrize("share", [0.25, 0.0])
def test_p5_n1000_under_a_memory_budget(share):
    """The p = 5 workload of the benchmark under a workspace budget: a quarter
    of the keep-everything arena (cones admitted into a shared area), and
    (share 0) just below the largest cone's own working set (the lowest share
    of it the planner meets), so that cone recomputes dropped outputs in its
    adjoint sweep.  Every edge term and the
    sampled derivatives against the oracle, as without a budget."""
    from paper_2106_15740_amd import QtnError

    w, net = net_for("p5_n1000", "min_degree", repeats=10, seq_max_bits=16, tile_blocks=128, par_bits=21)
    full = net.info()
    if share > 0:
        budget = int(share * full["arena_keep_all"])
        net.set_memory_budget(budget)
    else:
        # the lowest of these shares of the largest cone's region that the
        # planner can meet by recomputation
        for f in (0.9, 0.95, 0.98, 0.99, 0.999):
            budget = full["pinned_bytes"] + int(f * full["max_cone_dynamic"])
            try:
                net.set_memory_budget(budget)
                break
            except QtnError:
                continue
    info = net.info()
    print(f"[budget] {budget / 1e9:.2f} GB of {full['arena_keep_all'] / 1e9:.2f} GB keep-all: workspace "
          f"{info['ws_grad'] / 1e9:.2f} GB, {info['n_recomputed']} outputs recomputed", flush=True)
    assert info["ws_grad"] <= budget + (1 << 20) and info["ws_grad"] <= 0.5 * full["arena_keep_all"]
    assert (info["n_recomputed"] > 0) == (share == 0)
    check_against_golden("p5_n1000", net, "batched")


@pytest.mark.parametrize("order", ["min_fill", "min_degree"])
def test_amplitude_n22_p4_wide_vs_statevector(order):
    """The single amplitude <0...0|gamma beta> of a 22-vertex graph at p = 4
    (widths 22 and 24: the wide-op executor on an amplitude network) with the
    benchmark leg's tiles, against the oracle's state vector; derivatives
    against its central differences.  Relative tolerance 1e-4 of |amp| (and
    of the largest derivative): the amplitude is a sum of ~2^22 unit-modulus
    paths that cancel down to |amp| ~ 2^-11, so the complex64 rounding error
    relative to |amp| is larger than for the edge terms."""
    from paper_2106_15740_amd import QaoaAmplitude

    n, p = 22, 4
    edges = random_regular_graph(n, 3, 0)
    g, b = random_angles(p, 5)
    ref = load_amplitude(n, p)
    print(f"[case] amplitude n={n} p={p} {order}", flush=True)
    net = QaoaAmplitude(n, edges, p, dtype="c64", order=order, device=0)
    net.set_tuning(seq_max_bits=14, tile_blocks=64, par_bits=21)
    assert net.max_width >= 22
    net.set_params(g, b)
    a = net.amplitude("batched")
    assert abs(a - ref["amplitude"]) <= 1e-4 * abs(ref["amplitude"]), (a, ref["amplitude"])
    a2, dg, db = net.amplitude_grad("batched")
    assert abs(a2 - ref["amplitude"]) <= 1e-4 * abs(ref["amplitude"])
    d_ref = np.array([ref[f"d_gamma_{l + 1}"] for l in range(p)] + [ref[f"d_beta_{l + 1}"] for l in range(p)])
    d = np.concatenate([dg, db])
    scale = np.abs(d_ref).max()
    assert np.abs(d - d_ref).max() <= 1e-4 * scale, (d, d_ref)
