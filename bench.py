"""Benchmark: QAOA-MaxCut light cones per second (energy + gradient), p = 3.

Headline workload: seeded random 3-regular graph, N = 244 vertices (366
edges), QAOA depth p = 3, angles ~ U(0, pi), complex64 with FP32 accumulation,
min-fill randomized greedy order (10 repeats).  One step = one forward sweep of
every edge's light-cone network plus the adjoint sweep (energy, dE/dgamma,
dE/dbeta) in the batched form: one persistent launch over a device work
queue, replayed from a hipGraph, tile shapes from the library's autotuner.
The plan and leaf tables are resident in HBM before timing starts; each step
re-uploads the 4p+2 leaf values (a few hundred bytes) as the sweep's first
node and reads back 1 + 2p doubles.

Prints one JSON line.  Beside the headline it reports: the plain per-edge
loop (one launch per bucket step) on the same GPU; the roofline of the
persistent kernel (latency-bound at p = 3); the p = 5, N = 1000 workload
(throughput and HBM fraction of the whole sweep) with the roofline of its
buckets of width >= 20 measured inside a persistent launch; one single
amplitude of a 40-vertex graph at p = 4; and the CPU oracle timed on a bounded
sample of edges.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
P5_TIMED_MAX_WIDTH = 23  # widest oracle contraction timed in the p = 5 CPU extrapolation
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic_small_kernel_p3_n244.json")
P5_TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic_persistent_kernel_p5_n1000.json")


def log(msg: str) -> None:
    """A progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2106_15740_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if not f.endswith((".hip", ".hpp", ".cpp")) or f == "api.cpp":
            continue
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(path=TRAFFIC_JSON, tuning=None, bands=None):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    runs, only while the kernel sources (and the tile shapes) are the ones
    they were taken with."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    if tuning is not None and t.get("tuning") not in (None, tuning):
        return None
    if bands is not None and t.get("band_tuning") not in (None, bands):
        return None
    return t.get("bytes_per_launch")


def host_cores() -> int:
    """Worker processes for the CPU oracle: the CPUs this process may run on,
    at most 16 (one GPU's share of the host)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(avail, 16))


def _pool_rate(fn, args_list, cores, budget_s):
    """Edge light cones per second of fn over args_list (cycled) on `cores`
    worker processes for about budget_s seconds."""
    import concurrent.futures as cf
    import multiprocessing as mp

    t0 = time.perf_counter()
    done = 0
    with cf.ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("fork")) as ex:
        i = 0
        while (time.perf_counter() - t0) < budget_s:
            batch = [ex.submit(fn, *args_list[(i + k) % len(args_list)]) for k in range(cores)]
            for f in batch:
                f.result()
            done += len(batch)
            i += cores
    return done, time.perf_counter() - t0


def cpu_baseline(w, budget_s: float = 12.0):
    """The CPU oracle as it stands, timed on this host: oracle.tn's tensor-network
    contraction (numpy einsum bucket elimination, complex128) of the edge
    terms, with the gradient by central differences (4p + 1 contractions per
    edge, the oracle's only gradient at this size), one process per core, in
    passes over the edges in a seeded order; plus the same with complex64
    storage, the forward contraction alone, one core, the oracle's state
    vector on the small workloads, and the p = 5, N = 1000 workload from a
    timed sample of edges."""
    import numpy as np

    from oracle import ball, statevector as sv
    from workloads import bfs_subgraph, workload as wl

    cores = host_cores()
    rng = np.random.default_rng(0)
    order = rng.permutation(len(w.edges))
    h = 1e-4
    args = [(w.n, w.edges, w.gamma, w.beta, w.edges[int(e)], h, "c128") for e in order]
    done, dt = _pool_rate(_oracle_edge_grad, args, cores, budget_s)
    args64 = [a[:-1] + ("c64",) for a in args]
    done64, dt64 = _pool_rate(_oracle_edge_grad, args64, cores, budget_s / 3)
    fwd_args = [a[:5] for a in args]
    donef, dtf = _pool_rate(_oracle_edge_fwd, fwd_args, cores, budget_s / 3)
    # the same work on one core, for a few seconds
    t1 = time.perf_counter()
    one = 0
    while time.perf_counter() - t1 < min(4.0, budget_s / 3):
        _oracle_edge_grad(*args[one % len(args)])
        one += 1
    dt1 = time.perf_counter() - t1
    # the state vector (the oracle's definition) where it fits: config 1, the
    # N = 16 subgraph of the p = 4 workload, and the radius-p ball of every
    # edge of the p = 2 workload (energy and, where defined, adjoint gradient)
    sv_times = {}
    w1 = wl("p1_n10")
    t = time.perf_counter()
    sv.energy_grad_adjoint(w1.n, w1.edges, w1.gamma, w1.beta)
    sv_times["p1_n10_energy_grad_s"] = time.perf_counter() - t
    w4 = wl("p4_n100")
    n16, e16 = bfs_subgraph(w4.n, w4.edges, 16)
    t = time.perf_counter()
    sv.energy_grad_adjoint(n16, e16, w4.gamma, w4.beta)
    sv_times["p4_n16_subgraph_energy_grad_s"] = time.perf_counter() - t
    w2 = wl("p2_n60")
    t = time.perf_counter()
    for j, k in w2.edges:
        ball.zz_edge(w2.n, w2.edges, w2.gamma, w2.beta, j, k)
    sv_times["p2_n60_ball_energy_s"] = time.perf_counter() - t
    # p = 5, N = 1000: the oracle's own contraction width of every edge (its
    # network and min-fill order, no contraction), one timed contraction of the
    # first edge of each width up to P5_TIMED_MAX_WIDTH, twice the time per
    # width above it (memory and work double per index), extrapolated to energy
    # + gradient (4p + 1 contractions) over all 1500 edges on `cores` cores
    import concurrent.futures as cf
    import multiprocessing as mp

    w5 = wl("p5_n1000")
    a5 = [(w5.n, w5.edges, w5.gamma, w5.beta, e) for e in w5.edges]
    t = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("fork")) as ex:
        widths = list(ex.map(_oracle_edge_width, a5, chunksize=8))
        classes = sorted(set(widths))
        timed_w = [c for c in classes if c <= P5_TIMED_MAX_WIDTH]
        picks = [a5[widths.index(c)] for c in timed_w]
        times = dict(zip(timed_w, ex.map(_oracle_edge_fwd_timed, picks)))
    dt5 = time.perf_counter() - t
    top = max(timed_w)
    per_w = {c: times[c] if c in times else times[top] * 2.0 ** (c - top) for c in classes}
    core_s = sum(per_w[c] for c in widths) * (4 * w5.p + 1)
    p5_sweep_s = core_s / cores
    return {"value": done / dt, "unit": "edge light-cones/s", "cores": cores, "kind": "oracle",
            "os_cpu_count": os.cpu_count(),
            "cores_note": "one worker process per CPU this process may use, capped at 16 (one GPU's share of the "
                          "host); os_cpu_count is what the machine reports",
            "sample": f"{done} edge light cones ({done / len(w.edges):.1f} passes over the {len(w.edges)} edges in a "
                      f"seeded order), numpy einsum bucket elimination in complex128, energy + gradient by central "
                      f"differences ({4 * w.p + 1} contractions per edge), {cores} worker processes, {dt:.1f} s",
            "gradient_method": f"central differences: {4 * w.p + 1} contractions per edge; one forward plus one "
                               f"adjoint would cost about 3, so the gradient inflates this baseline's time by "
                               f"about {(4 * w.p + 1) / 3:.1f}x",
            "forward_only": {"value": donef / dtf, "unit": "edge light-cones/s (energy only)",
                             "sample": f"{donef} forward contractions, complex128, {cores} processes, {dtf:.1f} s"},
            "c64": {"value": done64 / dt64, "unit": "edge light-cones/s",
                    "sample": f"{done64} edge light cones with complex64 tensors, {cores} processes, {dt64:.1f} s"},
            "single_core": {"value": one / dt1, "sample": f"{one} edge light cones on one core, {dt1:.1f} s"},
            "statevector_s": sv_times,
            "p5_n1000_extrapolated": {
                "sweep_s": p5_sweep_s, "edge_light_cones_per_s": len(w5.edges) / p5_sweep_s,
                "seconds_per_contraction_by_oracle_width": {str(c): per_w[c] for c in classes},
                "edges_by_oracle_width": {str(c): widths.count(c) for c in classes},
                "sample": f"the oracle's width of all {len(w5.edges)} edges; one complex128 contraction timed per "
                          f"width {min(timed_w)}..{top}, 2x per width above {top} (widths up to {max(classes)}); "
                          f"times {4 * w5.p + 1} contractions per edge over {cores} cores ({dt5:.1f} s of "
                          f"measurement): an extrapolation, not a run"}}


def _oracle_edge_fwd(n, edges, gamma, beta, edge):
    from oracle import tn

    return tn.zz_edge(n, edges, gamma, beta, *edge)


def _oracle_edge_width(a):
    from oracle import tn

    n, edges, gamma, beta, edge = a
    return tn.min_fill_order(tn.network(n, edges, gamma, beta, *edge))[1]


def _oracle_edge_fwd_timed(a):
    t = time.perf_counter()
    _oracle_edge_fwd(*a)
    return time.perf_counter() - t


def _oracle_edge_grad(n, edges, gamma, beta, edge, h, dtype="c128"):
    import numpy as np

    from oracle import tn

    dt = np.complex64 if dtype == "c64" else np.complex128
    j, k = edge
    z = tn.zz_edge(n, edges, gamma, beta, j, k, dt)
    g = np.array(gamma, dtype=float)
    b = np.array(beta, dtype=float)
    for l in range(len(g)):
        for arr in (g, b):
            arr[l] += h
            tn.zz_edge(n, edges, g, b, j, k, dt)
            arr[l] -= 2 * h
            tn.zz_edge(n, edges, g, b, j, k, dt)
            arr[l] += h
    return z


def time_sweeps(net, steps: int, warmup: int, mode: str = "batched", settle_s: float = 0.0):
    """Wall time of `steps` energy + gradient sweeps bracketed by device
    synchronisation, the last energy, and the average device time of the graph
    replay (HIP events on the launch stream, over up to 100 further sweeps).
    Before the `warmup` sweeps, sweeps run for settle_s seconds: a GPU that was
    idle runs short kernels about 1.5x slower for the first few hundred
    milliseconds of work."""
    import torch

    t_settle = time.perf_counter()
    while time.perf_counter() - t_settle < settle_s:
        net.energy_grad(mode)
    for _ in range(warmup):
        net.energy_grad(mode)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        e, _, _ = net.energy_grad(mode)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the device time of the graph replay, from events around it, in sweeps
    # of their own after the timed ones (the events add to a sweep's wall time)
    net.set_sweep_timing(True)
    net.kernel_time(reset=True)
    for _ in range(min(steps, 100)):
        net.energy_grad(mode)
    k_ms, k_cnt = net.kernel_time(reset=True)
    net.set_sweep_timing(False)
    return dt, e, k_ms / max(k_cnt, 1), k_cnt


WIDE_TUNING = dict(seq_max_bits=16, tile_blocks=128, par_bits=21)
WIDE_TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic_wide_sweep_p5_n1000.json")


def wide_leg(repeats: int, steps: int, copy_gbps, retune: bool = False):
    """p = 5, N = 1000 (1500 edges), c64, min-degree randomized greedy order
    (widths up to 26, 0.5 GB tensors): the HBM-bound workload.  Reports the
    whole sweep, the in-sweep rate of its buckets of width >= 20 (their ops as
    one persistent launch of their own), the same ops launched one by one by
    width band, and the other greedy order."""
    import torch

    from paper_2106_15740_amd import QaoaNet, tunecache
    from workloads import workload

    w = workload("p5_n1000")
    t0 = time.perf_counter()
    net = QaoaNet(w.n, w.edges, w.p, dtype="c64", order="min_degree", device=0, repeats=repeats)
    plan_s = time.perf_counter() - t0
    net.set_params(w.gamma, w.beta)
    # tiles: the tuning cache's entry for this plan, else the global and
    # per-band autotuners started from WIDE_TUNING (and stored)
    net.set_tuning(**WIDE_TUNING)
    t1 = time.perf_counter()
    entry = tunecache.tuned(net, with_grad=True, retune=retune)
    tune_s = time.perf_counter() - t1
    log(f"p5_n1000: tiles from {entry['source']} in {tune_s:.1f} s")
    info = net.info()
    census = net.gemm_census(4)  # steps holding a dense product with K, M, N >= 16
    dt, e, k_ms, _ = time_sweeps(net, steps, 1)
    pk_ms = net.time_persistent(with_grad=True, reps=2)
    alg = info["fwd_bytes"] + info["bwd_bytes"]
    alg_b = info["fwd_bytes_bucket"] + info["bwd_bytes_bucket"]
    # buckets of width >= 20 inside a sweep: their ops alone, one persistent launch
    ws20 = net.time_wide_sweep(min_width=20, with_grad=True, reps=3)
    ws20["achieved_GBps"] = ws20["alg_bytes"] / (ws20["ms"] * 1e-3) / 1e9 if ws20["ms"] > 0 else None
    # the same ops launched one by one, by width band (cumulative above each
    # threshold, differenced)
    cum = {wmin: net.time_wide_ops(min_width=wmin, with_grad=True, reps=2) for wmin in (16, 20, 24)}
    bands = []
    for lo, hi in ((16, 20), (20, 24), (24, None)):
        b, ms, k = cum[lo]
        if hi is not None:
            b, ms, k = b - cum[hi][0], ms - cum[hi][1], k - cum[hi][2]
        bands.append({"widths": f"{lo}-{hi - 1}" if hi else f">={lo}", "ops": k, "alg_bytes": b, "ms": ms,
                      "achieved_GBps": b / (ms * 1e-3) / 1e9 if ms > 0 else None})
    tuning = net.tuning()
    bands = net.band_tuning()
    # the same sweep under workspace budgets: a quarter of the keep-everything
    # arena (cones admitted into a shared area as regions free up), and just
    # below the largest cone's own working set (that cone drops outputs after
    # its forward sweep and recomputes them in its adjoint sweep)
    budgets = []
    log("p5_n1000: memory budgets")
    below = [info["pinned_bytes"] + int(f * info["max_cone_dynamic"]) for f in (0.9, 0.95, 0.98, 0.99, 0.999)]
    for label, cands in (("quarter_of_keep_all", [int(0.25 * info["arena_keep_all"])]),
                         ("below_largest_cone", below)):
        nbytes = None
        for nb in cands:  # the lowest the planner meets
            try:
                net.set_memory_budget(nb)
                nbytes = nb
                break
            except Exception:
                continue
        if nbytes is None:
            budgets.append({"budget": label, "met": False})
            continue
        ib = net.info()
        dtb, eb, _, _ = time_sweeps(net, steps, 1)
        pkb = net.time_persistent(with_grad=True, reps=2)
        budgets.append({"budget": label, "budget_GB": nbytes / 1e9, "workspace_GB": ib["ws_grad"] / 1e9,
                        "n_recomputed": ib["n_recomputed"], "recompute_bytes": ib["rec_bytes"],
                        "persistent_kernel_ms": pkb, "overhead_vs_keep_all": pkb / pk_ms - 1.0,
                        "edge_light_cones_per_s": len(w.edges) * steps / dtb,
                        "energy_rel_diff": abs(eb - e) / abs(e)})
    net.set_memory_budget(0)
    del net
    torch.cuda.empty_cache()
    log("p5_n1000: other order")
    # the other greedy order (min-fill: narrower, widths up to 25 on this graph)
    net_mf = QaoaNet(w.n, w.edges, w.p, dtype="c64", order="min_fill", device=0, repeats=repeats)
    net_mf.set_tuning(**tuning)
    net_mf.set_band_tuning(bands)
    net_mf.set_params(w.gamma, w.beta)
    info_mf = net_mf.info()
    dt_mf, e_mf, k_ms_mf, _ = time_sweeps(net_mf, steps, 1)
    pk_mf = net_mf.time_persistent(with_grad=True, reps=2)
    alg_mf = info_mf["fwd_bytes"] + info_mf["bwd_bytes"]
    other = {"order": "min_fill", "max_width": info_mf["max_width"],
             "edge_light_cones_per_s": len(w.edges) * steps / dt_mf, "persistent_kernel_ms": pk_mf,
             "alg_bytes_per_sweep": alg_mf, "achieved_GBps": alg_mf / (pk_mf * 1e-3) / 1e9, "energy": e_mf}
    del net_mf
    torch.cuda.empty_cache()
    achieved_b = alg / (pk_ms * 1e-3) / 1e9
    out = {
        "workload": f"QAOA-MaxCut p=5, random 3-regular N=1000 (1500 edges), c64, min-degree randomized greedy "
                    f"({repeats} repeats), batched energy + gradient",
        "edge_light_cones_per_s": len(w.edges) * steps / dt,
        "ms_per_step": 1e3 * dt / steps,
        "max_width": info["max_width"],
        "alg_bytes_per_sweep": alg,
        "alg_bytes_per_sweep_index_buckets": alg_b,
        "sweep_ms": k_ms,
        "persistent_kernel_ms": pk_ms,
        "achieved_GBps": achieved_b,
        "frac_of_peak": achieved_b / HBM_PEAK_GBS,
        "traffic_bytes_per_launch": measured_traffic(P5_TRAFFIC_JSON, tuning, bands),
        "frac_of_copy": achieved_b / copy_gbps if copy_gbps else None,
        "workspace_GB": info["ws_grad"] / 1e9,
        "keep_all_GB": info["arena_keep_all"] / 1e9,
        "memory_budgets": budgets,
        "gemm_census_k16": census,
        "width_ge_20_standalone_bands": bands,
        "energy": e,
        "plan_s": plan_s,
        "tuning": tuning,
        "band_tuning": bands,
        "tuning_source": {"source": entry["source"], "key": entry["key"], "seconds": tune_s},
        "other_order": other,
    }
    roof20 = {"bound": "hbm", "achieved": ws20["achieved_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": ws20["achieved_GBps"] / HBM_PEAK_GBS if ws20["achieved_GBps"] else None,
              "traffic": measured_traffic(WIDE_TRAFFIC_JSON, tuning, bands),
              "kernel": "persistent_kernel (queue of the width >= 20 ops only)",
              "kernel_ms": ws20["ms"], "alg_bytes_per_launch": ws20["alg_bytes"],
              "op_bytes_per_launch": ws20["op_bytes"], "ops": ws20["ops"],
              "items": ws20["items"], "copy_kernel_GBps": copy_gbps,
              "frac_of_copy": ws20["achieved_GBps"] / copy_gbps if (copy_gbps and ws20["achieved_GBps"]) else None,
              "workload": "p=5 N=1000 min-degree randomized greedy: every forward and adjoint op of a bucket with "
                          "output rank >= 20, chained per light cone, tiled and list-scheduled as in the full sweep, "
                          "one launch reading the previous sweep's tensors"}
    return out, roof20


def amplitude_leg(steps: int = 3):
    """The paper's own benchmark object: one amplitude <0...0|gamma beta> of a
    whole 40-vertex random 3-regular graph at p = 4 (the depth the paper
    estimates for supercomputers only), c64, min-fill randomized greedy order
    (50 repeats), forward contraction."""
    import torch

    from paper_2106_15740_amd import QaoaAmplitude
    from workloads import random_angles, random_regular_graph

    n, p = 40, 4
    edges = random_regular_graph(n, 3, 0)
    g, b = random_angles(p, 1 + 1000 * p)
    t0 = time.perf_counter()
    net = QaoaAmplitude(n, edges, p, dtype="c64", order="min_fill", device=0, repeats=50)
    plan_s = time.perf_counter() - t0
    net.set_tuning(seq_max_bits=14, tile_blocks=64, par_bits=21)
    net.set_params(g, b)
    info = net.info()
    a = net.amplitude()  # warm-up (graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a = net.amplitude()
    dt = (time.perf_counter() - t0) / steps
    out = {"workload": "single amplitude <0...0|gamma beta>, random 3-regular N=40 (60 edges), p=4, c64, "
                       "min-fill randomized greedy (50 repeats), batched forward contraction",
           "ms_per_amplitude": 1e3 * dt, "max_width": info["max_width"], "workspace_GB": info["ws_fwd"] / 1e9,
           "alg_bytes": info["fwd_bytes"], "alg_GBps": info["fwd_bytes"] / dt / 1e9,
           "amplitude": [a.real, a.imag], "plan_s": plan_s}
    del net
    torch.cuda.empty_cache()
    return out


def profile_leg(which: str, repeats: int):
    """One p = 5 measurement alone, for profiler runs: `p5_sweep` times the
    persistent kernel of the whole sweep, `p5_wide20` the width >= 20 ops as a
    launch of their own (both after one warm sweep)."""
    from paper_2106_15740_amd import QaoaNet, tunecache
    from workloads import workload

    w = workload("p5_n1000")
    net = QaoaNet(w.n, w.edges, w.p, dtype="c64", order="min_degree", device=0, repeats=repeats)
    net.set_tuning(**WIDE_TUNING)
    entry = tunecache.tuned(net, with_grad=True, search=False)  # the cached tiles, if any
    net.set_params(w.gamma, w.beta)
    net.energy_grad("batched")
    info = net.info()
    out = {"profile": which, "tuning": net.tuning(), "band_tuning": net.band_tuning(),
           "tuning_source": None if entry is None else entry["source"]}
    if which == "p5_sweep":
        out["persistent_kernel_ms"] = net.time_persistent(with_grad=True, reps=3)
        out["alg_bytes_per_launch"] = info["fwd_bytes"] + info["bwd_bytes"]
        out["alg_bytes_per_launch_index_buckets"] = info["fwd_bytes_bucket"] + info["bwd_bytes_bucket"]
    else:
        out.update(net.time_wide_sweep(min_width=20, with_grad=True, reps=3))
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--settle", type=float, default=1.0,
                    help="seconds of untimed sweeps before the warm-up steps (the GPU's clocks ramp up)")
    ap.add_argument("--workload", default="p3_n244")
    ap.add_argument("--repeats", type=int, default=10,
                    help="randomized greedy order: runs per cone on top of the deterministic one (0: deterministic)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile shapes")
    ap.add_argument("--retune", action="store_true",
                    help="run the autotuners even when the tuning cache has an entry for the plan (and store it)")
    ap.add_argument("--tuning", default="",
                    help="fixed tile shapes instead of the autotuner, e.g. threads=128,lane_cap=7,seq_max_bits=14")
    ap.add_argument("--no-wide", action="store_true", help="skip the p=5 N=1000 leg")
    ap.add_argument("--no-amplitude", action="store_true", help="skip the single-amplitude leg (N=40, p=4)")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-other-order", dest="other_order", action="store_false",
                    help="skip the headline workload under the other greedy order")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after timing, run one device copy of this many MiB (counter calibration)")
    ap.add_argument("--profile", choices=["p5_sweep", "p5_wide20"], default=None,
                    help="run only one p=5 measurement (for rocprofv3 runs): the whole sweep, or the width >= 20 "
                         "ops as one launch; prints its timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the light-cone sweep is not sharded across GPUs; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    from workloads import workload

    if args.profile:
        profile_leg(args.profile, args.repeats)
        return
    w = workload(args.workload)
    if args.cpu_only:
        print(json.dumps(cpu_baseline(w)))
        return
    # the CPU leg runs in a child process (which forks its workers) and ends
    # before this process touches the GPU
    cpu = None
    if not args.no_cpu:
        import subprocess

        log("CPU oracle baseline")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-only", "--workload", args.workload],
                           capture_output=True, text=True, check=True)
        cpu = json.loads(r.stdout.strip().splitlines()[-1])
        log(f"CPU oracle baseline done: {cpu['value']:.1f} {cpu['unit']}")

    import torch

    from paper_2106_15740_amd import QaoaNet, copy_bandwidth, tunecache

    t0 = time.perf_counter()
    net = QaoaNet(w.n, w.edges, w.p, dtype=w.dtype, order=w.order, device=0, repeats=args.repeats)
    plan_s = time.perf_counter() - t0
    net.set_params(w.gamma, w.beta)
    log(f"{args.workload}: plan built in {plan_s:.1f} s; tuning")
    tune_entry = None
    if args.tuning:
        net.set_tuning(**{k: int(v) for k, v in (kv.split("=") for kv in args.tuning.split(","))})
    elif not args.no_autotune:
        tune_entry = tunecache.tuned(net, with_grad=True, retune=args.retune)
    tuned = net.tuning()
    info = net.info()

    log(f"{args.workload}: timing {args.steps} steps")
    dt, e, k_avg_ms, k_cnt = time_sweeps(net, args.steps, args.warmup, settle_s=args.settle)
    log(f"{args.workload}: {1e3 * dt / args.steps:.3f} ms per step")
    ms_step = 1e3 * dt / args.steps
    cones_per_s = len(w.edges) * args.steps / dt
    # the dominant kernel alone: HIP events around the persistent kernel on
    # the launch stream (sweeps enqueued without graph capture)
    pk_ms = net.time_persistent(with_grad=True, reps=20)

    other = None
    if args.other_order:
        # the same workload under the other greedy order (same tile shapes)
        o2 = "min_degree" if w.order == "min_fill" else "min_fill"
        net2 = QaoaNet(w.n, w.edges, w.p, dtype=w.dtype, order=o2, device=0, repeats=args.repeats)
        net2.set_params(w.gamma, w.beta)
        net2.set_tuning(**{k: v for k, v in tuned.items()})
        i2 = net2.info()
        dt2, _, k2, _ = time_sweeps(net2, args.steps, args.warmup, settle_s=min(args.settle, 0.3))
        other = {"order": o2, "max_width": i2["max_width"], "edge_light_cones_per_s": len(w.edges) * args.steps / dt2,
                 "ms_per_step": 1e3 * dt2 / args.steps,
                 "alg_GBps": (i2["fwd_bytes"] + i2["bwd_bytes"]) / (k2 * 1e-3) / 1e9}
        del net2

    # achievable-bandwidth reference, after the timed steps
    copy_gbps = copy_bandwidth(1 << 30, reps=5)

    plain_ms = None
    if args.plain_steps > 0:
        pdt, _, _, _ = time_sweeps(net, args.plain_steps, 1, mode="plain")
        plain_ms = 1e3 * pdt / args.plain_steps

    if args.copy_mb > 0:
        x = torch.empty(args.copy_mb << 20, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()

    alg_merged = info["fwd_bytes"] + info["bwd_bytes"]
    alg_bytes = info["fwd_bytes_bucket"] + info["bwd_bytes_bucket"]
    achieved = alg_merged / (pk_ms * 1e-3) / 1e9 if pk_ms > 0 else None
    out = {
        "metric": "edge light-cones/sec (energy+grad) & HBM GB/s vs plain loop, 3-regular p=3",
        "value": cones_per_s,
        "unit": "edge light-cones/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 accumulate)" if w.dtype == "c64" else "c128",
        "data": "synthetic: seeded random 3-regular graph, angles ~ U(0, pi)",
        "config": {"workload": f"QAOA-MaxCut p={w.p}, random 3-regular N={w.n} ({len(w.edges)} edges), "
                               f"{w.dtype}, {w.order.replace('_', '-')} randomized greedy order "
                               f"({args.repeats} repeats), batched persistent sweep (energy + gradient)",
                   "n_vertices": w.n, "n_edges": len(w.edges), "p": w.p, "order": w.order,
                   "repeats": args.repeats, "max_width": info["max_width"], "buckets": info["n_buckets"],
                   "lds_resident_cones": info["n_lds_cones"]},
        "roofline": {"bound": "latency", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": measured_traffic(TRAFFIC_JSON, tuned),
                     "kernel": ("small_kernel (every light cone LDS-resident, one workgroup each)"
                                if info["n_lds_cones"] == len(w.edges) else
                                "persistent_kernel" if info["n_lds_cones"] == 0 else
                                "small_kernel (LDS-resident cones) + persistent_kernel (queued cones)"),
                     "kernel_ms": pk_ms, "sweep_ms": k_avg_ms,
                     "alg_bytes_per_launch": alg_merged,
                     "alg_bytes_per_launch_index_buckets": alg_bytes,
                     "copy_kernel_GBps": copy_gbps,
                     "frac_of_copy": (achieved / copy_gbps) if achieved else None,
                     "note": "p=3 sweeps are chains of small dependent steps whose tensors live in LDS and cache: "
                             "bound by dependency latency, not HBM; achieved = algorithmic bytes of the plan's "
                             "contraction steps (each input read once, each output written once) over the "
                             "contraction kernel's time (HIP events around it: kernel_ms); the count with one bucket "
                             "per index beside it; sweep_ms: the whole graph replay (leaf kernels and final "
                             "reduction included)"},
        "plain_loop": None if plain_ms is None else {
            "ms_per_step": plain_ms, "edge_light_cones_per_s": len(w.edges) / (plain_ms * 1e-3),
            "speedup_batched_vs_plain": plain_ms / ms_step},
        "other_order": other,
        "energy": e,
        "plan_s": plan_s,
        "tuning": tuned,
        "tuning_source": None if tune_entry is None else {"source": tune_entry["source"], "key": tune_entry["key"]},
    }
    if not args.no_wide:
        del net
        torch.cuda.empty_cache()
        log("p5_n1000 leg")
        out["wide"], out["roofline_width_ge_20"] = wide_leg(args.repeats, steps=3, copy_gbps=copy_gbps,
                                                            retune=args.retune)
    if not args.no_amplitude:
        log("amplitude leg")
        out["amplitude"] = amplitude_leg()
    if cpu is not None:
        cpu["gpu_speedup"] = cones_per_s / cpu["value"]
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
