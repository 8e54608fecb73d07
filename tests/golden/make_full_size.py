"""Writes the full-size expected values of the GPU parity tests from the CPU
oracle alone (no part of the GPU library is imported).

For a workload of ``workloads.workload`` it contracts every edge's light-cone
network with ``oracle.tn`` (complex128 bucket elimination over the oracle's
own pruned gate list and min-fill order) and, for a chosen set of edges, takes
d<Z_j Z_k>/d(gamma_l, beta_l) by central differences of the same contraction
(step h = 1e-4; truncation error about h^2/6 times the third derivative).
Which edges get derivatives: every edge for ``p3_n244``; otherwise the first
edge of each contraction width of the oracle's own order, plus edge 0.

It also writes the single amplitude <0...0|gamma beta> of a 22-vertex random
3-regular graph at p = 4 and its derivatives, from the oracle's state vector
(``amplitude_n22_p4.txt``).

Usage:  python tests/golden/make_full_size.py [p3_n244 p4_n100 p5_n1000 amp] [-j PROCS]
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import statevector as sv, tn  # noqa: E402
from workloads import random_angles, random_regular_graph, workload  # noqa: E402

H = 1e-4
AMP_N, AMP_P, AMP_GRAPH_SEED, AMP_ANGLE_SEED = 22, 4, 0, 5


def _zz(task):
    name, i = task
    w = workload(name)
    j, k = w.edges[i]
    t = tn.network(w.n, w.edges, w.gamma, w.beta, j, k)
    order, width = tn.min_fill_order(t)
    return i, tn.contract(t, order), width


def _grad(task):
    name, i = task
    w = workload(name)
    j, k = w.edges[i]
    g = np.array(w.gamma, dtype=float)
    b = np.array(w.beta, dtype=float)
    out = []
    for arr in (g, b):
        for l in range(w.p):
            arr[l] += H
            up = tn.zz_edge(w.n, w.edges, g, b, j, k)
            arr[l] -= 2 * H
            dn = tn.zz_edge(w.n, w.edges, g, b, j, k)
            arr[l] += H
            out.append(((up - dn) / (2 * H)).real)
    return i, out


def write_workload(name: str, procs: int) -> str:
    w = workload(name)
    m = len(w.edges)
    t0 = time.time()
    zz = np.zeros(m, dtype=np.complex128)
    width = np.zeros(m, dtype=np.int64)
    with mp.get_context("fork").Pool(procs) as pool:
        for i, z, wd in pool.imap_unordered(_zz, [(name, i) for i in range(m)], chunksize=1):
            zz[i], width[i] = z, wd
        if name == "p3_n244":
            chosen = list(range(m))
        else:
            chosen = sorted({0} | {int(np.nonzero(width == v)[0][0]) for v in np.unique(width)})
        order = sorted(chosen, key=lambda i: -width[i])  # widest first: the pool does not end on one long task
        grads = {}
        for i, gr in pool.imap_unordered(_grad, [(name, i) for i in order], chunksize=1):
            grads[i] = gr
    path = os.path.join(HERE, f"full_size_{name}.txt")
    with open(path, "w") as fh:
        fh.write(f"# Per-edge <Z_j Z_k> of workload {name} (workloads.workload: seeded random 3-regular graph, "
                 f"N={w.n}, {m} edges, p={w.p},\n# gamma={[float(x) for x in w.gamma]}, beta={[float(x) for x in w.beta]})\n")
        fh.write("# written by tests/golden/make_full_size.py from oracle.tn: complex128 bucket elimination of each\n")
        fh.write("# edge's light-cone network (Sections II, III.B, IV.B); derivatives d<ZZ>/d(gamma_1..p, beta_1..p)\n")
        fh.write(f"# by central differences, h = {H}.  Columns: edge j k oracle_width re im [2p derivatives]\n")
        for i in range(m):
            j, k = w.edges[i]
            cols = [str(i), str(j), str(k), str(int(width[i])), repr(float(zz[i].real)), repr(float(zz[i].imag))]
            if i in grads:
                cols += [repr(float(x)) for x in grads[i]]
            fh.write(" ".join(cols) + "\n")
    print(f"{name}: {m} edges, {len(grads)} with derivatives, {time.time() - t0:.0f} s -> {path}", flush=True)
    return path


def _amp(task):
    which, l = task
    edges = random_regular_graph(AMP_N, 3, AMP_GRAPH_SEED)
    g, b = random_angles(AMP_P, AMP_ANGLE_SEED)
    if which == "value":
        return task, sv.amplitude(AMP_N, edges, g, b)
    arr = g if which == "gamma" else b
    arr[l] += H
    up = sv.amplitude(AMP_N, edges, g, b)
    arr[l] -= 2 * H
    dn = sv.amplitude(AMP_N, edges, g, b)
    return task, (up - dn) / (2 * H)


def write_amplitude(procs: int) -> str:
    tasks = [("value", 0)] + [(k, l) for k in ("gamma", "beta") for l in range(AMP_P)]
    res = {}
    with mp.get_context("fork").Pool(min(procs, 4)) as pool:  # ~1 GB per state vector
        for t, v in pool.imap_unordered(_amp, tasks):
            res[t] = v
    path = os.path.join(HERE, f"amplitude_n{AMP_N}_p{AMP_P}.txt")
    g, b = random_angles(AMP_P, AMP_ANGLE_SEED)
    with open(path, "w") as fh:
        fh.write(f"# <0...0|gamma beta> of workloads.random_regular_graph({AMP_N}, 3, seed={AMP_GRAPH_SEED}) at "
                 f"p={AMP_P},\n# angles workloads.random_angles({AMP_P}, seed={AMP_ANGLE_SEED}): gamma={[float(x) for x in g]}, "
                 f"beta={[float(x) for x in b]}\n")
        fh.write("# written by tests/golden/make_full_size.py from oracle.statevector (complex128 state vector,\n")
        fh.write(f"# Section II); derivatives by central differences, h = {H}.  Columns: quantity re im\n")
        fh.write(f"amplitude {res[('value', 0)].real!r} {res[('value', 0)].imag!r}\n")
        for k in ("gamma", "beta"):
            for l in range(AMP_P):
                v = res[(k, l)]
                fh.write(f"d_{k}_{l + 1} {v.real!r} {v.imag!r}\n")
    print(f"amplitude -> {path}", flush=True)
    return path


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", nargs="*", default=["p3_n244", "p4_n100", "p5_n1000", "amp"])
    ap.add_argument("-j", type=int, default=min(8, os.cpu_count() or 1))
    a = ap.parse_args()
    for name in a.what:
        if name == "amp":
            write_amplitude(a.j)
        else:
            write_workload(name, a.j)


if __name__ == "__main__":
    main()
