"""Cost model of the paper's comparison (Section IV, the FLOP figures of
Section V and Tables I and II): contraction width and operation count of the
single amplitude <0...0|gamma beta> under the four network constructions,
ordered by the library's randomized greedy orderer (host only; see
qtn_cost_model in include/qtn.h for the constructions).
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Iterable, List, Sequence, Tuple

import numpy as np

from . import _lib as L

VARIANTS = ("default", "diagonal", "zz", "diagonal_zz")
_ORDERS = {"min_degree": L.QTN_ORDER_MIN_DEGREE, "min_fill": L.QTN_ORDER_MIN_FILL}

# memory of the paper's two machines and the bytes of one complex128 element;
# the laptop's 4 GB is read as 4 GiB (2^32 bytes: a width-28 complex128
# tensor), the aggregate 800 TB as 800e12 bytes (largest width 45 either way)
LAPTOP_BYTES = 4.0 * 2 ** 30
SUPERCOMPUTER_BYTES = 800e12
ELEM_BYTES = 16


def cost(n: int, edges: Sequence[Tuple[int, int]], p: int, variant: str, order: str = "min_fill",
         repeats: int = 10, temperature: float = 0.02, seed: int = 0) -> Dict[str, float]:
    """{'n_indices', 'n_tensors', 'width', 'log2_ops', 'order_seconds'} of one
    network (log2_ops: log2 of the sum over buckets of 2^|union|)."""
    e = np.ascontiguousarray(np.array(edges, dtype=np.int32).reshape(-1, 2))
    out = L.Cost()
    L.check(L.lib().qtn_cost_model(int(n), len(e), e.ctypes.data_as(C.c_void_p), int(p), VARIANTS.index(variant),
                                   _ORDERS[order], int(repeats), float(temperature), int(seed), C.byref(out)))
    return out.as_dict()


def cost_and_order(n: int, edges: Sequence[Tuple[int, int]], p: int, variant: str, order: str = "min_fill",
                   repeats: int = 10, temperature: float = 0.02, seed: int = 0) -> Tuple[Dict[str, float], List[int]]:
    """cost() and the elimination order it evaluated (index ids in the order
    the construction creates them; see qtn_cost_model_order)."""
    e = np.ascontiguousarray(np.array(edges, dtype=np.int32).reshape(-1, 2))
    first = cost(n, edges, p, variant, order, repeats=0)
    buf = np.zeros(max(1, int(first["n_indices"])), dtype=np.int32)
    out = L.Cost()
    L.check(L.lib().qtn_cost_model_order(int(n), len(e), e.ctypes.data_as(C.c_void_p), int(p), VARIANTS.index(variant),
                                         _ORDERS[order], int(repeats), float(temperature), int(seed), C.byref(out),
                                         buf.ctypes.data_as(C.c_void_p), len(buf)))
    return out.as_dict(), [int(x) for x in buf[: out.n_indices]]


def _graphs(n: int, seeds: Iterable[int]):
    from workloads import random_regular_graph

    return [random_regular_graph(n, 3, s) for s in seeds]


def ops_vs_p(n: int = 40, ps: Iterable[int] = range(1, 6), seeds: Iterable[int] = range(5),
             **kw) -> Dict[str, List[Tuple[int, float, float, float]]]:
    """Per variant: (p, mean log2_ops, std, mean width) over seeded random
    3-regular graphs (the shape of the paper's FLOPs-versus-p figure)."""
    graphs = _graphs(n, seeds)
    res = {}
    for v in VARIANTS:
        rows = []
        for p in ps:
            cs = [cost(n, g, p, v, **kw) for g in graphs]
            lo = [c["log2_ops"] for c in cs]
            rows.append((p, float(np.mean(lo)), float(np.std(lo)), float(np.mean([c["width"] for c in cs]))))
        res[v] = rows
    return res


def ops_vs_n(ns: Iterable[int] = (20, 40, 80, 120, 160), p: int = 1, seeds: Iterable[int] = range(5),
             **kw) -> Dict[str, List[Tuple[int, float, float, float]]]:
    """Per variant: (N, mean log2_ops, std, mean width) at fixed p (the shape of
    the paper's FLOPs-versus-N figure, p = 1)."""
    res = {v: [] for v in VARIANTS}
    for n in ns:
        graphs = _graphs(n, seeds)
        for v in VARIANTS:
            cs = [cost(n, g, p, v, **kw) for g in graphs]
            lo = [c["log2_ops"] for c in cs]
            res[v].append((n, float(np.mean(lo)), float(np.std(lo)), float(np.mean([c["width"] for c in cs]))))
    return res


def fits(width: int, mem_bytes: float) -> bool:
    """The largest intermediate (2^width complex128 elements) fits in memory."""
    return ELEM_BYTES * 2.0 ** width <= mem_bytes


def max_p(n: int, mem_bytes: float, seeds: Iterable[int] = range(5), p_max: int = 8, **kw) -> Dict[str, int]:
    """Per variant: the largest p whose network fits mem_bytes for every seeded
    graph (Table I: N = 40, a 4 GB laptop and an 800 TB machine)."""
    graphs = _graphs(n, seeds)
    res = {}
    for v in VARIANTS:
        best = 0
        for p in range(1, p_max + 1):
            if all(fits(cost(n, g, p, v, **kw)["width"], mem_bytes) for g in graphs):
                best = p
            else:
                break
        res[v] = best
    return res


def max_n(p: int, mem_bytes: float, ns: Sequence[int], seeds: Iterable[int] = range(5), **kw) -> Dict[str, int]:
    """Per variant: the largest N from ns (ascending) whose network fits
    mem_bytes for every seeded graph at depth p (Table II)."""
    res = {}
    for v in VARIANTS:
        best = 0
        for n in ns:
            if all(fits(cost(n, g, p, v, **kw)["width"], mem_bytes) for g in _graphs(n, seeds)):
                best = n
            else:
                break
        res[v] = best
    return res


def ops_vs_order_time(n: int = 160, p: int = 1, variant: str = "diagonal_zz", order: str = "min_fill",
                      repeats: Iterable[int] = (0, 1, 2, 5, 10, 20, 50), seed_graph: int = 0,
                      temperature: float = 0.02) -> List[Tuple[int, float, int, float]]:
    """(n_repeats, ordering seconds, width, log2_ops) for one seeded graph as
    the randomized greedy orderer gets more repeats (the shape of the paper's
    FLOPs-versus-ordering-time figure: p = 1, N = 160)."""
    g = _graphs(n, [seed_graph])[0]
    out = []
    for r in repeats:
        c = cost(n, g, p, variant, order=order, repeats=r, temperature=temperature, seed=1)
        out.append((int(r), c["order_seconds"], int(c["width"]), c["log2_ops"]))
    return out
