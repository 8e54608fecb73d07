"""Thin Python wrapper over the C ABI: one QAOA-MaxCut energy network.

PyTorch supplies device memory (the caller-owned workspace) and the stream;
every contraction step runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence, Tuple

import numpy as np

from . import _lib as L

_DTYPES = {"c64": L.QTN_C64, "c128": L.QTN_C128}
_ORDERS = {"min_degree": L.QTN_ORDER_MIN_DEGREE, "min_fill": L.QTN_ORDER_MIN_FILL}
_MODES = {"plain": L.QTN_PLAIN, "batched": L.QTN_BATCHED}


class Context:
    """A device (or host-only planning) context."""

    def __init__(self, device: int = 0):
        self._lib = L.lib()
        h = C.c_void_p()
        L.check(self._lib.qtn_create(int(device), C.byref(h)))
        self.handle = h
        self.device = device

    def __del__(self):
        if getattr(self, "handle", None):
            self._lib.qtn_destroy(self.handle)
            self.handle = None


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 5, device: int = 0) -> float:
    """GB/s (read + write) of the library's plain copy kernel over an nbytes
    device buffer: the achievable-bandwidth reference."""
    import torch

    ctx = default_context(device)
    buf = torch.empty(int(nbytes), dtype=torch.uint8, device=f"cuda:{device}")
    g = C.c_double()
    st = C.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    L.check(ctx._lib.qtn_copy_bandwidth(ctx.handle, C.c_void_p(buf.data_ptr()), buf.numel(), st, int(reps),
                                        C.byref(g)))
    del buf
    return g.value


_default_ctx = {}


def default_context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


class QaoaNet:
    _BUILD = "qtn_build"

    """Light-cone tensor networks of every edge term of <gamma beta|C|gamma beta>.

    n, edges: the graph (vertices 0..n-1); p: QAOA depth; dtype "c64" or
    "c128"; order "min_degree" or "min_fill", deterministic, or with
    repeats > 0 the randomized greedy (repeats, temperature, seed) keeping the
    cheapest order per cone; device: HIP device id, or None for a host-only
    planning network (statistics and plan checks only).
    """

    def __init__(self, n: int, edges: Sequence[Tuple[int, int]], p: int, dtype: str = "c64",
                 order: str = "min_fill", device: Optional[int] = 0, repeats: int = 0,
                 temperature: float = 0.02, seed: int = 0):
        self._lib = L.lib()
        self.ctx = Context(L.QTN_HOST_ONLY) if device is None else default_context(device)
        self.n, self.p, self.dtype, self.order = int(n), int(p), dtype, order
        self.edges = [(int(u), int(v)) for u, v in edges]
        self.device = device
        e = np.ascontiguousarray(np.array(self.edges, dtype=np.int32).reshape(-1, 2))
        self._edges_buf = e
        h = C.c_void_p()
        L.check(getattr(self._lib, self._BUILD)(self.ctx.handle, self.n, len(self.edges),
                                                e.ctypes.data_as(C.c_void_p), self.p, _DTYPES[dtype], C.byref(h)))
        self.handle = h
        w = C.c_int32()
        if repeats > 0:
            L.check(self._lib.qtn_order_rgreedy(self.handle, _ORDERS[order], int(repeats), float(temperature),
                                                int(seed), C.byref(w)))
        else:
            L.check(self._lib.qtn_order(self.handle, _ORDERS[order], C.byref(w)))
        self.max_width = w.value
        self._ws = {}

    def __del__(self):
        if getattr(self, "handle", None):
            self._lib.qtn_net_free(self.handle)
            self.handle = None

    # ------------------------------------------------------------------ info
    def info(self) -> dict:
        i = L.Info()
        L.check(self._lib.qtn_get_info(self.handle, C.byref(i)))
        return i.as_dict()

    def cone_stats(self) -> dict:
        m = len(self.edges)
        arrs = {k: np.zeros(m, np.int32) for k in ("width", "n_qubits", "n_indices", "n_tensors", "n_buckets")}
        arrs.update({k: np.zeros(m, np.float64) for k in ("fwd_bytes", "bwd_bytes")})
        ptr = lambda a: a.ctypes.data_as(C.c_void_p)
        L.check(self._lib.qtn_cone_stats(self.handle, *(ptr(arrs[k]) for k in (
            "width", "n_qubits", "n_indices", "n_tensors", "n_buckets", "fwd_bytes", "bwd_bytes"))))
        return arrs

    def validate(self) -> None:
        L.check(self._lib.qtn_validate_plan(self.handle))

    def workspace_size(self, with_grad: bool) -> int:
        s = C.c_size_t()
        L.check(self._lib.qtn_workspace_size(self.handle, int(bool(with_grad)), C.byref(s)))
        return s.value

    def set_memory_budget(self, nbytes: int) -> None:
        """Checkpointed adjoint: keep the workspace within about nbytes by
        recomputing dropped bucket outputs in the adjoint sweep (0: no limit)."""
        L.check(self._lib.qtn_set_memory_budget(self.handle, int(nbytes)))
        self._ws.clear()

    def tuning(self) -> dict:
        t = L.Tuning()
        L.check(self._lib.qtn_get_tuning(self.handle, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw) -> None:
        t = L.Tuning()
        L.check(self._lib.qtn_get_tuning(self.handle, C.byref(t)))
        names = {f for f, _ in L.Tuning._fields_}
        for k, v in kw.items():
            if k not in names:
                raise ValueError(f"unknown tuning field {k!r} (fields: {sorted(names)})")
            setattr(t, k, int(v))
        L.check(self._lib.qtn_set_tuning(self.handle, C.byref(t)))
        self._ws = {k: v for k, v in self._ws.items() if k == "buf"}

    def band_tuning(self) -> list:
        """Tile parameters of wide buckets per union-size band (0: the global
        value): [{'par_bits', 'tile_blocks', 'loop_cap'}] * QTN_BANDS."""
        arr = (L.BandTuning * L.QTN_BANDS)()
        L.check(self._lib.qtn_get_band_tuning(self.handle, arr))
        return [b.as_dict() for b in arr]

    def set_band_tuning(self, bands) -> None:
        arr = (L.BandTuning * L.QTN_BANDS)()
        for i, b in enumerate(bands):
            for k, v in b.items():
                setattr(arr[i], k, int(v))
        L.check(self._lib.qtn_set_band_tuning(self.handle, arr))
        self._ws = {k: v for k, v in self._ws.items() if k == "buf"}

    def signature(self) -> str:
        """The plan's shape before tiling (cones, depth, dtype, contraction width,
        buckets and their algorithmic bytes): the key of tuning caches."""
        i = self.info()
        return (f"n{i['n_cones']}-p{i['p']}-{self.dtype}-w{i['max_width']}-b{i['n_buckets']}-"
                f"B{int(i['fwd_bytes_bucket'])}")

    # ------------------------------------------------------------------ device work
    def _workspace(self, with_grad: bool):
        import torch

        if self.device is None:
            raise L.QtnError(L.QTN_ESTATE, "a host-only network cannot run contractions")

        key = ("need", bool(with_grad))
        need = self._ws.get(key)
        if need is None:
            need = self._ws[key] = self.workspace_size(with_grad)
        buf = self._ws.get("buf")
        if buf is None or buf.numel() < need:
            self._ws.pop("buf", None)
            buf = torch.empty(max(need, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
            self._ws["buf"] = buf
        return buf

    def _stream(self):
        import torch

        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def set_params(self, gamma, beta) -> None:
        g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64).reshape(-1))
        b = np.ascontiguousarray(np.asarray(beta, dtype=np.float64).reshape(-1))
        if g.size != self.p or b.size != self.p:
            raise ValueError(f"gamma and beta must have length p={self.p}")
        L.check(self._lib.qtn_set_params(self.handle, g.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p)))

    def zz_buffer(self):
        import torch

        dt = torch.complex64 if self.dtype == "c64" else torch.complex128
        return torch.empty(len(self.edges), dtype=dt, device=f"cuda:{self.device}")

    def energy(self, mode: str = "batched", zz_out=None) -> float:
        ws = self._workspace(False)
        e = C.c_double()
        L.check(self._lib.qtn_contract(self.handle, _MODES[mode], C.c_void_p(ws.data_ptr()), ws.numel(),
                                       self._stream(), C.c_void_p(zz_out.data_ptr() if zz_out is not None else 0),
                                       C.byref(e)))
        return e.value

    def energy_grad(self, mode: str = "batched", zz_out=None) -> Tuple[float, np.ndarray, np.ndarray]:
        import torch

        # (the per-step path of an optimizer loop: plain integers for the
        # pointer arguments, one output array for both gradients)
        ws = self._workspace(True)
        e = C.c_double()
        g = np.zeros(2 * self.p)
        at = g.ctypes.data
        L.check(self._lib.qtn_energy_grad(self.handle, _MODES[mode], ws.data_ptr(), ws.numel(),
                                          torch.cuda.current_stream(self.device).cuda_stream,
                                          zz_out.data_ptr() if zz_out is not None else None, C.byref(e),
                                          at, at + 8 * self.p))
        return e.value, g[:self.p], g[self.p:]

    def energy_grad_noalloc(self, mode: str = "batched", zz_out=None) -> Tuple[float, np.ndarray, np.ndarray]:
        """energy_grad through the allocation-free entry point: the workspace is
        the library's static device scratch (64 MiB per GPU), nothing is
        allocated."""
        e = C.c_double()
        dg = np.zeros(self.p)
        db = np.zeros(self.p)
        L.check(self._lib.qtn_energy_grad_noalloc(self.handle, _MODES[mode], self._stream(),
                                                  C.c_void_p(zz_out.data_ptr() if zz_out is not None else 0),
                                                  C.byref(e), dg.ctypes.data_as(C.c_void_p),
                                                  db.ctypes.data_as(C.c_void_p)))
        return e.value, dg, db

    def edge_results(self, with_grad: bool = False):
        """Per-edge <Z_j Z_k> (complex128) and, with_grad, d<ZZ>/d(gamma, beta)
        of shape [n_edges, 2p] from the last sweep."""
        m = len(self.edges)
        zz = np.zeros(2 * m)
        dzz = np.zeros(m * 4 * self.p) if with_grad else None
        # NULL workspace: the one the last sweep used (the library tracks it)
        L.check(self._lib.qtn_edge_results(self.handle, None, self._stream(),
                                           zz.ctypes.data_as(C.c_void_p),
                                           dzz.ctypes.data_as(C.c_void_p) if with_grad else None))
        z = zz[0::2] + 1j * zz[1::2]
        if not with_grad:
            return z
        d = dzz.reshape(m, 2 * self.p, 2)
        return z, d[..., 0] + 1j * d[..., 1]

    def autotune(self, with_grad: bool = True, reps: int = 3) -> dict:
        ws = self._workspace(with_grad)
        t = L.Tuning()
        L.check(self._lib.qtn_autotune(self.handle, int(bool(with_grad)), C.c_void_p(ws.data_ptr()), ws.numel(),
                                       self._stream(), int(reps), C.byref(t)))
        self._ws = {k: v for k, v in self._ws.items() if k == "buf"}
        return t.as_dict()

    def autotune_bands(self, with_grad: bool = True, reps: int = 2) -> Tuple[list, float]:
        """Per-band tile search (qtn_autotune_bands): the chosen bands and the
        whole persistent sweep's device ms with them."""
        ws = self._workspace(with_grad)
        arr = (L.BandTuning * L.QTN_BANDS)()
        ms = C.c_double()
        L.check(self._lib.qtn_autotune_bands(self.handle, int(bool(with_grad)), C.c_void_p(ws.data_ptr()), ws.numel(),
                                             self._stream(), int(reps), arr, C.byref(ms)))
        self._ws = {k: v for k, v in self._ws.items() if k == "buf"}
        return [b.as_dict() for b in arr], ms.value

    def time_wide_ops(self, min_width: int = 20, with_grad: bool = True, reps: int = 2) -> Tuple[float, float, int]:
        """(algorithmic bytes, device ms, op count) of the contraction ops whose
        output rank is >= min_width, each launched alone (after a sweep)."""
        ws = self._workspace(with_grad)
        b, ms, n = C.c_double(), C.c_double(), C.c_int64()
        L.check(self._lib.qtn_time_wide_ops(self.handle, int(bool(with_grad)), int(min_width),
                                            C.c_void_p(ws.data_ptr()), ws.numel(), self._stream(), int(reps),
                                            C.byref(b), C.byref(ms), C.byref(n)))
        return b.value, ms.value, n.value

    def time_wide_sweep(self, min_width: int = 20, with_grad: bool = True, reps: int = 3, max_width: int = 0,
                        kinds: int = 0) -> dict:
        """In-sweep rate of the buckets of output rank in [min_width,
        max_width] (0: unbounded): their ops (kinds: bit 0 forward, bit 1
        single-input adjoints, bit 2 fused adjoints; 0 all) as one persistent
        launch of their own (after a sweep).  alg_bytes: the steps'
        algorithmic bytes (as the sweep totals); op_bytes: the ops' operand
        bytes (re-reads of separate adjoint passes included)."""
        ws = self._workspace(with_grad)
        b, ob, ms, n, it = C.c_double(), C.c_double(), C.c_double(), C.c_int64(), C.c_int64()
        L.check(self._lib.qtn_time_wide_sweep(self.handle, int(bool(with_grad)), int(min_width), int(max_width),
                                              int(kinds),
                                              C.c_void_p(ws.data_ptr()), ws.numel(), self._stream(), int(reps),
                                              C.byref(b), C.byref(ob), C.byref(ms), C.byref(n), C.byref(it)))
        return {"alg_bytes": b.value, "op_bytes": ob.value, "ms": ms.value, "ops": n.value, "items": it.value}

    def time_persistent(self, with_grad: bool = True, reps: int = 10) -> float:
        """Average device ms of the sweep's contraction kernels alone (the
        LDS-resident cones' kernel and the persistent kernel; sweeps enqueued
        without graph capture, HIP events around those kernels)."""
        ws = self._workspace(with_grad)
        ms = C.c_double()
        L.check(self._lib.qtn_time_persistent(self.handle, int(bool(with_grad)), C.c_void_p(ws.data_ptr()), ws.numel(),
                                              self._stream(), int(reps), C.byref(ms)))
        return ms.value

    def gemm_census(self, min_bits: int = 4) -> dict:
        """Contraction steps that contain a dense matrix product (two inputs
        sharing >= min_bits summed indices, each with >= min_bits kept indices
        the other lacks) and their share of the plan's flops."""
        ns, ng = C.c_int64(), C.c_int64()
        fg, ft = C.c_double(), C.c_double()
        L.check(self._lib.qtn_gemm_census(self.handle, int(min_bits), C.byref(ns), C.byref(ng), C.byref(fg),
                                          C.byref(ft)))
        return {"steps": ns.value, "gemm_steps": ng.value, "gemm_flops": fg.value, "total_flops": ft.value}

    def set_sweep_timing(self, on: bool) -> None:
        """Record HIP events around every batched sweep for kernel_time (off
        by default: each event adds microseconds to a sweep)."""
        L.check(self._lib.qtn_set_sweep_timing(self.handle, int(bool(on))))

    def kernel_time(self, reset: bool = False) -> Tuple[float, int]:
        """(device ms summed, sweeps) of the batched sweeps timed since the
        last reset (those run with set_sweep_timing(True))."""
        ms = C.c_double()
        cnt = C.c_int64()
        L.check(self._lib.qtn_kernel_time(self.handle, C.byref(ms), C.byref(cnt), int(bool(reset))))
        return ms.value, cnt.value


class QaoaAmplitude(QaoaNet):
    """Single-amplitude network <0...0|gamma beta> of the whole graph (ket
    only; the paper's benchmark object).  Ordering, tuning and parameters work
    as for QaoaNet; read the value with amplitude() / amplitude_grad()."""

    _BUILD = "qtn_build_amplitude"

    def amplitude(self, mode: str = "batched") -> complex:
        ws = self._workspace(False)
        a = np.zeros(2)
        L.check(self._lib.qtn_amplitude(self.handle, _MODES[mode], C.c_void_p(ws.data_ptr()), ws.numel(),
                                        self._stream(), a.ctypes.data_as(C.c_void_p), None))
        return complex(a[0], a[1])

    def amplitude_grad(self, mode: str = "batched"):
        """(amplitude, d amplitude / d gamma [p], d amplitude / d beta [p]), complex."""
        ws = self._workspace(True)
        a = np.zeros(2)
        d = np.zeros(4 * self.p)
        L.check(self._lib.qtn_amplitude(self.handle, _MODES[mode], C.c_void_p(ws.data_ptr()), ws.numel(),
                                        self._stream(), a.ctypes.data_as(C.c_void_p), d.ctypes.data_as(C.c_void_p)))
        z = d[0::2] + 1j * d[1::2]
        return complex(a[0], a[1]), z[: self.p], z[self.p:]
