"""ctypes binding of libgmrf (C ABI in include/gmrf.h).

Argument marshalling only: every step of the sampler runs in the HIP
library.  PyTorch supplies device workspaces (uint8 tensors sized by the
library's footprint queries) and the stream (torch's current stream).  If
libgmrf.so has not been built, every entry point raises; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgmrf.so")

OK, E_INVALID_ARG, E_GRAPH, E_COLORING, E_WORKSPACE, E_DEVICE, E_NUMERIC = range(7)
STATUS_NAMES = {0: "GMRF_OK", 1: "GMRF_E_INVALID_ARG", 2: "GMRF_E_GRAPH",
                3: "GMRF_E_COLORING", 4: "GMRF_E_WORKSPACE", 5: "GMRF_E_DEVICE",
                6: "GMRF_E_NUMERIC"}
FP64, FP32_ACC64 = 0, 1
WITH_HYPER, CAPTURE = 1, 2
NUM_TILES = 3
GAUSSIAN, BINOMIAL = 0, 1
PTR_HOST, PTR_DEVICE = 0, 1


class GmrfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class GraphDesc(C.Structure):
    _fields_ = [("n", C.c_int64), ("row_ptr", C.POINTER(C.c_int64)),
                ("col_idx", C.POINTER(C.c_int32)), ("color", C.POINTER(C.c_int32)),
                ("num_colors", C.c_int32), ("lat_rows", C.c_int32), ("lat_cols", C.c_int32),
                ("lat_stencil", C.c_int32), ("rho", C.c_double)]


class Model(C.Structure):
    _fields_ = [("a_tau", C.c_double), ("b_tau", C.c_double), ("a_lam", C.c_double),
                ("b_lam", C.c_double), ("tau0", C.c_double), ("lam0", C.c_double),
                ("burn_in", C.c_int64), ("intercept", C.c_int32), ("likelihood", C.c_int32),
                ("beta0", C.c_double), ("beta0_var", C.c_double), ("rng_version", C.c_int32)]


_lib = None

_SIGS = {
    "gmrf_last_error": ([], C.c_char_p),
    "gmrf_version": ([], C.c_int),
    "gmrf_graph_footprint": ([C.POINTER(GraphDesc)], C.c_size_t),
    "gmrf_graph_create": ([C.POINTER(GraphDesc), C.c_void_p, C.c_size_t, C.c_void_p,
                           C.POINTER(C.c_void_p)], C.c_int),
    "gmrf_graph_destroy": ([C.c_void_p], C.c_int),
    "gmrf_graph_info": ([C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                         C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
    "gmrf_greedy_coloring": ([C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                              C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "gmrf_chain_footprint": ([C.c_void_p, C.c_int], C.c_size_t),
    "gmrf_chain_create": ([C.c_void_p, C.POINTER(Model), C.POINTER(C.c_double),
                           C.POINTER(C.c_double), C.c_int, C.c_uint64, C.c_uint32, C.c_void_p,
                           C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "gmrf_chain_destroy": ([C.c_void_p], C.c_int),
    "gmrf_binomial_footprint": ([C.c_void_p, C.c_int, C.POINTER(C.c_int32)], C.c_size_t),
    "gmrf_chain_create_binomial": ([C.c_void_p, C.POINTER(Model), C.POINTER(C.c_double),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_int,
                                    C.c_uint64, C.c_uint32, C.c_void_p, C.c_size_t, C.c_void_p,
                                    C.POINTER(C.c_void_p)], C.c_int),
    "gmrf_sweep": ([C.c_void_p, C.c_int32, C.c_uint32, C.c_void_p], C.c_int),
    "gmrf_sweep_static": ([C.c_void_p, C.c_int32, C.c_uint32, C.c_void_p], C.c_int),
    "gmrf_sweep_timed": ([C.c_void_p, C.c_int32, C.c_uint32, C.c_void_p,
                          C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "gmrf_hyper_update": ([C.c_void_p, C.c_void_p], C.c_int),
    "gmrf_set_hyper": ([C.c_void_p, C.c_double, C.c_double, C.c_void_p], C.c_int),
    "gmrf_posterior_stats": ([C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64),
                              C.c_uint32, C.c_void_p], C.c_int),
    "gmrf_get_state": ([C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                        C.POINTER(C.c_double), C.POINTER(C.c_uint64), C.c_void_p], C.c_int),
    "gmrf_set_state": ([C.c_void_p, C.POINTER(C.c_double), C.c_double, C.c_double, C.c_uint64,
                        C.c_void_p], C.c_int),
    "gmrf_get_accumulators": ([C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                               C.POINTER(C.c_int64), C.c_void_p], C.c_int),
    "gmrf_set_accumulators": ([C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                               C.c_int64, C.c_void_p], C.c_int),
    "gmrf_last_reductions": ([C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.c_void_p], C.c_int),
    "gmrf_get_intercept": ([C.c_void_p, C.POINTER(C.c_double), C.c_void_p], C.c_int),
    "gmrf_set_intercept": ([C.c_void_p, C.c_double, C.c_void_p], C.c_int),
    "gmrf_set_trace": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p], C.c_int),
    "gmrf_chain_get_tile": ([C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                             C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "gmrf_chain_set_tile": ([C.c_void_p, C.c_int32], C.c_int),
    "gmrf_chain_autotune": ([C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_int32),
                             C.POINTER(C.c_double)], C.c_int),
    "gmrf_batch_footprint": ([C.POINTER(C.c_void_p), C.c_int32], C.c_size_t),
    "gmrf_batch_create": ([C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                           C.POINTER(C.c_void_p)], C.c_int),
    "gmrf_batch_destroy": ([C.c_void_p], C.c_int),
    "gmrf_batch_sweep": ([C.c_void_p, C.c_int32, C.c_uint32, C.c_void_p], C.c_int),
    "gmrf_batch_autotune": ([C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_int32),
                             C.POINTER(C.c_double)], C.c_int),
}


def lib():
    """Load libgmrf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no CPU fallback)")
        # Device memory and streams come from torch: let torch bring up the
        # HIP runtime before the library's first HIP call, so that both use
        # the devices torch sees.
        _torch().cuda.is_available()
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        raise GmrfError(rc, lib().gmrf_last_error().decode())


def _p(a, ctype):
    return None if a is None else a.ctypes.data_as(C.POINTER(ctype))


def greedy_coloring(row_ptr, col_idx):
    """First-fit greedy coloring (host); returns (color int32[n], k)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = rp.size - 1
    color = np.zeros(max(n, 1), dtype=np.int32)
    k = C.c_int32(0)
    _check(lib().gmrf_greedy_coloring(n, _p(rp, C.c_int64), _p(cl if cl.size else None,
                                                                  C.c_int32),
                                      _p(color, C.c_int32), C.byref(k)))
    return color[:n].copy(), int(k.value)


def _torch():
    import torch

    return torch


def _stream_handle(stream):
    if stream is None:
        torch = _torch()
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _workspace(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class _Desc:
    """Keeps the numpy arrays of a GraphDesc alive."""

    def __init__(self, n=None, row_ptr=None, col_idx=None, color=None, num_colors=0,
                 lattice=None, rho=1.0):
        self.rp = None if row_ptr is None else np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.cl = None if col_idx is None else np.ascontiguousarray(col_idx, dtype=np.int32)
        if self.cl is not None and self.cl.size == 0:
            self.cl = np.zeros(1, dtype=np.int32)
        self.co = None if color is None else np.ascontiguousarray(color, dtype=np.int32)
        rows = cols = st = 0
        if lattice is not None:
            rows, cols, st = (int(v) for v in lattice)
            if n is None:
                n = rows * cols
        if n is None:
            n = self.rp.size - 1
        self.desc = GraphDesc(int(n), _p(self.rp, C.c_int64), _p(self.cl, C.c_int32),
                              _p(self.co, C.c_int32), int(num_colors), rows, cols, st,
                              float(rho))


def validate_graph(**kw) -> int:
    """Run the library's graph checks without a device workspace: returns the
    status code (GMRF_E_WORKSPACE means the description itself is valid; a
    lattice, which needs no workspace, returns GMRF_OK)."""
    d = _Desc(**kw)
    h = C.c_void_p()
    rc = lib().gmrf_graph_create(C.byref(d.desc), None, 0, None, C.byref(h))
    if rc == OK:
        lib().gmrf_graph_destroy(h)
    return rc


def last_error() -> str:
    return lib().gmrf_last_error().decode()


class Graph:
    """A validated graph on the device (CSR color slabs or an implicit lattice).

    ``lattice=(rows, cols, stencil)`` selects the lattice path; otherwise pass
    ``row_ptr``, ``col_idx``, ``color`` and ``num_colors``.
    """

    def __init__(self, *, n=None, row_ptr=None, col_idx=None, color=None, num_colors=0,
                 lattice=None, rho=1.0, device="cuda", stream=None):
        L = lib()
        self._d = _Desc(n, row_ptr, col_idx, color, num_colors, lattice, rho)
        self.device = device
        need = L.gmrf_graph_footprint(C.byref(self._d.desc))
        self.ws = _workspace(need, device) if need else None
        h = C.c_void_p()
        _check(L.gmrf_graph_create(C.byref(self._d.desc),
                                   None if self.ws is None else C.c_void_p(self.ws.data_ptr()),
                                   need, _stream_handle(stream), C.byref(h)))
        self.handle = h
        n_, k_, comp, nnz = C.c_int64(), C.c_int32(), C.c_int64(), C.c_int64()
        _check(L.gmrf_graph_info(h, C.byref(n_), C.byref(k_), C.byref(comp), C.byref(nnz)))
        self.n, self.k, self.components, self.nnz = n_.value, k_.value, comp.value, nnz.value
        self.rho = float(rho)
        self.is_lattice = lattice is not None
        self.lattice = lattice

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.gmrf_graph_destroy(h)
            self.handle = None


class Chain:
    """One Markov chain (state, accumulators, tau, lam and, with
    ``intercept=True``, beta0) of a Graph on the device."""

    def __init__(self, graph: Graph, y, *, precision=FP64, seed=1, instance=0, x0=None,
                 a_tau=1.0, b_tau=1.0, a_lam=1.0, b_lam=1.0, tau0=1.0, lam0=1.0, burn_in=0,
                 intercept=False, beta0=0.0, trials=None, beta0_var=0.0, rng_version=1,
                 stream=None):
        """With ``trials`` (m_i) the chain is the binomial logit model and y
        holds the successes Y_i; ``beta0_var`` is then the prior variance of
        beta0 (0 = flat).  ``rng_version`` 2 selects the paired site normals
        (lattices of width a multiple of 4)."""
        L = lib()
        self.graph = graph
        self.n = graph.n
        self.precision = precision
        self.trace_buf = None
        binom = trials is not None
        self.model = Model(a_tau, b_tau, a_lam, b_lam, tau0, lam0, int(burn_in),
                           1 if intercept else 0, BINOMIAL if binom else GAUSSIAN, float(beta0),
                           float(beta0_var), int(rng_version))
        if binom:
            tt = np.ascontiguousarray(trials, dtype=np.int32)
            if tt.size != self.n:
                raise ValueError("trials must have n entries")
            need = L.gmrf_binomial_footprint(graph.handle, precision, _p(tt, C.c_int32))
        else:
            need = L.gmrf_chain_footprint(graph.handle, precision)
        if need == 0:
            raise GmrfError(E_INVALID_ARG, last_error())
        self.footprint = need
        self.ws = _workspace(need, graph.device)
        yy = np.ascontiguousarray(y, dtype=np.float64)
        if yy.size != self.n:
            raise ValueError("y must have n entries")
        xx = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        h = C.c_void_p()
        if binom:
            _check(L.gmrf_chain_create_binomial(
                graph.handle, C.byref(self.model), _p(yy, C.c_double), _p(tt, C.c_int32),
                _p(xx, C.c_double), precision, int(seed), int(instance),
                C.c_void_p(self.ws.data_ptr()), need, _stream_handle(stream), C.byref(h)))
        else:
            _check(L.gmrf_chain_create(graph.handle, C.byref(self.model), _p(yy, C.c_double),
                                       _p(xx, C.c_double), precision, int(seed), int(instance),
                                       C.c_void_p(self.ws.data_ptr()), need,
                                       _stream_handle(stream), C.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.gmrf_chain_destroy(h)
            self.handle = None

    # sampling -------------------------------------------------------------
    def sweep(self, nsweeps: int = 1, hyper: bool = True, capture: bool = False, stream=None):
        flags = (WITH_HYPER if hyper else 0) | (CAPTURE if capture else 0)
        _check(lib().gmrf_sweep(self.handle, int(nsweeps), flags, _stream_handle(stream)))
        return self

    def sweep_static(self, nsweeps: int = 1, hyper: bool = True, stream=None):
        """gmrf_sweep_static: the same sweeps with the library's fixed device
        scratch instead of the workspace's (allocates nothing)."""
        _check(lib().gmrf_sweep_static(self.handle, int(nsweeps), WITH_HYPER if hyper else 0,
                                       _stream_handle(stream)))
        return self

    def sweep_timed(self, nsweeps: int, hyper: bool = True, stream=None, span=False):
        """Run nsweeps sweeps (plain launches) and return the summed duration in
        ms of their sweep kernels, from HIP events the dispatches record around
        those kernels; with span=True return (kernel_ms, span_ms), span_ms
        being the device time from the first sweep kernel's start to the end
        of the last sweep."""
        ms, sp = C.c_double(), C.c_double()
        _check(lib().gmrf_sweep_timed(self.handle, int(nsweeps), WITH_HYPER if hyper else 0,
                                      _stream_handle(stream), C.byref(ms), C.byref(sp)))
        return (ms.value, sp.value) if span else ms.value

    def hyper_update(self, stream=None):
        _check(lib().gmrf_hyper_update(self.handle, _stream_handle(stream)))

    def set_hyper(self, tau: float, lam: float, stream=None):
        _check(lib().gmrf_set_hyper(self.handle, float(tau), float(lam), _stream_handle(stream)))

    # results --------------------------------------------------------------
    def posterior_stats(self, stream=None):
        mean = np.empty(self.n)
        var = np.empty(self.n)
        nacc = C.c_int64()
        _check(lib().gmrf_posterior_stats(self.handle, mean.ctypes.data, var.ctypes.data,
                                          C.byref(nacc), PTR_HOST, _stream_handle(stream)))
        return mean, var, nacc.value

    def posterior_stats_device(self, mean, var, stream=None):
        """Write mean / var into device tensors (float64, n entries); async."""
        _check(lib().gmrf_posterior_stats(self.handle, mean.data_ptr(), var.data_ptr(), None,
                                          PTR_DEVICE, _stream_handle(stream)))

    def get_state(self, stream=None):
        x = np.empty(self.n)
        tau, lam, sw = C.c_double(), C.c_double(), C.c_uint64()
        _check(lib().gmrf_get_state(self.handle, _p(x, C.c_double), C.byref(tau), C.byref(lam),
                                    C.byref(sw), _stream_handle(stream)))
        return x, tau.value, lam.value, sw.value

    def set_state(self, x, tau, lam, sweep, stream=None):
        xx = None if x is None else np.ascontiguousarray(x, dtype=np.float64)
        _check(lib().gmrf_set_state(self.handle, _p(xx, C.c_double), float(tau), float(lam),
                                    int(sweep), _stream_handle(stream)))

    def get_accumulators(self, stream=None):
        s1, s2, nacc = np.empty(self.n), np.empty(self.n), C.c_int64()
        _check(lib().gmrf_get_accumulators(self.handle, _p(s1, C.c_double), _p(s2, C.c_double),
                                           C.byref(nacc), _stream_handle(stream)))
        return s1, s2, nacc.value

    def set_accumulators(self, s1, s2, n_acc, stream=None):
        a = np.ascontiguousarray(s1, dtype=np.float64)
        b = np.ascontiguousarray(s2, dtype=np.float64)
        _check(lib().gmrf_set_accumulators(self.handle, _p(a, C.c_double), _p(b, C.c_double),
                                           int(n_acc), _stream_handle(stream)))

    def last_reductions(self, stream=None):
        q, s = C.c_double(), C.c_double()
        _check(lib().gmrf_last_reductions(self.handle, C.byref(q), C.byref(s),
                                          _stream_handle(stream)))
        return q.value, s.value

    @property
    def tile(self):
        """(shape index, tile rows, tile cols, threads).  Lattices: shapes 0, 1
        (64x64 / 32x32 tiles) and 2 (one persistent block).  General graphs
        (tile 0 x 0): 0 (one launch per color), 1 (chunks staged in LDS, one
        launch per sweep) or 2 (one block, field in LDS)."""
        k, r, c, t = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().gmrf_chain_get_tile(self.handle, C.byref(k), C.byref(r), C.byref(c),
                                         C.byref(t)))
        return k.value, r.value, c.value, t.value

    def set_tile(self, shape: int):
        _check(lib().gmrf_chain_set_tile(self.handle, int(shape)))

    def autotune(self, reps: int = 50, stream=None):
        """Time each tile shape on this chain (state unchanged), keep the
        fastest; returns (best shape, [us per sweep of each shape])."""
        best = C.c_int32()
        us = (C.c_double * NUM_TILES)()
        _check(lib().gmrf_chain_autotune(self.handle, int(reps), _stream_handle(stream),
                                         C.byref(best), us))
        return best.value, list(us)

    @property
    def beta0(self) -> float:
        b = C.c_double()
        _check(lib().gmrf_get_intercept(self.handle, C.byref(b), _stream_handle(None)))
        return b.value

    def set_intercept(self, beta0: float, stream=None):
        _check(lib().gmrf_set_intercept(self.handle, float(beta0), _stream_handle(stream)))

    def enable_trace(self, capacity: int, stream=None):
        """Record (tau, lam, beta0) after every sweep t < capacity into a device
        buffer (float64 tensor of shape (capacity, 3), read it with trace())."""
        torch = _torch()
        buf = torch.full((int(capacity), 3), float("nan"), dtype=torch.float64,
                         device=self.graph.device)
        _check(lib().gmrf_set_trace(self.handle, C.c_void_p(buf.data_ptr()), int(capacity),
                                    _stream_handle(stream)))
        self.trace_buf = buf

    def disable_trace(self, stream=None):
        _check(lib().gmrf_set_trace(self.handle, None, 0, _stream_handle(stream)))
        self.trace_buf = None

    def trace(self, stream=None) -> np.ndarray:
        """The recorded (tau, lam, beta0) rows as a host array (synchronises)."""
        if self.trace_buf is None:
            raise RuntimeError("trace: enable_trace() was not called")
        torch = _torch()
        if stream is not None:
            stream.synchronize()
        else:
            torch.cuda.current_stream().synchronize()
        return self.trace_buf.cpu().numpy()


class Batch:
    """Many chains (one precision) advanced together by shared launches; each
    chain's results equal its standalone sweeps bit for bit."""

    def __init__(self, chains, stream=None):
        L = lib()
        self.chains = list(chains)
        arr = (C.c_void_p * len(self.chains))(*[c.handle.value for c in self.chains])
        need = L.gmrf_batch_footprint(arr, len(self.chains))
        if need == 0:
            raise GmrfError(E_INVALID_ARG, last_error())
        self.ws = _workspace(need, self.chains[0].graph.device)
        h = C.c_void_p()
        _check(L.gmrf_batch_create(arr, len(self.chains), C.c_void_p(self.ws.data_ptr()), need,
                                   _stream_handle(stream), C.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.gmrf_batch_destroy(h)
            self.handle = None

    def sweep(self, nsweeps: int = 1, hyper: bool = True, capture: bool = False, stream=None):
        flags = (WITH_HYPER if hyper else 0) | (CAPTURE if capture else 0)
        _check(lib().gmrf_batch_sweep(self.handle, int(nsweeps), flags, _stream_handle(stream)))
        return self

    def autotune(self, reps: int = 10, stream=None):
        """Time the batch's lattice tiles in shapes 0 and 1 (chain state
        unchanged) and keep the faster; returns (best shape or -1, [us per
        pass of each shape])."""
        best = C.c_int32()
        us = (C.c_double * 2)()
        _check(lib().gmrf_batch_autotune(self.handle, int(reps), _stream_handle(stream),
                                         C.byref(best), us))
        return best.value, list(us)
