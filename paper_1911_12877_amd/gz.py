"""Python binding of libgz's C-ABI (include/gz.h): argument marshalling only.

Every step of counting runs inside libgz (host graph preparation and pattern
compilation in C++, the mining loops in HIP kernels).  There is no Python or
CPU fallback: if the library is not built this module raises on first use.

PyTorch is imported before the library is loaded so that both share one HIP
runtime; it is otherwise only used to accept device tensors and streams.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

try:  # one HIP runtime per process: torch's, loaded first
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - torch is part of the image
    torch = None

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_build", "libgz.so")

GZ_OK, GZ_EINVAL, GZ_ENOMEM, GZ_EDEVICE, GZ_EOVERFLOW, GZ_ENOTSUP = 0, -1, -2, -3, -4, -5
GRAPH_NORMALIZE = 1
GRAPH_NO_REINDEX = 2
GRAPH_DEVICE_PTRS = 4
GRAPH_PREP_DEVICE = 8
SCHED_ANALYTIC = 0
SCHED_LEARNED = 1
SCHED_NO_RESTRICT = 8
FEATURES = 108


def mlp_param_count(D, H):
    return H * D + 2 * H + 1


class GzError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"gz status {status}: {message}")
        self.status = status


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"libgz.so is not built ({LIB_PATH}); run "
            "`python -m paper_1911_12877_amd.build` (or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sigs = {
        "gz_load_graph": [P, P, i32, i64, u32, P, P],
        "gz_load_edges": [P, P, i64, i32, u32, P, P],
        "gz_graph_info": [P, P, P, P, P],
        "gz_graph_export": [P, P, P, P],
        "gz_compile_pattern": [P, i32, i32, u32, P],
        "gz_compile_pattern_order": [P, i32, i32, P, u32, P],
        "gz_schedule_info": [P, P, P, P, P, P],
        "gz_enumerate_schedules": [P, i32, i32, P, P, i32, P],
        "gz_count": [P, P, P, P],
        "gz_count_timed": [P, P, P, P, P],
        "gz_count_roots": [P, P, P, i64, P, P],
        "gz_count_subset": [P, P, P, i64, P, P, P],
        "gz_count_noalloc": [P, P, P, P],
        "gz_count_bytes_subset": [P, P, P, i64, P, P, P],
        "gz_count_bytes": [P, P, P, P, P],
        "gz_count_ops": [P, P, P, P, P],
        "gz_census_create": [P, i32, P, i32, P],
        "gz_census_run": [P, P, P],
        "gz_census_tune": [P, P, P],
        "gz_prepare_edges": [P, P, i64, i32, u32, P, P, P, P, P],
        "gz_schedule_features": [P, P, i32, i32, P, P],
        "gz_set_cost_model": [P, i32, i32, ctypes.c_float, i32, P],
        "gz_compile_pattern_graph": [P, P, i32, i32, u32, P],
        "gz_mlp_forward": [P, P, i32, i32, i32, i32, P, P],
        "gz_mlp_loss_grad": [P, P, P, i32, i32, i32, P, P, P],
        "gz_mlp_adam": [P, P, P, P, i32, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                        ctypes.c_float, i32, P],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    lib.gz_free_graph.argtypes = [P]
    lib.gz_free_graph.restype = None
    lib.gz_free_schedule.argtypes = [P]
    lib.gz_free_schedule.restype = None
    lib.gz_census_free.argtypes = [P]
    lib.gz_census_free.restype = None
    lib.gz_last_error.argtypes = []
    lib.gz_last_error.restype = ctypes.c_char_p
    lib.gz_status_string.argtypes = [ctypes.c_int32]
    lib.gz_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def library():
    """The loaded ctypes library (raises if it is not built)."""
    return _load()


def _check(status):
    if status != GZ_OK:
        msg = _load().gz_last_error().decode(errors="replace")
        raise GzError(status, msg)


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _np(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _is_device_tensor(a):
    return torch is not None and isinstance(a, torch.Tensor) and a.is_cuda


class Graph:
    """A prepared graph resident on the GPU (owns a gz_graph handle)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def info(self):
        return graph_info(self)

    def close(self):
        if self._h and self._h.value:
            _load().gz_free_graph(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Schedule:
    """A compiled pattern (owns a gz_schedule handle)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def info(self):
        return schedule_info(self)

    def close(self):
        if self._h and self._h.value:
            _load().gz_free_schedule(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ graphs


def load_graph(rowptr, colidx, n=None, flags=GRAPH_NORMALIZE, stream=None) -> Graph:
    """gz_load_graph: CSR (host arrays or CUDA tensors) -> Graph."""
    lib = _load()
    out = ctypes.c_void_p()
    if _is_device_tensor(rowptr):
        assert rowptr.dtype == torch.int32 and colidx.dtype == torch.int32
        n = rowptr.numel() - 1 if n is None else n
        _check(lib.gz_load_graph(rowptr.data_ptr(), colidx.data_ptr(), n, colidx.numel(),
                                 flags | GRAPH_DEVICE_PTRS, _stream_ptr(stream),
                                 ctypes.byref(out)))
    else:
        r = _np(rowptr, np.int32)
        c = _np(colidx, np.int32)
        n = r.shape[0] - 1 if n is None else n
        _check(lib.gz_load_graph(r.ctypes.data, c.ctypes.data if c.size else None, n,
                                 c.shape[0], flags, _stream_ptr(stream), ctypes.byref(out)))
    return Graph(out.value)


def load_edges(src, dst, n, flags=0, stream=None) -> Graph:
    """gz_load_edges: raw edge list (host arrays or CUDA tensors) -> Graph."""
    lib = _load()
    out = ctypes.c_void_p()
    if _is_device_tensor(src):
        assert src.dtype == torch.int32 and dst.dtype == torch.int32
        _check(lib.gz_load_edges(src.data_ptr(), dst.data_ptr(), src.numel(), n,
                                 flags | GRAPH_DEVICE_PTRS, _stream_ptr(stream),
                                 ctypes.byref(out)))
    else:
        s = _np(src, np.int32)
        d = _np(dst, np.int32)
        _check(lib.gz_load_edges(s.ctypes.data if s.size else None,
                                 d.ctypes.data if d.size else None, s.shape[0], n, flags,
                                 _stream_ptr(stream), ctypes.byref(out)))
    return Graph(out.value)


def graph_info(g: Graph):
    """gz_graph_info -> dict(n, nnz, max_deg, max_lo_deg)."""
    n, nnz = ctypes.c_int32(), ctypes.c_int64()
    md, ml = ctypes.c_int32(), ctypes.c_int32()
    _check(_load().gz_graph_info(g.handle, ctypes.byref(n), ctypes.byref(nnz),
                                 ctypes.byref(md), ctypes.byref(ml)))
    return dict(n=n.value, nnz=nnz.value, max_deg=md.value, max_lo_deg=ml.value)


def graph_export(g: Graph):
    """gz_graph_export -> (rowptr, colidx, old_of_new) as numpy int32."""
    info = graph_info(g)
    r = np.zeros(info["n"] + 1, dtype=np.int32)
    c = np.zeros(max(info["nnz"], 1), dtype=np.int32)
    p = np.zeros(max(info["n"], 1), dtype=np.int32)
    _check(_load().gz_graph_export(g.handle, r.ctypes.data, c.ctypes.data, p.ctypes.data))
    return r, c[:info["nnz"]], p[:info["n"]]


def free_graph(g: Graph):
    g.close()


def prepare_edges(src, dst, n, flags=0):
    """gz_prepare_edges (host only) -> (rowptr, colidx, old_of_new, lo)."""
    s = _np(src, np.int32)
    d = _np(dst, np.int32)
    m = s.shape[0]
    nnz = ctypes.c_int64()
    r = np.zeros(n + 1, dtype=np.int32)
    c = np.zeros(max(2 * m, 1), dtype=np.int32)
    p = np.zeros(max(n, 1), dtype=np.int32)
    lo = np.zeros(max(n, 1), dtype=np.int32)
    _check(_load().gz_prepare_edges(s.ctypes.data if m else None, d.ctypes.data if m else None,
                                    m, n, flags, ctypes.byref(nnz), r.ctypes.data,
                                    c.ctypes.data, p.ctypes.data, lo.ctypes.data))
    return r, c[:nnz.value].copy(), p[:n].copy(), lo[:n].copy()


# ---------------------------------------------------------------- patterns


def _adj_bytes(adj):
    a = _np(adj, np.uint8)
    k = a.shape[0]
    return a.reshape(-1), k


def compile_pattern(adj, induced=True, flags=SCHED_ANALYTIC) -> Schedule:
    a, k = _adj_bytes(adj)
    out = ctypes.c_void_p()
    _check(_load().gz_compile_pattern(a.ctypes.data, k, int(bool(induced)), flags,
                                      ctypes.byref(out)))
    return Schedule(out.value)


def compile_pattern_order(adj, order, induced=True, flags=SCHED_ANALYTIC) -> Schedule:
    a, k = _adj_bytes(adj)
    o = _np(order, np.int8)
    out = ctypes.c_void_p()
    _check(_load().gz_compile_pattern_order(a.ctypes.data, k, int(bool(induced)),
                                            o.ctypes.data, flags, ctypes.byref(out)))
    return Schedule(out.value)


def schedule_info(s: Schedule):
    """gz_schedule_info -> dict(order, bound, aut_size, n_distinct, cost)."""
    o = np.zeros(8, dtype=np.int8)
    b = np.zeros(8, dtype=np.int8)
    aut, nd, cost = ctypes.c_uint64(), ctypes.c_int32(), ctypes.c_double()
    _check(_load().gz_schedule_info(s.handle, o.ctypes.data, b.ctypes.data, ctypes.byref(aut),
                                    ctypes.byref(nd), ctypes.byref(cost)))
    k = int(np.sum(o >= 0))
    return dict(order=tuple(int(x) for x in o[:k]), bound=[int(x) for x in b[:k]],
                aut_size=aut.value, n_distinct=nd.value, cost=cost.value)


def enumerate_schedules(adj, induced=True):
    """gz_enumerate_schedules -> list of (order tuple, analytic cost)."""
    a, k = _adj_bytes(adj)
    lib = _load()
    total = ctypes.c_int32()
    _check(lib.gz_enumerate_schedules(a.ctypes.data, k, int(bool(induced)), None, None, 0,
                                      ctypes.byref(total)))
    nt = total.value
    orders = np.zeros(max(nt, 1) * 8, dtype=np.int8)
    costs = np.zeros(max(nt, 1), dtype=np.float64)
    _check(lib.gz_enumerate_schedules(a.ctypes.data, k, int(bool(induced)), orders.ctypes.data,
                                      costs.ctypes.data, nt, ctypes.byref(total)))
    return [(tuple(int(x) for x in orders[i * 8:i * 8 + k]), float(costs[i]))
            for i in range(nt)]


def free_schedule(s: Schedule):
    s.close()


# ---------------------------------------------------------------- counting


def count(g: Graph, s: Schedule, stream=None) -> int:
    out = ctypes.c_uint64()
    _check(_load().gz_count(g.handle, s.handle, _stream_ptr(stream), ctypes.byref(out)))
    return int(out.value)


def count_noalloc(g: Graph, s: Schedule, stream=None) -> int:
    """gz_count_noalloc: the exact count without any device allocation."""
    out = ctypes.c_uint64()
    _check(_load().gz_count_noalloc(g.handle, s.handle, _stream_ptr(stream), ctypes.byref(out)))
    return int(out.value)


def count_timed(g: Graph, s: Schedule, stream=None):
    """gz_count_timed -> (count, mining kernel milliseconds)."""
    out = ctypes.c_uint64()
    ms = ctypes.c_float()
    _check(_load().gz_count_timed(g.handle, s.handle, _stream_ptr(stream), ctypes.byref(out),
                                  ctypes.byref(ms)))
    return int(out.value), float(ms.value)


def count_roots(g: Graph, s: Schedule, roots, stream=None):
    r = _np(roots, np.int32)
    out = np.zeros(max(r.shape[0], 1), dtype=np.uint64)
    _check(_load().gz_count_roots(g.handle, s.handle, r.ctypes.data if r.size else None,
                                  r.shape[0], _stream_ptr(stream), out.ctypes.data))
    return out[:r.shape[0]]


def count_subset(g: Graph, s: Schedule, roots, stream=None):
    """gz_count_subset -> (count over the listed roots, kernel milliseconds)."""
    r = _np(roots, np.int32)
    out = ctypes.c_uint64()
    ms = ctypes.c_float()
    _check(_load().gz_count_subset(g.handle, s.handle, r.ctypes.data if r.size else None,
                                   r.shape[0], _stream_ptr(stream), ctypes.byref(out),
                                   ctypes.byref(ms)))
    return int(out.value), float(ms.value)


def count_bytes(g: Graph, s: Schedule, stream=None):
    """(algorithmic bytes, count) of one instrumented pass."""
    b, c = ctypes.c_uint64(), ctypes.c_uint64()
    _check(_load().gz_count_bytes(g.handle, s.handle, _stream_ptr(stream), ctypes.byref(b),
                                  ctypes.byref(c)))
    return int(b.value), int(c.value)


def count_bytes_subset(g: Graph, s: Schedule, roots, stream=None):
    """(algorithmic bytes, count) of one instrumented pass over the listed roots."""
    r = _np(roots, np.int32)
    b, c = ctypes.c_uint64(), ctypes.c_uint64()
    _check(_load().gz_count_bytes_subset(g.handle, s.handle, r.ctypes.data if r.size else None,
                                         r.shape[0], _stream_ptr(stream), ctypes.byref(b),
                                         ctypes.byref(c)))
    return int(b.value), int(c.value)


def count_ops(g: Graph, s: Schedule, stream=None):
    """(bit-row intersection lane operations, count) of the clique path."""
    o, c = ctypes.c_uint64(), ctypes.c_uint64()
    _check(_load().gz_count_ops(g.handle, s.handle, _stream_ptr(stream), ctypes.byref(o),
                                ctypes.byref(c)))
    return int(o.value), int(c.value)


def status_string(status: int) -> str:
    return _load().gz_status_string(status).decode()


# ------------------------------------------------------- learned schedules


def schedule_features(g: Graph, adj, order, induced=True):
    """gz_schedule_features -> float32[FEATURES]."""
    a, k = _adj_bytes(adj)
    o = _np(order, np.int8)
    out = np.zeros(FEATURES, dtype=np.float32)
    _check(_load().gz_schedule_features(g.handle, a.ctypes.data, k, int(bool(induced)),
                                        o.ctypes.data, out.ctypes.data))
    return out


GRAPH_STATS = 8


def set_cost_model(params, H=None, margin=0.0, k_max=8, graph_range=None):
    """gz_set_cost_model: install FP32 parameters (None removes the model);
    margin: the predicted gain (log10 time) a learned choice must exceed;
    k_max: the largest pattern size the model was trained on; graph_range:
    (min, max) arrays of the graph statistics over its corpus, or None."""
    if params is None:
        _check(_load().gz_set_cost_model(None, FEATURES, 1, ctypes.c_float(0.0), 8, None))
        return
    p = _np(params, np.float32)
    rng = None
    if graph_range is not None:
        rng = np.concatenate([np.asarray(graph_range[0], np.float32).ravel(),
                              np.asarray(graph_range[1], np.float32).ravel()])
        assert rng.size == 2 * GRAPH_STATS
    _check(_load().gz_set_cost_model(p.ctypes.data, FEATURES, H, ctypes.c_float(margin),
                                     int(k_max), rng.ctypes.data if rng is not None else None))


def compile_pattern_graph(g: Graph, adj, induced=True, flags=SCHED_LEARNED) -> Schedule:
    a, k = _adj_bytes(adj)
    out = ctypes.c_void_p()
    _check(_load().gz_compile_pattern_graph(g.handle, a.ctypes.data, k, int(bool(induced)), flags,
                                            ctypes.byref(out)))
    return Schedule(out.value)


def _dptr(t):
    assert _is_device_tensor(t) and t.dtype == torch.float32 and t.is_contiguous()
    return t.data_ptr()


def mlp_forward(params, X, H, bf16=False, stream=None):
    """gz_mlp_forward on CUDA float32 tensors -> y (CUDA tensor)."""
    n, D = X.shape
    y = torch.empty(n, dtype=torch.float32, device=X.device)
    _check(_load().gz_mlp_forward(_dptr(params), _dptr(X), n, D, H, int(bool(bf16)), _dptr(y),
                                  _stream_ptr(stream)))
    return y


def mlp_loss_grad(params, X, t, H, stream=None):
    """gz_mlp_loss_grad -> (loss, grad tensor)."""
    n, D = X.shape
    grad = torch.empty_like(params)
    loss = ctypes.c_float()
    _check(_load().gz_mlp_loss_grad(_dptr(params), _dptr(X), _dptr(t), n, D, H, _dptr(grad),
                                    ctypes.byref(loss), _stream_ptr(stream)))
    return float(loss.value), grad


def mlp_adam(params, grad, m, v, D, H, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """gz_mlp_adam: one in-place Adam step."""
    _check(_load().gz_mlp_adam(_dptr(params), _dptr(grad), _dptr(m), _dptr(v), D, H, lr, beta1,
                               beta2, eps, step, _stream_ptr(stream)))


# ------------------------------------------------------------------ census


class Census:
    """gz_census: many patterns over many graphs in one captured launch.
    Keeps references to its graphs and schedules."""

    def __init__(self, graphs, scheds):
        self.graphs = list(graphs)
        self.scheds = list(scheds)
        G = (ctypes.c_void_p * len(self.graphs))(*[g.handle.value for g in self.graphs])
        S = (ctypes.c_void_p * len(self.scheds))(*[s.handle.value for s in self.scheds])
        out = ctypes.c_void_p()
        _check(_load().gz_census_create(G, len(self.graphs), S, len(self.scheds),
                                        ctypes.byref(out)))
        self._h = out

    def run(self):
        """-> (counts uint64[n_graphs, n_scheds], device ms)."""
        c = np.zeros(len(self.graphs) * len(self.scheds), dtype=np.uint64)
        ms = ctypes.c_float()
        _check(_load().gz_census_run(self._h, c.ctypes.data, ctypes.byref(ms)))
        return c.reshape(len(self.graphs), len(self.scheds)), float(ms.value)

    def tune(self):
        """-> ((granularity k=3, granularity k>=4, items per pop), best ms)."""
        p = np.zeros(3, dtype=np.int32)
        ms = ctypes.c_float()
        _check(_load().gz_census_tune(self._h, p.ctypes.data, ctypes.byref(ms)))
        return tuple(int(x) for x in p), float(ms.value)

    def close(self):
        if self._h and self._h.value:
            _load().gz_census_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
