"""Thin ctypes binding of libmfard.so (include/mf.h); argument marshalling only.

Every step of the solve runs in the library's HIP kernels.  Host numpy arrays
or device tensors (torch CUDA tensors on ROCm) may be passed as capacities;
torch is used only for device memory and streams.  There is no CPU fallback:
if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmfard.so")

MF_OK, MF_E_INVAL, MF_E_NOMEM, MF_E_DEVICE, MF_E_STATE, MF_E_OVERFLOW, MF_E_SWEEPS = range(7)
MF_CUT_MIN_SOURCE, MF_CUT_MAX_SOURCE = 0, 1
MF_SCHED_PARD, MF_SCHED_COLORED, MF_SCHED_LEARNED, MF_SCHED_AUTO, MF_SCHED_LEARNED_COLORED = 0, 1, 2, 3, 4
MF_KERNEL_AUTO, MF_KERNEL_HBM, MF_KERNEL_LDS, MF_KERNEL_WAVE, MF_KERNEL_ROWS, MF_KERNEL_ROWS64 = 0, 1, 2, 3, 4, 5
MF_METHOD_ARD, MF_METHOD_PRD = 0, 1
MF_REDUCE_STRONG_SOURCE, MF_REDUCE_STRONG_SINK, MF_REDUCE_WEAK_SOURCE, MF_REDUCE_WEAK_SINK = 1, 2, 4, 8
TRACE_FIELDS = 10
FEATURES = 6
TRACE_NAMES = ("sweep", "region", "rounds", "levels", "stages", "ticks", "excess_in", "to_sink",
               "to_boundary", "label_sum")

EXPORTED = ("mf_create_grid", "mf_set_caps", "mf_solve", "mf_flow_value", "mf_min_cut",
            "mf_get_state", "mf_get_info", "mf_discharge_bytes_per_vertex", "mf_destroy",
            "mf_status_str", "mf_create_batch", "mf_batch_info", "mf_batch_set_caps",
            "mf_batch_flow_values", "mf_batch_min_cut", "mf_model_create", "mf_model_destroy",
            "mf_model_num_params", "mf_model_get_params", "mf_model_set_params", "mf_model_forward",
            "mf_model_loss_grad", "mf_model_adam_step", "mf_boundary_relabel", "mf_region_relabel",
            "mf_global_relabel", "mf_model_forward_noalloc", "mf_region_reduction",
            "mf_create_graph", "mf_graph_get_info", "mf_graph_solve", "mf_graph_flow_value",
            "mf_graph_min_cut", "mf_graph_state", "mf_graph_destroy", "mf_graph_discharge_bytes",
            "mf_read_dimacs", "mf_free_dimacs")


class mf_solve_opts(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("global_relabel_every", ctypes.c_int32),
                ("gap", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("max_sweeps", ctypes.c_int64), ("model", ctypes.c_void_p),
                ("stream", ctypes.c_void_p), ("profile", ctypes.c_int32),
                ("region_kernel", ctypes.c_int32), ("trace", ctypes.c_void_p),
                ("trace_cap", ctypes.c_int64), ("graph", ctypes.c_int32),
                ("max_defer", ctypes.c_int32), ("defer_threshold", ctypes.c_float),
                ("defer_mode", ctypes.c_int32), ("features", ctypes.c_void_p),
                ("features_cap", ctypes.c_int64), ("partial", ctypes.c_int32),
                ("boundary_relabel", ctypes.c_int32), ("method", ctypes.c_int32),
                ("label_trace", ctypes.c_void_p), ("label_trace_cap", ctypes.c_int64),
                ("round_cap", ctypes.c_int32)]


class mf_solve_stats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("region_discharges", ctypes.c_int64),
                ("boundary_size", ctypes.c_int64), ("d_inf", ctypes.c_int64),
                ("solve_ms", ctypes.c_double), ("discharge_ms", ctypes.c_double),
                ("discharge_launches", ctypes.c_int64), ("discharge_bytes", ctypes.c_double),
                ("discharged_vertices", ctypes.c_int64), ("discharge_iterations", ctypes.c_int64),
                ("search_levels", ctypes.c_int64), ("search_stages", ctypes.c_int64),
                ("trace_records", ctypes.c_int64), ("search_ticks", ctypes.c_int64),
                ("push_ticks", ctypes.c_int64), ("setup_ticks", ctypes.c_int64),
                ("flood_ticks", ctypes.c_int64), ("global_relabels", ctypes.c_int64),
                ("global_relabel_levels", ctypes.c_int64), ("push_iterations", ctypes.c_int64),
                ("region_kernel", ctypes.c_int64), ("relabel_only", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class mf_graph_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("npairs", ctypes.c_int64), ("regions", ctypes.c_int64),
                ("boundary_size", ctypes.c_int64), ("boundary_pairs", ctypes.c_int64),
                ("page_words", ctypes.c_int64), ("device_pages", ctypes.c_int64),
                ("resident", ctypes.c_int32), ("max_region_vertices", ctypes.c_int32)]


class mf_graph_opts(ctypes.Structure):
    _fields_ = [("max_sweeps", ctypes.c_int64), ("gap", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("round_cap", ctypes.c_int32)]


class mf_graph_stats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("discharges", ctypes.c_int64),
                ("push_rounds", ctypes.c_int64), ("search_steps", ctypes.c_int64),
                ("pages_in", ctypes.c_int64), ("pages_out", ctypes.c_int64),
                ("bytes_h2d", ctypes.c_int64), ("bytes_d2h", ctypes.c_int64), ("ms", ctypes.c_double),
                ("discharged_vertices", ctypes.c_int64), ("discharged_arcs", ctypes.c_int64),
                ("discharge_launches", ctypes.c_int64), ("discharge_ms", ctypes.c_double)]


class mf_dimacs(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("npairs", ctypes.c_int64),
                ("pu", ctypes.POINTER(ctypes.c_int32)), ("pv", ctypes.POINTER(ctypes.c_int32)),
                ("cuv", ctypes.POINTER(ctypes.c_int32)), ("cvu", ctypes.POINTER(ctypes.c_int32)),
                ("cs", ctypes.POINTER(ctypes.c_int32)), ("ct", ctypes.POINTER(ctypes.c_int32)),
                ("st_capacity", ctypes.c_int64), ("vertex_id", ctypes.POINTER(ctypes.c_int64))]


class MFError(RuntimeError):
    def __init__(self, status, where, stats=None):
        self.status = status
        self.stats = stats  # mf_solve on MF_E_SWEEPS: the statistics of the sweeps run
        super().__init__(f"{where}: {status_str(status)} (status {status})")


_lib = None


def load(path: str = LIB_PATH):
    """Load libmfard.so and declare the C ABI; raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing; build it with "
                           "`python -m paper_1109_1146_amd.build` (there is no CPU fallback)")
    # torch ships its own libamdhip64.so.7; loading it first makes the library
    # bind to that same HIP runtime, so device pointers and streams from torch
    # are valid in both (two runtimes in one process leave torch without GPUs).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.mf_create_grid.argtypes = [ctypes.c_int32, P, ctypes.c_int32, P, ctypes.POINTER(P)]
    lib.mf_create_grid.restype = ctypes.c_int
    lib.mf_set_caps.argtypes = [P, P, P, P, ctypes.c_int32, P]
    lib.mf_set_caps.restype = ctypes.c_int
    lib.mf_solve.argtypes = [P, ctypes.POINTER(mf_solve_opts), ctypes.POINTER(mf_solve_stats)]
    lib.mf_solve.restype = ctypes.c_int
    lib.mf_flow_value.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    lib.mf_flow_value.restype = ctypes.c_int
    lib.mf_min_cut.argtypes = [P, ctypes.c_int32, P]
    lib.mf_min_cut.restype = ctypes.c_int
    lib.mf_get_state.argtypes = [P, P, P, P, P]
    lib.mf_get_state.restype = ctypes.c_int
    lib.mf_boundary_relabel.argtypes = [P, ctypes.c_int32, P]
    lib.mf_boundary_relabel.restype = ctypes.c_int
    lib.mf_region_relabel.argtypes = [P, ctypes.c_int32, P]
    lib.mf_region_relabel.restype = ctypes.c_int
    lib.mf_region_reduction.argtypes = [P, ctypes.c_int32, P]
    lib.mf_region_reduction.restype = ctypes.c_int
    lib.mf_global_relabel.argtypes = [P, P]
    lib.mf_global_relabel.restype = ctypes.c_int
    lib.mf_get_info.argtypes = [P, P, P, P, P, P]
    lib.mf_get_info.restype = ctypes.c_int
    lib.mf_discharge_bytes_per_vertex.argtypes = [ctypes.c_int32]
    lib.mf_discharge_bytes_per_vertex.restype = ctypes.c_int64
    lib.mf_destroy.argtypes = [P]
    lib.mf_destroy.restype = None
    lib.mf_status_str.argtypes = [ctypes.c_int]
    lib.mf_status_str.restype = ctypes.c_char_p
    lib.mf_create_batch.argtypes = [ctypes.c_int32, P, P, P, ctypes.POINTER(P)]
    lib.mf_create_batch.restype = ctypes.c_int
    lib.mf_batch_info.argtypes = [P, ctypes.c_int32, P, P]
    lib.mf_batch_info.restype = ctypes.c_int
    lib.mf_batch_set_caps.argtypes = [P, ctypes.c_int32, P, P, P, ctypes.c_int32, P]
    lib.mf_batch_set_caps.restype = ctypes.c_int
    lib.mf_batch_flow_values.argtypes = [P, P]
    lib.mf_batch_flow_values.restype = ctypes.c_int
    lib.mf_batch_min_cut.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P]
    lib.mf_batch_min_cut.restype = ctypes.c_int
    lib.mf_model_create.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(P)]
    lib.mf_model_create.restype = ctypes.c_int
    lib.mf_model_destroy.argtypes = [P]
    lib.mf_model_destroy.restype = None
    lib.mf_model_num_params.argtypes = [P]
    lib.mf_model_num_params.restype = ctypes.c_int64
    lib.mf_model_get_params.argtypes = [P, P]
    lib.mf_model_get_params.restype = ctypes.c_int
    lib.mf_model_set_params.argtypes = [P, P]
    lib.mf_model_set_params.restype = ctypes.c_int
    lib.mf_model_forward.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, P, ctypes.c_int32, P]
    lib.mf_model_forward.restype = ctypes.c_int
    lib.mf_model_forward_noalloc.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, P, ctypes.c_int32, P]
    lib.mf_model_forward_noalloc.restype = ctypes.c_int
    lib.mf_model_loss_grad.argtypes = [P, P, ctypes.c_int32, P, P, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_float), P, P]
    lib.mf_model_loss_grad.restype = ctypes.c_int
    lib.mf_model_adam_step.argtypes = [P, ctypes.c_float, P]
    lib.mf_model_adam_step.restype = ctypes.c_int
    lib.mf_create_graph.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P, P, P, P, ctypes.c_int32,
                                    ctypes.c_int64, ctypes.POINTER(P)]
    lib.mf_create_graph.restype = ctypes.c_int
    lib.mf_graph_get_info.argtypes = [P, ctypes.POINTER(mf_graph_info)]
    lib.mf_graph_get_info.restype = ctypes.c_int
    lib.mf_graph_solve.argtypes = [P, ctypes.POINTER(mf_graph_opts), ctypes.POINTER(mf_graph_stats)]
    lib.mf_graph_solve.restype = ctypes.c_int
    lib.mf_graph_flow_value.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    lib.mf_graph_flow_value.restype = ctypes.c_int
    lib.mf_graph_min_cut.argtypes = [P, ctypes.c_int32, P]
    lib.mf_graph_min_cut.restype = ctypes.c_int
    lib.mf_graph_state.argtypes = [P, P, P, P, P, P]
    lib.mf_graph_state.restype = ctypes.c_int
    lib.mf_graph_destroy.argtypes = [P]
    lib.mf_graph_destroy.restype = None
    lib.mf_graph_discharge_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64]
    lib.mf_graph_discharge_bytes.restype = ctypes.c_int64
    lib.mf_read_dimacs.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.POINTER(mf_dimacs))]
    lib.mf_read_dimacs.restype = ctypes.c_int
    lib.mf_free_dimacs.argtypes = [ctypes.POINTER(mf_dimacs)]
    lib.mf_free_dimacs.restype = None
    _lib = lib
    return lib


def status_str(status: int) -> str:
    return load().mf_status_str(int(status)).decode()


def _check(status, where):
    if status != MF_OK:
        raise MFError(status, where)


def _ptr(a):
    """Host numpy array or device tensor -> (pointer, on_device)."""
    if isinstance(a, np.ndarray):
        if a.dtype != np.int32 or not a.flags["C_CONTIGUOUS"]:
            raise TypeError("capacity arrays must be C-contiguous int32")
        return ctypes.c_void_p(a.ctypes.data), 0
    # torch tensor (duck-typed so this module does not import torch)
    if getattr(a, "dtype", None) is not None and hasattr(a, "data_ptr"):
        import torch
        if a.dtype != torch.int32 or not a.is_contiguous():
            raise TypeError("capacity tensors must be contiguous int32")
        return ctypes.c_void_p(a.data_ptr()), 1 if a.is_cuda else 0
    raise TypeError(f"unsupported array type {type(a)}")


def discharge_bytes_per_vertex(connectivity: int) -> int:
    return int(load().mf_discharge_bytes_per_vertex(int(connectivity)))


class Grid:
    """One solver handle (mf_create_grid ... mf_destroy)."""

    def __init__(self, dims, connectivity, region_shape=None):
        lib = load()
        self.dims = tuple(int(d) for d in dims)
        self.ndim = len(self.dims)
        self.conn = int(connectivity)
        d = (ctypes.c_int64 * self.ndim)(*self.dims)
        rs = None
        if region_shape is not None:
            rs = (ctypes.c_int32 * self.ndim)(*[int(t) for t in region_shape])
        h = ctypes.c_void_p()
        _check(lib.mf_create_grid(self.ndim, d, self.conn, rs, ctypes.byref(h)), "mf_create_grid")
        self._h = h
        self.n = int(np.prod(self.dims))
        self.K = self.conn

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().mf_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def info(self):
        n = ctypes.c_int64()
        K = ctypes.c_int32()
        regs = ctypes.c_int64()
        b = ctypes.c_int64()
        rs = (ctypes.c_int32 * 3)()
        _check(load().mf_get_info(self._h, ctypes.byref(n), ctypes.byref(K), ctypes.byref(regs),
                                  ctypes.byref(b), rs), "mf_get_info")
        return dict(n=n.value, K=K.value, regions=regs.value, boundary_size=b.value,
                    region_shape=tuple(rs[3 - self.ndim:]))

    def set_caps(self, cs, ct, nbr, stream=None):
        p1, d1 = _ptr(cs)
        p2, d2 = _ptr(ct)
        p3, d3 = _ptr(nbr)
        if not (d1 == d2 == d3):
            raise ValueError("capacity arrays must all be on the host or all on the device")
        for a, size in ((cs, self.n), (ct, self.n), (nbr, self.K * self.n)):
            numel = a.size if isinstance(a, np.ndarray) else a.numel()
            if int(numel) != size:
                raise ValueError(f"expected {size} capacities, got {int(numel)}")
        st = ctypes.c_void_p(stream) if stream else None
        _check(load().mf_set_caps(self._h, p1, p2, p3, d1, st), "mf_set_caps")

    def solve(self, schedule=MF_SCHED_PARD, gap=True, global_relabel_every=0, check_every=0,
              max_sweeps=0, stream=None, profile=False, region_kernel=MF_KERNEL_AUTO,
              trace=None, graph=False, model=None, max_defer=0, defer_threshold=0.0,
              features=None, defer_mode=0, partial=False, boundary_relabel=0,
              method=MF_METHOD_ARD, label_trace=None, round_cap=0):
        """trace: optional int32 device tensor of shape (cap, TRACE_FIELDS);
        round_cap: n > 0 caps a region discharge at n search-and-push rounds per sweep;
        partial: partial discharges (sweep s runs the stages k <= s only);
        boundary_relabel: n > 0 runs the boundary relabel heuristic after every
        sweep with at most n levels of its search;
        method: MF_METHOD_ARD or MF_METHOD_PRD (push-relabel region discharge);
        label_trace: optional int32 device tensor of shape (cap, n): the labels
        after every step."""
        tptr, tcap = None, 0
        if trace is not None:
            tptr, tcap = trace.data_ptr(), int(trace.shape[0])
        fptr, fcap = None, 0
        if features is not None:
            fptr, fcap = features.data_ptr(), int(features.shape[0])
        o = mf_solve_opts(schedule=schedule, global_relabel_every=global_relabel_every,
                          gap=1 if gap else 0, check_every=check_every, max_sweeps=max_sweeps,
                          model=None, stream=stream, profile=1 if profile else 0,
                          region_kernel=region_kernel, trace=tptr, trace_cap=tcap,
                          graph=1 if graph else 0, max_defer=max_defer,
                          defer_threshold=defer_threshold, defer_mode=defer_mode, features=fptr,
                          features_cap=fcap, partial=1 if partial else 0,
                          boundary_relabel=int(boundary_relabel), method=int(method),
                          label_trace=label_trace.data_ptr() if label_trace is not None else None,
                          label_trace_cap=int(label_trace.shape[0]) if label_trace is not None else 0,
                          round_cap=int(round_cap))
        if model is not None:
            o.model = model._h
        s = mf_solve_stats()
        rc = load().mf_solve(self._h, ctypes.byref(o), ctypes.byref(s))
        if rc == MF_E_SWEEPS:
            raise MFError(rc, "mf_solve", s.as_dict())
        _check(rc, "mf_solve")
        return s.as_dict()

    def flow_value(self):
        f = ctypes.c_int64()
        _check(load().mf_flow_value(self._h, ctypes.byref(f)), "mf_flow_value")
        return int(f.value)

    def min_cut(self, kind=MF_CUT_MIN_SOURCE):
        out = np.zeros(self.n, dtype=np.uint8)
        _check(load().mf_min_cut(self._h, int(kind), ctypes.c_void_p(out.ctypes.data)),
               "mf_min_cut")
        return out

    def state(self):
        res = np.zeros((self.K, self.n), dtype=np.int32)
        rt = np.zeros(self.n, dtype=np.int32)
        ex = np.zeros(self.n, dtype=np.int32)
        lab = np.zeros(self.n, dtype=np.int32)
        P = lambda a: ctypes.c_void_p(a.ctypes.data)
        _check(load().mf_get_state(self._h, P(res), P(rt), P(ex), P(lab)), "mf_get_state")
        return dict(res=res, rt=rt, ex=ex, labels=lab)

    def region_relabel(self, region_kernel=MF_KERNEL_AUTO):
        """Region relabel (Alg. 3) of every region on the state of the last solve;
        returns the number of regions relabelled."""
        n = ctypes.c_int64()
        _check(load().mf_region_relabel(self._h, int(region_kernel), ctypes.byref(n)),
               "mf_region_relabel")
        return int(n.value)

    def region_reduction(self, region_kernel=MF_KERNEL_AUTO):
        """Region reduction (Alg. 5) of every region of the loaded instance: one
        class byte per vertex (MF_REDUCE_* bits); overwrites the solver state."""
        out = np.zeros(self.n, dtype=np.uint8)
        _check(load().mf_region_reduction(self._h, int(region_kernel), ctypes.c_void_p(out.ctypes.data)),
               "mf_region_reduction")
        return out

    def global_relabel(self):
        """Exact region-distance relabel on the state of the last solve; returns
        the number of level launches."""
        n = ctypes.c_int64()
        _check(load().mf_global_relabel(self._h, ctypes.byref(n)), "mf_global_relabel")
        return int(n.value)

    def boundary_relabel(self, max_levels=1 << 30):
        """Boundary relabel heuristic on the state of the last solve (also one
        stopped by max_sweeps); returns the number of levels that reached a vertex."""
        lv = ctypes.c_int64()
        _check(load().mf_boundary_relabel(self._h, int(max_levels), ctypes.byref(lv)),
               "mf_boundary_relabel")
        return int(lv.value)


class Batch(Grid):
    """Many independent 2D instances solved together (mf_create_batch ... mf_destroy)."""

    def __init__(self, dims_list, conn_list, region_shape=None):
        lib = load()
        self.count = len(dims_list)
        self.inst_dims = [tuple(int(x) for x in d) for d in dims_list]
        self.inst_conn = [int(c) for c in conn_list]
        d = (ctypes.c_int64 * (2 * self.count))(*[x for dd in self.inst_dims for x in dd])
        c = (ctypes.c_int32 * self.count)(*self.inst_conn)
        rs = None
        if region_shape is not None:
            rs = (ctypes.c_int32 * 2)(*[int(t) for t in region_shape])
        h = ctypes.c_void_p()
        _check(lib.mf_create_batch(self.count, d, c, rs, ctypes.byref(h)), "mf_create_batch")
        self._h = h
        off = (ctypes.c_int64 * 2)()
        dims = (ctypes.c_int64 * 2)()
        _check(lib.mf_batch_info(self._h, -1, off, dims), "mf_batch_info")
        self.dims = (dims[0], dims[1])
        self.ndim = 2
        self.n = int(dims[0] * dims[1])
        self.K = 8 if 8 in self.inst_conn else 4
        self.conn = self.K

    def placement(self, i):
        off = (ctypes.c_int64 * 2)()
        dims = (ctypes.c_int64 * 2)()
        _check(load().mf_batch_info(self._h, int(i), off, dims), "mf_batch_info")
        return (off[0], off[1]), (dims[0], dims[1])

    def set_caps(self, i, cs, ct, nbr, stream=None):  # noqa: D401 - per instance
        p1, d1 = _ptr(cs)
        p2, d2 = _ptr(ct)
        p3, d3 = _ptr(nbr)
        if not (d1 == d2 == d3):
            raise ValueError("capacity arrays must all be on the host or all on the device")
        n = self.inst_dims[i][0] * self.inst_dims[i][1]
        for a, size in ((cs, n), (ct, n), (nbr, self.inst_conn[i] * n)):
            numel = a.size if isinstance(a, np.ndarray) else a.numel()
            if int(numel) != size:
                raise ValueError(f"instance {i}: expected {size} capacities, got {int(numel)}")
        st = ctypes.c_void_p(stream) if stream else None
        _check(load().mf_batch_set_caps(self._h, int(i), p1, p2, p3, d1, st), "mf_batch_set_caps")

    def flow_values(self):
        out = np.zeros(self.count, dtype=np.int64)
        _check(load().mf_batch_flow_values(self._h, ctypes.c_void_p(out.ctypes.data)),
               "mf_batch_flow_values")
        return out

    def instance_cut(self, i, kind=MF_CUT_MIN_SOURCE):
        h, w = self.inst_dims[i]
        out = np.zeros(h * w, dtype=np.uint8)
        _check(load().mf_batch_min_cut(self._h, int(i), int(kind), ctypes.c_void_p(out.ctypes.data)),
               "mf_batch_min_cut")
        return out


class Model:
    """The scheduler CNN (mf_model_*).  Tensors are torch CUDA float32 tensors."""

    def __init__(self, channels=16, seed=0):
        h = ctypes.c_void_p()
        _check(load().mf_model_create(int(channels), int(seed), ctypes.byref(h)), "mf_model_create")
        self._h = h
        self.channels = int(channels)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().mf_model_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self):
        return int(load().mf_model_num_params(self._h))

    def get_params(self):
        out = np.zeros(self.num_params, dtype=np.float32)
        _check(load().mf_model_get_params(self._h, ctypes.c_void_p(out.ctypes.data)), "get_params")
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.num_params
        _check(load().mf_model_set_params(self._h, ctypes.c_void_p(p.ctypes.data)), "set_params")

    def forward(self, x, dims, bf16=True, stream=None):
        """x: CUDA float32 tensor [D*H*W, xs]; returns logits tensor [D*H*W]."""
        import torch
        D, H, W = dims
        out = torch.empty(D * H * W, dtype=torch.float32, device=x.device)
        _check(load().mf_model_forward(self._h, ctypes.c_void_p(x.data_ptr()), int(x.shape[1]), D, H, W,
                                       ctypes.c_void_p(out.data_ptr()), 1 if bf16 else 0,
                                       ctypes.c_void_p(stream) if stream else None), "forward")
        return out

    def forward_noalloc(self, x, out, dims, bf16=True, stream=None):
        """mf_model_forward_noalloc: logits of the D*H*W grid x into the caller's
        float32 tensor out, with no device allocation."""
        D, H, W = dims
        _check(load().mf_model_forward_noalloc(self._h, ctypes.c_void_p(x.data_ptr()), int(x.shape[1]), D, H, W,
                                               ctypes.c_void_p(out.data_ptr()), 1 if bf16 else 0,
                                               ctypes.c_void_p(stream) if stream else None),
               "forward_noalloc")
        return out

    def loss_grad(self, x, target, mask, dims, want_grads=False, stream=None):
        D, H, W = dims
        loss = ctypes.c_float()
        g = np.zeros(self.num_params, dtype=np.float32) if want_grads else None
        _check(load().mf_model_loss_grad(
            self._h, ctypes.c_void_p(x.data_ptr()), int(x.shape[1]), ctypes.c_void_p(target.data_ptr()),
            ctypes.c_void_p(mask.data_ptr()), D, H, W, ctypes.byref(loss),
            ctypes.c_void_p(g.ctypes.data) if g is not None else None,
            ctypes.c_void_p(stream) if stream else None), "loss_grad")
        return float(loss.value), g

    def adam_step(self, lr, stream=None):
        _check(load().mf_model_adam_step(self._h, float(lr), ctypes.c_void_p(stream) if stream else None),
               "adam_step")


def load_batch(instances, region_shape=None):
    """Create a Batch for synth.GridInstance objects (2D) and load their caps."""
    b = Batch([inst.dims for inst in instances], [inst.conn for inst in instances], region_shape)
    for i, inst in enumerate(instances):
        b.set_caps(i, np.ascontiguousarray(inst.cs, np.int32), np.ascontiguousarray(inst.ct, np.int32),
                   np.ascontiguousarray(inst.nbr, np.int32))
    return b


def solve_instance(inst, tile=None, **solve_kw):
    """Solve a synth.GridInstance; returns dict(flow, smin, smax, stats)."""
    tile = tile if tile is not None else inst.tile
    with Grid(inst.dims, inst.conn, tile) as g:
        g.set_caps(np.ascontiguousarray(inst.cs, np.int32), np.ascontiguousarray(inst.ct, np.int32),
                   np.ascontiguousarray(inst.nbr, np.int32))
        st = g.solve(**solve_kw)
        out = dict(flow=g.flow_value(), smin=g.min_cut(MF_CUT_MIN_SOURCE),
                   smax=g.min_cut(MF_CUT_MAX_SOURCE), stats=st, info=g.info())
        out["state"] = g.state()
    return out


def _host_i32(a, n, what):
    a = np.ascontiguousarray(a, dtype=np.int32)
    if a.shape != (n,):
        raise ValueError(f"{what} must have shape ({n},)")
    return a


class Graph:
    """A general network in region pages (mf_create_graph ... mf_graph_destroy).

    Pairs (pu, pv, cuv, cvu) and t-links (cs, ct) are host int32 arrays; region
    is an int32 array of region numbers or None for blocks of region_size
    consecutive vertices; device_pages 0 keeps every page in device memory,
    k >= 1 streams them through k device page slots."""

    def __init__(self, n, pu, pv, cuv, cvu, cs, ct, region=None, region_size=4096, device_pages=0):
        lib = load()
        n = int(n)
        m = int(np.asarray(pu).shape[0])
        arrs = [_host_i32(a, m, w) for a, w in ((pu, "pu"), (pv, "pv"), (cuv, "cuv"), (cvu, "cvu"))]
        arrs += [_host_i32(a, n, w) for a, w in ((cs, "cs"), (ct, "ct"))]
        reg = None if region is None else _host_i32(region, n, "region")
        self.n, self.npairs = n, m
        h = ctypes.c_void_p()
        ptrs = [ctypes.c_void_p(a.ctypes.data) for a in arrs]
        _check(lib.mf_create_graph(n, m, *ptrs, ctypes.c_void_p(reg.ctypes.data) if reg is not None else None,
                                   int(region_size), int(device_pages), ctypes.byref(h)), "mf_create_graph")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().mf_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def info(self):
        i = mf_graph_info()
        _check(load().mf_graph_get_info(self._h, ctypes.byref(i)), "mf_graph_get_info")
        return {f: getattr(i, f) for f, _ in mf_graph_info._fields_}

    def solve(self, max_sweeps=0, gap=True, check_every=0, profile=False, round_cap=0):
        """round_cap: n > 0 caps a region discharge at n push rounds per sweep."""
        o = mf_graph_opts(int(max_sweeps), 1 if gap else 0, int(check_every), 1 if profile else 0,
                          int(round_cap))
        st = mf_graph_stats()
        _check(load().mf_graph_solve(self._h, ctypes.byref(o), ctypes.byref(st)), "mf_graph_solve")
        return {f: getattr(st, f) for f, _ in mf_graph_stats._fields_}

    def flow_value(self):
        v = ctypes.c_int64()
        _check(load().mf_graph_flow_value(self._h, ctypes.byref(v)), "mf_graph_flow_value")
        return int(v.value)

    def min_cut(self, kind=MF_CUT_MIN_SOURCE):
        out = np.zeros(max(self.n, 1), dtype=np.uint8)
        _check(load().mf_graph_min_cut(self._h, int(kind), ctypes.c_void_p(out.ctypes.data)), "mf_graph_min_cut")
        return out[:self.n]

    def state(self):
        m, n = max(self.npairs, 1), max(self.n, 1)
        r_uv, r_vu = np.zeros(m, np.int64), np.zeros(m, np.int64)
        rt, ex, lab = np.zeros(n, np.int64), np.zeros(n, np.int64), np.zeros(n, np.int32)
        _check(load().mf_graph_state(self._h, *[ctypes.c_void_p(a.ctypes.data) for a in (r_uv, r_vu, rt, ex, lab)]),
               "mf_graph_state")
        return dict(r_uv=r_uv[:self.npairs], r_vu=r_vu[:self.npairs], rt=rt[:self.n], ex=ex[:self.n],
                    labels=lab[:self.n])


def solve_graph(inst, region=None, region_size=4096, device_pages=0, **solve_kw):
    """Solve a synth.GraphInstance; returns dict(flow, smin, smax, stats, info, state)."""
    region = region if region is not None else inst.region
    with Graph(inst.n, inst.pu, inst.pv, inst.cuv, inst.cvu, inst.cs, inst.ct, region=region,
               region_size=region_size, device_pages=device_pages) as g:
        st = g.solve(**solve_kw)
        out = dict(flow=g.flow_value(), smin=g.min_cut(MF_CUT_MIN_SOURCE), smax=g.min_cut(MF_CUT_MAX_SOURCE),
                   stats=st, info=g.info())
        out["state"] = g.state()
    return out


def graph_discharge_bytes(nv, na) -> int:
    return int(load().mf_graph_discharge_bytes(int(nv), int(na)))


def read_dimacs(path):
    """A DIMACS max-flow file through the library's reader (mf_read_dimacs): a
    dict with n, the pair arrays pu, pv, cuv, cvu, the t-links cs, ct (numpy
    int32 copies), st_capacity (flow of the arcs from s straight to t) and
    vertex_id (the file id of every vertex)."""
    lib = load()
    d = ctypes.POINTER(mf_dimacs)()
    _check(lib.mf_read_dimacs(str(path).encode(), ctypes.byref(d)), "mf_read_dimacs")
    try:
        r = d.contents
        n, m = int(r.n), int(r.npairs)
        arr = lambda ptr, k: np.ctypeslib.as_array(ptr, shape=(k,)).copy() if k else np.zeros(0, np.int32)
        out = dict(n=n, pu=arr(r.pu, m), pv=arr(r.pv, m), cuv=arr(r.cuv, m), cvu=arr(r.cvu, m),
                   cs=arr(r.cs, n), ct=arr(r.ct, n), st_capacity=int(r.st_capacity),
                   vertex_id=(np.ctypeslib.as_array(r.vertex_id, shape=(n,)).copy() if n else np.zeros(0, np.int64)))
    finally:
        lib.mf_free_dimacs(d)
    return out
