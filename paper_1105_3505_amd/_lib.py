"""ctypes declarations for include/lfmm.h and small Python wrappers with the same names."""
from __future__ import annotations

import ctypes
import os
import re
import warnings
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblfmm.so")
_HEADER = os.path.join(os.path.dirname(_HERE), "include", "lfmm.h")

PRECISIONS = {"fp64": 0, "mixed": 1, "mixed-bf16": 2}
STENCILS = {5: 0, 9: 1, "5": 0, "9": 1, "5-point": 0, "9-point": 1}

_i32, _i64, _dbl, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class LfmmError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__("lfmm status %d: %s" % (status, detail))
        self.status = status


class LfmmWarning(UserWarning):
    """A call succeeded with a warning status (> 0), e.g. loads whose total is not zero."""

    def __init__(self, status: int, detail: str):
        super().__init__("lfmm status %d: %s" % (status, detail))
        self.status = status


class _Options(ctypes.Structure):
    _fields_ = [("eps", _dbl), ("max_leaf", _i32), ("precision", _i32), ("proxy_per_edge", _i32),
                ("max_rank", _i32), ("flags", _i32), ("stencil", _i32)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("n_points", _i64), ("n_instances", _i32), ("root_bits", _i32), ("leaf_level", _i32),
                ("leaf_side", _i64),
                ("rank", _i32), ("leaf_kind", _i32), ("n_boxes", _i64), ("n_leaves", _i64),
                ("near_pairs", _i64), ("m2l_pairs", _i64), ("device_bytes", _i64), ("n_targets", _i64),
                ("adaptive", _i32), ("pad0", _i32), ("m2p_terms", _i64), ("p2l_terms", _i64)]


class _ServerOptions(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_batch", _i32), ("max_inflight", _i32),
                ("max_batch_points", _i64)]


class _SolverOptions(ctypes.Structure):
    _fields_ = [("tol", _dbl), ("max_iter", _i32), ("restart", _i32)]


class _SolverStats(ctypes.Structure):
    _fields_ = [("iterations", _i32), ("converged", _i32), ("rel_residual", _dbl)]


class _RequestStats(ctypes.Structure):
    _fields_ = [("status", _i32), ("batch_size", _i32), ("batch_id", _i64), ("t_submit", _dbl),
                ("t_admit", _dbl), ("t_done", _dbl)]


STATUS_BUSY = -7
STATUS_NONZERO_SUM = 1
FLAG_GRAPH = 1
FLAG_CHECK_LOADS = 2
FLAG_ADAPTIVE = 4


def library_path() -> str:
    return _LIB_PATH


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError("liblfmm.so is not built; run `python paper_1105_3505_amd/build.py`")
    # PyTorch ships its own HIP runtime.  Load it first, so that the library binds to that
    # same runtime (it is looked up by its soname): loaded the other way round, the process
    # would hold two HIP runtimes and the library would see no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "lfmm_options_init": [_vp],
        "lfmm_ctx_create": [_i32, _vp, _vp],
        "lfmm_ctx_destroy": [_vp],
        "lfmm_plan_create": [_vp, _i64, _vp, _i64, _vp, _vp, _vp],
        "lfmm_plan_create_batch": [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp],
        "lfmm_execute": [_vp, _vp, _vp, _vp],
        "lfmm_execute_instances": [_vp, _vp, _vp, _vp],
        "lfmm_execute_sorted": [_vp, _vp, _vp, _vp],
        "lfmm_execute_batch": [_vp, _i32, _vp, _vp, _vp, _vp],
        "lfmm_plan_get_info": [_vp, _vp],
        "lfmm_autotune": [_vp, _i64, _vp, _i32, _vp, _i32, _i32, _vp, _vp, _vp],
        "lfmm_autotune_batch": [_vp, _i32, _vp, _vp, _i32, _vp, _i32, _i32, _vp, _vp, _vp],
        "lfmm_plan_set_timing": [_vp, _i32],
        "lfmm_plan_set_timing_phases": [_vp, ctypes.c_uint32],
        "lfmm_plan_export": [_vp, _i32, _vp, _vp],
        "lfmm_plan_phase_times": [_vp, _vp],
        "lfmm_plan_footprint_bytes": [_vp, _i64, _i64, _i32, _vp],
        "lfmm_plan_destroy": [_vp],
        "lfmm_solve": [_vp, _i64, _vp, _vp, _vp, _vp],
        "lfmm_solve_static": [_vp, _i64, _vp, _vp, _vp, _vp],
        "lfmm_direct": [_vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp],
        "lfmm_host_phi": [_i32, _i64, _vp, _vp],
        "lfmm_host_opset_create": [_i64, _i32, _vp, _vp],
        "lfmm_host_opset_level": [_vp, _i32, _vp, _vp],
        "lfmm_host_opset_skeleton": [_vp, _i32, _vp],
        "lfmm_host_opset_ofo": [_vp, _i32, _i32, _vp],
        "lfmm_host_opset_leaf": [_vp, _vp],
        "lfmm_host_opset_destroy": [_vp],
        "lfmm_server_create": [_vp, _vp, _vp],
        "lfmm_server_submit": [_vp, _i64, _vp, _vp, _vp, _vp, _vp],
        "lfmm_server_wait": [_vp, ctypes.c_uint64, _dbl, _vp],
        "lfmm_server_destroy": [_vp],
        "lfmm_inclusions_create": [_vp, _i64, _vp, _vp, _vp, _vp],
        "lfmm_inclusions_nodes": [_vp, _vp, _vp],
        "lfmm_inclusions_solve": [_vp, _dbl, _dbl, _vp, _vp, _vp, _vp],
        "lfmm_inclusions_potential": [_vp, _dbl, _dbl, _vp, _i64, _vp, _vp, _vp],
        "lfmm_inclusions_destroy": [_vp],
        "lfmm_dirichlet_create": [_vp, _i64, _vp, _vp, _vp, _vp],
        "lfmm_dirichlet_apply": [_vp, _vp, _vp, _vp],
        "lfmm_dirichlet_solve": [_vp, _vp, _vp, _vp, _vp, _vp],
        "lfmm_dirichlet_potential": [_vp, _vp, _i64, _vp, _vp, _vp],
        "lfmm_dirichlet_destroy": [_vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.lfmm_status_string.argtypes = [ctypes.c_int]
    lib.lfmm_status_string.restype = ctypes.c_char_p
    lib.lfmm_last_error.argtypes = []
    lib.lfmm_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()


def _check(status: int) -> int:
    """Raises LfmmError for an error status (< 0); a warning status (> 0) is issued as an
    LfmmWarning and returned."""
    if status != 0:
        detail = (_lib.lfmm_last_error() or b"").decode(errors="replace")
        name = (_lib.lfmm_status_string(status) or b"").decode()
        if status > 0:
            warnings.warn(LfmmWarning(status, "%s: %s" % (name, detail)), stacklevel=3)
            return status
        raise LfmmError(status, "%s: %s" % (name, detail))
    return 0


def exported_symbols() -> list[str]:
    """Every function name declared in include/lfmm.h."""
    with open(_HEADER) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"\b(lfmm_[a-z_0-9]+)\s*\(", text)))


def _options(eps=None, max_leaf=None, precision=None, proxy_per_edge=None, max_rank=None,
             flags=None, graph=None, check_loads=None, stencil=None, adaptive=None) -> _Options:
    o = _Options()
    _check(_lib.lfmm_options_init(ctypes.byref(o)))
    if eps is not None:
        o.eps = float(eps)
    if max_leaf is not None:
        o.max_leaf = int(max_leaf)
    if precision is not None:
        o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    if proxy_per_edge is not None:
        o.proxy_per_edge = int(proxy_per_edge)
    if max_rank is not None:
        o.max_rank = int(max_rank)
    if flags is not None:
        o.flags = int(flags)
    if graph:
        o.flags |= FLAG_GRAPH
    if check_loads:
        o.flags |= FLAG_CHECK_LOADS
    if adaptive:
        o.flags |= FLAG_ADAPTIVE
    if stencil is not None:
        o.stencil = STENCILS[stencil]
    return o


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _empty_on(stream, n, device):
    """A float64 output of n entries that the library writes on `stream`: allocated on that
    stream, so that torch's caching allocator orders its reuse after the write."""
    import torch
    if stream is None:
        return torch.empty(n, dtype=torch.float64, device=device)
    with torch.cuda.stream(stream):
        return torch.empty(n, dtype=torch.float64, device=device)


def _keep_for(stream, *tensors):
    """Marks tensors the library reads or writes on a stream other than torch's current one,
    so that the caching allocator does not hand their memory out before that stream is done."""
    import torch
    if stream is None or stream == torch.cuda.current_stream():
        return
    for t in tensors:
        t.record_stream(stream)


def _dev_tensor(t, dtype, shape_tail, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must live on the GPU" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s" % (name, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape_tail is not None and tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError("%s must have shape [n, %s]" % (name, ",".join(map(str, shape_tail))))
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """lfmm_ctx: a device, the phi table and the operator cache."""

    def __init__(self, device: int = 0, **opts):
        self._opts = _options(**opts)
        h = ctypes.c_void_p()
        _check(_lib.lfmm_ctx_create(int(device), ctypes.byref(self._opts), ctypes.byref(h)))
        self._h = h
        self.device = int(device)
        self._plans = weakref.WeakSet()
        self._servers = weakref.WeakSet()

    def close(self) -> None:
        """Destroys the context; its servers and live plans are destroyed first."""
        if getattr(self, "_h", None):
            for s in list(self._servers):
                s.close()
            for p in list(self._plans):
                p.close()
            _lib.lfmm_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def plan(self, xy, targets=None, stream=None) -> "Plan":
        """lfmm_plan_create over the sources xy [n, 2]; `targets` [m, 2] (optional) are the
        points where the potentials are wanted (default: the sources)."""
        import torch
        ptr = _dev_tensor(xy, torch.int32, (2,), "xy")
        nt, tp = 0, None
        if targets is not None:
            if int(targets.shape[0]) < 1:
                raise ValueError("targets must hold at least one point (None: targets = sources)")
            tp = _dev_tensor(targets, torch.int32, (2,), "targets")
            nt = int(targets.shape[0])
        h = ctypes.c_void_p()
        _check(_lib.lfmm_plan_create(self._h, int(xy.shape[0]), ptr, nt, tp, _stream_handle(stream),
                                     ctypes.byref(h)))
        plan = Plan(self, h, [int(xy.shape[0])], [nt if targets is not None else int(xy.shape[0])],
                    n_points=int(xy.shape[0]) + nt)
        self._plans.add(plan)
        return plan

    def plan_batch(self, xys, targets=None, stream=None) -> "Plan":
        """One plan over several point sets (lfmm_plan_create_batch): every pass is one
        launch over all of them; each instance's result equals that of a plan of its own.
        targets: None, or a list with one entry per instance (None = its sources)."""
        import torch
        k = len(xys)
        ptrs = (ctypes.c_void_p * k)(*[_dev_tensor(xy, torch.int32, (2,), "xy").value for xy in xys])
        sizes = np.ascontiguousarray([int(xy.shape[0]) for xy in xys], dtype=np.int64)
        tsz, tptrs = None, None
        outs = [int(v) for v in sizes]
        if targets is not None:
            if len(targets) != k:
                raise ValueError("one target entry per instance")
            tsz = np.ascontiguousarray([0 if t is None else int(t.shape[0]) for t in targets], dtype=np.int64)
            tptrs = (ctypes.c_void_p * k)(*[None if t is None else _dev_tensor(t, torch.int32, (2,), "targets").value
                                            for t in targets])
            outs = [o if t is None else int(t.shape[0]) for o, t in zip(outs, targets)]
        h = ctypes.c_void_p()
        _check(_lib.lfmm_plan_create_batch(self._h, k, sizes.ctypes.data_as(_vp), ptrs,
                                           None if tsz is None else tsz.ctypes.data_as(_vp), tptrs,
                                           _stream_handle(stream), ctypes.byref(h)))
        plan = Plan(self, h, [int(v) for v in sizes], outs,
                    n_points=int(sizes.sum()) + (0 if tsz is None else int(tsz.sum())))
        self._plans.add(plan)
        return plan

    def solve(self, xy, f, u=None, stream=None):
        """lfmm_solve (targets = sources).  A non-zero total load gives an LfmmWarning."""
        import torch
        n = int(xy.shape[0])
        if u is None:
            u = _empty_on(stream, n, f.device)
        _check(_lib.lfmm_solve(self._h, n, _dev_tensor(xy, torch.int32, (2,), "xy"),
                               _dev_tensor(f, torch.float64, (), "f"), _dev_tensor(u, torch.float64, (), "u"),
                               _stream_handle(stream)))
        return u

    def solve_static(self, xy, f, u, stream=None):
        """lfmm_solve_static: lfmm_solve with no allocation (the library's static workspace,
        at most 65,536 points); u is the caller's preallocated output."""
        import torch
        n = int(xy.shape[0])
        if int(f.shape[0]) != n or int(u.shape[0]) != n:
            raise ValueError("f and u must have one entry per point")
        _check(_lib.lfmm_solve_static(self._h, n, _dev_tensor(xy, torch.int32, (2,), "xy"),
                                      _dev_tensor(f, torch.float64, (), "f"), _dev_tensor(u, torch.float64, (), "u"),
                                      _stream_handle(stream)))
        return u

    def direct(self, txy, sxy, f, u=None, stream=None):
        import torch
        nt, ns = int(txy.shape[0]), int(sxy.shape[0])
        if u is None:
            u = _empty_on(stream, nt, f.device)
        _check(_lib.lfmm_direct(self._h, nt, _dev_tensor(txy, torch.int32, (2,), "txy"), ns,
                                _dev_tensor(sxy, torch.int32, (2,), "sxy"), _dev_tensor(f, torch.float64, (), "f"),
                                _dev_tensor(u, torch.float64, (), "u"), _stream_handle(stream)))
        return u

    def execute_batch(self, plans, fs, us, stream=None):
        import torch
        k = len(plans)
        hp = (ctypes.c_void_p * k)(*[p._h for p in plans])
        fp = (ctypes.c_void_p * k)(*[_dev_tensor(f, torch.float64, (), "f").value for f in fs])
        up = (ctypes.c_void_p * k)(*[_dev_tensor(u, torch.float64, (), "u").value for u in us])
        _check(_lib.lfmm_execute_batch(self._h, k, hp, fp, up, _stream_handle(stream)))
        return us

    def autotune(self, xy, candidates=(16, 32, 64, 128), objective="solve", reps=3, stream=None):
        """lfmm_autotune: the fastest N_leaf among `candidates` for this point set; the
        context remembers it for point sets of similar size and density (used when the
        context's max_leaf is 0).  Returns (best, {candidate: ms})."""
        import torch
        cand = np.ascontiguousarray(candidates, dtype=np.int32)
        ms = np.zeros(len(cand), dtype=np.float64)
        best = ctypes.c_int32()
        obj = {"solve": 0, "execute": 1}[objective]
        _check(_lib.lfmm_autotune(self._h, int(xy.shape[0]), _dev_tensor(xy, torch.int32, (2,), "xy"), len(cand),
                                  cand.ctypes.data_as(_vp), obj, int(reps), _stream_handle(stream),
                                  ctypes.byref(best), ms.ctypes.data_as(_vp)))
        return int(best.value), dict(zip([int(c) for c in cand], [float(v) for v in ms]))

    def autotune_batch(self, xys, candidates=(16, 32, 64, 128), objective="execute", reps=3, stream=None):
        """lfmm_autotune_batch: the fastest N_leaf among `candidates` for a plan of all the point
        sets `xys` (each candidate applied to every instance); recorded for the size and density
        class of each instance.  Returns (best, {candidate: ms})."""
        import torch
        k = len(xys)
        ptrs = (ctypes.c_void_p * k)(*[_dev_tensor(xy, torch.int32, (2,), "xy").value for xy in xys])
        sizes = np.ascontiguousarray([int(xy.shape[0]) for xy in xys], dtype=np.int64)
        cand = np.ascontiguousarray(candidates, dtype=np.int32)
        ms = np.zeros(len(cand), dtype=np.float64)
        best = ctypes.c_int32()
        obj = {"solve": 0, "execute": 1}[objective]
        _check(_lib.lfmm_autotune_batch(self._h, k, sizes.ctypes.data_as(_vp), ptrs, len(cand),
                                        cand.ctypes.data_as(_vp), obj, int(reps), _stream_handle(stream),
                                        ctypes.byref(best), ms.ctypes.data_as(_vp)))
        return int(best.value), dict(zip([int(c) for c in cand], [float(v) for v in ms]))

    def footprint_bytes(self, n_src: int, n_tgt: int = 0, root_bits: int = -1) -> int:
        """lfmm_plan_footprint_bytes: bound on the device bytes of a plan (root_bits -1: any
        extent below 2^31)."""
        out = ctypes.c_size_t()
        _check(_lib.lfmm_plan_footprint_bytes(self._h, int(n_src), int(n_tgt), int(root_bits), ctypes.byref(out)))
        return int(out.value)


class Plan:
    """lfmm_plan: the trees of one or more point sets (instances), resident on the device."""

    def __init__(self, ctx: Context, handle, sizes, out_sizes=None, n_points=None):
        self.ctx = ctx
        self._h = handle
        self.sizes = list(sizes)                    # sources per instance
        self.out_sizes = list(out_sizes if out_sizes is not None else sizes)   # targets per instance
        self.n = sum(self.sizes)
        self.n_out = sum(self.out_sizes)
        self._n_points = n_points                   # points of the plan: sources and separate targets

    def execute(self, f, u=None, stream=None):
        """lfmm_execute: f has one load per source, u one potential per target."""
        import torch
        if int(f.shape[0]) != self.n:
            raise ValueError("f must have one load per source")
        if u is None:
            u = _empty_on(stream, self.n_out, f.device)
        elif int(u.shape[0]) != self.n_out:
            raise ValueError("u must have one entry per target")
        _check(_lib.lfmm_execute(self._h, _dev_tensor(f, torch.float64, (), "f"),
                                 _dev_tensor(u, torch.float64, (), "u"), _stream_handle(stream)))
        _keep_for(stream, f, u)
        return u

    def execute_sorted(self, f, u=None, stream=None):
        """lfmm_execute_sorted: f and u span every point of the plan in its Morton order
        (export("perm") gives each point's caller index)."""
        import torch
        if self._n_points is None:   # get_info reads back plan statistics: once
            self._n_points = int(self.info()["n_points"])
        n_all = self._n_points
        if int(f.shape[0]) != n_all:
            raise ValueError("f must have one entry per point of the plan (%d)" % n_all)
        if u is None:
            u = _empty_on(stream, n_all, f.device)
        elif int(u.shape[0]) != n_all:
            raise ValueError("u must have one entry per point of the plan (%d)" % n_all)
        _check(_lib.lfmm_execute_sorted(self._h, _dev_tensor(f, torch.float64, (), "f"),
                                        _dev_tensor(u, torch.float64, (), "u"), _stream_handle(stream)))
        _keep_for(stream, f, u)
        return u

    def execute_instances(self, fs, us=None, stream=None):
        """lfmm_execute_instances: fs[k] (and us[k]) belong to instance k."""
        import torch
        k = len(self.sizes)
        if len(fs) != k:
            raise ValueError("one load vector per instance")
        for f, n in zip(fs, self.sizes):
            if int(f.shape[0]) != n:
                raise ValueError("f must have one load per source of its instance")
        if us is None:
            us = [_empty_on(stream, n, f.device) for f, n in zip(fs, self.out_sizes)]
        for u, n in zip(us, self.out_sizes):
            if int(u.shape[0]) != n:
                raise ValueError("u must have one entry per target of its instance")
        fp = (ctypes.c_void_p * k)(*[_dev_tensor(f, torch.float64, (), "f").value for f in fs])
        up = (ctypes.c_void_p * k)(*[_dev_tensor(u, torch.float64, (), "u").value for u in us])
        _check(_lib.lfmm_execute_instances(self._h, fp, up, _stream_handle(stream)))
        _keep_for(stream, *fs, *us)
        return us

    PHASES = ("gather", "p2m", "m2m", "m2l", "l2l", "leaf")
    EXPORTS = {"points": (0, np.int32, 2), "perm": (1, np.int32, 0), "level_base": (2, np.int32, 0),
               "box_key": (3, np.uint64, 0), "box_begin": (4, np.int32, 0), "box_end": (5, np.int32, 0),
               "box_parent": (6, np.int32, 0), "box_child": (7, np.int32, 4), "interaction": (8, np.int32, 27),
               "neighbor": (9, np.int32, 9), "qhat": (10, np.float64, 48), "uhat": (11, np.float64, 48),
               "loads": (12, np.float64, 0), "level_count": (13, np.int32, 0), "box_level": (14, np.int8, 0),
               "box_instance": (15, np.int32, 0), "box_role": (16, np.int8, 0)}
    LISTS = {"U": 17, "W": 18, "X": 19}

    def export(self, name: str) -> np.ndarray:
        """Copy of a plan internal (lfmm_plan_export) as a numpy array."""
        item, dtype, width = self.EXPORTS[name]
        size = ctypes.c_size_t()
        _check(_lib.lfmm_plan_export(self._h, item, None, ctypes.byref(size)))
        out = np.empty(size.value // np.dtype(dtype).itemsize, dtype=dtype)
        if size.value:
            _check(_lib.lfmm_plan_export(self._h, item, out.ctypes.data_as(_vp), ctypes.byref(size)))
        return out.reshape(-1, width) if width else out

    def export_list(self, name: str):
        """Adaptive plans: list `name` ("U", "W" or "X") as (row starts [n_boxes + 1], entries)."""
        item = self.LISTS[name]
        size = ctypes.c_size_t()
        _check(_lib.lfmm_plan_export(self._h, item, None, ctypes.byref(size)))
        out = np.empty(size.value // 4, dtype=np.int32)
        _check(_lib.lfmm_plan_export(self._h, item, out.ctypes.data_as(_vp), ctypes.byref(size)))
        nb = int(self.info()["n_boxes"])
        return out[:nb + 1], out[nb + 1:]

    def set_timing(self, enable: bool = True) -> None:
        _check(_lib.lfmm_plan_set_timing(self._h, 1 if enable else 0))

    def set_timing_phases(self, phases) -> None:
        """Time only the named phases (events around them alone); an empty list turns timing off."""
        mask = 0
        for name in phases:
            mask |= 1 << self.PHASES.index(name)
        _check(_lib.lfmm_plan_set_timing_phases(self._h, mask))

    def phase_times(self) -> dict:
        """Milliseconds per timed phase of the last timed execute (HIP events on its stream)."""
        out = (ctypes.c_double * len(self.PHASES))()
        _check(_lib.lfmm_plan_phase_times(self._h, out))
        return {k: v for k, v in zip(self.PHASES, list(out)) if v == v}

    def info(self) -> dict:
        i = _PlanInfo()
        _check(_lib.lfmm_plan_get_info(self._h, ctypes.byref(i)))
        return {name: getattr(i, name) for name, _ in _PlanInfo._fields_}

    def close(self) -> None:
        if getattr(self, "_h", None):
            # a closed context has destroyed its plans already (garbage collection may finalise
            # the context first)
            if getattr(self.ctx, "_h", None):
                _lib.lfmm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def host_phi(mxy, stencil=5) -> np.ndarray:
    """The library's phi of the given lattice operator (5 or 9 point) at integer offsets
    (host computation, no GPU)."""
    m = np.ascontiguousarray(np.asarray(mxy, dtype=np.int32).reshape(-1, 2))
    out = np.empty(len(m), dtype=np.float64)
    _check(_lib.lfmm_host_phi(STENCILS[stencil], len(m), m.ctypes.data_as(_vp), out.ctypes.data_as(_vp)))
    return out


class HostOperators:
    """Host copy of the operators for one leaf side (lfmm_opset)."""

    def __init__(self, leaf_side: int, n_levels: int, **opts):
        o = _options(**opts)
        h = ctypes.c_void_p()
        _check(_lib.lfmm_host_opset_create(int(leaf_side), int(n_levels), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.n_levels = int(n_levels)
        self.leaf_side = int(leaf_side)

    def level(self, h: int):
        side, rank = ctypes.c_int64(), ctypes.c_int32()
        _check(_lib.lfmm_host_opset_level(self._h, int(h), ctypes.byref(side), ctypes.byref(rank)))
        return int(side.value), int(rank.value)

    def skeleton(self, h: int) -> np.ndarray:
        _, r = self.level(h)
        out = np.empty(2 * r, dtype=np.int64)
        _check(_lib.lfmm_host_opset_skeleton(self._h, int(h), out.ctypes.data_as(_vp)))
        return out.reshape(r, 2)

    def ofo(self, h: int, c: int) -> np.ndarray:
        _, r = self.level(h)
        _, rc = self.level(h - 1)
        out = np.empty((r, rc), dtype=np.float64)
        _check(_lib.lfmm_host_opset_ofo(self._h, int(h), int(c), out.ctypes.data_as(_vp)))
        return out

    def leaf(self) -> np.ndarray:
        _, r = self.level(0)
        out = np.empty((r, self.leaf_side ** 2), dtype=np.float64)
        _check(_lib.lfmm_host_opset_leaf(self._h, out.ctypes.data_as(_vp)))
        return out

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.lfmm_host_opset_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """lfmm_server: continuous batching of solve requests over one context.

    The server's worker thread owns the context while the server lives: make no other
    call on that context until close().  submit() and wait() may be called from any thread.
    """

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 0, max_batch: int = 0, max_inflight: int = 0,
                 max_batch_points: int = 0):
        o = _ServerOptions(int(hbm_budget_bytes), int(max_batch), int(max_inflight), int(max_batch_points))
        h = ctypes.c_void_p()
        _check(_lib.lfmm_server_create(ctx._h, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        self._held = {}          # ticket -> tensors the device reads or writes until done
        ctx._servers.add(self)

    def submit(self, xy, f, u=None, stream=None) -> int:
        """Queues a solve; `stream` (default: torch's current stream) is where xy and f were
        written: the server reads them only after the work queued there so far."""
        import torch
        n = int(xy.shape[0])
        if int(f.shape[0]) != n:
            raise ValueError("f must have one load per point")
        if u is None:
            u = torch.empty(n, dtype=torch.float64, device=f.device)
        t = ctypes.c_uint64()
        _check(_lib.lfmm_server_submit(self._h, n, _dev_tensor(xy, torch.int32, (2,), "xy"),
                                       _dev_tensor(f, torch.float64, (), "f"),
                                       _dev_tensor(u, torch.float64, (), "u"), _stream_handle(stream),
                                       ctypes.byref(t)))
        self._held[int(t.value)] = (xy, f, u)
        return int(t.value)

    def wait(self, ticket: int, timeout=None):
        """Waits for a request; returns (u, stats dict).  Raises LfmmError with status
        STATUS_BUSY if it is not done within `timeout` seconds."""
        st = _RequestStats()
        status = _lib.lfmm_server_wait(self._h, ctypes.c_uint64(int(ticket)),
                                       -1.0 if timeout is None else float(timeout), ctypes.byref(st))
        if status == STATUS_BUSY:
            _check(status)
        held = self._held.pop(int(ticket), None)
        _check(status)
        stats = {name: getattr(st, name) for name, _ in _RequestStats._fields_}
        return held[2], stats

    def close(self) -> None:
        """Serves every queued request, then stops the worker."""
        if getattr(self, "_h", None):
            if getattr(self.ctx, "_h", None):   # else destroyed with its context
                _lib.lfmm_server_destroy(self._h)
            self._h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _solver_options(tol=None, max_iter=None, restart=None) -> _SolverOptions:
    return _SolverOptions(float(tol or 0.0), int(max_iter or 0), int(restart or 0))


class Inclusions:
    """lfmm_inclusions: a lattice whose bars are modified (Section 10.1).  bars: [n, 4] int32
    (a1, a2, b1, b2) and delta: [n] float64 (host arrays); the resident plan applies S on the
    nodes the bars touch."""

    def __init__(self, ctx: Context, bars, delta, stream=None):
        b = np.ascontiguousarray(np.asarray(bars, dtype=np.int32).reshape(-1, 4))
        d = np.ascontiguousarray(np.asarray(delta, dtype=np.float64).reshape(-1))
        if len(b) != len(d):
            raise ValueError("one conductance change per bar")
        h = ctypes.c_void_p()
        _check(_lib.lfmm_inclusions_create(ctx._h, len(b), b.ctypes.data_as(_vp), d.ctypes.data_as(_vp),
                                           _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        ctx._plans.add(self)          # closed before the context, which would free its plan
        n = ctypes.c_int64()
        _check(_lib.lfmm_inclusions_nodes(self._h, ctypes.byref(n), None))
        self.nodes = np.empty((n.value, 2), dtype=np.int32)
        _check(_lib.lfmm_inclusions_nodes(self._h, ctypes.byref(n), self.nodes.ctypes.data_as(_vp)))

    def solve(self, c1: float, c2: float, mu=None, stream=None, **opts):
        """mu of eq. 10.4 for the far field v = c1 m1 + c2 m2; returns (mu, stats dict)."""
        import torch
        if mu is None:
            mu = _empty_on(stream, len(self.nodes), torch.device("cuda", self.ctx.device))
        o = _solver_options(**opts)
        st = _SolverStats()
        _check(_lib.lfmm_inclusions_solve(self._h, float(c1), float(c2), ctypes.byref(o),
                                          _dev_tensor(mu, torch.float64, (), "mu"), ctypes.byref(st),
                                          _stream_handle(stream)))
        return mu, {name: getattr(st, name) for name, _ in _SolverStats._fields_}

    def potential(self, c1: float, c2: float, mu, targets, u=None, stream=None):
        """u = v - S(B v + mu) at the targets [m, 2] (device int32)."""
        import torch
        m = int(targets.shape[0])
        if u is None:
            u = _empty_on(stream, m, mu.device)
        _check(_lib.lfmm_inclusions_potential(self._h, float(c1), float(c2), _dev_tensor(mu, torch.float64, (), "mu"),
                                              m, _dev_tensor(targets, torch.int32, (2,), "targets"),
                                              _dev_tensor(u, torch.float64, (), "u"), _stream_handle(stream)))
        return u

    def close(self) -> None:
        if getattr(self, "_h", None):
            if getattr(self.ctx, "_h", None):
                _lib.lfmm_inclusions_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Dirichlet:
    """lfmm_dirichlet: the double-layer-like operator D of a finite lattice (Section 10.2).
    gamma: [n, 2] int32 boundary nodes, normals: [n] codes 0..3 (+x, -x, +y, -y) (host)."""

    def __init__(self, ctx: Context, gamma, normals, stream=None):
        g = np.ascontiguousarray(np.asarray(gamma, dtype=np.int32).reshape(-1, 2))
        c = np.ascontiguousarray(np.asarray(normals, dtype=np.int8).reshape(-1))
        if len(g) != len(c):
            raise ValueError("one normal per boundary node")
        h = ctypes.c_void_p()
        _check(_lib.lfmm_dirichlet_create(ctx._h, len(g), g.ctypes.data_as(_vp), c.ctypes.data_as(_vp),
                                          _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        ctx._plans.add(self)
        self.n = len(g)

    def apply(self, q, out=None, stream=None):
        import torch
        if out is None:
            out = _empty_on(stream, self.n, q.device)
        _check(_lib.lfmm_dirichlet_apply(self._h, _dev_tensor(q, torch.float64, (), "q"),
                                         _dev_tensor(out, torch.float64, (), "out"), _stream_handle(stream)))
        return out

    def solve(self, g, q=None, stream=None, **opts):
        """q with D q = g on the boundary (eq. 10.7); returns (q, stats dict)."""
        import torch
        if q is None:
            q = _empty_on(stream, self.n, g.device)
        o = _solver_options(**opts)
        st = _SolverStats()
        _check(_lib.lfmm_dirichlet_solve(self._h, _dev_tensor(g, torch.float64, (), "g"), ctypes.byref(o),
                                         _dev_tensor(q, torch.float64, (), "q"), ctypes.byref(st),
                                         _stream_handle(stream)))
        return q, {name: getattr(st, name) for name, _ in _SolverStats._fields_}

    def potential(self, q, targets, u=None, stream=None):
        import torch
        m = int(targets.shape[0])
        if u is None:
            u = _empty_on(stream, m, q.device)
        _check(_lib.lfmm_dirichlet_potential(self._h, _dev_tensor(q, torch.float64, (), "q"), m,
                                             _dev_tensor(targets, torch.int32, (2,), "targets"),
                                             _dev_tensor(u, torch.float64, (), "u"), _stream_handle(stream)))
        return u

    def close(self) -> None:
        if getattr(self, "_h", None):
            if getattr(self.ctx, "_h", None):
                _lib.lfmm_dirichlet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
