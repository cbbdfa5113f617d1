"""Python binding of libbbfmm (ctypes, argument marshalling only).

Every computation happens in the HIP library; this module converts torch
device tensors to pointers and handles to Python objects, and raises
``BBFMMError`` on a non-zero status.  It refuses to run when the shared
library has not been built -- there is no fallback path.

Names follow the C ABI in include/bbfmm.h: ``build_tree``,
``precompute_operators``, ``matvec``, plus export/import helpers and plans.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbbfmm.so")

K_INV_R, K_EXP, K_GAUSS, K_DIPOLE_X, K_POLY_TEST = 0, 1, 2, 3, 100
M2L_FP32, M2L_BF16X3, M2L_FP16_SCALED, M2L_FFT = 0, 1, 2, 3

TA = dict(perm=0, keys=1, pb=2, pe=3, parent=4, cb=5, ce=6, nbr_off=7, nbr_idx=8,
          pair_t=9, pair_tgt=10, pair_src=11, pair_goff=12, leaf_level=13, leaf_cell=14,
          w_off=15, w_level=16, w_cell=17, x_off=18, x_leaf=19)
_TA_DTYPE = dict(keys=np.uint64)
OA = dict(U=0, V=1, C=2, sv_fat=3, sv_thin=4)
STAGES = ("gather", "p2m", "m2m", "m2l", "down", "p2p")

STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "HIP", 4: "BUDGET",
          5: "NOT_FOUND", 6: "INTERNAL", 7: "CANCELLED"}


class BBFMMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class TreeParams(ctypes.Structure):
    _fields_ = [("kernel_id", ctypes.c_int32), ("kernel_param", ctypes.c_double),
                ("cheb_order", ctypes.c_int32), ("leaf_size", ctypes.c_int32),
                ("max_depth", ctypes.c_int32), ("fixed_depth", ctypes.c_int32),
                ("adaptive", ctypes.c_int32)]


class TreeInfo(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("depth", ctypes.c_int32),
                ("cheb_order", ctypes.c_int32), ("kernel_id", ctypes.c_int32),
                ("kernel_param", ctypes.c_double), ("lo", ctypes.c_float * 3),
                ("side", ctypes.c_float), ("scale", ctypes.c_float),
                ("max_leaf_points", ctypes.c_int32), ("cells", ctypes.c_int32 * 22),
                ("pairs", ctypes.c_int64 * 22), ("near_pairs", ctypes.c_int64),
                ("n_targets", ctypes.c_int64), ("n_sources", ctypes.c_int64),
                ("adaptive", ctypes.c_int32), ("n_leaves", ctypes.c_int32),
                ("w_entries", ctypes.c_int64)]


class RequestStats(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("batch_r", ctypes.c_int32),
                ("slot", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("requests_done", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("plans_created", ctypes.c_int64), ("plans_evicted", ctypes.c_int64),
                ("bytes_in_use", ctypes.c_int64), ("bytes_peak", ctypes.c_int64)]


class PlanOptions(ctypes.Structure):
    _fields_ = [("m2l_split", ctypes.c_int32), ("m2l_min_waves", ctypes.c_int32),
                ("p2p_max_split", ctypes.c_int32), ("p2p_mfma", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("p2p_waves", ctypes.c_int32),
                ("m2l_occupancy", ctypes.c_int32), ("m2l_layout", ctypes.c_int32),
                ("m2l_schedule", ctypes.c_int32), ("m2l_block", ctypes.c_int32),
                ("m2l_rtile", ctypes.c_int32), ("m2l_xcd", ctypes.c_int32),
                ("leaf_fused", ctypes.c_int32), ("p2p_pack", ctypes.c_int32),
                ("m2l_mfma", ctypes.c_int32)]


class RuntimeCounters(ctypes.Structure):
    _fields_ = [("device_buffers", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("plans", ctypes.c_int64), ("streams", ctypes.c_int64),
                ("events", ctypes.c_int64), ("plans_freed_in_flight", ctypes.c_int64)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class AllocatorHook(ctypes.Structure):
    """bbfmm_allocator: alloc(bytes, stream, ctx), free(ptr, stream, ctx), ctx."""
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


class TorchAllocator:
    """The library's device memory from torch's caching allocator, so torch
    owns every byte.  Counts its calls; ``fail_after`` makes the allocation
    after that many successful ones return NULL (for testing the library's
    out-of-memory path).  Must outlive the handles built with it (they keep
    a reference)."""

    def __init__(self, fail_after: Optional[int] = None):
        self.fail_after = fail_after
        self.allocs = 0
        self.frees = 0
        self.live = {}

        def _alloc(nbytes, stream, _ctx):
            try:
                import torch
                if self.fail_after is not None and self.allocs >= self.fail_after:
                    return None
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
                self.allocs += 1
                self.live[int(ptr)] = int(nbytes)
                return ptr
            except Exception:
                return None

        def _free(ptr, _stream, _ctx):
            try:
                import torch
                torch.cuda.caching_allocator_delete(int(ptr))
                self.frees += 1
                self.live.pop(int(ptr), None)
            except Exception:
                pass

        self._alloc_cb = _ALLOC_FN(_alloc)
        self._free_cb = _FREE_FN(_free)
        self.hook = AllocatorHook(self._alloc_cb, self._free_cb, None)


_default_torch_alloc = None


def torch_allocator() -> TorchAllocator:
    """The process-wide TorchAllocator used by default."""
    global _default_torch_alloc
    if _default_torch_alloc is None:
        _default_torch_alloc = TorchAllocator()
    return _default_torch_alloc


def _hook_arg(allocator):
    return None if allocator is None else ctypes.byref(allocator.hook)


_lib_handle = None

# name -> (restype, argtypes); every symbol of include/bbfmm.h
_VP, _I32, _I64, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_PVP = ctypes.POINTER(ctypes.c_void_p)
SIGNATURES = {
    "bbfmm_build_tree": (_I32, [_VP, _I64, ctypes.POINTER(TreeParams), _VP, _VP, _PVP]),
    "bbfmm_build_tree_sets": (_I32, [_VP, _I64, _VP, _I64, ctypes.POINTER(TreeParams), _VP, _VP,
                                     _PVP]),
    "bbfmm_tree_info_get": (_I32, [_VP, ctypes.POINTER(TreeInfo)]),
    "bbfmm_tree_export": (_I32, [_VP, _I32, _I32, _VP, _I64, ctypes.POINTER(_I64)]),
    "bbfmm_precompute_operators": (_I32, [_VP, _D, _I32, _VP, _VP, _PVP]),
    "bbfmm_ops_rank": (_I32, [_VP, _I32, ctypes.POINTER(_I32)]),
    "bbfmm_ops_export": (_I32, [_VP, _I32, _I32, _VP, _I64, ctypes.POINTER(_I64)]),
    "bbfmm_ops_import": (_I32, [_VP, _I32, _VP, _VP, _VP, _VP, _VP, _PVP]),
    "bbfmm_matvec": (_I32, [_VP, _VP, _VP, _I64, _VP, _VP]),
    "bbfmm_matvec_static": (_I32, [_VP, _VP, _VP, _I64, _VP, _VP]),
    "bbfmm_plan_create": (_I32, [_VP, _VP, _I64, _PVP]),
    "bbfmm_plan_create_ex": (_I32, [_VP, _VP, _I64, _VP, _VP, _VP, _PVP]),
    "bbfmm_get_runtime_counters": (_I32, [ctypes.POINTER(RuntimeCounters)]),
    "bbfmm_plan_execute": (_I32, [_VP, _VP, _VP, _VP]),
    "bbfmm_plan_workspace_bytes": (_I32, [_VP, ctypes.POINTER(_I64)]),
    "bbfmm_plan_get_options": (_I32, [_VP, ctypes.POINTER(PlanOptions)]),
    "bbfmm_dense_atb": (_I32, [_VP, _VP, _I64, _I32, _VP, _VP, _VP]),
    "bbfmm_dense_ab": (_I32, [_VP, _I64, _I32, _VP, _I32, _VP, _VP]),
    "bbfmm_plan_set_timing": (_I32, [_VP, _I32]),
    "bbfmm_plan_set_graph": (_I32, [_VP, _I32]),
    "bbfmm_plan_stage_times": (_I32, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64), _I32]),
    "bbfmm_server_get_stats": (_I32, [_VP, ctypes.POINTER(ServerStats)]),
    "bbfmm_plan_autotune": (_I32, [_VP, _VP, _I64, _VP, _VP, _VP, _I32, ctypes.POINTER(PlanOptions),
                                   ctypes.POINTER(ctypes.c_double)]),
    "bbfmm_server_create": (_I32, [_I64, _I32, _I32, _PVP]),
    "bbfmm_server_add": (_I32, [_VP, _VP, _VP, ctypes.POINTER(_I32)]),
    "bbfmm_server_submit": (_I32, [_VP, _I32, _VP, _I64, _VP, ctypes.POINTER(ctypes.c_uint64)]),
    "bbfmm_server_wait": (_I32, [_VP, ctypes.c_uint64, _VP]),
    "bbfmm_server_cancel": (_I32, [_VP, ctypes.c_uint64]),
    "bbfmm_server_destroy": (_I32, [_VP]),
    "bbfmm_tree_free": (None, [_VP]),
    "bbfmm_ops_free": (None, [_VP]),
    "bbfmm_plan_free": (None, [_VP]),
    "bbfmm_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load libbbfmm.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib_handle = h
    return _lib_handle


def _check(status: int) -> None:
    if status != 0:
        raise BBFMMError(status, lib().bbfmm_last_error().decode(errors="replace"))


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _device_f32(t, name: str, shape: Optional[Sequence[int]] = None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float32")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def dense_atb(A, B, allocator="torch", stream=None):
    """A^T B (m x m, float64 CUDA tensor) for A, B of shape (n, m), float32
    on the GPU, with FP64 accumulation in a fixed order (bbfmm_dense_atb)."""
    import torch
    _device_f32(A, "A")
    _device_f32(B, "B", tuple(A.shape))
    n, m = A.shape
    C = torch.empty((m, m), dtype=torch.float64, device=A.device)
    hook = torch_allocator() if allocator == "torch" else allocator
    _check(lib().bbfmm_dense_atb(A.data_ptr(), B.data_ptr(), n, m, C.data_ptr(), _hook_arg(hook),
                                 _stream_handle(stream)))
    return C


def dense_ab(A, R, stream=None):
    """A R (n x k, float32 CUDA tensor) for A (n, m) float32 and R (m, k)
    float64, both on the GPU, with FP64 accumulation (bbfmm_dense_ab)."""
    import torch
    _device_f32(A, "A")
    if not isinstance(R, torch.Tensor) or not R.is_cuda or R.dtype != torch.float64 \
            or not R.is_contiguous() or R.dim() != 2 or R.shape[0] != A.shape[1]:
        raise TypeError("R must be a contiguous float64 CUDA tensor with A.shape[1] rows")
    n, m = A.shape
    k = R.shape[1]
    C = torch.empty((n, k), dtype=torch.float32, device=A.device)
    _check(lib().bbfmm_dense_ab(A.data_ptr(), n, m, R.data_ptr(), k, C.data_ptr(),
                                _stream_handle(stream)))
    return C


def runtime_counters() -> dict:
    """Live buffers, bytes, plans, streams and events of the library."""
    out = RuntimeCounters()
    _check(lib().bbfmm_get_runtime_counters(ctypes.byref(out)))
    return {name: getattr(out, name) for name, _ in RuntimeCounters._fields_}


class Tree:
    def __init__(self, handle: int, params: TreeParams, allocator=None):
        self._h = handle
        self.params = params
        self.allocator = allocator      # kept alive while the tree is

    @property
    def handle(self):
        return self._h

    def info(self) -> TreeInfo:
        out = TreeInfo()
        _check(lib().bbfmm_tree_info_get(self._h, ctypes.byref(out)))
        return out

    def export(self, what: str, level: int = 0) -> np.ndarray:
        code = TA[what]
        size = _I64(0)
        _check(lib().bbfmm_tree_export(self._h, code, level, None, 0, ctypes.byref(size)))
        dt = _TA_DTYPE.get(what, np.int32)
        out = np.empty(size.value // np.dtype(dt).itemsize, dtype=dt)
        _check(lib().bbfmm_tree_export(self._h, code, level, out.ctypes.data_as(_VP),
                                       out.nbytes, ctypes.byref(size)))
        return out

    def close(self):
        if self._h:
            lib().bbfmm_tree_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ops:
    def __init__(self, handle: int, tree: Tree, allocator=None):
        self._h = handle
        self.tree = tree
        self.allocator = allocator

    @property
    def handle(self):
        return self._h

    def rank(self, level: int) -> int:
        k = _I32(0)
        _check(lib().bbfmm_ops_rank(self._h, level, ctypes.byref(k)))
        return k.value

    def export(self, what: str, level: int) -> np.ndarray:
        size = _I64(0)
        _check(lib().bbfmm_ops_export(self._h, OA[what], level, None, 0, ctypes.byref(size)))
        out = np.empty(size.value // 8, dtype=np.float64)
        _check(lib().bbfmm_ops_export(self._h, OA[what], level, out.ctypes.data_as(_VP),
                                      out.nbytes, ctypes.byref(size)))
        return out

    def close(self):
        if self._h:
            lib().bbfmm_ops_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Reusable matvec for a fixed (tree, ops, r); owns its workspace."""

    def __init__(self, tree: Tree, ops: Ops, r: int, allocator=None, stream=None, **options):
        """options: m2l_split, m2l_min_waves, p2p_max_split, p2p_mfma, overlap, p2p_waves,
        m2l_occupancy, m2l_layout, m2l_schedule, m2l_block, m2l_rtile, m2l_xcd, leaf_fused,
        p2p_pack, m2l_mfma (0 = heuristic).  allocator: a TorchAllocator
        (None = the operators'); stream: where the set-up is enqueued."""
        h = _VP()
        opt = PlanOptions()
        for k, v in options.items():
            setattr(opt, k, int(v))
        _check(lib().bbfmm_plan_create_ex(tree.handle, ops.handle, int(r), ctypes.byref(opt),
                                          _hook_arg(allocator), _stream_handle(stream),
                                          ctypes.byref(h)))
        self.allocator = allocator
        self.options = dict(options)
        self._h = h.value
        self.tree, self.ops, self.r = tree, ops, int(r)
        info = tree.info()
        self.n_in, self.n_out = info.n_sources, info.n_targets

    def resolved_options(self) -> dict:
        """The launch shapes this plan runs with (heuristic choices explicit)."""
        o = PlanOptions()
        _check(lib().bbfmm_plan_get_options(self._h, ctypes.byref(o)))
        return {name: getattr(o, name) for name, _ in PlanOptions._fields_}

    def workspace_bytes(self) -> int:
        b = _I64(0)
        _check(lib().bbfmm_plan_workspace_bytes(self._h, ctypes.byref(b)))
        return b.value

    def set_graph(self, enable: bool) -> None:
        """Replay the captured launch sequence as one HIP graph."""
        _check(lib().bbfmm_plan_set_graph(self._h, 1 if enable else 0))

    def set_timing(self, enable: bool) -> None:
        _check(lib().bbfmm_plan_set_timing(self._h, 1 if enable else 0))

    def stage_times(self, reset: bool = True):
        """(dict stage -> summed device ms, number of timed executions)."""
        ms = (ctypes.c_double * len(STAGES))()
        n = _I64(0)
        _check(lib().bbfmm_plan_stage_times(self._h, ms, ctypes.byref(n), 1 if reset else 0))
        return dict(zip(STAGES, list(ms))), n.value

    def execute(self, sigma, phi, stream=None):
        _device_f32(sigma, "sigma", (self.n_in, self.r))
        _device_f32(phi, "phi", (self.n_out, self.r))
        _check(lib().bbfmm_plan_execute(self._h, sigma.data_ptr(), phi.data_ptr(),
                                        _stream_handle(stream)))
        return phi

    def close(self):
        if self._h:
            lib().bbfmm_plan_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(tree: Tree, ops: Ops, sigma, phi=None, reps: int = 5, stream=None):
    """Fastest launch-shape options for (tree, ops, r = sigma.shape[1]) on this
    data (bbfmm_plan_autotune); returns (options dict for Plan, median ms)."""
    import torch
    info = tree.info()
    _device_f32(sigma, "sigma", (info.n_sources, sigma.shape[1]))
    if phi is None:
        phi = torch.empty((info.n_targets, sigma.shape[1]), dtype=sigma.dtype, device=sigma.device)
    _device_f32(phi, "phi", (info.n_targets, sigma.shape[1]))
    best = PlanOptions()
    ms = ctypes.c_double(0.0)
    _check(lib().bbfmm_plan_autotune(tree.handle, ops.handle, sigma.shape[1], sigma.data_ptr(),
                                     phi.data_ptr(), _stream_handle(stream), int(reps),
                                     ctypes.byref(best), ctypes.byref(ms)))
    return {"m2l_split": best.m2l_split, "p2p_max_split": best.p2p_max_split,
            "p2p_mfma": best.p2p_mfma, "overlap": best.overlap,
            "p2p_waves": best.p2p_waves, "m2l_occupancy": best.m2l_occupancy,
            "m2l_layout": best.m2l_layout, "m2l_schedule": best.m2l_schedule,
            "m2l_block": best.m2l_block, "m2l_rtile": best.m2l_rtile,
            "m2l_xcd": best.m2l_xcd, "leaf_fused": best.leaf_fused,
            "p2p_pack": best.p2p_pack, "m2l_mfma": best.m2l_mfma}, ms.value


def build_tree(points, kernel_id: int = K_INV_R, kernel_param: float = 1.0,
               cheb_order: int = 4, leaf_size: int = 64, max_depth: int = 22,
               fixed_depth: int = 0, stream=None, allocator="torch", sources=None,
               adaptive: bool = False) -> Tree:
    """Octree over the bounding cube of ``points`` ((N,3) float32 on the GPU).
    sources: a second (M,3) set; then ``points`` are the targets, products
    take sigma of M rows and give phi of N rows (bbfmm_build_tree_sets).
    adaptive: a level-adaptive tree (a cell of at most leaf_size points is a
    leaf on whatever level; one point set only).
    allocator: "torch" (torch's caching allocator owns the library's device
    memory; the default), a TorchAllocator, or None (hipMalloc)."""
    for name, pts in (("points", points), ("sources", sources)):
        if pts is not None and (pts.dim() != 2 or pts.shape[1] != 3):
            raise ValueError(f"{name} must have shape (N, 3)")
    _device_f32(points, "points")
    if allocator == "torch":
        allocator = torch_allocator()
    p = TreeParams(kernel_id, kernel_param, cheb_order, leaf_size, max_depth, fixed_depth,
                   1 if adaptive else 0)
    h = _VP()
    if sources is None:
        _check(lib().bbfmm_build_tree(points.data_ptr(), points.shape[0], ctypes.byref(p),
                                      _hook_arg(allocator), _stream_handle(stream),
                                      ctypes.byref(h)))
    else:
        _device_f32(sources, "sources")
        _check(lib().bbfmm_build_tree_sets(points.data_ptr(), points.shape[0],
                                           sources.data_ptr(), sources.shape[0], ctypes.byref(p),
                                           _hook_arg(allocator), _stream_handle(stream),
                                           ctypes.byref(h)))
    return Tree(h.value, p, allocator)


def precompute_operators(tree: Tree, svd_eps: float = 1e-5, precision: int = M2L_FP32,
                         stream=None, allocator=None) -> Ops:
    """allocator: None = the tree's."""
    h = _VP()
    _check(lib().bbfmm_precompute_operators(tree.handle, float(svd_eps), int(precision),
                                            _hook_arg(allocator), _stream_handle(stream),
                                            ctypes.byref(h)))
    return Ops(h.value, tree, allocator)


def ops_import(tree: Tree, ranks: Sequence[int], U: Sequence[np.ndarray],
               V: Sequence[np.ndarray], C: Sequence[np.ndarray],
               precision: int = M2L_FP32, stream=None) -> Ops:
    """Operators from host FP64 arrays: lists over levels 2..depth-1."""
    depth = tree.info().depth
    rk = np.zeros(max(depth, 1), dtype=np.int32)
    for i, k in enumerate(ranks):
        rk[2 + i] = k
    cat = lambda xs: np.ascontiguousarray(np.concatenate([np.ravel(x) for x in xs])
                                          if len(xs) else np.zeros(1), dtype=np.float64)
    u, v, c = cat(U), cat(V), cat(C)
    h = _VP()
    _check(lib().bbfmm_ops_import(tree.handle, int(precision), rk.ctypes.data_as(_VP),
                                  u.ctypes.data_as(_VP), v.ctypes.data_as(_VP),
                                  c.ctypes.data_as(_VP), _stream_handle(stream),
                                  ctypes.byref(h)))
    return Ops(h.value, tree)


def matvec(tree: Tree, ops: Ops, sigma, phi=None, stream=None):
    """phi = K sigma for sigma of shape (N, r) (or (N,)) float32 on the GPU."""
    import torch
    squeeze = sigma.dim() == 1
    s2 = sigma.reshape(-1, 1) if squeeze else sigma
    info = tree.info()
    _device_f32(s2, "sigma", (info.n_sources, s2.shape[1]))
    if phi is None:
        phi = torch.empty((info.n_targets, s2.shape[1]), dtype=s2.dtype, device=s2.device)
    _device_f32(phi, "phi", (info.n_targets, s2.shape[1]))
    _check(lib().bbfmm_matvec(tree.handle, ops.handle, s2.data_ptr(), s2.shape[1],
                              phi.data_ptr(), _stream_handle(stream)))
    return phi.reshape(-1) if squeeze else phi


class Server:
    """Continuous-batching matvec server (see bbfmm_server_* in bbfmm.h)."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 8, r_max: int = 64):
        h = _VP()
        _check(lib().bbfmm_server_create(int(hbm_budget_bytes), int(max_inflight), int(r_max),
                                         ctypes.byref(h)))
        self._h = h.value
        self._keep = {}          # request id -> (sigma, phi) kept alive until wait
        self._models = []

    def add(self, tree: Tree, ops: Ops) -> int:
        mid = _I32(0)
        _check(lib().bbfmm_server_add(self._h, tree.handle, ops.handle, ctypes.byref(mid)))
        self._models.append((tree, ops))
        return mid.value

    def submit(self, model_id: int, sigma, phi) -> int:
        _device_f32(sigma, "sigma")
        _device_f32(phi, "phi", tuple(sigma.shape))
        rid = ctypes.c_uint64(0)
        _check(lib().bbfmm_server_submit(self._h, int(model_id), sigma.data_ptr(),
                                         sigma.shape[1], phi.data_ptr(), ctypes.byref(rid)))
        self._keep[rid.value] = (sigma, phi)
        return rid.value

    def wait(self, request_id: int) -> dict:
        st = RequestStats()
        try:
            _check(lib().bbfmm_server_wait(self._h, ctypes.c_uint64(request_id), ctypes.byref(st)))
        finally:
            self._keep.pop(request_id, None)
        return {"t_submit": st.t_submit, "t_admit": st.t_admit, "t_done": st.t_done,
                "batch_r": st.batch_r, "slot": st.slot}

    def cancel(self, request_id: int) -> None:
        """Withdraw a request that has not been admitted (its wait then raises
        CANCELLED)."""
        _check(lib().bbfmm_server_cancel(self._h, ctypes.c_uint64(request_id)))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().bbfmm_server_get_stats(self._h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            _check(lib().bbfmm_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
