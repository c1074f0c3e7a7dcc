"""Python binding of libfmmg.so, the MI355X (gfx950) octree FMM gravity solve.

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  The functions carry the names of the C-ABI in include/fmmg.h;
``Plan`` is a small convenience wrapper around them.  Device buffers are
torch tensors (float64, contiguous, on the plan's device); torch is used for
memory and streams only.

The library must have been built (``python -m paper_1908_03121_amd._build``
or ``__graft_entry__.build()``); there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmmg.so")

FMMG_OK, FMMG_EINVAL, FMMG_ETREE, FMMG_ENOMEM, FMMG_EHIP, FMMG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
FMMG_FP64, FMMG_MIXED, FMMG_MIXED_F32 = 0, 1, 2
FMMG_TOP_FULL, FMMG_TOP_STENCIL_ONLY = 0, 1
FMMG_NOALLOC_MAX_DENSITIES = 65536 * 4096  # fmmg_check_density_noalloc: its static array's reach
_STATUS = {0: "FMMG_OK", -1: "FMMG_EINVAL", -2: "FMMG_ETREE", -3: "FMMG_ENOMEM", -4: "FMMG_EHIP",
           -5: "FMMG_EUNSUPPORTED"}

EXPORTED = ["fmmg_default_options", "fmmg_plan_create", "fmmg_plan_n_leaves", "fmmg_leaf_order",
            "fmmg_solve", "fmmg_density_status", "fmmg_check_density", "fmmg_check_density_noalloc",
            "fmmg_get_timings", "fmmg_get_launch_shape",
            "fmmg_get_stats", "fmmg_plan_destroy", "fmmg_last_error", "fmmg_count_pairs",
            "fmmg_version"]
STAGES = ["p2m", "m2m", "top", "mono", "mp_refined", "mp_leaf", "fused", "down"]


class FmmgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class fmmg_tree_desc(C.Structure):
    _fields_ = [("n_subgrids", C.c_int32), ("level", C.POINTER(C.c_int32)),
                ("coord", C.POINTER(C.c_int32)), ("origin", C.c_double * 3), ("L0", C.c_double)]


class fmmg_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("top_mode", C.c_int), ("G", C.c_double),
                ("angular_correction", C.c_int32), ("use_graph", C.c_int32),
                ("persistent", C.c_int32), ("timing", C.c_int32), ("plane_groups", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("autotune", C.c_int32), ("tuning_cache", C.c_char_p),
                ("overlap", C.c_int32), ("launch_streams", C.c_int32), ("xcd_queues", C.c_int32),
                ("plane_pairs", C.c_int32)]


class fmmg_timings(C.Structure):
    _fields_ = [("ms", C.c_double * 8), ("launches", C.c_int64 * 8), ("solves", C.c_int64)]


class fmmg_launch_shape(C.Structure):
    _fields_ = [("persistent", C.c_int32), ("plane_groups", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("from_cache", C.c_int32), ("tuned_ms", C.c_double), ("overlap", C.c_int32),
                ("split_level", C.c_int32), ("launch_streams", C.c_int32), ("use_graph", C.c_int32),
                ("xcd_queues", C.c_int32), ("plane_pairs", C.c_int32)]

    def as_dict(self):
        return {"persistent": int(self.persistent), "plane_groups": int(self.plane_groups),
                "blocks_per_cu": int(self.blocks_per_cu), "overlap": int(self.overlap),
                "split_level": int(self.split_level), "launch_streams": int(self.launch_streams),
                "from_cache": int(self.from_cache), "use_graph": int(self.use_graph),
                "xcd_queues": int(self.xcd_queues), "plane_pairs": int(self.plane_pairs),
                "tuned_ms": float(self.tuned_ms)}


class fmmg_stats(C.Structure):
    _fields_ = [("pairs", C.c_int64 * 4), ("pairs_top", C.c_int64), ("launches", C.c_int64),
                ("solves", C.c_int64), ("paper_flops", C.c_double), ("n_leaves", C.c_int64),
                ("n_refined", C.c_int64), ("max_level", C.c_int32), ("n_trees", C.c_int32),
                ("sweep_y_targets", C.c_int32), ("sweep_x_targets", C.c_int32)]

    def as_dict(self):
        return {"pairs": list(self.pairs), "pairs_top": int(self.pairs_top),
                "launches": int(self.launches), "solves": int(self.solves),
                "paper_flops": float(self.paper_flops), "n_leaves": int(self.n_leaves),
                "n_refined": int(self.n_refined), "max_level": int(self.max_level),
                "n_trees": int(self.n_trees), "sweep_y_targets": int(self.sweep_y_targets),
                "sweep_x_targets": int(self.sweep_x_targets),
                "total_pairs": int(sum(self.pairs) + self.pairs_top)}


_lib = None


def lib() -> C.CDLL:
    """Load the in-tree libfmmg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_1908_03121_amd._build)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.fmmg_default_options.argtypes = [C.POINTER(fmmg_options)]
        L.fmmg_default_options.restype = None
        L.fmmg_plan_create.argtypes = [C.POINTER(vp), C.POINTER(fmmg_tree_desc), C.c_int32,
                                       C.POINTER(fmmg_options), vp]
        L.fmmg_plan_n_leaves.argtypes = [vp, C.POINTER(C.c_int64)]
        L.fmmg_leaf_order.argtypes = [vp, C.POINTER(C.c_int32)]
        L.fmmg_solve.argtypes = [vp, vp, vp, vp, vp]
        L.fmmg_density_status.argtypes = [vp, C.POINTER(C.c_int64)]
        L.fmmg_check_density.argtypes = [vp, vp, vp]
        L.fmmg_check_density_noalloc.argtypes = [vp, C.c_int64, vp, vp]
        L.fmmg_get_stats.argtypes = [vp, C.POINTER(fmmg_stats)]
        L.fmmg_get_timings.argtypes = [vp, C.POINTER(fmmg_timings)]
        L.fmmg_get_launch_shape.argtypes = [vp, C.POINTER(fmmg_launch_shape)]
        L.fmmg_plan_destroy.argtypes = [vp]
        L.fmmg_plan_destroy.restype = None
        L.fmmg_last_error.argtypes = []
        L.fmmg_last_error.restype = C.c_char_p
        L.fmmg_count_pairs.argtypes = [C.POINTER(fmmg_tree_desc), C.c_int32, C.c_int,
                                       C.POINTER(fmmg_stats)]
        L.fmmg_version.argtypes = []
        L.fmmg_version.restype = C.c_int32
        for name in ("fmmg_plan_create", "fmmg_plan_n_leaves", "fmmg_leaf_order", "fmmg_solve",
                     "fmmg_density_status",
                     "fmmg_check_density", "fmmg_check_density_noalloc", "fmmg_get_stats",
                     "fmmg_count_pairs", "fmmg_get_timings",
                     "fmmg_get_launch_shape"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def fmmg_last_error() -> str:
    return lib().fmmg_last_error().decode()


def _check(rc: int):
    if rc != FMMG_OK:
        raise FmmgError(rc, fmmg_last_error())


def fmmg_version() -> int:
    return int(lib().fmmg_version())


def fmmg_default_options() -> fmmg_options:
    o = fmmg_options()
    lib().fmmg_default_options(C.byref(o))
    return o


def _descs(trees: Sequence):
    """trees: objects with level [n], coord [n,3], origin (3), L0."""
    keep = []
    arr = (fmmg_tree_desc * len(trees))()
    for i, t in enumerate(trees):
        lv = np.ascontiguousarray(t.level, dtype=np.int32)
        cd = np.ascontiguousarray(t.coord, dtype=np.int32).reshape(-1, 3)
        if cd.shape[0] != lv.shape[0]:
            raise ValueError("level and coord lengths differ")
        keep += [lv, cd]
        arr[i].n_subgrids = lv.shape[0]
        arr[i].level = lv.ctypes.data_as(C.POINTER(C.c_int32))
        arr[i].coord = cd.ctypes.data_as(C.POINTER(C.c_int32))
        for a in range(3):
            arr[i].origin[a] = float(t.origin[a])
        arr[i].L0 = float(t.L0)
    return arr, keep


def fmmg_count_pairs(trees: Sequence, top_mode: int = FMMG_TOP_FULL) -> dict:
    """Host-only pair counts of a solve (no device touched)."""
    arr, keep = _descs(trees)
    st = fmmg_stats()
    _check(lib().fmmg_count_pairs(arr, len(trees), int(top_mode), C.byref(st)))
    return st.as_dict()


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dptr(t, n, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return t.data_ptr()


def fmmg_plan_create(trees: Sequence, options: fmmg_options | None = None, stream=None) -> C.c_void_p:
    arr, keep = _descs(trees)
    h = C.c_void_p()
    opt = options if options is not None else fmmg_default_options()
    _check(lib().fmmg_plan_create(C.byref(h), arr, len(trees), C.byref(opt), _stream_ptr(stream)))
    return h


def fmmg_plan_n_leaves(plan) -> int:
    n = C.c_int64()
    _check(lib().fmmg_plan_n_leaves(plan, C.byref(n)))
    return int(n.value)


def fmmg_leaf_order(plan) -> np.ndarray:
    out = np.zeros(fmmg_plan_n_leaves(plan), dtype=np.int32)
    _check(lib().fmmg_leaf_order(plan, out.ctypes.data_as(C.POINTER(C.c_int32))))
    return out


def fmmg_solve(plan, rho, phi, g, stream=None) -> None:
    n = fmmg_plan_n_leaves(plan)
    _check(lib().fmmg_solve(plan, _dptr(rho, n * 512, "rho"), _dptr(phi, n * 512, "phi"),
                            _dptr(g, n * 3 * 512, "g"), _stream_ptr(stream)))


def fmmg_density_status(plan) -> int:
    """-1, or raises FmmgError (FMMG_EINVAL) naming the flat index of a bad
    density that a completed solve read."""
    bad = C.c_int64(-1)
    _check(lib().fmmg_density_status(plan, C.byref(bad)))
    return int(bad.value)


def fmmg_check_density(plan, rho, stream=None) -> None:
    n = fmmg_plan_n_leaves(plan)
    _check(lib().fmmg_check_density(plan, _dptr(rho, n * 512, "rho"), _stream_ptr(stream)))


def fmmg_check_density_noalloc(rho, n, bad_index, stream=None) -> None:
    """rho: contiguous float64 CUDA tensor of at least n elements; bad_index:
    int64 CUDA tensor of one element that receives -1 or the smallest bad flat
    index when the stream reaches the check."""
    import torch
    if not isinstance(rho, torch.Tensor) or rho.dtype != torch.float64 or not rho.is_cuda \
            or not rho.is_contiguous() or rho.numel() < n:
        raise ValueError(f"rho must be a contiguous float64 CUDA tensor of at least {n} elements")
    if not isinstance(bad_index, torch.Tensor) or bad_index.dtype != torch.int64 or not bad_index.is_cuda \
            or bad_index.numel() < 1:
        raise ValueError("bad_index must be an int64 CUDA tensor of one element")
    _check(lib().fmmg_check_density_noalloc(rho.data_ptr() if n > 0 else None, int(n), bad_index.data_ptr(),
                                            _stream_ptr(stream)))


def fmmg_get_stats(plan) -> dict:
    st = fmmg_stats()
    _check(lib().fmmg_get_stats(plan, C.byref(st)))
    return st.as_dict()


def fmmg_get_timings(plan) -> dict:
    """Summed stage durations (ms) of the timed solves since the last call."""
    t = fmmg_timings()
    _check(lib().fmmg_get_timings(plan, C.byref(t)))
    return {"solves": int(t.solves), "ms": dict(zip(STAGES, list(t.ms))),
            "launches": dict(zip(STAGES, list(t.launches)))}


def fmmg_get_launch_shape(plan) -> dict:
    sh = fmmg_launch_shape()
    _check(lib().fmmg_get_launch_shape(plan, C.byref(sh)))
    return sh.as_dict()


def fmmg_plan_destroy(plan) -> None:
    if plan:
        lib().fmmg_plan_destroy(plan)


class Plan:
    """Owns one fmmg plan.  ``solve`` returns (phi [L,512], g [L,3,512])."""

    def __init__(self, trees: Sequence, precision: str = "fp64", top_mode: str = "full",
                 G: float = 1.0, angular_correction: bool = True, use_graph: bool | None = None,
                 persistent: bool = False, timing: bool = False, plane_groups: int = 0,
                 blocks_per_cu: int = 0, autotune: bool = False, tuning_cache: str | None = None,
                 overlap: int = 1, launch_streams: int = 0, xcd_queues: bool = True,
                 plane_pairs: bool | None = None, stream=None):
        opt = fmmg_default_options()
        opt.precision = {"fp64": FMMG_FP64, "mixed": FMMG_MIXED, "mixed_f32": FMMG_MIXED_F32}[precision]
        opt.top_mode = {"full": FMMG_TOP_FULL, "stencil": FMMG_TOP_STENCIL_ONLY}[top_mode]
        opt.G = float(G)
        opt.angular_correction = int(bool(angular_correction))
        # None: the library's default (capture batched plans without timing)
        opt.use_graph = -1 if use_graph is None else int(bool(use_graph))
        opt.persistent = int(bool(persistent))
        opt.timing = int(bool(timing))
        opt.plane_groups = int(plane_groups)
        opt.blocks_per_cu = int(blocks_per_cu)
        opt.autotune = int(bool(autotune))
        self._cache = tuning_cache.encode() if tuning_cache else None
        opt.tuning_cache = self._cache
        opt.overlap = int(overlap)  # 0, 1 (True) or 2
        opt.launch_streams = int(launch_streams)
        opt.xcd_queues = int(bool(xcd_queues))
        # None: the library's choice (paired refined-target items when they fill the GPU)
        opt.plane_pairs = -1 if plane_pairs is None else int(bool(plane_pairs))
        self._h = fmmg_plan_create(trees, opt, stream)
        self.n_leaves = fmmg_plan_n_leaves(self._h)

    def solve(self, rho, phi=None, g=None, stream=None):
        import torch
        if phi is None:
            phi = torch.empty((self.n_leaves, 512), dtype=torch.float64, device=rho.device)
        if g is None:
            g = torch.empty((self.n_leaves, 3, 512), dtype=torch.float64, device=rho.device)
        fmmg_solve(self._h, rho, phi, g, stream)
        return phi, g

    def density_status(self) -> int:
        return fmmg_density_status(self._h)

    def check_density(self, rho, stream=None):
        fmmg_check_density(self._h, rho, stream)

    def stats(self) -> dict:
        return fmmg_get_stats(self._h)

    def timings(self) -> dict:
        return fmmg_get_timings(self._h)

    def launch_shape(self) -> dict:
        return fmmg_get_launch_shape(self._h)

    def leaf_order(self) -> np.ndarray:
        return fmmg_leaf_order(self._h)

    def close(self):
        if getattr(self, "_h", None):
            fmmg_plan_destroy(self._h)
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
