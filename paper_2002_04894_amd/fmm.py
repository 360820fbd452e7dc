"""ctypes binding of libfmm.so (the C ABI in include/fmm.h).

Argument marshalling only: every step of the evaluation runs in the HIP
kernels of libfmm.so.  Device arrays are torch CUDA (HIP) float64 tensors; the
stream is torch's current stream unless one is given.  There is no CPU
fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm.so")

FMM_OK, FMM_EINVAL, FMM_ENOMEM, FMM_EDEVICE, FMM_EUNSUPPORTED = 0, -1, -2, -3, -4
FMM_PART_NEAR, FMM_PART_FAR, FMM_PART_ALL = 1, 2, 3
FMM_PREC_F64, FMM_PREC_MIXED, FMM_PREC_F32 = 0, 1, 2
FMM_MAX_LEVELS, FMM_MAX_ORDER = 8, 20
PHASES = ("tree", "lists", "p2m", "m2m", "m2l", "l2l", "l2p", "p2p")
MAX_LEVELS, MAX_ORDER = 8, 20

_lib = None

# signatures of the allocator hook (fmm_set_allocator)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
_hook_refs = None  # keeps the ctypes callbacks of the current hook alive


class FMMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fmm error {code}: {msg}")
        self.code = code


def lib():
    """Load libfmm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2002_04894_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int, C.c_double
    L.fmm_build.argtypes = [vp, vp, vp, i64, i32, d, vp, C.POINTER(vp)]
    L.fmm_evaluate_tree.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp]
    L.fmm_evaluate_tree_parts.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp, vp]
    L.fmm_evaluate_tree_ex.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, vp, vp]
    L.fmm_evaluate.argtypes = [vp, vp, vp, vp, i64, d, i32, i32, vp, vp, vp, vp, vp]
    L.fmm_build_ex.argtypes = [vp, vp, vp, i64, vp, vp, vp, i64, i32, d, d, vp, C.POINTER(vp)]
    L.fmm_evaluate_targets.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, vp, vp]
    L.fmm_tree_targets.argtypes = [vp, C.POINTER(i64), vp]
    L.fmm_free.argtypes = [vp]
    L.fmm_last_error.argtypes = []
    L.fmm_last_error.restype = C.c_char_p
    L.fmm_tree_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i32), C.POINTER(d)]
    L.fmm_tree_perm.argtypes = [vp, vp]
    L.fmm_tree_boxes.argtypes = [vp, i32, vp, vp]
    L.fmm_tree_lists.argtypes = [vp, i32, i32, C.POINTER(i64), vp, vp]
    L.fmm_tree_stats.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
    L.fmm_set_profiling.argtypes = [i32]
    L.fmm_last_timings.argtypes = [vp]
    L.fmm_bytes_estimate.argtypes = [i64, i32, d, i32]
    L.fmm_bytes_estimate.restype = C.c_size_t
    L.fmm_set_allocator.argtypes = [ALLOC_FN, FREE_FN, vp]
    L.fmm_tree_bytes.argtypes = [vp, i32, i32, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
    L.fmm_evaluate_tree_noalloc.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, vp, vp]
    for f in ("fmm_build", "fmm_build_ex", "fmm_evaluate_targets", "fmm_tree_targets", "fmm_evaluate_tree_ex",
              "fmm_evaluate_tree", "fmm_evaluate_tree_parts", "fmm_evaluate", "fmm_free",
              "fmm_tree_info", "fmm_tree_perm", "fmm_tree_boxes", "fmm_tree_lists", "fmm_tree_stats",
              "fmm_set_profiling", "fmm_last_timings", "fmm_set_allocator", "fmm_tree_bytes",
              "fmm_evaluate_tree_noalloc"):
        getattr(L, f).restype = i32
    _lib = L
    return L


def _check(rc: int):
    if rc != FMM_OK:
        raise FMMError(rc, lib().fmm_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    return int(t)


def _dev(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 tensor on a HIP device")
    return t


def _stream(stream):
    if stream is not None:
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    import torch
    return torch.cuda.current_stream().cuda_stream


class Tree:
    """Owning wrapper of an fmm_tree handle (n sources, m separate targets)."""

    def __init__(self, handle: int, n: int, m: int = 0):
        self.handle = handle
        self.n = n
        self.m = m

    def free(self):
        if self.handle:
            _check(lib().fmm_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _same_length(x, y, z, names=("x", "y", "z")):
    if not (y.numel() == x.numel() and z.numel() == x.numel()):
        raise ValueError(f"{', '.join(names)} must have the same length")


def fmm_build(x, y, z, levels: int, theta: float, stream=None) -> Tree:
    _same_length(x, y, z)
    for t, nm in ((x, "x"), (y, "y"), (z, "z")):
        _dev(t, nm)
    h = C.c_void_p()
    _check(lib().fmm_build(_ptr(x), _ptr(y), _ptr(z), x.numel(), int(levels), float(theta), _stream(stream),
                           C.byref(h)))
    return Tree(h.value, x.numel())


def fmm_build_ex(x, y, z, levels: int, theta: float, eta: float = 1.0, targets=None, stream=None) -> Tree:
    """Tree with split parameter eta and optional separate targets (tx, ty, tz)."""
    _same_length(x, y, z)
    for t, nm in ((x, "x"), (y, "y"), (z, "z")):
        _dev(t, nm)
    if targets is None:
        tp, m = (None, None, None), 0
    else:
        for t, nm in zip(targets, ("tx", "ty", "tz")):
            _dev(t, nm)
        m = targets[0].numel()
        if any(t.numel() != m for t in targets):
            raise ValueError("tx, ty, tz must have the same length")
        tp = tuple(_ptr(t) for t in targets)
    h = C.c_void_p()
    _check(lib().fmm_build_ex(_ptr(x), _ptr(y), _ptr(z), x.numel(), *tp, m, int(levels), float(theta), float(eta),
                              _stream(stream), C.byref(h)))
    return Tree(h.value, x.numel(), m)


def fmm_evaluate_targets(tree: Tree, q, p: int, pot, ex, ey, ez, stream=None, parts: int = FMM_PART_ALL,
                         precision: int = FMM_PREC_F64):
    _dev(q, "q")
    if q.numel() != tree.n:
        raise ValueError(f"q must have {tree.n} elements")
    for t, nm in ((pot, "pot"), (ex, "ex"), (ey, "ey"), (ez, "ez")):
        _dev(t, nm)
        if t.numel() != tree.m:
            raise ValueError(f"{nm} must have {tree.m} elements")
    _check(lib().fmm_evaluate_targets(tree.handle, _ptr(q), int(p), int(parts), int(precision), _ptr(pot), _ptr(ex),
                                      _ptr(ey), _ptr(ez), _stream(stream)))


def fmm_tree_targets(tree: Tree) -> np.ndarray:
    """Leaf of each separate target (caller's order)."""
    m = C.c_int64()
    _check(lib().fmm_tree_targets(tree.handle, C.byref(m), None))
    leaf = np.empty(max(m.value, 1), dtype=np.int32)
    _check(lib().fmm_tree_targets(tree.handle, C.byref(m), leaf.ctypes.data))
    return leaf[: m.value]


def fmm_evaluate_tree(tree: Tree, q, p: int, pot, ex, ey, ez, stream=None, parts: int = FMM_PART_ALL,
                      precision: int = FMM_PREC_F64):
    for t, nm in ((q, "q"), (pot, "pot"), (ex, "ex"), (ey, "ey"), (ez, "ez")):
        _dev(t, nm)
        if t.numel() != tree.n:
            raise ValueError(f"{nm} must have {tree.n} elements")
    if precision != FMM_PREC_F64:
        _check(lib().fmm_evaluate_tree_ex(tree.handle, _ptr(q), int(p), int(parts), int(precision), _ptr(pot),
                                          _ptr(ex), _ptr(ey), _ptr(ez), _stream(stream)))
    elif parts == FMM_PART_ALL:
        _check(lib().fmm_evaluate_tree(tree.handle, _ptr(q), int(p), _ptr(pot), _ptr(ex), _ptr(ey), _ptr(ez),
                                       _stream(stream)))
    else:
        _check(lib().fmm_evaluate_tree_parts(tree.handle, _ptr(q), int(p), int(parts), _ptr(pot), _ptr(ex),
                                             _ptr(ey), _ptr(ez), _stream(stream)))


def fmm_evaluate_tree_noalloc(tree: Tree, q, p: int, pot, ex, ey, ez, stream=None, parts: int = FMM_PART_ALL,
                              precision: int = FMM_PREC_F64):
    """fmm_evaluate_tree with all scratch in the library's fixed device array
    (no allocation; capturable in a graph; calls on one GPU must not overlap)."""
    for t, nm in ((q, "q"), (pot, "pot"), (ex, "ex"), (ey, "ey"), (ez, "ez")):
        _dev(t, nm)
        if t.numel() != tree.n:
            raise ValueError(f"{nm} must have {tree.n} elements")
    _check(lib().fmm_evaluate_tree_noalloc(tree.handle, _ptr(q), int(p), int(parts), int(precision), _ptr(pot),
                                           _ptr(ex), _ptr(ey), _ptr(ez), _stream(stream)))


def fmm_evaluate(x, y, z, q, theta: float, p: int, levels: int, pot, ex, ey, ez, stream=None):
    for t, nm in ((x, "x"), (y, "y"), (z, "z"), (q, "q"), (pot, "pot"), (ex, "ex"), (ey, "ey"), (ez, "ez")):
        _dev(t, nm)
    for t, nm in ((y, "y"), (z, "z"), (q, "q"), (pot, "pot"), (ex, "ex"), (ey, "ey"), (ez, "ez")):
        if t.numel() != x.numel():
            raise ValueError(f"{nm} must have {x.numel()} elements")
    _check(lib().fmm_evaluate(_ptr(x), _ptr(y), _ptr(z), _ptr(q), x.numel(), float(theta), int(p), int(levels),
                              _ptr(pot), _ptr(ex), _ptr(ey), _ptr(ez), _stream(stream)))


def fmm_free(tree: Tree):
    tree.free()


def fmm_last_error() -> str:
    return lib().fmm_last_error().decode()


def fmm_tree_info(tree: Tree):
    n, lv, th = C.c_int64(), C.c_int(), C.c_double()
    _check(lib().fmm_tree_info(tree.handle, C.byref(n), C.byref(lv), C.byref(th)))
    return n.value, lv.value, th.value


def fmm_tree_perm(tree: Tree) -> np.ndarray:
    out = np.empty(tree.n, dtype=np.int32)
    _check(lib().fmm_tree_perm(tree.handle, out.ctypes.data))
    return out


def fmm_tree_boxes(tree: Tree, level: int):
    nb = 8 ** level
    geom = np.empty((nb, 10))
    start = np.empty(nb + 1, dtype=np.int64)
    _check(lib().fmm_tree_boxes(tree.handle, int(level), geom.ctypes.data, start.ctypes.data))
    return geom, start


def fmm_tree_lists(tree: Tree, level: int, kind: int):
    nnz = C.c_int64()
    _check(lib().fmm_tree_lists(tree.handle, int(level), int(kind), C.byref(nnz), None, None))
    off = np.empty(8 ** level + 1, dtype=np.int64)
    idx = np.empty(max(nnz.value, 1), dtype=np.int32)
    _check(lib().fmm_tree_lists(tree.handle, int(level), int(kind), C.byref(nnz), off.ctypes.data, idx.ctypes.data))
    return off, idx[: nnz.value]


def fmm_tree_stats(tree: Tree):
    a, b = C.c_int64(), C.c_int64()
    _check(lib().fmm_tree_stats(tree.handle, C.byref(a), C.byref(b)))
    return a.value, b.value


def fmm_set_profiling(on: bool):
    _check(lib().fmm_set_profiling(1 if on else 0))


def fmm_last_timings() -> dict:
    ms = np.zeros(len(PHASES))
    _check(lib().fmm_last_timings(ms.ctypes.data))
    return dict(zip(PHASES, ms.tolist()))


def fmm_tree_bytes(tree: Tree, p: int, precision: int = FMM_PREC_F64):
    """(device bytes the tree owns, peak scratch bytes of one evaluation)."""
    a, b = C.c_size_t(), C.c_size_t()
    _check(lib().fmm_tree_bytes(tree.handle, int(p), int(precision), C.byref(a), C.byref(b)))
    return a.value, b.value


def fmm_set_allocator(alloc=None, free=None):
    """Routes the library's device allocations through Python callables
    alloc(nbytes, stream) -> int pointer (0 on failure) and free(ptr, stream);
    with no arguments the library's own stream-ordered pool is restored.
    The callables are kept alive until the next call."""
    global _hook_refs
    if (alloc is None) != (free is None):
        raise ValueError("alloc and free must both be given or both omitted")
    if alloc is None:
        _check(lib().fmm_set_allocator(ALLOC_FN(), FREE_FN(), None))
        _hook_refs = None
        return

    def _a(nbytes, stream, user):
        try:
            return int(alloc(int(nbytes), stream or 0) or 0)
        except Exception:
            return 0

    def _f(ptr, stream, user):
        try:
            free(int(ptr), stream or 0)
        except Exception:
            pass

    refs = (ALLOC_FN(_a), FREE_FN(_f))
    _check(lib().fmm_set_allocator(refs[0], refs[1], None))
    _hook_refs = refs


class TorchAllocator:
    """Device memory from PyTorch's caching allocator, with an optional
    budget in bytes: an allocation that would exceed it fails, and the
    library then fails the call with FMM_ENOMEM (its allocations freed).
    A block freed on another stream than the one it was allocated on is
    handed back only after that stream's work is done."""

    def __init__(self, budget: int | None = None):
        import threading
        import torch
        self._torch = torch
        self.budget = budget
        self.in_use = 0
        self.peak = 0
        self.live = {}
        self._mu = threading.Lock()

    def alloc(self, nbytes: int, stream: int) -> int:
        with self._mu:
            if self.budget is not None and self.in_use + nbytes > self.budget:
                return 0
            self.in_use += nbytes
            self.peak = max(self.peak, self.in_use)
        try:
            dev = self._torch.cuda.current_device()
            ptr = int(self._torch.cuda.caching_allocator_alloc(nbytes, dev, stream))
        except Exception:
            with self._mu:
                self.in_use -= nbytes
            return 0
        with self._mu:
            self.live[ptr] = (nbytes, stream)
        return ptr

    def free(self, ptr: int, stream: int) -> None:
        with self._mu:
            nbytes, astream = self.live.pop(ptr)
            self.in_use -= nbytes
        if stream != astream:
            if stream:
                self._torch.cuda.ExternalStream(stream).synchronize()
            else:
                self._torch.cuda.synchronize()
        self._torch.cuda.caching_allocator_delete(ptr)

    def install(self):
        fmm_set_allocator(self.alloc, self.free)
        return self


def fmm_bytes_estimate(n: int, levels: int, theta: float, p: int) -> int:
    return int(lib().fmm_bytes_estimate(int(n), int(levels), float(theta), int(p)))


def evaluate(x, y, z, q, levels: int, theta: float, p: int, stream=None):
    """Convenience: allocate outputs and run the one-shot evaluation."""
    import torch
    pot, ex, ey, ez = (torch.empty_like(x) for _ in range(4))
    fmm_evaluate(x, y, z, q, theta, p, levels, pot, ex, ey, ez, stream)
    return pot, ex, ey, ez
