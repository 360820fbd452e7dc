"""ctypes wrapper of the C oracle (test infrastructure only; see fmm_oracle.c)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

__all__ = ["build", "direct", "Tree", "p2m", "m2m", "m2l", "m2l_rot", "set_m2l_form", "set_threads", "l2l", "l2p", "m2p", "p2l",
           "nterms", "idx"]

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_cp = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build() -> None:
    """Compile liboracle.so (always rebuilds)."""
    subprocess.run(["sh", os.path.join(_HERE, "build.sh")], check=True)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = C.CDLL(_LIB)
    i64, d, i32 = C.c_int64, C.c_double, C.c_int
    lib.orc_direct.argtypes = [i64, _dp, _dp, _dp, _dp, i64, C.c_void_p, _dp, _dp, _dp, _dp]
    lib.orc_direct.restype = None
    lib.orc_create.argtypes = [i64, _dp, _dp, _dp, i32, d]
    lib.orc_create.restype = C.c_void_p
    lib.orc_create_ex.argtypes = [i64, _dp, _dp, _dp, i64, C.c_void_p, C.c_void_p, C.c_void_p, i32, d, d]
    lib.orc_create_ex.restype = C.c_void_p
    lib.orc_locate.argtypes = [C.c_void_p, d, d, d]
    lib.orc_locate.restype = i64
    lib.orc_evaluate_targets.argtypes = [C.c_void_p, _dp, i32, i32, _dp, _dp, _dp, _dp]
    lib.orc_evaluate_targets.restype = i32
    lib.orc_destroy.argtypes = [C.c_void_p]
    lib.orc_get_perm.argtypes = [C.c_void_p, _i32p]
    lib.orc_get_geom.argtypes = [C.c_void_p, i32, _dp]
    lib.orc_get_start.argtypes = [C.c_void_p, i32, _i64p]
    lib.orc_list_nnz.argtypes = [C.c_void_p, i32, i32]
    lib.orc_list_nnz.restype = i64
    lib.orc_get_list.argtypes = [C.c_void_p, i32, i32, _i64p, _i32p]
    lib.orc_evaluate.argtypes = [C.c_void_p, _dp, i32, i32, i64, C.c_void_p, _dp, _dp, _dp, _dp]
    lib.orc_evaluate.restype = i32
    lib.orc_p2m.argtypes = [i32, d, d, d, i64, _dp, _dp, _dp, _dp, _cp]
    lib.orc_m2m.argtypes = [i32, _cp, d, d, d, _cp]
    lib.orc_m2l_add.argtypes = [i32, _cp, d, d, d, _cp]
    lib.orc_m2l_rot_add.argtypes = [i32, _cp, d, d, d, _cp]
    lib.orc_set_m2l_form.argtypes = [i32]
    lib.orc_rot_prepare.argtypes = [i32]
    lib.orc_set_threads.argtypes = [i32]
    lib.orc_set_threads.restype = i32
    lib.orc_create_targeted.argtypes = [i64, _dp, _dp, _dp, i32, d, i64, _i64p]
    lib.orc_create_targeted.restype = C.c_void_p
    lib.orc_set_theta.argtypes = [C.c_void_p, d]
    lib.orc_l2l_add.argtypes = [i32, _cp, d, d, d, _cp]
    lib.orc_l2p_add.argtypes = [i32, _cp, d, d, d, d, d, d] + [C.POINTER(C.c_double)] * 4
    lib.orc_m2p.argtypes = [i32, _cp, d, d, d, d, d, d, C.POINTER(C.c_double)]
    lib.orc_p2l.argtypes = [i32, d, d, d, i64, _dp, _dp, _dp, _dp, _cp]
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def nterms(p: int) -> int:
    return (p + 1) * (p + 1)


def idx(n: int, m: int) -> int:
    """Storage index of coefficient (n, m), -n <= m <= n."""
    return n * n + n + m


def direct(x, y, z, q, targets=None):
    """Direct sum (eq. 2.1) at all points or at the listed target indices.
    Returns (phi, ex, ey, ez) for the targets in the order given."""
    lib = _load()
    x, y, z, q = map(_f64, (x, y, z, q))
    n = x.shape[0]
    if targets is None:
        nt, tp = n, None
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        nt, tp = targets.shape[0], targets.ctypes.data_as(C.c_void_p)
    out = [np.empty(nt) for _ in range(4)]
    lib.orc_direct(n, x, y, z, q, nt, tp, *out)
    return tuple(out)


class Tree:
    """ORB tree + theta-criterion lists + FMM evaluation (all on the CPU)."""

    def __init__(self, x, y, z, levels: int, theta: float, eta: float = 1.0, targets=None, leaves=None):
        """targets: optional (tx, ty, tz) of separate evaluation points; they
        widen the root cell (see orc_create_ex).  eta: split parameter.
        leaves: targeted mode (orc_create_targeted): lists only along the
        chains of these leaves, which are then the only ones that can be
        evaluated (for trees whose full lists exceed host memory)."""
        lib = _load()
        self._x, self._y, self._z = map(_f64, (x, y, z))
        self.n = self._x.shape[0]
        self.levels = int(levels)
        self.theta = float(theta)
        self.eta = float(eta)
        if leaves is not None:
            if targets is not None or eta != 1.0:
                raise ValueError("targeted mode takes neither targets nor eta")
            self._t = None
            self.m = 0
            lv = np.ascontiguousarray(leaves, dtype=np.int64)
            self._h = lib.orc_create_targeted(self.n, self._x, self._y, self._z, self.levels, self.theta,
                                              lv.shape[0], lv)
            return
        if targets is None:
            self._t = None
            self.m = 0
            ptrs = (None, None, None)
        else:
            self._t = tuple(map(_f64, targets))
            self.m = self._t[0].shape[0]
            ptrs = tuple(a.ctypes.data_as(C.c_void_p) for a in self._t)
        self._h = lib.orc_create_ex(self.n, self._x, self._y, self._z, self.m, *ptrs, self.levels, self.theta,
                                    self.eta)

    def set_theta(self, theta: float) -> None:
        """Rebuild the lists for another theta (same tree; a targeted tree
        keeps its leaves)."""
        _load().orc_set_theta(self._h, float(theta))
        self.theta = float(theta)

    def close(self):
        if self._h:
            _load().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def perm(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int32)
        _load().orc_get_perm(self._h, out)
        return out

    def geom(self, level: int) -> np.ndarray:
        """(8^l, 10): lo[3], hi[3], centre[3], radius."""
        out = np.empty((8 ** level, 10))
        _load().orc_get_geom(self._h, level, out)
        return out

    def start(self, level: int) -> np.ndarray:
        out = np.empty(8 ** level + 1, dtype=np.int64)
        _load().orc_get_start(self._h, level, out)
        return out

    def lists(self, level: int, kind: int):
        """kind 0 = strong, 1 = weak; returns (offsets int64[8^l+1], idx int32[nnz])."""
        lib = _load()
        nnz = lib.orc_list_nnz(self._h, level, kind)
        off = np.empty(8 ** level + 1, dtype=np.int64)
        ix = np.empty(max(nnz, 1), dtype=np.int32)
        lib.orc_get_list(self._h, level, kind, off, ix)
        return off, ix[:nnz]

    def evaluate(self, q, p: int, parts: int = 3, leaves=None):
        """phi, ex, ey, ez in input order.  parts: 1 near, 2 far, 3 both.
        With `leaves`, only points of those leaves are filled (others NaN)."""
        lib = _load()
        q = _f64(q)
        out = [np.full(self.n, np.nan) for _ in range(4)]
        if leaves is None:
            nl, lp = 0, None
        else:
            leaves = np.ascontiguousarray(leaves, dtype=np.int64)
            nl, lp = leaves.shape[0], leaves.ctypes.data_as(C.c_void_p)
        rc = lib.orc_evaluate(self._h, q, int(p), int(parts), nl, lp, *out)
        if rc != 0:
            raise ValueError(f"orc_evaluate failed ({rc})")
        return tuple(out)


    def locate(self, x, y, z) -> int:
        """Leaf whose cell holds the point (first child in order at every
        level), -1 outside the root cell."""
        return int(_load().orc_locate(self._h, float(x), float(y), float(z)))

    def evaluate_targets(self, q, p: int, parts: int = 3):
        """phi, ex, ey, ez at the separate targets, in their input order."""
        if self._t is None:
            raise ValueError("this tree has no separate targets")
        out = [np.empty(self.m) for _ in range(4)]
        rc = _load().orc_evaluate_targets(self._h, _f64(q), int(p), int(parts), *out)
        if rc != 0:
            raise ValueError(f"orc_evaluate_targets failed ({rc})")
        return tuple(out)


def p2m(p, centre, x, y, z, q):
    x, y, z, q = map(_f64, (x, y, z, q))
    M = np.zeros(nterms(p), dtype=np.complex128)
    _load().orc_p2m(p, *map(float, centre), x.shape[0], x, y, z, q, M)
    return M


def m2m(p, O, d):
    """d = old centre - new centre."""
    M = np.zeros(nterms(p), dtype=np.complex128)
    _load().orc_m2m(p, np.ascontiguousarray(O, dtype=np.complex128), *map(float, d), M)
    return M


def m2l(p, O, d):
    """d = source centre - target centre."""
    L = np.zeros(nterms(p), dtype=np.complex128)
    _load().orc_m2l_add(p, np.ascontiguousarray(O, dtype=np.complex128), *map(float, d), L)
    return L


def m2l_rot(p, O, d):
    """The rotational form of m2l (Section 2.1.3); d = source - target centre."""
    L = np.zeros(nterms(p), dtype=np.complex128)
    _load().orc_m2l_rot_add(p, np.ascontiguousarray(O, dtype=np.complex128), *map(float, d), L)
    return L


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops (n <= 0: keep); returns the count in use."""
    return int(_load().orc_set_threads(int(n)))


def set_m2l_form(rotational: bool) -> None:
    """M2L form of the whole-method evaluation: rotational (True) or the
    basic translation theorem (False, the default)."""
    _load().orc_set_m2l_form(1 if rotational else 0)


def l2l(p, O, d):
    """d = old centre - new centre."""
    L = np.zeros(nterms(p), dtype=np.complex128)
    _load().orc_l2l_add(p, np.ascontiguousarray(O, dtype=np.complex128), *map(float, d), L)
    return L


def l2p(p, Lc, centre, pt):
    """(phi, ex, ey, ez) of a local expansion at one point."""
    outs = [C.c_double(0.0) for _ in range(4)]
    _load().orc_l2p_add(p, np.ascontiguousarray(Lc, dtype=np.complex128), *map(float, centre), *map(float, pt),
                        *[C.byref(o) for o in outs])
    return tuple(o.value for o in outs)


def m2p(p, M, centre, pt):
    out = C.c_double(0.0)
    _load().orc_m2p(p, np.ascontiguousarray(M, dtype=np.complex128), *map(float, centre), *map(float, pt),
                    C.byref(out))
    return out.value


def p2l(p, centre, x, y, z, q):
    x, y, z, q = map(_f64, (x, y, z, q))
    L = np.zeros(nterms(p), dtype=np.complex128)
    _load().orc_p2l(p, *map(float, centre), x.shape[0], x, y, z, q, L)
    return L
