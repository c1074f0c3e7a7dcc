"""ctypes wrapper around the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg.  The product library never loads it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "oracle.c")

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


class Stats(C.Structure):
    _fields_ = [("cls", C.c_int64 * 4), ("top", C.c_int64), ("per_level", C.c_int64 * 16)]

    def as_dict(self):
        return {"cls": list(self.cls), "top": int(self.top), "per_level": list(self.per_level)}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unknown-pragmas", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB_PATH)
        L.oracle_dtensors.argtypes = [_f64p, _f64p, _f64p, _f64p, _f64p, _f64p]
        L.oracle_pair_rule.argtypes = [C.c_int, _i32p, _i32p, C.c_int, C.c_int]
        L.oracle_pair_rule.restype = C.c_int
        L.oracle_m2l_pair.argtypes = [C.c_double, C.c_int, C.c_double, _f64p, C.c_void_p,
                                      C.c_double, _f64p, C.c_void_p, C.c_void_p,
                                      _f64p, _f64p, _f64p, _f64p, _f64p]
        L.oracle_l2l.argtypes = [_f64p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p]
        tree = [C.c_int, _i32p, _i32p, _f64p, C.c_double]
        L.oracle_upward.argtypes = tree + [_f64p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_upward.restype = C.c_int
        L.oracle_solve.argtypes = tree + [_f64p, C.c_double, C.c_int, C.c_int, _f64p, _f64p,
                                          C.POINTER(Stats)]
        L.oracle_solve.restype = C.c_int
        L.oracle_solve_sampled.argtypes = tree + [_f64p, C.c_double, C.c_int, C.c_int, C.c_int,
                                                  _i32p, _i32p, _f64p, _f64p]
        L.oracle_solve_sampled.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_set_threads.restype = C.c_int
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = C.c_int
        L.oracle_direct_sum.argtypes = tree + [_f64p, C.c_double, _f64p, _f64p]
        L.oracle_direct_sum.restype = C.c_int
        L.oracle_direct_sum_sampled.argtypes = tree + [_f64p, C.c_double, C.c_int, _i32p, _i32p,
                                                       _f64p, _f64p]
        L.oracle_direct_sum_sampled.restype = C.c_int
        L.oracle_pair_coverage.argtypes = [C.c_int, _i32p, _i32p, C.c_int, _u8p]
        L.oracle_pair_coverage.restype = C.c_int
        _lib = L
    return _lib


def _tree_args(tree):
    return (tree.n_subgrids, np.ascontiguousarray(tree.level, dtype=np.int32),
            np.ascontiguousarray(tree.coord, dtype=np.int32),
            np.asarray(tree.origin, dtype=np.float64), float(tree.L0))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed with code {rc}")


def dtensors(R):
    R = np.asarray(R, dtype=np.float64)
    D0 = np.zeros(1); D1 = np.zeros(3); D2 = np.zeros(9); D3 = np.zeros(27); D4 = np.zeros(81)
    lib().oracle_dtensors(R, D0, D1, D2, D3, D4)
    return D0[0], D1, D2.reshape(3, 3), D3.reshape(3, 3, 3), D4.reshape(3, 3, 3, 3)


def pair_rule(all_pairs, ca, cb, a_leaf, b_leaf) -> int:
    return lib().oracle_pair_rule(int(all_pairs), np.asarray(ca, dtype=np.int32),
                                  np.asarray(cb, dtype=np.int32), int(a_leaf), int(b_leaf))


def m2l_pair(ma, xa, M3a, mb, xb, M2b, M3b, G=1.0, correction=1):
    """Contribution of one source to one target; returns (L0, L1, L2, L3, dg)."""
    out = [np.zeros(1), np.zeros(3), np.zeros(9), np.zeros(27), np.zeros(3)]
    keep = []

    def ptr(a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64).ravel()
        keep.append(a)
        return a.ctypes.data_as(C.c_void_p)
    lib().oracle_m2l_pair(float(G), int(correction), float(ma), np.asarray(xa, np.float64),
                          ptr(M3a), float(mb), np.asarray(xb, np.float64), ptr(M2b), ptr(M3b),
                          *out)
    return out[0][0], out[1], out[2].reshape(3, 3), out[3].reshape(3, 3, 3), out[4]


def l2l(L0, L1, L2, L3, r):
    o = [np.zeros(1), np.zeros(3), np.zeros(9), np.zeros(27)]
    lib().oracle_l2l(np.asarray([L0], np.float64), np.ascontiguousarray(L1, np.float64).ravel(),
                     np.ascontiguousarray(L2, np.float64).ravel(),
                     np.ascontiguousarray(L3, np.float64).ravel(), np.asarray(r, np.float64), *o)
    return o[0][0], o[1], o[2].reshape(3, 3), o[3].reshape(3, 3, 3)


def upward(tree, rho):
    """Per-cell mass, COM, raw M2 and raw M3 of every sub-grid (descriptor order)."""
    n = tree.n_subgrids
    m = np.zeros(n * 512)
    X = np.zeros(n * 512 * 3)
    M2 = np.zeros(n * 512 * 9)
    M3 = np.zeros(n * 512 * 27)
    vp = lambda a: a.ctypes.data_as(C.c_void_p)
    rc = lib().oracle_upward(*_tree_args(tree), np.ascontiguousarray(rho, np.float64),
                             vp(m), vp(X), vp(M2), vp(M3))
    _check(rc, "oracle_upward")
    return (m.reshape(n, 512), X.reshape(n, 512, 3), M2.reshape(n, 512, 3, 3),
            M3.reshape(n, 512, 3, 3, 3))


def solve(tree, rho, G=1.0, top_all_pairs=True, correction=True, with_stats=False):
    """Full FMM solve of one tree; returns phi [L,512], g [L,3,512] (and stats)."""
    nl = rho.shape[0]
    phi = np.zeros(nl * 512)
    g = np.zeros(nl * 3 * 512)
    st = Stats()
    rc = lib().oracle_solve(*_tree_args(tree), np.ascontiguousarray(rho, np.float64), float(G),
                            int(top_all_pairs), int(correction), phi, g, C.byref(st))
    _check(rc, "oracle_solve")
    out = (phi.reshape(nl, 512), g.reshape(nl, 3, 512))
    return out + (st.as_dict(),) if with_stats else out


def solve_sampled(tree, rho, leaf_idx, cell_idx, G=1.0, top_all_pairs=True, correction=True):
    leaf_idx = np.ascontiguousarray(leaf_idx, dtype=np.int32)
    cell_idx = np.ascontiguousarray(cell_idx, dtype=np.int32)
    ns = leaf_idx.shape[0]
    phi = np.zeros(ns)
    g = np.zeros(ns * 3)
    rc = lib().oracle_solve_sampled(*_tree_args(tree), np.ascontiguousarray(rho, np.float64),
                                    float(G), int(top_all_pairs), int(correction), ns,
                                    leaf_idx, cell_idx, phi, g)
    _check(rc, "oracle_solve_sampled")
    return phi, g.reshape(ns, 3)


def set_threads(n: int) -> int:
    """OpenMP team size of the oracle's loops (n < 1: the runtime default);
    returns the size now in effect."""
    return int(lib().oracle_set_threads(int(n)))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def direct_sum(tree, rho, G=1.0):
    nl = rho.shape[0]
    phi = np.zeros(nl * 512)
    g = np.zeros(nl * 3 * 512)
    rc = lib().oracle_direct_sum(*_tree_args(tree), np.ascontiguousarray(rho, np.float64),
                                 float(G), phi, g)
    _check(rc, "oracle_direct_sum")
    return phi.reshape(nl, 512), g.reshape(nl, 3, 512)


def direct_sum_sampled(tree, rho, leaf_idx, cell_idx, G=1.0):
    """Newton's sum over every leaf cell, at the sampled cells only."""
    leaf_idx = np.ascontiguousarray(leaf_idx, dtype=np.int32)
    cell_idx = np.ascontiguousarray(cell_idx, dtype=np.int32)
    ns = leaf_idx.shape[0]
    phi = np.zeros(ns)
    g = np.zeros(ns * 3)
    rc = lib().oracle_direct_sum_sampled(*_tree_args(tree), np.ascontiguousarray(rho, np.float64),
                                         float(G), ns, leaf_idx, cell_idx, phi, g)
    _check(rc, "oracle_direct_sum_sampled")
    return phi, g.reshape(ns, 3)


def pair_coverage(tree, top_all_pairs=True):
    n_cells = tree.n_leaves * 512
    cover = np.zeros(n_cells * n_cells, dtype=np.uint8)
    rc = lib().oracle_pair_coverage(tree.n_subgrids, np.ascontiguousarray(tree.level, np.int32),
                                    np.ascontiguousarray(tree.coord, np.int32), int(top_all_pairs),
                                    cover)
    _check(rc, "oracle_pair_coverage")
    return cover.reshape(n_cells, n_cells)
