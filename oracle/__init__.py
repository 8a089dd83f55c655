"""CPU FP64 oracle for the 3-D Laplace FMM (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library is built and run without
it.  The arithmetic lives in ``fmm_oracle.c``; this module only marshals NumPy
arrays into it (see that file's header for the formulas and readings).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None

STATUS = {0: "ok", 1: "invalid argument", 3: "point outside the given cube",
          4: "non-finite input", 5: "coincident distinct points", 8: "out of memory"}


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}: {STATUS.get(code, 'unknown')}")
        self.code = code


def load_library(path):
    """Load an oracle build (the default one, or a variant built by a test)."""
    lib = ctypes.CDLL(path)
    d = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.oracle_direct.argtypes = [i64, d, d, i64, ctypes.c_void_p, d, d, d]
    lib.oracle_fmm.argtypes = [i64, d, d, ctypes.c_int, ctypes.c_int, d, ctypes.c_double,
                               i64, ctypes.c_void_p, d, d, d]
    lib.oracle_leaf_cells.argtypes = [i64, d, ctypes.c_int, d, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_int32), d, d]
    lib.oracle_chain.argtypes = [ctypes.c_int, ctypes.c_int, i64, d, d, d, d, d, i64, d, d,
                                 ctypes.c_void_p]
    lib.oracle_fmm_probe.argtypes = [i64, d, d, ctypes.c_int, ctypes.c_int, d, ctypes.c_double,
                                     i64, ctypes.c_void_p, d, d]
    lib.oracle_fmm_adaptive.argtypes = [i64, d, d, ctypes.c_int, ctypes.c_int, ctypes.c_int, d,
                                        ctypes.c_double, d, d, d, ctypes.POINTER(i64)]
    for f in (lib.oracle_direct, lib.oracle_fmm, lib.oracle_leaf_cells, lib.oracle_chain,
              lib.oracle_fmm_adaptive, lib.oracle_fmm_probe):
        f.restype = ctypes.c_int
    return lib


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        _LIB = load_library(path)
    return _LIB


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _targets(targets):
    if targets is None:
        return None, None
    t = np.ascontiguousarray(targets, dtype=np.int64)
    return t, t.ctypes.data_as(ctypes.c_void_p)


def direct(pos, q, targets=None):
    """Exact O(N^2) sums.  Returns (phi, force, energy); energy is None when
    only a subset of targets is evaluated."""
    pos = _f64(pos, (-1, 3))
    q = _f64(q)
    n = len(q)
    t, tp = _targets(targets)
    nt = n if t is None else len(t)
    phi = np.zeros(nt)
    force = np.zeros((nt, 3))
    e = np.zeros(1)
    st = _lib().oracle_direct(n, _dp(pos), _dp(q), nt, tp, _dp(phi), _dp(force),
                              _dp(e) if t is None else None)
    if st:
        raise OracleError(st)
    return phi, force, (float(e[0]) if t is None else None)


def fmm(pos, q, depth, p, lo=(0.0, 0.0, 0.0), side=1.0, targets=None, lib=None):
    """FP64 FMM of the given depth and order.  side <= 0 derives the cube.
    Returns (phi, force, energy); energy is None for a target subset."""
    pos = _f64(pos, (-1, 3))
    q = _f64(q)
    n = len(q)
    lo = _f64(lo)
    t, tp = _targets(targets)
    nt = n if t is None else len(t)
    phi = np.zeros(nt)
    force = np.zeros((nt, 3))
    e = np.zeros(1)
    st = (lib or _lib()).oracle_fmm(n, _dp(pos), _dp(q), int(depth), int(p), _dp(lo), float(side), nt, tp,
                           _dp(phi), _dp(force), _dp(e) if t is None else None)
    if st:
        raise OracleError(st)
    return phi, force, (float(e[0]) if t is None else None)


def fmm_probe(pos, q, depth, p, idx, y, lo=(0.0, 0.0, 0.0), side=1.0):
    """FMM potential phi'(y_k) felt by particle idx[k] if it sat at y_k (same
    leaf), from every other particle, with the tree and expansions of the
    unmoved system.  Central differences of the FMM energy in x_i are then
    q_i (phi'(x_i + h e) - phi'(x_i - h e)) / 2h (see fmm_oracle.c)."""
    pos = _f64(pos, (-1, 3))
    q = _f64(q)
    lo = _f64(lo)
    t, tp = _targets(idx)
    y = _f64(y, (-1, 3))
    if len(y) != len(t):
        raise ValueError("one displaced position per index")
    out = np.zeros(len(t))
    st = _lib().oracle_fmm_probe(len(q), _dp(pos), _dp(q), int(depth), int(p), _dp(lo),
                                 float(side), len(t), tp, _dp(y), _dp(out))
    if st:
        raise OracleError(st)
    return out


def leaf_cells(pos, depth, lo=(0.0, 0.0, 0.0), side=1.0):
    """Leaf cell (ix, iy, iz) of every particle, plus the resolved cube."""
    pos = _f64(pos, (-1, 3))
    lo = _f64(lo)
    cells = np.zeros((len(pos), 3), dtype=np.int32)
    lo_out = np.zeros(3)
    side_out = np.zeros(1)
    st = _lib().oracle_leaf_cells(len(pos), _dp(pos), int(depth), _dp(lo), float(side),
                                  cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  _dp(lo_out), _dp(side_out))
    if st:
        raise OracleError(st)
    return cells, lo_out, float(side_out[0])


CHAIN_M2P, CHAIN_M2M_M2P, CHAIN_M2L_L2P, CHAIN_M2L_L2L_L2P = 0, 1, 2, 3


def chain(kind, p, src, q, x, c1, c2=(0, 0, 0), c3=(0, 0, 0)):
    """Evaluate sources through one operator chain (see fmm_oracle.c)."""
    src = _f64(src, (-1, 3))
    q = _f64(q)
    x = _f64(x, (-1, 3))
    c1, c2, c3 = _f64(c1), _f64(c2), _f64(c3)
    phi = np.zeros(len(x))
    grad = np.zeros((len(x), 3))
    st = _lib().oracle_chain(int(kind), int(p), len(q), _dp(src), _dp(q), _dp(c1), _dp(c2),
                             _dp(c3), len(x), _dp(x), _dp(phi),
                             grad.ctypes.data_as(ctypes.c_void_p))
    if st:
        raise OracleError(st)
    return phi, grad


ADAPTIVE_STATS = ("boxes", "leaves", "deepest", "u", "v", "w", "x", "p2p_pairs", "m2l_pairs")


def fmm_adaptive(pos, q, leaf_max, max_depth, p, lo=(0.0, 0.0, 0.0), side=1.0, lib=None):
    """FP64 FMM on the adaptive octree (boxes with more than leaf_max
    particles divided, down to level max_depth; U, V, W, X lists).  Returns
    (phi, force, energy, stats) with the tree's integer statistics."""
    pos = _f64(pos, (-1, 3))
    q = _f64(q)
    n = len(q)
    lo = _f64(lo)
    phi = np.zeros(n)
    force = np.zeros((n, 3))
    e = np.zeros(1)
    st_arr = np.zeros(len(ADAPTIVE_STATS), dtype=np.int64)
    st = (lib or _lib()).oracle_fmm_adaptive(
        n, _dp(pos), _dp(q), int(leaf_max), int(max_depth), int(p), _dp(lo), float(side),
        _dp(phi), _dp(force), _dp(e), st_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if st:
        raise OracleError(st)
    return phi, force, float(e[0]), dict(zip(ADAPTIVE_STATS, (int(v) for v in st_arr)))
