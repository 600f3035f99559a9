"""ctypes binding of the matrix-free FP64 oracle sums in ``direct_sum.c``.

Test infrastructure only (see ``oracle/__init__.py``).  ``build()`` compiles
the C file with gcc into ``oracle/_direct_sum.so``; ``load()`` builds it on
first use when it is missing.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct_sum.c")
_LIB = os.path.join(_HERE, "_direct_sum.so")
_lib = None


def build():
    """Compile direct_sum.c (plain C, OpenMP, no fast-math) into a shared object."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        for name in ("oracle_kv_rows", "oracle_grad_rows"):
            fn = getattr(lib, name)
            fn.restype = None
            fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, P, P, ctypes.c_int64,
                           P, ctypes.c_int64, P, P]
        lib.oracle_kv_rows_real.restype = None
        lib.oracle_kv_rows_real.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, P, P, ctypes.c_int64,
                                            P, ctypes.c_int64, P, P]
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _pts(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a[:, None].copy() if a.ndim == 1 else a


def num_threads():
    return load().oracle_num_threads()


def kv(tgt, src, w, r, eps, rows=None):
    """sum_j w_j exp(-|tgt_i - src_j|^r/eps) for i in ``rows`` (all targets if None)."""
    lib = load()
    tgt = _pts(tgt)
    src = _pts(src)
    w = np.ascontiguousarray(w, dtype=np.float64)
    d = tgt.shape[1]
    if rows is None:
        nrows, rp = tgt.shape[0], None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        nrows, rp = rows.shape[0], rows.ctypes.data
    out = np.empty(nrows)
    if float(r) in (1.0, 2.0):
        lib.oracle_kv_rows(d, int(r), float(eps), tgt.ctypes.data, rp, nrows,
                           src.ctypes.data, src.shape[0], w.ctypes.data, out.ctypes.data)
    else:
        lib.oracle_kv_rows_real(d, float(r), float(eps), tgt.ctypes.data, rp, nrows,
                                src.ctypes.data, src.shape[0], w.ctypes.data, out.ctypes.data)
    return out


def grad_rows(tgt, src, w, r, eps, rows=None):
    """sum_j w_j k_ij grad_x c(tgt_i, src_j) for i in ``rows``; shape (nrows, d)
    (r = 1 or 2 only)."""
    if float(r) not in (1.0, 2.0):
        raise ValueError("grad_rows takes r = 1 or 2")
    lib = load()
    tgt = _pts(tgt)
    src = _pts(src)
    w = np.ascontiguousarray(w, dtype=np.float64)
    d = tgt.shape[1]
    if rows is None:
        nrows, rp = tgt.shape[0], None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        nrows, rp = rows.shape[0], rows.ctypes.data
    out = np.empty((nrows, d))
    lib.oracle_grad_rows(d, int(r), float(eps), tgt.ctypes.data, rp, nrows,
                         src.ctypes.data, src.shape[0], w.ctypes.data, out.ctypes.data)
    return out
