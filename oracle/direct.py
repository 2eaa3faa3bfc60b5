"""ORACLE (test infrastructure only) -- Python entry to the direct sum of eq. (1.7).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use
this module.  The sum itself is plain C (``oracle/direct.c``), compiled with gcc on first use
or by ``build_oracle()``; phi is the quadrature table of ``oracle/phi.py`` plus eq. (3.1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .phi import TABLE_RADIUS, load_table, table_file

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_LIB = os.path.join(_HERE, "_direct.so")
_lib = None
_tables = {}


def build_oracle(force: bool = False) -> str:
    """Compile ``direct.c`` into ``_direct.so`` with gcc (no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build_oracle())
        i64, p = ctypes.c_int64, ctypes.c_void_p
        lib.oracle_direct_sum.argtypes = [i64, p, i64, p, p, p, i64, i64, p]
        lib.oracle_direct_sum.restype = None
        lib.oracle_phi.argtypes = [i64, p, p, i64, i64, p]
        lib.oracle_phi.restype = None
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def table(stencil: int = 5) -> np.ndarray:
    """The committed quadrature table of the 5-point (or 9-point) operator."""
    if stencil not in _tables:
        _tables[stencil] = np.ascontiguousarray(load_table(table_file(stencil)), dtype=np.float64)
    return _tables[stencil]


def threads() -> int:
    return int(_load().oracle_threads())


def phi(mxy, stencil: int = 5) -> np.ndarray:
    """phi at integer offsets ``mxy`` [K, 2] (table inside radius 128; beyond it eq. (3.1) for
    the 5-point operator, NaN for the 9-point one, whose oracle has only its table)."""
    m = np.ascontiguousarray(np.asarray(mxy, dtype=np.int32).reshape(-1, 2))
    out = np.empty(len(m), dtype=np.float64)
    tab = table(stencil)
    _load().oracle_phi(len(m), m.ctypes.data, tab.ctypes.data, TABLE_RADIUS, 1 if stencil == 5 else 0,
                       out.ctypes.data)
    return out


def direct_sum(targets, sources, f, stencil: int = 5) -> np.ndarray:
    """u(t) = sum_s phi(t - s) f(s) for each target row (eq. 1.7), Neumaier-summed, FP64.
    For the 9-point operator every offset must lie inside the table (|m|_inf <= 128)."""
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.int32).reshape(-1, 2))
    s = np.ascontiguousarray(np.asarray(sources, dtype=np.int32).reshape(-1, 2))
    q = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1))
    if len(s) != len(q):
        raise ValueError("sources and loads differ in length")
    if stencil != 5 and len(t) and len(s):
        lo = np.minimum(t.min(axis=0), s.min(axis=0)).astype(np.int64)
        hi = np.maximum(t.max(axis=0), s.max(axis=0)).astype(np.int64)
        if np.any(hi - lo > TABLE_RADIUS):
            raise ValueError("offsets beyond the %d-point table radius %d" % (stencil, TABLE_RADIUS))
    u = np.empty(len(t), dtype=np.float64)
    tab = table(stencil)
    _load().oracle_direct_sum(len(t), t.ctypes.data, len(s), s.ctypes.data, q.ctypes.data,
                              tab.ctypes.data, TABLE_RADIUS, 1 if stencil == 5 else 0, u.ctypes.data)
    return u
