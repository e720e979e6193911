"""Oracle B: Python side of the C/OpenMP oracle (oracle/fast/oracle_fast.c).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Same definition and array
conventions as oracle.scheme (Oracle A); the basis polynomials of
oracle.lattices are expanded into monomial terms here (sympy) and passed in.
"""
import ctypes
import os
import subprocess

import numpy as np
import sympy as sp

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fast", "oracle_fast.c")
LIB = os.path.join(HERE, "liboracle_fast.so")

_lib = None


def build():
    """Compile liboracle_fast.so with gcc (always rebuilds)."""
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = ctypes.CDLL(LIB)
    return _lib


class _Lat(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("q", ctypes.c_int), ("c", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("nterms", ctypes.c_int), ("term_poly", ctypes.c_void_p), ("term_exp", ctypes.c_void_p),
                ("term_coef", ctypes.c_void_p), ("la", ctypes.c_double)]


_TERMS = {}


def _terms(lat, la):
    key = (lat.name, float(la))
    if key not in _TERMS:
        X, Y, Z = sp.symbols("X Y Z")
        polys, exps, coefs = [], [], []
        for k, P in enumerate(lat.basis):
            expr = sp.expand(P(X, Y, Z, sp.nsimplify(la)))
            for (a, b, c), co in sp.Poly(expr, X, Y, Z).terms():
                polys.append(k)
                exps.append((a, b, c))
                coefs.append(float(co))
        _TERMS[key] = (np.array(polys, dtype=np.int32), np.array(exps, dtype=np.int32).reshape(-1, 3),
                       np.array(coefs, dtype=np.float64))
    return _TERMS[key]


def _struct(lat, la, keep):
    tp, te, tc = _terms(lat, la)
    c = np.ascontiguousarray(lat.c.astype(np.int32))
    w = np.ascontiguousarray(lat.w)
    keep.extend([tp, te, tc, c, w])
    return _Lat(lat.d, lat.q, c.ctypes.data, w.ctypes.data, len(tp), tp.ctypes.data, te.ctypes.data,
                tc.ctypes.data, float(la))


def run(lat, f, s, nsteps, la=1.0, mode=0, alpha=1.0, field=None, threads=None):
    """nsteps full steps of f (q, *grid), FP64; returns the new array."""
    lib = _load()
    keep = []
    L = _struct(lat, la, keep)
    f = np.ascontiguousarray(f, dtype=np.float64).copy()
    scratch = np.empty_like(f)
    grid = f.shape[1:]
    dims = np.array(list(reversed(grid)) + [1] * (3 - len(grid)), dtype=np.int64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    fld = None if field is None else np.ascontiguousarray(field, dtype=np.float64)
    threads = threads or os.cpu_count() or 1
    rc = lib.ob_run(ctypes.byref(L), s.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(mode),
                    ctypes.c_double(alpha), None if fld is None else fld.ctypes.data_as(ctypes.c_void_p),
                    dims.ctypes.data_as(ctypes.c_void_p), ctypes.c_int64(nsteps),
                    f.ctypes.data_as(ctypes.c_void_p), scratch.ctypes.data_as(ctypes.c_void_p),
                    ctypes.c_int(threads))
    if rc:
        raise FloatingPointError("singular M(u~) in oracle B")
    return f


def collide(lat, f, s, la=1.0, mode=0, alpha=1.0, field=None, threads=None):
    lib = _load()
    keep = []
    L = _struct(lat, la, keep)
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    N = int(np.prod(f.shape[1:]))
    s = np.ascontiguousarray(s, dtype=np.float64)
    fld = None if field is None else np.ascontiguousarray(field, dtype=np.float64)
    rc = lib.ob_collide(ctypes.byref(L), s.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(mode),
                        ctypes.c_double(alpha), None if fld is None else fld.ctypes.data_as(ctypes.c_void_p),
                        ctypes.c_int64(N), f.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p),
                        ctypes.c_int(threads or os.cpu_count() or 1))
    if rc:
        raise FloatingPointError("singular M(u~) in oracle B")
    return out
