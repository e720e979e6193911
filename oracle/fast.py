"""Oracle B: Python side of the C/OpenMP oracles.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Same definition and array
conventions as oracle.scheme (Oracle A); the basis polynomials of
oracle.lattices are expanded into monomial terms here (sympy) and passed in.

run / collide       oracle/fast/oracle_fast.c: per-node Gaussian elimination
                    with partial pivoting (also the CPU baseline)
run_tri / collide_tri
                    oracle/fast/oracle_tri.c: the same definition, solving
                    M(u~) x = m* through M(u~) = T(u~) M(0) (eq. (matTu)) by
                    forward substitution; batched over nodes, for long runs on
                    large grids
"""
import ctypes
import os
import subprocess

import numpy as np
import sympy as sp

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fast", "oracle_fast.c")
LIB = os.path.join(HERE, "liboracle_fast.so")
SRC_TRI = os.path.join(HERE, "fast", "oracle_tri.c")
LIB_TRI = os.path.join(HERE, "liboracle_tri.so")

_lib = None
_lib_tri = None


def build():
    """Compile liboracle_fast.so and liboracle_tri.so with gcc (always rebuilds).

    The triangular form is built for AVX2/FMA vector units with every product
    and sum rounded separately (no contraction into fused multiply-adds)."""
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    tmp = LIB_TRI + ".tmp"
    subprocess.run(["gcc", "-O3", "-mavx2", "-mfma", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
                    SRC_TRI, "-lm"], check=True)
    os.replace(tmp, LIB_TRI)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = ctypes.CDLL(LIB)
    return _lib


def _load_tri():
    global _lib_tri
    if _lib_tri is None:
        if not os.path.exists(LIB_TRI):
            build()
        _lib_tri = ctypes.CDLL(LIB_TRI)
    return _lib_tri


class _Lat(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("q", ctypes.c_int), ("c", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("nterms", ctypes.c_int), ("term_poly", ctypes.c_void_p), ("term_exp", ctypes.c_void_p),
                ("term_coef", ctypes.c_void_p), ("la", ctypes.c_double)]


_TERMS = {}


def _terms(lat, la):
    """Monomial terms (basis index, exponents, coefficient) of the basis, X units."""
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


_M0INV = {}


def _m0_inverse(lat, la):
    """M(0)^{-1} in FP64, rounded once from the exact rational inverse of
    M(0)_kj = P_k(v_j) (sympy), after checking that T(u~) = M(u~) M(0)^{-1}
    is unit lower triangular (eq. (matTu)) at a spread of relative velocities,
    which the triangular solve assumes."""
    key = (lat.name, float(la))
    if key not in _M0INV:
        lam = sp.nsimplify(la)
        M0 = sp.Matrix(lat.q, lat.q, lambda k, j: sp.nsimplify(lat.basis[k](
            *[lam * int(lat.c[j, a]) for a in range(3)], lam)))
        inv = np.array(M0.inv().tolist(), dtype=np.float64)
        from . import scheme
        rng = np.random.default_rng(11)
        for _ in range(16):
            ut = la * rng.uniform(-0.5, 0.5, (1, lat.d))
            T = scheme.moment_matrix(lat, ut, la)[0] @ inv
            if np.abs(np.triu(T, 1)).max() > 1e-12 or np.abs(np.diag(T) - 1).max() > 1e-12:
                raise ValueError("T(u~) is not unit lower triangular for basis %s" % lat.name)
        if max(int(e) for e in _terms(lat, la)[1].ravel()) > 8:
            raise ValueError("basis exponent above 8")
        _M0INV[key] = inv
    return _M0INV[key]


def run_tri(lat, f, s, nsteps, la=1.0, mode=0, alpha=1.0, field=None, threads=None, out=None):
    """nsteps full steps of f (q, *grid), FP64, triangular-solve form; returns
    the new array (written into `out`, shape of f, if given)."""
    lib = _load_tri()
    keep = []
    L = _struct(lat, la, keep)
    inv = np.ascontiguousarray(_m0_inverse(lat, la))
    if out is None:
        out = np.array(f, dtype=np.float64, order="C", copy=True)
    else:
        np.copyto(out, f)
    scratch = np.empty_like(out)
    grid = out.shape[1:]
    dims = np.array(list(reversed(grid)) + [1] * (3 - len(grid)), dtype=np.int64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    fld = None if field is None else np.ascontiguousarray(field, dtype=np.float64)
    threads = threads or os.cpu_count() or 1
    lib.ot_run(ctypes.byref(L), inv.ctypes.data_as(ctypes.c_void_p), s.ctypes.data_as(ctypes.c_void_p),
               ctypes.c_int(mode), ctypes.c_double(alpha),
               None if fld is None else fld.ctypes.data_as(ctypes.c_void_p),
               dims.ctypes.data_as(ctypes.c_void_p), ctypes.c_int64(nsteps),
               out.ctypes.data_as(ctypes.c_void_p), scratch.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(threads))
    return out


def collide_tri(lat, f, s, la=1.0, mode=0, alpha=1.0, field=None, threads=None):
    """The relaxation alone (triangular-solve form)."""
    lib = _load_tri()
    keep = []
    L = _struct(lat, la, keep)
    inv = np.ascontiguousarray(_m0_inverse(lat, la))
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    N = int(np.prod(f.shape[1:]))
    s = np.ascontiguousarray(s, dtype=np.float64)
    fld = None if field is None else np.ascontiguousarray(field, dtype=np.float64)
    lib.ot_collide(ctypes.byref(L), inv.ctypes.data_as(ctypes.c_void_p), s.ctypes.data_as(ctypes.c_void_p),
                   ctypes.c_int(mode), ctypes.c_double(alpha),
                   None if fld is None else fld.ctypes.data_as(ctypes.c_void_p), ctypes.c_int64(N),
                   f.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p),
                   ctypes.c_int(threads or os.cpu_count() or 1))
    return out
