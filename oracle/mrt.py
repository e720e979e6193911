"""Oracle C: the d'Humieres MRT step for D2Q9, written on its own.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 1.1 of the paper: m = M f with the constant matrix M(0) of eq. (matort);
m*_k = m_k + s_k (m^eq_k - m_k); f* = M^{-1} m*; transport eq. (transport).
Shares nothing with Oracle A: the matrix is the printed one, the velocity list,
the equilibrium and the transport are written again here.  Used to pin that
Oracle A with u~ = 0 is this scheme.
"""
import numpy as np


def printed_M0(la):
    """eq. (matort), typed from the paper."""
    L = la
    return np.array([
        [1, 1, 1, 1, 1, 1, 1, 1, 1],
        [0, L, 0, -L, 0, L, -L, -L, L],
        [0, 0, L, 0, -L, L, L, -L, -L],
        [-4, -1, -1, -1, -1, 2, 2, 2, 2],
        [0, 1, -1, 1, -1, 0, 0, 0, 0],
        [0, 0, 0, 0, 0, 1, -1, 1, -1],
        [0, -2, 0, 2, 0, 1, -1, -1, 1],
        [0, 0, -2, 0, 2, 1, 1, -1, -1],
        [4, -2, -2, -2, -2, 1, 1, 1, 1],
    ], dtype=np.float64)


_EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
_EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
_W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def mrt_step(f, s, la=1.0):
    """One d'Humieres step on a periodic (Ny, Nx) grid; f has shape (9, Ny, Nx)."""
    M = printed_M0(la)
    Minv = np.linalg.inv(M)
    s = np.asarray(s, dtype=np.float64)
    rho = f.sum(axis=0)
    ux = la * np.tensordot(_EX, f, axes=(0, 0)) / rho
    uy = la * np.tensordot(_EY, f, axes=(0, 0)) / rho
    cs2 = la * la / 3.0
    feq = np.empty_like(f)
    for j in range(9):
        cu = la * (_EX[j] * ux + _EY[j] * uy)
        feq[j] = _W[j] * rho * (1 + cu / cs2 + cu * cu / (2 * cs2 * cs2) - (ux * ux + uy * uy) / (2 * cs2))
    m = np.tensordot(M, f, axes=(1, 0))
    meq = np.tensordot(M, feq, axes=(1, 0))
    mstar = m + s[:, None, None] * (meq - m)
    fstar = np.tensordot(Minv, mstar, axes=(1, 0))
    out = np.empty_like(f)
    for j in range(9):                        # f_j(x) = f*_j(x - c_j)
        out[j] = np.roll(np.roll(fstar[j], _EX[j], axis=1), _EY[j], axis=0)
    return out
