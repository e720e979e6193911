"""Oracle D: the cascaded D2Q9 step in the g-vector form of Appendix B.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Appendix B (proof of Proposition th:cascd2q9):
  * eq. (relgeier):   f* = f + tM(0) g, with M(0) the matrix of eq. (matort);
  * eq. (relgeier2):  m*_g(u) = m_g(u) + C(u) g,  C(u) = M_g(u) tM(0), where
    M_g(u) holds the raw polynomials 1, X, Y, X^2, Y^2, XY, XY^2, X^2Y, X^2Y^2
    shifted by the fluid velocity u = q / rho;
  * the relaxation target is Lambda (m^eq_g - m_g) with Lambda block-diagonal:
    zero on the conserved block, [[s+, s-], [s-, s+]] on (X^2, Y^2) with
    s+- = (s_3 +- s_4)/2, then s_5 .. s_8;
  * g is found by block forward substitution: first the 2x2 system for
    (g_3, g_4), then the remaining components one at a time (eq. (casc2)).
eq. (casc1) is garbled in the paper; this follows its stated conclusion.
Indices here are 0-based.

The rates ``s`` are indexed like the Geier basis of eq. (polgeier): s_3 on
X^2+Y^2, s_4 on X^2-Y^2, s_5 on XY, s_6 on XY^2, s_7 on X^2Y, s_8 on X^2Y^2.
"""
import numpy as np

from .mrt import printed_M0

_EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
_EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
_W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def _raw_moments(X, Y):
    """Rows of M_g: the raw Geier polynomials evaluated at (X, Y) (arrays (N, 9))."""
    return np.stack([np.ones_like(X), X, Y, X * X, Y * Y, X * Y, X * Y * Y, X * X * Y, X * X * Y * Y], axis=1)


def geier_collide(f, s, la=1.0):
    """Cascaded relaxation at every node of f (9, Ny, Nx); returns f*."""
    s = np.asarray(s, dtype=np.float64)
    shape = f.shape
    F = f.reshape(9, -1).T                                 # (N, 9)
    rho = F.sum(axis=1)
    ux = la * (F @ _EX) / rho
    uy = la * (F @ _EY) / rho
    cs2 = la * la / 3.0
    cu = la * (_EX[None, :] * ux[:, None] + _EY[None, :] * uy[:, None])
    feq = _W[None, :] * rho[:, None] * (1 + cu / cs2 + cu * cu / (2 * cs2 * cs2)
                                        - ((ux * ux + uy * uy) / (2 * cs2))[:, None])
    X = la * _EX[None, :] - ux[:, None]                    # (N, 9): v_j - u
    Y = la * _EY[None, :] - uy[:, None]
    Mg = _raw_moments(X, Y)                                # (N, 9 moments, 9 velocities)
    C = Mg @ printed_M0(la).T[None, :, :]                  # C(u) = M_g(u) tM(0)
    mg = np.einsum("nkj,nj->nk", Mg, F)
    mgeq = np.einsum("nkj,nj->nk", Mg, feq)
    sp, sm = (s[3] + s[4]) / 2, (s[3] - s[4]) / 2
    Lam = np.zeros((9, 9))
    Lam[3, 3] = Lam[4, 4] = sp
    Lam[3, 4] = Lam[4, 3] = sm
    for k in range(5, 9):
        Lam[k, k] = s[k]
    rhs = np.einsum("kl,nl->nk", Lam, mgeq - mg)           # (N, 9)
    g = np.zeros_like(rhs)
    # conserved block: C is lower triangular there and rhs = 0, so g_0 = g_1 = g_2 = 0
    for k in range(3):
        g[:, k] = (rhs[:, k] - np.einsum("nl,nl->n", C[:, k, :k], g[:, :k])) / C[:, k, k]
    # the 2x2 block (g_3, g_4)
    r3 = rhs[:, 3] - np.einsum("nl,nl->n", C[:, 3, :3], g[:, :3])
    r4 = rhs[:, 4] - np.einsum("nl,nl->n", C[:, 4, :3], g[:, :3])
    a, b, c, d = C[:, 3, 3], C[:, 3, 4], C[:, 4, 3], C[:, 4, 4]
    det = a * d - b * c
    g[:, 3] = (d * r3 - b * r4) / det
    g[:, 4] = (a * r4 - c * r3) / det
    # successive substitution for the remaining components, eq. (casc2)
    for k in range(5, 9):
        g[:, k] = (rhs[:, k] - np.einsum("nl,nl->n", C[:, k, :k], g[:, :k])) / C[:, k, k]
    Fstar = F + g @ printed_M0(la)                         # f* = f + tM(0) g
    return Fstar.T.reshape(shape)


def geier_step(f, s, la=1.0):
    fstar = geier_collide(f, s, la)
    out = np.empty_like(fstar)
    for j in range(9):
        out[j] = np.roll(np.roll(fstar[j], int(_EX[j]), axis=1), int(_EY[j]), axis=0)
    return out


def upper_structure(u, la=1.0):
    """C(u) for a single u, to check the block lower-triangular structure."""
    X = la * _EX[None, :] - u[0]
    Y = la * _EY[None, :] - u[1]
    return (_raw_moments(X, Y) @ printed_M0(la).T[None])[0]
