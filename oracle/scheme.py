"""Oracle A: one time step of the scheme with relative velocities, as defined.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows section 1.2 of the paper step by step, in FP64, vectorised over nodes:

1. conserved moments rho = sum_j f_j, q = sum_j v_j f_j, u = q / rho   eq. (rhoq)
2. the relative velocity u~ (zero, alpha * u, or a given field)       section 1.2
3. f^eq independent of u~ (second-order polynomial equilibrium, a
   reading: the paper leaves f^eq open)                               section 1.2
4. M(u~)_kj = P_k(v_j - u~) evaluated from the polynomials            eq. (MatMu)
5. m = M(u~) f, m^eq = M(u~) f^eq                                     eq. (ftomu)
6. m*_k = m_k + s_k (m^eq_k - m_k)                                    eq. (relaxationu)
7. f* = M(u~)^{-1} m*  (LU solve with partial pivoting per node)      section 1.2
8. f_j(x, t + dt) = f*_j(x - v_j dt, t), periodic                     eq. (transport)

Arrays: populations ``f`` have shape (q, *grid) with grid = (Ny, Nx) in 2-D and
(Nz, Ny, Nx) in 3-D (x fastest).  A u~ field has shape (d, *grid).  Lattice
units: dx = 1, dt = dx / la.
"""
import numpy as np

ZERO, FLUID, FIELD = 0, 1, 2


def _flat(lat, a):
    """(k, *grid) -> (N, k)."""
    return a.reshape(a.shape[0], -1).T


def conserved(lat, f, la=1.0):
    """rho and u = q / rho at every node, eq. (rhoq).  u has shape (d, *grid)."""
    v = lat.velocities(la)
    rho = f.sum(axis=0)
    q = np.stack([np.tensordot(v[:, a], f, axes=(0, 0)) for a in range(lat.d)])
    return rho, q / rho


def equilibrium(lat, rho, u, la=1.0):
    """f^eq_j = w_j rho [1 + v.u/cs2 + (v.u)^2/(2 cs2^2) - |u|^2/(2 cs2)], cs2 = la^2/3.

    The paper leaves f^eq open (section 2 allows a general equilibrium); this
    is the usual second-order choice.  u has shape (d, *grid); returns (q, *grid).
    """
    v = lat.velocities(la)
    cs2 = la * la / 3.0
    uu = sum(u[a] * u[a] for a in range(lat.d))
    out = np.empty((lat.q,) + rho.shape)
    for j in range(lat.q):
        vu = sum(v[j, a] * u[a] for a in range(lat.d))
        out[j] = lat.w[j] * rho * (1.0 + vu / cs2 + vu * vu / (2 * cs2 * cs2) - uu / (2 * cs2))
    return out


def moment_matrix(lat, ut, la=1.0):
    """M(u~)_kj = P_k(v_j - u~), eq. (MatMu).

    ut: array (N, d) of relative velocities (one row per node).  Returns (N, q, q).
    """
    v = lat.velocities(la)
    n = ut.shape[0]
    XYZ = []
    for a in range(3):
        if a < lat.d:
            XYZ.append(v[None, :, a] - ut[:, a:a + 1])      # (N, q): component a of v_j - u~
        else:
            XYZ.append(np.zeros((n, lat.q)))
    M = np.empty((n, lat.q, lat.q))
    for k, P in enumerate(lat.basis):
        M[:, k, :] = P(XYZ[0], XYZ[1], XYZ[2], la)
    return M


def relative_velocity(lat, u, mode, alpha=1.0, field=None):
    """u~ per node: 0 (d'Humieres), alpha*u (alpha=1: cascaded), or a given field."""
    if mode == ZERO:
        return np.zeros_like(u)
    if mode == FLUID:
        return alpha * u
    if mode == FIELD:
        return np.asarray(field, dtype=np.float64)
    raise ValueError(mode)


def maxwellian_moments(lat, rho, u, ut, la=1.0, npts=5):
    """m^eq(u~)_k = rho E[P_k(xi - u~)], xi ~ N(u, cs2 I), cs2 = la^2 / 3.

    The continuous Maxwellian moments Geier's cascaded scheme relaxes towards
    (introduction of the paper) instead of M(u~) f^eq; the expectation is taken
    by tensor Gauss-Hermite quadrature (npts points per axis: exact for
    polynomials of degree <= 2 npts - 1).  rho (N,), u and ut (N, d); returns (N, q).
    """
    x, w = np.polynomial.hermite_e.hermegauss(npts)     # weight exp(-x^2 / 2)
    w = w / np.sqrt(2 * np.pi)
    sigma = la / np.sqrt(3.0)
    grids = np.meshgrid(*([x] * lat.d), indexing="ij")
    wts = np.ones_like(grids[0])
    for g in np.meshgrid(*([w] * lat.d), indexing="ij"):
        wts = wts * g
    pts = [g.ravel() for g in grids]                    # quadrature points, each (P,)
    wts = wts.ravel()
    XYZ = []
    for a in range(3):
        if a < lat.d:
            XYZ.append(u[:, a:a + 1] + sigma * pts[a][None, :] - ut[:, a:a + 1])   # (N, P)
        else:
            XYZ.append(np.zeros((u.shape[0], wts.size)))
    out = np.empty((u.shape[0], lat.q))
    for k, P in enumerate(lat.basis):
        out[:, k] = rho * (P(XYZ[0], XYZ[1], XYZ[2], la) * wts[None, :]).sum(axis=1)
    return out


def collide(lat, f, s, la=1.0, mode=ZERO, alpha=1.0, field=None, eq="polynomial"):
    """Relaxation phase of section 1.2 at every node; returns f* (q, *grid).

    eq = "polynomial": m^eq(u~) = M(u~) f^eq (section 1.2);
    eq = "maxwellian": m^eq(u~) = the Maxwellian's moments (Geier's choice)."""
    s = np.asarray(s, dtype=np.float64)
    rho, u = conserved(lat, f, la)
    ut = relative_velocity(lat, u, mode, alpha, field)
    M = moment_matrix(lat, _flat(lat, ut), la)                  # (N, q, q)
    m = np.einsum("nkj,nj->nk", M, _flat(lat, f))               # shifted moments
    if eq == "maxwellian":
        meq = maxwellian_moments(lat, rho.ravel(), _flat(lat, u), _flat(lat, ut), la)
    else:
        feq = equilibrium(lat, rho, u, la)
        meq = np.einsum("nkj,nj->nk", M, _flat(lat, feq))       # shifted equilibrium moments
    mstar = m + s[None, :] * (meq - m)
    fstar = np.linalg.solve(M, mstar[:, :, None])[:, :, 0]      # M(u~)^{-1} m*
    return fstar.T.reshape(f.shape)


def opposite(lat):
    """Index of -c_j for every j."""
    return [next(k for k in range(lat.q) if all(lat.c[k] == -lat.c[j])) for j in range(lat.q)]


def stream(lat, fstar, walls=None, la=1.0):
    """Transport phase, eq. (transport): f_j(x) = f*_j(x - c_j), periodic.

    walls: None, or (mask, uw, rho_w) for half-way bounce-back on domain faces
    (the paper does not discuss boundaries; this is the usual rule).  Bit
    2a + side of mask makes the low (side 0) or high (side 1) face of axis a a
    wall; uw[2a + side] is that wall's velocity (length 3).  A population whose
    source x - c_j lies beyond a wall face comes back from the node itself:
    f_j(x) = f*_opp(j)(x) + 2 w_j rho_w (v_j . u_w) / cs2, taking u_w of the
    first crossed wall face in axis order.
    """
    out = np.empty_like(fstar)
    nd = fstar.ndim - 1
    for j in range(lat.q):
        shifts = [int(lat.c[j, a]) for a in range(lat.d)]
        axes = [nd - 1 - a for a in range(lat.d)]                # x -> last axis
        out[j] = np.roll(fstar[j], shift=shifts, axis=axes)
    if walls is None or not walls[0]:
        return out
    mask, uw, rho_w = walls
    opp = opposite(lat)
    cs2 = la * la / 3.0
    shape = fstar.shape[1:]
    idx = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    coord = list(reversed(idx))                                  # coord[a]: index along axis a
    for j in range(lat.q):
        hit = np.zeros(shape, dtype=bool)
        face = np.full(shape, -1)
        for a in range(lat.d):
            c = int(lat.c[j, a])
            for side, cond in ((0, c > 0), (1, c < 0)):
                if cond and (mask >> (2 * a + side)) & 1:
                    edge = coord[a] == (0 if side == 0 else shape[nd - 1 - a] - 1)
                    face = np.where(edge & (face < 0), 2 * a + side, face)
                    hit |= edge
        if not hit.any():
            continue
        corr = np.zeros(shape)
        for fc in range(2 * lat.d):
            vu = la * sum(int(lat.c[j, a]) * uw[fc][a] for a in range(lat.d))
            corr = np.where(face == fc, 2 * lat.w[j] * rho_w * vu / cs2, corr)
        out[j] = np.where(hit, fstar[opp[j]] + corr, out[j])
    return out


def step(lat, f, s, la=1.0, mode=ZERO, alpha=1.0, field=None, walls=None, eq="polynomial"):
    """One full time step: relaxation then transport."""
    return stream(lat, collide(lat, f, s, la, mode, alpha, field, eq), walls, la)


def run(lat, f, s, nsteps, la=1.0, mode=ZERO, alpha=1.0, field=None, walls=None, eq="polynomial"):
    for _ in range(nsteps):
        f = step(lat, f, s, la, mode, alpha, field, walls, eq)
    return f


def fixed_moments(lat, f, la=1.0):
    """m(0) = M(0) f at every node, shape (q, *grid)."""
    M0 = moment_matrix(lat, np.zeros((1, lat.d)), la)[0]
    return np.tensordot(M0, f, axes=(1, 0))


def shift_matrix(lat, ut, la=1.0):
    """T(u~) = M(u~) M(0)^{-1} (section 1.3), for a single u~ of length d."""
    Mu = moment_matrix(lat, np.asarray(ut, dtype=np.float64)[None, :], la)[0]
    M0 = moment_matrix(lat, np.zeros((1, lat.d)), la)[0]
    return Mu @ np.linalg.inv(M0)
