"""Oracle F: linear (von Neumann) stability of the scheme about a uniform state.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

About a uniform equilibrium (rho0, u0) one step maps a small perturbation
d(x) = F e^{i k.x} to diag(e^{-i k.c_j}) J F e^{i k.x}: J = df*/df is the
Jacobian of the collision of section 1.2 at that state (taken here by
reverse-mode autodiff of Oracle E's FP64 step on a one-node grid, so for
u~ = alpha u it includes the derivative through u~, which vanishes at an
equilibrium), and the phase factors are the transport eq. (transport),
f_j(x, t+1) = f*_j(x - c_j).  The scheme is linearly stable at that state
when the spectral radius of G(k) is at most 1 for every wavenumber; on a
periodic L^d grid the wavenumbers are 2 pi m / L.  The paper names stability
as the open question its schemes raise (conclusion); nothing here is from
the paper beyond the step itself.
"""
import numpy as np
import torch

from . import adjoint as E
from . import scheme as A


def jacobian(lat, s, u0, rho0=1.0, mode="zero", alpha=1.0, la=1.0):
    """J = df*/df (q x q) at f = f^eq(rho0, u0); mode "zero" or "fluid" (u~ = alpha u)."""
    shape = (1,) * lat.d
    u = np.asarray(u0, dtype=np.float64).reshape((lat.d,) + shape)
    feq = A.equilibrium(lat, rho0 * np.ones(shape), u, la)
    f = torch.tensor(feq, dtype=torch.float64)
    st = torch.tensor(np.asarray(s, dtype=np.float64))
    fn = lambda x: E.step(lat, x, st, la, None, alpha if mode == "fluid" else None)
    J = torch.autograd.functional.jacobian(fn, f)
    return J.reshape(lat.q, lat.q).numpy(), feq.reshape(lat.q)


def wavenumbers(d, L, include_zero=False):
    """All 2 pi m / L of a periodic L^d grid, shape (L^d, d) (the zero vector first)."""
    k = np.stack(np.meshgrid(*[2 * np.pi * np.arange(L) / L] * d, indexing="ij"), -1).reshape(-1, d)
    return k if include_zero else k[1:]


def amplification(lat, J, k):
    """G(k) = diag(e^{-i k.c_j}) J for wavenumbers k (n, d): (n, q, q) complex."""
    ph = np.exp(-1j * (k @ lat.c[:, : lat.d].T.astype(np.float64)))
    return ph[:, :, None] * J[None]


def spectral_radius(lat, J, L, include_zero=False):
    """max over the grid's wavenumbers (k = 0 excluded by default) of max |eig G(k)|."""
    ev = np.linalg.eigvals(amplification(lat, J, wavenumbers(lat.d, L, include_zero)))
    return float(np.abs(ev).max())


def critical_speed(lat, s, direction, L, mode="zero", alpha=1.0, threshold=1e-3, umax=0.6, iters=16):
    """Largest |u0| along `direction` (bisection on [0, umax]) whose spectral
    radius over the L^d grid is at most 1 + threshold."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    lo, hi = 0.0, umax
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        J, _ = jacobian(lat, s, mid * d, mode=mode, alpha=alpha)
        if spectral_radius(lat, J, L) > 1 + threshold:
            hi = mid
        else:
            lo = mid
    return lo
