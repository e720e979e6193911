"""Oracle E: gradients of a flow objective through N steps of the scheme, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The step is written once more with plain PyTorch CPU ops, following the same
definition as Oracle A (section 1.2: M(u~)_kj = P_k(v_j - u~) from the
polynomials, m* = m + s (m^eq - m), f* = M(u~)^{-1} m*, transport; m^eq from
the polynomial f^eq or from the Maxwellian), and reverse-
mode automatic differentiation of that definition gives the discrete adjoint:
d/df_0, d/ds_k and d/du~(x) of J(f_N) for a cotangent dJ/df_N.  u~ is zero, a
given field held fixed over the N steps, or alpha times the local fluid
velocity (then autodiff also differentiates through u = q / rho).  Segments of K steps are
recomputed during the backward pass (torch.utils.checkpoint), so memory stays
bounded for long runs.
"""
import numpy as np
import torch
from torch.utils.checkpoint import checkpoint

from . import scheme as A


def _basis_torch(lat, X, Y, Z, la):
    return torch.stack([P(X, Y, Z, la) for P in lat.basis], dim=-2)   # (..., q_basis, q_vel)


def _maxwellian_meq(lat, rho, u, ut, la, npts=5):
    """rho E[P_k(xi - u~)] for xi ~ N(u, cs2 I), cs2 = la^2 / 3, by tensor
    Gauss-Hermite quadrature (npts points per axis, exact up to degree
    2 npts - 1), in torch so that autodiff follows rho, u and u~.  (N, q)."""
    x, w = np.polynomial.hermite_e.hermegauss(npts)     # weight exp(-x^2 / 2)
    w = w / np.sqrt(2 * np.pi)
    sigma = la / np.sqrt(3.0)
    d = lat.d
    pts = np.stack(np.meshgrid(*([x] * d), indexing="ij"), -1).reshape(-1, d)     # (P, d)
    wts = np.prod(np.stack(np.meshgrid(*([w] * d), indexing="ij"), -1).reshape(-1, d), axis=1)
    pts = torch.tensor(pts, dtype=torch.float64)
    wts = torch.tensor(wts, dtype=torch.float64)
    rel = [u[:, a:a + 1] + sigma * pts[None, :, a] - ut[:, a:a + 1] for a in range(d)]   # (N, P)
    while len(rel) < 3:
        rel.append(torch.zeros_like(rel[0]))
    cols = [(P(rel[0], rel[1], rel[2], la) * wts[None, :]).sum(dim=1) for P in lat.basis]
    return rho[:, None] * torch.stack(cols, dim=1)


def step(lat, f, s, la=1.0, field=None, alpha=None, eq="polynomial"):
    """One step in torch FP64.  f (q, *grid); s (q,); field (d, *grid) or None;
    u~ = field if given, else alpha * u if alpha is given, else 0.  eq: the
    polynomial equilibrium M(u~) f^eq, or "maxwellian": rho E[P_k(xi - u~)]."""
    q, d = lat.q, lat.d
    grid = f.shape[1:]
    F = f.reshape(q, -1).T                                             # (N, q)
    c = torch.tensor(lat.c[:, :d], dtype=torch.float64)
    v = la * c                                                          # (q, d)
    w = torch.tensor(lat.w, dtype=torch.float64)
    rho = F.sum(dim=1)
    u = (F @ v) / rho[:, None]                                          # (N, d)
    cs2 = la * la / 3.0
    vu = u @ v.T                                                        # (N, q)
    uu = (u * u).sum(dim=1, keepdim=True)
    feq = w[None, :] * rho[:, None] * (1 + vu / cs2 + vu * vu / (2 * cs2 * cs2) - uu / (2 * cs2))
    if field is not None:
        ut = field.reshape(d, -1).T                                     # (N, d)
    elif alpha is not None:
        ut = alpha * u
    else:
        ut = torch.zeros_like(u)
    rel = [v[None, :, a] - ut[:, a:a + 1] for a in range(d)]           # components of v_j - u~
    while len(rel) < 3:
        rel.append(torch.zeros_like(rel[0]))
    M = _basis_torch(lat, rel[0], rel[1], rel[2], la)                   # (N, q, q)
    m = (M @ F[:, :, None])[:, :, 0]
    meq = (M @ feq[:, :, None])[:, :, 0] if eq == "polynomial" else _maxwellian_meq(lat, rho, u, ut, la)
    mstar = m + s[None, :] * (meq - m)
    fstar = torch.linalg.solve(M, mstar[:, :, None])[:, :, 0]
    fstar = fstar.T.reshape((q,) + tuple(grid))
    out = []
    for j in range(q):                                                  # f_j(x) = f*_j(x - c_j)
        shifts = [int(lat.c[j, a]) for a in range(d)]
        axes = [len(grid) - 1 - a for a in range(d)]
        out.append(torch.roll(fstar[j], shifts=shifts, dims=axes))
    return torch.stack(out)


def run(lat, f, s, nsteps, la=1.0, field=None, K=100, alpha=None, eq="polynomial"):
    """nsteps steps with recomputation in segments of K steps during backward."""
    def seg(fx, sx, fld, n):
        for _ in range(n):
            fx = step(lat, fx, sx, la, fld, alpha, eq)
        return fx
    done = 0
    while done < nsteps:
        n = min(K, nsteps - done)
        if torch.is_grad_enabled():
            f = checkpoint(seg, f, s, field, n, use_reentrant=False)
        else:
            f = seg(f, s, field, n)
        done += n
    return f


def vjp(lat, f0, s, nsteps, cot_fN, la=1.0, field=None, K=100, alpha=None, eq="polynomial"):
    """Gradients of <cot_fN, f_N> with respect to f0, s and the u~ field.

    Returns (f_N, dJ/df0, dJ/ds, dJ/dfield or None) as NumPy FP64 arrays.
    """
    f0t = torch.tensor(np.asarray(f0, dtype=np.float64), requires_grad=True)
    st = torch.tensor(np.asarray(s, dtype=np.float64), requires_grad=True)
    ft = None if field is None else torch.tensor(np.asarray(field, dtype=np.float64), requires_grad=True)
    fN = run(lat, f0t, st, nsteps, la, ft, K, alpha, eq)
    fN.backward(torch.tensor(np.asarray(cot_fN, dtype=np.float64)))
    return (fN.detach().numpy(), f0t.grad.numpy(), st.grad.numpy(),
            None if ft is None else ft.grad.numpy())


def kinetic_energy(lat, f, la=1.0):
    """J = 1/2 sum_x |q|^2 / rho (the objective of the adjoint workload), and dJ/df."""
    v = lat.velocities(la)[:, : lat.d]
    rho = f.sum(axis=0)
    qm = np.stack([np.tensordot(v[:, a], f, 1) for a in range(lat.d)])
    J = 0.5 * float((sum(qm[a] ** 2 for a in range(lat.d)) / rho).sum())
    uu = sum((qm[a] / rho) ** 2 for a in range(lat.d))
    grad = np.empty_like(f)
    for j in range(lat.q):
        grad[j] = sum(v[j, a] * qm[a] / rho for a in range(lat.d)) - 0.5 * uu
    return J, grad


def objective_after(lat, f0, s, nsteps, la=1.0, field=None, alpha=None, eq="polynomial"):
    """J(f_N) with Oracle A's NumPy step (used for finite differences)."""
    mode = A.FIELD if field is not None else (A.FLUID if alpha is not None else A.ZERO)
    fN = A.run(lat, f0, s, nsteps, la, mode, alpha=1.0 if alpha is None else alpha, field=field, eq=eq)
    return kinetic_energy(lat, fN, la)[0]
