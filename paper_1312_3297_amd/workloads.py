"""Seeded synthetic inputs: density, velocity and noise fields of the workloads.

This module holds no arithmetic of the scheme itself (no equilibrium, no
moments): it only draws the macroscopic fields that initial states are built
from, so that the library (lbmrv_init_equilibrium) and the CPU oracle can each
build their own initial populations from identical inputs.

All fields are node-centred on a periodic grid, x_i = i (i = 0 .. L-1), with
array shape (ny, nx) in 2-D and (nz, ny, nx) in 3-D (x fastest); velocities are
in lattice units (dx = dt = 1).  Random numbers come from NumPy's PCG64 with the
stated seeds.
"""
import numpy as np


def _coords(shape):
    """Index grids (x, y[, z]) for an array of shape (ny, nx) or (nz, ny, nx)."""
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    return list(reversed(grids))


def noise(q, shape, seed):
    """U(-1, 1) per population and node, shape (q, *shape)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, (q,) + tuple(shape))


def shear_wave(L=64, U=0.01):
    """rho = 1, u_x = U sin(2 pi y / L), u_y = 0 on an L x L grid."""
    x, y = _coords((L, L))
    rho = np.ones((L, L))
    u = np.stack([U * np.sin(2 * np.pi * y / L), np.zeros((L, L))])
    return rho, u


def double_shear_layer(L=2048, U=0.04, kappa=80.0, delta=0.002):
    """Double periodic shear layer: u_x = U tanh(kappa (y/L - 1/4)) for y/L <= 1/2,
    U tanh(kappa (3/4 - y/L)) above; u_y = delta sin(2 pi x / L); rho = 1."""
    x, y = _coords((L, L))
    yl = y / L
    ux = np.where(yl <= 0.5, U * np.tanh(kappa * (yl - 0.25)), U * np.tanh(kappa * (0.75 - yl)))
    uy = delta * np.sin(2 * np.pi * x / L)
    return np.ones((L, L)), np.stack([ux, uy])


def taylor_green(L=256, U0=0.05, shape=None):
    """Taylor-Green vortex with wavenumber 2 pi / L:
    u = U0 sin x cos y cos z, v = -U0 cos x sin y cos z, w = 0,
    rho = 1 + 3 U0^2 / 16 (cos 2x + cos 2y)(cos 2z + 2), x = 2 pi i / L."""
    shape = shape or (L, L, L)
    x, y, z = [2 * np.pi * g / L for g in _coords(shape)]
    u = U0 * np.sin(x) * np.cos(y) * np.cos(z)
    v = -U0 * np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros(shape)
    rho = 1 + 3 * U0 * U0 / 16 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2)
    return rho, np.stack([u, v, w])


def random_phase(L=512, amp=0.02, kmin=1, kmax=8, seed=1315):
    """Divergence-free random-phase field from the stream function
    psi = sum_{kmin <= |k| <= kmax} cos(2 pi k.x / L + phi_k), u = (d_y psi, -d_x psi),
    rescaled so that max |u| = amp; rho = 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y = _coords((L, L))
    ux = np.zeros((L, L))
    uy = np.zeros((L, L))
    for kx in range(-kmax, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            k2 = kx * kx + ky * ky
            if k2 < kmin * kmin or k2 > kmax * kmax:
                continue
            phi = rng.uniform(0, 2 * np.pi)
            arg = 2 * np.pi * (kx * x + ky * y) / L + phi
            s = -np.sin(arg) * 2 * np.pi / L
            ux += s * ky          # d psi / dy
            uy -= s * kx          # -d psi / dx
    scale = amp / np.sqrt(ux * ux + uy * uy).max()
    return np.ones((L, L)), np.stack([ux * scale, uy * scale])


# Named rate vectors of the workloads.
RATES_D2Q9_GROUPED = [0, 0, 0, 1.4, 1.7, 1.7, 1.2, 1.2, 1.4]
RATES_D2Q9_LITERAL = [0, 0, 0, 1.4, 1.4, 1.2, 1.2, 1.7, 1.7]
RATES_D2Q9_SHEAR_LAYER = [0, 0, 0, 1.2, 1.9, 1.9, 1.5, 1.5, 1.8]
# 3-D: bulk 1.1, the five shear moments 1.95, third order 1.5, fourth order and
# above 1.2 (a rate of 1.8 on the fourth-order monomials makes the Taylor-Green
# runs blow up within ~60 steps, in the oracle as well as on the GPU)
RATES_D3Q19 = [0.0] * 4 + [1.1] + [1.95] * 5 + [1.5] * 6 + [1.2] * 3
RATES_D3Q27 = [0.0] * 4 + [1.1] + [1.95] * 5 + [1.5] * 7 + [1.2] * 10


# ---------------------------------------------------------------------------
# run-time moment bases (q polynomials in xi = X / lambda, as (coef, exponents)
# terms) and rates for them
# ---------------------------------------------------------------------------
def _t(c, a=0, b=0, e=0):
    return (c, (a, b, e))


def _herm(a, b, e):
    """Tensor Hermite-like polynomial H_a(xi_x) H_b(xi_y) H_c(xi_z) with
    H_0 = 1, H_1 = xi, H_2 = xi^2 - 1/3, expanded into monomial terms."""
    per_axis = {0: [(1.0, 0)], 1: [(1.0, 1)], 2: [(1.0, 2), (-1.0 / 3.0, 0)]}
    out = []
    for ca, pa in per_axis[a]:
        for cb, pb in per_axis[b]:
            for ce, pe in per_axis[e]:
                out.append(_t(ca * cb * ce, pa, pb, pe))
    return out


# D2Q9, Geier's span: Hermite-like family (constants mixed into the second- and
# fourth-order elements, and xi^2 terms into the fourth-order one)
HERMITE_D2Q9 = [_herm(0, 0, 0), _herm(1, 0, 0), _herm(0, 1, 0),
                [_t(1, 2), _t(1, 0, 2), _t(-2.0 / 3.0)], [_t(1, 2), _t(-1, 0, 2)], _herm(1, 1, 0),
                _herm(1, 2, 0), _herm(2, 1, 0), _herm(2, 2, 0)]
RATES_HERMITE_D2Q9 = [0, 0, 0, 1.1, 1.6, 1.75, 1.3, 1.45, 1.9]

# D2Q9, the span of eq. (mom): raw powers of |xi|^2 instead of the orthogonal family
RAW_D2Q9 = [[_t(1)], [_t(1, 1)], [_t(1, 0, 1)], [_t(1, 2), _t(1, 0, 2)], [_t(1, 2), _t(-1, 0, 2)], [_t(1, 1, 1)],
            [_t(1, 3), _t(1, 1, 2)], [_t(1, 2, 1), _t(1, 0, 3)], [_t(1, 4), _t(2, 2, 2), _t(1, 0, 4)]]
RATES_RAW_D2Q9 = [0, 0, 0, 1.2, 1.7, 1.65, 1.3, 1.35, 1.5]

# D3Q19: raw second moments xi_a xi_b with different rates per normal stress
# (an anisotropic relaxation the built-in basis cannot express), the rest as
# the built-in list
RAW2_D3Q19 = ([[_t(1)], [_t(1, 1)], [_t(1, 0, 1)], [_t(1, 0, 0, 1)],
               [_t(1, 2)], [_t(1, 0, 2)], [_t(1, 0, 0, 2)], [_t(1, 1, 1)], [_t(1, 0, 1, 1)], [_t(1, 1, 0, 1)]]
              + [[_t(1, *e)] for e in [(1, 2, 0), (1, 0, 2), (2, 1, 0), (0, 1, 2), (2, 0, 1), (0, 2, 1),
                                       (2, 2, 0), (2, 0, 2), (0, 2, 2)]])
RATES_RAW2_D3Q19 = [0.0] * 4 + [1.1, 1.2, 1.3] + [1.95] * 3 + [1.5] * 6 + [1.2] * 3

# D3Q27: the tensor Hermite-like family over exponents 0..2 per axis, in the
# built-in monomial order
_EXP27 = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 1, 0), (0, 1, 1),
          (1, 0, 1), (1, 2, 0), (1, 0, 2), (2, 1, 0), (0, 1, 2), (2, 0, 1), (0, 2, 1), (1, 1, 1), (2, 2, 0),
          (2, 0, 2), (0, 2, 2), (2, 1, 1), (1, 2, 1), (1, 1, 2), (2, 2, 1), (2, 1, 2), (1, 2, 2), (2, 2, 2)]
HERMITE_D3Q27 = [_herm(*e) for e in _EXP27]
RATES_HERMITE_D3Q27 = [0.0] * 4 + [1.1, 1.15, 1.2] + [1.95] * 3 + [1.5] * 7 + [1.3] * 3 + [1.2] * 7
