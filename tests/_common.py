"""Shared helpers of the GPU parity tests (test infrastructure).

Inputs for the HIP path are built on the host from the oracle's FP64 state and
rounded to the storage type with NumPy (round-to-nearest-even); the oracle then
starts from exactly the values the GPU holds, widened to FP64.
"""
import numpy as np

from oracle import lattices
from oracle import scheme as A

LAT = {("d2q9", "default"): "d2q9_paper", ("d2q9", "geier"): "d2q9_geier",
       ("d3q19", "default"): "d3q19", ("d3q27", "default"): "d3q27"}
NP_STORE = {"f64": np.float64, "f32": np.float32, "f32dev": np.float32, "f16dev": np.float16}


def oracle_lattice(lattice, basis="default"):
    return lattices.make(LAT[(lattice, basis)])


def to_storage(lat, f64, storage, rho0=1.0):
    """Host encoding of an FP64 state: (stored array, the FP64 values it represents)."""
    if storage in ("f64", "f32"):
        st = f64.astype(NP_STORE[storage])
        return st, st.astype(np.float64)
    w = lat.w.reshape((-1,) + (1,) * (f64.ndim - 1))
    st = (f64 - w * rho0).astype(NP_STORE[storage])
    return st, st.astype(np.float64) + w * rho0


def from_storage(lat, st, storage, rho0=1.0):
    st = np.asarray(st, dtype=np.float64)
    if storage in ("f64", "f32"):
        return st
    w = lat.w.reshape((-1,) + (1,) * (st.ndim - 1))
    return st + w * rho0


def far_state(lat, shape, seed, amp=0.05, umax=0.2):
    """f^eq(rho, u) * (1 + amp U(-1, 1)), away from equilibrium, |u| up to umax."""
    rng = np.random.default_rng(seed)
    rho = 1 + 0.05 * rng.standard_normal(shape)
    u = umax * rng.uniform(-1, 1, (lat.d,) + tuple(shape))
    feq = A.equilibrium(lat, rho, u)
    return feq * (1 + amp * rng.uniform(-1, 1, feq.shape))


def rel(a, b):
    """Normwise relative error ||a - b||_inf / ||b||_inf."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def moment_bounds(lat, fw, lam, growth=8.0):
    """Element-wise bounds for FP32 evaluations of rho, u and m(0) = M(0) f from
    the stored state fw (widened to FP64): a sum of q products in FP32 errs by
    at most about q 2^-24 times the sum of the magnitudes of its terms (the
    deviation storages also add w_j rho0, with rho0 = 1, per term); `growth`
    is the margin.  Returns the bounds for rho [grid], u [d, grid] and
    m(0) [q, grid]."""
    eps = growth * lat.q * 2.0 ** -24
    M0 = np.abs(A.moment_matrix(lat, np.zeros((1, lat.d)), lam)[0])
    mag = np.abs(fw) + lat.w.reshape((-1,) + (1,) * (fw.ndim - 1))
    rho, u = A.conserved(lat, fw, lam)
    t_rho = eps * mag.sum(axis=0)
    v = np.abs(lat.velocities(lam))
    t_u = np.stack([eps * (np.tensordot(v[:, a], mag, axes=(0, 0)) + np.abs(u[a]) * mag.sum(axis=0)) / rho
                    for a in range(lat.d)])
    t_m = eps * np.tensordot(M0, mag, axes=(1, 0))
    return t_rho, t_u, t_m
