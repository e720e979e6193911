"""Oracle F (linear stability about a uniform state) pinned to facts that do
not depend on it:
  * at k = 0 the step is the collision alone, whose eigenvalues are 1 on the
    conserved moments and 1 - s_k on the others (the relaxation is diagonal in
    the moving frame and the shift is a similarity), for u~ = 0 and u~ = u;
  * without relaxation (s = 0) the step is a pure transport: |eig G(k)| = 1;
  * with one rate on every non-conserved moment (BGK) the Jacobian does not
    depend on u~ or on the basis; at u0 = 0 the modes u~ = 0 and u~ = u agree;
  * the autodiff Jacobian equals central differences of Oracle A's collision;
  * brute force: power iteration of the full nonlinear step (Oracle B) from a
    small zero-mean perturbation on the same periodic grid grows at the
    predicted spectral radius.
"""
import numpy as np
import pytest

from oracle import fast, lattices
from oracle import scheme as A
from oracle import stability as F

S9 = [0, 0, 0, 1.4, 1.95, 1.95, 1.2, 1.2, 1.4]


@pytest.mark.parametrize("name", ["d2q9", "d2q9_geier", "d3q19"])
@pytest.mark.parametrize("mode,u0", [("zero", 0.12), ("fluid", 0.12)])
def test_k0_eigenvalues_are_one_and_one_minus_s(name, mode, u0):
    lat = lattices.make(name)
    s = S9 if lat.q == 9 else [0.0] * 4 + [1.1] + [1.9] * 5 + [1.5] * 6 + [1.3] * 3
    u = np.zeros(lat.d)
    u[0], u[1] = u0, -0.5 * u0
    J, _ = F.jacobian(lat, s, u, mode=mode)
    ev = np.sort(np.linalg.eigvals(J).real)
    ref = np.sort(1.0 - np.asarray(s, dtype=np.float64))
    assert np.abs(ev - ref).max() <= 1e-10
    assert np.abs(np.linalg.eigvals(J).imag).max() <= 1e-10


def test_pure_transport_has_unit_spectrum():
    lat = lattices.make("d2q9")
    J, _ = F.jacobian(lat, [0.0] * 9, (0.2, 0.1), mode="fluid")
    assert np.abs(J - np.eye(9)).max() <= 1e-14
    ev = np.linalg.eigvals(F.amplification(lat, J, F.wavenumbers(2, 8)))
    assert np.abs(np.abs(ev) - 1).max() <= 1e-14


def test_bgk_jacobian_is_independent_of_the_relative_velocity_and_basis():
    s = [0, 0, 0] + [1.7] * 6
    u = (0.15, 0.05)
    Js = [F.jacobian(lattices.make(n), s, u, mode=m)[0] for n in ("d2q9", "d2q9_geier") for m in ("zero", "fluid")]
    for J in Js[1:]:
        assert np.abs(J - Js[0]).max() <= 1e-13


def test_modes_agree_at_rest():
    lat = lattices.make("d2q9_geier")
    a, _ = F.jacobian(lat, S9, (0.0, 0.0), mode="zero")
    b, _ = F.jacobian(lat, S9, (0.0, 0.0), mode="fluid")
    assert np.abs(a - b).max() <= 1e-15


@pytest.mark.parametrize("mode", ["zero", "fluid"])
def test_jacobian_matches_finite_differences_of_the_collision(mode):
    lat = lattices.make("d2q9")
    u0 = (0.1, -0.07)
    J, feq = F.jacobian(lat, S9, u0, mode=mode)
    h = 1e-6
    fd = np.empty((9, 9))
    m = {"zero": A.ZERO, "fluid": A.FLUID}[mode]
    for j in range(9):
        e = np.zeros((9, 1, 1))
        e[j] = h
        fp = A.collide(lat, feq.reshape(9, 1, 1) + e, S9, mode=m)
        fm = A.collide(lat, feq.reshape(9, 1, 1) - e, S9, mode=m)
        fd[:, j] = ((fp - fm) / (2 * h)).reshape(9)
    assert np.abs(fd - J).max() <= 1e-8


def _power_iteration(lat, s, u0, mode, L, chunk=20, chunks=40, amp=1e-9, seed=7):
    """Growth rate per step of a small zero-mean perturbation under the full
    step (Oracle B), renormalised after every chunk; geometric mean over the
    second half of the chunks."""
    shape = (L,) * lat.d
    u = np.asarray(u0, dtype=np.float64).reshape((lat.d,) + (1,) * lat.d) * np.ones((lat.d,) + shape)
    base = A.equilibrium(lat, np.ones(shape), u)
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(base.shape)
    d -= d.mean(axis=tuple(range(1, d.ndim)), keepdims=True)
    d *= amp / np.linalg.norm(d)
    logs = []
    for _ in range(chunks):
        f = fast.run(lat, base + d, s, chunk, mode={"zero": A.ZERO, "fluid": A.FLUID}[mode], threads=4)
        g = np.linalg.norm(f - base)
        logs.append(np.log(g / amp))
        d = (f - base) * (amp / g)
    return float(np.exp(np.mean(logs[chunks // 2:]) / chunk))


@pytest.mark.parametrize("name,mode,u0", [("d2q9", "fluid", (0.25, 0.0)), ("d2q9", "zero", (0.25, 0.0)),
                                          ("d2q9_geier", "zero", (0.2, 0.2))])
def test_power_iteration_of_the_full_step_grows_at_the_spectral_radius(name, mode, u0):
    lat = lattices.make(name)
    L = 16
    J, _ = F.jacobian(lat, S9, u0, mode=mode)
    rad = F.spectral_radius(lat, J, L)
    assert rad > 1.01                                    # unstable: the perturbation must grow
    rate = _power_iteration(lat, S9, u0, mode, L)
    assert abs(rate - rad) <= 1e-4, (rate, rad)


def test_stable_state_does_not_grow():
    lat = lattices.make("d2q9_geier")
    u0 = (0.2, 0.0)
    J, _ = F.jacobian(lat, S9, u0, mode="fluid")
    rad = F.spectral_radius(lat, J, 16)
    assert rad <= 1.0 + 1e-12
    assert _power_iteration(lat, S9, u0, "fluid", 16) <= 1.0 + 1e-6
