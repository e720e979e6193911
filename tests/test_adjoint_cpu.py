"""Pins of the FP64 adjoint oracle (Oracle E) against central finite differences
of the definition (Oracle A, NumPy) and against exact zeros the scheme fixes."""
import numpy as np
import pytest

from oracle import adjoint as E
from oracle import lattices
from oracle import scheme as A

pytest.importorskip("torch")


def _setup(name="d2q9", L=8, seed=0, field_amp=0.05, noise=0.01):
    lat = lattices.make(name)
    rng = np.random.default_rng(seed)
    shape = (L, L) if lat.d == 2 else (4, 4, 4)
    rho = 1 + 0.01 * rng.standard_normal(shape)
    u = 0.03 * rng.uniform(-1, 1, (lat.d,) + shape)
    f0 = A.equilibrium(lat, rho, u) * (1 + noise * rng.uniform(-1, 1, (lat.q,) + shape))
    s = np.concatenate([np.zeros(lat.d + 1), rng.uniform(1.1, 1.8, lat.q - lat.d - 1)])
    field = field_amp * rng.uniform(-1, 1, (lat.d,) + shape)
    return lat, f0, s, field


def _grads(lat, f0, s, field, n):
    fN = A.run(lat, f0, s, n, mode=A.FIELD, field=field)
    _, cot = E.kinetic_energy(lat, fN)
    return E.vjp(lat, f0, s, n, cot, field=field, K=4)


def _fd(fun, x, direction, h):
    return (fun(x + h * direction) - fun(x - h * direction)) / (2 * h)


def _rich(fun, x, direction, h):
    """Central differences with one Richardson step, O(h^4): far from
    equilibrium the O(h^2) truncation of a plain difference reaches 1e-7 of the
    derivative on D3Q27 (its error falls 4x per halving of h)."""
    return (4 * _fd(fun, x, direction, h / 2) - _fd(fun, x, direction, h)) / 3


@pytest.mark.parametrize("name", ["d2q9", "d2q9_geier", "d3q19", "d3q27"])
def test_adjoint_matches_central_differences(name):
    """Far from equilibrium with a large u~ so that every gradient is well above
    the finite-difference noise (about 100 eps |J| / h)."""
    lat, f0, s, field = _setup(name, noise=0.1, field_amp=0.2)
    n = 6
    _, gf, gs, gu = _grads(lat, f0, s, field, n)
    rng = np.random.default_rng(1)
    J = lambda f, ss, fl: E.objective_after(lat, f, ss, n, field=fl)  # noqa: E731
    J0 = J(f0, s, field)
    h = 1e-5
    noise = 300 * 2.2e-16 * abs(J0) / h

    def close(fd, ad):
        return abs(fd - ad) <= 1e-7 * abs(fd) + noise

    for _ in range(3):
        d = rng.standard_normal(f0.shape)
        assert close(_rich(lambda x: J(x, s, field), f0, d, h), (gf * d).sum())
        ds = np.concatenate([np.zeros(lat.d + 1), rng.standard_normal(lat.q - lat.d - 1)])
        assert close(_rich(lambda x: J(f0, x, field), s, ds, h), (gs * ds).sum())
        du = rng.standard_normal(field.shape)
        fd = _rich(lambda x: J(f0, s, x), field, du, h)
        assert abs(fd) > 1e3 * noise       # the u~ gradient is resolved
        assert close(fd, (gu * du).sum())
    # single components
    for idx in [(0, 0, 0), (3, 2, 5), (8, 7, 7)] if lat.d == 2 else [(0, 0, 0, 0), (7, 1, 2, 3), (26, 3, 0, 1)]:
        if idx[0] >= lat.q:
            continue
        e = np.zeros_like(f0)
        e[idx] = 1.0
        assert close(_rich(lambda x: J(x, s, field), f0, e, h), gf[idx])


def test_conserved_rates_have_zero_gradient():
    """s_k for the conserved moments multiplies m^eq_k - m_k = 0 (section 1.1)."""
    lat, f0, s, field = _setup("d2q9")
    _, _, gs, _ = _grads(lat, f0, s, field, 5)
    assert np.abs(gs[: lat.d + 1]).max() <= 1e-14
    assert np.abs(gs[lat.d + 1:]).max() > 1e-8


def test_bgk_rates_make_the_relative_velocity_irrelevant():
    """Equal non-conserved rates: the step does not depend on u~, so dJ/du~ = 0."""
    lat, f0, s, field = _setup("d2q9", field_amp=0.2)
    s = np.where(np.arange(lat.q) > lat.d, 1.3, 0.0)
    _, _, _, gu = _grads(lat, f0, s, field, 5)
    assert np.abs(gu).max() <= 1e-14


def test_adjoint_dot_product_identity_one_step():
    """<J v, w> = <v, J^T w> for one step (forward-mode vs reverse-mode)."""
    import torch
    lat, f0, s, field = _setup("d2q9")
    rng = np.random.default_rng(3)
    v = rng.standard_normal(f0.shape)
    w = rng.standard_normal(f0.shape)
    st = torch.tensor(s)
    fl = torch.tensor(field)
    _, jv = torch.func.jvp(lambda x: E.step(lat, x, st, 1.0, fl), (torch.tensor(f0),), (torch.tensor(v),))
    _, gf, _, _ = E.vjp(lat, f0, s, 1, w, field=field)
    assert abs(float((jv.numpy() * w).sum()) - float((v * gf).sum())) <= 1e-13 * np.abs(v * gf).sum()


@pytest.mark.parametrize("name", ["d2q9", "d2q9_geier", "d3q19", "d3q27"])
def test_torch_step_is_oracle_a_step(name):
    import torch
    lat, f0, s, field = _setup(name, noise=0.1, field_amp=0.2)
    a = A.step(lat, f0, s, 1.0, A.FIELD, field=field)
    b = E.step(lat, torch.tensor(f0), torch.tensor(s), 1.0, torch.tensor(field)).numpy()
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()
    a = A.step(lat, f0, s, 1.0, A.FLUID, alpha=0.7)
    b = E.step(lat, torch.tensor(f0), torch.tensor(s), 1.0, alpha=0.7).numpy()
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()
    a = A.step(lat, f0, s, 1.0, A.ZERO)
    b = E.step(lat, torch.tensor(f0), torch.tensor(s), 1.0).numpy()
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()


@pytest.mark.parametrize("name", ["d2q9", "d3q19", "d3q27"])
def test_zero_mode_adjoint_matches_central_differences(name):
    """u~ = 0 (the d'Humieres scheme): gradients with respect to f0 and s."""
    lat, f0, s, _ = _setup(name, noise=0.1)
    n = 5
    fN = A.run(lat, f0, s, n, mode=A.ZERO)
    J0, cot = E.kinetic_energy(lat, fN)
    _, gf, gs, _ = E.vjp(lat, f0, s, n, cot, K=2)
    J = lambda f, ss: E.objective_after(lat, f, ss, n)  # noqa: E731
    rng = np.random.default_rng(8)
    h = 1e-5
    noise = 300 * 2.2e-16 * abs(J0) / h
    for _ in range(3):
        d = rng.standard_normal(f0.shape)
        fd = _rich(lambda x: J(x, s), f0, d, h)
        assert abs(fd - (gf * d).sum()) <= 1e-7 * abs(fd) + noise
        ds = np.concatenate([np.zeros(lat.d + 1), rng.standard_normal(lat.q - lat.d - 1)])
        fd = _rich(lambda x: J(f0, x), s, ds, h)
        assert abs(fd - (gs * ds).sum()) <= 1e-7 * abs(fd) + noise


def test_kinetic_energy_gradient_closed_form():
    lat, f0, _, _ = _setup("d2q9")
    J, g = E.kinetic_energy(lat, f0)
    rng = np.random.default_rng(4)
    d = rng.standard_normal(f0.shape)
    fd = (E.kinetic_energy(lat, f0 + 1e-6 * d)[0] - E.kinetic_energy(lat, f0 - 1e-6 * d)[0]) / 2e-6
    assert abs(fd - (g * d).sum()) <= 1e-8 * abs(fd)


@pytest.mark.parametrize("name", ["d2q9", "d3q19", "d3q27"])
def test_fluid_mode_adjoint_matches_central_differences(name):
    """u~ = alpha u(f): the gradient also flows through u = q / rho."""
    lat, f0, s, _ = _setup(name, noise=0.1)
    n, alpha = 5, 0.8
    fN = A.run(lat, f0, s, n, mode=A.FLUID, alpha=alpha)
    J0, cot = E.kinetic_energy(lat, fN)
    _, gf, gs, _ = E.vjp(lat, f0, s, n, cot, alpha=alpha, K=2)
    rng = np.random.default_rng(7)
    h = 1e-5
    J = lambda f, ss: E.objective_after(lat, f, ss, n, alpha=alpha)  # noqa: E731

    def rich(fun, x, d):
        return _rich(fun, x, d, h)

    noise = 300 * 2.2e-16 * abs(J0) / h
    for _ in range(3):
        d = rng.standard_normal(f0.shape)
        fd = rich(lambda x: J(x, s), f0, d)
        assert abs(fd - (gf * d).sum()) <= 1e-7 * abs(fd) + noise
        ds = np.concatenate([np.zeros(lat.d + 1), rng.standard_normal(lat.q - lat.d - 1)])
        fd = rich(lambda x: J(f0, x), s, ds)
        assert abs(fd - (gs * ds).sum()) <= 1e-7 * abs(fd) + noise
    # and it differs from the frozen-field adjoint at the same u~ values
    _, u0 = A.conserved(lat, f0)
    _, gf_field, _, _ = E.vjp(lat, f0, s, n, cot, field=alpha * u0, K=2)
    assert np.abs(gf - gf_field).max() > 1e-8


@pytest.mark.parametrize("name,mode", [("d2q9_geier", "fluid"), ("d2q9", "field"), ("d3q19", "fluid")])
def test_maxwellian_adjoint_matches_central_differences(name, mode):
    """The Maxwellian equilibria (m^eq = rho E[P_k(xi - u~)]): Oracle E's
    gradients against central differences of Oracle A with the same
    equilibrium, for u~ = u (differentiated through u = q / rho) and a field."""
    lat, f0, s, field = _setup(name, noise=0.1, field_amp=0.2)
    n = 5
    fld = field if mode == "field" else None
    alpha = 0.9 if mode == "fluid" else None
    fN = A.run(lat, f0, s, n, mode=A.FIELD if fld is not None else A.FLUID, alpha=0.9, field=fld, eq="maxwellian")
    _, cot = E.kinetic_energy(lat, fN)
    _, gf, gs, gu = E.vjp(lat, f0, s, n, cot, field=fld, K=3, alpha=alpha, eq="maxwellian")
    J = lambda f, ss, fl: E.objective_after(lat, f, ss, n, field=fl, alpha=alpha, eq="maxwellian")  # noqa: E731
    J0 = J(f0, s, fld)
    h = 2e-5
    rng = np.random.default_rng(2)

    def rfd(fun, x, direction):
        # Richardson-extrapolated central difference: the Maxwellian's quartic
        # terms make the O(h^2) truncation of a plain difference ~1e-7 here
        return (4 * _fd(fun, x, direction, h / 2) - _fd(fun, x, direction, h)) / 3

    def close(fd, ad):
        return abs(fd - ad) <= 1e-9 * abs(fd) + 100 * 2.2e-16 * abs(J0) / h

    for _ in range(2):
        d = rng.standard_normal(f0.shape)
        assert close(rfd(lambda x: J(x, s, fld), f0, d), (gf * d).sum())
        ds = np.concatenate([np.zeros(lat.d + 1), rng.standard_normal(lat.q - lat.d - 1)])
        assert close(rfd(lambda x: J(f0, x, fld), s, ds), (gs * ds).sum())
        if fld is not None:
            du = rng.standard_normal(fld.shape)
            assert close(rfd(lambda x: J(f0, s, x), fld, du), (gu * du).sum())
    # and the Maxwellian gradient differs from the polynomial one (the option matters)
    _, gf_p, _, _ = E.vjp(lat, f0, s, n, cot, field=fld, K=3, alpha=alpha)
    assert np.abs(gf_p - gf).max() > 1e-6 * np.abs(gf).max()
