"""Oracle A (NumPy) and Oracle B (C/OpenMP) implement the same definition
independently (different LU codes, different loops); they agree to rounding."""
import numpy as np
import pytest

from oracle import fast, lattices
from oracle import scheme as A


@pytest.mark.parametrize("name", lattices.ALL)
@pytest.mark.parametrize("mode", [A.ZERO, A.FLUID, A.FIELD])
@pytest.mark.parametrize("la", [1.0, 1.6])
def test_oracle_b_matches_oracle_a(name, mode, la):
    lat = lattices.make(name)
    shape = (6, 7) if lat.d == 2 else (3, 4, 5)
    rng = np.random.default_rng(0)
    rho = 1 + 0.05 * rng.standard_normal(shape)
    u = 0.1 * la * rng.uniform(-1, 1, (lat.d,) + shape)
    f = A.equilibrium(lat, rho, u, la) * (1 + 0.1 * rng.uniform(-1, 1, (lat.q,) + shape))
    s = np.concatenate([np.zeros(lat.d + 1), rng.uniform(0.6, 1.9, lat.q - lat.d - 1)])
    fld = la * rng.uniform(-0.3, 0.3, (lat.d,) + shape)
    a = A.run(lat, f, s, 5, la, mode, 0.8, fld)
    b = fast.run(lat, f, s, 5, la, mode, 0.8, fld, threads=2)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


def test_oracle_b_thread_count_does_not_change_the_result():
    lat = lattices.make("d3q19")
    rng = np.random.default_rng(1)
    shape = (5, 6, 7)
    f = A.equilibrium(lat, np.ones(shape), 0.05 * rng.uniform(-1, 1, (3,) + shape))
    s = [0.0] * 4 + [1.1] + [1.9] * 5 + [1.5] * 6 + [1.8] * 3
    a = fast.run(lat, f, s, 4, mode=A.FLUID, threads=1)
    b = fast.run(lat, f, s, 4, mode=A.FLUID, threads=3)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("name", lattices.ALL)
@pytest.mark.parametrize("mode", [A.ZERO, A.FLUID, A.FIELD])
@pytest.mark.parametrize("la", [1.0, 1.6])
def test_triangular_form_matches_oracle_a(name, mode, la):
    """Oracle B's triangular-solve form (M(u~) = T(u~) M(0), eq. (matTu),
    forward substitution) gives Oracle A's step; the grid is not a multiple of
    the node batch, so the ragged last batch is covered."""
    lat = lattices.make(name)
    shape = (6, 7) if lat.d == 2 else (3, 4, 5)
    rng = np.random.default_rng(2)
    rho = 1 + 0.05 * rng.standard_normal(shape)
    u = 0.1 * la * rng.uniform(-1, 1, (lat.d,) + shape)
    f = A.equilibrium(lat, rho, u, la) * (1 + 0.1 * rng.uniform(-1, 1, (lat.q,) + shape))
    s = np.concatenate([np.zeros(lat.d + 1), rng.uniform(0.6, 1.9, lat.q - lat.d - 1)])
    fld = la * rng.uniform(-0.3, 0.3, (lat.d,) + shape)
    a = A.run(lat, f, s, 5, la, mode, 0.8, fld)
    b = fast.run_tri(lat, f, s, 5, la, mode, 0.8, fld, threads=3)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
    c = fast.collide_tri(lat, f, s, la, mode, 0.8, fld, threads=1)
    assert np.abs(c - A.collide(lat, f, s, la, mode, 0.8, fld)).max() <= 1e-13 * np.abs(c).max()


def test_triangular_form_is_independent_of_threads_and_far_from_equilibrium():
    lat = lattices.make("d3q27")
    rng = np.random.default_rng(3)
    shape = (5, 6, 7)
    f = A.equilibrium(lat, np.ones(shape), 0.2 * rng.uniform(-1, 1, (3,) + shape)) * \
        (1 + 0.3 * rng.uniform(-1, 1, (27,) + shape))
    s = [0.0] * 4 + list(rng.uniform(0.5, 1.95, 23))
    a = fast.run_tri(lat, f, s, 3, mode=A.FLUID, threads=1)
    b = fast.run_tri(lat, f, s, 3, mode=A.FLUID, threads=4)
    assert np.array_equal(a, b)
    ref = A.run(lat, f, s, 3, mode=A.FLUID)
    assert np.abs(a - ref).max() <= 1e-13 * np.abs(ref).max()


def test_triangular_form_refuses_a_basis_whose_shift_is_not_triangular():
    """With two basis elements of different degree swapped, T(u~) = M(u~) M(0)^{-1}
    is no longer lower triangular, and the triangular form must not be used."""
    base = lattices.make("d2q9_geier")
    basis = list(base.basis)
    basis[3], basis[6] = basis[6], basis[3]            # X^2 + Y^2 after X Y^2
    lat = lattices.Lattice("d2q9_geier_unordered", 2, [tuple(c) for c in base.c.tolist()], base.w_exact, basis)
    f = A.equilibrium(lat, np.ones((3, 4)), np.zeros((2, 3, 4)))
    with pytest.raises(ValueError):
        fast.run_tri(lat, f, [0, 0, 0, 1.1, 1.2, 1.3, 1.4, 1.5, 1.6], 1, mode=A.FLUID)
