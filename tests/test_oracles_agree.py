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
