"""Run-time moment bases: the oracle's invariances and the library's host-side
validation (no GPU needed: every rejection happens before any HIP call).

Pins (section 1.2: the relaxation is diagonal in the basis P and leaves the
conserved moments rho, q unchanged), each a property of the scheme that the
oracle must reproduce with two different polynomial families:
  * adding multiples of the conserved polynomials (1, xi) to a non-conserved
    P_k does not change the scheme, for u~ = 0 and u~ = u: the row operation
    commutes with the relaxation because the conserved moments are at
    equilibrium;
  * rescaling a non-conserved P_k does not change it;
  * recombining basis elements that share one rate does not change it, while
    recombining elements with different rates does.
"""
import ctypes

import numpy as np
import pytest

from oracle import lattices
from oracle import scheme as A
from paper_1312_3297_amd import lbmrv, workloads as W

from _common import far_state


def _t(c, a=0, b=0, e=0):
    return (c, (a, b, e))


GEIER = [[_t(1)], [_t(1, 1)], [_t(1, 0, 1)], [_t(1, 2), _t(1, 0, 2)], [_t(1, 2), _t(-1, 0, 2)], [_t(1, 1, 1)],
         [_t(1, 1, 2)], [_t(1, 2, 1)], [_t(1, 2, 2)]]
S9 = [0, 0, 0, 1.1, 1.6, 1.75, 1.3, 1.45, 1.9]


def _run(lat, s, mode, n=3, seed=3, la=1.0):
    f0 = far_state(lat, (9, 11), seed=seed, amp=0.03, umax=0.1 * la)
    return A.run(lat, f0, s, n, la=la, mode=mode)


@pytest.mark.parametrize("mode", [A.ZERO, A.FLUID])
def test_term_list_basis_is_in_units_of_lambda(mode):
    """A term-list polynomial is evaluated at xi = X / lambda: the Geier family
    written as terms gives the built-in Geier scheme at any lambda."""
    for la in (1.0, 1.7):
        a = _run(lattices.with_basis("d2q9", GEIER), S9, mode, la=la)
        c = _run(lattices.make("d2q9_geier"), S9, mode, la=la)
        assert np.abs(a - c).max() <= 1e-13
    # an inhomogeneous family: the Hermite-like one written in X with lambda
    # explicit must equal its term list in xi (and differ from the same
    # coefficients read in X units when lambda != 1)
    la = 1.7
    h = [lambda X, Y, Z, l: 1 + 0 * X, lambda X, Y, Z, l: X / l, lambda X, Y, Z, l: Y / l,
         lambda X, Y, Z, l: (X ** 2 + Y ** 2) / l ** 2 - 2.0 / 3.0, lambda X, Y, Z, l: (X ** 2 - Y ** 2) / l ** 2,
         lambda X, Y, Z, l: X * Y / l ** 2, lambda X, Y, Z, l: X / l * (Y ** 2 / l ** 2 - 1.0 / 3.0),
         lambda X, Y, Z, l: Y / l * (X ** 2 / l ** 2 - 1.0 / 3.0),
         lambda X, Y, Z, l: (X ** 2 / l ** 2 - 1.0 / 3.0) * (Y ** 2 / l ** 2 - 1.0 / 3.0)]
    base = lattices.make("d2q9")
    explicit = lattices.Lattice("h", 2, [tuple(c) for c in base.c.tolist()], base.w_exact, h)
    a = _run(lattices.with_basis("d2q9", W.HERMITE_D2Q9), W.RATES_HERMITE_D2Q9, mode, la=la)
    b = _run(explicit, W.RATES_HERMITE_D2Q9, mode, la=la)
    assert np.abs(a - b).max() <= 1e-13
    x_units = [lambda X, Y, Z, l, P=P: P(X, Y, Z, 1.0) for P in h]
    c = _run(lattices.Lattice("x", 2, [tuple(c) for c in base.c.tolist()], base.w_exact, x_units),
             W.RATES_HERMITE_D2Q9, mode, la=la)
    assert np.abs(a - c).max() > 1e-6


@pytest.mark.parametrize("mode", [A.ZERO, A.FLUID])
def test_adding_conserved_polynomials_leaves_the_scheme_unchanged(mode):
    shifted = [list(p) for p in GEIER]
    shifted[3] += [_t(-2.0 / 3.0)]
    shifted[6] += [_t(-1.0 / 3.0, 1)]
    shifted[7] += [_t(-1.0 / 3.0, 0, 1), _t(0.7)]
    shifted[8] += [_t(0.25), _t(-0.4, 0, 1), _t(1.5, 1)]
    a = _run(lattices.with_basis("d2q9", GEIER), S9, mode)
    b = _run(lattices.with_basis("d2q9", shifted), S9, mode)
    assert np.abs(a - b).max() <= 1e-13


@pytest.mark.parametrize("mode", [A.ZERO, A.FLUID])
def test_rescaling_basis_elements_leaves_the_scheme_unchanged(mode):
    scaled = [list(p) for p in GEIER]
    for k, fac in ((3, 2.5), (5, -0.3), (8, 7.0)):
        scaled[k] = [(fac * c, e) for c, e in scaled[k]]
    a = _run(lattices.with_basis("d2q9", GEIER), S9, mode)
    b = _run(lattices.with_basis("d2q9", scaled), S9, mode)
    assert np.abs(a - b).max() <= 1e-13


@pytest.mark.parametrize("mode", [A.ZERO, A.FLUID])
def test_recombining_elements_with_one_rate_leaves_the_scheme_unchanged(mode):
    lat = lattices.make("d3q19")
    raw = lattices.with_basis("d3q19", W.RAW2_D3Q19)
    f0 = far_state(lat, (4, 5, 6), seed=5, amp=0.03, umax=0.1)
    # the built-in degree-2 block (trace, two normal-stress differences, three
    # shears) and the raw one (xi_x^2, xi_y^2, xi_z^2, shears) with one rate
    s = [0.0] * 4 + [1.3] * 6 + [1.5] * 6 + [1.2] * 3
    a = A.run(lat, f0, s, 2, mode=mode)
    b = A.run(raw, f0, s, 2, mode=mode)
    assert np.abs(a - b).max() <= 1e-13
    # with distinct rates on the raw normal stresses the schemes differ
    s2 = list(s)
    s2[4:7] = [1.1, 1.3, 1.5]
    c = A.run(raw, f0, s2, 2, mode=mode)
    assert np.abs(c - a).max() > 1e-6


# ---------------------------------------------------------------- host validation
def _create(lattice, polys, s=None, dims=(8, 8)):
    q = lbmrv.QD[lattice][0]
    s = s if s is not None else [0.0] * (lbmrv.QD[lattice][1] + 1) + [1.2] * (q - lbmrv.QD[lattice][1] - 1)
    pb = lbmrv.poly_basis(polys)
    rates = (ctypes.c_double * q)(*s)
    dd = (ctypes.c_int64 * 3)(*(list(dims) + [1] * (3 - len(dims))))
    h = ctypes.c_void_p()
    rc = lbmrv.library().lbmrv_create_custom(ctypes.byref(h), lbmrv.LATTICES[lattice], ctypes.byref(pb), 1.0, rates,
                                             dd, lbmrv.STORAGES["f32"], 1.0)
    if rc == lbmrv.OK:
        lbmrv.library().lbmrv_destroy(h)
    return rc


def _bad_geier():
    cases = {}
    b = [list(p) for p in GEIER]
    b[8] = [_t(1, 4), _t(1, 0, 4)]                        # xi_x^4 + xi_y^4: in neither D2Q9 span
    cases["outside_span"] = b
    b = [list(p) for p in GEIER]
    b[0] = [_t(2)]                                        # P_0 must be exactly 1
    cases["p0_not_one"] = b
    b = [list(p) for p in GEIER]
    b[1] = [_t(1, 1), _t(0.5)]                            # P_1 must be exactly xi_x
    cases["p1_not_xi"] = b
    b = [list(p) for p in GEIER]
    b[7] = list(b[6])                                     # two equal elements: singular R
    cases["singular"] = b
    b = [list(p) for p in GEIER]
    b[5] = [_t(1, 1, 1), _t(1, 0, 0, 1)]                  # a z term in 2-D
    cases["z_in_2d"] = b
    b = [list(p) for p in GEIER]
    b[5] = [_t(1, 9)]                                     # exponent above 8
    cases["exponent"] = b
    b = [list(p) for p in GEIER]
    b[5] = [_t(float("nan"), 1, 1)]
    cases["nan"] = b
    cases["missing_element"] = [list(p) for p in GEIER[:8]]
    b = [list(p) for p in GEIER]
    b[4] = [_t(1, 2), _t(-1, 0, 2), _t(1e-9, 1, 1, 0)]    # not exactly a recombination... still in span
    cases["in_span_ok"] = b
    return cases


@pytest.mark.parametrize("case", sorted(_bad_geier()))
def test_create_custom_validates_the_basis_on_the_host(case):
    rc = _create("d2q9", _bad_geier()[case])
    if case == "in_span_ok":
        # a valid basis passes validation; without a GPU the table upload fails
        assert rc in (lbmrv.OK, lbmrv.ERR_HIP)
    else:
        assert rc == lbmrv.ERR_INVALID_ARG


def test_create_custom_rejects_bad_rates_and_ill_conditioned_bases():
    assert _create("d2q9", GEIER, s=[0, 0, 0.1, 1, 1, 1, 1, 1, 1]) == lbmrv.ERR_INVALID_ARG
    b = [list(p) for p in GEIER]
    b[6] = [_t(1, 1, 2)]
    b[7] = [_t(1, 1, 2), _t(1e-12, 2, 1)]                 # nearly dependent: condition number ~1e12
    assert _create("d2q9", b) == lbmrv.ERR_INVALID_ARG


@pytest.mark.parametrize("lattice,polys", [("d2q9", W.HERMITE_D2Q9), ("d2q9", W.RAW_D2Q9),
                                           ("d3q19", W.RAW2_D3Q19), ("d3q27", W.HERMITE_D3Q27)])
def test_workload_bases_pass_validation(lattice, polys):
    assert _create(lattice, polys, dims=(4,) * lbmrv.QD[lattice][1]) in (lbmrv.OK, lbmrv.ERR_HIP)


def test_workload_bases_are_bases_of_the_lattice():
    """M_P(0) of each run-time basis is invertible on its lattice (oracle side)."""
    for name, polys in (("d2q9", W.HERMITE_D2Q9), ("d2q9", W.RAW_D2Q9), ("d3q19", W.RAW2_D3Q19),
                        ("d3q27", W.HERMITE_D3Q27)):
        lat = lattices.with_basis(name, polys)
        M = A.moment_matrix(lat, np.zeros((1, lat.d)))[0]
        assert np.linalg.cond(M) < 1e4
