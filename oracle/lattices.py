"""Velocity sets, weights and moment bases used by the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The D2Q9 velocity order and its orthogonal polynomial family follow the paper,
section 1.3 ("Two-dimensional examples"), eq. (mom).  The Geier family is
eq. (polgeier) of Proposition th:cascd2q9.  The paper gives no three-dimensional
lattice; the D3Q19/D3Q27 orders and the graded monomial bases below are a
reading of it (the order is an interface convention, shared with the HIP
library only as a written convention).

A basis is a list of Python callables ``P(X, Y, Z, la)``.  They use only
arithmetic operators, so they evaluate on NumPy arrays and on sympy symbols
alike; ``la`` is the velocity scale lambda of eq. (lambda).
"""
from fractions import Fraction as Fr

import numpy as np

# ----------------------------------------------------------------------------
# velocity sets (integer directions c_j; the physical velocity is v_j = la*c_j)
# ----------------------------------------------------------------------------

# Section 1.3: (0,0),(la,0),(0,la),(-la,0),(0,-la),(la,la),(-la,la),(-la,-la),(la,-la)
D2Q9_C = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
          (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)]

# Three-dimensional orders (a reading; the paper has none): rest, the six axis
# directions as +/- pairs, the twelve edge directions as +/- pairs, then (D3Q27)
# the eight corners as +/- pairs.
_AXIS = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
_EDGE = [(1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
         (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
         (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
_CORNER = [(1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1),
           (1, -1, 1), (-1, 1, -1), (-1, 1, 1), (1, -1, -1)]
D3Q19_C = [(0, 0, 0)] + _AXIS + _EDGE
D3Q27_C = [(0, 0, 0)] + _AXIS + _EDGE + _CORNER


def _weights(cs, table):
    """Standard weights by squared speed |c|^2 (the equilibrium is a reading: the paper leaves it open)."""
    return [table[c[0] ** 2 + c[1] ** 2 + c[2] ** 2] for c in cs]


D2Q9_W = _weights(D2Q9_C, {0: Fr(4, 9), 1: Fr(1, 9), 2: Fr(1, 36)})
D3Q19_W = _weights(D3Q19_C, {0: Fr(1, 3), 1: Fr(1, 18), 2: Fr(1, 36)})
D3Q27_W = _weights(D3Q27_C, {0: Fr(8, 27), 1: Fr(2, 27), 2: Fr(1, 54), 3: Fr(1, 216)})

# ----------------------------------------------------------------------------
# moment bases
# ----------------------------------------------------------------------------

# eq. (mom): the usual orthogonal D2Q9 family (Lallemand-Luo), lambda-scaled.
D2Q9_PAPER_BASIS = [
    lambda X, Y, Z, la: 1 + 0 * X,
    lambda X, Y, Z, la: X,
    lambda X, Y, Z, la: Y,
    lambda X, Y, Z, la: (3 * (X ** 2 + Y ** 2) - 4 * la ** 2) / la ** 2,
    lambda X, Y, Z, la: (X ** 2 - Y ** 2) / la ** 2,
    lambda X, Y, Z, la: X * Y / la ** 2,
    lambda X, Y, Z, la: X * (3 * (X ** 2 + Y ** 2) - 5 * la ** 2) / la ** 3,
    lambda X, Y, Z, la: Y * (3 * (X ** 2 + Y ** 2) - 5 * la ** 2) / la ** 3,
    lambda X, Y, Z, la: (9 * (X ** 2 + Y ** 2) ** 2 - 21 * la ** 2 * (X ** 2 + Y ** 2)
                         + 8 * la ** 4) / (2 * la ** 4),
]

# eq. (polgeier): 1, X, Y, X^2+Y^2, X^2-Y^2, XY, XY^2, X^2Y, X^2Y^2
D2Q9_GEIER_BASIS = [
    lambda X, Y, Z, la: 1 + 0 * X,
    lambda X, Y, Z, la: X,
    lambda X, Y, Z, la: Y,
    lambda X, Y, Z, la: X ** 2 + Y ** 2,
    lambda X, Y, Z, la: X ** 2 - Y ** 2,
    lambda X, Y, Z, la: X * Y,
    lambda X, Y, Z, la: X * Y ** 2,
    lambda X, Y, Z, la: X ** 2 * Y,
    lambda X, Y, Z, la: X ** 2 * Y ** 2,
]


def _mono(a, b, c):
    return lambda X, Y, Z, la: X ** a * Y ** b * Z ** c


# Degree-two block shared by both 3-D bases: bulk trace, two normal-stress
# differences, three off-diagonal stresses (a reading: the paper has no 3-D basis).
_DEG2 = [
    lambda X, Y, Z, la: X ** 2 + Y ** 2 + Z ** 2,
    lambda X, Y, Z, la: 2 * X ** 2 - Y ** 2 - Z ** 2,
    lambda X, Y, Z, la: Y ** 2 - Z ** 2,
    _mono(1, 1, 0), _mono(0, 1, 1), _mono(1, 0, 1),
]
_LOW = [_mono(0, 0, 0), _mono(1, 0, 0), _mono(0, 1, 0), _mono(0, 0, 1)]

D3Q19_BASIS = _LOW + _DEG2 + [
    _mono(1, 2, 0), _mono(1, 0, 2), _mono(2, 1, 0), _mono(0, 1, 2), _mono(2, 0, 1), _mono(0, 2, 1),
    _mono(2, 2, 0), _mono(2, 0, 2), _mono(0, 2, 2),
]

D3Q27_BASIS = _LOW + _DEG2 + [
    _mono(1, 2, 0), _mono(1, 0, 2), _mono(2, 1, 0), _mono(0, 1, 2), _mono(2, 0, 1), _mono(0, 2, 1),
    _mono(1, 1, 1),
    _mono(2, 2, 0), _mono(2, 0, 2), _mono(0, 2, 2),
    _mono(2, 1, 1), _mono(1, 2, 1), _mono(1, 1, 2),
    _mono(2, 2, 1), _mono(2, 1, 2), _mono(1, 2, 2),
    _mono(2, 2, 2),
]

# Human-readable names of the basis elements, for error reports.
BASIS_NAMES = {
    "d2q9_paper": ["rho", "qx", "qy", "e", "pxx", "pxy", "hx", "hy", "eps"],
    "d2q9_geier": ["1", "X", "Y", "X2+Y2", "X2-Y2", "XY", "XY2", "X2Y", "X2Y2"],
}


class Lattice:
    """A DdQq lattice with one moment basis, all in exact or FP64 form."""

    def __init__(self, name, d, cs, ws, basis):
        self.name = name
        self.d = d
        self.q = len(cs)
        self.c = np.array(cs, dtype=np.int64)[:, :3]
        self.w_exact = list(ws)
        self.w = np.array([float(x) for x in ws])
        self.basis = basis
        assert len(basis) == self.q

    def velocities(self, la):
        """v_j = la * c_j, shape (q, 3)."""
        return la * self.c.astype(np.float64)

    def __repr__(self):
        return "Lattice(%s)" % self.name


def polynomial(terms):
    """A basis element given as terms [(coef, (a, b, c)), ...] of the monomials
    xi_x^a xi_y^b xi_z^c in the dimensionless variable xi = X / la (section 1.2
    allows any polynomial family; this is how a run-time basis is written)."""
    terms = [(c, tuple(e) + (0,) * (3 - len(e))) for c, e in terms]

    def P(X, Y, Z, la):
        out = 0 * X
        for c, (a, b, e) in terms:
            out = out + c * (X / la) ** a * (Y / la) ** b * (Z / la) ** e
        return out
    return P


def with_basis(name, polys):
    """The velocity set and weights of lattice `name` with the moment basis
    `polys` (q term lists, see polynomial)."""
    import hashlib
    base = make(name)
    tag = hashlib.sha1(repr([[(float(c), tuple(e)) for c, e in t] for t in polys]).encode()).hexdigest()[:12]
    return Lattice(base.name + "_custom_" + tag, base.d, [tuple(c) for c in base.c.tolist()], base.w_exact,
                   [polynomial(t) for t in polys])


def make(name):
    if name in ("d2q9", "d2q9_paper"):
        return Lattice("d2q9_paper", 2, D2Q9_C, D2Q9_W, D2Q9_PAPER_BASIS)
    if name == "d2q9_geier":
        return Lattice("d2q9_geier", 2, D2Q9_C, D2Q9_W, D2Q9_GEIER_BASIS)
    if name == "d3q19":
        return Lattice("d3q19", 3, D3Q19_C, D3Q19_W, D3Q19_BASIS)
    if name == "d3q27":
        return Lattice("d3q27", 3, D3Q27_C, D3Q27_W, D3Q27_BASIS)
    raise ValueError(name)


ALL = ("d2q9_paper", "d2q9_geier", "d3q19", "d3q27")
