"""Linear stability measured through the GPU step against Oracle F.

The power iteration of paper_1312_3297_amd.stability (library step, deviation
norm and rescale kernels, FP64) must reproduce the spectral radius of the
linearised step over the grid's nonzero wavenumbers (Oracle F, eigenvalues of
diag(e^{-i k.c}) J with J from autodiff of the definition) to 1e-4, and the
critical speeds it finds by bisection must match the oracle's bisection with
the same criterion.  The map of critical speeds is printed (pytest -s).
"""
import numpy as np
import pytest

from oracle import lattices
from oracle import stability as F
from paper_1312_3297_amd import stability
from paper_1312_3297_amd.lbmrv import Lbmrv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

S9 = [0, 0, 0, 1.4, 1.95, 1.95, 1.2, 1.2, 1.4]
S19 = [0.0] * 4 + [1.1] + [1.9] * 5 + [1.5] * 6 + [1.3] * 3
ORACLE = {("d2q9", "default"): "d2q9_paper", ("d2q9", "geier"): "d2q9_geier", ("d3q19", "default"): "d3q19"}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("lattice,basis,mode,u0,L", [
    ("d2q9", "default", "fluid", (0.25, 0.0), 16),
    ("d2q9", "default", "zero", (0.25, 0.0), 16),
    ("d2q9", "geier", "zero", (0.2, 0.2), 16),
    ("d2q9", "geier", "fluid", (0.3, 0.1), 16),
    ("d3q19", "default", "zero", (0.4, 0.0, 0.0), 8),
    ("d3q19", "default", "fluid", (0.4, 0.0, 0.0), 8),
])
def test_gpu_growth_rate_is_the_spectral_radius(lattice, basis, mode, u0, L):
    s = S9 if lattice == "d2q9" else S19
    lat = lattices.make(ORACLE[(lattice, basis)])
    J, _ = F.jacobian(lat, s, u0, mode=mode)
    rad = F.spectral_radius(lat, J, L)
    ctx = Lbmrv(lattice, s, (L,) * lat.d, "f64", basis=basis)
    rate = stability.growth_rate(ctx, u0, mode)
    print("\n%s/%s %s u0=%s: GPU rate %.7f, oracle radius %.7f" % (lattice, basis, mode, u0, rate, rad))
    assert rad > 1.002
    assert abs(rate - rad) <= 1e-5


def test_gpu_power_iteration_follows_the_oracle_step():
    """Where the two largest moduli are close (1.09382 and 1.09408 here) ten
    thousand steps do not reach the radius; the GPU iteration must still be
    the oracle's: the same start (seed, zero mean, 1e-9), chunks and
    renormalisation through Oracle B give the same rate."""
    from oracle import fast
    from oracle import scheme as A
    lat = lattices.make("d3q19")
    u0, L, chunk, chunks, tail, amp = (0.35, 0.1, 0.05), 8, 50, 200, 50, 1e-9
    ctx = Lbmrv("d3q19", S19, (L, L, L), "f64")
    rate = stability.growth_rate(ctx, u0, "zero", chunk=chunk, chunks=chunks, tail=tail, amp=amp, seed=1316)
    shape = (L, L, L)
    base = A.equilibrium(lat, np.ones(shape), np.asarray(u0).reshape(3, 1, 1, 1) * np.ones((3,) + shape))
    rng = np.random.default_rng(1316)
    d = rng.standard_normal(base.shape)
    d -= d.mean(axis=(1, 2, 3), keepdims=True)
    d *= amp / np.sqrt((d ** 2).sum())
    logs = []
    for _ in range(chunks):
        f = fast.run(lat, base + d, S19, chunk, mode=A.ZERO)
        g = np.sqrt(((f - base) ** 2).sum())
        logs.append(np.log(g / amp))
        d = (f - base) * (amp / g)
    ref = float(np.exp(np.mean(logs[-tail:]) / chunk))
    print("\nd3q19 zero u0=%s: GPU %.9f, Oracle B iteration %.9f" % (u0, rate, ref))
    assert abs(rate - ref) <= 1e-7


def test_gpu_stable_state_does_not_grow():
    ctx = Lbmrv("d2q9", S9, (16, 16), "f64", basis="geier")
    lat = lattices.make("d2q9_geier")
    J, _ = F.jacobian(lat, S9, (0.2, 0.0), mode="fluid")
    assert F.spectral_radius(lat, J, 16) <= 1 + 1e-12
    assert stability.growth_rate(ctx, (0.2, 0.0), "fluid") <= 1 + 1e-6


def test_critical_speed_map_matches_oracle():
    """Critical |u0| along x and along the diagonal, D2Q9, both bases,
    u~ = 0 and u~ = u, shear rate s_nu in {1.8, 1.9, 1.95, 1.99}: GPU power
    iteration against the oracle's eigenvalues, same bisection (12 halvings
    of [0, 0.6], unstable when the growth per step exceeds 1 + 1e-3) on a
    16^2 grid."""
    rows = []
    worst = 0.0
    for basis in ("default", "geier"):
        lat = lattices.make(ORACLE[("d2q9", basis)])
        for sv in (1.8, 1.9, 1.95, 1.99):
            s = [0, 0, 0, 1.4, sv, sv, 1.2, 1.2, 1.4]
            for direction in ((1.0, 0.0), (1.0, 1.0)):
                got = [stability.critical_speed("d2q9", s, direction, 16, mode, basis=basis, iters=12)
                       for mode in ("zero", "fluid")]
                ref = [F.critical_speed(lat, s, direction, 16, mode, threshold=1e-3, iters=12)
                       for mode in ("zero", "fluid")]
                rows.append((basis, sv, direction, got, ref))
                worst = max(worst, max(abs(a - b) for a, b in zip(got, ref)))
    print("\ncritical |u0| (GPU; oracle), 16^2 grid, threshold 1 + 1e-3:")
    for basis, sv, direction, got, ref in rows:
        print("  %-7s s_nu=%.2f dir=%s  u~=0: %.4f (%.4f)   u~=u: %.4f (%.4f)"
              % (basis, sv, direction, got[0], ref[0], got[1], ref[1]))
    # one bisection interval (0.6 / 2^12) of slack for decisions within the
    # rate's estimation error of the threshold
    assert worst <= 2 * 0.6 / 2 ** 12 + 1e-12


def test_critical_speed_map_d3q19_matches_oracle():
    """D3Q19 (the built-in graded monomial basis) on an 8^3 grid: critical
    |u0| along x, the xy diagonal and the main diagonal, s_nu in {1.9, 1.99},
    u~ = 0 and u~ = u, GPU power iteration against the oracle's eigenvalues."""
    lat = lattices.make("d3q19")
    rows = []
    worst = 0.0
    for sv in (1.9, 1.99):
        s = [0.0] * 4 + [1.1] + [sv] * 5 + [1.5] * 6 + [1.3] * 3
        for direction in ((1.0, 0.0, 0.0), (1.0, 1.0, 0.0), (1.0, 1.0, 1.0)):
            got = [stability.critical_speed("d3q19", s, direction, 8, mode, iters=12) for mode in ("zero", "fluid")]
            ref = [F.critical_speed(lat, s, direction, 8, mode, threshold=1e-3, iters=12)
                   for mode in ("zero", "fluid")]
            rows.append((sv, direction, got, ref))
            worst = max(worst, max(abs(a - b) for a, b in zip(got, ref)))
    print("\ncritical |u0| (GPU; oracle), D3Q19 8^3 grid, threshold 1 + 1e-3:")
    for sv, direction, got, ref in rows:
        print("  s_nu=%.2f dir=%s  u~=0: %.4f (%.4f)   u~=u: %.4f (%.4f)"
              % (sv, direction, got[0], ref[0], got[1], ref[1]))
    assert worst <= 2 * 0.6 / 2 ** 12 + 1e-12
