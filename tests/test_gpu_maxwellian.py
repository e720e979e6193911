"""The Maxwellian equilibrium option on the GPU against the oracle's
Gauss-Hermite evaluation of the same moments."""
import numpy as np
import pytest

from oracle import scheme as A
from paper_1312_3297_amd import lbmrv, workloads
from paper_1312_3297_amd.lbmrv import Lbmrv

from _common import far_state, from_storage, oracle_lattice, rel, to_storage

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RATES = {9: workloads.RATES_D2Q9_GROUPED, 19: workloads.RATES_D3Q19, 27: workloads.RATES_D3Q27}
MODES = {"zero": A.ZERO, "fluid": A.FLUID, "field": A.FIELD}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("lattice,basis", [("d2q9", "default"), ("d2q9", "geier"), ("d3q19", "default"),
                                           ("d3q27", "default")])
@pytest.mark.parametrize("storage,mode,n", [("f64", "fluid", 6), ("f64", "field", 6), ("f32", "fluid", 6)])
def test_maxwellian_equilibrium_matches_oracle(lattice, basis, storage, mode, n):
    lat = oracle_lattice(lattice, basis)
    shape = (11, 270) if lat.d == 2 else (4, 5, 70)
    f0 = far_state(lat, shape, seed=17, amp=0.02, umax=0.08)
    st, f0w = to_storage(lat, f0, storage)
    field = (0.1 * np.random.default_rng(18).uniform(-1, 1, (lat.d,) + shape)).astype(np.float32).astype(np.float64)
    ref = A.run(lat, f0w, RATES[lat.q], n, mode=MODES[mode], alpha=0.9, field=field, eq="maxwellian")
    ctx = Lbmrv(lattice, RATES[lat.q], tuple(reversed(shape)), storage, basis)
    ctx.set_equilibrium("maxwellian")
    fin = torch.from_numpy(st).cuda()
    fout = torch.empty_like(fin)
    ctx.step(fin, fout, mode, 0.9, torch.from_numpy(field.astype(np.float32)).cuda(), n)
    torch.cuda.synchronize()
    got = from_storage(lat, fout.cpu().numpy(), storage)
    tol = 1e-12 if storage == "f64" else 3e-7 * (n + 4)
    assert rel(got, ref) <= tol
    # and the option changes the result
    poly = A.run(lat, f0w, RATES[lat.q], n, mode=MODES[mode], alpha=0.9, field=field)
    assert rel(poly, ref) > 1e-9


def test_adjoint_still_rejects_walls():
    """The adjoint covers periodic domains (either equilibrium); walls are not
    differentiated."""
    ctx = Lbmrv("d2q9", RATES[9], (8, 8), "f64")
    ctx.set_equilibrium("maxwellian")
    ctx.set_walls(0b1100)
    f = torch.zeros((9, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(lbmrv.LbmrvError) as e:
        ctx.adjoint(f, f, 3, 2, "zero")
    assert e.value.code == lbmrv.ERR_UNSUPPORTED
