"""The order in which workgroups take their tiles changes nothing but speed:
every node's arithmetic is the same, so the natural and the per-XCD order must
give the same bits, for every streaming form, with walls and with a run-time
basis, on grids whose block counts are and are not multiples of eight."""
import numpy as np
import pytest

from oracle import scheme as A
from paper_1312_3297_amd import workloads
from paper_1312_3297_amd.lbmrv import Lbmrv

from _common import far_state, oracle_lattice, to_storage

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RATES = {9: workloads.RATES_D2Q9_GROUPED, 19: workloads.RATES_D3Q19, 27: workloads.RATES_D3Q27}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(lattice, shape, storage, streaming, order, walls=False, basis="default", nsteps=7):
    lat = oracle_lattice(lattice)
    f0 = far_state(lat, shape, seed=81, amp=0.02, umax=0.06)
    st, _ = to_storage(lat, f0, storage)
    s = RATES[lat.q] if isinstance(basis, str) else workloads.RATES_RAW2_D3Q19
    ctx = Lbmrv(lattice, s, tuple(reversed(shape)), storage, basis=basis)
    ctx.set_streaming(streaming)
    ctx.set_block_order(order)
    if walls:
        ctx.set_walls(0b1100, [[0, 0, 0]] * 3 + [[0.02, 0, 0]] + [[0, 0, 0]] * 2, 1.0)
    a = torch.from_numpy(st).cuda()
    b = a if streaming == "aa" else torch.empty_like(a)
    ctx.step(a, b, "fluid", 1.0, None, nsteps)
    torch.cuda.synchronize()
    return b.cpu()


@pytest.mark.parametrize("lattice,shape", [("d2q9", (37, 600)), ("d2q9", (64, 512)), ("d3q19", (5, 7, 300)),
                                           ("d3q27", (4, 8, 130))])
@pytest.mark.parametrize("streaming", ["pull", "push", "aa"])
def test_block_orders_give_identical_bits(lattice, shape, streaming):
    ref = _run(lattice, shape, "f32", streaming, "natural")
    assert torch.equal(_run(lattice, shape, "f32", streaming, "xcd"), ref)
    assert torch.equal(_run(lattice, shape, "f32", streaming, "auto"), ref)


def test_block_orders_with_walls_fp16_and_runtime_basis():
    assert torch.equal(_run("d2q9", (33, 700), "f16dev", "pull", "xcd", walls=True),
                       _run("d2q9", (33, 700), "f16dev", "pull", "natural", walls=True))
    assert torch.equal(_run("d3q19", (6, 5, 260), "f64", "pull", "xcd", basis=workloads.RAW2_D3Q19),
                       _run("d3q19", (6, 5, 260), "f64", "pull", "natural", basis=workloads.RAW2_D3Q19))


@pytest.mark.parametrize("mode", ["zero", "fluid", "field"])
def test_adjoint_is_independent_of_the_block_order(mode):
    """The reverse kernel takes its tiles in the chosen order too; its dJ/ds
    partial sums are kept per tile, so every output is identical bit for bit."""
    lat = oracle_lattice("d2q9")
    shape = (40, 600)
    f0 = far_state(lat, shape, seed=82, amp=0.02, umax=0.05)
    rng = np.random.default_rng(83)
    cot = torch.from_numpy(rng.standard_normal(f0.shape).astype(np.float32)).cuda()
    fld = torch.from_numpy((0.03 * rng.uniform(-1, 1, (2,) + shape)).astype(np.float32)).cuda() \
        if mode == "field" else None
    st, _ = to_storage(lat, f0, "f32")
    outs = []
    for order in ("natural", "xcd"):
        ctx = Lbmrv("d2q9", RATES[9], (600, 40), "f32")
        ctx.set_block_order(order)
        res = ctx.adjoint(torch.from_numpy(st).cuda(), cot, 9, 4, mode, fld, want_fN=True)
        torch.cuda.synchronize()
        outs.append([None if r is None else r.cpu() for r in res])
    for a, b in zip(*outs):
        assert (a is None and b is None) or torch.equal(a, b)
