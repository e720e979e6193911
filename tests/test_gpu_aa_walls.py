"""The in-place (AA) streaming form and half-way bounce-back walls on the GPU.

The in-place form must reproduce the two-array forms bit for bit (same per-node
arithmetic, only the memory layout differs).  Walls are compared with the
oracle's transport with walls (FP64, 1e-12) and must leave mass unchanged.
"""
import numpy as np
import pytest

from oracle import scheme as A
from paper_1312_3297_amd import lbmrv, workloads
from paper_1312_3297_amd.lbmrv import Lbmrv

from _common import far_state, oracle_lattice, rel, to_storage

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RATES = {9: workloads.RATES_D2Q9_GROUPED, 19: workloads.RATES_D3Q19, 27: workloads.RATES_D3Q27}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("lattice,storage", [("d2q9", "f32"), ("d3q19", "f32"), ("d3q27", "f64"),
                                             ("d3q19", "f16dev"), ("d3q27", "f32"), ("d3q27", "f16dev")])
@pytest.mark.parametrize("nsteps", [1, 4, 7])
def test_in_place_form_matches_pull_bitwise(lattice, storage, nsteps):
    lat = oracle_lattice(lattice)
    shape = (21, 300) if lat.d == 2 else (5, 6, 70)
    f0 = far_state(lat, shape, seed=11, amp=0.02, umax=0.08)
    st, _ = to_storage(lat, f0, storage)
    ctx = Lbmrv(lattice, RATES[lat.q], tuple(reversed(shape)), storage)
    ref_in = torch.from_numpy(st).cuda()
    ref_out = torch.empty_like(ref_in)
    ctx.set_streaming("pull")
    ctx.step(ref_in, ref_out, "fluid", 1.0, None, nsteps)
    ctx.set_streaming("aa")
    one = torch.from_numpy(st).cuda()
    ctx.step(one, one, "fluid", 1.0, None, nsteps)              # in place, one array
    a, b = torch.from_numpy(st).cuda(), torch.empty_like(ref_in)
    ctx.step(a, b, "fluid", 1.0, None, nsteps)                  # two arrays: copy then in place
    torch.cuda.synchronize()
    assert torch.equal(one, ref_out)
    assert torch.equal(b, ref_out)


@pytest.mark.parametrize("nx", [2, 4, 70, 71, 128, 256, 258, 384])
def test_d3q19_fp16_in_place_node_pairs_match_pull_bitwise(nx):
    """With FP16 storage the D3Q19 even in-place step takes two nodes per
    thread when nx is even (2 and 4: one and two pairs a row, the odd step's
    periodic wrap next to every pair; 70: 35 pairs a row, several rows per
    block; 128, 256, 384: one, two and three wavefronts a row; 258: 129 pairs,
    two blocks a row) and one otherwise (71); five rows leave the last block
    of each plane partly empty.  Every form stores the bits of the pull form,
    in both block orders."""
    lat = oracle_lattice("d3q19")
    shape = (3, 5, nx)
    f0 = far_state(lat, shape, seed=16, amp=0.02, umax=0.08)
    st, _ = to_storage(lat, f0, "f16dev")
    ctx = Lbmrv("d3q19", RATES[19], tuple(reversed(shape)), "f16dev")
    ctx.set_streaming("pull")
    ref_in = torch.from_numpy(st).cuda()
    ref = torch.empty_like(ref_in)
    ctx.step(ref_in, ref, "fluid", 1.0, None, 6)
    ctx.set_streaming("aa")
    for order in ("natural", "xcd"):
        ctx.set_block_order(order)
        one = torch.from_numpy(st).cuda()
        ctx.step(one, one, "fluid", 1.0, None, 6)
        torch.cuda.synchronize()
        assert torch.equal(one, ref), order


def test_d3q19_fp16_in_place_on_an_array_with_2_byte_alignment():
    """The interface asks FP16 arrays for 2-byte alignment only; an array that
    starts 2 bytes past a word boundary runs the even step one node per
    thread and still stores the pull form's bits."""
    lat = oracle_lattice("d3q19")
    shape = (4, 5, 70)
    f0 = far_state(lat, shape, seed=17, amp=0.02, umax=0.08)
    st, _ = to_storage(lat, f0, "f16dev")
    ctx = Lbmrv("d3q19", RATES[19], tuple(reversed(shape)), "f16dev")
    ctx.set_streaming("pull")
    ref_in = torch.from_numpy(st).cuda()
    ref = torch.empty_like(ref_in)
    ctx.step(ref_in, ref, "fluid", 1.0, None, 6)
    ctx.set_streaming("aa")
    flat = torch.zeros(st.size + 1, dtype=ref.dtype, device="cuda")
    one = flat[1:].view(st.shape)
    assert one.data_ptr() % 4 == 2
    one.copy_(torch.from_numpy(st).cuda())
    ctx.step(one, one, "fluid", 1.0, None, 6)
    torch.cuda.synchronize()
    assert torch.equal(one, ref)


@pytest.mark.parametrize("mode", ["zero", "fluid", "field"])
def test_d3q27_fp16_scatter_forms_match_pull_bitwise(mode):
    """The scatter forms (push, in-place odd) of the D3Q27 FP16-deviation
    step compute their destinations after the collision, the gather forms
    before it; every form stores the same bits."""
    lat = oracle_lattice("d3q27")
    shape = (5, 6, 200)                                  # 192 + 8 along x
    f0 = far_state(lat, shape, seed=13, amp=0.02, umax=0.08)
    st, _ = to_storage(lat, f0, "f16dev")
    fld = None
    if mode == "field":
        rng = np.random.default_rng(14)
        fld = torch.from_numpy(rng.uniform(-0.1, 0.1, (3,) + shape).astype(np.float32)).cuda()
    ctx = Lbmrv("d3q27", RATES[lat.q], tuple(reversed(shape)), "f16dev")
    outs = {}
    for streaming in ("pull", "push", "aa"):
        ctx.set_streaming(streaming)
        a = torch.from_numpy(st).cuda()
        b = a if streaming == "aa" else torch.empty_like(a)
        ctx.step(a, b, mode, 0.9, fld, 5)
        outs[streaming] = b
    torch.cuda.synchronize()
    assert torch.equal(outs["push"], outs["pull"])
    assert torch.equal(outs["aa"], outs["pull"])


def _walls(lat):
    """Walls on both y faces (the high one moving along x) and, in 3-D, on the low z face."""
    mask = (1 << 2) | (1 << 3) | ((1 << 4) if lat.d == 3 else 0)
    uw = [[0.0, 0.0, 0.0] for _ in range(6)]
    uw[3] = [0.03, 0.0, 0.0]
    return mask, uw


@pytest.mark.parametrize("lattice", ["d2q9", "d3q19", "d3q27"])
@pytest.mark.parametrize("mode", ["zero", "fluid"])
def test_bounce_back_walls_match_oracle_fp64(lattice, mode):
    lat = oracle_lattice(lattice)
    shape = (9, 70) if lat.d == 2 else (5, 6, 7)
    f0 = far_state(lat, shape, seed=13, amp=0.02, umax=0.05)
    mask, uw = _walls(lat)
    n = 6
    ref = A.run(lat, f0, RATES[lat.q], n, mode={"zero": A.ZERO, "fluid": A.FLUID}[mode],
                walls=(mask, uw, 1.0))
    ctx = Lbmrv(lattice, RATES[lat.q], tuple(reversed(shape)), "f64")
    ctx.set_walls(mask, uw, 1.0)
    fin = torch.from_numpy(f0).cuda()
    fout = torch.empty_like(fin)
    ctx.step(fin, fout, mode, 1.0, None, n)
    torch.cuda.synchronize()
    assert rel(fout.cpu().numpy(), ref) <= 1e-12


def test_walls_at_rest_conserve_mass_on_the_gpu():
    lat = oracle_lattice("d3q19")
    shape = (8, 9, 10)
    rho, u = workloads.taylor_green(10, 0.03, shape=shape)
    f0 = A.equilibrium(lat, rho, u)
    ctx = Lbmrv("d3q19", RATES[19], (10, 9, 8), "f64")
    ctx.set_walls(0b111111)
    m0, _, _ = ctx.conservation(torch.from_numpy(f0).cuda())
    fin = torch.from_numpy(f0).cuda()
    fout = torch.empty_like(fin)
    ctx.step(fin, fout, "fluid", 1.0, None, 100)
    m1, _, ok = ctx.conservation(fout)
    assert ok and abs(m1 - m0) <= 1e-12 * m0


def test_walls_need_the_pull_form_or_paired_in_place_walls():
    ctx = Lbmrv("d2q9", RATES[9], (8, 8), "f32")
    f = torch.zeros((9, 8, 8), device="cuda")
    g = torch.empty_like(f)
    for kind, mask in (("push", 0b1100), ("aa", 0b0100), ("aa", 0b1000), ("aa", 0b1101)):
        ctx.set_walls(mask)
        ctx.set_streaming(kind)
        with pytest.raises(lbmrv.LbmrvError) as e:
            ctx.step(f, g, "zero", 1.0, None, 2)
        assert e.value.code == lbmrv.ERR_UNSUPPORTED


@pytest.mark.parametrize("lattice,storage", [("d2q9", "f32"), ("d2q9", "f64"), ("d3q19", "f32"), ("d3q27", "f64")])
@pytest.mark.parametrize("nsteps", [1, 2, 5, 8])
def test_in_place_form_with_walls_matches_pull_bitwise(lattice, storage, nsteps):
    """Walls on both y faces (the upper one moving) and, in 3-D, on both z
    faces: the in-place form keeps each bounced population in the node's own
    opposite slot and must reproduce the pull form bit for bit."""
    lat = oracle_lattice(lattice)
    shape = (11, 130) if lat.d == 2 else (6, 7, 70)
    f0 = far_state(lat, shape, seed=14, amp=0.02, umax=0.05)
    st, _ = to_storage(lat, f0, storage)
    mask = (1 << 2) | (1 << 3) | ((1 << 4) | (1 << 5) if lat.d == 3 else 0)
    uw = [[0.0, 0.0, 0.0] for _ in range(6)]
    uw[3] = [0.03, 0.0, 0.0]
    if lat.d == 3:
        uw[4] = [0.0, 0.02, 0.0]
    ctx = Lbmrv(lattice, RATES[lat.q], tuple(reversed(shape)), storage)
    ctx.set_walls(mask, uw, 1.0)
    ref_in = torch.from_numpy(st).cuda()
    ref_out = torch.empty_like(ref_in)
    ctx.step(ref_in, ref_out, "fluid", 1.0, None, nsteps)
    ctx.set_streaming("aa")
    one = torch.from_numpy(st).cuda()
    ctx.step(one, one, "fluid", 1.0, None, nsteps)
    torch.cuda.synchronize()
    assert torch.equal(one, ref_out)
    if storage == "f64":
        ref = A.run(lat, f0, RATES[lat.q], nsteps, mode=A.FLUID, walls=(mask, uw, 1.0))
        assert rel(one.cpu().numpy(), ref) <= 1e-12


def test_in_place_form_with_walls_fp16_within_tolerance():
    """FP16 deviations with a moving wall: the in-place odd step stores a
    bounced population with the wall's momentum already added (one FP16
    rounding of the sum), the pull form stores it before the bounce and adds
    the momentum in FP32 when it reads it, so the two forms agree to the FP16
    tolerance rather than bit for bit; both are held to the oracle."""
    lat = oracle_lattice("d3q19")
    shape = (6, 7, 70)
    f0 = far_state(lat, shape, seed=15, amp=0.02, umax=0.05)
    st, f0w = to_storage(lat, f0, "f16dev")
    mask = 0b111100
    uw = [[0.0, 0.0, 0.0] for _ in range(6)]
    uw[3] = [0.03, 0.0, 0.0]
    ctx = Lbmrv("d3q19", RATES[19], (70, 7, 6), "f16dev")
    ctx.set_walls(mask, uw, 1.0)
    ctx.set_streaming("aa")
    one = torch.from_numpy(st).cuda()
    n = 7
    ctx.step(one, one, "fluid", 1.0, None, n)
    torch.cuda.synchronize()
    from _common import from_storage
    ref = A.run(lat, f0w, RATES[19], n, mode=A.FLUID, walls=(mask, uw, 1.0))
    assert rel(from_storage(lat, one.cpu().numpy(), "f16dev"), ref) <= 8e-5 * (n + 1)


def test_in_place_walls_at_rest_conserve_mass():
    lat = oracle_lattice("d3q19")
    shape = (8, 9, 10)
    rho, u = workloads.taylor_green(10, 0.03, shape=shape)
    f0 = A.equilibrium(lat, rho, u)
    ctx = Lbmrv("d3q19", RATES[19], (10, 9, 8), "f64")
    ctx.set_walls(0b111111)
    ctx.set_streaming("aa")
    m0, _, _ = ctx.conservation(torch.from_numpy(f0).cuda())
    f = torch.from_numpy(f0).cuda()
    ctx.step(f, f, "fluid", 1.0, None, 101)
    m1, _, ok = ctx.conservation(f)
    assert ok and abs(m1 - m0) <= 1e-12 * m0
