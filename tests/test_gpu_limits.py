"""The largest and the smallest grids the interface accepts.

Largest: grids whose element offsets j * N + n pass 2^31 and 2^32 (q * N above
2^32), up to the largest node count lbmrv_create accepts (2^32 - 256; node
indices are 32-bit).  The initial state is a periodic tiling of a small
block built on the host; a periodic start stays periodic under the scheme, so
the oracle's run on the small periodic block is the exact answer at every node
of the large grid, and sampled nodes (faces, corners, the last elements) are
compared with it.  Smallest: one node (the transport maps a node onto itself,
so a step is a collision), grids one node wide, and nsteps = 0.
"""
import numpy as np
import pytest

from oracle import fast
from oracle import scheme as A
from paper_1312_3297_amd import workloads
from paper_1312_3297_amd.lbmrv import Lbmrv

from _common import far_state, from_storage, oracle_lattice, rel, to_storage

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RATES = {9: workloads.RATES_D2Q9_GROUPED, 19: workloads.RATES_D3Q19, 27: workloads.RATES_D3Q27}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _tiled_case(lattice, block, reps, storage, mode, nsteps, tol, seed):
    lat = oracle_lattice(lattice)
    q = lat.q
    dims_zyx = tuple(b * r for b, r in zip(block, reps))            # grid axes (z, y, x) or (y, x)
    nodes = int(np.prod(dims_zyx))
    assert nodes <= 2 ** 32 - 256
    f0 = far_state(lat, block, seed=seed, amp=0.02, umax=0.08)
    st, f0w = to_storage(lat, f0, storage)
    ref = fast.run(lat, f0w, RATES[q], nsteps, mode={"zero": A.ZERO, "fluid": A.FLUID}[mode])
    ctx = Lbmrv(lattice, RATES[q], tuple(reversed(dims_zyx)), storage)
    small = torch.from_numpy(st).to("cuda")
    fin = small.repeat((1,) + tuple(reps)).contiguous()
    del small
    fout = torch.empty_like(fin)
    ctx.step(fin, fout, mode, 1.0, None, nsteps)
    mass, _, finite = ctx.conservation(fout)
    torch.cuda.synchronize()
    del fin
    rng = np.random.default_rng(seed + 1)
    pts = [tuple(0 for _ in dims_zyx), tuple(d - 1 for d in dims_zyx)]
    pts += [tuple(int(rng.integers(0, d)) for d in dims_zyx) for _ in range(200)]
    pts += [tuple((d - 1) if i == k else int(rng.integers(0, d)) for i, d in enumerate(dims_zyx))
            for k in range(len(dims_zyx)) for _ in range(8)]
    idx = [torch.tensor([p[a] for p in pts], device="cuda") for a in range(len(dims_zyx))]
    got = fout[(slice(None),) + tuple(idx)].cpu().numpy()                  # (q, npts)
    want = ref[(slice(None),) + tuple(np.array([[p[a] % block[a] for p in pts] for a in range(len(block))]))]
    err = rel(from_storage(lat, got, storage), want)
    # conservation over the whole large grid: the tiles' sum
    m_ref = float(ref.sum()) * int(np.prod(reps))
    print("\n%s %s grid %s (q*N = %d): sampled error %.2e, mass %.15e vs %.15e"
          % (lattice, storage, dims_zyx, q * nodes, err, mass, m_ref))
    assert finite
    assert err <= tol
    # The storage rounding of every population breaks exact conservation.  The
    # tiles are identical and evolve identically, so their rounding errors add
    # coherently: the drift is that of one tile (a random walk over its nodes)
    # times the number of tiles, ~2e-8 relative for FP16 deviations here
    # (measured 1.8e-8), ~1e-9 for FP32.
    gate = 1e-7 if storage == "f16dev" else 1e-8
    assert abs(mass - m_ref) <= gate * m_ref


def test_largest_grid_d3q19_f16dev():
    # 215 x 1024 x 1024 nodes, q * N = 4,283,432,960 (2^32 - 11.5e6); 2 x 8.6 GB
    _tiled_case("d3q19", (43, 64, 64), (5, 16, 16), "f16dev", "fluid", 3, 5e-3, 71)


def test_more_than_2_32_elements_d3q19_f16dev():
    # 320 x 1024 x 1024 nodes, q * N = 6,375,342,080 (1.48 x 2^32); 2 x 12.7 GB
    _tiled_case("d3q19", (32, 64, 64), (10, 16, 16), "f16dev", "fluid", 3, 5e-3, 75)


def test_largest_node_count_d2q9_f16dev():
    # 16 rows of 65535 * 4096 nodes: N = 4,294,901,760 = 2^32 - 65,536 (node
    # offsets up to 2^32 - 65,537), q * N = 3.9e10; 2 x 77.3 GB
    _tiled_case("d2q9", (4, 4096), (4, 65535), "f16dev", "fluid", 2, 5e-3, 76)


def test_longest_row_d2q9_f32():
    # one row of 240 * 2^20 = 251,658,240 nodes (the largest extent accepted is
    # 65535 * 4096), the y axis one node wide; q * N = 2.26e9; 2 x 9.1 GB
    _tiled_case("d2q9", (1, 240), (1, 2 ** 20), "f32", "fluid", 4, 3e-7 * 8, 72)


@pytest.mark.parametrize("lattice,shape", [("d2q9", (1, 1)), ("d3q19", (1, 1, 1)), ("d3q27", (1, 1, 1)),
                                           ("d2q9", (1, 7)), ("d3q19", (3, 1, 2)), ("d3q27", (1, 5, 1))])
@pytest.mark.parametrize("mode", ["zero", "fluid"])
def test_smallest_grids_fp64(lattice, shape, mode):
    lat = oracle_lattice(lattice)
    f0 = far_state(lat, shape, seed=73, amp=0.03, umax=0.1)
    n = 5
    ref = A.run(lat, f0, RATES[lat.q], n, mode={"zero": A.ZERO, "fluid": A.FLUID}[mode])
    if int(np.prod(shape)) == 1:                                           # one node: steps are collisions
        c = f0
        for _ in range(n):
            c = A.collide(lat, c, RATES[lat.q], mode={"zero": A.ZERO, "fluid": A.FLUID}[mode])
        assert np.abs(c - ref).max() <= 1e-15
    ctx = Lbmrv(lattice, RATES[lat.q], tuple(reversed(shape)), "f64")
    for streaming in ("pull", "push", "aa"):
        ctx.set_streaming(streaming)
        a = torch.from_numpy(f0).cuda()
        b = a if streaming == "aa" else torch.empty_like(a)
        ctx.step(a, b, mode, 1.0, None, n)
        torch.cuda.synchronize()
        assert rel(b.cpu().numpy(), ref) <= 1e-12, streaming


def test_zero_steps_copy_the_state_bitwise():
    lat = oracle_lattice("d3q19")
    f0 = far_state(lat, (4, 5, 6), seed=74)
    st, _ = to_storage(lat, f0, "f16dev")
    ctx = Lbmrv("d3q19", RATES[19], (6, 5, 4), "f16dev")
    for streaming in ("pull", "push", "aa"):
        ctx.set_streaming(streaming)
        a = torch.from_numpy(st).cuda()
        b = torch.full_like(a, 7.0)
        ctx.step(a, b, "fluid", 1.0, None, 0)
        torch.cuda.synchronize()
        assert torch.equal(b.cpu(), torch.from_numpy(st)), streaming
