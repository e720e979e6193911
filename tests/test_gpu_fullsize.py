"""Parity at the benchmark's full sizes, in the launch configurations it times.

The whole grid runs on the GPU for n steps from a host-built initial state;
the oracle then recomputes sampled output nodes one by one: the value of a node
after n steps depends only on the (2n+1)^d block around it, so the oracle runs
n steps on that block (periodic on the block; the wrapped values never reach the
centre within n steps) and the centre is compared.  Samples include the domain
faces and corners, where the periodic wrap of the GPU kernel is exercised.
"""
import numpy as np
import pytest

from oracle import scheme as A
from paper_1312_3297_amd import workloads
from paper_1312_3297_amd.lbmrv import Lbmrv

from _common import from_storage, oracle_lattice, rel, to_storage

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NSTEPS = 3


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _samples(shape, rng, n=120):
    pts = [tuple(0 for _ in shape), tuple(s - 1 for s in shape)]
    pts += [tuple(rng.integers(0, s) for s in shape) for _ in range(n)]
    pts += [tuple((s - 1) if i == k else int(rng.integers(0, s)) for i, s in enumerate(shape))
            for k in range(len(shape)) for _ in range(4)]
    return pts


def _block(arr, centre, R):
    """Periodic (2R+1)^d block of arr[..., grid] around centre (grid axes last)."""
    idx = [np.arange(c - R, c + R + 1) % s for c, s in zip(centre, arr.shape[-len(centre):])]
    return arr[(Ellipsis,) + np.ix_(*idx)]


def _check(lattice, shape, storage, mode, streaming, rates, rho, u, noise_amp, seed, field=None, tol=None):
    lat = oracle_lattice(lattice)
    f0 = A.equilibrium(lat, rho, u)
    if noise_amp:
        f0 += noise_amp * workloads.noise(lat.q, shape, seed)
    st, f0w = to_storage(lat, f0, storage)
    del f0
    ctx = Lbmrv(lattice, rates, tuple(reversed(shape)), storage)
    ctx.set_streaming(streaming)
    fin = torch.from_numpy(st).to("cuda")
    fout = fin if streaming == "aa" else torch.empty_like(fin)   # the in-place form runs on one array
    fld = None if field is None else torch.from_numpy(field.astype(np.float32)).to("cuda")
    ctx.step(fin, fout, mode, 1.0, fld, NSTEPS)
    torch.cuda.synchronize()
    got = fout.cpu().numpy()
    del fin, fout
    rng = np.random.default_rng(seed + 1)
    R = NSTEPS
    pts = _samples(shape, rng)
    blocks = np.stack([_block(f0w, p, R) for p in pts], axis=1)               # (q, P, b, b[, b])
    fblk = None
    if field is not None:
        fw = field.astype(np.float32).astype(np.float64)
        fblk = np.stack([_block(fw, p, R) for p in pts], axis=1)
    smode = {"zero": A.ZERO, "fluid": A.FLUID, "field": A.FIELD}[mode]
    ref_all = []
    for i in range(len(pts)):                     # oracle, one block at a time
        fb = blocks[:, i]
        out = A.run(lat, fb, rates, NSTEPS, mode=smode, field=None if fblk is None else fblk[:, i])
        ref_all.append(out[(slice(None),) + (R,) * lat.d])
    ref = np.stack(ref_all, axis=1)
    gv = from_storage(lat, np.stack([got[(slice(None),) + p] for p in pts], axis=1), storage)
    tol = tol if tol is not None else {"f64": 1e-12, "f32": 3e-7 * (NSTEPS + 4), "f32dev": 3e-7 * (NSTEPS + 4),
                                       "f16dev": 8e-5 * (NSTEPS + 1)}[storage]
    assert rel(gv, ref) <= tol


# every benchmark workload in the pull form it times (two-row blocks for D3Q27
# FP32, one-row blocks and 5 wavefronts per SIMD for D3Q27 FP16, per-XCD block
# order for D2Q9 2048^2), and the push and in-place forms of the headline
@pytest.mark.parametrize("streaming", ["pull", "push", "aa"])
def test_d3q19_taylor_green_256_f32_fluid(streaming):
    rho, u = workloads.taylor_green(256, 0.05)
    _check("d3q19", (256, 256, 256), "f32", "fluid", streaming, workloads.RATES_D3Q19, rho, u, 1e-5, 1313)


@pytest.mark.parametrize("storage", ["f16dev", "f64", "f32dev"])
def test_d3q19_taylor_green_256_other_storages_fluid(storage):
    rho, u = workloads.taylor_green(256, 0.05)
    _check("d3q19", (256, 256, 256), storage, "fluid", "pull", workloads.RATES_D3Q19, rho, u, 1e-5, 1313)


def test_d3q19_taylor_green_slab_f32dev_fluid():
    """One GPU's share of the headline case in eight z-slabs (256 x 256 x 32),
    in place, in the launch shape the benchmark times."""
    rho, u = workloads.taylor_green(256, 0.05, shape=(32, 256, 256))
    _check("d3q19", (32, 256, 256), "f32dev", "fluid", "aa", workloads.RATES_D3Q19, rho, u, 1e-5, 1313)


@pytest.mark.parametrize("storage", ["f32", "f16dev"])
def test_d3q27_taylor_green_192_field(storage):
    rho, u = workloads.taylor_green(192, 0.05)
    _check("d3q27", (192, 192, 192), storage, "field", "pull", workloads.RATES_D3Q27, rho, u, 1e-5, 1314,
           field=0.5 * u)


@pytest.mark.parametrize("L", [2048, 4096])
def test_d2q9_double_shear_layer_f32_fluid(L):
    rho, u = workloads.double_shear_layer(L)
    _check("d2q9", (L, L), "f32", "fluid", "pull", workloads.RATES_D2Q9_SHEAR_LAYER, rho, u, 0.0, 7)


# D3Q19 512^3 FP32 (Taylor-Green without noise; 2 x 10.2 GB of state in the
# pull form): rows of 512 nodes span two blocks, and both timed forms run
# one-row blocks, four per CU.  As in the benchmark, the GPU forms f^eq(rho, u)
# itself (lbmrv_init_equilibrium, FP64 then rounded to FP32); the oracle forms
# it on the host from the same rho and u over each sampled block, so a stored
# value may differ by one FP32 rounding between the two starts.
@pytest.mark.parametrize("streaming", ["pull", "aa"])
def test_d3q19_taylor_green_512_f32_fluid(streaming):
    lat = oracle_lattice("d3q19")
    L = 512
    shape = (L, L, L)
    rho, u = workloads.taylor_green(L, 0.05)
    ctx = Lbmrv("d3q19", workloads.RATES_D3Q19, shape, "f32")
    ctx.set_streaming(streaming)
    fin = ctx.init_equilibrium(torch.from_numpy(rho).to("cuda"), torch.from_numpy(u).to("cuda"), None, 0.0)
    fout = fin if streaming == "aa" else torch.empty_like(fin)
    ctx.step(fin, fout, "fluid", 1.0, None, NSTEPS)
    pts = _samples(shape, np.random.default_rng(512))
    idx = tuple(torch.tensor([p[a] for p in pts], device="cuda") for a in range(3))
    gv = fout[(slice(None),) + idx].double().cpu().numpy()                  # (q, P)
    del fin, fout
    torch.cuda.synchronize()
    R = NSTEPS
    ref = []
    for p in pts:
        f0 = to_storage(lat, A.equilibrium(lat, _block(rho, p, R), _block(u, p, R)), "f32")[1]
        ref.append(A.run(lat, f0, workloads.RATES_D3Q19, NSTEPS, mode=A.FLUID)[(slice(None),) + (R,) * 3])
    assert rel(gv, np.stack(ref, axis=1)) <= 3e-7 * (NSTEPS + 4)
