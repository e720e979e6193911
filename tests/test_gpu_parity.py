"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Each test builds its input on the host, rounds it to the storage type with
NumPy, hands the same values to the GPU and (widened to FP64) to the oracle, and
compares element by element.  Tolerances:
  * FP64 storage: 1e-12 normwise relative on f and rho.  On u the gate is
    1e-11: u = q / rho is a small difference of O(1) populations, and two
    correct FP64 implementations of the same step (the oracle's LU form and the
    separately written MRT form) already disagree by 8e-12 on u after the 500
    steps of the 64 x 64 shear wave (pinned by a CPU test);
  * FP32 storage, n steps: per step the store rounds f (|f| <= 1/2) by at most
    2^-25 ~ 3e-8 and the FP32 collision adds a few ulp of |f* - f| ~ 0.05 times
    the ~30 terms of a D3Q27 moment sum, together below 1e-7 = 3e-7 ||f||_inf;
    the gate is 3e-7 * (n + 4) normwise on f;
  * FP16 deviation storage: half an ulp of a stored deviation below 1/8 is at
    most 2^-15 ~ 3.1e-5 per step, about 8e-5 of ||f||_inf ~ 0.4; the gate is
    8e-5 * (n + 1) normwise on f.
"""
import numpy as np
import pytest

from oracle import scheme as A
from paper_1312_3297_amd import workloads
from paper_1312_3297_amd.lbmrv import Lbmrv

from _common import far_state, from_storage, moment_bounds, oracle_lattice, rel, to_storage

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MODES = {"zero": A.ZERO, "fluid": A.FLUID, "field": A.FIELD}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gpu(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to(device="cuda", dtype=dtype) if dtype is not None else t.to("cuda")


def run_gpu(ctx, st, nsteps, mode="zero", alpha=1.0, field=None, streaming="pull"):
    ctx.set_streaming(streaming)
    fin = gpu(st)
    fout = torch.empty_like(fin)
    fld = gpu(field.astype(np.float32)) if field is not None else None
    ctx.step(fin, fout, mode, alpha, fld, nsteps)
    torch.cuda.synchronize()
    return fout.cpu().numpy()


def f_tol(storage, n):
    return {"f64": 1e-12, "f32": 3e-7 * (n + 4), "f32dev": 3e-7 * (n + 4), "f16dev": 8e-5 * (n + 1)}[storage]


# ---------------------------------------------------------------------------
# the 64 x 64 FP64 shear-wave case, 500 steps
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("basis,mode,rates", [
    ("default", "zero", workloads.RATES_D2Q9_GROUPED),
    ("default", "fluid", workloads.RATES_D2Q9_GROUPED),
    ("geier", "fluid", workloads.RATES_D2Q9_GROUPED),
    ("default", "fluid", workloads.RATES_D2Q9_LITERAL),
])
def test_d2q9_shear_wave_64_fp64_500_steps(basis, mode, rates):
    lat = oracle_lattice("d2q9", basis)
    rho, u = workloads.shear_wave(64, 0.01)
    f0 = A.equilibrium(lat, rho, u) + 1e-4 * workloads.noise(9, (64, 64), 1312)
    ref = A.run(lat, f0, rates, 500, mode=MODES[mode])
    ctx = Lbmrv("d2q9", rates, (64, 64), "f64", basis)
    got = run_gpu(ctx, f0, 500, mode)
    assert rel(got, ref) <= 1e-12
    r_rho, r_u = A.conserved(lat, ref)
    g_rho, g_u = A.conserved(lat, got)
    assert rel(g_rho, r_rho) <= 1e-12
    # rho - 1 is ~1e-5 here, so the FP64 rounding of rho ~ 1 alone is ~1e-11 of it
    assert rel(g_rho - 1, r_rho - 1) <= 1e-9
    assert rel(g_u, r_u) <= 1e-11


# ---------------------------------------------------------------------------
# ragged 3-D grids: several blocks along x with a partial last one
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lattice,storage,mode,nsteps", [
    ("d3q19", "f64", "fluid", 8),
    ("d3q19", "f64", "field", 8),
    ("d3q19", "f64", "zero", 8),
    ("d3q19", "f32", "fluid", 12),
    ("d3q19", "f32dev", "fluid", 12),
    ("d3q19", "f16dev", "fluid", 6),
    ("d3q27", "f64", "field", 6),
    ("d3q27", "f64", "fluid", 6),
    ("d3q27", "f32", "field", 6),
])
def test_3d_ragged_grid(lattice, storage, mode, nsteps):
    lat = oracle_lattice(lattice)
    shape = (5, 7, 300)                                 # (nz, ny, nx): 256 + 44 along x
    f0 = far_state(lat, shape, seed=21, amp=0.02, umax=0.08)
    st, f0w = to_storage(lat, f0, storage)
    field = np.random.default_rng(22).uniform(-0.1, 0.1, (3,) + shape).astype(np.float32).astype(np.float64)
    rates = workloads.RATES_D3Q19 if lattice == "d3q19" else workloads.RATES_D3Q27
    ref = A.run(lat, f0w, rates, nsteps, mode=MODES[mode], alpha=0.8, field=field)
    ctx = Lbmrv(lattice, rates, (300, 7, 5), storage)
    got = from_storage(lat, run_gpu(ctx, st, nsteps, mode, 0.8, field), storage)
    assert rel(got, ref) <= f_tol(storage, nsteps)


@pytest.mark.parametrize("lattice,basis", [("d2q9", "default"), ("d2q9", "geier"), ("d3q19", "default"),
                                           ("d3q27", "default")])
@pytest.mark.parametrize("nsteps", [3, 4])
def test_push_and_pull_agree_bitwise(lattice, basis, nsteps):
    lat = oracle_lattice(lattice, basis)
    shape = (33, 70) if lat.d == 2 else (4, 6, 33)
    f0 = far_state(lat, shape, seed=5)
    st, _ = to_storage(lat, f0, "f32")
    dims = tuple(reversed(shape))
    rates = {9: workloads.RATES_D2Q9_GROUPED, 19: workloads.RATES_D3Q19, 27: workloads.RATES_D3Q27}[lat.q]
    ctx = Lbmrv(lattice, rates, dims, "f32", basis)
    a = run_gpu(ctx, st, nsteps, "fluid", streaming="pull")
    b = run_gpu(ctx, st, nsteps, "fluid", streaming="push")
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# single relaxation far from equilibrium with a large relative velocity: the
# u~-dependent part of the collision is O(1e-2) here, so a wrong shift fails
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lattice,basis", [("d2q9", "default"), ("d2q9", "geier"), ("d3q19", "default"),
                                           ("d3q27", "default")])
@pytest.mark.parametrize("lam", [1.0, 1.7])
def test_collision_far_from_equilibrium_fp64(lattice, basis, lam):
    lat = oracle_lattice(lattice, basis)
    shape = (9, 11) if lat.d == 2 else (3, 5, 7)
    rng = np.random.default_rng(31)
    f0 = far_state(lat, shape, seed=32, amp=0.1, umax=0.2)
    rates = np.concatenate([np.zeros(lat.d + 1), rng.uniform(0.5, 1.95, lat.q - lat.d - 1)])
    field = (lam * rng.uniform(-0.3, 0.3, (lat.d,) + shape)).astype(np.float32).astype(np.float64)
    ctx = Lbmrv(lattice, rates, tuple(reversed(shape)), "f64", basis, lam=lam)
    fin = gpu(f0)
    for mode, alpha in (("zero", 1.0), ("fluid", 1.0), ("fluid", -0.7), ("field", 1.0)):
        fout = torch.empty_like(fin)
        ctx.collide(fin, fout, mode, alpha, gpu(field.astype(np.float32)))
        torch.cuda.synchronize()
        ref = A.collide(lat, f0, rates, lam, MODES[mode], alpha, field)
        assert rel(fout.cpu().numpy() - f0, ref - f0) <= 1e-12, mode
        if mode != "zero":
            zero = A.collide(lat, f0, rates, lam, A.ZERO)
            assert rel(ref - f0, zero - f0) > 1e-3          # the shift matters here


def test_in_place_collision_matches_out_of_place():
    lat = oracle_lattice("d3q19")
    f0 = far_state(lat, (4, 5, 6), seed=3)
    ctx = Lbmrv("d3q19", workloads.RATES_D3Q19, (6, 5, 4), "f32")
    st, _ = to_storage(lat, f0, "f32")
    a = gpu(st)
    b = torch.empty_like(a)
    ctx.collide(a, b, "fluid")
    ctx.collide(a, a, "fluid")
    torch.cuda.synchronize()
    assert torch.equal(a, b)


# ---------------------------------------------------------------------------
# transport
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lattice,shape", [("d2q9", (12, 12)), ("d3q19", (6, 6, 6)), ("d3q27", (5, 5, 5))])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev"])
def test_zero_rates_stream_period_is_identity_bitwise(lattice, shape, storage):
    """All s = 0: the collision is the identity, so L steps on an L-periodic grid
    return the input bit for bit (eq. (transport))."""
    lat = oracle_lattice(lattice)
    f0 = far_state(lat, shape, seed=8)
    st, _ = to_storage(lat, f0, storage)
    ctx = Lbmrv(lattice, np.zeros(lat.q), tuple(reversed(shape)), storage)
    for streaming in ("pull", "push"):
        got = run_gpu(ctx, st, shape[0], "fluid", streaming=streaming)
        assert np.array_equal(got, st), streaming


@pytest.mark.parametrize("lattice", ["d2q9", "d3q19", "d3q27"])
def test_transport_matches_oracle_bitwise(lattice):
    lat = oracle_lattice(lattice)
    shape = (7, 300) if lat.d == 2 else (3, 4, 300)
    f0 = np.random.default_rng(2).standard_normal((lat.q,) + shape)
    ctx = Lbmrv(lattice, np.zeros(lat.q), tuple(reversed(shape)), "f64")
    a = gpu(f0)
    b = torch.empty_like(a)
    ctx.transport(a, b)
    torch.cuda.synchronize()
    assert np.array_equal(b.cpu().numpy(), A.stream(lat, f0))


# ---------------------------------------------------------------------------
# moments, conservation, initial state, storage conversion
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lattice,basis", [("d2q9", "default"), ("d2q9", "geier"), ("d3q19", "default"),
                                           ("d3q27", "default")])
@pytest.mark.parametrize("lam", [1.0, 0.6])
def test_moments_fp64(lattice, basis, lam):
    lat = oracle_lattice(lattice, basis)
    shape = (10, 13) if lat.d == 2 else (3, 4, 5)
    f0 = far_state(lat, shape, seed=4)
    ctx = Lbmrv(lattice, np.zeros(lat.q), tuple(reversed(shape)), "f64", basis, lam=lam)
    rho, u, m0 = ctx.moments(gpu(f0), with_m0=True)
    torch.cuda.synchronize()
    r_rho, r_u = A.conserved(lat, f0, lam)
    assert rel(rho.cpu().numpy(), r_rho) <= 1e-15
    assert rel(u.cpu().numpy(), r_u) <= 1e-14
    assert rel(m0.cpu().numpy(), A.fixed_moments(lat, f0, lam)) <= 1e-14


@pytest.mark.parametrize("lattice,basis", [("d2q9", "default"), ("d2q9", "geier"), ("d3q19", "default"),
                                           ("d3q27", "default")])
@pytest.mark.parametrize("storage", ["f32", "f32dev", "f16dev"])
@pytest.mark.parametrize("lam", [1.0, 0.6])
def test_moments_reduced_storage(lattice, basis, storage, lam):
    """lbmrv_moments in the FP32 storages (FP32 arithmetic and output) against
    eq. (rhoq) and m(0) = M(0) f (eq. (matort) for the D2Q9 paper basis) of the
    widened stored state, element by element within the FP32 rounding bound;
    the deviation storages add the rest moments of w_j rho0 back in."""
    lat = oracle_lattice(lattice, basis)
    shape = (10, 13) if lat.d == 2 else (3, 4, 5)
    f0 = far_state(lat, shape, seed=5)
    st, fw = to_storage(lat, f0, storage)
    ctx = Lbmrv(lattice, np.zeros(lat.q), tuple(reversed(shape)), storage, basis, lam=lam)
    rho, u, m0 = ctx.moments(gpu(st), with_m0=True)
    torch.cuda.synchronize()
    assert rho.dtype == torch.float32 and m0.dtype == torch.float32
    r_rho, r_u = A.conserved(lat, fw, lam)
    r_m = A.fixed_moments(lat, fw, lam)
    t_rho, t_u, t_m = moment_bounds(lat, fw, lam)
    assert np.all(np.abs(rho.cpu().numpy() - r_rho) <= t_rho)
    assert np.all(np.abs(u.cpu().numpy() - r_u) <= t_u)
    assert np.all(np.abs(m0.cpu().numpy() - r_m) <= t_m)
    # and the bound is not vacuous: relative to each field's norm it is small
    assert (t_u / np.abs(r_u).max()).max() <= 2e-4


@pytest.mark.parametrize("storage", ["f64", "f32", "f32dev", "f16dev"])
def test_conservation_reduction(storage):
    lat = oracle_lattice("d3q19")
    shape = (6, 10, 257)
    f0 = far_state(lat, shape, seed=6)
    st, f0w = to_storage(lat, f0, storage)
    ctx = Lbmrv("d3q19", workloads.RATES_D3Q19, tuple(reversed(shape)), storage, lam=1.3)
    mass, mom, finite = ctx.conservation(gpu(st))
    assert finite
    rho, u = A.conserved(lat, f0w, 1.3)
    assert abs(mass - rho.sum()) <= 1e-12 * rho.sum()
    for a in range(3):
        assert abs(mom[a] - (rho * u[a]).sum()) <= 1e-11 * np.abs(rho * u[a]).sum()


def test_conservation_reports_nonfinite():
    lat = oracle_lattice("d2q9")
    f0 = far_state(lat, (8, 8), seed=1)
    f0[3, 2, 5] = np.nan
    ctx = Lbmrv("d2q9", workloads.RATES_D2Q9_GROUPED, (8, 8), "f32")
    _, _, finite = ctx.conservation(gpu(f0.astype(np.float32)))
    assert not finite


def test_mass_momentum_conserved_over_many_steps_fp64():
    lat = oracle_lattice("d3q19")
    shape = (16, 16, 16)
    rho, u = workloads.taylor_green(16, 0.05)
    f0 = A.equilibrium(lat, rho, u) + 1e-5 * workloads.noise(19, shape, 77)
    ctx = Lbmrv("d3q19", workloads.RATES_D3Q19, tuple(reversed(shape)), "f64")
    m0, p0, _ = ctx.conservation(gpu(f0))
    got = run_gpu(ctx, f0, 200, "fluid")
    m1, p1, ok = ctx.conservation(gpu(got))
    assert ok and abs(m1 - m0) <= 1e-12 * m0
    assert max(abs(a - b) for a, b in zip(p0, p1)) <= 1e-12 * m0


@pytest.mark.parametrize("lattice", ["d2q9", "d3q19", "d3q27"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f32dev", "f16dev"])
def test_init_equilibrium_and_conversion(lattice, storage):
    lat = oracle_lattice(lattice)
    shape = (11, 17) if lat.d == 2 else (3, 5, 9)
    rng = np.random.default_rng(9)
    rho = 1 + 0.02 * rng.standard_normal(shape)
    u = 0.05 * rng.uniform(-1, 1, (lat.d,) + shape)
    noise = rng.uniform(-1, 1, (lat.q,) + shape)
    lam = 1.25
    ctx = Lbmrv(lattice, np.zeros(lat.q), tuple(reversed(shape)), storage, lam=lam, rho0=1.0)
    st = ctx.init_equilibrium(gpu(rho), gpu(u), gpu(noise), 1e-4)
    back = ctx.export_f64(st)
    torch.cuda.synchronize()
    ref = A.equilibrium(lat, rho, u, lam) + 1e-4 * noise
    tol = {"f64": 1e-15, "f32": 1e-7, "f32dev": 2e-8, "f16dev": 2e-4}[storage]
    assert rel(back.cpu().numpy(), ref) <= tol
    # import: bitwise equal to NumPy's round-to-nearest-even of f - w rho0
    host_st, _ = to_storage(lat, ref, storage)
    imp = ctx.import_f64(gpu(ref))
    torch.cuda.synchronize()
    assert np.array_equal(imp.cpu().numpy(), host_st)


@pytest.mark.parametrize("lattice", ["d2q9", "d3q19", "d3q27"])
@pytest.mark.parametrize("mode", ["zero", "fluid"])
def test_fp16_subnormal_deviations(lattice, mode):
    """A rest state (f = w_j, rho0 = 1) plus perturbations of ~1e-6, so every
    stored deviation lies in the binary16 subnormal range (below 2^-14 ~ 6.1e-5,
    spacing 2^-24 ~ 6e-8).  The import is bitwise NumPy's round-to-nearest-even;
    after a step the stored deviations are still nonzero subnormals (nothing is
    flushed to zero), and each equals the oracle's deviation after the step,
    computed in FP64 from the widened state, to within half a subnormal spacing
    (the FP32 collision errs by ~1e-13 on values of ~1e-6)."""
    lat = oracle_lattice(lattice)
    shape = (7, 9) if lat.d == 2 else (3, 4, 5)
    rng = np.random.default_rng(10)
    w = lat.w.reshape((-1,) + (1,) * lat.d)
    f0 = w * np.ones((lat.q,) + shape) + 1e-6 * rng.uniform(-1, 1, (lat.q,) + shape)
    ctx = Lbmrv(lattice, ctx_rates(lat), tuple(reversed(shape)), "f16dev")
    host_st, fw = to_storage(lat, f0, "f16dev")
    sub = np.abs(host_st.astype(np.float64))
    assert sub.max() < 2.0 ** -14 and np.count_nonzero(sub) > 0.9 * sub.size
    imp = ctx.import_f64(gpu(f0))
    torch.cuda.synchronize()
    assert np.array_equal(imp.cpu().numpy().view(np.uint16), host_st.view(np.uint16))
    out = torch.empty_like(imp)
    ctx.step(imp, out, mode, 1.0, None, 1)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    dev = np.abs(got.astype(np.float64))
    assert dev.max() < 2.0 ** -14
    assert np.count_nonzero(dev) > 0.8 * dev.size
    ref_dev = A.step(lat, fw, ctx_rates(lat), mode=MODES[mode]) - w
    assert np.abs(got.astype(np.float64) - ref_dev).max() <= 2.0 ** -25 * 1.01


def test_fp16_subnormal_deviations_in_place_node_pairs():
    """The same subnormal rest state on D3Q19 with an even nx, in place: the
    even step runs on node pairs (two 2-byte halves per word), and after two
    and three steps the state still holds nonzero subnormals and equals the
    pull form's bits."""
    lat = oracle_lattice("d3q19")
    shape = (3, 4, 6)
    rng = np.random.default_rng(11)
    w = lat.w.reshape((-1,) + (1,) * lat.d)
    f0 = w * np.ones((lat.q,) + shape) + 1e-6 * rng.uniform(-1, 1, (lat.q,) + shape)
    ctx = Lbmrv("d3q19", ctx_rates(lat), tuple(reversed(shape)), "f16dev")
    for nsteps in (2, 3):
        ctx.set_streaming("pull")
        a = ctx.import_f64(gpu(f0))
        ref = torch.empty_like(a)
        ctx.step(a, ref, "fluid", 1.0, None, nsteps)
        ctx.set_streaming("aa")
        one = ctx.import_f64(gpu(f0))
        ctx.step(one, one, "fluid", 1.0, None, nsteps)
        torch.cuda.synchronize()
        got = one.cpu().numpy().astype(np.float64)
        assert np.abs(got).max() < 2.0 ** -14 and np.count_nonzero(got) > 0.8 * got.size
        assert torch.equal(one, ref), nsteps


def ctx_rates(lat):
    return {9: workloads.RATES_D2Q9_GROUPED, 19: workloads.RATES_D3Q19, 27: workloads.RATES_D3Q27}[lat.q]


# ---------------------------------------------------------------------------
# the velocity scale lambda
# ---------------------------------------------------------------------------
def test_lambda_scale_fp64():
    lat = oracle_lattice("d2q9")
    lam = 1.7
    shape = (20, 23)
    rng = np.random.default_rng(41)
    rho = 1 + 0.01 * rng.standard_normal(shape)
    u = lam * 0.05 * rng.uniform(-1, 1, (2,) + shape)
    f0 = A.equilibrium(lat, rho, u, lam) * (1 + 0.02 * rng.uniform(-1, 1, (9,) + shape))
    field = (lam * rng.uniform(-0.2, 0.2, (2,) + shape)).astype(np.float32).astype(np.float64)
    ref = A.run(lat, f0, workloads.RATES_D2Q9_GROUPED, 10, lam, A.FIELD, field=field)
    ctx = Lbmrv("d2q9", workloads.RATES_D2Q9_GROUPED, (23, 20), "f64", lam=lam)
    got = run_gpu(ctx, f0, 10, "field", field=field)
    assert rel(got, ref) <= 1e-12


@pytest.mark.parametrize("nsteps", [1, 7])
def test_geier_basis_with_u_equals_appendix_b_cascaded_step(nsteps):
    """Prop. th:cascd2q9 on the GPU: the Geier basis with u~ = u reproduces the
    g-vector cascaded step of Appendix B (Oracle D, written separately from
    Oracle A), far from equilibrium, over a ragged 70 x 13 grid."""
    from oracle import geier
    lat = oracle_lattice("d2q9", "geier")
    shape = (13, 70)
    f0 = far_state(lat, shape, seed=31, amp=0.05, umax=0.15)
    s = [0, 0, 0, 1.1, 1.8, 1.6, 1.25, 1.35, 1.5]
    ref = f0.copy()
    for _ in range(nsteps):
        ref = geier.geier_step(ref, s)
    ctx = Lbmrv("d2q9", s, tuple(reversed(shape)), "f64", "geier")
    got = run_gpu(ctx, f0, nsteps, "fluid", 1.0)
    assert rel(got, ref) <= 1e-12
    # the same state under the fixed-frame (MRT) relaxation is far from it
    mrt = run_gpu(ctx, f0, nsteps, "zero")
    assert rel(mrt, ref) > 1e-5
