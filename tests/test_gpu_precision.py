"""Accuracy of the storage forms against the FP64 oracle after 1000 steps.

Taylor-Green vortex on a 64^3 D3Q19 grid (U0 = 0.05, wavenumber 2 pi / 64,
1e-5 seeded noise), u~ = u, the 3-D rates of the workloads.  The oracle
(Oracle B, C/OpenMP FP64) starts from the FP64 state; the GPU starts from that
state rounded to its storage, so the errors include the initial rounding.
Errors are normwise relative: ||rho - rho_ref||_inf / ||rho_ref||_inf,
||u - u_ref||_inf / ||u_ref||_inf, and for each non-conserved fixed-frame moment
||m_k - m_k,ref||_inf / ||m_k,ref||_inf (the largest over k is gated).  Because
rho ~ 1 hides density errors, the density error is also measured against the
density perturbation, ||rho - rho_ref||_inf / ||rho_ref - 1||_inf.

Gates (None: measured and printed, not gated), from the arithmetic and a margin
over the measured values:
  FP64 storage        1e-9 on every field (FP64 rounding over 1000 steps);
  FP32 deviations     rho, u 1e-5 (the FP32 tolerance on rho and u at step N),
                      moments 2e-5, rho against rho - 1: 5e-5;  this is the
                      FP32 form of the benchmarks;
  FP32 storage of f itself: rho 1e-5 and moments 5e-4; u and rho against
                      rho - 1 are reported only: the store rounds |f| ~ 1/3 to
                      ~2e-8 at every step, and the momentum error random-walks
                      to 0.8-1.1e-5 of ||u|| over 1000 steps;
  FP16 deviations     rho, u 5e-3 (the tolerance stated for FP16 storage on rho
                      and u), moments 5e-2, rho against rho - 1: 5e-2.
The measured values are printed (run pytest with -s).
"""
import os

import numpy as np
import pytest

from oracle import fast
from oracle import scheme as A
from paper_1312_3297_amd import workloads
from paper_1312_3297_amd.lbmrv import Lbmrv

from _common import from_storage, oracle_lattice, to_storage

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

L, NSTEPS = 64, 1000

# (storage, gates on rho, rho against rho - 1, u, non-conserved moments)
GATES = [("f64", (1e-9, 1e-9, 1e-9, 1e-9)), ("f32dev", (1e-5, 5e-5, 1e-5, 2e-5)),
         ("f32", (1e-5, None, None, 5e-4)), ("f16dev", (5e-3, 5e-2, 5e-3, 5e-2))]


def check_gates(errors, gates):
    for name, e, g in zip(("rho", "rho of rho-1", "u", "moments"), errors, gates):
        if g is not None:
            assert e <= g, (name, e, g)


@pytest.fixture(scope="module")
def reference():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lat = oracle_lattice("d3q19")
    rho, u = workloads.taylor_green(L, 0.05)
    f0 = A.equilibrium(lat, rho, u) + 1e-5 * workloads.noise(19, (L, L, L), 1313)
    ref = fast.run(lat, f0, workloads.RATES_D3Q19, NSTEPS, mode=A.FLUID, threads=min(16, os.cpu_count() or 1))
    return lat, f0, ref


def field_errors(lat, got, ref):
    g_rho, g_u = A.conserved(lat, got)
    r_rho, r_u = A.conserved(lat, ref)
    e_rho = np.abs(g_rho - r_rho).max() / np.abs(r_rho).max()
    e_rho1 = np.abs(g_rho - r_rho).max() / np.abs(r_rho - 1).max()
    e_u = np.abs(g_u - r_u).max() / np.abs(r_u).max()
    gm, rm = A.fixed_moments(lat, got), A.fixed_moments(lat, ref)
    e_m = max(np.abs(gm[k] - rm[k]).max() / np.abs(rm[k]).max() for k in range(lat.d + 1, lat.q))
    return e_rho, e_rho1, e_u, e_m


@pytest.mark.parametrize("storage,gates", GATES)
def test_taylor_green_64_precision(reference, storage, gates):
    lat, f0, ref = reference
    st, _ = to_storage(lat, f0, storage)
    ctx = Lbmrv("d3q19", workloads.RATES_D3Q19, (L, L, L), storage)
    fin = torch.from_numpy(st).to("cuda")
    fout = torch.empty_like(fin)
    ctx.step(fin, fout, "fluid", 1.0, None, NSTEPS)
    torch.cuda.synchronize()
    got = from_storage(lat, fout.cpu().numpy(), storage)
    e_rho, e_rho1, e_u, e_m = field_errors(lat, got, ref)
    print("\nprecision %-7s after %d steps: rho %.3e (of rho-1: %.3e)  u %.3e  non-conserved moments %.3e"
          % (storage, NSTEPS, e_rho, e_rho1, e_u, e_m))
    check_gates((e_rho, e_rho1, e_u, e_m), gates)


L27 = 32


@pytest.fixture(scope="module")
def reference_d3q27():
    """D3Q27 Taylor-Green (U0 = 0.05, wavenumber 2 pi / 32, 1e-5 seeded noise)
    with u~ = 0.5 u(x, 0) held as a field, the form of the D3Q27 workload."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lat = oracle_lattice("d3q27")
    rho, u = workloads.taylor_green(L27, 0.05)
    f0 = A.equilibrium(lat, rho, u) + 1e-5 * workloads.noise(27, (L27,) * 3, 1314)
    field = (0.5 * u).astype(np.float32).astype(np.float64)
    ref = fast.run(lat, f0, workloads.RATES_D3Q27, NSTEPS, mode=A.FIELD, field=field,
                   threads=min(16, os.cpu_count() or 1))
    return lat, f0, field, ref


@pytest.mark.parametrize("storage,gates", GATES)
def test_d3q27_field_precision(reference_d3q27, storage, gates):
    """The same gates as the D3Q19 case: the storage roundings per step are the
    same, and the moment sums have at most 27 terms instead of 19."""
    lat, f0, field, ref = reference_d3q27
    st, _ = to_storage(lat, f0, storage)
    ctx = Lbmrv("d3q27", workloads.RATES_D3Q27, (L27,) * 3, storage)
    fin = torch.from_numpy(st).to("cuda")
    fout = torch.empty_like(fin)
    ctx.step(fin, fout, "field", 1.0, torch.from_numpy(field.astype(np.float32)).to("cuda"), NSTEPS)
    torch.cuda.synchronize()
    got = from_storage(lat, fout.cpu().numpy(), storage)
    e_rho, e_rho1, e_u, e_m = field_errors(lat, got, ref)
    print("\nD3Q27 field precision %-7s after %d steps: rho %.3e (of rho-1: %.3e)  u %.3e  "
          "non-conserved moments %.3e" % (storage, NSTEPS, e_rho, e_rho1, e_u, e_m))
    check_gates((e_rho, e_rho1, e_u, e_m), gates)
