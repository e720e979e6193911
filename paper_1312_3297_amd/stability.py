"""Linear stability of the scheme about a uniform flow, measured through the
library's own step (the question the paper leaves open in its conclusion:
in which regimes the relative velocity helps).

growth_rate() runs a power iteration: a small zero-mean random perturbation of
the uniform equilibrium f^eq(rho0, u0) on a periodic grid is advanced `chunk`
steps at a time with lbmrv_step, its distance from the uniform state is taken
with lbmrv_deviation_norm and it is rescaled to its starting size with
lbmrv_deviation_scale.  The rate per step (geometric mean of the chunk growth
factors over the last `tail` chunks) tends to the largest modulus of the
eigenvalues of the linearised step over the grid's nonzero wavenumbers: above
1 the uniform flow is linearly unstable.  Convergence is geometric in the
ratio of the two largest moduli, which can be close (e.g. 1.1613 against
1.1646), hence the default of 10^4 steps.  critical_speed() bisects on
|u0| along a direction.  Runs in FP64 storage, so that the perturbation (1e-9
per population) stays far above rounding and far below the nonlinear range.
"""
import math

import numpy as np

from .lbmrv import Lbmrv


def _uniform(ctx, rho0, u0, noise, amp):
    import torch
    shape = ctx.grid_shape
    rho = torch.full(shape, float(rho0), dtype=torch.float64, device="cuda")
    u = torch.empty((ctx.d,) + shape, dtype=torch.float64, device="cuda")
    for a in range(ctx.d):
        u[a].fill_(float(u0[a]))
    nz = None if noise is None else torch.from_numpy(noise).to("cuda")
    return ctx.init_equilibrium(rho, u, nz, amp)


def reference_state(ctx, rho0, u0):
    """The uniform equilibrium populations f^eq(rho0, u0) (q values), built by the library."""
    f = _uniform(ctx, rho0, u0, None, 0.0)
    return ctx.export_f64(f).reshape(ctx.q, -1)[:, 0].cpu().numpy()


def growth_rate(ctx, u0, mode="zero", alpha=1.0, rho0=1.0, chunk=50, chunks=200, tail=50, amp=1e-9, seed=1316):
    """Growth factor per step of a small perturbation of the uniform flow u0
    (physical units) under the context's scheme; ctx should use FP64 storage."""
    import torch
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((ctx.q,) + ctx.grid_shape)
    noise -= noise.mean(axis=tuple(range(1, noise.ndim)), keepdims=True)   # no k = 0 component
    noise /= np.sqrt((noise ** 2).sum())
    f_ref = reference_state(ctx, rho0, u0)
    f = _uniform(ctx, rho0, u0, noise, amp)
    g = torch.empty_like(f)
    n0, _ = ctx.deviation_norm2(f, f_ref)
    logs = []
    for _ in range(chunks):
        ctx.step(f, g, mode, alpha, None, chunk)
        f, g = g, f
        n, finite = ctx.deviation_norm2(f, f_ref)
        if not finite or n == 0.0:
            raise FloatingPointError("perturbation left the linear range")
        logs.append(0.5 * math.log(n / n0))
        ctx.deviation_scale(f, f_ref, math.sqrt(n0 / n))
    return math.exp(float(np.mean(logs[-tail:])) / chunk)


def critical_speed(lattice, s, direction, L, mode="zero", basis="default", alpha=1.0, threshold=1e-3, umax=0.6,
                   iters=16, **kw):
    """Largest |u0| along `direction` (bisection on [0, umax]) whose measured
    growth rate on an L^d periodic grid is at most 1 + threshold."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    dims = (L,) * (2 if lattice == "d2q9" else 3)
    ctx = Lbmrv(lattice, s, dims, "f64", basis=basis)
    lo, hi = 0.0, umax
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if growth_rate(ctx, mid * d, mode, alpha, **kw) > 1 + threshold:
            hi = mid
        else:
            lo = mid
    return lo
