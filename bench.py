"""Throughput of the relative-velocity lattice Boltzmann step on one MI355X.

Default workload: D3Q19, 256^3 periodic, populations stored in FP32 as
deviations f - w_j rho0 (FP32 arithmetic), Taylor-Green vortex (U0 = 0.05) plus
1e-5 seeded noise, u~ = local fluid velocity (cascaded choice), rates bulk 1.1 /
shear 1.95 / third order 1.5 / fourth order 1.2, streamed in place (one array,
one fused pass per step).

A "step" is one full time step of the scheme (relaxation in the moving frame,
then transport) over every node.  K steps are timed as one lbmrv_step call on
the current stream, bracketed by a device synchronisation; inputs are resident
in HBM before the timed region.  Prints one JSON line.  roofline.achieved is
the algorithmic bytes of one step (2 q b per node, plus the u~ field when it is
read) over the measured time per step; roofline.per_launch gives the same per
kernel launch (they differ only when a call adds boundary passes: the pull
form's first collision and last transport, the in-place form's final swap
after an odd step count).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % of HBM roofline (D3Q19 FP32 256³); adjoint cost ratio vs fwd"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the fused collide-stream kernel (GB), from rocprofv3
# FETCH_SIZE and WRITE_SIZE counters scaled by what the same counters read for
# a plain copy of known size (FETCH x 2.0, WRITE x 1.0); see profiles/.  Only
# valid for the kernel version the counters were taken on, in the default
# (automatic) block order; the in-place form averages its two kernels.
TRAFFIC_GB = {
    ("d2q9_shear2048_f32_fluid", "aa"): 0.3021,
    ("d2q9_shear4096_f32_fluid", "aa"): 1.2395,
    ("d3q19_couette256_f32_fluid_walls", "aa"): 2.5503,
    ("d3q19_tgv256_f16dev_fluid", "aa"): 1.2752,
    ("d3q19_tgv256_f32_fluid", "aa"): 2.5502,
    ("d3q19_tgv256_f32dev_fluid", "aa"): 2.5502,
    ("d3q19_tgv256_slab32_f32dev_fluid", "aa"): 0.3189,
    ("d3q19_tgv256_f64_fluid", "aa"): 5.1021,
    ("d3q19_tgv512_f32_fluid", "aa"): 20.8212,
    ("d3q27_tgv192_f16dev_field", "aa"): 0.8495,
    ("d3q27_tgv192_f32_field", "aa"): 1.6143,
    ("d2q9_shear2048_f32_fluid", "pull"): 0.3021,
    ("d2q9_shear4096_f32_fluid", "pull"): 1.2207,
    ("d3q19_couette256_f32_fluid_walls", "pull"): 2.5533,
    ("d3q19_tgv256_f16dev_fluid", "pull"): 1.2752,
    ("d3q19_tgv256_f32_fluid", "pull"): 2.5508,
    ("d3q19_tgv256_f32_fluid", "push"): 2.551,
    ("d3q19_tgv256_f32_fluid_rawbasis", "pull"): 2.5512,
    ("d3q19_tgv256_f32dev_fluid", "pull"): 2.5508,
    ("d3q19_tgv256_f64_fluid", "pull"): 5.1006,
    ("d3q19_tgv512_f32_fluid", "pull"): 21.0724,
    ("d3q27_tgv192_f16dev_field", "pull"): 0.8731,
    ("d3q27_tgv192_f32_field", "pull"): 1.6595,
}

WORKLOADS = {
    # name: (lattice, dims, storage, mode, alpha, builder)
    "d3q19_tgv256_f32_fluid": ("d3q19", (256, 256, 256), "f32", "fluid"),
    "d3q19_tgv256_f16dev_fluid": ("d3q19", (256, 256, 256), "f16dev", "fluid"),
    "d3q27_tgv192_f32_field": ("d3q27", (192, 192, 192), "f32", "field"),
    "d2q9_shear2048_f32_fluid": ("d2q9", (2048, 2048), "f32", "fluid"),
    "d2q9_shear4096_f32_fluid": ("d2q9", (4096, 4096), "f32", "fluid"),
    # channel between two half-way bounce-back walls (y faces), the upper one
    # moving along x; Taylor-Green start as in the headline workload
    "d3q19_couette256_f32_fluid_walls": ("d3q19", (256, 256, 256), "f32", "fluid"),
    "d3q19_tgv256_f64_fluid": ("d3q19", (256, 256, 256), "f64", "fluid"),
    "d3q19_tgv256_f32dev_fluid": ("d3q19", (256, 256, 256), "f32dev", "fluid"),
    # one GPU's share of the headline case split into eight z-slabs: the first
    # 32 planes of the same Taylor-Green state (periodic in z here; a sharded
    # run would exchange the face populations instead)
    "d3q19_tgv256_slab32_f32dev_fluid": ("d3q19", (256, 256, 32), "f32dev", "fluid"),
    # the headline case at 512^3 (2 x 10.2 GB of state), to show the rate holds
    # for a state 8x larger; no seeded noise (it would be 20 GB on the host)
    "d3q19_tgv512_f32_fluid": ("d3q19", (512, 512, 512), "f32", "fluid"),
    "d3q27_tgv192_f16dev_field": ("d3q27", (192, 192, 192), "f16dev", "field"),
    # run-time moment basis (raw second moments, three normal-stress rates):
    # the relaxation goes through a dense R^{-1} S R instead of compiled tables
    "d3q19_tgv256_f32_fluid_rawbasis": ("d3q19", (256, 256, 256), "f32", "fluid"),
}
WALLS = {"d3q19_couette256_f32_fluid_walls": ((1 << 2) | (1 << 3), 0.05)}
RUNTIME_BASIS = {"d3q19_tgv256_f32_fluid_rawbasis": ("RAW2_D3Q19", "RATES_RAW2_D3Q19")}


def build_state(name, ctx, torch):
    """Seeded initial populations in HBM (built by the library from rho, u, noise)."""
    from paper_1312_3297_amd import workloads as W
    lattice, dims, storage, mode = WORKLOADS[name]
    if lattice == "d3q19":
        rho, u = W.taylor_green(dims[0], 0.05, shape=tuple(reversed(dims)))
        noise, amp, seed = dims[0] <= 256, 1e-5, 1313
    elif lattice == "d3q27":
        rho, u = W.taylor_green(dims[0], 0.05)
        noise, amp, seed = True, 1e-5, 1314
    else:
        rho, u = W.double_shear_layer(dims[0])
        noise, amp, seed = False, 0.0, 0
    d_rho = torch.from_numpy(rho).to("cuda")
    d_u = torch.from_numpy(u).to("cuda")
    d_noise = torch.from_numpy(W.noise(ctx.q, rho.shape, seed)).to("cuda") if noise else None
    f = ctx.init_equilibrium(d_rho, d_u, d_noise, amp)
    field = None
    if mode == "field":
        # prescribed relative velocity: half the initial fluid velocity, frozen
        field = (0.5 * d_u).to(torch.float32).contiguous()
    del d_rho, d_noise
    torch.cuda.synchronize()
    return f, field


def rates_for(lattice):
    from paper_1312_3297_amd import workloads as W
    return {"d2q9": W.RATES_D2Q9_SHEAR_LAYER, "d3q19": W.RATES_D3Q19, "d3q27": W.RATES_D3Q27}[lattice]


def cpu_baseline(name, budget_s=15.0):
    """The FP64 oracle (Oracle B: plain C, OpenMP over nodes, per-node Gaussian
    elimination) on a bounded sample of the workload: a sub-block of the same
    initial state, stepped (periodically) for about budget_s seconds."""
    from oracle import fast, lattices, scheme
    from paper_1312_3297_amd import workloads as W
    lattice, dims, storage, mode = WORKLOADS[name]
    lat = lattices.make({"d2q9": "d2q9_paper"}.get(lattice, lattice))
    s = rates_for(lattice)
    if name in RUNTIME_BASIS:
        basis, rates = (getattr(W, x) for x in RUNTIME_BASIS[name])
        lat, s = lattices.with_basis(lattice, basis), rates
    if lat.d == 3:
        sub = (32, 32, 32)
        rho, u = W.taylor_green(dims[0], 0.05, shape=sub)
    else:
        sub = (128, 256)
        rho, u = W.double_shear_layer(dims[0])
        rho, u = rho[: sub[0], : sub[1]], u[:, : sub[0], : sub[1]]
    f = scheme.equilibrium(lat, rho, u)
    smode = {"zero": scheme.ZERO, "fluid": scheme.FLUID, "field": scheme.FIELD}[mode]
    field = 0.5 * u if mode == "field" else None
    nodes = int(np.prod(sub))

    def timed(fn, f, budget):
        """Steps fn(f, n) in growing chunks for about `budget` seconds; (steps, seconds)."""
        t0 = time.perf_counter()
        steps, chunk = 0, 1
        while True:
            f = fn(f, chunk)
            steps += chunk
            el = time.perf_counter() - t0
            if el >= budget:
                return steps, el
            chunk = max(1, min(64, int(steps * (budget - el) / el / 4)))

    threads = min(16, os.cpu_count() or 1)
    steps, el = timed(lambda g, n: fast.run(lat, g, s, n, 1.0, smode, 1.0, field, threads=threads), f, budget_s)
    # the same on one core; the triangular-solve form of the same oracle (the
    # one that wrote the stored full-size references) on all cores; and
    # Oracle A (NumPy) on the 64^2 D2Q9 shear wave
    steps1, el1 = timed(lambda g, n: fast.run(lat, g, s, n, 1.0, smode, 1.0, field, threads=1), f, budget_s / 3)
    steps_t, el_t = timed(lambda g, n: fast.run_tri(lat, g, s, n, 1.0, smode, 1.0, field, threads=threads), f,
                          budget_s / 3)
    lat_a = lattices.make("d2q9_paper")
    rho_a, u_a = W.shear_wave(64, 0.01)
    steps_a, el_a = timed(lambda g, n: scheme.run(lat_a, g, W.RATES_D2Q9_GROUPED, n, mode=scheme.FLUID),
                          scheme.equilibrium(lat_a, rho_a, u_a), budget_s / 3)
    return {"value": round(nodes * steps / el / 1e6, 4), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "Oracle B (C, FP64, OpenMP, per-node Gaussian elimination) on a %s periodic sub-block of "
                      "the same initial state, %d steps in %.1f s" % ("x".join(str(x) for x in reversed(sub)),
                                                                       steps, el),
            "one_core_value": round(nodes * steps1 / el1 / 1e6, 4),
            "triangular_form_value": round(nodes * steps_t / el_t / 1e6, 4),
            "oracle_a_d2q9_64_mlups": round(64 * 64 * steps_a / el_a / 1e6, 4)}


def adjoint_cost(torch, L=512, nsteps=2000, K=100, reps=2):
    """Cost of the discrete adjoint (forward with snapshots + recompute + reverse
    sweep, FP64 accumulation of dJ/ds and dJ/du~) over the plain forward, on the
    D2Q9 random-phase workload (amplitude 0.02, wavenumbers 1..8), FP32 storage,
    u~ = u(x, 0) frozen."""
    from paper_1312_3297_amd import workloads as W
    from paper_1312_3297_amd.lbmrv import Lbmrv
    s = W.RATES_D2Q9_GROUPED
    ctx = Lbmrv("d2q9", s, (L, L), "f32")
    rho, u = W.random_phase(L, 0.02, 1, 8, 1315)
    f0 = ctx.init_equilibrium(torch.from_numpy(rho).to("cuda"), torch.from_numpy(u).to("cuda"))
    field = torch.from_numpy(u).to("cuda").to(torch.float32)
    a, b = f0.clone(), torch.empty_like(f0)
    cot = torch.randn((9, L, L), device="cuda", dtype=torch.float32)
    ws = torch.empty(ctx.adjoint_workspace_bytes(nsteps, K), dtype=torch.uint8, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    fwd = {"push": [], "pull": [], "aa": []}
    adj = []
    for form in fwd:
        ctx.set_streaming(form)
        ctx.step(a, a if form == "aa" else b, "field", 1.0, field, 10)
    ctx.adjoint(f0, cot, 20, 7, "field", field, workspace=ws)
    torch.cuda.synchronize()
    for _ in range(reps):
        for form, times in fwd.items():
            ctx.set_streaming(form)
            a.copy_(f0)
            ev[0].record()
            ctx.step(a, a if form == "aa" else b, "field", 1.0, field, nsteps)
            ev[1].record()
            torch.cuda.synchronize()
            times.append(ev[0].elapsed_time(ev[1]))
        ev[1].record()
        ctx.adjoint(f0, cot, nsteps, K, "field", field, workspace=ws)
        ev[2].record()
        torch.cuda.synchronize()
        adj.append(ev[1].elapsed_time(ev[2]))
    # the plain forward in its fastest form on this grid
    form, f_ms = min(((k, min(v)) for k, v in fwd.items()), key=lambda kv: kv[1])
    a_ms = min(adj)
    return {"workload": "d2q9_randomphase%d_f32_field" % L, "nsteps": nsteps, "K": K,
            "forward_ms": round(f_ms, 3), "forward_form": form,
            "forward_ms_by_form": {k: round(min(v), 3) for k, v in fwd.items()},
            "adjoint_ms": round(a_ms, 3), "cost_ratio": round(a_ms / f_ms, 3)}


def adjoint_costs(torch):
    """The adjoint workload (512^2, N = 2000, K = 100), and the same at 2048^2
    with N = 200 where launch overheads no longer weigh.  Each also with K = N:
    every state of the forward sweep stays in HBM (18.9 GB at 512^2, 30.2 GB
    at 2048^2), so no segment is recomputed.  The cost ratio divides by the
    plain forward in its fastest streaming form on the same grid."""
    out = adjoint_cost(torch)
    out["at_2048"] = adjoint_cost(torch, L=2048, nsteps=200, K=100, reps=2)
    out["all_states_resident"] = adjoint_cost(torch, K=2000)
    out["all_states_resident_2048"] = adjoint_cost(torch, L=2048, nsteps=200, K=200, reps=2)
    return out


def side_kernels(ctx, f, b, torch, reps=20):
    """The moments output (rho, u; and with all q moments m(0)) and the FP64
    conservation reduction on the benchmark state: time per call and the
    algorithmic bytes moved per second.  The reduction returns host values,
    so its figure is wall time per call, synchronisation included."""
    N, q, d = ctx.N, ctx.q, ctx.d
    bo = 8 if b == 8 else 4
    stream = torch.cuda.current_stream()
    res = {}
    for key, with_m0 in (("moments", False), ("moments_m0", True)):
        ctx.moments(f, with_m0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            ctx.moments(f, with_m0)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        nbytes = q * b * N + (1 + d + (q if with_m0 else 0)) * bo * N
        res[key] = {"us": round(us, 1), "GB_s": round(nbytes / (us * 1e-6) / 1e9, 1)}
    ctx.conservation(f)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.conservation(f)
    us = (time.perf_counter() - t0) * 1e6 / reps
    res["conservation"] = {"us_wall": round(us, 1), "GB_s_wall": round(q * b * N / (us * 1e-6) / 1e9, 1)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="d3q19_tgv256_f32dev_fluid", choices=sorted(WORKLOADS))
    ap.add_argument("--streaming", default=None, choices=["pull", "push", "aa"],
                    help="default: in place (aa), pull for a run-time basis")
    ap.add_argument("--block-order", default="auto", choices=["auto", "natural", "xcd"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(domain decomposition across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1312_3297_amd.lbmrv import Lbmrv

    name = args.workload
    lattice, dims, storage, mode = WORKLOADS[name]
    if args.streaming is None:
        args.streaming = "pull" if name in RUNTIME_BASIS else "aa"
    if name in RUNTIME_BASIS:
        from paper_1312_3297_amd import workloads as W
        basis, rates = (getattr(W, x) for x in RUNTIME_BASIS[name])
        ctx = Lbmrv(lattice, rates, dims, storage, basis=basis)
    else:
        ctx = Lbmrv(lattice, rates_for(lattice), dims, storage)
    ctx.set_streaming(args.streaming)
    ctx.set_block_order(args.block_order)
    if name in WALLS:
        mask, uwall = WALLS[name]
        wu = [[0.0, 0.0, 0.0] for _ in range(6)]
        wu[3] = [uwall, 0.0, 0.0]
        ctx.set_walls(mask, wu, 1.0)
    f, field = build_state(name, ctx, torch)
    # the in-place form needs one array only
    g = f if args.streaming == "aa" else torch.empty_like(f)
    stream = torch.cuda.current_stream()

    # warmup
    ctx.step(f, g, mode, 1.0, field, args.warmup)
    f, g = g, f
    torch.cuda.synchronize()

    K = args.steps
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    ctx.step(f, g, mode, 1.0, field, K)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    f, g = g, f

    mass, mom, finite = ctx.conservation(f)
    N = ctx.N
    q = ctx.q
    b = {"f64": 8, "f32": 4, "f32dev": 4, "f16dev": 2}[storage]
    # kernel launches inside the call: pull = collide + (K-1) fused + transport;
    # push = K fused (+ one split step when K is even); in place = K (+ one swap
    # pass when K is odd).  Every launch reads and writes q populations per node
    # (the swap pass a little less).
    launches = {"pull": K + 1, "push": K if K % 2 else K + 1, "aa": K + (K % 2)}[args.streaming]
    bytes_per_step = 2 * q * b * N + (ctx.d * 4 * N if mode == "field" else 0)
    achieved = bytes_per_step * K / (ms * 1e-3) / 1e9
    achieved_launch = bytes_per_step * launches / (ms * 1e-3) / 1e9
    mlups = N * K / (ms * 1e-3) / 1e6
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f32dev": "f32", "f16dev": "f16-storage/f32"}[storage],
        "data": "synthetic",
        "config": {"workload": name, "lattice": lattice, "grid": list(dims), "storage": storage,
                   "relative_velocity": mode, "streaming": args.streaming, "block_order": args.block_order,
                   "nodes": N},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": TRAFFIC_GB.get((name, args.streaming)) if args.block_order == "auto" else None,
                     "bytes_per_step_GB": round(bytes_per_step / 1e9, 4),
                     "per_launch": {"launches": launches, "achieved": round(achieved_launch, 1),
                                    "frac": round(achieved_launch / HBM_PEAK_GBS, 4)}},
        "state_finite": bool(finite),
        "wall_s": round(wall, 4),
    }
    out["side_kernels"] = side_kernels(ctx, f, b, torch)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_costs(torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(name, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
