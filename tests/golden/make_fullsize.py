"""Writes the stored FP64 references of the benchmark workloads at full size.

For each workload below, the FP64 oracle (Oracle B in its triangular-solve
form, oracle/fast/oracle_tri.c) runs the configured grid for the configured
number of steps from the seeded initial state, and this script stores, at a
seeded set of sample nodes (all corners, nodes on every face, the rest drawn
uniformly), the density rho, the velocity u = q / rho (eq. (rhoq)) and all q
fixed-frame moments m(0) = M(0) f of the basis (the paper's m(0) of
section 1.3), plus whole-grid norms and sums that the comparisons are scaled
by.  The state compared is the pre-collision f after N full steps
(relaxation then transport, section 1.2).

Only oracle/ and the seeded input generators (paper_1312_3297_amd/workloads.py,
loaded from its file so that nothing of the library is imported) are used.

  python tests/golden/make_fullsize.py [--only NAME] [--threads T]

Runtime with 8 threads of an AVX2 host: about 15 min (D2Q9 2048^2, 2000 steps),
60 min (D3Q19 256^3, 1000 steps) and 70 min (D3Q27 192^3, 1000 steps).
"""
import argparse
import importlib.util
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fast, lattices  # noqa: E402
from oracle import scheme as A  # noqa: E402

_spec = importlib.util.spec_from_file_location("workloads", os.path.join(ROOT, "paper_1312_3297_amd", "workloads.py"))
W = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(W)

NSAMPLE = 4096
PER_FACE = 64

# name: lattice, grid (nx, ny[, nz]), initial state, rates, u~ mode, steps, sample seed
WORKLOADS = {
    "d2q9_shear2048_fluid": dict(lattice="d2q9_paper", L=2048, init="shear_layer", rates="RATES_D2Q9_SHEAR_LAYER",
                                 mode="fluid", steps=2000, seed=5001),
    "d3q19_tgv256_fluid": dict(lattice="d3q19", L=256, init="taylor_green", noise_seed=1313,
                               rates="RATES_D3Q19", mode="fluid", steps=1000, seed=5002),
    "d3q27_tgv192_field": dict(lattice="d3q27", L=192, init="taylor_green", noise_seed=1314,
                               rates="RATES_D3Q27", mode="field", steps=1000, seed=5003),
}
NOISE_AMP = 1e-5


def path(name):
    return os.path.join(HERE, "fullsize_%s.npz" % name)


def sample_nodes(d, L, seed):
    """Grid indices (z, y, x) in 3-D or (y, x) in 2-D of the sample nodes:
    every corner, PER_FACE nodes drawn on each face, the rest drawn anywhere;
    distinct, in increasing node order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    picked = set()
    for c in range(1 << d):
        picked.add(tuple((L - 1) if (c >> a) & 1 else 0 for a in range(d)))
    for a in range(d):
        for side in (0, L - 1):
            n = 0
            while n < PER_FACE:
                p = list(rng.integers(0, L, d))
                p[a] = side
                if tuple(p) not in picked:
                    picked.add(tuple(p))
                    n += 1
    while len(picked) < NSAMPLE:
        picked.add(tuple(rng.integers(0, L, d)))
    nodes = np.array(sorted(picked), dtype=np.int64)
    return nodes


def initial_state(cfg, lat):
    L = cfg["L"]
    if cfg["init"] == "shear_layer":
        rho, u = W.double_shear_layer(L)
        f = A.equilibrium(lat, rho, u)
    else:
        rho, u = W.taylor_green(L, 0.05)
        f = A.equilibrium(lat, rho, u)
        f += NOISE_AMP * W.noise(lat.q, rho.shape, cfg["noise_seed"])
    field = None
    if cfg["mode"] == "field":
        # the prescribed relative velocity, half the initial fluid velocity,
        # as the FP32 field the library is given
        field = (0.5 * u).astype(np.float32).astype(np.float64)
    return f, u, field


def reference(name, threads):
    cfg = WORKLOADS[name]
    lat = lattices.make(cfg["lattice"])
    q, d = lat.q, lat.d
    f, u0, field = initial_state(cfg, lat)
    del u0
    mode = {"zero": A.ZERO, "fluid": A.FLUID, "field": A.FIELD}[cfg["mode"]]
    t0 = time.time()
    fN = fast.run_tri(lat, f, getattr(W, cfg["rates"]), cfg["steps"], 1.0, mode, 1.0, field, threads=threads, out=f)
    wall = time.time() - t0
    nodes = sample_nodes(d, cfg["L"], cfg["seed"])
    flat = np.ravel_multi_index(tuple(nodes.T), fN.shape[1:])
    F = fN.reshape(q, -1)
    fs = F[:, flat]                                         # (q, S)
    rho_s, u_s = A.conserved(lat, fs)
    m0_s = A.fixed_moments(lat, fs)
    # whole-grid norms and sums
    rho = F.sum(axis=0)
    v = lat.velocities(1.0)
    mom = np.stack([v[:, a] @ F for a in range(d)])        # (d, N)
    M0 = A.moment_matrix(lat, np.zeros((1, d)))[0]
    m0_norm = np.array([np.abs(M0[k] @ F).max() for k in range(q)])
    uabs = np.abs(mom / rho).max()
    out = dict(nodes=nodes, rho=rho_s, u=u_s, m0=m0_s,
               rho_norm=np.abs(rho).max(), rho_dev_norm=np.abs(rho - 1.0).max(), u_norm=uabs, m0_norm=m0_norm,
               mass=rho.sum(), momentum=mom.sum(axis=1), kinetic=0.5 * ((mom * mom).sum(axis=0) / rho).sum())
    meta = dict(workload=name, lattice=cfg["lattice"], grid=[cfg["L"]] * d, steps=cfg["steps"], mode=cfg["mode"],
                rates=list(getattr(W, cfg["rates"])), noise_amp=NOISE_AMP if cfg["init"] != "shear_layer" else 0.0,
                noise_seed=cfg.get("noise_seed"), sample_seed=cfg["seed"],
                oracle="Oracle B, triangular-solve form (oracle/fast/oracle_tri.c), FP64",
                oracle_wall_s=round(wall, 1), threads=threads)
    np.savez_compressed(path(name), meta=np.array(json.dumps(meta)), **out)
    print("%s: %d steps in %.0f s, wrote %s" % (name, cfg["steps"], wall, path(name)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", choices=sorted(WORKLOADS))
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    args = ap.parse_args()
    for name in ([args.only] if args.only else list(WORKLOADS)):
        reference(name, args.threads)


if __name__ == "__main__":
    main()
