"""Benchmark of the coupled capsule lattice Boltzmann step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c2] [--gpus 1]

Prints one JSON line.  A step is one full coupled time step (density pass,
membrane forces, binning, spreading, fused collide-stream, interpolation and
advection) over the whole lattice.  `value` is MLUPS = lattice nodes x
steps / wall time of the timed region, with all state resident in HBM.

roofline: the fused collide-stream kernel dominates; its achieved bandwidth
is the algorithmic bytes per launch (152 B population reads + 152 B
population writes + 8 B density reads per lattice node, FP32) over its
average duration from HIP events recorded on the library's stream around
each launch in the timed region.

cpu_baseline: the FP64 oracle (test infrastructure) timed on this host on a
bounded sample of the same workload.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (2-comp D3Q19+IBM), % HBM peak, FP16-store vs FP32, adjoint/fwd time"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per lattice update of the fused collide kernel (FP32)
COLLIDE_BYTES_PER_LUP = {"fp32": 2 * 19 * 4 * 2 + 2 * 4}
DENSITY_BYTES_PER_LUP = {"fp32": 2 * 19 * 4 + 2 * 4}

WORKLOAD_TEXT = {
    "c2": "128^3 periodic two-component box, flat interface at z=64, 8 capsules R=8 (2562-node "
          "icospheres) seeded in z=64+-4, kS~U[0.002,0.02], theta~U[60,120] deg, tau=1, G=3.6",
    "c5": "512^3 periodic two-component box, flat interface at z=256, 512 capsules of 162/642/2562 "
          "nodes (R 4/6/10), theta~U[60,120] deg, tau=1, G=3.6",
    "c1": "32^3 periodic box, flat interface, one R=6 capsule (642 nodes)",
}


def cpu_baseline(wl, budget_s=20.0):
    """Time the FP64 oracle on a bounded sample of the same workload."""
    import torch
    from oracle.sim import from_workload
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = max(1, min(cores, 16))
    torch.set_num_threads(cores)
    o = from_workload(wl)
    o.step()                    # first step pays allocation
    t0 = time.perf_counter()
    n = 0
    while True:
        o.step()
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s * 0.5 or n >= 50:
            break
    return {"value": wl.n_lattice * n / el / 1e6, "unit": "MLUPS", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": "%d FP64 oracle steps of the benchmark workload (%dx%dx%d, %d capsules) after one "
                      "untimed step, %.1f s" % (n, wl.nx, wl.ny, wl.nz, len(wl.capsules), el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="fp32", choices=["fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the step would shard by z-slabs; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1904_11386_amd import workloads
    from paper_1904_11386_amd.binding import sim_from_workload

    wl = workloads.make(args.workload)
    print("bench: workload %s %dx%dx%d, %d capsules, %d nodes" %
          (args.workload, wl.nx, wl.ny, wl.nz, len(wl.capsules), int(wl.meshes()[0].sum())),
          file=sys.stderr, flush=True)
    sim = sim_from_workload(wl)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms = sim.step_timed(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    N = wl.n_lattice
    mlups = N * args.steps / wall / 1e6
    obs = sim.observables()
    m0 = np.array([wl.rhoA.astype(np.float64).sum(), wl.rhoB.astype(np.float64).sum()])
    mass_drift = float(np.abs(obs["mass"] / m0 - 1).max())

    t_col = kms["collide"] / args.steps * 1e-3
    t_den = kms["density"] / args.steps * 1e-3
    bpl = COLLIDE_BYTES_PER_LUP[args.precision]
    achieved = bpl * N / t_col / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_collide", "bytes_per_launch": bpl * N, "avg_launch_ms": round(t_col * 1e3, 5)}
    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT.get(args.workload, args.workload), "name": args.workload,
                   "lattice": [wl.nx, wl.ny, wl.nz], "capsules": len(wl.capsules),
                   "membrane_nodes": int(wl.meshes()[0].sum()), "precision": args.precision},
        "roofline": roof,
        "kernels_ms_per_step": {k: round(v / args.steps, 5) for k, v in kms.items()},
        "density_pass_gbs": round(DENSITY_BYTES_PER_LUP[args.precision] * N / t_den / 1e9, 1),
        "fp64_mass_drift": mass_drift,
    }
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        print("bench: timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
