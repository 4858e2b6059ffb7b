"""Benchmark of the coupled capsule lattice Boltzmann step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c5] [--gpus 1]

Prints one JSON line.  A step is one full coupled time step (densities,
membrane forces, binning, spreading, fused collide-stream, interpolation and
advection) over the whole lattice; the FP32 form of the large lattices forms
the densities inside the collide (one lattice pass), and the line also
times the same steps with a separate density pass (`fp32_two_passes`).  The headline workload is the largest
configuration, the 512^3 periodic box with 512 capsules; `value` is its
MLUPS in FP32 storage = lattice nodes x steps / wall time of the timed
region, with all state resident in HBM.  The FP16-storage form runs on the
same workload (`fp16_form`); legs follow on the 256^3 droplet (FP16/FP32
ratio), the 128^3 box, the sheared channel (adjoint cost and its check
against central differences) and the FP64 oracle on the host.

roofline: the fused collide-stream kernel dominates; its achieved bandwidth
is the algorithmic bytes per launch (152 B population reads + 152 B
population writes per lattice node in one pass, plus 8 B density reads in
two, FP32) over its
average duration from HIP events recorded on the library's stream around
each launch, in a second timed region of the same number of steps run
right after the first (the first replays HIP graphs, which carry no
per-kernel events).  traffic: HBM bytes per launch from the committed
rocprofv3 counter summary of the same kernel and workload.

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
# FP32: 152 B population reads + 152 B writes + 8 B density; FP16: 76 + 76 B
# of binary16 populations + 8 B densities of step n + 8 B decode densities
COLLIDE_BYTES_PER_LUP = {"fp32": 2 * 19 * 4 * 2 + 2 * 4, "fp16": 2 * 19 * 2 * 2 + 2 * 4 + 2 * 4}
DENSITY_BYTES_PER_LUP = {"fp32": 2 * 19 * 4 + 2 * 4, "fp16": 2 * 19 * 2 + 2 * 4 + 2 * 4}
# one lattice pass (FP32): the collide reads and writes the populations only
# (152 + 152 B); it forms the densities from what it pulls
ONE_PASS_BYTES_PER_LUP = 2 * 19 * 4 * 2

WORKLOAD_TEXT = {
    "c2": "128^3 periodic two-component box, flat interface at z=64, 8 capsules R=8 (2562-node "
          "icospheres) seeded in z=64+-4, kS~U[0.002,0.02], theta~U[60,120] deg, tau=1, G=3.6",
    "c5": "512^3 periodic two-component box, flat interface at z=256, 512 capsules of 162/642/2562 "
          "nodes (R 4/6/10), theta~U[60,120] deg, tau=1, G=3.6",
    "c1": "32^3 periodic box, flat interface, one R=6 capsule (642 nodes)",
    "c3": "256^3 periodic box, B droplet R=60 in A, 64 capsules R=6 (642 nodes) on a shell of radius 66, "
          "theta~U[45,135] deg, tau=1, G=3.6",
}


def measured_traffic(workload, form):
    """HBM bytes per k_collide launch of one storage form on one workload from
    the committed rocprofv3 counter summary profiles/k_collide_<workload>_pmc.md,
    or None when there is none or the lattice kernel sources changed since
    the counters were taken."""

    path = os.path.join(ROOT, "profiles", "k_collide_%s_pmc.md" % workload)
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if line.startswith("traffic_bytes_per_launch k_collide %s:" % form):
            rec["bytes"] = float(line.split(":")[1])
        if line.startswith("source_sha256_16:"):
            rec["sha"] = line.split(":")[1].strip()
    if rec.get("sha") != lattice_source_hash():
        return None
    return rec.get("bytes")


def lattice_source_hash():
    """First 16 hex digits of the SHA-256 of the lattice kernels' sources:
    csrc/k_fluid.hip, the Lattice struct they read and the block-shape
    constants they are compiled with (the other parts of lbm_internal.h do
    not reach these kernels)."""
    import hashlib
    h = hashlib.sha256()
    h.update(open(os.path.join(ROOT, "paper_1904_11386_amd/csrc/k_fluid.hip"), "rb").read())
    hdr = open(os.path.join(ROOT, "paper_1904_11386_amd/csrc/lbm_internal.h")).read()
    i0 = hdr.index("struct Lattice {")
    h.update(hdr[i0:hdr.index("\n};", i0)].encode())
    for line in hdr.splitlines():
        if line.startswith(("#define LBM_BX", "#define LBM_BY", "#define LBM_ZC")):
            h.update(line.encode())
    return h.hexdigest()[:16]


def copy_ceiling(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy bandwidth (read + write bytes / time) of a
    plain 1 GiB tensor copy, as the achievable-bandwidth reference."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def host_threads():
    """Threads the oracle runs on: torch's default, which follows the
    environment's OpenMP setting (the host cores given to this job), and the
    number of cores this process may run on."""
    import torch
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return torch.get_num_threads(), aff


def cpu_baseline(wl, budget_s=20.0):
    """Time the FP64 oracle on a bounded sample of the same workload: the
    whole lattice when it has at most 128^3 nodes, else a 128 x 128 x 64 box
    of its initial state around the interface with the capsules that lie
    wholly inside it."""
    import torch
    from oracle.sim import from_workload
    from paper_1904_11386_amd import workloads
    sample = wl
    if wl.n_lattice > 128 ** 3:
        z0 = int(min(max(wl.z_interface - 31.5, 0), wl.nz - 64))
        sample = workloads.crop(wl, 0, 0, z0, 128, 128, 64)
    threads, aff = host_threads()
    o = from_workload(sample)
    o.step()                    # first step pays allocation
    t0 = time.perf_counter()
    n = 0
    while True:
        o.step()
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s * 0.5 or n >= 50:
            break
    used = torch.get_num_threads()
    # one more step on a single thread, for the per-core rate
    torch.set_num_threads(1)
    t1 = time.perf_counter()
    o.step()
    el1 = time.perf_counter() - t1
    torch.set_num_threads(used)
    return {"value": sample.n_lattice * n / el / 1e6, "unit": "MLUPS", "cores": used, "affinity_cores": aff,
            "kind": "oracle", "value_1_thread": sample.n_lattice / el1 / 1e6,
            "sample": "%d FP64 oracle steps of a %dx%dx%d box of the benchmark workload (%d capsules wholly "
                      "inside) after one untimed step, %.1f s; then one step on one thread, %.1f s"
                      % (n, sample.nx, sample.ny, sample.nz, len(sample.capsules), el, el1)}


def oracle_timing_leg():
    """The FP64 oracle's own rate on the small configurations, on this host:
    the 32^3 one-capsule case in full (1000 steps) and the 64^3 crop of the
    benchmark workload and 64^3 copy of the precision workload over 50 steps
    each, at all cores and at one thread.  A reported baseline only."""
    import torch
    from oracle.sim import from_workload
    from paper_1904_11386_amd import workloads
    cores, aff = host_threads()
    out = {"cores": cores, "affinity_cores": aff}
    for name, steps in (("c1", 1000), ("c2_64", 50), ("c3_64", 50)):
        wl = workloads.make(name)
        row = {"steps": steps}
        for label, threads in (("all_cores", cores), ("one_thread", 1)):
            torch.set_num_threads(threads)
            print("bench: oracle timing %s, %d thread(s)" % (name, threads), file=sys.stderr, flush=True)
            o = from_workload(wl)
            o.step()
            t0 = time.perf_counter()
            o.run(steps - 1)
            el = time.perf_counter() - t0
            row[label + "_mlups"] = round(wl.n_lattice * (steps - 1) / el / 1e6, 4)
        out[name] = row
    torch.set_num_threads(cores)
    return out


def adjoint_leg(torch, steps=2000, every=100):
    """Forward and backward wall time of the hand-written adjoint on the
    192x96x96 sheared channel (one 2562-node capsule, theta 75 deg,
    kS 0.005, G 3.6): J = capsule height after 2000 steps, checkpoint every
    100 steps."""
    from paper_1904_11386_amd import workloads
    from paper_1904_11386_amd.binding import LBM_OBJ_COM_Z, sim_from_workload
    wl = workloads.make("c4")
    print("bench: adjoint leg on c4 (%d steps, checkpoint every %d)" % (steps, every), file=sys.stderr, flush=True)
    plain = sim_from_workload(wl)
    plain.step(20)
    plain.synchronize()
    t0 = time.perf_counter()
    plain.step(steps)
    plain.synchronize()
    t_plain = time.perf_counter() - t0
    plain.close()
    del plain
    torch.cuda.empty_cache()
    sim = sim_from_workload(wl, n_slots=(steps + every - 1) // every, ring_len=every)
    t0 = time.perf_counter()
    J = sim.adjoint_forward(steps, every, LBM_OBJ_COM_Z, 0)
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    g = sim.adjoint_backward()
    t_bwd = time.perf_counter() - t0
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"workload": "192x96x96 channel, walls at y=0/95 moving -+0.01, interface z=48, one 2562-node R=10 "
                        "capsule, theta 75 deg, kS 0.005, G 3.6",
            "steps": steps, "checkpoint_every": every, "J_com_height": J,
            "grad_theta_per_rad": g[0], "grad_kS": g[1], "grad_G": g[2],
            "forward_s": round(t_plain, 4), "forward_with_checkpoints_s": round(t_fwd, 4),
            "backward_s": round(t_bwd, 4), "backward_over_forward": round(t_bwd / t_plain, 3)}


def adjoint_fd_sweep(torch, steps=2000, every=100):
    """Full-size gradient check on the 192x96x96 channel: the hand-written
    adjoint's dJ/d(theta, kS, G) for J = capsule height after `steps` steps,
    against central differences of the GPU FP32 forward run over a sweep of
    steps h; the plateau (smallest relative difference over h) is reported
    per parameter."""
    import math
    from paper_1904_11386_amd import workloads
    from paper_1904_11386_amd.adjoint import workload_with
    from paper_1904_11386_amd.binding import LBM_OBJ_COM_Z, sim_from_workload
    wl = workloads.make("c4")
    p0 = [75.0, 0.005, 3.6]
    sim = sim_from_workload(workload_with(wl, *p0), n_slots=(steps + every - 1) // every, ring_len=every)
    J = sim.adjoint_forward(steps, every, LBM_OBJ_COM_Z, 0)
    g = sim.adjoint_backward()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    grad = [g[0] * math.pi / 180.0, g[1], g[2]]        # per degree, per kS, per G

    def height(p):
        s = sim_from_workload(workload_with(wl, *p))
        s.step(steps)
        h = s.observables()["caps"][0]["height"]
        s.close()
        return h

    names = ("theta_deg", "kS", "G")
    h0 = (2.0, 1e-3, 0.04)
    n_h = 8                                            # h = h0, h0/2, ..., h0/128
    # the FP32 forward is not bit-reproducible (float atomics in the force
    # spread), so J carries run-to-run noise that bounds the smallest useful h
    reruns = [height(p0) for _ in range(3)]
    noise = float(np.std(reruns, ddof=1))
    out = {"workload": "192x96x96 channel (c4), J = capsule height after %d steps" % steps, "J": J,
           "J_rerun_std": noise, "adjoint": dict(zip(names, grad))}
    # A changed parameter also changes every rounding of the run, which a
    # rerun at the same parameters does not: J at parameters moved by steps
    # far too small to matter physically, minus the adjoint's linear part,
    # is that rounding noise (per parameter).
    tiny = (1e-5, 1e-8, 1e-6)
    J0 = reruns[0]
    for k, name in enumerate(names):
        rest = []
        for m in (1.0, -1.0, 2.0, -2.0):
            pp = list(p0)
            pp[k] += m * tiny[k]
            rest.append(height(pp) - J0 - grad[k] * m * tiny[k])
        pnoise = float(np.sqrt(np.mean(np.square(rest))))
        rows = []
        for i in range(n_h):
            h = h0[k] / 2 ** i
            print("bench: FD sweep %s h=%g" % (name, h), file=sys.stderr, flush=True)
            pp, pm = list(p0), list(p0)
            pp[k] += h
            pm[k] -= h
            fd = (height(pp) - height(pm)) / (2 * h)
            rows.append({"h": h, "fd": fd, "rel_diff": abs(grad[k] - fd) / abs(fd),
                         "noise_rel": math.sqrt(2.0) * noise / (2 * h) / abs(fd),
                         "perturbation_noise_rel": math.sqrt(2.0) * pnoise / (2 * h) / abs(fd)})
        best = min(rows, key=lambda r: r["rel_diff"])
        out[name] = {"sweep": rows, "plateau_rel_diff": best["rel_diff"], "plateau_h": best["h"],
                     "J_perturbation_noise": pnoise}
    return out


def membrane_extras_leg(torch, warmup=100, steps=200):
    """The 512^3 configuration with the optional membrane terms on: Helfrich
    bending at the paper's B = kB / (kS R0^2) = 1e-2 (Sec. II.B) and the
    particle-particle repulsion of Sec. III.E (eps 0.5, cut-off 1.25); both
    storage forms, MLUPS and the two terms' kernel time per step.  The seeded
    capsules start at least 2 lu apart, so the repulsion prices the bin
    search every step pays."""
    import dataclasses
    from paper_1904_11386_amd import workloads
    from paper_1904_11386_amd.binding import LBM_FP16, LBM_FP32, sim_from_workload
    base = workloads.make("c5")
    caps = [dataclasses.replace(c, kB=1e-2 * c.kS * c.radius ** 2) for c in base.capsules]
    wl = dataclasses.replace(base, capsules=caps, rep_eps=0.5, rep_d0=1.25)
    N = wl.n_lattice
    out = {"workload": "512^3 scale configuration with bending (B = 1e-2) and particle-particle repulsion "
                       "(eps 0.5, d0 1.25)", "warmup": warmup, "steps": steps}
    for name, prec in (("fp32", LBM_FP32), ("fp16", LBM_FP16)):
        print("bench: membrane extras leg, %s form" % name, file=sys.stderr, flush=True)
        sim = sim_from_workload(wl, precision=prec)
        sim.step(warmup)
        sim.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.synchronize()
        wall = time.perf_counter() - t0
        k = sim.step_timed(20)
        out[name] = {"mlups": round(N * steps / wall / 1e6, 1), "ms_per_step": round(wall / steps * 1e3, 4),
                     "repulse_ms_per_step": round(k["repulse"] / 20, 5), "bend_ms_per_step": round(k["bend"] / 20, 5)}
        sim.close()
        del sim
        torch.cuda.empty_cache()
    return out


def reference_model_leg(torch, steps=240000, chunk=20000, kV=20.0, beta=1000.0, C=9.0, w=1.0):
    """The LBM-free reference model of Sec. III.B at the paper's particle
    size: R0 = 10 (2562-node mesh), beta = R0^2 gamma / kB = 1000,
    B = kB / (kS R0^2) = 1e-2, nu_s = 0.9 (C = 9), volume modulus kV (20),
    gamma = 0.0388, w = 1, overdamped with mobility 0.05.  Reports the ellipsoid half-axes
    (from the volume second moments, the paper's 'tensor of inertia') along
    the relaxation and the time per membrane step."""
    import numpy as np
    from paper_1904_11386_amd import workloads
    from paper_1904_11386_amd.binding import sim_from_workload
    R0, gamma, B, mu = 10.0, 0.0388, 1e-2, 0.05
    kB = R0 * R0 * gamma / beta
    kS = kB / (B * R0 * R0)
    ra, rb = workloads.layered(32, 32, 32, 16)
    cap = workloads.Capsule(workloads._snap(np.array([16.0, 16.0, 16.0])), R0, 16, kS, C, kV, 90.0, kB=kB)
    wl = workloads.Workload("reference", 32, 32, 32, ra, rb, [cap], z_interface=15.5)
    sim = sim_from_workload(wl)
    hist = []
    t_run = 0.0
    for k in range(steps // chunk):
        sim.synchronize()
        t0 = time.perf_counter()
        sim.reference_relax(chunk, gamma, w, 16.0, mu)
        sim.synchronize()
        t_run += time.perf_counter() - t0
        ax = sim.observables()["caps"][0]["axes"]
        hist.append({"steps": (k + 1) * chunk, "r_p": round(float(ax[0]), 5), "r_i": round(float(ax[2]), 5),
                     "r_i_mean": round(0.5 * float(ax[1] + ax[2]), 5)})
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"workload": "one R0=10 capsule (2562 nodes), beta %g, B 1e-2, C %g (nu_s %.2f), kV %g, gamma 0.0388, "
                        "w %g, mobility 0.05" % (beta, C, C / (1.0 + C), kV, w),
            "us_per_step": round(t_run / steps * 1e6, 2), "relaxation": hist}


def reference_sweep_leg(torch, betas=(10.0, 100.0, 1000.0), nus=(0.5, 0.9), ws=(1.0, 4.0), steps=240000):
    """The reference model's equilibrium over the softness beta, the surface
    Poisson ratio nu_s (C = nu_s / (1 - nu_s)) and the emulated interface
    width w (the membrane-only part of the paper's comparison, Sec. III.B):
    final half-axes r_p and mean r_i, and their change over the last 20 000
    steps as a convergence measure."""
    out = []
    for beta in betas:
        for nu in nus:
            for w in ws:
                print("bench: reference sweep beta %g nu_s %g w %g" % (beta, nu, w), file=sys.stderr, flush=True)
                r = reference_model_leg(torch, steps=steps, kV=20.0, beta=beta, C=nu / (1.0 - nu), w=w)
                a, b = r["relaxation"][-2], r["relaxation"][-1]
                out.append({"beta": beta, "nu_s": nu, "w": w, "r_p": b["r_p"], "r_i": b["r_i_mean"],
                            "ratio": round(b["r_i_mean"] / b["r_p"], 4),
                            "last_change": round(max(abs(b["r_p"] - a["r_p"]), abs(b["r_i_mean"] - a["r_i_mean"])), 5)})
    return {"workload": "one R0=10 capsule (2562 nodes), B 1e-2, kV 20, gamma 0.0388, mobility 0.05, %d steps" % steps,
            "runs": out}


def shape_error_leg(torch, betas=(100.0, 1000.0), steps=40000, chunk=5000, kV=2.0, coupling=0):
    """The shape errors of Sec. III.B (eq. interface:error) between the
    reference model and the coupled simulation of the same capsule (R0 = 10,
    2562 nodes, B 1e-2, nu_s 0.9, softness beta) at the flat interface of a
    64x64x48 two-component box (G 3.6, theta 90 deg), run to equilibrium.
    Delta_p = (r_p^ref - r_p^sim) / R0 and Delta_i = (r_i^ref - r_i^sim) / R0
    with r_p the half-axis normal to the interface and r_i the mean of the two
    in-plane half-axes, both from the volume second moments.
    coupling 0: the immersed boundary, workloads' fluid (psi = rho, densities
    0.7 / 0.04), volume modulus kV = 2 (the explicit coupling diverges within
    250 steps at kV = 20).  coupling 1: the paper's bounce-back coupling with
    its fluid (psi = 1 - exp(-rho), 0.7 / 0.042), inertial nodes of mass 5,
    the capsule filled with the lower fluid and centred off the lattice's
    symmetry planes; pass the paper's kV = 20.  The reference model runs with
    the same kV."""
    import numpy as np
    from paper_1904_11386_amd import workloads
    from paper_1904_11386_amd.binding import LbmError, sim_from_workload
    R0, gamma, B = 10.0, 0.0388, 1e-2
    bb = coupling == 1
    rho = (0.7, 0.042) if bb else (float(workloads.RHO_MAJ), float(workloads.RHO_MIN))
    out = {"workload": "64x64x48 box, interface z=23.5, one R0=10 capsule (2562 nodes), B 1e-2, nu_s 0.9, kV %g, "
                       "theta 90 deg, G 3.6, %s" % (kV, "bounce-back coupling (node mass 5), psi 1 - exp(-rho), "
                                                   "rho 0.7/0.042" if bb else "immersed boundary, psi rho"),
           "steps": steps, "runs": []}
    for beta in betas:
        print("bench: shape errors, beta %g, coupling %d" % (beta, coupling), file=sys.stderr, flush=True)
        ref = reference_model_leg(torch, kV=kV, beta=beta)
        kB = R0 * R0 * gamma / beta
        kS = kB / (B * R0 * R0)
        ra, rb = workloads.layered(64, 64, 48, 24, rho)
        if bb:
            c = workloads._snap(np.array([32.37, 32.61, 23.83]))
            g = np.meshgrid(np.arange(48), np.arange(64), np.arange(64), indexing="ij")
            ins = (g[2] - c[0]) ** 2 + (g[1] - c[1]) ** 2 + (g[0] - c[2]) ** 2 < (R0 - 0.3) ** 2
            ra = np.where(ins, np.float32(rho[0]), ra).astype(np.float32)
            rb = np.where(ins, np.float32(rho[1]), rb).astype(np.float32)
            cap = workloads.Capsule(c, R0, 16, kS, 9.0, kV, 90.0, kB=kB)
            wl = workloads.Workload("shape_error_bb", 64, 64, 48, ra, rb, [cap], z_interface=23.5, wet_scale=1.0,
                                    coupling=1, node_mass=5.0, mass_c0=2500.0, psi_kind=1,
                                    rho_maj=float(np.float32(rho[0])), rho_min=float(np.float32(rho[1])))
        else:
            cap = workloads.Capsule(workloads._snap(np.array([32.0, 32.0, 24.0])), R0, 16, kS, 9.0, kV, 90.0, kB=kB)
            wl = workloads.Workload("shape_error", 64, 64, 48, ra, rb, [cap], z_interface=23.5)
        sim = sim_from_workload(wl)
        hist = []
        err = None
        t0 = time.perf_counter()
        try:
            for k in range(steps // chunk):
                sim.step(chunk)
                ob = sim.observables()["caps"][0]
                ax = ob["axes"]
                hist.append({"steps": (k + 1) * chunk, "r_p": round(float(ax[0]), 5),
                             "r_i_mean": round(0.5 * float(ax[1] + ax[2]), 5), "com_z": round(float(ob["com"][2]), 4)})
        except LbmError as e:
            err = str(e)
        sim.synchronize()
        wall = time.perf_counter() - t0
        sim.close()
        del sim
        torch.cuda.empty_cache()
        rf = ref["relaxation"][-1]
        run = {"beta": beta, "wall_s": round(wall, 2), "coupled": hist, "reference": rf, "error": err}
        if hist and err is None:
            fin = hist[-1]
            run["delta_p"] = round((rf["r_p"] - fin["r_p"]) / R0, 5)
            run["delta_i"] = round((rf["r_i_mean"] - fin["r_i_mean"]) / R0, 5)
        out["runs"].append(run)
    return out


def shear_leg(torch, cas=(0.0125, 0.025, 0.05, 0.1, 0.2), steps=100000, every=10000):
    """The capsule-in-shear workload of Sec. III.A: a 48^3 box between
    on-site velocity boundaries moving at -+rate (n - 1) / 2 (shear rate
    1e-4), one fluid of density 1 (both components at 0.5, G = 0), one
    R0 = 7.64 capsule (2562 nodes) with C = 1 and kS = rho nu rate R0 / Ca.
    Reports the Taylor deformation D along each run and its final value per
    capillary number, and the time per step."""
    from paper_1904_11386_amd import workloads
    from paper_1904_11386_amd.binding import sim_from_workload
    out = {"workload": "48^3, on-site boundaries y=0/47 at -+2.35e-3, rho 1, G 0, one R0=7.64 capsule "
                       "(2562 nodes), C 1, kS = rho nu rate R0 / Ca", "steps": steps, "runs": []}
    for ca in cas:
        print("bench: capsule in shear, Ca %g" % ca, file=sys.stderr, flush=True)
        wl = workloads.shear(ca)
        sim = sim_from_workload(wl)
        hist = []
        t0 = time.perf_counter()
        for k in range(steps // every):
            sim.step(every)
            hist.append(round(float(sim.observables()["caps"][0]["D"]), 5))
        sim.synchronize()
        wall = time.perf_counter() - t0
        sim.close()
        del sim
        torch.cuda.empty_cache()
        out["runs"].append({"Ca": ca, "kS": round(wl.capsules[0].kS, 7), "D": hist[-1], "D_over_Ca": round(hist[-1] / ca, 3),
                            "D_every_%d" % every: hist, "us_per_step": round(wall / steps * 1e6, 2)})
    return out


def extras_leg(torch, steps=2000):
    """Short runs of the paths outside the benchmark step, for timing and
    kernel profiles: the capsule in shear between on-site boundaries (48^3,
    Ca 0.1, both storage forms), the reference model (20 000 membrane steps),
    capsules with Helfrich bending (bent, 38x34x36) and with the
    particle-particle repulsion (pressed, 37x30x33); microseconds per step
    of each and the per-kernel split of 20 event-timed steps."""
    from paper_1904_11386_amd import workloads
    from paper_1904_11386_amd.binding import LBM_FP16, LBM_FP32, sim_from_workload
    out = {"steps": steps}
    runs = (("shear_fp32", workloads.shear(0.1), LBM_FP32), ("shear_fp16", workloads.shear(0.1), LBM_FP16),
            ("bent", workloads.bent(), LBM_FP32), ("pressed", workloads.pressed(), LBM_FP32))
    for name, wl, prec in runs:
        print("bench: extras leg, %s" % name, file=sys.stderr, flush=True)
        sim = sim_from_workload(wl, precision=prec)
        sim.step(100)
        sim.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.synchronize()
        wall = time.perf_counter() - t0
        k = sim.step_timed(20)
        out[name] = {"us_per_step": round(wall / steps * 1e6, 2),
                     "kernels_us_per_step": {kk: round(v / 20 * 1e3, 2) for kk, v in k.items() if v > 0}}
        sim.close()
        del sim
        torch.cuda.empty_cache()
    out["reference"] = reference_model_leg(torch, steps=20000, chunk=10000)["us_per_step"]
    return out


def precision_study(torch, steps):
    """The FP16 g-storage form beside the FP32 form on the 256^3 droplet
    workload (B droplet of radius 60 in A, 64 capsules of 642 nodes on a
    shell of radius 66, angles in [45, 135] deg): per-component FP64 mass
    drift, droplet radius, density difference and capsule heights after
    `steps` steps, and each form's MLUPS.  (Against the FP64 oracle the same
    forms are checked on the 64^3 copy by the GPU tests.)"""
    from paper_1904_11386_amd import workloads
    from paper_1904_11386_amd.binding import LBM_FP16, LBM_FP32, sim_from_workload
    wl = workloads.make("c3")
    m0 = np.array([wl.rhoA.astype(np.float64).sum(), wl.rhoB.astype(np.float64).sum()])

    def radius(rb):
        v = ((np.asarray(rb, dtype=np.float64) - workloads.RHO_MIN) / (workloads.RHO_MAJ - workloads.RHO_MIN)).sum()
        return float((3.0 * v / (4.0 * np.pi)) ** (1.0 / 3.0))

    out, kept = {"workload": "256^3 periodic box, B droplet R=60 in A, %d capsules R=6 (642 nodes) on a shell "
                             "of radius 66, theta~U[45,135] deg" % len(wl.capsules), "steps": steps}, {}
    # a second FP32 run is the control: spreading sums with float atomics,
    # so two runs of one form differ by rounding order, and after many steps
    # the capsules' trajectories separate on their own
    for name, prec in (("fp32", LBM_FP32), ("fp32_rerun", LBM_FP32), ("fp16", LBM_FP16)):
        print("bench: precision study, %s form, %d steps" % (name, steps), file=sys.stderr, flush=True)
        sim = sim_from_workload(wl, precision=prec)
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            k = min(2000, steps - done)
            sim.step(k)
            sim.synchronize()
            done += k
            print("bench: precision study, %s form, %d / %d steps" % (name, done, steps), file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        ra, rb, _ = sim.fields()
        obs = sim.observables()
        kept[name] = (ra, rb, [c["height"] for c in obs["caps"]])
        out[name] = {"mlups": round(wl.n_lattice * steps / wall / 1e6, 1),
                     "mass_drift": [float(v) for v in (obs["mass"] / m0 - 1)],
                     "droplet_radius": round(radius(rb), 5)}
        sim.close()
        del sim
        torch.cuda.empty_cache()
    a32, b32, h32 = kept["fp32"]

    def diff(other):
        a, b, h = kept[other]
        return {"rho_rel_max": [float(np.abs(a - a32).max() / np.abs(a32).max()),
                                float(np.abs(b - b32).max() / np.abs(b32).max())],
                "droplet_radius_diff": round(out[other]["droplet_radius"] - out["fp32"]["droplet_radius"], 6),
                "capsule_height_diff_max": float(np.abs(np.array(h) - np.array(h32)).max())}
    out["fp16_vs_fp32"] = diff("fp16")
    out["fp16_vs_fp32"]["mlups_ratio"] = round(out["fp16"]["mlups"] / out["fp32"]["mlups"], 3)
    out["fp32_rerun_vs_fp32"] = diff("fp32_rerun")
    return out


def run_form(torch, wl, form, warmup, steps, traffic=None, lattice_passes=0):
    """`steps` graph-replayed whole steps of one storage form after `warmup`,
    then the same number of event-timed steps for the per-kernel split.
    Returns MLUPS, ms per step, per-kernel ms per step, and the roofline block
    of the fused collide kernel: its algorithmic bytes per launch over its
    average launch duration (HIP events on the library's stream).
    lattice_passes as in lbm_params (0: the library's choice)."""
    from paper_1904_11386_amd.binding import LBM_FP16, LBM_FP32, sim_from_workload
    N = wl.n_lattice
    sim = sim_from_workload(wl, precision=LBM_FP16 if form == "fp16" else LBM_FP32, lattice_passes=lattice_passes)
    sim.step(warmup)
    sim.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = sim.step_timed(steps)
    obs = sim.observables()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    mlups = N * steps / wall / 1e6
    t_col = kms["collide"] / steps * 1e-3
    t_den = kms["density"] / steps * 1e-3
    # (the density group launches nothing when the collide forms the densities)
    one = t_den == 0.0
    bpl = ONE_PASS_BYTES_PER_LUP if one else COLLIDE_BYTES_PER_LUP[form]
    lattice_bytes = bpl if one else bpl + DENSITY_BYTES_PER_LUP[form]
    achieved = bpl * N / t_col / 1e9
    m0 = np.array([wl.rhoA.astype(np.float64).sum(), wl.rhoB.astype(np.float64).sum()])
    return {
        "mlups": round(mlups, 2), "ms_per_step": round(wall / steps * 1e3, 5), "wall_s": wall,
        "lattice_passes": 1 if one else 2,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_collide (%s storage, %s)" % (form, "one lattice pass" if one else "two passes"),
                     "bytes_per_launch": bpl * N, "bytes_per_lup": bpl, "avg_launch_ms": round(t_col * 1e3, 5)},
        "density_pass_gbs": None if one else round(DENSITY_BYTES_PER_LUP[form] * N / t_den / 1e9, 1),
        # whole step: MLUPS times the lattice passes' algorithmic bytes, over the peak
        "effective_hbm_frac": round(mlups * 1e6 * lattice_bytes / 1e9 / HBM_PEAK_GBS, 4),
        # the same against the one-pass minimum of the method (304 B), for every form alike
        "effective_hbm_frac_vs_one_pass_min": round(mlups * 1e6 * ONE_PASS_BYTES_PER_LUP / 1e9 / HBM_PEAK_GBS, 4),
        "fp64_mass_drift": float(np.abs(obs["mass"] / m0 - 1).max()),
        "kernels_ms_per_step": {k: round(v / steps, 5) for k, v in kms.items()},
    }


def bb_leg(torch, name="c2", warmup=30, steps=300, v=(0.01, 0.0, 0.0)):
    """The benchmark's 128^3 workload (8 capsules of 2562 nodes on the
    interface, angles in [60, 120] deg) under the paper's bounce-back
    coupling, FP32, the capsules translated along the interface at a
    prescribed velocity v (the set-up of the paper's mass-conservation test;
    free capsules of these soft 2562-node membranes leave their label boxes
    within about 100 steps under this coupling): MLUPS, ms per step and the
    per-group split of as many event-timed steps.  The coupling's head
    (labels, link list, fresh nodes, the bounce-back of the crossing
    populations, tile flags) is timed as "bb_head", the Shan-Chen sum across
    the membranes as "bb_shan_chen" and the node update as "bb_advance"."""
    from paper_1904_11386_amd import workloads
    from paper_1904_11386_amd.binding import LBM_FP32, LbmError, sim_from_workload
    wl = workloads.bounce_back(workloads.make(name))
    N = wl.n_lattice
    print("bench: bounce-back leg, %s, %d warm-up + %d timed steps" % (name, warmup, steps), file=sys.stderr, flush=True)
    sim = sim_from_workload(wl, precision=LBM_FP32)
    try:
        sim.set_velocity(0, [v] * len(wl.capsules), prescribed=True)
        ob0 = sim.observables()
        sim.step(warmup)
        sim.synchronize()
        torch.cuda.synchronize()
        print("bench: bounce-back leg warmed up", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        sim.step(steps)
        sim.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        print("bench: bounce-back leg timed, %.3f ms per step" % (wall / steps * 1e3), file=sys.stderr, flush=True)
        kms = sim.step_timed(steps)
        ob = sim.observables()
    except LbmError as e:
        # (the coupling reports an unstable run instead of stepping on)
        return {"workload": WORKLOAD_TEXT.get(name, name) + ", bounce-back coupling", "error": str(e)}
    finally:
        sim.close()
        del sim
        torch.cuda.empty_cache()
    rename = {"clear": "bb_head", "spread": "bb_shan_chen", "interp": "bb_advance"}
    t_col = kms["collide"] / steps * 1e-3
    achieved = COLLIDE_BYTES_PER_LUP["fp32"] * N / t_col / 1e9
    return {"workload": WORKLOAD_TEXT.get(name, name) + ", bounce-back coupling (node mass 5, C0 2500), "
                        "capsules translated at a prescribed %s lu/step" % (list(v),),
            "lattice": [wl.nx, wl.ny, wl.nz], "capsules": len(wl.capsules), "warmup": warmup, "steps": steps,
            "mlups": round(N * steps / wall / 1e6, 2), "ms_per_step": round(wall / steps * 1e3, 5),
            "collide_gbs": round(achieved, 1), "collide_frac": round(achieved / HBM_PEAK_GBS, 4),
            "kernels_ms_per_step": {rename.get(k, k): round(v / steps, 5) for k, v in kms.items() if v > 0},
            "mass_change": (ob["mass"] / ob0["mass"] - 1).tolist(),
            "capsule_height_change": [round(c1["com"][2] - c0["com"][2], 4) for c0, c1 in zip(ob0["caps"], ob["caps"])]}


def bb_contact_angle_leg(torch, colours=(0.30, 0.0, -0.30, 0.61), steps=40000, chunk=5000, R=10.0, psi_kind=1,
                         n=64, freq=16, rho=(0.7, 0.042), kS=0.5, node_mass=200.0, wet_scale=1.0):
    """The contact-angle law of the paper's coupling (Sec. III.D: a rigid
    particle's centre sits R cos(theta) from the interface, cos(theta) =
    colour): an n^3 flat interface (A below) relaxed for 3000 steps without a
    capsule; in those densities a free, stiff capsule (kS 0.5, node mass 200;
    its inside set to the relaxed A phase) placed with its centre at
    -R colour from the interface, then `steps` free steps; its offset dz from
    the interface far from it every `chunk` steps (positive colour prefers A,
    below, so the law puts dz at -R colour).  Defaults: the paper's R0 = 10
    (2562 nodes) and fluid (psi = 1 - exp(-rho), G 3.6, densities 0.7 and
    0.042) in a 64^3 box.  The mass check runs every 1000 steps at 1e-2 and
    the drift is reported."""
    import dataclasses
    import math
    from paper_1904_11386_amd import workloads
    from paper_1904_11386_amd.binding import LbmError, sim_from_workload

    def far_interface(ra, rb):
        zs = []
        for (y, x) in ((0, 0), (0, n // 2), (n // 2, 0), (n // 4, 3 * n // 4), (3 * n // 4, n // 4)):
            col = (ra[:, y, x] - rb[:, y, x]).astype(np.float64)
            for z in range(n // 6, 5 * n // 6):
                if col[z] > 0 >= col[z + 1]:
                    zs.append(z + col[z] / (col[z] - col[z + 1]))
        return float(np.mean(zs)) if zs else float("nan")

    print("bench: bounce-back contact-angle leg", file=sys.stderr, flush=True)
    base = dataclasses.replace(workloads.bb_capsule(nx=n, ny=n, nz=n, layered_z=n // 2, rho=rho), psi_kind=psi_kind)
    g = sim_from_workload(dataclasses.replace(base, capsules=[], coupling=0))
    g.step(3000)
    ra0, rb0, _ = g.fields()
    g.close()
    zi = far_interface(ra0, rb0)
    amaj, bmin = float(ra0[5, 0, 0]), float(rb0[5, 0, 0])
    out = {"workload": "%d^3 periodic box, flat interface (A below, relaxed 3000 steps), one free capsule R=%g "
                       "(%d nodes), kS %g, node mass %g, C0 2500, psi %s, densities %g/%g, G 3.6, colour offset "
                       "x %g" % (n, R, 10 * freq * freq + 2, kS, node_mass, "1 - exp(-rho)" if psi_kind else "rho",
                                 rho[0], rho[1], wet_scale),
           "steps": steps, "interface_z": round(zi, 3), "A_phase": [round(amaj, 4), round(bmin, 4)], "runs": []}
    gz = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    for colour in colours:
        theta = math.degrees(math.acos(colour))
        wl = workloads.bb_capsule(nx=n, ny=n, nz=n, centre=(n / 2 - 0.63, n / 2 + 0.61, zi - R * colour), radius=R,
                                  freq=freq, theta=theta, kS=kS, layered_z=n // 2, node_mass=node_mass,
                                  psi_kind=psi_kind, rho=rho, wet_scale=wet_scale)
        c = wl.capsules[0].centre
        ins = (gz[2] - c[0]) ** 2 + (gz[1] - c[1]) ** 2 + (gz[0] - c[2]) ** 2 < (R - 0.3) ** 2
        wl = dataclasses.replace(wl, rhoA=np.ascontiguousarray(np.where(ins, np.float32(amaj), ra0), np.float32),
                                 rhoB=np.ascontiguousarray(np.where(ins, np.float32(bmin), rb0), np.float32))
        m0 = np.array([wl.rhoA.astype(np.float64).sum(), wl.rhoB.astype(np.float64).sum()])
        g = sim_from_workload(wl, check_every=1000, mass_tol=1e-2)
        trace, err = [], None
        try:
            for k in range(steps // chunk):
                g.step(chunk)
                ra, rb, _ = g.fields()
                trace.append(round(g.observables()["caps"][0]["com"][2] - far_interface(ra, rb), 3))
                print("bench: contact angle, colour %+.3f, step %d, dz %.3f" % (colour, (k + 1) * chunk, trace[-1]),
                      file=sys.stderr, flush=True)
        except LbmError as e:
            err = str(e)
        drift = float(np.abs(g.observables()["mass"] / m0 - 1).max())
        g.close()
        last = float(np.mean(trace[-2:])) if len(trace) >= 2 else float("nan")
        out["runs"].append({"colour": colour, "theta_deg": round(theta, 2), "dz_start": round(-R * colour, 3),
                            "dz_trace": trace, "cos_theta_measured": round(-last / R, 3), "mass_drift": drift,
                            "error": err})
        torch.cuda.empty_cache()
    return out


def bb_mass_leg(torch, c0s=(0.0, 500.0, 2500.0, 5000.0), colours=(0.0, 0.30, 0.61), steps=250000,
                chunk=25000, R=10.0, psi_kind=1, rho=(0.7, 0.042), wet_scale=1.0, mass_fix=False):
    """The mass-conservation test of the paper's coupling (Sec. II.E, Fig.
    mass-conservation): a sphere of radius 10 (2562 nodes) at a flat interface
    of a (180, 60, 60) box, every node moved at a prescribed 1e-3 lu/step
    along x (rigid translation), for 250 000 steps (a whole number of lattice
    units); the relative change of each component's mass against the
    correction's strength C0 and the particle colour (the preferred phase A
    below; the sphere's centre at the contact-angle law's height, its inside
    filled with the lower fluid's composition).  Fluid parameters of the
    paper's results (Sec. III): psi = 1 - exp(-rho), G = 3.6, majority and
    minority densities 0.7 and 0.042.  Each run also reports the library's
    FP64 ledger of the coupling's own mass changes (the change an exact
    storage would show); the rest of the lattice's change is the FP32
    storage's rounding.  The paper reports below 1e-4 for every component
    once C0 >= 2500."""
    import math
    from paper_1904_11386_amd import workloads
    from paper_1904_11386_amd.binding import LbmError, sim_from_workload
    out = {"workload": "(180, 60, 60) periodic box, flat interface at z=29.5 (A below), sphere R=10 (2562 nodes) "
                       "translated at 1e-3 lu/step along x, bounce-back coupling, FP32, psi %s, rho %s/%s, G 3.6, "
                       "colour offset x %g%s" % ("1 - exp(-rho)" if psi_kind else "rho", rho[0], rho[1], wet_scale,
                                                 ", FP32 mass compensated every 1000 steps" if mass_fix else ""),
           "steps": steps, "runs": []}
    for colour in colours:
        for c0 in c0s:
            wl = workloads.bb_capsule(nx=180, ny=60, nz=60, centre=(90.37, 30.61, 29.5 - R * colour), radius=R,
                                      freq=16, theta=math.degrees(math.acos(colour)), kS=0.05, layered_z=30,
                                      v=(1e-3, 0.0, 0.0), prescribed=True, C0=c0, interior=rho, rho=rho,
                                      psi_kind=psi_kind, wet_scale=wet_scale)
            m0 = np.array([wl.rhoA.astype(np.float64).sum(), wl.rhoB.astype(np.float64).sum()])
            # mass_fix: the FP32 storage compensated to the initial mass plus the ledger every 1000 steps
            g = sim_from_workload(wl, check_every=1000 if mass_fix else 0, mass_fix=int(mass_fix), mass_tol=0.1)
            err = None
            t0 = time.perf_counter()
            try:
                for k in range(steps // chunk):
                    g.step(chunk)
                    ob = g.observables()
                    print("bench: mass leg, colour %.2f, C0 %g, step %d, rel mass change %s, ledger %s" % (
                        colour, c0, (k + 1) * chunk, np.round(ob["mass"] / m0 - 1, 7).tolist(),
                        np.round(ob["mass_ledger"] / m0, 7).tolist()), file=sys.stderr, flush=True)
            except LbmError as e:
                err = str(e)
            ob = g.observables()
            wall = time.perf_counter() - t0
            g.close()
            torch.cuda.empty_cache()
            rel = (ob["mass"] / m0 - 1).tolist()
            led = (ob["mass_ledger"] / m0).tolist()
            # the preferred component is A for a positive colour
            out["runs"].append({"colour": colour, "C0": c0, "rel_mass_change_A": rel[0], "rel_mass_change_B": rel[1],
                                "rel_ledger_A": led[0], "rel_ledger_B": led[1],
                                "ms_per_step": round(wall / steps * 1e3, 4), "error": err})
    return out


def ratio_leg(torch, name, warmup, steps):
    """Both storage forms of one workload, same step counts: MLUPS, collide
    bandwidth and the FP16/FP32 ratio."""
    from paper_1904_11386_amd import workloads
    wl = workloads.make(name)
    out = {"workload": WORKLOAD_TEXT.get(name, name), "lattice": [wl.nx, wl.ny, wl.nz],
           "capsules": len(wl.capsules), "warmup": warmup, "steps": steps}
    for form in ("fp32", "fp16"):
        print("bench: %s leg, %s form" % (name, form), file=sys.stderr, flush=True)
        r = run_form(torch, wl, form, warmup, steps)
        out[form] = {"mlups": r["mlups"], "ms_per_step": r["ms_per_step"], "lattice_passes": r["lattice_passes"],
                     "collide_gbs": r["roofline"]["achieved"], "collide_frac": r["roofline"]["frac"],
                     "effective_hbm_frac": r["effective_hbm_frac"], "kernels_ms_per_step": r["kernels_ms_per_step"]}
    out["fp16_over_fp32"] = round(out["fp16"]["mlups"] / out["fp32"]["mlups"], 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="c5",
                    help="headline workload (default: the 512^3 throughput-at-scale configuration)")
    ap.add_argument("--forms", default="both", choices=["both", "fp32", "fp16"],
                    help="storage forms of the headline workload (fp32 alone for counter runs of one kernel)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline workload's storage forms (for profiling that configuration)")
    ap.add_argument("--no-c3-leg", action="store_true", help="skip the 256^3 FP16/FP32 leg")
    ap.add_argument("--no-c2-leg", action="store_true", help="skip the 128^3 leg")
    ap.add_argument("--no-two-pass-leg", action="store_true",
                    help="skip the headline workload's FP32 form in two lattice passes")
    ap.add_argument("--no-adjoint-leg", action="store_true")
    ap.add_argument("--no-bb-leg", action="store_true",
                    help="skip the 128^3 workload under the paper's bounce-back coupling")
    ap.add_argument("--bb-leg", action="store_true",
                    help="run the bounce-back leg even with --headline-only")
    ap.add_argument("--bb-mass-leg", action="store_true",
                    help="also run the paper's mass-conservation test of the bounce-back coupling (250 000 steps "
                         "for each mass-correction strength and colour)")
    ap.add_argument("--colour-offset-scale", type=float, default=1.0,
                    help="scale of the colour offset (wet_scale) in the bounce-back mass and contact-angle legs: 1 = "
                         "the normalisation as written, 0.25 = the one that reproduces the paper's contact-angle law")
    ap.add_argument("--fp32-mass-fix", action="store_true",
                    help="the bounce-back mass leg with the FP32 storage's mass compensation (mass_fix)")
    ap.add_argument("--bb-shape-leg", action="store_true",
                    help="also run the shape errors of Sec. III.B under the bounce-back coupling with the paper's "
                         "fluid (beta 100, 316, 1000; kV 20)")
    ap.add_argument("--bb-contact-angle-leg", action="store_true",
                    help="also measure the rest position of free capsules on a flat interface under the bounce-back "
                         "coupling against the paper's contact-angle law")
    ap.add_argument("--no-fd-sweep", action="store_true",
                    help="skip the full-size adjoint check against FP32 central differences")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-timing-leg", action="store_true",
                    help="also time the FP64 oracle on the 32^3 case (1000 steps) and the 64^3 cases (50 steps)")
    ap.add_argument("--reference-sweep-leg", action="store_true",
                    help="also sweep the reference model over softness, surface Poisson ratio and interface width")
    ap.add_argument("--extras-leg", action="store_true",
                    help="also time short runs of the on-site boundaries, reference model, bending and repulsion")
    ap.add_argument("--shear-leg", action="store_true",
                    help="also run the capsule-in-shear workload (on-site boundaries) at five capillary numbers")
    ap.add_argument("--shape-error-leg", action="store_true",
                    help="also relax a capsule with the reference model and couple the same capsule at a fluid "
                         "interface, and report the shape errors between the two")
    ap.add_argument("--reference-model-leg", action="store_true",
                    help="also relax a capsule with the LBM-free reference model (no fluid)")
    ap.add_argument("--membrane-extras-leg", action="store_true",
                    help="also run the 512^3 configuration with bending and particle-particle repulsion on")
    ap.add_argument("--precision-study", type=int, default=0, metavar="STEPS",
                    help="also run the FP16/FP32 precision study on the 256^3 droplet for STEPS steps")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the step would shard by z-slabs, one per GPU, with one halo exchange per step).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1904_11386_amd import workloads

    wl = workloads.make(args.workload)
    print("bench: workload %s %dx%dx%d, %d capsules, %d nodes" %
          (args.workload, wl.nx, wl.ny, wl.nz, len(wl.capsules), int(wl.meshes()[0].sum())),
          file=sys.stderr, flush=True)
    copy_gbs = copy_ceiling(torch)
    forms = ("fp32", "fp16") if args.forms == "both" else (args.forms,)
    res = {}
    for form in forms:
        print("bench: %s, %s form, %d warm-up + %d timed steps" % (args.workload, form, args.warmup, args.steps),
              file=sys.stderr, flush=True)
        res[form] = run_form(torch, wl, form, args.warmup, args.steps,
                             traffic=measured_traffic(args.workload, form))
    head = res[forms[0]]
    out = {
        "metric": METRIC, "value": head["mlups"], "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "storage": "f16 (g = f/rho - w)" if forms[0] == "fp16" else "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT.get(args.workload, args.workload), "name": args.workload,
                   "lattice": [wl.nx, wl.ny, wl.nz], "capsules": len(wl.capsules),
                   "membrane_nodes": int(wl.meshes()[0].sum()), "storage": forms[0],
                   "lattice_passes": head["lattice_passes"]},
        "roofline": head["roofline"],
        "kernels_ms_per_step": head["kernels_ms_per_step"],
        "density_pass_gbs": head["density_pass_gbs"],
        "copy_ceiling_gbs": round(copy_gbs, 1),
        "collide_frac_of_copy": round(head["roofline"]["achieved"] / copy_gbs, 4),
        "effective_hbm_frac": head["effective_hbm_frac"],
        "effective_hbm_frac_vs_one_pass_min": head["effective_hbm_frac_vs_one_pass_min"],
        "fp64_mass_drift": head["fp64_mass_drift"],
    }
    if "fp16" in res and forms[0] == "fp32":
        r16 = res["fp16"]
        out["fp16_form"] = {"value": r16["mlups"], "unit": "MLUPS", "ms_per_step": r16["ms_per_step"],
                            "ratio_vs_fp32": round(r16["mlups"] / head["mlups"], 3),
                            "roofline": r16["roofline"], "density_pass_gbs": r16["density_pass_gbs"],
                            "effective_hbm_frac": r16["effective_hbm_frac"],
                            "fp64_mass_drift": r16["fp64_mass_drift"],
                            "kernels_ms_per_step": r16["kernels_ms_per_step"]}
    if not args.headline_only and not args.no_two_pass_leg and "fp32" in res and head["lattice_passes"] == 1:
        # the same FP32 steps with a density pass and the collide, for comparison
        print("bench: %s, fp32 form in two lattice passes" % args.workload, file=sys.stderr, flush=True)
        r2 = run_form(torch, wl, "fp32", args.warmup, args.steps, lattice_passes=2)
        out["fp32_two_passes"] = {"value": r2["mlups"], "unit": "MLUPS", "ms_per_step": r2["ms_per_step"],
                                  "one_pass_speedup": round(res["fp32"]["mlups"] / r2["mlups"], 3),
                                  "roofline": r2["roofline"], "density_pass_gbs": r2["density_pass_gbs"],
                                  "effective_hbm_frac": r2["effective_hbm_frac"],
                                  "effective_hbm_frac_vs_one_pass_min": r2["effective_hbm_frac_vs_one_pass_min"],
                                  "kernels_ms_per_step": r2["kernels_ms_per_step"]}
        if "fp16_form" in out:
            out["fp16_form"]["ratio_vs_fp32_two_passes"] = round(out["fp16_form"]["value"] / r2["mlups"], 3)
    if not args.headline_only:
        if not args.no_c3_leg and args.workload != "c3":
            out["c3_leg"] = ratio_leg(torch, "c3", 50, 200)
        if not args.no_c2_leg and args.workload != "c2":
            out["c2_leg"] = ratio_leg(torch, "c2", 30, 300)
        if not args.no_bb_leg:
            out["bb_leg"] = bb_leg(torch)
        if not args.no_adjoint_leg:
            out["adjoint"] = adjoint_leg(torch)
            if not args.no_fd_sweep:
                out["adjoint_fd_sweep"] = adjoint_fd_sweep(torch)
    if args.bb_leg and args.headline_only:
        out["bb_leg"] = bb_leg(torch)
    if args.bb_mass_leg:
        out["bb_mass"] = bb_mass_leg(torch, wet_scale=args.colour_offset_scale, mass_fix=args.fp32_mass_fix)
    if args.bb_shape_leg:
        out["bb_shape"] = shape_error_leg(torch, betas=(100.0, 316.0, 1000.0), kV=20.0, coupling=1)
    if args.bb_contact_angle_leg:
        out["bb_contact_angle"] = bb_contact_angle_leg(torch, wet_scale=args.colour_offset_scale)
    if args.reference_model_leg:
        out["reference_model"] = reference_model_leg(torch)
    if args.shape_error_leg:
        out["shape_error"] = shape_error_leg(torch)
    if args.shear_leg:
        out["shear"] = shear_leg(torch)
    if args.extras_leg:
        out["extras"] = extras_leg(torch)
    if args.reference_sweep_leg:
        out["reference_sweep"] = reference_sweep_leg(torch)
    if args.membrane_extras_leg:
        out["membrane_extras"] = membrane_extras_leg(torch)
    if args.precision_study > 0:
        out["precision_study"] = precision_study(torch, args.precision_study)
    if args.oracle_timing_leg:
        out["oracle_timing"] = oracle_timing_leg()
    if not args.no_cpu_baseline and not args.headline_only:
        print("bench: timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
