"""One lattice pass per step (lbm_params.lattice_passes = 1).

The collide forms the step's densities rho^n(x) = sum_i f*_i(x - c_i)
(Sec. II.A) for its block and a one-node halo from the populations it
pulls, instead of reading them from a density pass; the tiles that the
immersed boundary touches get a density pass of their own, which the
wettability reaction of the spreading reads (Sec. II.D, the colour term
on the membrane).  The sums are the two passes' own, so the Shan-Chen
force (Sec. II.D, eq. method:shanchen) and the collision see the same
values bit for bit: with the deterministic spreading a run in one pass
equals a run in two passes exactly, fields, velocities, lattice force and
virtual-density fields, node positions and node forces.  Each form is also
held to the oracle's bounds of the default step."""

import dataclasses
import sys

import numpy as np
import pytest
import torch

from oracle.sim import from_workload
from paper_1904_11386_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)).max()
                 / max(np.abs(np.asarray(b, np.float64)).max(), 1e-300))


def _partial_tiles():
    # lattice edges of 8k+1 cells with a capsule across the periodic wrap:
    # the tile density pass widens each tile by one cell
    wl = W.small(nx=33, ny=33, nz=38, ncap=2, theta=(60.0, 110.0), wet_scale=0.5)
    wl.capsules[0].centre = W._snap(np.array([32.3, 32.4, wl.z_interface + 0.7]))
    wl.capsules[1].centre = W._snap(np.array([14.2, 15.1, wl.z_interface - 0.6]))
    return wl


CASES = {
    "fluid only, ragged box": lambda: W.small(nx=40, ny=36, nz=44, ncap=0),
    "fluid only, two tau, weak G": lambda: W.small(nx=24, ny=20, nz=28, ncap=0, tau=(0.8, 1.3), G=2.5),
    "three wetting capsules, ragged box": lambda: W.small(nx=40, ny=36, nz=44, ncap=3),
    "capsules across one-cell partial tiles": _partial_tiles,
    "psi = 1 - exp(-rho) with wetting capsules": lambda: dataclasses.replace(
        W.small(nx=40, ny=36, nz=44, ncap=2, theta=(60.0, 120.0)), psi_kind=1),
    "pressed capsules with repulsion": lambda: W.pressed(),
    "64^3 crop of the 128^3 workload (tile-aligned)": lambda: W.make("c2_64"),
}


def _state(g, caps):
    ra, rb, u = g.fields()
    F, ph = g.spread()
    s = {"rhoA": ra, "rhoB": rb, "u": u, "F_ib": F, "phi": ph}
    if caps:
        s["X"] = g.nodes()
        s["node_F"] = g.node_forces()
    return s


def _run(wl, steps, **kw):
    from paper_1904_11386_amd.binding import sim_from_workload
    g = sim_from_workload(wl, **kw)
    g.step(steps)
    s = _state(g, len(wl.capsules) > 0)
    g.close()
    return s


@pytest.mark.parametrize("case", list(CASES))
def test_one_pass_equals_two_passes_bit_for_bit(case):
    wl = CASES[case]()
    steps = 40
    _say("case", case, (wl.nx, wl.ny, wl.nz), "caps", len(wl.capsules), "steps", steps)
    a = _run(wl, steps, deterministic=1, lattice_passes=1)
    b = _run(wl, steps, deterministic=1, lattice_passes=2)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    # and the step moved: not a trivially equal state
    assert float(np.abs(a["u"]).max()) > 0.0


@pytest.mark.parametrize("case,steps,tol_rho,tol_x", [
    ("fluid only, ragged box", 100, 2e-6, None),
    ("three wetting capsules, ragged box", 60, 5e-6, 2e-5),
    ("psi = 1 - exp(-rho) with wetting capsules", 100, 5e-6, 2e-5),
])
def test_one_pass_oracle_parity(case, steps, tol_rho, tol_x):
    """The default (atomic) spreading in one pass against the FP64 oracle,
    the bounds of the two-pass parity tests."""
    from paper_1904_11386_amd.binding import sim_from_workload
    wl = CASES[case]()
    _say("case", case, "one pass", steps, "steps")
    g = sim_from_workload(wl, lattice_passes=1)
    g.step(steps)
    o = from_workload(wl)
    umax = 0.0
    for _ in range(steps):
        o.step()
        umax = max(umax, float(o.u_last.abs().max()))
    ra, rb, u = g.fields()
    ea, eb = _rel(ra, o.rho_last[0].numpy()), _rel(rb, o.rho_last[1].numpy())
    du = float(np.abs(u - o.u_last.numpy()).max())
    _say("  rho rel err %.3e %.3e  du/U %.3e" % (ea, eb, du / umax))
    assert ea <= tol_rho and eb <= tol_rho and du <= 1e-5 * umax
    if tol_x is not None:
        dx = float(np.abs(g.nodes() - torch.cat(o.X, 0).numpy()).max())
        _say("  node position err %.3e lu" % dx)
        assert dx <= tol_x
    g.close()


def test_one_pass_step_timing_groups():
    """lbm_step_timed in one pass: the density group launches nothing and
    reads 0; the collide and the spreading (which holds the tile density
    pass) take time."""
    from paper_1904_11386_amd.binding import sim_from_workload
    wl = W.small(nx=40, ny=36, nz=44, ncap=2)
    g = sim_from_workload(wl, lattice_passes=1)
    g.step(2)
    t = g.step_timed(4)
    _say("  groups (ms per step):", {k: round(v, 4) for k, v in t.items()})
    assert t["density"] == 0.0
    assert t["collide"] > 0.0 and t["spread"] > 0.0
    g.close()


def test_one_pass_checkpoint_replay_bit_identical():
    """N steps, save, M steps; load, the same M steps again: the same state
    bit for bit under the deterministic spreading (the state slot holds the
    populations and nodes; one pass leaves the density field written on the
    touched tiles only, and nothing it reads depends on the rest)."""
    from paper_1904_11386_amd.binding import sim_from_workload
    wl = W.small(nx=40, ny=36, nz=44, ncap=3)
    g = sim_from_workload(wl, lattice_passes=1, deterministic=1, n_slots=1)
    g.step(30)
    g.save(0)
    g.step(20)
    a = _state(g, True)
    g.load(0)
    g.step(20)
    b = _state(g, True)
    g.close()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_one_pass_with_mass_fix_holds_the_mass():
    """FP32 mass compensation at the mass checks in one pass: after 2000
    steps with checks every 200 the FP64 masses equal the initial ones to
    the rounding of the scaling, as in two passes."""
    from paper_1904_11386_amd.binding import sim_from_workload
    wl = W.small(nx=40, ny=36, nz=44, ncap=3)
    m0 = np.array([wl.rhoA.astype(np.float64).sum(), wl.rhoB.astype(np.float64).sum()])
    g = sim_from_workload(wl, lattice_passes=1, check_every=200, mass_fix=1, mass_tol=1e-2)
    g.step(2000)
    rel = (g.observables()["mass"] - m0) / m0
    g.close()
    _say("  one pass, mass_fix: relative mass change %s" % rel.tolist())
    assert np.abs(rel).max() < 2e-7
