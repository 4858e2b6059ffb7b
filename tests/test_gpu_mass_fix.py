"""FP64 mass compensation of the FP32 storage (lbm_params.mass_fix): at
each mass check the populations of each component are scaled to the
intended mass, the initial mass plus (bounce-back coupling) the coupling's
own change.  Right after a check the stored FP64 mass equals it to the
rounding of the scaling.  The mass the paper's coupling changes is Sec. II.E
(eqs. method:freshnodes, method:masscorrection); the immersed boundary
changes none."""

import sys

import numpy as np
import pytest

from paper_1904_11386_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(wl, steps, every, fix):
    """The intended initial mass is the FP64 sum of the densities given to
    the library (its FP32 rest populations represent it to FP32 rounding)."""
    from paper_1904_11386_amd.binding import sim_from_workload
    g = sim_from_workload(wl, check_every=every, mass_fix=fix, mass_tol=1e-2)
    m0 = np.array([wl.rhoA.astype(np.float64).sum(), wl.rhoB.astype(np.float64).sum()])
    g.step(steps)
    ob = g.observables()
    g.close()
    return m0, ob


def test_bounce_back_lattice_mass_equals_initial_plus_ledger():
    wl = W.bb_capsule(nx=40, ny=36, nz=44, centre=(19.37, 17.61, 18.83), radius=6.0, freq=8, theta=60.0,
                      layered_z=22, v=(0.01, 0.0, 0.0), prescribed=True, interior=(0.7, 0.042), rho=(0.7, 0.042),
                      psi_kind=1)
    for fix in (0, 1):
        m0, ob = _run(wl, 4000, 500, fix)
        gap = (ob["mass"] - m0 - ob["mass_ledger"]) / m0
        _say("mass_fix %d: lattice - initial - ledger, relative: %s; ledger %s" % (
            fix, gap.tolist(), (ob["mass_ledger"] / m0).tolist()))
        if fix:
            assert np.abs(gap).max() < 2e-7
            assert np.abs(ob["mass_ledger"] / m0).max() > 1e-6        # (the coupling did change the masses)


def test_immersed_boundary_fp32_mass_held_at_start():
    wl = W.small(nx=40, ny=36, nz=44, ncap=3)
    m0, ob = _run(wl, 2000, 200, 1)
    rel = (ob["mass"] - m0) / m0
    _say("immersed boundary, mass_fix: relative mass change %s" % rel.tolist())
    assert np.abs(rel).max() < 2e-7
    assert np.all(ob["mass_ledger"] == 0.0)
