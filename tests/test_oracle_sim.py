"""Whole-step invariants of the FP64 oracle (no GPU)."""

import numpy as np
import pytest
import torch

from oracle import ibm
from oracle.sim import OracleSim, cos_deg
from paper_1904_11386_amd import workloads as W

DT = torch.float64


def _capsule_sim(theta, steps=0, walls=0, centre=(10.0, 10.0, 11.5), kV=2.0):
    ra, rb = W.layered(20, 20, 24, 12)
    xyz, tri = W.icosphere(4, 4.0)
    c = np.array(centre)
    s = OracleSim(ra.astype(np.float64), rb.astype(np.float64),
                  [dict(xyz=xyz + c, tri=tri, kS=0.01, C=0.0, kV=kV, theta=theta)],
                  G=3.6, z_interface=11.5, walls=walls)
    return s.run(steps)


def test_mass_and_momentum_conserved_with_wetting():
    s = _capsule_sim(60.0)
    m0 = s.mass().clone()
    p0 = s.momentum().clone()
    s.run(60)
    assert torch.allclose(s.mass(), m0, rtol=1e-13, atol=0)
    scale = float(m0.sum())
    assert float((s.momentum() - p0).abs().max()) < 1e-15 * scale
    # the wetting term did act: the fluid force is not the pure Shan-Chen one
    assert float(s.phi_last[0].abs().max()) > 0.01


def test_wetting_phi_partition_of_unity_and_colour_law(golden):
    s = _capsule_sim(60.0, steps=1)
    rv = 2 * cos_deg(60.0) * (0.7 - 0.04)
    A = float(s.caps[0]["mesh"].A0.sum())
    assert float(s.phi_last[0].sum()) == pytest.approx(rv * A, rel=1e-13)
    assert float(s.phi_last[1].abs().max()) == 0.0
    # colour = rho_v / (2 (maj - min)) = cos(theta): theta = acos(colour)
    assert np.degrees(np.arccos(rv / (2 * (0.7 - 0.04)))) == pytest.approx(60.0, abs=1e-12)
    s = _capsule_sim(120.0, steps=1)
    assert float(s.phi_last[1].sum()) == pytest.approx(abs(rv) * A, rel=1e-13)


def test_neutral_capsule_symmetry_and_wetting_direction():
    """Mirror z -> 23 - z with A <-> B swap is a symmetry of the layered box
    and a capsule centred on the mid-plane 11.5: a neutral capsule keeps its
    height, and theta and 180 - theta give opposite heights.  A capsule that
    prefers A (theta < 90) moves into A, below the interface."""
    s90 = _capsule_sim(90.0, steps=60)
    assert abs(float(s90.capsule_obs(0)["height"])) < 1e-10
    assert float(s90.phi_last.abs().max()) == 0.0
    s60 = _capsule_sim(60.0, steps=60)
    s120 = _capsule_sim(120.0, steps=60)
    h60 = float(s60.capsule_obs(0)["height"])
    h120 = float(s120.capsule_obs(0)["height"])
    assert h60 < -0.5
    assert h60 == pytest.approx(-h120, abs=1e-10)


def test_flat_interface_unchanged_by_neutral_zero_stiffness_capsule_at_rest():
    """With G = 0, uniform fluid and a capsule at rest nothing moves."""
    rho = np.full((12, 12, 12), 0.37)
    xyz, tri = W.icosphere(4, 3.0)
    s = OracleSim(rho, rho, [dict(xyz=xyz + 6.0, tri=tri, kS=0.01, C=1.0, kV=2.0, theta=90.0)], G=0.0)
    s.run(20)
    assert float((s.X[0] - torch.tensor(xyz + 6.0)).abs().max()) == 0.0
    assert float(s.u_last.abs().max()) < 1e-18


def test_exponential_pseudo_potential_step_conserves_mass_and_momentum():
    """With psi = 1 - exp(-rho) and wetting capsules the coupled step still
    conserves mass and fluid momentum (the Shan-Chen forces are
    antisymmetric for any psi; the virtual density enters linearly)."""
    import dataclasses
    from oracle.sim import from_workload
    wl = dataclasses.replace(W.small(nx=20, ny=18, nz=22, ncap=2, theta=(60.0, 120.0)), psi_kind=1)
    s = from_workload(wl)
    m0, p0 = s.mass().clone(), s.momentum().clone()
    s.run(30)
    assert torch.allclose(s.mass(), m0, rtol=1e-13, atol=0)
    assert float((s.momentum() - p0).abs().max()) < 1e-15 * float(m0.sum())
    # and the pseudo-potential matters: a psi = rho run differs
    s0 = from_workload(dataclasses.replace(wl, psi_kind=0)).run(30)
    assert float((s.rho_last - s0.rho_last).abs().max()) > 1e-4
