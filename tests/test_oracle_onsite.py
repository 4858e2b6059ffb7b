"""Pins of the on-site velocity boundaries in the oracle (oracle/lattice.py,
onsite_closure; the boundaries of the paper's shear-flow case, Sec. III.A):
the boundary nodes take the wall velocity exactly, a fluid at rest stays at
rest, and the steady Couette profile between the boundary rows is the exact
linear one."""

import pytest
import torch

from oracle import lattice as L
from oracle.sim import OracleSim

DT = torch.float64


def test_closure_gives_boundary_nodes_the_wall_velocity():
    g = torch.Generator().manual_seed(11)
    f = 0.01 + 0.05 * torch.rand(2, 19, 3, 6, 5, generator=g, dtype=DT)
    u_lo, u_hi = (0.013, 0.0, -0.004), (-0.008, 0.0, 0.011)
    out = L.onsite_closure(f, u_lo, u_hi)
    rho, j = L.moments(out)
    for yb, uw in ((0, u_lo), (5, u_hi)):
        for a in range(3):
            got = j[:, a, :, yb, :] / rho[:, :, yb, :]
            assert torch.allclose(got, torch.full_like(got, uw[a]), rtol=0, atol=1e-15), (yb, a)
    # interior rows untouched, and only the unknown populations change
    assert torch.equal(out[:, :, :, 1:5], f[:, :, :, 1:5])
    for i in range(19):
        cy = int(L.C[i][1])
        if cy != 1:
            assert torch.equal(out[:, i, :, 0], f[:, i, :, 0]), i
        if cy != -1:
            assert torch.equal(out[:, i, :, 5], f[:, i, :, 5]), i


def test_closure_with_normal_velocity_keeps_the_moments():
    g = torch.Generator().manual_seed(12)
    f = 0.01 + 0.05 * torch.rand(1, 19, 2, 4, 3, generator=g, dtype=DT)
    u_lo, u_hi = (0.002, 0.01, 0.0), (0.0, 0.01, -0.003)
    rho, j = L.moments(L.onsite_closure(f, u_lo, u_hi))
    for yb, uw in ((0, u_lo), (3, u_hi)):
        u = j[:, :, :, yb, :] / rho[:, None, :, yb, :]
        for a in range(3):
            assert torch.allclose(u[:, a], torch.full_like(u[:, a], uw[a]), rtol=0, atol=1e-15)


def test_fluid_at_rest_stays_at_rest():
    rho = torch.full((3, 8, 4), 0.6, dtype=DT)
    s = OracleSim(rho, 0.5 * rho, [], tau=(1.0, 0.8), G=0.0, walls=2)
    f0 = s.fpost.clone()
    s.run(40)
    assert torch.allclose(s.fpost, f0, rtol=0, atol=1e-15)


def test_couette_between_onsite_boundaries_is_linear():
    """Steady shear between the boundary rows, which move at -+0.01: u_x is
    linear in y from node row 0 to node row ny - 1 and the other components
    vanish."""
    ny = 12
    rho = torch.full((2, ny, 2), 0.5, dtype=DT)
    s = OracleSim(rho, rho, [], tau=(1.2, 1.2), G=0.0, walls=2, u_lo=(-0.01, 0, 0), u_hi=(0.01, 0, 0))
    s.run(4000)
    y = torch.arange(ny, dtype=DT)
    exp = -0.01 + 0.02 * y / (ny - 1)
    got = s.u_last[0, 0, :, 0]
    assert torch.allclose(got, exp, rtol=0, atol=1e-10), (got - exp).abs().max()
    assert float(s.u_last[1:].abs().max()) < 1e-14


def test_shan_chen_sum_clamps_at_onsite_boundaries():
    """With on-site boundaries the neighbour beyond a boundary row is that
    row: a field constant in x and z and linear in y has the interior
    gradient sum inside and a one-sided one on the boundary rows."""
    ny = 6
    psi = torch.arange(ny, dtype=DT).view(1, ny, 1).expand(3, ny, 4).clone()
    S = L.sc_sum(psi, walls=2)
    # interior: sum_i w_i c_iy (y + c_iy) = sum_i w_i c_iy^2 = 1/3
    assert torch.allclose(S[1, :, 1:ny - 1], torch.full_like(S[1, :, 1:ny - 1], 1.0 / 3.0), atol=1e-15)
    # boundary rows: the neighbour beyond reads the row itself, half the sum
    assert torch.allclose(S[1, :, 0], torch.full_like(S[1, :, 0], 1.0 / 6.0), atol=1e-15)
    assert torch.allclose(S[1, :, ny - 1], torch.full_like(S[1, :, ny - 1], 1.0 / 6.0), atol=1e-15)
    assert float(S[0].abs().max()) == 0.0 and float(S[2].abs().max()) == 0.0
