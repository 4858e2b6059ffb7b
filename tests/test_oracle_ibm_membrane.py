"""Pins of the oracle's immersed-boundary and membrane parts (no GPU)."""

import math

import numpy as np
import pytest
import torch

from oracle import ibm, membrane
from paper_1904_11386_amd import workloads

DT = torch.float64


def test_peskin_delta_identities():
    g = torch.Generator().manual_seed(11)
    r = torch.rand(1000, generator=g, dtype=DT)
    k = torch.arange(4, dtype=DT)
    d = r.unsqueeze(1) + 1.0 - k.unsqueeze(0)
    phi = ibm.peskin4(d)
    assert torch.allclose(phi.sum(1), torch.ones(1000, dtype=DT), atol=1e-15)
    assert torch.allclose((phi * d).sum(1), torch.zeros(1000, dtype=DT), atol=1e-15)
    assert torch.allclose((phi * phi).sum(1), torch.full((1000,), 3.0 / 8.0, dtype=DT), atol=1e-15)
    # even and compactly supported, phi(0) = 1/2, phi(1) = 1/4
    assert float(ibm.peskin4(torch.tensor([0.0], dtype=DT))) == pytest.approx(0.5, abs=1e-16)
    assert float(ibm.peskin4(torch.tensor([1.0], dtype=DT))) == pytest.approx(0.25, abs=1e-16)
    assert float(ibm.peskin4(torch.tensor([2.0], dtype=DT))) == 0.0
    x = torch.linspace(-2.5, 2.5, 101, dtype=DT)
    assert torch.equal(ibm.peskin4(x), ibm.peskin4(-x))


def test_interpolation_exact_for_linear_fields_and_axis_order():
    nx, ny, nz = 13, 11, 9
    z, y, x = torch.meshgrid(torch.arange(nz, dtype=DT), torch.arange(ny, dtype=DT),
                             torch.arange(nx, dtype=DT), indexing="ij")
    field = torch.stack([0.3 * x + 0.1, -0.2 * y + 0.5, 0.7 * z - 0.3], 0)
    g = torch.Generator().manual_seed(2)
    X = torch.stack([2 + 8 * torch.rand(50, generator=g, dtype=DT),
                     2 + 6 * torch.rand(50, generator=g, dtype=DT),
                     2 + 4 * torch.rand(50, generator=g, dtype=DT)], 1)
    U = ibm.interpolate(field, X)
    exp = torch.stack([0.3 * X[:, 0] + 0.1, -0.2 * X[:, 1] + 0.5, 0.7 * X[:, 2] - 0.3], 1)
    assert torch.allclose(U, exp, atol=1e-13)


def test_spread_conserves_and_is_adjoint_of_interpolation():
    dims = (10, 9, 8)
    g = torch.Generator().manual_seed(4)
    X = torch.rand(40, 3, generator=g, dtype=DT) * torch.tensor(dims, dtype=DT)
    X[0] = torch.tensor([0.0, 8.999, 7.5], dtype=DT)          # wraps every axis
    F = torch.randn(40, 4, generator=g, dtype=DT)
    fld = ibm.spread(F, X, dims)
    assert torch.allclose(fld.sum((1, 2, 3)), F.sum(0), atol=1e-13)
    u = torch.randn(4, dims[2], dims[1], dims[0], generator=g, dtype=DT)
    lhs = (fld * u).sum()
    rhs = (F * ibm.interpolate(u, X)).sum()
    assert float(lhs) == pytest.approx(float(rhs), rel=1e-13)


def test_stencil_base_and_tile_indexing():
    X = torch.tensor([[0.0, 0.0, 0.0], [7.999, 8.0, 15.5], [-0.25, 31.75, 3.0]], dtype=DT)
    idx, wts, base = ibm.stencil(X, (32, 32, 32))
    assert base.tolist() == [[-1, -1, -1], [6, 7, 14], [-2, 30, 2]]
    assert idx[0][2].tolist() == [30, 31, 0, 1]
    t = ibm.tile_of(X, (32, 32, 32))
    # tiles of 8: 4 per axis, x fastest
    assert t.tolist() == [0, 0 + 1 * 4 + 1 * 16, 3 + 3 * 4 + 0 * 16]


# ---------------- membrane --------------------------------------------------

def _flat_triangle():
    X0 = torch.tensor([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.3, 0.8, 0.0]], dtype=DT)
    tri = torch.tensor([[0, 1, 2]])
    return X0, tri


def _W(lam1, lam2, kS, C):
    I1 = lam1 ** 2 + lam2 ** 2 - 2
    I2 = lam1 ** 2 * lam2 ** 2 - 1
    return kS / 4 * (I1 ** 2 + 2 * I1 - 2 * I2 + C * I2 ** 2)


@pytest.mark.parametrize("C", [0.0, 1.0, 9.0])
def test_skalak_energy_closed_forms(C):
    X0, tri = _flat_triangle()
    m = membrane.Mesh(X0, tri)
    A0 = float(m.A0[0])
    kS = 0.01
    for lam in (0.9, 1.0, 1.3):
        E = float(membrane.skalak_energy(m, X0 * lam, kS, C))
        assert E == pytest.approx(A0 * _W(lam, lam, kS, C), rel=1e-12, abs=1e-18)
    for lam in (0.8, 1.2):
        Xs = X0.clone()
        Xs[:, 0] *= lam
        E = float(membrane.skalak_energy(m, Xs, kS, C))
        assert E == pytest.approx(A0 * _W(lam, 1.0, kS, C), rel=1e-12)
    # rotated and translated rest shape has zero energy
    R = torch.tensor([[0.0, -1.0, 0.0], [0.0, 0.0, 1.0], [-1.0, 0.0, 0.0]], dtype=DT)
    E = float(membrane.skalak_energy(m, X0 @ R.T + 3.0, kS, C))
    assert abs(E) < 1e-18


@pytest.mark.parametrize("C", [0.0, 0.5, 9.0])
def test_skalak_small_strain_moduli_match_paper(C, golden):
    """kA = (1 + 2C) kS and nu_s = C / (1 + C) (Sec. II.B)."""
    kS = 0.01
    eps = 1e-4
    # isotropic area strain alpha = lam^2 - 1: W ~ kA/2 alpha^2
    lam = math.sqrt(1 + eps)
    kA = 2 * _W(lam, lam, kS, C) / eps ** 2
    assert kA == pytest.approx((1 + 2 * C) * kS, rel=1e-3)
    # uniaxial stretch lam1 with free lam2: nu_s = -dlam2/dlam1
    lam1 = 1 + 1e-5
    lo, hi = 0.99, 1.01
    for _ in range(200):
        a = 0.5 * (lo + hi)
        h = 1e-9
        d = (_W(lam1, a + h, kS, C) - _W(lam1, a - h, kS, C))
        if d > 0:
            hi = a
        else:
            lo = a
    nu = -(a - 1) / (lam1 - 1)
    assert nu == pytest.approx(C / (1 + C), abs=2e-3)


def _mesh(freq=4, R=5.0):
    xyz, tri = workloads.icosphere(freq, R)
    return torch.tensor(xyz), torch.tensor(tri, dtype=torch.int64)


def test_membrane_forces_rest_balance_and_fd():
    X0, tri = _mesh()
    m = membrane.Mesh(X0, tri)
    F = membrane.elastic_forces(m, X0, 0.01, 1.0, 2.0)
    assert float(F.abs().max()) < 1e-16
    g = torch.Generator().manual_seed(9)
    X = X0 + 0.2 * torch.randn(X0.shape, generator=g, dtype=DT)
    F = membrane.elastic_forces(m, X, 0.01, 1.0, 2.0)
    assert float(F.sum(0).abs().max()) < 1e-15
    torque = torch.cross(X, F, dim=1).sum(0)
    assert float(torque.abs().max()) < 1e-14
    # central differences of the energy
    h = 1e-6
    for b, d in [(0, 0), (17, 1), (100, 2), (161, 0)]:
        Xp, Xm = X.clone(), X.clone()
        Xp[b, d] += h
        Xm[b, d] -= h
        fd = (membrane.elastic_energy(m, Xp, 0.01, 1.0, 2.0)
              - membrane.elastic_energy(m, Xm, 0.01, 1.0, 2.0)) / (2 * h)
        assert float(-F[b, d]) == pytest.approx(float(fd), rel=1e-6, abs=1e-12)


def test_virial_under_uniform_scaling():
    X0, tri = _mesh()
    m = membrane.Mesh(X0, tri)
    for lam in (0.95, 1.07):
        X = X0 * lam
        F = membrane.elastic_forces(m, X, 0.01, 0.0, 0.0)
        A_tot = float(m.A0.sum())
        E = float(membrane.skalak_energy(m, X, 0.01, 0.0))
        assert E == pytest.approx(A_tot * _W(lam, lam, 0.01, 0.0), rel=1e-10)
        vir = float((F * X).sum())
        # dE/dlam for E(lam) = A_tot W(lam, lam)
        h = 1e-6
        dE = A_tot * (_W(lam + h, lam + h, 0.01, 0.0) - _W(lam - h, lam - h, 0.01, 0.0)) / (2 * h)
        assert vir == pytest.approx(-lam * dE, rel=1e-6)


def test_icosahedron_volume_area_and_scaling():
    v, f = workloads.icosahedron()
    X = torch.tensor(v)
    a = 2.0                                               # edge length of the coordinate icosahedron
    V = float(membrane.volume(X, f))
    A = float(membrane.area(X, f))
    assert V == pytest.approx(5.0 / 12.0 * (3 + math.sqrt(5)) * a ** 3, rel=1e-14)
    assert A == pytest.approx(5 * math.sqrt(3) * a ** 2, rel=1e-14)
    X0, tri = _mesh(8, 6.0)
    V0 = float(membrane.volume(X0, tri))
    assert float(membrane.volume(1.3 * X0, tri)) == pytest.approx(1.3 ** 3 * V0, rel=1e-13)
    assert V0 < 4 / 3 * math.pi * 6 ** 3 and V0 > 0.97 * 4 / 3 * math.pi * 6 ** 3


def test_volume_penalty_force_is_normal_pressure():
    X0, tri = _mesh()
    m = membrane.Mesh(X0, tri)
    X = 1.01 * X0
    F = membrane.elastic_forces(m, X, 0.0, 0.0, 2.0)
    V = float(membrane.volume(X, tri))
    # F_b = -kV (V - V0)/V0 dV/dX_b and sum_b X_b . dV/dX_b = 3 V
    lam = -2.0 * (V - float(m.V0)) / float(m.V0)
    assert float((F * X).sum()) == pytest.approx(lam * 3 * V, rel=1e-12)


def test_taylor_D_of_affinely_stretched_icosphere():
    X0, tri = _mesh(8, 6.0)
    for (a, b, c) in [(1.0, 1.0, 1.0), (1.2, 1.0, 0.9), (0.8, 1.1, 1.0)]:
        X = X0 * torch.tensor([a, b, c], dtype=DT) + torch.tensor([3.0, -2.0, 7.5], dtype=DT)
        D = float(membrane.taylor_D(X, tri))
        exp = (max(a, b, c) - min(a, b, c)) / (max(a, b, c) + min(a, b, c))
        assert D == pytest.approx(exp, abs=1e-9)
    V, A, com, mu = membrane.shape_moments(X0 + 4.0, tri)
    assert torch.allclose(com, torch.full((3,), 4.0, dtype=DT), atol=1e-12)


def test_icosphere_counts_and_paper_mesh(golden):
    for n in (1, 2, 4, 8, 16):
        xyz, tri = workloads.icosphere(n, 1.0)
        assert xyz.shape[0] == 10 * n * n + 2 and tri.shape[0] == 20 * n * n
    pm = golden["paper_mesh"]["value"]
    assert 10 * 12 ** 2 + 2 == pm["N_b"] and 20 * 12 ** 2 == pm["N_f"]
    xyz, tri = workloads.icosphere(4, 6.0)
    # outward orientation: positive volume; mirror symmetric in x, y, z
    assert float(membrane.volume(torch.tensor(xyz), tri)) > 0
    s = {tuple(np.round(p, 9)) for p in xyz}
    for ax in range(3):
        m = xyz.copy()
        m[:, ax] *= -1
        assert {tuple(np.round(p, 9)) for p in m} == s
