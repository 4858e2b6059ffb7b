"""Pins of the oracle's Helfrich bending force (Sec. II.B, eq. surf_dens with
the discrete operators of Meyer et al.)."""

import math

import numpy as np
import torch

from oracle import bending
from paper_1904_11386_amd import workloads as W

DT = torch.float64


def _sphere(freq, R):
    xyz, tri = W.icosphere(freq, R)
    return torch.tensor(xyz, dtype=DT), torch.tensor(tri)


def _ellipsoid(freq, axes):
    xyz, tri = W.icosphere(freq, 1.0)
    return torch.tensor(xyz * np.array(axes), dtype=DT), torch.tensor(tri)


def _area(X, tri):
    t = tri.long()
    return 0.5 * torch.linalg.cross(X[t[:, 1]] - X[t[:, 0]], X[t[:, 2]] - X[t[:, 0]], dim=1).norm(dim=1).sum()


def test_gauss_bonnet_and_mixed_area_partition():
    """sum_i K_i A_i = 2 pi chi = 4 pi for any closed genus-0 mesh, and the
    mixed areas tile the surface; on a distorted ellipsoid with obtuse
    triangles too."""
    for X, tri in (_sphere(4, 5.0), _ellipsoid(8, (9.0, 5.0, 3.0))):
        g = torch.manual_seed(0)
        Xp = X + 0.05 * torch.randn(X.shape, generator=g, dtype=DT)
        for Y in (X, Xp):
            geo = bending.geometry(Y, tri)
            assert abs(float((geo["K"] * geo["A"]).sum()) - 4.0 * math.pi) < 1e-10
            assert abs(float(geo["A"].sum()) / float(_area(Y, tri)) - 1.0) < 1e-13


def test_obtuse_triangle_mixed_areas():
    """One triangle with an obtuse corner: that corner takes half the area,
    the others a quarter each; a right-angled acute case uses the Voronoi
    parts, which give the corner at the right angle half the area."""
    X = torch.tensor([[0.0, 0.0, 0.0], [4.0, 0.0, 0.0], [1.0, 0.5, 0.0]], dtype=DT)
    tri = torch.tensor([[0, 1, 2]])
    g = bending.geometry(X, tri)
    a = 0.5 * 4.0 * 0.5
    assert torch.allclose(g["A"], torch.tensor([a / 4, a / 4, a / 2], dtype=DT), rtol=1e-14)
    X = torch.tensor([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [0.0, 3.0, 0.0]], dtype=DT)
    g = bending.geometry(X, tri)
    # Voronoi parts of a right triangle: the right-angle corner gets half
    assert abs(float(g["A"][0]) - 1.5) < 1e-13 and abs(float(g["A"].sum()) - 3.0) < 1e-13


def test_laplacian_of_linear_field_is_mean_curvature_normal():
    """Lap_s (a . x) = -a . K_i at every node: the cot Laplacian applied to
    the coordinates gives minus the mean curvature normal (exactly)."""
    X, tri = _ellipsoid(4, (6.0, 4.0, 5.0))
    g = bending.geometry(X, tri)
    a = torch.tensor([0.3, -1.2, 0.7], dtype=DT)
    lap = bending.laplace_beltrami(g, X @ a)
    assert torch.allclose(lap, -(g["Kvec"] @ a), rtol=1e-12, atol=1e-12)
    # and of a constant, zero
    assert float(bending.laplace_beltrami(g, torch.ones(X.shape[0], dtype=DT)).abs().max()) < 1e-12


def test_sphere_curvatures_converge():
    R = 7.0
    errs = []
    for f in (4, 8, 16):
        X, tri = _sphere(f, R)
        g = bending.geometry(X, tri)
        eH = float((g["H"] * R - 1.0).abs().max())
        eK = float((g["K"] * R * R - 1.0).abs().max())
        # the normal is the outward radial direction
        eN = float((g["n"] - X / X.norm(dim=1, keepdim=True)).abs().max())
        errs.append((eH, eK, eN))
    # H is within 1e-4 at every frequency; K and the area-weighted normal
    # converge with refinement
    assert max(e[0] for e in errs) < 2e-4
    assert errs[2][1] < 2e-3 and errs[2][1] < 0.5 * errs[1][1] < 0.5 * errs[0][1]
    assert errs[2][2] < 1e-2 and errs[2][2] < 0.7 * errs[1][2] < 0.7 * errs[0][2]


def test_ellipsoid_curvatures_against_closed_form():
    """An affinely stretched icosphere: the mean errors converge with
    refinement; the worst nodes (stretched triangles around the irregular
    vertices) stay at a few per cent, as the discrete operators do on
    non-uniform meshes."""
    a, b, c = 8.0, 6.0, 4.5
    res = []
    for f in (8, 16):
        X, tri = _ellipsoid(f, (a, b, c))
        g = bending.geometry(X, tri)
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        q = x * x / a ** 4 + y * y / b ** 4 + z * z / c ** 4
        K = 1.0 / (a * a * b * b * c * c * q * q)
        H = (a * a + b * b + c * c - x * x - y * y - z * z) / (2.0 * a * a * b * b * c * c * q ** 1.5)
        eH, eK = ((g["H"] - H) / H).abs(), ((g["K"] - K) / K).abs()
        res.append((float(eH.mean()), float(eK.mean()), float(eH.max()), float(eK.max())))
    assert res[1][0] < 2e-3 and res[1][1] < 4e-3
    assert res[1][0] < 0.5 * res[0][0] and res[1][1] < 0.5 * res[0][1]
    assert res[1][2] < 5e-2 and res[1][3] < 8e-2


def test_sphere_force_vanishes_in_the_limit_and_rigid_invariance():
    """On a sphere 2H(H^2 - K) and Lap_s H vanish in the continuum; the
    discrete force shrinks with refinement relative to kB / R^3 times the
    area, and it moves rigidly with the mesh."""
    kB, R = 0.2, 6.0
    rel = []
    for f in (4, 8, 16):
        X, tri = _sphere(f, R)
        F = bending.bending_forces(X, tri, kB)
        A = bending.geometry(X, tri)["A"]
        rel.append(float((F.norm(dim=1) / (kB / R ** 3 * A)).max()))
    assert rel[-1] < 0.2 and rel[-1] < rel[0]
    X, tri = _ellipsoid(8, (7.0, 5.0, 4.0))
    F = bending.bending_forces(X, tri, kB)
    th = 0.7
    Rm = torch.tensor([[math.cos(th), -math.sin(th), 0.0], [math.sin(th), math.cos(th), 0.0], [0.0, 0.0, 1.0]],
                      dtype=DT)
    F2 = bending.bending_forces(X @ Rm.T + torch.tensor([3.0, -2.0, 11.0], dtype=DT), tri, kB)
    assert torch.allclose(F2, F @ Rm.T, rtol=1e-9, atol=1e-12 * float(F.abs().max()))
    # an ellipsoid is pushed toward a sphere: the force at the long-axis tips points inward
    tip = int(torch.argmax(X[:, 0]))
    assert float(F[tip, 0]) < 0.0


def test_whole_step_with_bending():
    """In the coupled step, the capsules with kB > 0 get exactly the bending
    force on top of the other node forces; the fluid's mass and momentum
    change only through the spread total, which now carries the (small,
    discretisation-level) net bending force."""
    from oracle.sim import from_workload
    wl = W.bent()
    s = from_workload(wl)
    s.step()
    import dataclasses
    off = from_workload(dataclasses.replace(wl, capsules=[dataclasses.replace(c, kB=0.0) for c in wl.capsules]))
    off.step()
    X0 = [torch.tensor(c.mesh()[0], dtype=DT) for c in wl.capsules]
    for k, c in enumerate(wl.capsules):
        d = s.Fb_last[k] - off.Fb_last[k]
        if c.kB > 0:
            ref = bending.bending_forces(X0[k], torch.tensor(c.mesh()[1]), c.kB)
            assert torch.allclose(d, ref, rtol=1e-10, atol=1e-14)
            # the ellipsoid is bent well beyond the sphere's discretisation level
            if c.stretch != (1.0, 1.0, 1.0):
                assert float(ref.abs().max()) > 1e-3
        else:
            assert float(d.abs().max()) == 0.0
    m0 = torch.tensor([wl.rhoA.astype(np.float64).sum(), wl.rhoB.astype(np.float64).sum()], dtype=DT)
    s.run(10)
    assert torch.allclose(s.mass(), m0, rtol=1e-13, atol=0)
