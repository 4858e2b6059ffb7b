"""The LBM-free reference model of Sec. III.B, FP64 (test infrastructure
only).

The paper checks its coupling against a model without hydrodynamics: the
capsule keeps its elastic laws (Skalak, volume, bending) and time
integration, and instead of the fluid the interface's surface tension
pulls on every boundary element within a slab of width w around the
(stationary) interface plane, with the tensile force
    F = gamma A / w                                (eq. emulatetension)
where A is the part of the element's area between the planes
z_interface -+ w/2; the force is shared evenly by the element's three nodes.

Readings (the paper's text and figure leave them open):
  - direction: the surface tension acts in the interface plane and pulls the
    contact line outward, so F points horizontally and radially away from
    the vertical axis through the capsule's centre of mass at the start of
    the relaxation, evaluated at the element's centroid;
  - time integration: the immersed-boundary nodes are massless, so the
    relaxation is overdamped, X <- X + mu F with a mobility mu; the
    equilibrium shape does not depend on mu.

The slab area uses the closed form for the part of a triangle below a plane
z = h: with the vertex heights sorted z0 <= z1 <= z2, the fraction is
(h - z0)^2 / ((z1 - z0)(z2 - z0)) for z0 <= h <= z1 and
1 - (z2 - h)^2 / ((z2 - z1)(z2 - z0)) for z1 <= h <= z2 (the cross-section
grows linearly on each side of z1).

Pins (tests/test_oracle_reference.py): the closed form against explicit
polygon clipping of random triangles; whole elements inside the slab give
their full area and elements outside none; the tensile force is horizontal
and, for a capsule mirror-symmetric about its axis, has no net force; a
relaxation stretches the capsule in the interface plane and shortens it
along the poles.  The paper's printed equilibrium half-axes are mutually
inconsistent, so the relaxed shape itself is parity unpinned.
"""

import torch

from . import bending, membrane

DT = torch.float64


def fraction_below(z, h):
    """Fraction of each triangle's area with height below h; z [F, 3]."""
    zs, _ = torch.sort(z, dim=1)
    z0, z1, z2 = zs[:, 0], zs[:, 1], zs[:, 2]
    one = torch.ones_like(z0)
    d20 = torch.where(z2 > z0, z2 - z0, one)
    d10 = torch.where(z1 > z0, z1 - z0, one)
    d21 = torch.where(z2 > z1, z2 - z1, one)
    lower = (h - z0) ** 2 / (d10 * d20)
    upper = 1.0 - (z2 - h) ** 2 / (d21 * d20)
    f = torch.where(h <= z1, lower, upper)
    f = torch.where(h <= z0, torch.zeros_like(f), f)
    return torch.where(h >= z2, one, f)


def slab_area(X, tri, z_lo, z_hi):
    """Area of each triangle between the planes z = z_lo and z = z_hi."""
    t = torch.as_tensor(tri, dtype=torch.int64)
    a = 0.5 * torch.linalg.cross(X[t[:, 1]] - X[t[:, 0]], X[t[:, 2]] - X[t[:, 0]], dim=1).norm(dim=1)
    z = X[t][:, :, 2]
    return a * (fraction_below(z, z_hi) - fraction_below(z, z_lo))


def tensile_forces(X, tri, axis_xy, gamma, w, z_interface):
    """Per-node tensile forces of eq. emulatetension (see the readings)."""
    t = torch.as_tensor(tri, dtype=torch.int64)
    A = slab_area(X, t, z_interface - 0.5 * w, z_interface + 0.5 * w)
    c = X[t].mean(1)
    d = torch.stack([c[:, 0] - axis_xy[0], c[:, 1] - axis_xy[1], torch.zeros_like(c[:, 0])], 1)
    dn = d.norm(dim=1, keepdim=True)
    d = torch.where(dn > 0, d / torch.where(dn > 0, dn, torch.ones_like(dn)), torch.zeros_like(d))
    f = (gamma * A / w / 3.0).unsqueeze(1) * d
    F = torch.zeros_like(X)
    for k in range(3):
        F = F.index_add(0, t[:, k], f)
    return F


def relax(xyz, tri, kS, C, kV, kB, gamma, w, z_interface, mobility, steps):
    """Overdamped relaxation of one capsule (rest shape xyz, which is also the
    start) under its elastic forces and the emulated tension; returns the
    node positions after `steps` steps."""
    mesh = membrane.Mesh(xyz, tri)
    X = torch.as_tensor(xyz, dtype=DT).clone()
    axis = X.mean(0)[:2].clone()
    for _ in range(steps):
        F = membrane.elastic_forces(mesh, X, kS, C, kV)
        if kB > 0.0:
            F = F + bending.bending_forces(X, mesh.tri, kB)
        F = F + tensile_forces(X, mesh.tri, axis, gamma, w, z_interface)
        X = X + mobility * F
    return X
