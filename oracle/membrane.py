"""Capsule membrane mechanics and shape observables, FP64 (test
infrastructure only).

Discretisation: linear triangles with constant strain.  For a triangle with
vertices X1, X2, X3 the edge vectors e1 = X2 - X1, e2 = X3 - X1 give the
2x2 metric M = [e_a . e_b]; M0 is the same for the rest shape.  The
principal stretches satisfy lambda1^2 + lambda2^2 = tr(M0^-1 M) and
lambda1^2 lambda2^2 = det M / det M0, so
    I1 = tr(M0^-1 M) - 2,    I2 = det M / det M0 - 1
(Sec. II.B, strain invariants).  The Skalak energy of Sec. II.B
(eq. method:strain) integrated over the rest area A0 of each triangle is
    E_T = A0 (kS / 4) (I1^2 + 2 I1 - 2 I2 + C I2^2).
The volume penalty is Sec. II.B, eq. method:volume,
    E_V = (kV / 2) (V - V0)^2 / V0,   V = (1/6) sum_T X1 . (X2 x X3).
Node forces are F_b = -dE/dX_b (Sec. II.B, principle of virtual work),
taken here with autograd on the energy: the definition itself.

Observables: centre of mass = mean node position (equal node masses,
Sec. III); the Taylor parameter D = (a_long - a_short)/(a_long + a_short)
(Sec. III.A, eq. taylorparameter) with the half-axes of the ellipsoid that
has the same volume second-moment tensor as the enclosed polyhedron
(a_k = sqrt(5 mu_k / V)), the paper's "tensor of inertia" reading.

Pins (tests/test_oracle_membrane.py): closed-form energy under isotropic
and uniaxial stretch; small-strain area-dilation modulus (1 + 2C) kS and
Poisson ratio C / (1 + C) as printed in Sec. II.B; zero force at rest;
zero net force and torque; central finite differences of the energy;
icosahedron volume and area closed forms; V scales as lambda^3; D of an
affinely stretched icosphere equals the closed form.
"""

import torch

DT = torch.float64


class Mesh:
    """Rest geometry of one capsule: faces and per-face reference metric."""

    def __init__(self, xyz_rest, tri):
        self.X0 = torch.as_tensor(xyz_rest, dtype=DT)
        self.tri = torch.as_tensor(tri, dtype=torch.int64)
        e1 = self.X0[self.tri[:, 1]] - self.X0[self.tri[:, 0]]
        e2 = self.X0[self.tri[:, 2]] - self.X0[self.tri[:, 0]]
        m11 = (e1 * e1).sum(1)
        m12 = (e1 * e2).sum(1)
        m22 = (e2 * e2).sum(1)
        self.det0 = m11 * m22 - m12 * m12
        # inverse of the rest metric
        self.q11 = m22 / self.det0
        self.q12 = -m12 / self.det0
        self.q22 = m11 / self.det0
        self.A0 = 0.5 * torch.sqrt(self.det0)
        self.V0 = volume(self.X0, self.tri)
        nb = self.X0.shape[0]
        self.node_area = torch.zeros(nb, dtype=DT).index_add(
            0, self.tri.reshape(-1), (self.A0 / 3.0).repeat_interleave(3))


def invariants(mesh, X):
    """Strain invariants (I1, I2) per triangle at positions X."""
    t = mesh.tri
    e1 = X[t[:, 1]] - X[t[:, 0]]
    e2 = X[t[:, 2]] - X[t[:, 0]]
    m11 = (e1 * e1).sum(1)
    m12 = (e1 * e2).sum(1)
    m22 = (e2 * e2).sum(1)
    tr = mesh.q11 * m11 + 2.0 * mesh.q12 * m12 + mesh.q22 * m22
    det = m11 * m22 - m12 * m12
    return tr - 2.0, det / mesh.det0 - 1.0


def skalak_energy(mesh, X, kS, C):
    I1, I2 = invariants(mesh, X)
    return (mesh.A0 * (kS / 4.0) * (I1 * I1 + 2.0 * I1 - 2.0 * I2 + C * I2 * I2)).sum()


def volume(X, tri):
    t = torch.as_tensor(tri, dtype=torch.int64)
    a, b, c = X[t[:, 0]], X[t[:, 1]], X[t[:, 2]]
    return (a * torch.cross(b, c, dim=1)).sum() / 6.0


def area(X, tri):
    t = torch.as_tensor(tri, dtype=torch.int64)
    e1 = X[t[:, 1]] - X[t[:, 0]]
    e2 = X[t[:, 2]] - X[t[:, 0]]
    return 0.5 * torch.linalg.norm(torch.cross(e1, e2, dim=1), dim=1).sum()


def volume_energy(mesh, X, kV):
    V = volume(X, mesh.tri)
    return 0.5 * kV * (V - mesh.V0) ** 2 / mesh.V0


def elastic_energy(mesh, X, kS, C, kV):
    return skalak_energy(mesh, X, kS, C) + volume_energy(mesh, X, kV)


def elastic_forces(mesh, X, kS, C, kV, create_graph=False):
    """F_b = -dE/dX_b for the Skalak plus volume energy (autograd)."""
    if not X.requires_grad:
        X = X.detach().requires_grad_(True)
        create_graph = False
    with torch.enable_grad():
        E = elastic_energy(mesh, X, kS, C, kV)
        (g,) = torch.autograd.grad(E, X, create_graph=create_graph)
    return -g


def shape_moments(X, tri):
    """Volume V, area A, node centre of mass, and the central second-moment
    tensor of the enclosed polyhedron (divergence theorem over the
    tetrahedra spanned with the node centroid)."""
    com = X.mean(0)
    Y = X - com
    t = torch.as_tensor(tri, dtype=torch.int64)
    a, b, c = Y[t[:, 0]], Y[t[:, 1]], Y[t[:, 2]]
    v = (a * torch.cross(b, c, dim=1)).sum(1) / 6.0
    V = v.sum()
    s = a + b + c
    first = (v.unsqueeze(1) * s).sum(0) / 4.0
    outer = lambda p, q: p.unsqueeze(2) * q.unsqueeze(1)
    second = (v.view(-1, 1, 1) * (outer(a, a) + outer(b, b) + outer(c, c) + outer(s, s))).sum(0) / 20.0
    xc = first / V
    mu = second - V * outer(xc.unsqueeze(0), xc.unsqueeze(0))[0]
    return V, area(X, tri), com, mu


def semi_axes(V, mu):
    ev = torch.linalg.eigvalsh(mu)
    return torch.sqrt(5.0 * torch.clamp(ev, min=0.0) / V)


def taylor_D(X, tri):
    V, _, _, mu = shape_moments(X, tri)
    ax = semi_axes(V, mu)
    return (ax.max() - ax.min()) / (ax.max() + ax.min())
