"""Particle-particle repulsion, FP64 (test infrastructure only).

Sec. III.E adds a short-range hard-core force between boundary nodes of
different particles so that particles do not overlap: a pair of nodes at
separation d pushes apart along the line joining them with magnitude
    F(d) = eps (d0 - d)^{3/2}   for d < d0,   0 for d >= d0,
where the paper takes eps = 0.5 and d0 = 1.25 lattice units.  Nodes of one
particle do not act on each other through it.  Separations are taken as the
nearest periodic image on the periodic axes (x and z, and y when there are
no walls).

The force is minus the gradient of the pair energy
    E(d) = (2/5) eps (d0 - d)^{5/2}   for d < d0,
which is what makes the pair forces equal and opposite and central.

Pins (tests/test_oracle_contact.py): the closed form for one pair, nothing
at or beyond d0 and nothing within a particle, Newton's third law and zero
net torque for random clouds, invariance under a shift by a lattice period,
F = -grad E, and a plain double loop on small clouds.
"""

import torch

DT = torch.float64


def nearest_image(d, dims, walls=0):
    """Separation vectors d [..., 3] mapped to the nearest periodic image
    on the periodic axes of a lattice of size dims = (nx, ny, nz)."""
    out = []
    for a in range(3):
        v = d[..., a]
        if not (a == 1 and walls):
            v = v - dims[a] * torch.round(v / dims[a])
        out.append(v)
    return torch.stack(out, -1)


def repulsion_forces(Xs, dims, eps, d0, walls=0):
    """Forces on the nodes of each particle.  Xs: list of [N_k, 3] absolute
    node positions, one tensor per particle.  Returns a list of [N_k, 3]."""
    F = [torch.zeros_like(X) for X in Xs]
    if eps == 0.0 or len(Xs) < 2:
        return F
    centre = [X.detach().mean(0) for X in Xs]
    reach = [float((X.detach() - c).norm(dim=1).max()) for X, c in zip(Xs, centre)]
    for k in range(len(Xs)):
        for l in range(k + 1, len(Xs)):
            # no node pair can come within d0 when the bounding spheres,
            # widened by d0, do not meet
            gap = float(nearest_image(centre[k] - centre[l], dims, walls).norm())
            if gap > reach[k] + reach[l] + d0:
                continue
            d = nearest_image(Xs[k][:, None, :] - Xs[l][None, :, :], dims, walls)   # [N_k, N_l, 3]
            r = d.norm(dim=2)
            near = r < d0
            if not bool(near.any()):
                continue
            rs = torch.where(near, r, torch.ones_like(r))
            mag = torch.where(near, eps * (d0 - rs) ** 1.5, torch.zeros_like(r))
            f = (mag / rs).unsqueeze(2) * d          # on the node of k, from the node of l
            F[k] = F[k] + f.sum(1)
            F[l] = F[l] - f.sum(0)
    return F


def repulsion_energy(Xs, dims, eps, d0, walls=0):
    """Total pair energy sum (2/5) eps (d0 - d)^{5/2} over node pairs of
    different particles closer than d0."""
    E = torch.zeros((), dtype=DT)
    for k in range(len(Xs)):
        for l in range(k + 1, len(Xs)):
            d = nearest_image(Xs[k][:, None, :] - Xs[l][None, :, :], dims, walls)
            r = d.norm(dim=2)
            near = r < d0
            rs = torch.where(near, r, torch.full_like(r, d0))
            E = E + (0.4 * eps * (d0 - rs) ** 2.5).sum()
    return E
