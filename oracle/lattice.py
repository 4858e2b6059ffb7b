"""D3Q19 BGK two-component Shan-Chen fluid, FP64 (test infrastructure only).

Layout: populations f[c, i, z, y, x]; c = component (0 = A, 1 = B),
i = direction.  Direction order: 0 rest; 1..6 = +x -x +y -y +z -z;
7..18 = (+-1,+-1,0), (+-1,0,+-1), (0,+-1,+-1) with opposite directions in
adjacent pairs.  The paper fixes only the three groups and their weights
(Sec. II.A, eq. lbm:weights); the order is a convention.

Pins (tests/test_oracle_lattice.py): equilibrium moments (mass, momentum,
momentum flux) exactly; shear-wave decay against the closed form with
nu = c_s^2 (tau - 1/2); half-way bounce-back Couette profile; Shan-Chen
force sums to zero in a periodic box; with two relaxation times the
collision's momentum change summed over the components equals the summed
force exactly, and without force the total momentum is conserved (which
fixes the tau-weighted common velocity and the tau_c in the shift);
flat interface stays flat; bulk
densities move toward the mean-field coexistence values; the on-site
velocity closure gives the boundary node the wall velocity exactly, keeps
a fluid at rest at rest, and its steady Couette profile is the exact
linear one between the boundary rows (tests/test_oracle_onsite.py).
"""

import torch

DT = torch.float64

C = torch.tensor([
    [0, 0, 0],
    [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
    [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
    [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
    [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1],
], dtype=torch.int64)

# Sec. II.A, eq. lbm:weights: 1/3 rest, 1/18 axis, 1/36 diagonal
W = torch.tensor([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12, dtype=DT)

OPP = [0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17]

# Sec. II.A: c_s = sqrt(1/3) in lattice units
CS2 = 1.0 / 3.0

CF = C.to(DT)


def equilibrium(rho, u):
    """Second-order equilibrium of Sec. II.A (eq. lbm:equilibrium):
    f_i^eq = w_i rho [1 + c.u / c_s^2 + (c.u)^2 / (2 c_s^4) - u^2 / (2 c_s^2)].

    rho: [..., z, y, x]; u: [..., 3, z, y, x] (x, y, z components).
    Returns [..., 19, z, y, x]."""
    cu = torch.einsum("id,...dzyx->...izyx", CF, u)
    uu = (u * u).sum(-4)
    w = W.view(19, 1, 1, 1)
    return w * rho.unsqueeze(-4) * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2)
                                    - uu.unsqueeze(-4) / (2.0 * CS2))


def moments(f):
    """Density and bare momentum: rho = sum_i f_i, j = sum_i f_i c_i
    (Sec. II.A with rho_0 = 1).  f: [c, 19, z, y, x]."""
    rho = f.sum(1)
    j = torch.einsum("id,cizyx->cdzyx", CF, f)
    return rho, j


def stream(fpost, walls=0, u_lo=(0.0, 0.0, 0.0), u_hi=(0.0, 0.0, 0.0)):
    """Pull streaming f_i(x) = f*_i(x - c_i), periodic in every direction
    (Sec. II.A, left-hand side of eq. method:boltzmann).

    walls = 2: on-site velocity boundaries on the rows y = 0 and
    y = ny - 1, which are fluid (onsite_closure).

    walls = 1: rows y = 0 and y = ny - 1 are solid.  A fluid population
    whose source node is solid is reflected half-way with the moving-wall
    term of Sec. II.C (eq. method:SBB):
        f_i(x) = f*_{opp(i)}(x) + 2 w_i rho(x) (c_i . u_w) / c_s^2,
    where c_i is the direction of the reflected population (from the wall
    into the fluid), u_w the velocity of that wall and rho(x) the density of
    component c at the fluid node, sum_i f*_i(x) (collision conserves it).
    Rows of solid nodes are left as garbage here; the caller resets them."""
    out = []
    for i in range(19):
        cx, cy, cz = (int(v) for v in C[i])
        out.append(torch.roll(fpost[:, i], shifts=(cz, cy, cx), dims=(1, 2, 3)))
    f = torch.stack(out, 1)
    if walls == 2:
        return onsite_closure(f, u_lo, u_hi)
    if walls:
        ny = f.shape[3]
        f = f.clone()
        rho_prev = fpost.sum(1)
        for i in range(19):
            cy = int(C[i][1])
            if cy == 0:
                continue
            y_f = 1 if cy == 1 else ny - 2
            uw = u_lo if cy == 1 else u_hi
            cu = float(C[i][0]) * uw[0] + float(C[i][1]) * uw[1] + float(C[i][2]) * uw[2]
            f[:, i, :, y_f, :] = (fpost[:, OPP[i], :, y_f, :]
                                  + 2.0 * float(W[i]) * rho_prev[:, :, y_f, :] * cu / CS2)
    return f


def onsite_closure(f, u_lo, u_hi):
    """On-site velocity boundaries on the rows y = 0 and y = ny - 1 (the
    boundaries the paper's shear-flow case names; Zou and He, in the D3Q19
    form of Hecht and Harting).  After streaming, the populations that would
    have come from outside the box (c_y = +1 at y = 0, c_y = -1 at
    y = ny - 1) are unknown.  With s the sign of c_y of the unknowns and u
    the wall velocity, mass and normal momentum give the node density
        rho = (Z + 2 O) / (1 - s u_y),
    Z the sum of the populations with c_y = 0 and O of those with c_y = -s;
    each unknown is its opposite plus the equilibrium difference, with a
    transverse correction that makes the tangential momentum rho u exactly:
        f_i = f_opp(i) + 6 w_i rho (c_i . u) - c_ix N_x - c_iz N_z,
        N_x = (1/2) sum_{c_y = 0} f c_x - rho u_x / 3 (and N_z alike).
    f: [c, 19, z, y, x] after streaming; returns a copy with the unknowns set."""
    f = f.clone()
    ny = f.shape[3]
    for yb, s, uw in ((0, 1, u_lo), (ny - 1, -1, u_hi)):
        g = f[:, :, :, yb, :].clone()               # [c, 19, z, x]
        cy = C[:, 1]
        Z = g[:, cy == 0].sum(1)
        O = g[:, cy == -s].sum(1)
        rho = (Z + 2.0 * O) / (1.0 - s * uw[1])
        flat = cy == 0
        Nx = 0.5 * (g[:, flat] * CF[flat, 0].view(1, -1, 1, 1)).sum(1) - rho * uw[0] / 3.0
        Nz = 0.5 * (g[:, flat] * CF[flat, 2].view(1, -1, 1, 1)).sum(1) - rho * uw[2] / 3.0
        for i in range(19):
            if int(C[i][1]) != s:
                continue
            cu = float(C[i][0]) * uw[0] + float(C[i][1]) * uw[1] + float(C[i][2]) * uw[2]
            f[:, i, :, yb, :] = (g[:, OPP[i]] + 6.0 * float(W[i]) * rho * cu
                                 - float(C[i][0]) * Nx - float(C[i][2]) * Nz)
    return f


def wall_copy(a, walls):
    """Solid rows take the value of the adjacent fluid row (a neutral wall for
    the pseudo-potential).  a: [..., z, y, x].  (With on-site boundaries every
    row is fluid; sc_sum then clamps its neighbours at the box instead.)"""
    if walls != 1:
        return a
    ny = a.shape[-2]
    idx = torch.arange(ny)
    idx[0] = 1
    idx[ny - 1] = ny - 2
    return a.index_select(-2, idx)


def pseudo_potential(rho, kind=0):
    """The Shan-Chen pseudo-potential: kind 0 psi = rho (the workloads'
    reading), kind 1 psi = rho0 (1 - exp(-rho / rho0)) with rho0 = 1, the
    form Sec. II.D names."""
    if kind == 0:
        return rho
    return 1.0 - torch.exp(-rho)


def sc_sum(psi, walls=0):
    """S(x) = sum_{i=1..18} w_i psi(x + c_i) c_i, periodic.  This is the
    neighbour sum inside the Shan-Chen force of Sec. II.D (eq.
    method:shanchen).  psi: [z, y, x] -> [3, z, y, x].  walls = 2 (on-site
    boundaries): a neighbour beyond the rows y = 0 or y = ny - 1 takes the
    boundary row's value (a neutral wall), not the periodic image."""
    s = torch.zeros((3,) + tuple(psi.shape), dtype=psi.dtype)
    acc = []
    ny = psi.shape[1]
    for i in range(1, 19):
        cx, cy, cz = (int(v) for v in C[i])
        if walls == 2:
            iy = torch.clamp(torch.arange(ny) + cy, 0, ny - 1)
            nb = torch.roll(psi.index_select(1, iy), shifts=(-cz, -cx), dims=(0, 2))
        else:
            nb = torch.roll(psi, shifts=(-cz, -cy, -cx), dims=(0, 1, 2))
        acc.append(float(W[i]) * nb.unsqueeze(0) * CF[i].view(3, 1, 1, 1))
    for a in acc:
        s = s + a
    return s


def shan_chen_force(psi_self, s_other, G):
    """F^c(x) = -psi^c(x) G S^{c'}(x) for two opposing components with
    G^{AB} = G^{BA} = G and G^{AA} = G^{BB} = 0 (Sec. II.D,
    eq. method:shanchen).  s_other is sc_sum of the other component's
    pseudo-potential."""
    return -G * psi_self.unsqueeze(0) * s_other


def collide(f, rho, j, F, tau):
    """BGK relaxation (Sec. II.A, eq. method:boltzmann right-hand side) with
    the force entering as a shift of the equilibrium velocity (Sec. II.A,
    after Shan and Chen):
        u' = sum_c (j^c / tau_c) / sum_c (rho^c / tau_c),
        u^{eq,c} = u' + tau_c F^c / rho^c,
        f* = f - (f - f^eq(rho^c, u^{eq,c})) / tau_c.
    f: [2, 19, z, y, x]; rho: [2, z, y, x]; j, F: [2, 3, z, y, x]."""
    t = [float(tau[0]), float(tau[1])]
    den = rho[0] / t[0] + rho[1] / t[1]
    up = (j[0] / t[0] + j[1] / t[1]) / den.unsqueeze(0)
    outs = []
    for c in range(2):
        ueq = up + t[c] * F[c] / rho[c].unsqueeze(0)
        feq = equilibrium(rho[c], ueq)
        outs.append(f[c] - (f[c] - feq) / t[c])
    return torch.stack(outs, 0)


def physical_velocity(rho, j, F):
    """u = (sum_c j^c + (1/2) sum_c F^c) / sum_c rho^c (Sec. II.A, second
    moment equation with the half-force term, summed over components)."""
    return (j[0] + j[1] + 0.5 * (F[0] + F[1])) / (rho[0] + rho[1]).unsqueeze(0)


def rest_populations(rhoA, rhoB):
    """Rest equilibrium f_i = w_i rho^c (u = 0) for both components."""
    rho = torch.stack([rhoA, rhoB], 0)
    return W.view(1, 19, 1, 1, 1) * rho.unsqueeze(1)
