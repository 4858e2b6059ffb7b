"""Helfrich bending force on a closed triangulated membrane, FP64 (test
infrastructure only).

Sec. II.B gives the bending resistance as the Helfrich energy
(kB/2) oint (2H - H0)^2 dA with H0 = 0, and its nodal force as the surface
force density
    f_B = 2 kB [2 H (H^2 - K) + Lap_s H] n                (eq. surf_dens)
times the node's area, with H the mean curvature, K the Gaussian curvature,
Lap_s the Laplace-Beltrami operator and n the outward normal, all from the
discrete differential-geometry operators of Meyer, Desbrun, Schroeder and
Barr (2003).  Those operators, at node i with its triangles T:
  - cot weights: for the edge (i, j), w_ij = cot(alpha_ij) + cot(beta_ij),
    the cotangents of the two angles opposite the edge;
  - mixed area A_i: per triangle, the Voronoi part
    (|x_i - x_j|^2 cot(angle at k) + |x_i - x_k|^2 cot(angle at j)) / 8 when
    the triangle has no obtuse angle, else area / 2 when the angle at i is
    obtuse and area / 4 when another angle is;
  - mean curvature normal K_i = (1 / (2 A_i)) sum_j w_ij (x_i - x_j), which
    equals 2 H n; here H = K_i . n / 2 with n the normalised sum of the
    triangles' area-weighted outward normals (defined also where H = 0);
  - Gaussian curvature K = (2 pi - sum_T theta_i^T) / A_i;
  - Lap_s f (i) = (1 / (2 A_i)) sum_j w_ij (f_j - f_i).
The nodal force is F_i = 2 kB [2 H_i (H_i^2 - K_i) + Lap_s H (i)] n_i A_i.
(With H > 0 on a sphere and the outward n, an outward bump has H above its
neighbours, a negative Laplacian and an inward force: bending flattens it.)

Pins (tests/test_oracle_bending.py): discrete Gauss-Bonnet sum_i K_i A_i =
4 pi exactly on a closed genus-0 mesh; the mixed areas sum to the surface
area exactly; Lap_s of a linear field a . x equals -a . K_i exactly; a
right-angled triangle's corner takes area / 2; H -> 1/R and K -> 1/R^2 on
icospheres of growing frequency and H, K of an ellipsoid against its closed
forms; the force vanishes on a sphere in the continuum limit and is
invariant under rigid motion.
"""

import math

import torch

DT = torch.float64


def _cot(a, b):
    """cot of the angle between vectors a and b (rows)."""
    return (a * b).sum(1) / torch.linalg.cross(a, b, dim=1).norm(dim=1)


def geometry(X, tri):
    """Per-node H, K, mixed area A, outward unit normal n, and the per-edge
    cot weights as (i, j, w) lists, for positions X [N, 3] and outward
    counter-clockwise triangles tri [F, 3]."""
    X = torch.as_tensor(X, dtype=DT)
    t = torch.as_tensor(tri, dtype=torch.int64)
    N = X.shape[0]
    xs = [X[t[:, c]] for c in range(3)]
    cross = torch.linalg.cross(xs[1] - xs[0], xs[2] - xs[0], dim=1)
    area = 0.5 * cross.norm(dim=1)
    # angle data per corner c of each triangle: cot and angle at c
    cots, angs = [], []
    for c in range(3):
        a = xs[(c + 1) % 3] - xs[c]
        b = xs[(c + 2) % 3] - xs[c]
        cots.append(_cot(a, b))
        cosv = (a * b).sum(1) / (a.norm(dim=1) * b.norm(dim=1))
        angs.append(torch.acos(cosv.clamp(-1.0, 1.0)))
    obtuse = [(a > 0.5 * math.pi) for a in angs]
    any_obt = obtuse[0] | obtuse[1] | obtuse[2]
    A = torch.zeros(N, dtype=DT)
    Kvec = torch.zeros(N, 3, dtype=DT)
    theta = torch.zeros(N, dtype=DT)
    nrm = torch.zeros(N, 3, dtype=DT)
    I, J, Wt = [], [], []
    for c in range(3):
        j, k = (c + 1) % 3, (c + 2) % 3
        xi, xj, xk = xs[c], xs[j], xs[k]
        # Voronoi part: edge (i, j) is opposite corner k, edge (i, k) opposite corner j
        vor = ((xi - xj) ** 2).sum(1) * cots[k] / 8.0 + ((xi - xk) ** 2).sum(1) * cots[j] / 8.0
        mixed = torch.where(any_obt, torch.where(obtuse[c], area / 2.0, area / 4.0), vor)
        A = A.index_add(0, t[:, c], mixed)
        contrib = cots[k].unsqueeze(1) * (xi - xj) + cots[j].unsqueeze(1) * (xi - xk)
        Kvec = Kvec.index_add(0, t[:, c], contrib)
        theta = theta.index_add(0, t[:, c], angs[c])
        nrm = nrm.index_add(0, t[:, c], cross)
        I += [t[:, c], t[:, c]]
        J += [t[:, j], t[:, k]]
        Wt += [cots[k], cots[j]]
    Kvec = Kvec / (2.0 * A).unsqueeze(1)
    n = nrm / nrm.norm(dim=1, keepdim=True)
    H = 0.5 * (Kvec * n).sum(1)
    K = (2.0 * math.pi - theta) / A
    return dict(H=H, K=K, A=A, n=n, Kvec=Kvec, I=torch.cat(I), J=torch.cat(J), W=torch.cat(Wt))


def laplace_beltrami(g, f):
    """Lap_s f at every node: (1 / (2 A_i)) sum over the node's triangle
    edges of cot(opposite angle) (f_j - f_i); each mesh edge is seen from
    its two triangles, which adds the two cotangents."""
    s = torch.zeros_like(f).index_add(0, g["I"], g["W"] * (f[g["J"]] - f[g["I"]]))
    return s / (2.0 * g["A"])


def bending_forces(X, tri, kB):
    """Nodal Helfrich bending forces F_i = 2 kB [2 H (H^2 - K) + Lap_s H] n A."""
    g = geometry(X, tri)
    H, K = g["H"], g["K"]
    lap = laplace_beltrami(g, H)
    s = 2.0 * kB * (2.0 * H * (H * H - K) + lap) * g["A"]
    return s.unsqueeze(1) * g["n"]
