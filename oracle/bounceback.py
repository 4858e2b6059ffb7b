"""The paper's own fluid-structure coupling, FP64 (test infrastructure only).

Only the test-suite, the smoke entry point and the benchmark's CPU-baseline
leg may use this module; the HIP library shares no code with it.

The membrane separates the lattice into the fluid inside each capsule and
the fluid outside; both are simulated (Sec. II.D: no third component for
the interior).  Written from Sec. II.C (half-way bounce-back on moving
elements, eq. method:SBB; momentum transfer, eq. method:momentumtransfer;
element-to-node weighting and the two-step spreading of the exchanged
momentum), Sec. II.D (the Shan-Chen sum across the membrane with densities
interpolated from the viewer's side, eq. method:interpolateshanchen, and the
colour offset on one component) and Sec. II.E (fresh nodes, eq.
method:freshnodes; their velocity and momentum bookkeeping; the adaptive
mass correction, eq. method:masscorrection, with the clamp to the
neighbours' range).  The nodes are inertial (node mass 5, Sec. III) and
move by the first-order Euler update of Sec. II.B.

One step n, state f*^{n-1} (post-collision), node positions X^n and
velocities V^n, the labels of the previous step, the exchanged momentum of
the previous step:
 1. labels L^n(x) = k when the lattice node x lies inside capsule k's
    closed triangulated surface at X^n, else -1; fresh nodes are those
    whose label changed;
 2. fresh nodes are refilled with the equilibrium of the interpolated,
    mass-corrected density and the mean velocity of the three nodes of the
    nearest element; the element gets the removed minus the created
    momentum;
 3. pull streaming; a population whose source lies across the membrane is
    the node's own outgoing population reflected, plus the moving-element
    term 2 w_i rho (c_i . v0) / c_s^2 (c_i the reflected direction, rho the
    node's density, v0 the element's velocity = the mean of its three nodes);
    the exchanged momentum [f*_out + f_back] c_out goes to that element;
 4. moments;
 5. Shan-Chen force: a neighbour across the membrane enters with the
    density interpolated from its own neighbours on the viewer's side, plus
    the capsule's virtual density on its preferred component; the force
    that pair would put on the neighbour goes to the element instead;
 6. BGK collision with the equilibrium-velocity shift (Sec. II.A);
 7. node force = elastic (Skalak, volume, optional bending) + half of this
    step's and half of the previous step's exchanged momentum + the fresh-node
    and Shan-Chen reactions; V += F / m, X += V (V held fixed for capsules
    with a prescribed velocity, the rigid motion of Sec. II.E's
    mass-conservation test).
Each element quantity goes to its three nodes in equal thirds (Sec. II.C).

Readings where the paper is silent (listed with the design readings):
labels by the closed surface (a node exactly on it is measure-zero); the
crossed element of a link, for both of its ends, is the one the segment
between the two nodes pierces nearest the link's start node (the end from
which it points along a positive half-direction), which a wrinkled membrane
can make differ from the first one seen from the other end; the nearest element of a
fresh node is the one with the nearest centroid; Delta rho^c of eq.
method:masscorrection is the component's total mass minus its initial
total, <rho^c> / rho_init^c the per-node average of the start, V_sys the
fluid node count; a fresh node with no non-fresh neighbour on its side
keeps its own density; densities for the bounce-back term and the
interpolations are those of f*^{n-1} (after the refill).

Pins (tests/test_oracle_bounceback.py): labels against a sphere and an
independent ray-parity count; rest preserved exactly; a capsule of one
uniform composition inside a different uniform composition stays at rest
exactly (the decoupling); a uniform flow carried by a capsule translating
at the same velocity is an exact steady state through fresh nodes (the sign
of the moving-element term); total momentum of fluid, nodes and the pending
half of the exchanged momentum conserved to rounding; mass per region exact
for a fixed membrane; mass drift of a translating sphere with and without
the correction; a neutral sphere on a flat interface keeps its height by
symmetry.
"""

import math

import torch

from . import bending, lattice, membrane

DT = torch.float64
C = lattice.C
CF = lattice.CF
W = lattice.W
OPP = lattice.OPP
CS2 = lattice.CS2


def cos_deg(theta):
    t = float(theta)
    return 0.0 if t == 90.0 else math.cos(math.radians(t))


def winding_inside(P, X, tri):
    """Inside test of points P [M, 3] for the closed surface (X, tri): the
    winding number, the sum over triangles of the solid angle they subtend
    (van Oosterom and Strackee) over 4 pi, is 1 inside and 0 outside."""
    A = X[tri[:, 0]].unsqueeze(0) - P.unsqueeze(1)     # [M, F, 3]
    B = X[tri[:, 1]].unsqueeze(0) - P.unsqueeze(1)
    Cc = X[tri[:, 2]].unsqueeze(0) - P.unsqueeze(1)
    la, lb, lc = A.norm(dim=2), B.norm(dim=2), Cc.norm(dim=2)
    num = (A * torch.cross(B, Cc, dim=2)).sum(2)
    den = la * lb * lc + (A * B).sum(2) * lc + (A * Cc).sum(2) * lb + (B * Cc).sum(2) * la
    omega = 2.0 * torch.atan2(num, den)
    return omega.sum(1) / (4.0 * math.pi) > 0.5


def segment_hits(P0, P1, X, tri):
    """Moeller-Trumbore: for each segment P0[k] -> P1[k] ([K, 3]) and each
    triangle, the parameter t in [0, 1) of the crossing, or inf."""
    A = X[tri[:, 0]]
    e1 = X[tri[:, 1]] - A
    e2 = X[tri[:, 2]] - A
    d = (P1 - P0).unsqueeze(1)                          # [K, 1, 3]
    pv = torch.cross(d.expand(-1, e2.shape[0], -1), e2.unsqueeze(0).expand(d.shape[0], -1, -1), dim=2)
    det = (e1.unsqueeze(0) * pv).sum(2)
    ok = det != 0.0
    inv = torch.where(ok, 1.0 / torch.where(ok, det, torch.ones_like(det)), torch.zeros_like(det))
    tv = P0.unsqueeze(1) - A.unsqueeze(0)
    u = (tv * pv).sum(2) * inv
    qv = torch.cross(tv, e1.unsqueeze(0).expand_as(tv), dim=2)
    v = (d * qv).sum(2) * inv
    t = (e2.unsqueeze(0) * qv).sum(2) * inv
    hit = ok & (u >= 0.0) & (v >= 0.0) & (u + v <= 1.0) & (t >= 0.0) & (t < 1.0)
    return torch.where(hit, t, torch.full_like(t, math.inf))


class BounceBackSim:
    """Two-component Shan-Chen fluid coupled to capsules by bounce-back.

    caps: dicts with xyz (rest = initial absolute positions), tri (outward
    counter-clockwise), kS, C, kV, theta (degrees), optional kB, v
    (initial node velocity, 3), prescribed (keep v)."""

    def __init__(self, rhoA, rhoB, caps=(), tau=(1.0, 1.0), G=3.6, rho_maj=0.7, rho_min=0.04,
                 z_interface=0.0, wet_scale=1.0, node_mass=5.0, C0=2500.0, psi_kind=0):
        rhoA = torch.as_tensor(rhoA, dtype=DT)
        rhoB = torch.as_tensor(rhoB, dtype=DT)
        self.nz, self.ny, self.nx = rhoA.shape
        self.tau = tuple(float(t) for t in tau)
        self.G = float(G)
        self.rho_maj, self.rho_min = float(rho_maj), float(rho_min)
        self.wet_scale = float(wet_scale)
        self.z_interface = float(z_interface)
        self.m = float(node_mass)
        self.C0 = float(C0)
        self.psi_kind = int(psi_kind)
        self.fpost = lattice.rest_populations(rhoA, rhoB)
        self.caps = []
        self.X, self.V = [], []
        for c in caps:
            mesh = membrane.Mesh(c["xyz"], c["tri"])
            v = torch.as_tensor(c.get("v", (0.0, 0.0, 0.0)), dtype=DT)
            dr = cos_deg(c["theta"])
            rv = 2.0 * dr * (self.rho_maj - self.rho_min) * self.wet_scale
            self.caps.append(dict(mesh=mesh, tri=mesh.tri, kS=float(c["kS"]), C=float(c["C"]), kV=float(c["kV"]),
                                  kB=float(c.get("kB", 0.0)), rv=abs(rv), pref=0 if rv >= 0.0 else 1,
                                  prescribed=bool(c.get("prescribed", False)), v=v))
            X = torch.as_tensor(c["xyz"], dtype=DT).clone()
            self.X.append(X)
            self.V.append(v.view(1, 3).expand_as(X).clone())
        self.n = 0
        N = self.nx * self.ny * self.nz
        self.M0 = self.fpost.sum((1, 2, 3, 4)).clone()
        self.Vsys = float(N)
        self.rho_init = self.M0 / self.Vsys
        self.L = self.labels()
        self.P_prev = [torch.zeros_like(X) for X in self.X]
        self.n_fresh = 0
        self.rho_last = self.u_last = self.F_last = None

    # ---- geometry ------------------------------------------------------
    def labels(self):
        """L[z, y, x] = k for lattice nodes inside capsule k, -1 elsewhere."""
        L = torch.full((self.nz, self.ny, self.nx), -1, dtype=torch.int64)
        for k, cap in enumerate(self.caps):
            X = self.X[k]
            lo = torch.floor(X.min(0).values).to(torch.int64) - 1
            hi = torch.ceil(X.max(0).values).to(torch.int64) + 1
            ax = [torch.arange(int(lo[d]), int(hi[d]) + 1) for d in range(3)]
            gz, gy, gx = torch.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
            P = torch.stack([gx, gy, gz], -1).reshape(-1, 3)
            inside = torch.zeros(P.shape[0], dtype=torch.bool)
            for s in range(0, P.shape[0], 512):
                inside[s:s + 512] = winding_inside(P[s:s + 512].to(DT), X, cap["tri"])
            Pi = P[inside]
            L[Pi[:, 2] % self.nz, Pi[:, 1] % self.ny, Pi[:, 0] % self.nx] = k
        return L

    def _unwrap(self, k, idx):
        """Coordinates of lattice nodes idx [K, 3] (x, y, z) as the periodic
        image nearest capsule k's centre."""
        c = self.X[k].mean(0)
        n = torch.tensor([self.nx, self.ny, self.nz], dtype=DT)
        p = idx.to(DT)
        return p + n * torch.round((c - p) / n)

    def crossed_face(self, k, x, y):
        """Faces of capsule k pierced by the segments from lattice nodes x to
        y ([K, 3] index triples, y = x + c_i): the one pierced nearest x
        (crossing parameters compared at single precision, then the lowest
        face index), or the one whose centroid is nearest the segment's
        midpoint when no face is pierced (a link grazing an edge)."""
        P0 = self._unwrap(k, x)
        d = (y - x).to(DT)
        n = torch.tensor([self.nx, self.ny, self.nz], dtype=DT)
        d = d - n * torch.round(d / n)                  # the lattice step, across the seam too
        P1 = P0 + d
        out = torch.empty(P0.shape[0], dtype=torch.int64)
        X, tri = self.X[k], self.caps[k]["tri"]
        cen = X[tri].mean(1)
        for s in range(0, P0.shape[0], 256):
            t = segment_hits(P0[s:s + 256], P1[s:s + 256], X, tri).to(torch.float32)
            tmin, arg = t.min(1)          # (the first index among equal minima)
            mid = 0.5 * (P0[s:s + 256] + P1[s:s + 256])
            near = ((cen.unsqueeze(0) - mid.unsqueeze(1)) ** 2).sum(2).argmin(1)
            out[s:s + 256] = torch.where(torch.isfinite(tmin), arg, near)
        return out

    def element_velocity(self, k, face):
        tri = self.caps[k]["tri"]
        return self.V[k][tri[face]].mean(1)            # [K, 3]

    def crossings(self, L):
        """Directed crossing links (x, i): L(x) != L(x + c_i).  Returns a list
        of (i, x [K, 3] index triples (x, y, z), capsule [K], face [K])."""
        out = []
        zz, yy, xx = torch.meshgrid(torch.arange(self.nz), torch.arange(self.ny), torch.arange(self.nx),
                                    indexing="ij")
        for i in range(1, 19):
            cx, cy, cz = (int(v) for v in C[i])
            Lnb = torch.roll(L, shifts=(-cz, -cy, -cx), dims=(0, 1, 2))     # L(x + c_i)
            m = L != Lnb
            if not bool(m.any()):
                continue
            xs = torch.stack([xx[m], yy[m], zz[m]], 1)
            ys = torch.stack([(xx[m] + cx) % self.nx, (yy[m] + cy) % self.ny, (zz[m] + cz) % self.nz], 1)
            la, lb = L[m], Lnb[m]
            cap = torch.where(la >= 0, la, lb)
            face = torch.empty(xs.shape[0], dtype=torch.int64)
            # one element per link, for both of its ends: the face pierced
            # nearest the link's start node, the end from which the link
            # points along a positive half-direction (odd i)
            s0, s1 = (xs, ys) if i % 2 == 1 else (ys, xs)
            for k in torch.unique(cap).tolist():
                sel = cap == k
                face[sel] = self.crossed_face(k, s0[sel], s1[sel])
            out.append((i, xs, cap, face))
        return out

    # ---- one step ------------------------------------------------------
    def step(self):
        nz, ny, nx = self.nz, self.ny, self.nx
        L = self.labels()
        fresh = L != self.L
        fpost = self.fpost.clone()
        rho_prev = fpost.sum(1)                          # [2, z, y, x]
        Q = [torch.zeros_like(X) for X in self.X]
        P = [torch.zeros_like(X) for X in self.X]
        R = [torch.zeros_like(X) for X in self.X]

        # 2. fresh nodes (Sec. II.E, eqs. method:freshnodes, method:masscorrection)
        M = rho_prev.sum((1, 2, 3))
        corr = 1.0 - self.C0 * (self.rho_init.sum() / self.rho_init) * (M - self.M0) / self.Vsys
        fl = torch.nonzero(fresh)
        self.n_fresh += fl.shape[0]
        new_f = []
        for z, y, x in fl.tolist():
            ell = int(L[z, y, x])
            vals = []
            for i in range(1, 19):
                cx, cy, cz = (int(v) for v in C[i])
                zn, yn, xn = (z + cz) % nz, (y + cy) % ny, (x + cx) % nx
                if int(L[zn, yn, xn]) == ell and not bool(fresh[zn, yn, xn]):
                    vals.append(rho_prev[:, zn, yn, xn])
            if vals:
                v = torch.stack(vals, 0)
                rf = torch.minimum(torch.maximum(v.mean(0) * corr, v.min(0).values), v.max(0).values)
            else:
                rf = rho_prev[:, z, y, x].clone()
            k = ell if ell >= 0 else int(self.L[z, y, x])
            X, tri = self.X[k], self.caps[k]["tri"]
            p = self._unwrap(k, torch.tensor([[x, y, z]]))[0]
            T = int(((X[tri].mean(1) - p) ** 2).sum(1).argmin())
            vel = self.V[k][tri[T]].mean(0)
            old = torch.einsum("id,ci->d", CF, fpost[:, :, z, y, x])
            feq = torch.stack([lattice.equilibrium(rf[c].view(1, 1, 1), vel.view(3, 1, 1, 1))[:, 0, 0, 0]
                               for c in (0, 1)], 0)
            new_f.append((z, y, x, feq))
            dq = (old - (rf[0] + rf[1]) * vel) / 3.0
            for b in tri[T].tolist():
                Q[k][b] += dq
        for z, y, x, feq in new_f:
            fpost[:, :, z, y, x] = feq
        rho_b = fpost.sum(1)                             # densities of the nodes for the wall term

        # 3. streaming with half-way bounce-back on the membrane (Sec. II.C)
        f = lattice.stream(fpost)
        cross = self.crossings(L)
        for i, xs, cap, face in cross:
            # (x, i) crossing: the pull at x of direction j = opp(i) has its
            # source x + c_i across the membrane; x's own outgoing f*_i comes
            # back as f_j
            j = OPP[i]
            X0, Y0, Z0 = xs[:, 0], xs[:, 1], xs[:, 2]
            v0 = torch.empty(xs.shape[0], 3, dtype=DT)
            for k in torch.unique(cap).tolist():
                sel = cap == k
                v0[sel] = self.element_velocity(k, face[sel])
            cv = (v0 * CF[j].view(1, 3)).sum(1)
            out = fpost[:, i, Z0, Y0, X0]                # [2, K]
            back = out + 2.0 * float(W[j]) * rho_b[:, Z0, Y0, X0] * cv.view(1, -1) / CS2
            f[:, j, Z0, Y0, X0] = back
            dp = (out + back).sum(0).view(-1, 1) * CF[i].view(1, 3) / 3.0   # [K, 3] per node
            for k in torch.unique(cap).tolist():
                sel = torch.nonzero(cap == k)[:, 0]
                tri = self.caps[k]["tri"][face[sel]]     # [K', 3]
                for a in range(3):
                    P[k].index_add_(0, tri[:, a], dp[sel])

        # 4. moments
        rho, j = lattice.moments(f)
        psi = torch.stack([lattice.pseudo_potential(rho[c], self.psi_kind) for c in (0, 1)], 0)

        # 5. Shan-Chen with the membrane (Sec. II.D, eq. method:interpolateshanchen)
        S = torch.stack([lattice.sc_sum(psi[c]) for c in (0, 1)], 0)    # [2 (c'), 3, z, y, x]
        for i, xs, cap, face in cross:
            cx, cy, cz = (int(v) for v in C[i])
            X0, Y0, Z0 = xs[:, 0], xs[:, 1], xs[:, 2]
            Xn, Yn, Zn = (X0 + cx) % nx, (Y0 + cy) % ny, (Z0 + cz) % nz
            side = L[Z0, Y0, X0]
            # density of the neighbour y = x + c_i seen from x's side: the
            # mean over y's neighbours with x's label
            acc = torch.zeros(2, xs.shape[0], dtype=DT)
            cnt = torch.zeros(xs.shape[0], dtype=DT)
            for q in range(1, 19):
                qx, qy, qz = (int(v) for v in C[q])
                zq, yq, xq = (Zn + qz) % nz, (Yn + qy) % ny, (Xn + qx) % nx
                m = (L[zq, yq, xq] == side).to(DT)
                acc += rho[:, zq, yq, xq] * m.view(1, -1)
                cnt += m
            rb = acc / cnt.view(1, -1)                   # cnt >= 1: x itself is one of them
            for k in torch.unique(cap).tolist():
                sel = cap == k
                rb[self.caps[k]["pref"], sel] += self.caps[k]["rv"]
            psib = torch.stack([lattice.pseudo_potential(rb[c], self.psi_kind) for c in (0, 1)], 0)
            w = float(W[i])
            # replace the neighbour's term in S at x
            for c in (0, 1):
                dS = w * (psib[c] - psi[c, Zn, Yn, Xn]).view(-1, 1) * CF[i].view(1, 3)     # [K, 3]
                for d in range(3):
                    S[c, d].index_put_((Z0, Y0, X0), dS[:, d], accumulate=True)
            # the force the pair would put on the neighbour goes to the element:
            # -(force on x) = G sum_c psi^c(x) w psib^{c'} c_i
            fr = self.G * w * (psi[0, Z0, Y0, X0] * psib[1] + psi[1, Z0, Y0, X0] * psib[0])
            fr = fr.view(-1, 1) * CF[i].view(1, 3) / 3.0
            for k in torch.unique(cap).tolist():
                sel = torch.nonzero(cap == k)[:, 0]
                tri = self.caps[k]["tri"][face[sel]]
                for a in range(3):
                    R[k].index_add_(0, tri[:, a], fr[sel])
        F = torch.stack([lattice.shan_chen_force(psi[0], S[1], self.G),
                         lattice.shan_chen_force(psi[1], S[0], self.G)], 0)

        # 6. collision
        self.fpost = lattice.collide(f, rho, j, F, self.tau)
        self.rho_last, self.F_last = rho, F
        self.u_last = lattice.physical_velocity(rho, j, F)

        # 7. node update (Sec. II.B forward Euler; Sec. II.C two-step spreading)
        self.Fb_last = []
        for k, cap in enumerate(self.caps):
            X = self.X[k]
            Fb = membrane.elastic_forces(cap["mesh"], X, cap["kS"], cap["C"], cap["kV"])
            if cap["kB"] > 0.0:
                Fb = Fb + bending.bending_forces(X, cap["tri"], cap["kB"])
            Fb = Fb + 0.5 * (P[k] + self.P_prev[k]) + Q[k] + R[k]
            self.Fb_last.append(Fb)
            if cap["prescribed"]:
                self.V[k] = cap["v"].view(1, 3).expand_as(X).clone()
            else:
                self.V[k] = self.V[k] + Fb / self.m
            self.X[k] = X + self.V[k]
            if not bool(torch.isfinite(self.V[k]).all()) or float(self.V[k].abs().max()) >= 1.0:
                raise FloatingPointError("capsule %d: node speed beyond one lattice unit per step" % k)
        self.P_prev = P
        self.L = L
        self.n += 1

    def run(self, n):
        for _ in range(n):
            self.step()
        return self

    # ---- observables ---------------------------------------------------
    def mass(self):
        return self.fpost.sum((1, 2, 3, 4))

    def fluid_momentum(self):
        return torch.einsum("id,cizyx->d", CF, self.fpost)

    def particle_momentum(self):
        return sum(self.m * V.sum(0) for V in self.V)

    def pending_momentum(self):
        """Half of the last step's exchanged momentum, which the nodes get
        with the next step."""
        return sum(0.5 * P.sum(0) for P in self.P_prev)

    def region_mass(self, k):
        """Mass per component of the fluid with label k (-1 = outside)."""
        m = (self.L == k).to(DT)
        return (self.fpost.sum(1) * m.unsqueeze(0)).sum((1, 2, 3))

    def capsule_obs(self, k):
        V, A, com, mu = membrane.shape_moments(self.X[k], self.caps[k]["tri"])
        return dict(com=com, V=V, A=A, height=com[2] - self.z_interface)


def from_workload(wl, **over):
    """BounceBackSim from a seeded workload object (duck-typed; capsules may
    carry `v` and `prescribed`)."""
    caps = []
    for c in wl.capsules:
        xyz, tri = c.mesh()
        caps.append(dict(xyz=xyz, tri=tri, kS=c.kS, C=c.C, kV=c.kV, theta=c.theta_deg, kB=getattr(c, "kB", 0.0),
                         v=getattr(c, "v", (0.0, 0.0, 0.0)), prescribed=getattr(c, "prescribed", False)))
    kw = dict(tau=wl.tau, G=wl.G, rho_maj=wl.rho_maj, rho_min=wl.rho_min, z_interface=wl.z_interface,
              wet_scale=wl.wet_scale, node_mass=getattr(wl, "node_mass", 5.0), C0=getattr(wl, "mass_c0", 2500.0),
              psi_kind=wl.psi_kind)
    kw.update(over)
    return BounceBackSim(wl.rhoA.astype("float64"), wl.rhoB.astype("float64"), caps, **kw)
