"""One coupled time step, FP64 (test infrastructure only).

State at the start of step n: post-collision populations f*^{n-1} and node
positions X^n.  The step, in this order:

 1. stream: f^n = pull(f*^{n-1}) with half-way bounce-back at walls
    (Sec. II.A; Sec. II.C eq. method:SBB), or with on-site velocity
    boundaries on the rows y = 0 and y = ny - 1 (walls = 2);
 2. densities rho^c = sum_i f_i^c, momenta j^c = sum_i f_i^c c_i, and the
    pseudo-potential: psi = rho for the workloads (psi_kind 0), or the
    1 - exp(-rho/rho0), rho0 = 1, that Sec. II.D names (psi_kind 1);
 3. node forces at X^n: Skalak plus volume (Sec. II.B) plus the wettability
    reaction.  The wettability term follows Sec. II.D: a virtual density
    offset rho_v added to the preferred component, with the particle colour
    Delta rho = rho_v / (2 (rho_maj - rho_min)) and Delta rho = cos(theta)
    (the theta = acos(Delta rho) law of Sec. III.D), times a strength
    factor wet_scale (1 = the law as written).  Carried to the
    immersed boundary, the offset is a field phi(x) = |rho_v| sum_b A_b delta
    (x - X_b) added to the preferred component's pseudo-potential when the
    other component's force is formed, and its reaction on node b is
        R_b = -G |rho_v| A_b sum_y delta(y - X_b) sum_i w_i psi^np(y + c_i) c_i
    (np = the non-preferred component), which keeps fluid plus membrane
    momentum conserved, as Sec. II.D requires of the cross-boundary force;
    when enabled, Helfrich bending (Sec. II.B, bending.py) and the
    particle-particle repulsion of Sec. III.E between nodes of different
    capsules (contact.py);
 4. spreading F_ib(x) = sum_b F_b delta(x - X_b) and the phi fields;
 5. fluid force F^c = -psi^c G sum_i w_i (psi^c' + phi^c')(x + c_i) c_i
    + (rho^c / rho) F_ib (Sec. II.D eq. method:shanchen; the body force is
    shared by mass fraction);
 6. BGK collision with the equilibrium-velocity shift (Sec. II.A);
 7. u^n = (sum j + F/2) / rho, U_b = sum u^n delta, X^{n+1} = X^n + U_b
    (forward Euler, Sec. II.B; massless immersed-boundary nodes).

Parity status: every function used here is pinned by the tests listed in
lattice.py, ibm.py and membrane.py and by the whole-step invariants in
tests/test_oracle_sim.py (mass, momentum, flat interface, wetting
neutrality and mirror antisymmetry, checkpoint replay).  The full coupled
trajectory itself has no printed value to compare with: beyond those
invariants it is parity unpinned.
"""

import math

import torch

from . import bending, contact, ibm, lattice, membrane

DT = torch.float64


def cos_deg(theta):
    """cos of an angle in degrees, exactly 0 at 90 degrees."""
    if isinstance(theta, torch.Tensor) and theta.requires_grad:
        return torch.cos(theta * (math.pi / 180.0))
    t = float(theta)
    if t == 90.0:
        return 0.0
    return math.cos(math.radians(t))


class OracleSim:
    """FP64 reference simulation.

    rhoA, rhoB: [nz, ny, nx] initial densities.  caps: list of dicts with
    keys xyz (rest = initial absolute positions, [N, 3]), tri ([F, 3],
    outward counter-clockwise), kS, C, kV, theta (degrees).  Per-capsule
    kS and theta, and G, may be float64 tensors that require grad: the step
    is then differentiable end to end.
    """

    def __init__(self, rhoA, rhoB, caps=(), tau=(1.0, 1.0), G=3.6, walls=0,
                 u_lo=(0.0, 0.0, 0.0), u_hi=(0.0, 0.0, 0.0), rho_maj=0.7,
                 rho_min=0.04, z_interface=0.0, wet_scale=1.0, differentiable=False,
                 rep_eps=0.0, rep_d0=1.25, psi_kind=0):
        rhoA = torch.as_tensor(rhoA, dtype=DT)
        rhoB = torch.as_tensor(rhoB, dtype=DT)
        self.nz, self.ny, self.nx = rhoA.shape
        self.dims = (self.nx, self.ny, self.nz)
        self.tau = tuple(float(t) for t in tau)
        self.G = G
        self.walls = int(walls)
        self.u_lo = tuple(float(v) for v in u_lo)
        self.u_hi = tuple(float(v) for v in u_hi)
        self.rho_maj = float(rho_maj)
        self.rho_min = float(rho_min)
        self.wet_scale = float(wet_scale)
        self.psi_kind = int(psi_kind)
        self.rep_eps = float(rep_eps)
        self.rep_d0 = float(rep_d0)
        self.z_interface = float(z_interface)
        self.diff = differentiable
        self.fpost = lattice.rest_populations(rhoA, rhoB)
        self.f_solid = self.fpost.clone()
        self.caps = []
        for c in caps:
            mesh = membrane.Mesh(c["xyz"], c["tri"])
            self.caps.append(dict(mesh=mesh, kS=c["kS"], C=float(c["C"]),
                                  kV=float(c["kV"]), theta=c["theta"], kB=float(c.get("kB", 0.0))))
        self.X = [torch.as_tensor(c["xyz"], dtype=DT).clone() for c in caps]
        self.n = 0
        self.fluid_mask = torch.ones(self.ny, dtype=torch.bool)
        if self.walls == 1:
            self.fluid_mask[0] = False
            self.fluid_mask[self.ny - 1] = False
        self.rho_last = self.u_last = self.Fib_last = self.phi_last = None
        self.Fb_last = None

    # ---- pieces -------------------------------------------------------
    def _reset_solid(self, f):
        if self.walls != 1:
            return f
        f = f.clone()
        f[:, :, :, 0, :] = self.f_solid[:, :, :, 0, :]
        f[:, :, :, -1, :] = self.f_solid[:, :, :, -1, :]
        return f

    def colour(self, k):
        """(rho_v signed, preferred component) of capsule k."""
        dr = cos_deg(self.caps[k]["theta"])
        rv = 2.0 * dr * (self.rho_maj - self.rho_min) * self.wet_scale
        if isinstance(rv, torch.Tensor):
            pref = 0 if float(rv.detach()) >= 0.0 else 1
        else:
            pref = 0 if rv >= 0.0 else 1
        return rv, pref

    def node_forces(self, rho):
        """Per-capsule node forces at X^n and the wettability weights."""
        w = self.walls
        S_psi = None
        Fb, phiw = [], []
        for k, cap in enumerate(self.caps):
            X = self.X[k]
            F = membrane.elastic_forces(cap["mesh"], X, cap["kS"], cap["C"],
                                        cap["kV"], create_graph=self.diff)
            if cap["kB"] > 0.0:
                # Helfrich bending (Sec. II.B, eq. surf_dens)
                F = F + bending.bending_forces(X, cap["mesh"].tri, cap["kB"])
            rv, pref = self.colour(k)
            is_zero = (not isinstance(rv, torch.Tensor)) and rv == 0.0
            a = cap["mesh"].node_area * (rv.abs() if isinstance(rv, torch.Tensor) else abs(rv))
            if not is_zero:
                if S_psi is None:
                    S_psi = [lattice.sc_sum(lattice.wall_copy(lattice.pseudo_potential(rho[c], self.psi_kind), w), w)
                             for c in (0, 1)]
                npc = 1 - pref
                interp = ibm.interpolate(S_psi[npc], X)          # [N, 3]
                F = F - self.G * a.unsqueeze(1) * interp
            pa = a if pref == 0 else torch.zeros_like(a)
            pb = a if pref == 1 else torch.zeros_like(a)
            Fb.append(F)
            phiw.append(torch.stack([pa, pb], 1))
        if self.rep_eps > 0.0:
            # particle-particle repulsion at X^n (Sec. III.E)
            R = contact.repulsion_forces(self.X, self.dims, self.rep_eps, self.rep_d0, w)
            Fb = [F + Rk for F, Rk in zip(Fb, R)]
        return Fb, phiw

    def step(self):
        w = self.walls
        f = lattice.stream(self.fpost, w, self.u_lo, self.u_hi)
        f = self._reset_solid(f)
        rho, j = lattice.moments(f)
        nz, ny, nx = self.nz, self.ny, self.nx
        if self.caps:
            Fb, phiw = self.node_forces(rho)
            Xall = torch.cat(self.X, 0)
            vals = torch.cat([torch.cat(Fb, 0), torch.cat(phiw, 0)], 1)
            fld = ibm.spread(vals, Xall, self.dims)
            Fib, phi = fld[:3], fld[3:]
        else:
            Fb = []
            Fib = torch.zeros(3, nz, ny, nx, dtype=DT)
            phi = torch.zeros(2, nz, ny, nx, dtype=DT)
        # the virtual density is a field added to the pseudo-potential (the
        # reading under the immersed boundary; linear in phi for any psi)
        psi = [lattice.pseudo_potential(rho[c], self.psi_kind) for c in (0, 1)]
        psi_tot = [lattice.wall_copy(psi[c] + phi[c], w) for c in (0, 1)]
        S_tot = [lattice.sc_sum(psi_tot[c], w) for c in (0, 1)]
        rsum = rho[0] + rho[1]
        F = []
        for c in (0, 1):
            Fc = lattice.shan_chen_force(psi[c], S_tot[1 - c], self.G)
            Fc = Fc + (rho[c] / rsum).unsqueeze(0) * Fib
            F.append(Fc)
        F = torch.stack(F, 0)
        fpost = lattice.collide(f, rho, j, F, self.tau)
        self.fpost = self._reset_solid(fpost)
        u = lattice.physical_velocity(rho, j, F)
        if self.caps:
            self.X = [X + ibm.interpolate(u, X) for X in self.X]
        self.rho_last, self.u_last = rho, u
        self.Fib_last, self.phi_last, self.Fb_last = Fib, phi, Fb
        self.F_last = F
        self.n += 1

    def run(self, n):
        for _ in range(n):
            self.step()
        return self

    # ---- observables (FP64) -------------------------------------------
    def mass(self):
        m = self.fpost[:, :, :, self.fluid_mask, :].sum((1, 2, 3, 4))
        return m

    def momentum(self):
        fp = self.fpost[:, :, :, self.fluid_mask, :]
        return torch.einsum("id,cizyx->d", lattice.CF, fp)

    def capsule_obs(self, k):
        cap = self.caps[k]
        V, A, com, mu = membrane.shape_moments(self.X[k], cap["mesh"].tri)
        ax = membrane.semi_axes(V, mu)
        D = (ax.max() - ax.min()) / (ax.max() + ax.min())
        return dict(com=com, V=V, A=A, axes=ax, D=D,
                    height=com[2] - self.z_interface)


def from_workload(wl, differentiable=False, **over):
    """OracleSim from a seeded workload object (duck-typed: needs rhoA, rhoB,
    capsules with mesh(), tau, G, walls, wall_u_lo/hi, rho_maj/min,
    z_interface)."""
    caps = []
    for c in wl.capsules:
        xyz, tri = c.mesh()
        caps.append(dict(xyz=xyz, tri=tri, kS=c.kS, C=c.C, kV=c.kV, theta=c.theta_deg,
                         kB=getattr(c, "kB", 0.0)))
    kw = dict(tau=wl.tau, G=wl.G, walls=wl.walls, u_lo=wl.wall_u_lo, u_hi=wl.wall_u_hi,
              rho_maj=wl.rho_maj, rho_min=wl.rho_min, z_interface=wl.z_interface,
              wet_scale=wl.wet_scale, differentiable=differentiable,
              rep_eps=getattr(wl, "rep_eps", 0.0), rep_d0=getattr(wl, "rep_d0", 1.25),
              psi_kind=getattr(wl, "psi_kind", 0))
    kw.update(over)
    return OracleSim(wl.rhoA.astype("float64"), wl.rhoB.astype("float64"), caps, **kw)


# ---- gradients of capsule objectives (reference for the adjoint) ----------

def objective(sim, kind, cap=0):
    """J at the current state: 'com_z' = node-mean z of capsule `cap` minus
    the interface plane (Sec. III.D, eq. interface:contactangle), or
    'taylor_D' (Sec. III.A, eq. results:taylorparameter)."""
    X = sim.X[cap]
    if kind == "com_z":
        return X[:, 2].mean() - sim.z_interface
    if kind == "taylor_D":
        return membrane.taylor_D(X, sim.caps[cap]["mesh"].tri)
    raise KeyError(kind)


def gradient(make_sim, steps, every, kind, cap=0):
    """J and dJ/d(theta [rad], kS, G) by reverse-mode autograd with
    checkpoint and recompute: the forward keeps the state every `every`
    steps; the backward replays each segment from its checkpoint with the
    graph recorded and pulls the adjoint through it.  theta, kS act on every
    capsule (the derivative is the sum over capsules).

    make_sim(theta_deg, kS, G) must return a fresh OracleSim with
    differentiable=True whose capsules use those (possibly tensor) values."""
    th0, ks0, g0 = make_sim.params
    sim = make_sim(th0, ks0, g0)
    ckpts = []
    with torch.no_grad():
        for k in range(steps):
            if k % every == 0:
                ckpts.append((k, sim.fpost.clone(), [x.clone() for x in sim.X]))
            sim.step()
        J = float(objective(sim, kind, cap))
    # seed at the final state
    Xf = [x.detach().clone().requires_grad_(True) for x in sim.X]
    with torch.enable_grad():
        sim.X = Xf
        Jt = objective(sim, kind, cap)
        lam_X = list(torch.autograd.grad(Jt, Xf, allow_unused=True))
    lam_X = [torch.zeros_like(x) if l is None else l for l, x in zip(lam_X, Xf)]
    lam_f = torch.zeros_like(sim.fpost)
    g = torch.zeros(3, dtype=DT)
    for (k0, f0, X0) in reversed(ckpts):
        n = min(every, steps - k0)
        th = torch.tensor(float(th0), dtype=DT, requires_grad=True)
        ks = torch.tensor(float(ks0), dtype=DT, requires_grad=True)
        G = torch.tensor(float(g0), dtype=DT, requires_grad=True)
        with torch.enable_grad():
            seg = make_sim(th, ks, G)
            fs = f0.clone().requires_grad_(True)
            Xs = [x.clone().requires_grad_(True) for x in X0]
            seg.fpost = fs
            seg.X = list(Xs)
            for _ in range(n):
                seg.step()
            outs = [seg.fpost] + list(seg.X)
            grads = torch.autograd.grad(outs, [fs] + Xs + [th, ks, G], grad_outputs=[lam_f] + lam_X,
                                        allow_unused=True)
        lam_f = grads[0]
        lam_X = [gx if gx is not None else torch.zeros_like(x) for gx, x in zip(grads[1:1 + len(Xs)], Xs)]
        for i, gp in enumerate(grads[1 + len(Xs):]):
            if gp is not None:
                g[i] += gp.detach()
    # theta was in degrees inside the simulation: report d/d(radian)
    g[0] = g[0] * (180.0 / math.pi)
    return J, g
