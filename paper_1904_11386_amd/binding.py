"""Thin ctypes binding of liblbm.so (include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP
library.  PyTorch supplies the device workspace (one uint8 tensor) and the
stream.  Importing this module does not load the library; the first Sim
does, and raises if liblbm.so has not been built.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_ESTATE, LBM_EUNSTABLE = range(6)
LBM_FP32, LBM_FP16 = 0, 1
ERR_NAMES = {1: "LBM_EINVAL", 2: "LBM_ENOMEM", 3: "LBM_EHIP", 4: "LBM_ESTATE", 5: "LBM_EUNSTABLE"}


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("precision", C.c_int32), ("walls", C.c_int32), ("n_slots", C.c_int32),
                ("check_every", C.c_int32), ("use_graphs", C.c_int32),
                ("tau", C.c_double * 2), ("G", C.c_double),
                ("rho_maj", C.c_double), ("rho_min", C.c_double),
                ("wall_u_lo", C.c_double * 3), ("wall_u_hi", C.c_double * 3),
                ("z_interface", C.c_double), ("mass_tol", C.c_double), ("wet_scale", C.c_double),
                ("ring_len", C.c_int32), ("stream_policy", C.c_int32), ("zchunk", C.c_int32),
                ("psi_kind", C.c_int32), ("rep_eps", C.c_double), ("rep_d0", C.c_double),
                ("coupling", C.c_int32), ("node_mass", C.c_double), ("mass_c0", C.c_double),
                ("deterministic", C.c_int32), ("mass_fix", C.c_int32), ("lattice_passes", C.c_int32)]


class Obs(C.Structure):
    _fields_ = [("mass", C.c_double * 2), ("momentum", C.c_double * 3), ("step", C.c_int64),
                ("particle_momentum", C.c_double * 3), ("pending_momentum", C.c_double * 3),
                ("mass_ledger", C.c_double * 2)]


class CapObs(C.Structure):
    _fields_ = [("com", C.c_double * 3), ("volume", C.c_double), ("area", C.c_double),
                ("axes", C.c_double * 3), ("taylor_D", C.c_double), ("height", C.c_double)]


_lib = None

EXPORTS = ["lbm_workspace_bytes", "lbm_init", "lbm_capsules_add", "lbm_capsules_velocity", "lbm_capsules_bending",
           "lbm_reference_relax", "lbm_debug_labels", "lbm_get_node_velocities",
           "lbm_step", "lbm_step_timed", "lbm_observables", "lbm_observables_noalloc",
           "lbm_get_fields", "lbm_get_nodes", "lbm_get_node_forces", "lbm_get_spread",
           "lbm_debug_bins", "lbm_state_save", "lbm_state_load", "lbm_adjoint_forward", "lbm_adjoint_backward",
           "lbm_adjoint_seed", "lbm_adjoint_record", "lbm_adjoint_step", "lbm_adjoint_grads",
           "lbm_destroy", "lbm_last_error"]
LBM_OBJ_COM_Z, LBM_OBJ_TAYLOR_D = 0, 1


def load(path: str = None):
    """Load liblbm.so (LIB_PATH unless a path is given) and declare its
    signatures (no device work)."""
    global _lib
    path = path or LIB_PATH
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("liblbm.so is not built: run `python -m paper_1904_11386_amd.build` "
                           "(no CPU fallback exists)")
    lib = C.CDLL(path)
    P = C.POINTER
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "lbm_workspace_bytes": ([P(Params), i64, i64, P(i64)], C.c_int),
        "lbm_init": ([P(Params), P(C.c_float), P(C.c_float), vp, i64, i64, i64, vp, P(vp)], C.c_int),
        "lbm_capsules_add": ([vp, i32, P(i32), P(i32), P(d), P(i32), P(d), P(d), P(d), P(d), P(i32)], C.c_int),
        "lbm_capsules_bending": ([vp, i32, i32, P(d)], C.c_int),
        "lbm_capsules_velocity": ([vp, i32, i32, P(d), i32], C.c_int),
        "lbm_debug_labels": ([vp, P(i32)], C.c_int),
        "lbm_get_node_velocities": ([vp, P(C.c_float)], C.c_int),
        "lbm_reference_relax": ([vp, i32, C.c_double, C.c_double, C.c_double, C.c_double], C.c_int),
        "lbm_step": ([vp, i32], C.c_int),
        "lbm_step_timed": ([vp, i32, P(d)], C.c_int),
        "lbm_observables": ([vp, P(Obs), P(CapObs)], C.c_int),
        "lbm_observables_noalloc": ([vp, P(Obs), P(CapObs)], C.c_int),
        "lbm_get_fields": ([vp, P(C.c_float), P(C.c_float), P(C.c_float)], C.c_int),
        "lbm_get_nodes": ([vp, P(d)], C.c_int),
        "lbm_get_node_forces": ([vp, P(C.c_float)], C.c_int),
        "lbm_get_spread": ([vp, P(C.c_float), P(C.c_float)], C.c_int),
        "lbm_debug_bins": ([vp, P(i32), P(i32)], C.c_int),
        "lbm_state_save": ([vp, i32], C.c_int),
        "lbm_state_load": ([vp, i32], C.c_int),
        "lbm_adjoint_forward": ([vp, i32, i32, i32, i32, P(d)], C.c_int),
        "lbm_adjoint_backward": ([vp, P(d)], C.c_int),
        "lbm_adjoint_seed": ([vp, i32, i32], C.c_int),
        "lbm_adjoint_record": ([vp, i32], C.c_int),
        "lbm_adjoint_step": ([vp, i32], C.c_int),
        "lbm_adjoint_grads": ([vp, P(d)], C.c_int),
        "lbm_destroy": ([vp], None),
        "lbm_last_error": ([vp], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    if path == LIB_PATH:
        _lib = lib
    return lib


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERR_NAMES.get(code, str(code)), msg))
        self.code = code


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def make_params(nx, ny, nz, tau=(1.0, 1.0), G=3.6, walls=0, wall_u_lo=(0, 0, 0), wall_u_hi=(0, 0, 0),
                rho_maj=0.7, rho_min=0.04, z_interface=0.0, precision=LBM_FP32, n_slots=0,
                check_every=0, mass_tol=1e-3, wet_scale=1.0, use_graphs=1, ring_len=0, stream_policy=0,
                zchunk=0, rep_eps=0.0, rep_d0=1.25, psi_kind=0, coupling=0, node_mass=5.0, mass_c0=2500.0,
                deterministic=0, mass_fix=0, lattice_passes=0):
    p = Params()
    p.nx, p.ny, p.nz = nx, ny, nz
    p.precision = precision
    p.walls = walls
    p.n_slots = n_slots
    p.check_every = check_every
    p.tau[0], p.tau[1] = tau
    p.G = G
    p.rho_maj, p.rho_min = rho_maj, rho_min
    for k in range(3):
        p.wall_u_lo[k] = wall_u_lo[k]
        p.wall_u_hi[k] = wall_u_hi[k]
    p.z_interface = z_interface
    p.mass_tol = mass_tol
    p.wet_scale = wet_scale
    p.use_graphs = use_graphs
    p.ring_len = ring_len
    p.stream_policy = stream_policy
    p.zchunk = zchunk
    p.rep_eps = rep_eps
    p.rep_d0 = rep_d0
    p.psi_kind = psi_kind
    p.coupling = coupling
    p.node_mass = node_mass
    p.mass_c0 = mass_c0
    p.deterministic = deterministic
    p.mass_fix = mass_fix
    p.lattice_passes = lattice_passes
    return p


def workspace_bytes(params, max_nodes, max_faces):
    lib = load()
    out = C.c_int64()
    r = lib.lbm_workspace_bytes(C.byref(params), max_nodes, max_faces, C.byref(out))
    if r != LBM_OK:
        raise LbmError(r, lib.lbm_last_error(None).decode())
    return out.value


class Sim:
    """One simulation context on a torch CUDA (HIP) device."""

    def __init__(self, params: Params, rhoA, rhoB, max_nodes=0, max_faces=0, device="cuda",
                 stream=None):
        import torch
        self.lib = load()
        self.params = params
        self.N = params.nx * params.ny * params.nz
        nbytes = workspace_bytes(params, max_nodes, max_faces)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        # a stream of its own (default priority), so the library can capture
        # graphs; torch's allocator is told the workspace is used there
        self.stream = stream if stream is not None else torch.cuda.Stream(self.workspace.device)
        self.workspace.record_stream(self.stream)
        torch.cuda.synchronize(self.workspace.device)
        rA = np.ascontiguousarray(rhoA, dtype=np.float32).reshape(-1)
        rB = np.ascontiguousarray(rhoB, dtype=np.float32).reshape(-1)
        if rA.size != self.N or rB.size != self.N:
            raise ValueError("density arrays must have nx*ny*nz entries")
        ctx = C.c_void_p()
        r = self.lib.lbm_init(C.byref(params), _ptr(rA, C.c_float), _ptr(rB, C.c_float),
                              C.c_void_p(self.workspace.data_ptr()), nbytes, max_nodes, max_faces,
                              C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if r != LBM_OK:
            raise LbmError(r, self.lib.lbm_last_error(None).decode())
        self.ctx = ctx
        self.n_nodes = 0
        self.n_caps = 0

    def _check(self, r):
        if r != LBM_OK:
            raise LbmError(r, self.lib.lbm_last_error(self.ctx).decode())

    def add_capsules(self, nodes_per_cap, faces_per_cap, xyz, tri, kS, Cs, kV, theta):
        npc = np.ascontiguousarray(nodes_per_cap, dtype=np.int32)
        fpc = np.ascontiguousarray(faces_per_cap, dtype=np.int32)
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (kS, Cs, kV, theta)]
        first = C.c_int32()
        self._check(self.lib.lbm_capsules_add(self.ctx, len(npc), _ptr(npc, C.c_int32), _ptr(fpc, C.c_int32),
                                              _ptr(xyz, C.c_double), _ptr(tri, C.c_int32),
                                              *[_ptr(a, C.c_double) for a in arrs], C.byref(first)))
        self.n_nodes += int(npc.sum())
        self.n_caps += len(npc)
        return first.value

    def reference_relax(self, nsteps, gamma, w, z_interface, mobility):
        """Membrane-only relaxation under the emulated tension (no fluid)."""
        self._check(self.lib.lbm_reference_relax(self.ctx, int(nsteps), float(gamma), float(w), float(z_interface),
                                                 float(mobility)))

    def set_velocity(self, first_id, v, prescribed=False):
        """Node velocity of each capsule first_id .. first_id + len(v) - 1,
        kept while prescribed (bounce-back coupling); before the first step
        or between steps."""
        v = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1, 3))
        self._check(self.lib.lbm_capsules_velocity(self.ctx, int(first_id), v.shape[0], _ptr(v, C.c_double),
                                                   1 if prescribed else 0))

    def labels(self):
        """Per lattice node: the capsule whose membrane encloses it, or -1
        (bounce-back coupling), for the current node positions."""
        p = self.params
        out = np.empty(self.N, np.int32)
        self._check(self.lib.lbm_debug_labels(self.ctx, _ptr(out, C.c_int32)))
        return out.reshape((p.nz, p.ny, p.nx))

    def node_velocities(self):
        V = np.empty((self.n_nodes, 3), np.float32)
        self._check(self.lib.lbm_get_node_velocities(self.ctx, _ptr(V, C.c_float)))
        return V

    def set_bending(self, first_id, kB):
        """Helfrich bending moduli of the capsules first_id .. first_id + len(kB) - 1."""
        kB = np.ascontiguousarray(kB, dtype=np.float64)
        self._check(self.lib.lbm_capsules_bending(self.ctx, int(first_id), len(kB), _ptr(kB, C.c_double)))

    def step(self, n=1):
        self._check(self.lib.lbm_step(self.ctx, int(n)))

    KERNELS = ["clear", "density", "volume", "faces", "nodes", "scan", "scatter", "repulse", "bend", "spread",
               "collide", "interp"]

    def step_timed(self, n):
        """Run n steps with HIP events around each kernel group; returns
        {kernel: summed ms}."""
        ms = (C.c_double * len(self.KERNELS))()
        self._check(self.lib.lbm_step_timed(self.ctx, int(n), ms))
        return {k: ms[i] for i, k in enumerate(self.KERNELS)}

    def observables(self):
        o = Obs()
        caps = (CapObs * max(self.n_caps, 1))()
        self._check(self.lib.lbm_observables(self.ctx, C.byref(o), caps if self.n_caps else None))
        out = dict(mass=np.array(o.mass[:]), momentum=np.array(o.momentum[:]), step=o.step, caps=[],
                   particle_momentum=np.array(o.particle_momentum[:]), pending_momentum=np.array(o.pending_momentum[:]),
                   mass_ledger=np.array(o.mass_ledger[:]))
        for k in range(self.n_caps):
            c = caps[k]
            out["caps"].append(dict(com=np.array(c.com[:]), V=c.volume, A=c.area, axes=np.array(c.axes[:]),
                                    D=c.taylor_D, height=c.height))
        return out

    def observables_noalloc(self):
        """As observables(), through lbm_observables_noalloc (no device
        allocation: the library's fixed per-device scratch)."""
        o = Obs()
        caps = (CapObs * max(self.n_caps, 1))()
        self._check(self.lib.lbm_observables_noalloc(self.ctx, C.byref(o), caps if self.n_caps else None))
        out = dict(mass=np.array(o.mass[:]), momentum=np.array(o.momentum[:]), step=o.step, caps=[],
                   particle_momentum=np.array(o.particle_momentum[:]), pending_momentum=np.array(o.pending_momentum[:]),
                   mass_ledger=np.array(o.mass_ledger[:]))
        for k in range(self.n_caps):
            c = caps[k]
            out["caps"].append(dict(com=np.array(c.com[:]), V=c.volume, A=c.area, axes=np.array(c.axes[:]),
                                    D=c.taylor_D, height=c.height))
        return out

    def fields(self):
        p = self.params
        shp = (p.nz, p.ny, p.nx)
        ra = np.empty(self.N, np.float32)
        rb = np.empty(self.N, np.float32)
        u = np.empty(3 * self.N, np.float32)
        self._check(self.lib.lbm_get_fields(self.ctx, _ptr(ra, C.c_float), _ptr(rb, C.c_float), _ptr(u, C.c_float)))
        return ra.reshape(shp), rb.reshape(shp), u.reshape((3,) + shp)

    def nodes(self):
        x = np.empty((self.n_nodes, 3), np.float64)
        self._check(self.lib.lbm_get_nodes(self.ctx, _ptr(x, C.c_double)))
        return x

    def node_forces(self):
        F = np.empty((self.n_nodes, 3), np.float32)
        self._check(self.lib.lbm_get_node_forces(self.ctx, _ptr(F, C.c_float)))
        return F

    def spread(self):
        p = self.params
        shp = (p.nz, p.ny, p.nx)
        F = np.empty(3 * self.N, np.float32)
        ph = np.empty(2 * self.N, np.float32)
        self._check(self.lib.lbm_get_spread(self.ctx, _ptr(F, C.c_float), _ptr(ph, C.c_float)))
        return F.reshape((3,) + shp), ph.reshape((2,) + shp)

    def bins(self):
        t = np.empty(self.n_nodes, np.int32)
        b = np.empty((self.n_nodes, 3), np.int32)
        self._check(self.lib.lbm_debug_bins(self.ctx, _ptr(t, C.c_int32), _ptr(b, C.c_int32)))
        return t, b

    def adjoint_forward(self, nsteps, every, objective=LBM_OBJ_COM_Z, capsule=0):
        """Run nsteps keeping checkpoints every `every` steps; returns J."""
        J = C.c_double()
        self._check(self.lib.lbm_adjoint_forward(self.ctx, int(nsteps), int(every), int(objective), int(capsule),
                                                 C.byref(J)))
        return J.value

    def adjoint_backward(self):
        """dJ/d(theta [rad], kS, G) of the last adjoint_forward."""
        g = (C.c_double * 3)()
        self._check(self.lib.lbm_adjoint_backward(self.ctx, g))
        return np.array(g[:])

    def adjoint_seed(self, objective=LBM_OBJ_COM_Z, capsule=0):
        """lambda_X = dJ/dX at the current positions; other adjoint state zeroed."""
        self._check(self.lib.lbm_adjoint_seed(self.ctx, int(objective), int(capsule)))

    def adjoint_record(self, nsteps):
        """Recompute nsteps states from the current one into the ring."""
        self._check(self.lib.lbm_adjoint_record(self.ctx, int(nsteps)))

    def adjoint_step(self, ring_index):
        """Adjoint of recorded step ring_index (reverse order, last first)."""
        self._check(self.lib.lbm_adjoint_step(self.ctx, int(ring_index)))

    def adjoint_grads(self):
        """dJ/d(theta [rad], kS, G) accumulated since the seed."""
        g = (C.c_double * 3)()
        self._check(self.lib.lbm_adjoint_grads(self.ctx, g))
        return np.array(g[:])

    def save(self, slot):
        self._check(self.lib.lbm_state_save(self.ctx, slot))

    def load(self, slot):
        self._check(self.lib.lbm_state_load(self.ctx, slot))

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            self.lib.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sim_from_workload(wl, precision=LBM_FP32, n_slots=0, check_every=0, device="cuda", use_graphs=1, ring_len=0,
                      stream_policy=0, zchunk=0, mass_tol=1e-3, deterministic=0, mass_fix=0, lattice_passes=0):
    """Build a Sim for a seeded workload (paper_1904_11386_amd.workloads)."""
    npc, fpc, xyz, tri = wl.meshes()
    p = make_params(wl.nx, wl.ny, wl.nz, tau=wl.tau, G=wl.G, walls=wl.walls, wall_u_lo=wl.wall_u_lo,
                    wall_u_hi=wl.wall_u_hi, rho_maj=wl.rho_maj, rho_min=wl.rho_min,
                    z_interface=wl.z_interface, precision=precision, n_slots=n_slots,
                    check_every=check_every, mass_tol=mass_tol, wet_scale=wl.wet_scale, use_graphs=use_graphs,
                    ring_len=ring_len,
                    stream_policy=stream_policy, zchunk=zchunk, rep_eps=wl.rep_eps, rep_d0=wl.rep_d0,
                    psi_kind=wl.psi_kind, coupling=getattr(wl, "coupling", 0),
                    node_mass=getattr(wl, "node_mass", 5.0), mass_c0=getattr(wl, "mass_c0", 2500.0),
                    deterministic=deterministic, mass_fix=mass_fix, lattice_passes=lattice_passes)
    s = Sim(p, wl.rhoA, wl.rhoB, max_nodes=int(npc.sum()), max_faces=int(fpc.sum()), device=device)
    if len(npc):
        kS, Cs, kV, th = wl.cap_params()
        first = s.add_capsules(npc, fpc, xyz, tri, kS, Cs, kV, th)
        kB = np.array([c.kB for c in wl.capsules], np.float64)
        if (kB > 0).any():
            s.set_bending(first, kB)
        if getattr(wl, "coupling", 0) == 1:
            for k, c in enumerate(wl.capsules):
                if any(c.v) or c.prescribed:
                    s.set_velocity(first + k, [c.v], c.prescribed)
    return s
