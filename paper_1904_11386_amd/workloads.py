"""Seeded synthetic inputs for the two-component capsule lattice Boltzmann step.

This module builds inputs only: initial density layers, triangulated capsule
meshes and per-capsule parameters.  It holds none of the method's arithmetic
(no populations, forces, deltas or collisions), so both the HIP path and the
FP64 oracle may consume what it produces.

Mesh: a geodesic icosphere of frequency n = 2^k (10 n^2 + 2 nodes, 20 n^2
triangles), the same family of meshes the paper uses for its capsules
(Sec. III, N_b = 1442 / N_f = 2880 is frequency 12).  It is built from the
coordinate icosahedron (0, +-1, +-phi) and its cyclic permutations by
midpoint subdivision with projection to the sphere.  That icosahedron is
mirror-symmetric in x, y and z.

Coordinates are snapped to multiples of 2^-20 lattice units.  With that
grid every node position is exactly an integer anchor plus an FP32 offset
(for offsets below 16 lu), so the FP32 device path and the FP64 oracle start
from bit-identical positions.

Workloads (sizes as stated, seeds numpy.random.default_rng(1904 + k)):
  c1      32^3 periodic, A below z = 16, one R = 6 (642-node) capsule at z = 16
  c2      128^3 periodic, interface z = 64, 8 capsules R = 8 (2562 nodes)
  c2_64   64^3 periodic, interface z = 32, 2 capsules of the c2 kind
  c3      256^3 periodic, B droplet R = 60 in A, 64 capsules R = 6 on a shell
  c3_64   64^3 copy: droplet R = 15, shell 21, capsules R = 6 as many as fit
  c4      192x96x96 channel, walls y = 0 / 95 at -+0.01, interface z = 48
  c4_mini 48x24x24 channel, walls y = 0 / 23, one R = 4 (162-node) capsule
  c5      512^3 periodic, 512 capsules of 162 / 642 / 2562 nodes (R 4 / 6 / 10)
  pressed 37x30x33, four R = 4 capsules pressed together in pairs (one pair
          across the periodic x boundary), particle-particle repulsion on
  bent    38x34x36, two capsules with Helfrich bending (one an ellipsoid) and
          an ellipsoid without it across the periodic x boundary
  onsite_mini  40x20x24 channel with on-site velocity boundaries on the rows
          y = 0 / 19 moving at -+0.01, interface z = 12, one R = 4 capsule
  shear   48^3 capsule in shear (Sec. III.A): on-site boundaries y = 0 / 47
          moving so that the shear rate is 1e-4, A and B both 0.5
          everywhere, G = 0, one R0 = 7.64 (2562-node) capsule, C = 1, kS
          from the capillary number Ca = rho nu rate R0 / kS
"""

from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SNAP = 2.0 ** -20

# initial bulk densities of the layered configurations (majority, minority)
RHO_MAJ = np.float32(0.7)
RHO_MIN = np.float32(0.04)


def _snap(a: np.ndarray) -> np.ndarray:
    return np.round(np.asarray(a, dtype=np.float64) / SNAP) * SNAP


def icosahedron():
    """Vertices (0,+-1,+-phi) and cyclic permutations; faces found as vertex
    triples with all three pairwise distances equal to the edge length 2,
    oriented counter-clockwise seen from outside."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            v.append((0.0, s1, s2 * p))
            v.append((s1, s2 * p, 0.0))
            v.append((s2 * p, 0.0, s1))
    v = np.array(v, dtype=np.float64)
    faces = []
    n = len(v)
    for a in range(n):
        for b in range(a + 1, n):
            if abs(np.linalg.norm(v[a] - v[b]) - 2.0) > 1e-9:
                continue
            for c in range(b + 1, n):
                if (abs(np.linalg.norm(v[a] - v[c]) - 2.0) < 1e-9
                        and abs(np.linalg.norm(v[b] - v[c]) - 2.0) < 1e-9):
                    nrm = np.cross(v[b] - v[a], v[c] - v[a])
                    if np.dot(nrm, v[a] + v[b] + v[c]) > 0:
                        faces.append((a, b, c))
                    else:
                        faces.append((a, c, b))
    faces = np.array(faces, dtype=np.int64)
    assert v.shape == (12, 3) and faces.shape == (20, 3)
    return v, faces


@functools.lru_cache(maxsize=None)
def _unit_icosphere(freq: int):
    return _icosphere_build(freq)


def icosphere(freq: int, radius: float):
    """Geodesic icosphere of frequency freq (a power of two) and given
    radius, centred at the origin.  Returns (xyz float64 [N,3] snapped to the
    2^-20 grid, tri int32 [F,3] outward counter-clockwise)."""
    if freq < 1 or (freq & (freq - 1)) != 0:
        raise ValueError("frequency must be a power of two")
    unit, tri = _unit_icosphere(freq)
    return _snap(unit * float(radius)), tri.copy()


def _icosphere_build(freq: int):
    v, f = icosahedron()
    v = v / np.linalg.norm(v, axis=1, keepdims=True)
    verts = [tuple(x) for x in v]
    faces = [tuple(x) for x in f]
    level = 1
    while level < freq:
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = (np.array(verts[a]) + np.array(verts[b])) * 0.5
                m = m / np.linalg.norm(m)
                verts.append(tuple(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for (a, b, c) in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
        level *= 2
    xyz = np.array(verts, dtype=np.float64)
    tri = np.array(faces, dtype=np.int32)
    assert xyz.shape[0] == 10 * freq * freq + 2
    assert tri.shape[0] == 20 * freq * freq
    return xyz, tri


# Volume-penalty modulus of the workloads.  The paper uses 20 with inertial
# boundary nodes and bounce-back coupling (Sec. III.B); with massless
# immersed-boundary nodes 20, 10 and 5 diverge within 100 steps of the 32^3
# one-capsule case in FP64, and 2 is the largest of {20, 10, 5, 2, 1} that
# stays stable for 1000 steps.
KV_DEFAULT = 2.0

# Strength of the virtual-density (wettability) term relative to the colour
# law as written, rho_v = 2 cos(theta) (rho_maj - rho_min).  At full strength
# the smeared membrane offset, with psi = rho and massless nodes, drives a
# steady contact-line circulation of 0.15 lu/step even around a membrane held
# fixed, and capsules of radius >= 8 diverge within 100 steps at 60 degrees;
# at 0.1 every workload's radius and angle range runs stably with currents
# near 0.02 lu/step and capsules still move into their preferred phase.
WET_SCALE = 0.1


@dataclass
class Capsule:
    centre: np.ndarray          # [3] float64 (snapped)
    radius: float
    freq: int
    kS: float
    C: float
    kV: float
    theta_deg: float
    kB: float = 0.0                         # Helfrich bending modulus (0 = none)
    stretch: tuple = (1.0, 1.0, 1.0)        # axis scaling of the rest mesh (ellipsoids)
    v: tuple = (0.0, 0.0, 0.0)              # initial node velocity (bounce-back coupling)
    prescribed: bool = False                # nodes keep v (rigid translation)

    def mesh(self):
        xyz, tri = icosphere(self.freq, self.radius)
        return _snap(xyz * np.asarray(self.stretch, dtype=np.float64)[None, :] + self.centre[None, :]), tri


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    rhoA: np.ndarray            # float32 [nz, ny, nx]
    rhoB: np.ndarray            # float32 [nz, ny, nx]
    capsules: List[Capsule] = field(default_factory=list)
    tau: tuple = (1.0, 1.0)
    G: float = 3.6
    walls: int = 0
    wall_u_lo: tuple = (0.0, 0.0, 0.0)
    wall_u_hi: tuple = (0.0, 0.0, 0.0)
    z_interface: float = 0.0
    steps: int = 1
    rho_maj: float = float(RHO_MAJ)
    rho_min: float = float(RHO_MIN)
    wet_scale: float = WET_SCALE
    rep_eps: float = 0.0        # particle-particle repulsion strength (0 = off)
    rep_d0: float = 1.25        # and its cut-off
    psi_kind: int = 0           # Shan-Chen pseudo-potential: 0 psi = rho, 1 psi = 1 - exp(-rho)
    coupling: int = 0           # 0 immersed boundary, 1 the paper's bounce-back coupling
    node_mass: float = 5.0      # boundary-node mass of the bounce-back coupling (Sec. III)
    mass_c0: float = 2500.0     # strength C0 of its adaptive mass correction (Sec. II.E)
    note: str = ""

    @property
    def n_lattice(self) -> int:
        return self.nx * self.ny * self.nz

    def meshes(self):
        """Concatenated meshes: (nodes_per_cap, faces_per_cap, xyz [sum N,3]
        float64, tri [sum F,3] int32 with capsule-local indices)."""
        npc, fpc, xs, ts = [], [], [], []
        for c in self.capsules:
            xyz, tri = c.mesh()
            npc.append(xyz.shape[0])
            fpc.append(tri.shape[0])
            xs.append(xyz)
            ts.append(tri)
        if not xs:
            return (np.zeros(0, np.int32), np.zeros(0, np.int32),
                    np.zeros((0, 3)), np.zeros((0, 3), np.int32))
        return (np.array(npc, np.int32), np.array(fpc, np.int32),
                np.concatenate(xs, 0), np.concatenate(ts, 0))

    def cap_params(self):
        a = lambda k: np.array([getattr(c, k) for c in self.capsules], np.float64)
        return a("kS"), a("C"), a("kV"), a("theta_deg")




def layered(nx, ny, nz, z_split, rho=(RHO_MAJ, RHO_MIN)):
    """Component A at majority density rho[0] for z < z_split, minority
    rho[1] above; B the opposite.  Returned float32 [nz, ny, nx]."""
    maj, mn = np.float32(rho[0]), np.float32(rho[1])
    z = np.arange(nz)[:, None, None]
    lower = np.broadcast_to(z < z_split, (nz, ny, nx))
    rhoA = np.where(lower, maj, mn).astype(np.float32)
    rhoB = np.where(lower, mn, maj).astype(np.float32)
    return np.ascontiguousarray(rhoA), np.ascontiguousarray(rhoB)


def droplet(n, radius, centre):
    """Component B droplet of the given radius in component A."""
    g = np.arange(n, dtype=np.float64)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    inside = ((x - centre[0]) ** 2 + (y - centre[1]) ** 2
              + (z - centre[2]) ** 2) < radius * radius
    rhoB = np.where(inside, RHO_MAJ, RHO_MIN).astype(np.float32)
    rhoA = np.where(inside, RHO_MIN, RHO_MAJ).astype(np.float32)
    return rhoA, rhoB


def _periodic_dist(a, b, box):
    d = np.abs(np.asarray(a) - np.asarray(b))
    box = np.asarray(box, dtype=np.float64)
    d = np.minimum(d, box - d)
    return float(np.sqrt((d * d).sum()))


def _seed_plane(rng, n_caps, radii, box, z_lo, z_hi, max_tries=200000):
    centres = []
    for k in range(n_caps):
        for _ in range(max_tries):
            c = np.array([rng.uniform(0, box[0]), rng.uniform(0, box[1]),
                          rng.uniform(z_lo, z_hi)])
            if all(_periodic_dist(c, o, box) >= radii[k] + radii[j] + 2.0
                   for j, o in enumerate(centres)):
                centres.append(c)
                break
        else:
            raise RuntimeError("could not place capsule %d" % k)
    return centres


def _seed_shell(rng, n_caps, radius_cap, shell_r, centre, box, keep_fitting=False):
    centres = []
    tries = 0
    while len(centres) < n_caps and tries < n_caps * 2000:
        tries += 1
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        c = np.asarray(centre) + shell_r * d
        if all(_periodic_dist(c, o, box) >= 2 * radius_cap + 2.0 for o in centres):
            centres.append(c)
        elif keep_fitting and tries > 50 * n_caps:
            break
    return centres


def make(name: str, kV: Optional[float] = None) -> Workload:
    """Build one named workload (see the module docstring)."""
    kV = KV_DEFAULT if kV is None else kV
    if name == "c1":
        rhoA, rhoB = layered(32, 32, 32, 16)
        cap = Capsule(_snap(np.array([16.0, 16.0, 16.0])), 6.0, 8, 0.01, 0.0, kV, 90.0)
        return Workload("c1", 32, 32, 32, rhoA, rhoB, [cap], z_interface=15.5,
                        steps=1000, note="32^3, one 642-node capsule, FP64 oracle case")
    if name in ("c2", "c2_64"):
        rng = np.random.default_rng(1904 + 1)
        n = 128 if name == "c2" else 64
        ncap = 8 if name == "c2" else 2
        cs = _seed_plane(rng, ncap, [8.0] * ncap, (n, n, n), n / 2 - 4, n / 2 + 4)
        caps = []
        for c in cs:
            kS = rng.uniform(0.002, 0.02)
            th = rng.uniform(60.0, 120.0)
            caps.append(Capsule(_snap(c), 8.0, 16, kS, 0.0, kV, th))
        rhoA, rhoB = layered(n, n, n, n // 2)
        return Workload(name, n, n, n, rhoA, rhoB, caps, z_interface=n / 2 - 0.5,
                        steps=5000 if name == "c2" else 50)
    if name in ("c3", "c3_64"):
        rng = np.random.default_rng(1904 + 2)
        if name == "c3":
            n, rd, shell, ncap = 256, 60.0, 66.0, 64
        else:
            n, rd, shell, ncap = 64, 15.0, 21.0, 64
        ctr = (n / 2, n / 2, n / 2)
        cs = _seed_shell(rng, ncap, 6.0, shell, ctr, (n, n, n), keep_fitting=True)
        caps = [Capsule(_snap(c), 6.0, 8, 0.01, 0.0, kV, rng.uniform(45.0, 135.0))
                for c in cs]
        rhoA, rhoB = droplet(n, rd, ctr)
        return Workload(name, n, n, n, rhoA, rhoB, caps, z_interface=n / 2,
                        steps=10000 if name == "c3" else 50)
    if name in ("c4", "c4_mini"):
        if name == "c4":
            nx, ny, nz, R, f = 192, 96, 96, 10.0, 16
        else:
            nx, ny, nz, R, f = 48, 24, 24, 4.0, 4
        rhoA, rhoB = layered(nx, ny, nz, nz // 2)
        cap = Capsule(_snap(np.array([nx / 2, (ny - 1) / 2.0, nz / 2])), R, f,
                      0.005, 0.0, kV, 75.0)
        return Workload(name, nx, ny, nz, rhoA, rhoB, [cap], walls=1,
                        wall_u_lo=(-0.01, 0.0, 0.0), wall_u_hi=(0.01, 0.0, 0.0),
                        z_interface=nz / 2 - 0.5, steps=2000 if name == "c4" else 200)
    if name == "c5":
        rng = np.random.default_rng(1904 + 4)
        n = 512
        kinds = [(4.0, 4), (6.0, 8), (10.0, 16)]
        radii = [kinds[k % 3][0] for k in range(512)]
        cs = _seed_plane(rng, 512, radii, (n, n, n), n / 2 - 2, n / 2 + 2)
        caps = []
        for k, c in enumerate(cs):
            R, f = kinds[k % 3]
            kS = rng.uniform(0.002, 0.02)
            th = rng.uniform(60.0, 120.0)
            caps.append(Capsule(_snap(c), R, f, kS, 0.0, kV, th))
        rhoA, rhoB = layered(n, n, n, n // 2)
        return Workload("c5", n, n, n, rhoA, rhoB, caps, z_interface=n / 2 - 0.5,
                        steps=300)
    raise KeyError(name)


def onsite_mini(nx=40, ny=20, nz=24, theta=75.0) -> Workload:
    """A small channel between on-site velocity boundaries (walls = 2) on the
    rows y = 0 and y = ny - 1, moving at -+0.01 in x, with the flat
    interface z = nz / 2 meeting them and one R = 4 (162-node) capsule in
    the middle of the channel."""
    rhoA, rhoB = layered(nx, ny, nz, nz // 2)
    cap = Capsule(_snap(np.array([nx / 2, (ny - 1) / 2.0, nz / 2])), 4.0, 4, 0.005, 0.0, KV_DEFAULT, theta)
    return Workload("onsite_mini", nx, ny, nz, rhoA, rhoB, [cap], walls=2,
                    wall_u_lo=(-0.01, 0.0, 0.0), wall_u_hi=(0.01, 0.0, 0.0), z_interface=nz / 2 - 0.5,
                    steps=100)


def shear(Ca, n=48, R0=7.64, rate=1e-4, C=1.0, freq=16, tau=1.0) -> Workload:
    """A capsule in simple shear between on-site velocity boundaries (Sec.
    III.A): an n^3 box whose rows y = 0 and y = n - 1 move at -+rate (n - 1) / 2
    in x, both components at 0.5 everywhere with G = 0 (one fluid of density
    1), one capsule of radius R0 in the centre with the Skalak parameter C and
    kS = rho nu rate R0 / Ca (nu = (tau - 1/2) / 3, rho = 1)."""
    nu = (tau - 0.5) / 3.0
    kS = 1.0 * nu * rate * R0 / Ca
    rho = np.full((n, n, n), 0.5, np.float32)
    u = rate * (n - 1) / 2.0
    cap = Capsule(_snap(np.array([n / 2, (n - 1) / 2.0, n / 2])), R0, freq, kS, C, KV_DEFAULT, 90.0)
    return Workload("shear", n, n, n, rho, rho.copy(), [cap], tau=(tau, tau), G=0.0, walls=2,
                    wall_u_lo=(-u, 0.0, 0.0), wall_u_hi=(u, 0.0, 0.0), z_interface=n / 2 - 0.5,
                    steps=100000)


def bent(nx=38, ny=34, nz=36, kB=0.02, freq=4, walls=0) -> Workload:
    """Capsules with Helfrich bending on a flat interface: an ellipsoid
    (rest mesh stretched 1.35 / 1.0 / 0.75 from R = 5), a sphere (R = 4) and
    a second ellipsoid across the periodic x boundary without bending.  The
    rest shape is the stretched one, so the Skalak force starts at zero and
    the bending force (zero spontaneous curvature) drives the ellipsoids."""
    zs = nz // 2
    rhoA, rhoB = layered(nx, ny, nz, zs)
    caps = [Capsule(_snap(np.array([11.3, 10.2, zs - 0.3])), 5.0, freq, 0.01, 0.0, KV_DEFAULT, 75.0,
                    kB=kB, stretch=(1.35, 1.0, 0.75)),
            Capsule(_snap(np.array([25.6, 23.4, zs - 0.6])), 4.0, freq, 0.008, 0.0, KV_DEFAULT, 105.0, kB=kB),
            Capsule(_snap(np.array([1.4, 24.1, zs + 0.2])), 4.0, freq, 0.01, 0.0, KV_DEFAULT, 95.0,
                    stretch=(0.8, 1.2, 1.0))]
    return Workload("bent", nx, ny, nz, rhoA, rhoB, caps, walls=walls,
                    wall_u_lo=(-0.01, 0, 0) if walls else (0, 0, 0),
                    wall_u_hi=(0.01, 0, 0) if walls else (0, 0, 0), z_interface=zs - 0.5, steps=20)


def pressed(nx=37, ny=30, nz=33, radius=4.0, freq=4, gap=0.6, rep_eps=0.5, rep_d0=1.25, walls=0,
            theta=(70.0, 115.0, 100.0, 65.0), kS=0.01, G=3.6, wall_u=0.01) -> Workload:
    """Capsules pressed together for the particle-particle repulsion: one
    pair side by side in x in the middle of the box and one pair facing each
    other across the periodic x boundary, surfaces `gap` apart (< rep_d0), on
    a flat interface.  Odd box edges make the last tiles and bins partial."""
    zs = nz // 2
    rhoA, rhoB = layered(nx, ny, nz, zs)
    h = radius + 0.5 * gap
    yc, zc = ny / 2.0 + 0.3, zs - 0.4
    centres = [(nx / 2.0 - h, yc, zc), (nx / 2.0 + h, yc, zc),
               (h - 0.25, yc - 0.7, zc + 0.2), (nx - h - 0.25, yc - 0.7, zc + 0.2)]
    caps = [Capsule(_snap(np.array(c)), radius, freq, kS, 0.0, KV_DEFAULT, theta[k % len(theta)])
            for k, c in enumerate(centres)]
    return Workload("pressed", nx, ny, nz, rhoA, rhoB, caps, G=G, walls=walls,
                    wall_u_lo=(-wall_u, 0, 0) if walls else (0, 0, 0),
                    wall_u_hi=(wall_u, 0, 0) if walls else (0, 0, 0),
                    z_interface=zs - 0.5, steps=20, rep_eps=rep_eps, rep_d0=rep_d0)


def small(nx=40, ny=36, nz=44, ncap=2, freq=4, radius=4.0, theta=(70.0, 115.0),
          kS=(0.01, 0.004), kV=None, seed=7, walls=0, wall_u=0.01, G=3.6,
          tau=(1.0, 1.0), z_split=None, wet_scale=WET_SCALE) -> Workload:
    """A small seeded workload for parity tests: a ragged box (sizes that are
    not multiples of the kernel tile widths), a flat interface and a few
    small capsules near it."""
    kV = KV_DEFAULT if kV is None else kV
    rng = np.random.default_rng(seed)
    zs = nz // 2 if z_split is None else z_split
    rhoA, rhoB = layered(nx, ny, nz, zs)
    box = (nx, ny, nz)
    centres = []
    for k in range(ncap):
        for _ in range(10000):
            lo_y, hi_y = (radius + 4, ny - radius - 5) if walls else (0, ny)
            c = np.array([rng.uniform(0, nx), rng.uniform(lo_y, hi_y),
                          rng.uniform(zs - 2.5, zs + 1.5)])
            if all(_periodic_dist(c, o, box) >= 2 * radius + 2 for o in centres):
                centres.append(c)
                break
    caps = [Capsule(_snap(c), radius, freq, kS[k % len(kS)], 0.0, kV,
                    theta[k % len(theta)]) for k, c in enumerate(centres)]
    return Workload("small", nx, ny, nz, rhoA, rhoB, caps, tau=tau, G=G,
                    walls=walls, wall_u_lo=(-wall_u, 0, 0) if walls else (0, 0, 0),
                    wall_u_hi=(wall_u, 0, 0) if walls else (0, 0, 0),
                    z_interface=zs - 0.5, steps=20, wet_scale=wet_scale)


def crop(wl: Workload, x0: int, y0: int, z0: int, wx: int, wy: int, wz: int, margin: float = 4.0) -> Workload:
    """A box of wl's initial state, [x0, x0 + wx) x [y0, y0 + wy) x
    [z0, z0 + wz) (periodic in x and y), with the capsules that lie wholly
    inside it at least `margin` cells from its faces, in box coordinates.
    A bounded sample of a large workload with its shapes and value mix."""
    xs = (x0 + np.arange(wx)) % wl.nx
    ys = (y0 + np.arange(wy)) % wl.ny
    zs = z0 + np.arange(wz)
    if zs[0] < 0 or zs[-1] >= wl.nz:
        raise ValueError("crop leaves the box in z")
    sel = np.ix_(zs, ys, xs)
    caps = []
    n = np.array([wl.nx, wl.ny], np.float64)
    for c in wl.capsules:
        rel = np.asarray(c.centre, np.float64) - np.array([x0, y0, z0], np.float64)
        rel[:2] = np.mod(rel[:2], n)
        lo = c.radius + margin
        if (lo <= rel[0] <= wx - 1 - lo and lo <= rel[1] <= wy - 1 - lo and lo <= rel[2] <= wz - 1 - lo):
            caps.append(Capsule(_snap(rel), c.radius, c.freq, c.kS, c.C, c.kV, c.theta_deg, kB=c.kB,
                                stretch=c.stretch))
    return Workload(wl.name + "_crop", wx, wy, wz, np.ascontiguousarray(wl.rhoA[sel]),
                    np.ascontiguousarray(wl.rhoB[sel]), caps, tau=wl.tau, G=wl.G,
                    z_interface=wl.z_interface - z0, rho_maj=wl.rho_maj, rho_min=wl.rho_min,
                    wet_scale=wl.wet_scale, rep_eps=wl.rep_eps, rep_d0=wl.rep_d0, psi_kind=wl.psi_kind)


def bb_capsule(nx=24, ny=22, nz=26, centre=(11.37, 10.61, 12.83), radius=4.0, freq=4, theta=90.0, kS=0.01,
               kV=2.0, v=(0.0, 0.0, 0.0), prescribed=False, interior=None, layered_z=None, G=3.6,
               rho=(0.7, 0.04), interior_mask=None, wet_scale=1.0, C0=2500.0, node_mass=5.0,
               tau=(1.0, 1.0), psi_kind=0) -> Workload:
    """One capsule for the bounce-back coupling (Sec. II.C-II.E) in a
    ragged periodic box, at a centre off the lattice's symmetry planes so
    that no lattice node lies on the membrane.  Densities: uniform `rho`
    (A, B) everywhere, or a flat interface at layered_z (A below, at the
    majority and minority densities rho[0], rho[1]); interior
    = (A, B) densities of the nodes inside the rest sphere shrunk by 0.3, or
    of the nodes where interior_mask [nz, ny, nx] is true, when given (the
    paper fills a capsule with the lower fluid's composition).  The
    capsule's velocity v, and whether it is prescribed, are inputs."""
    if layered_z is not None:
        rhoA, rhoB = layered(nx, ny, nz, layered_z, rho)
    else:
        rhoA = np.full((nz, ny, nx), rho[0], np.float32)
        rhoB = np.full((nz, ny, nx), rho[1], np.float32)
    c = _snap(np.array(centre, np.float64))
    if interior is not None:
        if interior_mask is not None:
            ins = np.asarray(interior_mask, bool)
        else:
            g = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
            ins = (g[2] - c[0]) ** 2 + (g[1] - c[1]) ** 2 + (g[0] - c[2]) ** 2 < (radius - 0.3) ** 2
        rhoA = np.where(ins, np.float32(interior[0]), rhoA).astype(np.float32)
        rhoB = np.where(ins, np.float32(interior[1]), rhoB).astype(np.float32)
    cap = Capsule(c, radius, freq, kS, 0.0, kV, theta, v=tuple(float(a) for a in v), prescribed=prescribed)
    zi = (layered_z - 0.5) if layered_z is not None else nz / 2
    return Workload("bb_capsule", nx, ny, nz, np.ascontiguousarray(rhoA), np.ascontiguousarray(rhoB), [cap],
                    tau=tau, G=G, z_interface=zi, wet_scale=wet_scale, coupling=1, node_mass=node_mass,
                    mass_c0=C0, psi_kind=psi_kind, rho_maj=float(np.float32(rho[0])),
                    rho_min=float(np.float32(rho[1])))


def bounce_back(wl: Workload, C0: float = 2500.0, node_mass: float = 5.0) -> Workload:
    """The same lattice, densities and capsules under the paper's bounce-back
    coupling (Sec. II.C-II.E): inertial nodes of mass `node_mass` (Sec. III),
    the adaptive mass correction of strength C0, and the colour offset at
    the full strength of the contact-angle law (wet_scale 1)."""
    import dataclasses
    return dataclasses.replace(wl, name=wl.name + "_bb", coupling=1, wet_scale=1.0, node_mass=node_mass,
                               mass_c0=C0)


def bb_pair(nx=32, ny=22, nz=26, centres=((9.37, 10.61, 12.83), (19.93, 11.29, 13.41)), radius=4.0, freq=4,
            thetas=(60.0, 120.0), kS=0.01, kV=2.0, vs=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)), prescribed=False,
            layered_z=13, C0=2500.0, node_mass=5.0) -> Workload:
    """Two capsules for the bounce-back coupling on a flat interface
    (A below layered_z), close enough that the lattice boxes in which their
    labels are found overlap; velocities and whether they are prescribed are
    inputs."""
    rhoA, rhoB = layered(nx, ny, nz, layered_z)
    caps = [Capsule(_snap(np.array(c, np.float64)), radius, freq, kS, 0.0, kV, th, v=tuple(float(a) for a in v),
                    prescribed=prescribed) for c, th, v in zip(centres, thetas, vs)]
    return Workload("bb_pair", nx, ny, nz, rhoA, rhoB, caps, G=3.6, z_interface=layered_z - 0.5, wet_scale=1.0,
                    coupling=1, node_mass=node_mass, mass_c0=C0)
