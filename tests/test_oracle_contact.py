"""Pins of the oracle's particle-particle repulsion (Sec. III.E): a pair of
boundary nodes of different particles at separation d < d0 repels along the
separation with eps (d0 - d)^{3/2}."""

import math

import numpy as np
import torch

from oracle import contact

DT = torch.float64
DIMS = (32, 24, 28)


def test_single_pair_closed_form():
    """One node per particle at separation d along a general direction: the
    force on each is eps (d0 - d)^{3/2} along its own side of the line."""
    eps, d0 = 0.5, 1.25
    n = torch.tensor([2.0, -1.0, 2.0], dtype=DT) / 3.0
    for d in (0.1, 0.6, 1.0, 1.2):
        Xa = torch.tensor([[10.0, 11.0, 12.0]], dtype=DT)
        Xb = Xa + d * n
        Fa, Fb = contact.repulsion_forces([Xa, Xb], DIMS, eps, d0)
        mag = eps * (d0 - d) ** 1.5
        assert torch.allclose(Fa[0], -mag * n, rtol=1e-12, atol=0)
        assert torch.allclose(Fb[0], mag * n, rtol=1e-12, atol=0)


def test_cutoff_and_no_self_interaction():
    eps, d0 = 0.5, 1.25
    Xa = torch.tensor([[5.0, 5.0, 5.0], [5.3, 5.0, 5.0]], dtype=DT)      # 0.3 apart, one particle
    Xb = torch.tensor([[5.0, 5.0 + d0, 5.0], [9.0, 9.0, 9.0]], dtype=DT)  # exactly d0 and far
    Fa, Fb = contact.repulsion_forces([Xa, Xb], DIMS, eps, d0)
    assert float(Fa[0].abs().max()) == 0.0
    assert float(Fb.abs().max()) == 0.0 and float(Fa.abs().max()) == 0.0
    (F1,) = contact.repulsion_forces([Xa], DIMS, eps, d0)
    assert float(F1.abs().max()) == 0.0


def _clouds(seed, n=3, m=40, spread=1.6):
    g = torch.Generator().manual_seed(seed)
    base = torch.tensor([15.0, 12.0, 14.0], dtype=DT)
    return [base + spread * torch.rand(m, 3, generator=g, dtype=DT) for _ in range(n)]


def test_newton_third_law_and_zero_torque():
    Xs = _clouds(3)
    F = contact.repulsion_forces(Xs, DIMS, 0.5, 1.25)
    tot = sum(f.sum(0) for f in F)
    torque = sum(torch.cross(X, f, dim=1).sum(0) for X, f in zip(Xs, F))
    scale = max(float(f.abs().max()) for f in F)
    assert scale > 1e-3                                  # the clouds do interact
    assert float(tot.abs().max()) <= 1e-13 * scale * 40
    assert float(torque.abs().max()) <= 1e-12 * scale * 40 * 20


def test_periodic_image_and_period_shift():
    """A pair straddling the x boundary interacts through the nearest image,
    and shifting one particle by a lattice period changes nothing."""
    eps, d0 = 0.5, 1.25
    Xa = torch.tensor([[0.2, 7.0, 7.0]], dtype=DT)
    Xb = torch.tensor([[DIMS[0] - 0.5, 7.0, 7.0]], dtype=DT)           # 0.7 apart through x = 0
    Fa, Fb = contact.repulsion_forces([Xa, Xb], DIMS, eps, d0)
    mag = eps * (d0 - 0.7) ** 1.5
    assert torch.allclose(Fa[0], torch.tensor([mag, 0.0, 0.0], dtype=DT), rtol=1e-12, atol=1e-15)
    Xs = _clouds(5)
    F0 = contact.repulsion_forces(Xs, DIMS, 0.5, 1.25)
    shifted = [Xs[0] + torch.tensor([DIMS[0], 0.0, -DIMS[2]], dtype=DT)] + Xs[1:]
    F1 = contact.repulsion_forces(shifted, DIMS, 0.5, 1.25)
    scale = max(float(f.abs().max()) for f in F0)
    for a, b in zip(F0, F1):
        # the shift only changes the rounding of the positions
        assert float((a - b).abs().max()) <= 1e-12 * scale
    # with walls, y is not periodic: the same pair across y = 0 does not interact
    Ya = torch.tensor([[7.0, 0.2, 7.0]], dtype=DT)
    Yb = torch.tensor([[7.0, DIMS[1] - 0.5, 7.0]], dtype=DT)
    assert float(contact.repulsion_forces([Ya, Yb], DIMS, eps, d0, walls=1)[0].abs().max()) == 0.0
    assert float(contact.repulsion_forces([Ya, Yb], DIMS, eps, d0, walls=0)[0].abs().max()) > 0.0


def test_force_is_minus_gradient_of_pair_energy():
    Xs = [X.clone().requires_grad_(True) for X in _clouds(7)]
    E = contact.repulsion_energy(Xs, DIMS, 0.5, 1.25)
    g = torch.autograd.grad(E, Xs)
    F = contact.repulsion_forces([X.detach() for X in Xs], DIMS, 0.5, 1.25)
    for f, gk in zip(F, g):
        assert torch.allclose(f, -gk, rtol=1e-10, atol=1e-13)


def test_matches_plain_double_loop():
    """A pure-Python loop over node pairs, written from the formula, on small
    random clouds (including pairs through the periodic boundary)."""
    eps, d0 = 0.5, 1.25
    rng = np.random.default_rng(11)
    Xs = [torch.tensor(np.mod(rng.uniform(-1.0, 2.5, (12, 3)) + c, DIMS), dtype=DT)
          for c in ([0.5, 0.5, 0.5], [1.0, 0.2, 27.4], [31.2, 1.0, 0.9])]
    F = contact.repulsion_forces(Xs, DIMS, eps, d0)
    ref = [np.zeros((12, 3)) for _ in Xs]
    for k in range(3):
        for a in range(12):
            for l in range(3):
                if l == k:
                    continue
                for b in range(12):
                    v = [float(Xs[k][a, q] - Xs[l][b, q]) for q in range(3)]
                    v = [x - DIMS[q] * round(x / DIMS[q]) for q, x in enumerate(v)]
                    r = math.sqrt(sum(x * x for x in v))
                    if r < d0:
                        m = eps * (d0 - r) ** 1.5 / r
                        ref[k][a] += [m * x for x in v]
    assert max(float(np.abs(ref[k]).max()) for k in range(3)) > 1e-3
    for k in range(3):
        assert np.allclose(F[k].numpy(), ref[k], rtol=1e-12, atol=1e-14)


def test_whole_step_momentum_with_repulsion():
    """The repulsion acts inside the membrane (equal and opposite pair forces),
    so with it on the fluid's mass and momentum stay conserved through the
    coupled step; and it does act on the pressed capsules."""
    from oracle.sim import from_workload
    from paper_1904_11386_amd import workloads as W
    wl = W.pressed()
    s = from_workload(wl)
    m0, p0 = s.mass().clone(), s.momentum().clone()
    s.run(20)
    assert torch.allclose(s.mass(), m0, rtol=1e-13, atol=0)
    assert float((s.momentum() - p0).abs().max()) < 1e-15 * float(m0.sum())
    R = contact.repulsion_forces(s.X, s.dims, wl.rep_eps, wl.rep_d0)
    assert all(float(r.abs().max()) > 1e-3 for r in R)      # every capsule is pressed
    s_off = from_workload(wl, rep_eps=0.0)
    s_off.step()
    s1 = from_workload(wl)
    s1.step()
    dF = [a - b for a, b in zip(s1.Fb_last, s_off.Fb_last)]
    R0 = contact.repulsion_forces(from_workload(wl).X, s.dims, wl.rep_eps, wl.rep_d0)
    for a, b in zip(dF, R0):
        assert torch.allclose(a, b, rtol=1e-12, atol=1e-15)
