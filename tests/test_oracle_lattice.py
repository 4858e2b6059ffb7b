"""Pins of the FP64 oracle's fluid part against what the paper and the
mathematics fix (no GPU)."""

import math

import numpy as np
import pytest
import torch

from oracle import lattice as L
from oracle.sim import OracleSim

DT = torch.float64


def test_weights_and_velocity_set_match_paper(golden):
    w = golden["d3q19_weights"]["value"]
    cnt = golden["d3q19_counts"]["value"]
    norms = (L.C * L.C).sum(1)
    assert int((norms == 0).sum()) == cnt["rest"]
    assert int((norms == 1).sum()) == cnt["axis"]
    assert int((norms == 2).sum()) == cnt["diagonal"]
    for i in range(19):
        exp = {0: w["rest"], 1: w["axis"], 2: w["diagonal"]}[int(norms[i])]
        assert float(L.W[i]) == pytest.approx(exp, abs=1e-16)
    # opposite pairs
    for i in range(19):
        assert torch.equal(L.C[L.OPP[i]], -L.C[i])
    assert L.CS2 == pytest.approx(golden["cs2"]["value"], abs=0)
    # isotropy: sum w = 1, sum w c = 0, sum w c c = cs2 I, sum w c c c c = cs2^2 (dd + ..)
    assert float(L.W.sum()) == pytest.approx(1.0, abs=1e-15)
    cw = (L.W.unsqueeze(1) * L.CF).sum(0)
    assert torch.allclose(cw, torch.zeros(3, dtype=DT), atol=1e-16)
    ccw = torch.einsum("i,ia,ib->ab", L.W, L.CF, L.CF)
    assert torch.allclose(ccw, L.CS2 * torch.eye(3, dtype=DT), atol=1e-16)
    c4 = torch.einsum("i,ia,ib,ic,id->abcd", L.W, L.CF, L.CF, L.CF, L.CF)
    I = torch.eye(3, dtype=DT)
    iso = (torch.einsum("ab,cd->abcd", I, I) + torch.einsum("ac,bd->abcd", I, I)
           + torch.einsum("ad,bc->abcd", I, I)) * L.CS2 ** 2
    assert torch.allclose(c4, iso, atol=1e-16)


def test_equilibrium_moments_exact():
    g = torch.Generator().manual_seed(3)
    rho = 0.05 + torch.rand(4, 3, 5, generator=g, dtype=DT)
    u = 0.05 * (torch.rand(3, 4, 3, 5, generator=g, dtype=DT) - 0.5)
    feq = L.equilibrium(rho, u)
    m0 = feq.sum(0)
    m1 = torch.einsum("id,izyx->dzyx", L.CF, feq)
    m2 = torch.einsum("ia,ib,izyx->abzyx", L.CF, L.CF, feq)
    assert torch.allclose(m0, rho, rtol=1e-14, atol=0)
    assert torch.allclose(m1, rho * u, rtol=1e-13, atol=1e-17)
    exp2 = rho * (L.CS2 * torch.eye(3, dtype=DT).view(3, 3, 1, 1, 1)) + rho * torch.einsum("azyx,bzyx->abzyx", u, u)
    assert torch.allclose(m2, exp2, rtol=1e-13, atol=1e-17)


def _uniform_sim(n, tau, u_field=None, walls=0, u_lo=(0, 0, 0), u_hi=(0, 0, 0), dims=None):
    nx, ny, nz = dims if dims else (n, n, n)
    rho = torch.full((nz, ny, nx), 0.5, dtype=DT)
    s = OracleSim(rho, rho, [], tau=(tau, tau), G=0.0, walls=walls, u_lo=u_lo, u_hi=u_hi)
    if u_field is not None:
        s.fpost = torch.stack([L.equilibrium(rho, u_field)] * 2, 0)
    return s


def test_shear_wave_decay_matches_viscosity(golden):
    """u_x = u0 sin(k z) decays as exp(-nu k^2 t), nu = cs2 (tau - 1/2)
    (Sec. II.A), up to the O(k^2) lattice error."""
    nz = 32
    for tau in (0.8, 1.0):
        z = torch.arange(nz, dtype=DT)
        k = 2 * math.pi / nz
        u = torch.zeros(3, nz, 2, 2, dtype=DT)
        u[0] = (1e-4 * torch.sin(k * z)).view(nz, 1, 1)
        s = _uniform_sim(0, tau, u, dims=(2, 2, nz))
        T = 300
        s.run(T)
        amp = float((s.u_last[0, :, 0, 0] * torch.sin(k * z)).sum() * 2 / nz)
        nu = L.CS2 * (tau - 0.5)
        # the measured field is u^{T-1}, the velocity of the last collision
        exp = 1e-4 * math.exp(-nu * k * k * (T - 1))
        assert amp == pytest.approx(exp, rel=0.02), (tau, amp, exp)


def test_couette_half_way_bounce_back_exact():
    """Moving half-way bounce-back walls (Sec. II.C, eq. method:SBB) at
    y = 1/2 and y = ny - 3/2 give the exact linear Couette profile."""
    ny = 14
    s = _uniform_sim(0, 1.2, walls=1, u_lo=(-0.01, 0, 0), u_hi=(0.01, 0, 0), dims=(2, ny, 2))
    s.run(3000)
    y = torch.arange(1, ny - 1, dtype=DT)
    H = ny - 2
    exp = -0.01 + 0.02 * (y - 0.5) / H
    got = s.u_last[0, 0, 1:ny - 1, 0]
    assert torch.allclose(got, exp, atol=1e-9), (got - exp).abs().max()
    assert float(s.u_last[1:, :, 1:ny - 1].abs().max()) < 1e-15
    # mass conserved exactly in the fluid rows
    m0 = 0.5 * H * 4
    assert float(s.mass()[0]) == pytest.approx(m0, rel=1e-13)


def test_shan_chen_force_sums_to_zero_periodic():
    g = torch.Generator().manual_seed(5)
    ra = 0.04 + 0.7 * torch.rand(6, 7, 5, generator=g, dtype=DT)
    rb = 0.04 + 0.7 * torch.rand(6, 7, 5, generator=g, dtype=DT)
    Fa = L.shan_chen_force(ra, L.sc_sum(rb), 3.6)
    Fb = L.shan_chen_force(rb, L.sc_sum(ra), 3.6)
    tot = (Fa + Fb).sum((1, 2, 3))
    scale = float(Fa.abs().sum())
    assert float(tot.abs().max()) < 1e-14 * scale
    assert float(Fa.sum((1, 2, 3)).abs().max()) > 1e-6 * scale   # not trivially zero per component
    # the neighbour sum of a linear ramp is cs2 times its gradient (interior)
    x = torch.arange(5, dtype=DT).view(1, 1, 5).expand(6, 7, 5)
    S = L.sc_sum(0.3 * x)
    assert torch.allclose(S[0][:, :, 1:4], torch.full((6, 7, 3), 0.3 * L.CS2, dtype=DT), atol=1e-15)


def _layered(nx, ny, nz, zs=None):
    zs = nz // 2 if zs is None else zs
    z = torch.arange(nz).view(nz, 1, 1).expand(nz, ny, nx)
    ra = torch.where(z < zs, 0.7, 0.04).to(DT)
    rb = torch.where(z < zs, 0.04, 0.7).to(DT)
    return ra, rb


def test_flat_interface_stays_flat_and_symmetric():
    ra, rb = _layered(6, 5, 16)
    s = OracleSim(ra, rb, [], G=3.6)
    s.run(150)
    rho = s.rho_last
    # x-y invariance is exact for a layered state
    for c in (0, 1):
        ref = rho[c][:, :1, :1]
        assert float((rho[c] - ref).abs().max()) < 1e-15
    assert float(s.u_last[:2].abs().max()) < 1e-17
    # A<->B swap with the mirror z -> 15 - z (about the mid-plane 7.5) and
    # the periodic partner interface is a symmetry of the set-up
    za = rho[0][:, 0, 0]
    zb = rho[1][:, 0, 0]
    assert torch.allclose(za, zb.flip(0), atol=1e-14)
    # mass per component exact
    assert float(s.mass()[0]) == pytest.approx(float(ra.sum()), rel=1e-14)


def _coexistence(G, tot):
    # mean-field bulk densities a, b with a + b = tot and ln(a/b) = G (a - b)
    lo, hi = tot / 2 + 1e-9, tot - 1e-12
    for _ in range(200):
        a = 0.5 * (lo + hi)
        f = math.log(a / (tot - a)) - G * (2 * a - tot)
        if f > 0:
            hi = a
        else:
            lo = a
    return a, tot - a


@pytest.mark.slow
def test_phase_separation_sign_and_static_interface_velocity():
    """Repulsive G > 0 keeps the components separated (a wrong sign mixes
    them toward 0.37 / 0.37); at rest the velocity with the half-force term
    vanishes although the force does not (Sec. II.A, II.D).  The bulk values
    do not follow the continuum mean-field law ln(a/b) = G (a - b): with the
    velocity-shift forcing the interface carries O(F^2 / rho) momentum flux,
    so the measured steady state (A 0.7647, B 0.0041 at G = 3.6) is recorded
    rather than compared with mean field."""
    ra, rb = _layered(1, 1, 48)
    s = OracleSim(ra, rb, [], G=3.6)
    s.run(4000)
    rho = s.rho_last
    a_bulk = float(rho[0][10, 0, 0])
    b_bulk = float(rho[1][10, 0, 0])
    assert a_bulk > 0.6 and b_bulk < 0.1
    # the minority phase is depleted further than the mean-field estimate
    a_mf, b_mf = _coexistence(3.6, a_bulk + b_bulk)
    assert b_bulk < b_mf
    Fmax = float(s.F_last.abs().max())
    assert Fmax > 1e-3
    assert float(s.u_last.abs().max()) < 1e-4 * Fmax


def test_exponential_pseudo_potential_closed_forms():
    """psi = 1 - exp(-rho) (Sec. II.D): psi(0) = 0, slope 1 at 0, saturation at
    1, and psi(-ln(1 - a)) = a."""
    from oracle.lattice import pseudo_potential
    r = torch.tensor([0.0, 1e-8, 0.7, 0.042, 50.0], dtype=torch.float64)
    p = pseudo_potential(r, 1)
    assert float(p[0]) == 0.0 and abs(float(p[1]) / 1e-8 - 1.0) < 1e-7
    assert abs(float(p[4]) - 1.0) < 1e-15
    a = torch.tensor([0.1, 0.5, 0.9], dtype=torch.float64)
    assert torch.allclose(pseudo_potential(-torch.log1p(-a), 1), a, rtol=1e-14)
    assert torch.equal(pseudo_potential(r, 0), r)


def test_shan_chen_force_on_a_linear_pseudo_potential():
    """With rho^B chosen so that psi^B = alpha + beta x exactly, the D3Q19
    neighbour sum is beta sum_i w_i c_ix c_i = (beta / 3, 0, 0) at every node
    away from the periodic seam, so F^A = -psi^A G beta / 3 along x."""
    from oracle.lattice import pseudo_potential, sc_sum, shan_chen_force
    nx, ny, nz, alpha, beta, G = 16, 4, 5, 0.05, 0.03, 3.6
    x = torch.arange(nx, dtype=torch.float64).view(1, 1, nx).expand(nz, ny, nx)
    rhoB = -torch.log1p(-(alpha + beta * x))
    rhoA = 0.4 + 0.02 * torch.arange(nz, dtype=torch.float64).view(nz, 1, 1).expand(nz, ny, nx)
    S = sc_sum(pseudo_potential(rhoB, 1))
    inner = slice(1, nx - 1)
    assert torch.allclose(S[0, :, :, inner], torch.full_like(S[0, :, :, inner], beta / 3.0), rtol=1e-13, atol=0)
    assert float(S[1:, :, :, inner].abs().max()) < 1e-16
    F = shan_chen_force(pseudo_potential(rhoA, 1), S, G)
    ref = -G * (1.0 - torch.exp(-rhoA[:, :, inner])) * beta / 3.0
    assert torch.allclose(F[0, :, :, inner], ref, rtol=1e-13, atol=0)


def test_unequal_tau_collision_momentum_change_equals_force():
    """Force as a shift of the equilibrium velocity with two relaxation
    times (Sec. II.A; Sec. II.D, eq. method:shanchen): the collision keeps
    each component's mass, and the momentum it adds, summed over the
    components, is exactly the summed force sum_c F^c, for any tau_c.  The
    common velocity u' must be the tau-weighted one and the shift of each
    component must carry its own tau_c for this to hold: with tau_c left out
    of the shift the change is sum_c F^c / tau_c, and with an unweighted u'
    an extra sum_c (rho^c u' - j^c) / tau_c appears."""
    g = torch.Generator().manual_seed(11)
    shp = (2, 19, 3, 4, 5)
    f = 0.002 + 0.05 * torch.rand(shp, generator=g, dtype=DT)
    rho, j = L.moments(f)
    F = 1e-3 * (torch.rand(2, 3, 3, 4, 5, generator=g, dtype=DT) - 0.5)
    for tau in ((0.7, 1.3), (0.8, 1.3), (1.3, 0.55)):
        fs = L.collide(f, rho, j, F, tau)
        assert torch.allclose(fs.sum(1), rho, rtol=1e-14, atol=0)
        dp = torch.einsum("id,cizyx->dzyx", L.CF, fs - f)
        ref = F[0] + F[1]
        err = float((dp - ref).abs().max())
        # rounding acts on the momenta themselves (|j| ~ 0.1 here, |F| ~ 5e-4)
        scale = float(j.abs().max()) + float(ref.abs().max())
        assert err < 1e-14 * scale, (tau, err)
        # each component alone does not receive its own force: the shares
        # are exchanged through u' when the densities differ
        dpa = torch.einsum("id,izyx->dzyx", L.CF, fs[0] - f[0])
        assert float((dpa - F[0]).abs().max()) > 1e-6


def test_unequal_tau_without_force_conserves_total_momentum():
    """With G = 0 and no capsules the two components exchange momentum only
    through the common velocity u' of Sec. II.A, so with tau_A != tau_B the
    total momentum of a periodic box is conserved exactly (to rounding) only
    when u' is the tau-weighted mean sum_c (j^c / tau_c) / sum_c (rho^c / tau_c);
    each component's own momentum does change."""
    g = torch.Generator().manual_seed(12)
    nz, ny, nx = 5, 4, 6
    ra = 0.05 + 0.7 * torch.rand(nz, ny, nx, generator=g, dtype=DT)
    rb = 0.05 + 0.7 * torch.rand(nz, ny, nx, generator=g, dtype=DT)
    ua = 0.02 * (torch.rand(3, nz, ny, nx, generator=g, dtype=DT) - 0.5)
    ub = 0.02 * (torch.rand(3, nz, ny, nx, generator=g, dtype=DT) - 0.5)
    s = OracleSim(ra, rb, [], tau=(0.7, 1.3), G=0.0)
    s.fpost = torch.stack([L.equilibrium(ra, ua), L.equilibrium(rb, ub)], 0)
    p0 = s.momentum().clone()
    pa0 = torch.einsum("id,izyx->d", L.CF, s.fpost[0]).clone()
    s.run(30)
    scale = float(s.fpost.sum())
    assert float((s.momentum() - p0).abs().max()) < 1e-15 * scale
    pa = torch.einsum("id,izyx->d", L.CF, s.fpost[0])
    assert float((pa - pa0).abs().max()) > 1e-4 * float(p0.abs().max() + 1e-30) or \
        float((pa - pa0).abs().max()) > 1e-6
