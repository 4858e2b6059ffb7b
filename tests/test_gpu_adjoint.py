"""The hand-written HIP adjoint against the FP64 oracle's reverse-mode
gradient and against central finite differences of the GPU forward."""

import math
import sys

import numpy as np
import pytest
import torch

from oracle import sim as S
from paper_1904_11386_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class OracleChannel:
    def __init__(self, wl, params):
        self.wl, self.params = wl, params

    def __call__(self, th, ks, G):
        wl = self.wl
        caps = []
        for c in wl.capsules:
            xyz, tri = c.mesh()
            caps.append(dict(xyz=xyz, tri=tri, kS=ks, C=c.C, kV=c.kV, theta=th))
        return S.OracleSim(wl.rhoA.astype(np.float64), wl.rhoB.astype(np.float64), caps, tau=wl.tau, G=G,
                           walls=wl.walls, u_lo=wl.wall_u_lo, u_hi=wl.wall_u_hi, rho_maj=wl.rho_maj,
                           rho_min=wl.rho_min, z_interface=wl.z_interface, wet_scale=wl.wet_scale,
                           differentiable=True, rep_eps=wl.rep_eps, rep_d0=wl.rep_d0, psi_kind=wl.psi_kind)


def _gpu_grad(wl, params, steps, every, kind):
    from paper_1904_11386_amd import binding
    from paper_1904_11386_amd.adjoint import OBJECTIVES, workload_with
    nseg = (steps + every - 1) // every
    sim = binding.sim_from_workload(workload_with(wl, *params), n_slots=nseg, ring_len=every)
    J = sim.adjoint_forward(steps, every, OBJECTIVES[kind], 0)
    g = sim.adjoint_backward()
    sim.close()
    return J, g


@pytest.mark.parametrize("kind", ["com_z", "taylor_D"])
def test_adjoint_matches_oracle_gradient_channel(kind):
    wl = W.make("c4_mini")
    params = (75.0, 0.005, 3.6)
    steps, every = 40, 10
    _say("adjoint", kind, "c4_mini", steps, "steps, checkpoint every", every)
    J, g = _gpu_grad(wl, params, steps, every, kind)
    Jo, go = S.gradient(OracleChannel(wl, params), steps, every, kind)
    go = go.numpy()
    rel = np.abs(g - go) / np.abs(go)
    _say("  J gpu %.8e oracle %.8e" % (J, Jo))
    _say("  grad gpu", g.tolist(), "oracle", go.tolist(), "rel", rel.tolist())
    assert abs(J - Jo) < 1e-5 * max(1.0, abs(Jo))
    assert np.all(rel < 1e-4), rel
    # and against FP64 central differences of the oracle forward
    oc = OracleChannel(wl, params)

    def run(p):
        s = oc(*p)
        with torch.no_grad():
            s.run(steps)
            return float(S.objective(s, kind))

    for i, h in enumerate((0.05, 1e-5, 1e-4)):
        pp, pm = list(params), list(params)
        pp[i] += h
        pm[i] -= h
        fd = (run(pp) - run(pm)) / (2 * h)
        if i == 0:
            fd *= 180.0 / math.pi
        _say("  param %d gpu adjoint %.8e fp64 fd %.8e rel %.2e" % (i, g[i], fd, abs(g[i] - fd) / abs(fd)))
        assert abs(g[i] - fd) <= 1e-4 * abs(fd)


def test_adjoint_matches_central_differences_gpu():
    from paper_1904_11386_amd import binding
    from paper_1904_11386_amd.adjoint import workload_with
    wl = W.make("c4_mini")
    params = [75.0, 0.005, 3.6]
    steps, every = 40, 10
    J, g = _gpu_grad(wl, params, steps, every, "com_z")

    def fwd(p):
        s = binding.sim_from_workload(workload_with(wl, *p))
        s.step(steps)
        h = s.observables()["caps"][0]["height"]
        s.close()
        return h

    # steps large enough that the change of J (a capsule height of a few
    # lattice units, resolved to ~1e-7 in FP32 node positions) is ~1e-5 or
    # more, while J stays close to linear over +-h
    for i, h in enumerate((0.5, 5e-4, 1e-3)):
        pp, pm = list(params), list(params)
        pp[i] += h
        pm[i] -= h
        fd = (fwd(pp) - fwd(pm)) / (2 * h)
        if i == 0:
            fd *= 180.0 / math.pi
        _say("  param %d adjoint %.6e fp32 fd %.6e rel %.2e" % (i, g[i], fd, abs(g[i] - fd) / abs(fd)))
        # FP32 forward differences carry ~1e-7 relative noise in J, so the
        # bound is the noise over the step, not the adjoint's accuracy
        assert abs(g[i] - fd) <= 1e-2 * abs(fd)


def test_autograd_function_backward():
    from paper_1904_11386_amd.adjoint import capsule_objective
    wl = W.make("c4_mini")
    th = torch.tensor(75.0, dtype=torch.float64, requires_grad=True)
    ks = torch.tensor(0.005, dtype=torch.float64, requires_grad=True)
    G = torch.tensor(3.6, dtype=torch.float64, requires_grad=True)
    J = capsule_objective(th, ks, G, wl, 20, 10, "com_z")
    J.backward()
    assert th.grad is not None and ks.grad is not None and G.grad is not None
    J2, g = _gpu_grad(wl, (75.0, 0.005, 3.6), 20, 10, "com_z")
    assert float(th.grad) == pytest.approx(g[0] * math.pi / 180.0, rel=1e-6)
    assert float(G.grad) == pytest.approx(g[2], rel=1e-6)


def test_adjoint_with_repulsion_pressed_channel():
    """The adjoint with the particle-particle repulsion on: four capsules
    pressed together in pairs in a walled channel (one pair across the
    periodic x boundary), J = height of capsule 0 after 40 steps.  Against
    the oracle's reverse-mode gradient and FP64 central differences of the
    oracle forward."""
    wl = W.pressed(walls=1)
    params = (75.0, 0.005, 3.6)
    steps, every, kind = 40, 10, "com_z"
    _say("adjoint with repulsion, pressed channel", steps, "steps, checkpoint every", every)
    J, g = _gpu_grad(wl, params, steps, every, kind)
    oc = OracleChannel(wl, params)
    Jo, go = S.gradient(oc, steps, every, kind)
    go = go.numpy()
    rel = np.abs(g - go) / np.abs(go)
    _say("  J gpu %.8e oracle %.8e" % (J, Jo))
    _say("  grad gpu", g.tolist(), "oracle", go.tolist(), "rel", rel.tolist())
    assert abs(J - Jo) < 1e-5 * max(1.0, abs(Jo))
    assert np.all(rel < 1e-4), rel

    def run(p):
        s = oc(*p)
        with torch.no_grad():
            s.run(steps)
            return float(S.objective(s, kind))

    for i, h in enumerate((0.05, 1e-5, 1e-4)):
        pp, pm = list(params), list(params)
        pp[i] += h
        pm[i] -= h
        fd = (run(pp) - run(pm)) / (2 * h)
        if i == 0:
            fd *= 180.0 / math.pi
        _say("  param %d gpu adjoint %.8e fp64 fd %.8e rel %.2e" % (i, g[i], fd, abs(g[i] - fd) / abs(fd)))
        assert abs(g[i] - fd) <= 1e-4 * abs(fd)
    # the repulsion matters here: the gradient without it differs
    import dataclasses
    _, g0 = _gpu_grad(dataclasses.replace(wl, rep_eps=0.0), params, steps, every, kind)
    _say("  grad without repulsion", g0.tolist())
    assert np.abs(g0 - g).max() > 1e-3 * np.abs(g).max()


@pytest.mark.parametrize("kind", ["com_z", "taylor_D"])
def test_adjoint_with_exponential_pseudo_potential(kind):
    """The adjoint with psi = 1 - exp(-rho) on the 48 x 24 x 24 walled channel,
    40 steps: against the oracle's reverse-mode gradient and FP64 central
    differences of the oracle forward."""
    import dataclasses
    wl = dataclasses.replace(W.make("c4_mini"), psi_kind=1)
    params = (75.0, 0.005, 3.6)
    steps, every = 40, 10
    _say("adjoint, psi = 1 - exp(-rho),", kind)
    J, g = _gpu_grad(wl, params, steps, every, kind)
    oc = OracleChannel(wl, params)
    Jo, go = S.gradient(oc, steps, every, kind)
    go = go.numpy()
    rel = np.abs(g - go) / np.abs(go)
    _say("  J gpu %.8e oracle %.8e" % (J, Jo))
    _say("  grad gpu", g.tolist(), "oracle", go.tolist(), "rel", rel.tolist())
    assert abs(J - Jo) < 1e-5 * max(1.0, abs(Jo))
    assert np.all(rel < 1e-4), rel
    if kind == "com_z":
        def run(p):
            s = oc(*p)
            with torch.no_grad():
                s.run(steps)
                return float(S.objective(s, kind))

        for i, h in enumerate((0.05, 1e-5, 1e-4)):
            pp, pm = list(params), list(params)
            pp[i] += h
            pm[i] -= h
            fd = (run(pp) - run(pm)) / (2 * h)
            if i == 0:
                fd *= 180.0 / math.pi
            _say("  param %d gpu adjoint %.8e fp64 fd %.8e rel %.2e" % (i, g[i], fd, abs(g[i] - fd) / abs(fd)))
            assert abs(g[i] - fd) <= 1e-4 * abs(fd)


def test_staged_reverse_sweep_matches_backward_call():
    """The reverse sweep driven from Python one stage at a time
    (lbm_adjoint_seed, then per checkpoint segment lbm_state_load,
    lbm_adjoint_record and lbm_adjoint_step in reverse, then
    lbm_adjoint_grads) gives the gradient of lbm_adjoint_backward, which runs
    the same stages inside the library.  The recomputed forward spreads with
    float atomics, so two sweeps agree to the rounding-order noise of the
    recompute, not bit for bit: the bound is 1e-6 of the gradient's max norm
    (a small component such as dJ/dkS carries relative noise near 1e-6 from
    run to run of the same call), and two runs of lbm_adjoint_backward are
    compared the same way for scale."""
    from paper_1904_11386_amd import binding
    from paper_1904_11386_amd.adjoint import OBJECTIVES, reverse_sweep, workload_with
    wl = W.make("c4_mini")
    params = (75.0, 0.005, 3.6)
    steps, every = 25, 10            # a ragged last segment of 5 steps
    for kind in ("com_z", "taylor_D"):
        sim = binding.sim_from_workload(workload_with(wl, *params), n_slots=3, ring_len=every)
        J = sim.adjoint_forward(steps, every, OBJECTIVES[kind], 0)
        g_call = sim.adjoint_backward()
        J2 = sim.adjoint_forward(steps, every, OBJECTIVES[kind], 0)
        g_staged = reverse_sweep(sim, steps, every, OBJECTIVES[kind])
        J3 = sim.adjoint_forward(steps, every, OBJECTIVES[kind], 0)
        g_call2 = sim.adjoint_backward()
        _say("  %s J %.10e %.10e %.10e" % (kind, J, J2, J3))
        _say("  backward call", g_call.tolist(), "staged", g_staged.tolist(), "second call", g_call2.tolist())
        rel = np.abs(g_staged - g_call) / np.abs(g_call)
        rel2 = np.abs(g_call2 - g_call) / np.abs(g_call)
        # max-norm relative over the gradient vector, as every parity bound
        # here: a small component carries the noise of the large ones
        err = float(np.abs(g_staged - g_call).max() / np.abs(g_call).max())
        _say("  staged vs call rel", rel.tolist(), "call vs call rel", rel2.tolist(), "max-norm %.2e" % err)
        assert abs(J2 - J) <= 1e-6 * abs(J) and abs(J3 - J) <= 1e-6 * abs(J)
        assert err < 1e-6, rel
        # the state after either sweep is the one at the start of the run
        obs = sim.observables()
        assert obs["step"] == 0
        sim.close()


def test_staged_reverse_sweep_order_and_state_errors():
    from paper_1904_11386_amd import binding
    from paper_1904_11386_amd.adjoint import workload_with
    wl = W.make("c4_mini")
    sim = binding.sim_from_workload(workload_with(wl, 75.0, 0.005, 3.6), n_slots=2, ring_len=10)
    sim.adjoint_forward(12, 10, binding.LBM_OBJ_COM_Z, 0)
    with pytest.raises(binding.LbmError) as e:
        sim.adjoint_step(0)                      # before the seed
    assert e.value.code == binding.LBM_ESTATE
    sim.adjoint_seed(binding.LBM_OBJ_COM_Z, 0)
    with pytest.raises(binding.LbmError) as e:
        sim.adjoint_step(0)                      # before a recording
    assert e.value.code == binding.LBM_ESTATE
    with pytest.raises(binding.LbmError) as e:
        sim.adjoint_seed(7, 0)
    assert e.value.code == binding.LBM_EINVAL
    with pytest.raises(binding.LbmError) as e:
        sim.adjoint_seed(binding.LBM_OBJ_COM_Z, 5)
    assert e.value.code == binding.LBM_EINVAL
    sim.load(1)
    with pytest.raises(binding.LbmError) as e:
        sim.adjoint_record(11)                   # longer than the ring
    assert e.value.code == binding.LBM_EINVAL
    sim.adjoint_record(2)
    with pytest.raises(binding.LbmError) as e:
        sim.adjoint_step(0)                      # out of order: 1 comes first
    assert e.value.code == binding.LBM_ESTATE
    with pytest.raises(binding.LbmError) as e:
        sim.adjoint_step(2)                      # outside the recording
    assert e.value.code == binding.LBM_EINVAL
    sim.adjoint_step(1)
    sim.adjoint_step(0)
    g = sim.adjoint_grads()
    assert np.all(np.isfinite(g))
    sim.close()
