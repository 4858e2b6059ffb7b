"""Capsule objectives as differentiable functions of the contact angle, the
shear modulus and the Shan-Chen coupling, with gradients from the library's
hand-written discrete adjoint (checkpoint every `every` steps, recompute in
a device ring).  Marshalling only: the forward run, the checkpoints and the
reverse sweep all execute in the HIP library."""

import copy
import math

import torch

from . import binding

OBJECTIVES = {"com_z": binding.LBM_OBJ_COM_Z, "taylor_D": binding.LBM_OBJ_TAYLOR_D}


def workload_with(wl, theta_deg, kS, G):
    """Copy of a workload with every capsule's angle and shear modulus, and
    G, replaced."""
    w = copy.copy(wl)
    w.capsules = [copy.copy(c) for c in wl.capsules]
    for c in w.capsules:
        c.theta_deg = float(theta_deg)
        c.kS = float(kS)
    w.G = float(G)
    return w


def reverse_sweep(sim, steps, every, objective, capsule=0):
    """The reverse sweep after sim.adjoint_forward(steps, every, ...), one
    library call per stage: seed dJ/dX at the final state, then for each
    checkpoint segment, last first, reload it, recompute it into the ring and
    apply its steps' adjoints in reverse; the state is left at the start of
    the run.  Returns dJ/d(theta [rad], kS, G)."""
    sim.adjoint_seed(objective, capsule)
    nseg = (steps + every - 1) // every
    for sgm in reversed(range(nseg)):
        n = min(every, steps - sgm * every)
        sim.load(sgm)
        sim.adjoint_record(n)
        for k in reversed(range(n)):
            sim.adjoint_step(k)
    sim.load(0)
    return sim.adjoint_grads()


class CapsuleObjective(torch.autograd.Function):
    """J = objective(capsule 0) after `steps` steps of `wl` run with
    (theta_deg, kS, G); backward returns dJ/dtheta_deg, dJ/dkS, dJ/dG."""

    @staticmethod
    def forward(ctx, theta_deg, kS, G, wl, steps, every, objective="com_z"):
        nseg = (steps + every - 1) // every
        sim = binding.sim_from_workload(workload_with(wl, float(theta_deg), float(kS), float(G)),
                                        n_slots=nseg, ring_len=every)
        J = sim.adjoint_forward(steps, every, OBJECTIVES[objective], 0)
        ctx.sim = sim
        ctx.steps, ctx.every, ctx.objective = steps, every, OBJECTIVES[objective]
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        g = reverse_sweep(ctx.sim, ctx.steps, ctx.every, ctx.objective)
        ctx.sim.close()
        s = float(gJ)
        return (torch.tensor(s * g[0] * math.pi / 180.0, dtype=torch.float64),
                torch.tensor(s * g[1], dtype=torch.float64), torch.tensor(s * g[2], dtype=torch.float64),
                None, None, None, None)


def capsule_objective(theta_deg, kS, G, wl, steps, every, objective="com_z"):
    return CapsuleObjective.apply(theta_deg, kS, G, wl, steps, every, objective)
