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
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        g = ctx.sim.adjoint_backward()
        ctx.sim.close()
        s = float(gJ)
        return (torch.tensor(s * g[0] * math.pi / 180.0, dtype=torch.float64),
                torch.tensor(s * g[1], dtype=torch.float64), torch.tensor(s * g[2], dtype=torch.float64),
                None, None, None, None)


def capsule_objective(theta_deg, kS, G, wl, steps, every, objective="com_z"):
    return CapsuleObjective.apply(theta_deg, kS, G, wl, steps, every, objective)
