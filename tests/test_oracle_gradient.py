"""Pin of the oracle's reverse-mode gradient (checkpoint and recompute)
against FP64 central finite differences, for both capsule objectives, on the
48x24x24 sheared channel (no GPU)."""

import math

import numpy as np
import pytest
import torch

from oracle import sim as S
from paper_1904_11386_amd import workloads as W


class ChannelSim:
    params = (75.0, 0.005, 3.6)

    def __init__(self):
        self.wl = W.make("c4_mini")

    def __call__(self, th, ks, G):
        wl = self.wl
        c = wl.capsules[0]
        xyz, tri = c.mesh()
        return S.OracleSim(wl.rhoA.astype(np.float64), wl.rhoB.astype(np.float64),
                           [dict(xyz=xyz, tri=tri, kS=ks, C=c.C, kV=c.kV, theta=th)], tau=wl.tau, G=G,
                           walls=wl.walls, u_lo=wl.wall_u_lo, u_hi=wl.wall_u_hi, rho_maj=wl.rho_maj,
                           rho_min=wl.rho_min, z_interface=wl.z_interface, wet_scale=wl.wet_scale,
                           differentiable=True)


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["com_z", "taylor_D"])
def test_oracle_gradient_matches_central_differences(kind):
    torch.set_num_threads(8)
    ms = ChannelSim()
    steps, every = 30, 10
    J, g = S.gradient(ms, steps, every, kind)

    def run(th, ks, G):
        s = ms(th, ks, G)
        with torch.no_grad():
            s.run(steps)
            return float(S.objective(s, kind))

    for i, h in enumerate((0.05, 1e-5, 1e-4)):
        p = list(ms.params)
        pp, pm = list(p), list(p)
        pp[i] += h
        pm[i] -= h
        fd = (run(*pp) - run(*pm)) / (2 * h)
        if i == 0:
            fd *= 180.0 / math.pi
        assert float(g[i]) == pytest.approx(fd, rel=1e-5, abs=1e-12), (kind, i, float(g[i]), fd)
