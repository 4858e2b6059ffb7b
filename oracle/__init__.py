"""FP64 CPU oracle for the two-component Shan-Chen D3Q19 / immersed-boundary
capsule step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry point and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never imports, calls or links it, and
the two share no code: the oracle takes plain arrays from the seeded input
generator and nothing else.

Everything here is plain, slow, float64 PyTorch-CPU code written from the
paper's equations (Wouters, Aouane, Krueger, Harting, arXiv:1904.11386):

  lattice.py   D3Q19 set and weights (Sec. II.A, eq. for w_i), second-order
               equilibrium (Sec. II.A), BGK relaxation (Sec. II.A), moments
               with the half-force velocity (Sec. II.A), pull streaming,
               half-way bounce-back on moving walls (Sec. II.C, eq. SBB),
               Shan-Chen inter-component force (Sec. II.D, eq. shanchen).
  ibm.py       Peskin 4-point delta, interpolation and spreading.  The paper
               names the immersed-boundary method as prior art (Sec. I) and
               gives no formula; the delta is Peskin's published 4-point
               kernel.
  membrane.py  Skalak strain energy (Sec. II.B, eq. strain), volume penalty
               (Sec. II.B, eq. volume), node forces as minus the energy
               gradient (Sec. II.B, virtual work), and the capsule
               observables (centre of mass, Sec. III.C eq. contactangle;
               Taylor deformation from the enclosed-volume inertia tensor,
               Sec. III.A eq. taylorparameter).
  sim.py       One time step in the order fixed by the design readings,
               and the autograd gradient used to check the adjoint.

Parity status per function is listed in each module header.
"""

from .lattice import C, W, OPP, CS2  # noqa: F401
from .sim import OracleSim  # noqa: F401
