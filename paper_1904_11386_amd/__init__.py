"""MI355X (gfx950) two-component Shan-Chen lattice Boltzmann step with
immersed-boundary Skalak capsules: HIP kernels behind a C ABI."""
