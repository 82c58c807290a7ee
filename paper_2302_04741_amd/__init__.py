"""MI355X (gfx950) thermal lattice Boltzmann step with Hermite body force.

Implements the hot path of Li & Shan, "Body-force modelling in thermal
compressible flows with lattice Boltzmann method" (arXiv:2302.04741): the fused
D2Q37 / D3Q39 time step of eq. (lbm) with the third-moment force term of
eq. (fi), as HIP kernels behind the C ABI of include/lbm.h.

    from paper_2302_04741_amd import Sim, workloads
    wl = workloads.periodic_2d()
    sim = from_workload(wl)          # needs a ROCm GPU and the built liblbm.so
    sim.step(1000); rho, u, theta = sim.moments()

Importing the package loads neither torch nor the library; ``Sim`` does, and
fails loudly if either the GPU or liblbm.so is missing.
"""
from . import workloads  # noqa: F401

__all__ = ["Sim", "from_workload", "workloads", "build_library"]


def __getattr__(name):
    if name in ("Sim", "from_workload"):
        from . import sim

        return getattr(sim, name)
    raise AttributeError(name)


def build_library() -> str:
    from .build import build

    return build()
