"""Generalized-polynomial lattice Boltzmann method (arXiv:1510.07328) for MI355X.

The hot path (fused stream-and-collide BGK step with the zero-temperature
Fermi-Dirac equilibrium expanded in the paper's generalized polynomials) runs in
hand-written HIP kernels behind the C ABI of include/lbm.h; ``lbm`` is its
ctypes binding and ``inputs`` the seeded synthetic workloads.  Submodules are
imported on demand so that ``inputs`` is usable without the compiled library.
"""

__all__ = ["lbm", "inputs", "build"]
