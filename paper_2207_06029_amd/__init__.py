"""MI355X-native D3Q19 BGK lattice-Boltzmann / dynamic immersed-boundary solver for rigid and
deformable capsules (arXiv 2207.06029, Sec. 1).

The solver is the HIP library liblbib.so (C ABI in include/lbib.h).  `api` holds the thin
Python binding with the same names; `inputs` generates seeded synthetic meshes and jobs.
Importing the package does not load the library; the first API call does, and fails loudly if
it has not been built.
"""
__all__ = ["api", "inputs", "build"]
