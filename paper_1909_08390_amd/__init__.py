"""MI355X-native IMEX finite-difference lattice Boltzmann with MP-9 advection.

The compute path is the C-ABI library ``libimexlb.so`` (HIP kernels for
gfx950) reached through :mod:`paper_1909_08390_amd.imexlb`; this package
import itself loads nothing, so the seeded input generators in
:mod:`paper_1909_08390_amd.workloads` can be used without a GPU.
"""
