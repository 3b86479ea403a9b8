"""MI355X (gfx950) Shan-Chen foam lattice-Boltzmann library: C ABI in
include/foamlbm.h, HIP kernels in csrc/, ctypes binding in foamlbm.py.

The binding is imported lazily so that the seeded input generators
(`inputs`) can be used without the built library.
"""
