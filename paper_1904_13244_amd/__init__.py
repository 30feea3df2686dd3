"""MI355X-native MR-STAT hot path: EPG linearisation with forward-mode tangents,
separable Cartesian encoding contraction into r, J v and Re(J^H w), and the
inexact Gauss-Newton step, as hand-written HIP kernels for gfx950 behind the C
ABI of include/mrstat.h (libmrstat.so). ``binding`` holds the thin ctypes
layer; ``inputs`` the seeded synthetic workloads; ``build`` compiles the
library in-tree.

Paper: van der Heide, Sbrizzi, Luijten, van den Berg, "High resolution in-vivo
MR-STAT using a matrix-free and parallelized reconstruction algorithm",
arXiv 1904.13244.
"""
__all__ = ["binding", "inputs", "build"]
