"""lbsd: the tau = 1 step of the semi-discrete compressible lattice Boltzmann
method (arXiv 1602.02675) as hand-written HIP kernels for MI355X (gfx950).

* :mod:`.lbsd` -- Python binding of the C ABI in include/lbsd.h (needs the
  built ``liblbsd.so``; raises on import otherwise).
* :mod:`.inputs` -- seeded synthetic workloads.
* :mod:`.build` -- hipcc build of the library.
"""
__all__ = ["lbsd", "inputs", "build"]
