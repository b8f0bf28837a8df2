"""MI355X (gfx950) implementation of the consistent VANSE lattice Boltzmann
step of arXiv:2208.09267.

  paper_2208_09267_amd.vanse      ctypes binding of the C ABI (include/vanse.h)
  paper_2208_09267_amd.workloads  seeded synthetic inputs (no method arithmetic)
  paper_2208_09267_amd.build      hipcc build of libvanse.so

Importing the package loads nothing; ``vanse`` loads the HIP library on first
use and raises if it has not been built.
"""
