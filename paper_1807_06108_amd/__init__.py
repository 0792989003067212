"""MI355X (gfx950) implementation of one MPPI iteration on a jump-diffusion
process (Wang, Williams, Theodorou, arXiv 1807.06108, Algorithm 1).

  native      ctypes binding of libmppi_jump.so (C ABI: include/mppi_jump.h)
  controller  Controller: a context and its device workspace (torch memory)
  workloads   seeded synthetic configurations and inputs
  build       in-tree hipcc build of the library
"""

__all__ = ["native", "controller", "workloads", "build"]
