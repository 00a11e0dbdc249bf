"""MI355X-native equi hash join (SHJ and radix-partitioned PHJ) for gfx950.

Submodules:
  hj     ctypes binding of include/hj.h (libhj.so, built by ``build``)
  gen    seeded synthetic relations (host side; ``gen.hip`` is the device side)
  build  hipcc build of the HIP libraries

Importing the package loads nothing; ``paper_1307_1955_amd.hj`` loads torch and
the library on first use.
"""
__all__ = ["hj", "gen", "build"]
