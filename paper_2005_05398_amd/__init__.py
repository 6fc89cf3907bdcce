"""MI355X (gfx950) solver for the Faddeev-Merkuriev spline-collocation system
of arXiv:2005.05398: tensor-trick-preconditioned flexible GMRES in HIP.

Submodules:
  fm         ctypes binding of libfm.so (include/fm.h); no CPU fallback
  build      in-tree hipcc build of libfm.so
  workloads  problem descriptions and seeded inputs (data only)

Importing the package loads nothing; the library is loaded on first use.
"""
