"""MI355X-native state-vector hot path (arXiv 2403.02512, PennyLane Lightning).

Submodules (imported on demand, so importing the package loads nothing):
  qsv        -- ctypes binding of the HIP C-ABI library libqsv.so
  build      -- compiles the HIP sources for gfx950 into libqsv.so
  workloads  -- seeded synthetic circuits, parameters and observables
  autograd   -- torch.autograd.Function whose backward is the adjoint sweep
"""
__version__ = "0.1.0"
