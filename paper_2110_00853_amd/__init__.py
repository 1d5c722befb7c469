"""MI355X-native nodal DG LES hot path (right-hand side + LSRK54 step).

Modules:
  binding   -- ctypes binding of libcm.so (include/cm.h); device compute only
  workloads -- seeded synthetic meshes, model settings and initial states
  build     -- hipcc build of libcm.so for gfx950
"""
__all__ = ["binding", "workloads", "build"]
