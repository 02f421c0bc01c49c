"""MI355X tensor-train k-eigenvalue transport solver (gfx950, HIP).

Modules:
  workload   seeded synthetic inputs (shared with the checker; no method arithmetic)
  qtt        exact QTT building blocks and host TT helpers (setup only)
  operators  H, S, F as mixed TT/QTT matrices (setup)
  native     ctypes binding of libttnt.so (the per-step path)
  solver     power-iteration driver over tt_power_step
  build      hipcc build of libttnt.so
"""
__all__ = ["workload", "qtt", "operators", "native", "solver", "build"]
