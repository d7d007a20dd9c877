"""MI355X (gfx950) time stepper for the non-hydrostatic shallow-water scheme of
Escalante, Morales de Luna & Castro (arXiv 1706.04551).

The library is libnhswe.so (C ABI in include/nhswe.h); `Solver` (one grid)
and `Ensemble` (many grids advanced together) are its thin ctypes binding;
`run_noalloc` steps caller-owned device tensors without device allocation.
`inputs` builds the seeded synthetic workloads.
"""
from .binding import Ensemble, Solver, NhError, lib, run_noalloc  # noqa: F401

__all__ = ["Ensemble", "Solver", "NhError", "lib", "run_noalloc"]
