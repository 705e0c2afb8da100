"""lrdm: low-rank density-matrix evolution with eigenvalue truncation on AMD MI355X (gfx950).

The compute path is the HIP library liblrdm.so (include/lrdm.h); this package holds its
sources (csrc/), the build script and a thin ctypes binding (lrdm.py).
"""
from .lrdm import (C64, C128, FLAG_OVERLAP, FLAG_PLAIN, Batch, FullRankDM, LowRankDM, LrdmError, load_library,  # noqa: F401
                   run_program, run_program_fdm, workspace_size)
