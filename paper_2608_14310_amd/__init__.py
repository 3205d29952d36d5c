"""MI355X (gfx950) CAV-multigrid FGMRES for the reduced Eulerian IB system.

The compute path is the HIP library `libcavmg.so` (C ABI in include/cavmg.h).
This package only marshals arguments to it; PyTorch supplies device memory and
the stream. Importing works without a GPU; using a Solver needs the built
library and a ROCm device, and fails loudly otherwise.
"""
from ._binding import (CAV_LAW, CAVError, Net, Solver, batch_solve, describe_structure, lib, library_path, structure_force,
                       EXPORTED_SYMBOLS)

__all__ = ["Solver", "Net", "batch_solve", "CAVError", "CAV_LAW", "describe_structure", "structure_force", "lib", "library_path", "EXPORTED_SYMBOLS"]
