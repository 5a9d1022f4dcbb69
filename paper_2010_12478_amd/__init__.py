"""MI355X-native series registration by prefix scan (arXiv 2010.12478).

The hot path is the HIP library libregscan.so (include/regscan.h); this
package is its thin Python binding.  Importing it fails if the library has
not been built (``python -m paper_2010_12478_amd.build``).
"""
from ._lib import (LIB_PATH, REG_S_ABORTED, REG_S_MAXITER, REG_S_NONFINITE, REG_S_OK, RegError,
                   lib, plan)
from .api import (autotune, compose, energy_grad, energy_grad_noalloc, last_solve_launch_ms, last_solve_timing, prolong, pyramid,
                  pyramid_energy, pyramid_energy_backward, release, restrict, rigid_solve_batch, scan_mock, scan_run,
                  scan_run_flex, scan_run_rigid, set_tuning, solve_batch, warp, warp_adjoint)
from .autograd import WarpEnergy, warp_energy

__all__ = [
    "LIB_PATH", "RegError", "lib", "plan", "warp", "warp_adjoint", "energy_grad", "energy_grad_noalloc",
    "pyramid_energy",
    "pyramid_energy_backward", "compose", "restrict", "prolong", "pyramid", "solve_batch", "scan_run", "scan_run_flex", "rigid_solve_batch", "scan_run_rigid",
    "last_solve_timing", "last_solve_launch_ms", "scan_mock", "set_tuning", "autotune", "release",
    "WarpEnergy", "warp_energy",
    "REG_S_OK", "REG_S_MAXITER", "REG_S_NONFINITE", "REG_S_ABORTED",
]
