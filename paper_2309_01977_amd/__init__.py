"""MI355X-native SPECT OSEM hot path (paper: arXiv 2309.01977, Section 2.1).

The parallel-hole SPECT system matrix pair (Eq. 1 and its transpose) and the
OSEM subset update (Eq. 5, Table 1) run as hand-written gfx950 HIP kernels
behind the C ABI in include/spect.h; this package is the thin Python binding
(torch supplies device memory and streams) plus the OSEM driver loop.
"""
from ._binding import (EXPORTS, KERNELS, LIB_PATH, OP_BACK, OP_BSREM, OP_BSREM_STEP, OP_FWD, OP_OSEM, OP_RECON,
                       OP_SENS, OP_STEP, OP_STEP_VJP, REQ_DONE, REQ_FAILED, REQ_QUEUED, REQ_RUNNING, Batch,
                       KernelTimer, Server, Plan, SpectError, load_library, subset_angles)
from .recon import osem, osem_steps, sensitivities
from .autograd import back_project, osem_update, project, unrolled_osem

__all__ = ["Plan", "Batch", "Server", "SpectError", "KernelTimer", "load_library", "osem", "osem_steps", "sensitivities",
           "subset_angles", "EXPORTS", "KERNELS", "LIB_PATH", "OP_FWD", "OP_BACK", "OP_SENS", "OP_OSEM", "OP_RECON", "OP_BSREM_STEP", "OP_BSREM",
           "OP_STEP", "OP_STEP_VJP", "REQ_QUEUED", "REQ_RUNNING", "REQ_DONE", "REQ_FAILED",
           "project", "back_project", "osem_update", "unrolled_osem"]
