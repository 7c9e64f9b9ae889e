"""MI355X (gfx950) split-and-parallelize (SaP) solver for dense banded
systems: hand-written HIP kernels behind a C ABI (include/sap.h), with this
package as the thin Python binding."""

from .sap import (SAP_COUPLED, SAP_DECOUPLED, SAP_PREC_FP32, SAP_PREC_FP64, SapError,
                  SapLibraryMissing, SapSolve, SapSolver, SapSparse, SapStats, load_library,
                  make_options, sap_solve_autograd, sap_workspace_bytes)

__all__ = ["SapSolver", "SapSolve", "SapStats", "SapError", "SapLibraryMissing",
           "load_library", "make_options", "sap_workspace_bytes", "sap_solve_autograd",
           "SAP_COUPLED", "SAP_DECOUPLED", "SAP_PREC_FP32", "SAP_PREC_FP64"]
