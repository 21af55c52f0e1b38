"""MI355X-native hot path of MR. POP (multi-robot AO-x + dRRT planning).

Python binding of ``libmrpop.so``: argument marshalling only.  Every step of
the hot path runs in the HIP kernels behind the C ABI (``include/mrpop.h``);
PyTorch provides device memory and streams.  Importing this package fails if
the library has not been built (``python -m paper_2609_30644_amd.build``).
"""
from ._binding import (  # noqa: F401
    MrpopError,
    Context,
    Scene,
    ValidateStats,
    KernelProfile,
    WORK_NAMES,
    PlanParams,
    PlanResult,
    Incumbent,
    Server,
    lib_path,
    load_library,
    STATUS_NAMES,
)

__all__ = ["MrpopError", "Context", "Scene", "ValidateStats", "KernelProfile", "WORK_NAMES", "PlanParams", "PlanResult", "Incumbent", "Server", "lib_path", "load_library", "STATUS_NAMES"]
