"""MI355X-native hot path of the Sheffield Advanced Code (SMAUG+) MHD scheme.

The compute path is the HIP library ``libsacx.so`` (sources under ``csrc/``,
C ABI in ``include/sacx.h``); ``sacx`` is its thin ctypes binding.
"""

from .sacx import (  # noqa: F401
    FIELDS, BACKGROUND_FIELDS, PERIODIC, OPEN, EXCHANGE, FP64, FP32, GHOST, PROBLEM_ORSZAG_TANG, PROBLEM_BRIO_WU,
    StepGraph,
    DEFAULT_C2, DEFAULT_CSHK, Solver, Batch, SacxError, load_library, make_grid, make_params,
    workspace_size,
)
from .decomposed import DecomposedSolver, even_cuts  # noqa: F401
