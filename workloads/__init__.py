"""Seeded, synthetic inputs shared by the CPU oracle and the GPU path.

This package only builds initial states (conserved variables on a cell-centred
grid) for the test problems of the paper's verification section and for the
validation problems used by the tests.  It contains none of the scheme's
arithmetic: no fluxes, no derivatives, no hyper-diffusion, no time stepping.
Both sides of every parity test receive the very same FP64 arrays from here.
"""

from .problems import (  # noqa: F401
    Problem,
    FIELDS,
    BACKGROUND_FIELDS,
    orszag_tang,
    brio_wu,
    uniform_state,
    entropy_wave,
    sound_wave,
    alfven_wave,
    random_smooth,
    split_background,
    with_gravity,
    stratified_atmosphere,
    transpose_problem,
    batch_instances,
    cell_centres,
    synthetic_ratio_planes,
    cnn_case,
)
from .problems3d import (  # noqa: F401,E402
    Problem3,
    FIELDS3,
    conserved3,
    orszag_tang_3d,
    uniform_3d,
    entropy_wave_3d,
    entropy_wave_3d_exact,
    random_smooth_3d,
    embed_2d,
    extract_2d,
)
