"""Seeded synthetic frame generator shared by the tests, the benchmark and the oracle timing.

This package draws inputs only: array geometries, source directions, source waveforms and
noise, combined by the narrowband signal model X = A(theta) S + W (Section 3.1, Eq. 1 and
Table 1).  It holds none of the estimation method's arithmetic (covariance, eigensolve,
noise-subspace selection, spectrum scan, peak search): those live separately in the oracle
and in the HIP library, and neither imports the other.  The workloads are JSON recipes under
``configs/``.
"""

from .frames import (  # noqa: F401
    CONFIGS,
    EL_GRIDS_2D,
    Frame,
    FrameSet,
    load_config,
    make_config,
    make_frame,
    make_frames,
    ula_positions,
    uca_positions,
    config_seed,
)
