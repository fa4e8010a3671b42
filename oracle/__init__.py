"""Plain FP64 CPU oracle for noise-subspace narrowband DOA estimation (PHD, MUSIC, EV, MN).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import this package.  The product path (the HIP library and its Python binding)
never imports, calls or links anything here, and this package shares no code with it.

Every function follows the paper's definitions directly, in float64 / complex128, with numpy
and LAPACK (``numpy.linalg.eigh``) as library primitives and no blocking or reordering beyond
what the definitions state.  Pins that tie each function to the paper and to mathematics
(closed forms, invariants, brute force) live in ``tests/test_oracle_*.py``.
"""

from .doa import (  # noqa: F401
    ALGS,
    grid_angles,
    steering,
    covariance,
    eig_desc,
    noise_subspace_matrix,
    step4_matrix,
    spectrum_quadratic_form,
    spectrum_factored,
    find_peaks,
    select_peaks,
    estimate,
    estimate_windowed,
    spectrum_factored_2d,
    find_peaks_2d,
    select_peaks_2d,
    estimate_2d,
    percent_error,
)
