"""MI355X-native noise-subspace narrowband DOA estimation (PHD, MUSIC, EV, MN).

The estimation path runs in libnssdoa.so (hand-written HIP for gfx950 behind a C ABI declared
in include/nssdoa.h); this package only marshals arguments to it.
"""

from ._abi import (  # noqa: F401
    ALGS, PRECS, PEAK_DTYPE, NssdoaError, load,
    ST_NONFINITE_INPUT, ST_EVD_NOT_CONVERGED, ST_DEGENERATE, ST_FEWER_PEAKS, ST_PEAK_OVERFLOW,
    ST_FALLBACK_USED,
    WS_COV, WS_EVALS, WS_EVECS, WS_B, WS_QREF, WS_SPECTRUM,
)
from .api import MLP, Batch, Options, Pipeline, Plan, decode_peaks, flatten_params, unflatten_params  # noqa: F401
