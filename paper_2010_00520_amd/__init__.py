"""MI355X-native FFT-based FMM translation with compressed translation operators.

The compute path is libtfmm (HIP kernels for gfx950 behind the C ABI in
include/tfmm.h); this package only builds it and binds it.
"""
from .tfmm import (FORMATS, PRECISIONS, Basis, Context, NearField, Operator, Problem, TfmmError, load,  # noqa: F401
                   make_problem, SIGNATURES)
