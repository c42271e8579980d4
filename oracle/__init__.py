"""FP64 reference implementation of the batched physics step (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library.
"""
from .oracle import (CON_SIZE, MODE_CONVERGED, MODE_FIXED, Oracle, build, lib_path,  # noqa: F401
                     set_capsule_box_tolerances)
