"""Plain FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU library never does, and this
package never imports the GPU library.
"""
from .oracle import (  # noqa: F401
    Oracle, build, lgl, load, hevi_coefficients, ark2_step, ark2_generic, column_matrix, num_threads, set_num_threads,
    l3_matrix, imex3d_step,
)
from . import mlp_oracle  # noqa: F401,E402
