"""CPU oracle for the tall & skinny products (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never does.
"""
from .oracle import (  # noqa: F401
    Oracle, build, tsmttsm, tsmm, tsmttsm_entries, tsmm_rows, orth_step, max_threads,
)
