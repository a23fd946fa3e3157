"""CPU FP64 oracle for the FMM-preconditioned Poisson solve (arXiv:1308.3339).

Test infrastructure only: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only users.  The product package never imports it.
"""
from .oracle import *  # noqa: F401,F403
from .oracle import _f64, _ip, _ptr  # noqa: F401  (raw-pointer helpers for tests)
from . import adjoint  # noqa: F401  (differentiation workload: exact FD solve, bumps, gradients)
