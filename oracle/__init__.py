"""FP64 CPU oracle for the CWTHF hot path (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  See ``oracle.cwthf`` for the functions and the passages of the
paper each one follows.
"""
from .cwthf import *  # noqa: F401,F403
from .cwthf import __all__  # noqa: F401
