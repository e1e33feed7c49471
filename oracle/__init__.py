"""FP64 CPU oracle for online tensor LDA.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
load anything in this package: only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library
under ``paper_2511_07809_amd``.
"""
from . import tlda_oracle  # noqa: F401
