"""CPU FP64 oracle for the Schwarz waveform relaxation method (Besse & Xing,
arXiv 1503.02564).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  It shares no code
with the GPU path; only the seeded input generators
(``paper_1503_02564_amd.workloads``) serve both.

Parity status of each function is stated in its docstring; every function is
pinned by a test under ``tests/test_oracle_*.py`` unless it says
"parity unpinned".
"""
from .oracle import *  # noqa: F401,F403
