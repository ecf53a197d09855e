"""FP64 CPU oracle for the event-based 4D-STEM phase-contrast path.

TEST INFRASTRUCTURE.  This package is a plain, slow, obviously correct restatement
of what the paper computes (event reductions of Table 1 and Eq. 4, the DPC
integration of Sec. V, the scan transform, double-overlap set and Eq. 3 sum of
Sec. IV, and the adjoint of the SSB phase).  It shares no code with the HIP
library and imports nothing from it.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.

Parity status: every function is pinned by the CPU tests (brute force on tiny
inputs, closed forms and invariants) except where a docstring says otherwise.
"""
from . import dpc, eer, ssb

__all__ = ["eer", "dpc", "ssb"]
