"""FP64 CPU oracle of the BSE hot path.

Test infrastructure only: imported by `tests/`, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library.  Shares no code with
the HIP path.
"""
from . import bse_oracle

__all__ = ["bse_oracle"]
