"""CPU oracle for exact best-match subsequence search under banded z-normalised DTW.

TEST INFRASTRUCTURE, not part of the search library: only the test suite, the
smoke check and the benchmark's CPU-baseline leg import it.  It shares no code
with the GPU path and imports nothing from it.

  reference  -- FP64 NumPy definitions (DTW recurrence, band, z-normalisation,
                bounds, brute-force best match, exhaustive warping paths,
                overlapping fragmentation).
  cascade    -- FP64 C implementation of the sequential cascade scan with
                early abandoning, partitioned over host threads (for sizes
                where brute force is too slow, and the timed CPU baseline).
"""
from . import reference  # noqa: F401
from .cascade import Cascade, build_cascade, cascade_path  # noqa: F401
