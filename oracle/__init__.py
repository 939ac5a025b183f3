"""FP64 CPU oracle for the RTCUR hot loop.

TEST INFRASTRUCTURE ONLY.  Only tests/, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library under ``paper_2108_10448_amd/`` and never imports it.
"""

from .rtcur import (E_INVAL, E_NONFINITE, E_RANK, NOT_CONVERGED, OK, Factors,
                    OracleError, Result, evaluate, gather_blocks, l_update,
                    outliers, rank_rtol, rtcur, truncated_pinv)
from .sampler import (Sample, Stream, chidori_tuples, decode_columns,
                      draw_sample, encode_columns, floyd_subset, sample_I,
                      splitmix64_step)
from .tensor import (fold, fro, hard_threshold, mode_product,
                     multi_mode_product, round_bf16, unfold)
