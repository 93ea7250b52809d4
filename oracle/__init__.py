"""CPU oracle for the silhouette hot path: plain, slow, float64.

TEST INFRASTRUCTURE ONLY.  It is imported by the tests, by the smoke check
and by the benchmark's CPU-baseline leg, and by nothing on the product path.
It shares no code, header or table with the HIP implementation.

Modules:
  philox      Philox4x32-10 and the 53-bit uniform built from it.
  distance    the four distances of the experiments, float64.
  silhouette  exact silhouette, Phase 1 / Phase 2 of Algorithm 1, the
              uniform-sampling variant and the global mean (Eq. 9).
  global_est  the subsampled global estimators gl-s (Eq. 8) and
              gl-pps-s / gl-uni-s (Eq. 10).
  coh_sep     cohesion and separation from cluster sums (Appendix B).
  cosine_sum  W_hat for the cosine distance by its linear form (the same
              estimator in O(n k d), for values at millions of rows).

Parity status: every function here is pinned by tests in tests/test_oracle_*.py
against values the paper prints, closed forms, brute force or invariants; none
is "parity unpinned".
"""
from .distance import CANB, COS, EUCL, MANH, dist_matrix, dist_to_point, metric_id  # noqa: F401
from .philox import STREAM_F0, STREAM_PPS, STREAM_ROWS, STREAM_UNI, bits53, philox4x32_10, uniform53  # noqa: F401
from .silhouette import (cluster_members, default_t, estimate, exact, global_mean,  # noqa: F401
                         pps_silhouette, sample, scores_from_weights)
from .global_est import draw_rows, gl_pps_s, gl_s, m_for, subset_mean, sweep  # noqa: F401
from .coh_sep import coh_sep_from_weights  # noqa: F401
from .cosine_sum import cosine_estimate, cosine_weights  # noqa: F401
