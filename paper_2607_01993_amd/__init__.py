"""MI355X-native (gfx950, HIP) implementation of the sampled silhouette of
"Scalable and Distributed Silhouette Approximation" (arxiv 2607.01993).

The compute path is the HIP library libsilh.so (C ABI in include/silh.h);
`native` is its thin ctypes binding.  `synth` draws seeded synthetic inputs.
"""
from .native import (Context, SilhError, gl_pps_s, gl_s, load_library, silh_destroy,  # noqa: F401
                     silh_coh_sep, silh_draw_rows, silh_exact, silh_exact_rows, silh_philox_uniform, silh_pps_sample,
                     silh_prof_enable, silh_prof_get, silh_prof_reset, silh_rows_for, silh_sample_init,
                     silh_sample_view, silh_scores, silh_scores_rows, silh_sweep, silh_weighted_sums, version)
from .native import Server  # noqa: F401
