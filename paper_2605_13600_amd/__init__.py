"""MI355X (gfx950) implementation of SCOUP's hot path behind a C ABI (libscoup.so).

Sparse coefficient uplift (Eq. 5 / Algorithm 1) with Top-K filtering (Eq. 6),
sparse coefficient render (Eq. 7) and codebook decode (Eq. 8), plus the
backward of render and decode.  Every step runs in the hand-written HIP
kernels of ``csrc/``; this package only marshals arguments (``_lib``) and
offers torch-facing wrappers (``api``).  Importing it does not load the
library; the first call does, and raises if the library was not built.
"""
from .api import (  # noqa: F401
    DeviceGaussians, DeviceViews, ScoupError, camera_struct, decode, entropy, gaussians_to_device,
    RenderDecode, relevancy, render, render_backward, render_coeff, render_decode, render_views,
    set_deferred_entry_limit,
    set_views_in_flight, stage_timing, topk, uplift, uplift_touch_stats,
    uplift_accumulate, uplift_dense, uplift_levels, views_in_flight, views_to_device,
)
