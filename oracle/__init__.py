"""FP64 CPU oracle for the sparse-code uplift, sparse render, decode and backward.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
imports, links or calls it, and the oracle shares no code with the library:
the only thing both consume is the seeded input arrays of ``scenegen``.

Every step is a plain, slow, obviously correct transcription of the paper's
definitions in float64 (inputs are float32 and are upcast exactly):

* ``project``    3DGS covariance and EWA projection (Sec. 3, the tile
                 rasterizer whose weights feed Eq. 1-2).
* ``composite``  front-to-back alpha blending, e = alpha * T (Eq. 2), with
                 the 3DGS numerics: alpha clamp 0.99, skip alpha < 1/255,
                 stop before T drops below 1e-4.
* ``uplift``     weighted sparse accumulation (Eq. 5, Algorithm 1) and
                 Top-K with L1 normalisation (Eq. 6).
* ``render``     sparse coefficient render (Eq. 7) and codebook decode (Eq. 8).
* ``backward``   gradients of a cosine loss through render and decode.
* ``brute``      an independent scalar brute force used to pin the above.

Parity status of each function is stated in its module docstring.
"""
from . import project, composite, uplift, render, backward, brute  # noqa: F401
