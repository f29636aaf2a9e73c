"""CPU FP64 oracle for the outer-volume path -- test infrastructure only.

Plain, slow, obviously correct implementations of what the HIP library computes,
written from the paper's statement of the problem:

* ``exact``   -- OBV(X, O) of one box by the divergence theorem (Sec. 3, Eq. 4),
                 in float64 or exact rationals;
* ``raygrid`` -- the jittered parallel-ray estimator of OBV with parity
                 integration along each ray (Sec. 4.1, Eq. 9 generalised);
* ``fit``     -- area-weighted covariance OBB of a triangle cluster;
* ``rng``     -- SplitMix64, the counter-based generator both sides implement
                 from its publication to draw the ray jitter;
* ``collision`` -- synthetic sphere queries against a box hierarchy (tests and
                 hits), the stand-in for the paper's collision experiment;
* ``central`` -- the paper's central-projection estimator (Sec. 4.1, Eq. 9-10:
                 cube-map directions from the box centre, cone volumes).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
and never imports it; inputs come from ``synth`` or from the caller.
"""
from . import rng, geometry, exact, raygrid, fit, collision, central  # noqa: F401
