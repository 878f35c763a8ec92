"""MI355X-native Z4c right-hand side + RK4 substep (arXiv 2607.08743 spacetime hot path).

* ``paper_2607_08743_amd.z4c``    -- ctypes binding of libz4c.so (include/z4c.h)
* ``paper_2607_08743_amd.inputs`` -- seeded synthetic initial data and workloads
* ``paper_2607_08743_amd.build``  -- hipcc build of libz4c.so for gfx950
"""
from . import inputs  # noqa: F401
