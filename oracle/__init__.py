"""FP64 CPU reference for the polyethylene MD hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  It shares no code with the GPU library.
"""

from .oracle import *  # noqa: F401,F403
