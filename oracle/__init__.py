"""FP64 CPU oracle for MBIR of spectral-domain OCT (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path.
"""
from .oct_oracle import *  # noqa: F401,F403
