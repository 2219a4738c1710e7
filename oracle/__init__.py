"""FP64 CPU oracle of SAFR.  Test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library.
"""
from . import mlp, safr  # noqa: F401
