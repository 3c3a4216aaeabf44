"""CPU FP64 oracle of the domain-wall hot path (test infrastructure only).

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP library.
"""
from .oracle import *  # noqa: F401,F403
