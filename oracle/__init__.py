"""CPU complex128 oracle of the state-vector method -- TEST INFRASTRUCTURE.

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may
import this package. It shares no code with the GPU library: it reads the same
seeded circuits (plain data) and computes everything else on its own.
"""

from .oracle import *  # noqa: F401,F403
from .oracle import using_library  # noqa: F401
