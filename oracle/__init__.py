"""FP64 CPU oracle for Fourier-domain dedispersion (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this package.
It shares no code with the HIP library and must never be used as a fallback by it.
"""
from .fdd_oracle import *  # noqa: F401,F403
from .fdd_oracle import __all__  # noqa: F401
