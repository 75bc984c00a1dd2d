"""FP64 CPU oracle of the BSGD-TV method — TEST INFRASTRUCTURE ONLY.

Only the test suite, the package's smoke check and the benchmark's CPU
baseline leg may import this package.  The library and its Python binding
never import it, and it imports nothing from them.
"""
from . import bsgd_ref  # noqa: F401
from .bsgd_ref import *  # noqa: F401,F403
