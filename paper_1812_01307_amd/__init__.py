"""BSGD-TV on MI355X: block CSR projections, delayed-residual steps and an
FGP TV prox in hand-written HIP kernels for gfx950, behind a C ABI
(include/bsgd.h).

``capi`` is the ctypes binding (same names as the C entry points);
``host`` uploads host CSR arrays and builds a plan.  Importing the package
raises ImportError when libbsgd.so has not been built.
"""
from . import capi  # noqa: F401
from .capi import *  # noqa: F401,F403
from .host import plan_from_host, to_device  # noqa: F401
