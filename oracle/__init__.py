"""CPU oracle (test infrastructure only): plain FP64 NumPy implementation of the
beta-NMF majorization-minimization updates, used to check the GPU library.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package; the GPU library never does.
"""
from .nmf_oracle import *  # noqa: F401,F403
from .nmf_oracle import __all__  # noqa: F401
