"""CPU oracle for fast graph-based denoising (FGBD) of point-cloud colour.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow FP64 restatement of
the method (numpy, with library primitives for sorting and small eigenproblems)
used to check the GPU library.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library never does, and the two
share no code.
"""
from .fgbd_oracle import *  # noqa: F401,F403
from .fgbd_oracle import __all__  # noqa: F401
