"""MI355X-native neighbourhood-graph construction by the multiple sorting method.

The compute path lives in a C-ABI shared library (``libmsm.so``, header
``include/msm.h``) of hand-written HIP kernels for gfx950. ``msm`` is the thin
ctypes binding; ``inputs`` holds the seeded synthetic workloads.

Importing the package loads nothing; ``paper_0904_3151_amd.msm`` loads the
library and raises if it has not been built.
"""

__all__ = ["inputs", "msm"]
