"""MI355X (gfx950) Jacobi-PCG for P1/P2 FEM Laplace systems with many right-hand sides.

The compute path is libfemcg.so (HIP kernels + C ABI, include/femcg.h);
``femcg`` is its ctypes binding.  Importing the package does not load the
library; the first call does, and fails loudly if it is not built.
"""
from . import femcg  # noqa: F401
