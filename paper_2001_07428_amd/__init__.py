"""MI355X-native thick-restart Lanczos for Hermitian J-symmetric matrices.

The solver is the C-ABI library libjlanczos.so (HIP kernels for gfx950,
declared in include/jlanczos.h); `jlanczos` is its ctypes binding and
`inputs` holds the seeded synthetic workloads.  Importing the package does not
load the library; the first binding call does, and raises if it is missing.
"""
from . import inputs  # noqa: F401
