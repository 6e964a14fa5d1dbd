"""MI355X-native geometric multigrid for Poisson's equation on octree AMR
meshes of 8^3-cell boxes (Teunissen & Ebert, arXiv:1708.08434, section 2.1).

The solver lives in libmg.so (HIP kernels for gfx950 behind the C ABI of
include/mg.h and include/mg_nn.h); ``mg`` and ``nn`` are its ctypes bindings.
"""
from . import mg  # noqa: F401
from . import nn  # noqa: F401
