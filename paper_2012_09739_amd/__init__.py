"""MI355X-native MLMC level-correction estimator with low-precision approximate Gaussian
variables: HIP kernels for gfx950 behind the C-ABI of include/mlmc.h (libmlmc.so), with a
ctypes binding of the same names (``mlmc``)."""

from . import mlmc  # noqa: F401
from .mlmc import *  # noqa: F401,F403
