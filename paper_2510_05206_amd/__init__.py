"""MI355X-native differentiable particle-mesh hot path (DISCO-DJ II,
arXiv:2510.05206): HIP kernels behind the C ABI of include/pm.h, with a thin
Python binding.  PyTorch provides device memory and streams only."""
from ._lib import PMError, load  # noqa: F401
from .sim import Config, PMFunction, PMSim, simulate  # noqa: F401
