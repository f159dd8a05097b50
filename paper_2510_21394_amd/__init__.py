"""MI355X (gfx950) matrix/tensor-oriented integrators for the space-fractional CGLE.

The computation lives in libfcgle.so (C ABI in include/fcgle.h); this package
only marshals arguments from torch tensors.
"""
from .fcgle import BatchPlan, ExpEulerTrajectory, Plan, Problem, host_eig, host_fd_weights, host_fz  # noqa: F401
from ._lib import FcgleError  # noqa: F401
