"""MI355X-native joint time-frequency scattering (JTFS) and metamer descent.

The transform, its adjoint and the descent updates run in hand-written HIP kernels for
gfx950 behind the C ABI of include/jtfs.h (libjtfs.so in this directory). Importing the
package does not load the library; the first use does, and fails if it is not built.
"""
from .jtfs import Optimizer, Params, Plan, jtfs_backward, jtfs_forward, jtfs_metamer_step, jtfs_plan  # noqa: F401

__all__ = ["Params", "Plan", "Optimizer", "jtfs_plan", "jtfs_forward", "jtfs_backward", "jtfs_metamer_step"]
