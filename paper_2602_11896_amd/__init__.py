"""MI355X-native joint time-frequency scattering (JTFS) and metamer descent.

The transform, its adjoint and the descent updates run in hand-written HIP kernels for
gfx950 behind the C ABI of include/jtfs.h (libjtfs.so in this directory). Importing the
package does not load the library; the first use does, and fails if it is not built.
"""
from .jtfs import (Optimizer, Params, Plan, Tuning, autotune, jtfs_backward, jtfs_forward,  # noqa: F401
                   jtfs_loss, jtfs_metamer_step, jtfs_plan, opt_status)

__all__ = ["Params", "Plan", "Optimizer", "Tuning", "autotune", "jtfs_plan", "jtfs_forward", "jtfs_backward",
           "jtfs_metamer_step", "jtfs_loss", "opt_status"]
