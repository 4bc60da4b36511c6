"""MI355X-native softened direct-summation gravity.

The compute lives in libnbody_accel.so (hand-written HIP kernels for gfx950,
C ABI in include/nbody.h); this package only binds it.  Functions carry the
C entry points' names: nbody_accel, nbody_accel_noalloc, nbody_step, nbody_energy, nbody_accel_vjp,
nbody_traj_grad, nbody_step_batched, nbody_accel_jerk, nbody_step_hermite,
nbody_accel_jerk_snap, nbody_step_hermite6, nbody_potential, nbody_tune, nbody_tune_batched,
nbody_set_config, plus the autograd Function NBodyTrajectory.
"""
from ._binding import (ENERGY_FIELDS, NBODY_ACC_VALID, NBODY_CHECK_FINITE, NBODY_EHIP, NBODY_EINVAL,
                       NBODY_ENOMEM, NBODY_ENONFINITE, NBODY_EUNSUPPORTED, NBODY_EXCLUDE_SELF, NBODY_FP32,
                       NBODY_FP32C, NBODY_FP64, NBODY_OK, LIB_PATH, PRECISIONS, NBodyError, load,
                       nbody_accel, nbody_accel_noalloc, nbody_accel_jerk, nbody_accel_jerk_snap, nbody_accel_vjp, nbody_energy,
                       nbody_finalize, nbody_last_error, nbody_potential, nbody_step_hermite, nbody_step_hermite6,
                       nbody_set_config, nbody_step, nbody_step_batched, nbody_traj_grad, nbody_tune, nbody_tune_batched,
                       nbody_version)
from .autograd import NBodyTrajectory, trajectory

__all__ = [
    "nbody_accel", "nbody_accel_noalloc", "nbody_step", "nbody_energy", "nbody_accel_vjp", "nbody_traj_grad",
    "nbody_accel_jerk", "nbody_step_hermite", "nbody_accel_jerk_snap", "nbody_step_hermite6", "nbody_potential",
    "nbody_step_batched", "nbody_tune", "nbody_tune_batched", "nbody_set_config", "nbody_last_error", "nbody_finalize",
    "nbody_version", "NBodyTrajectory", "trajectory", "NBodyError", "load", "LIB_PATH", "PRECISIONS",
    "ENERGY_FIELDS", "NBODY_OK", "NBODY_EINVAL", "NBODY_EHIP", "NBODY_ENOMEM", "NBODY_ENONFINITE",
    "NBODY_EUNSUPPORTED", "NBODY_FP64", "NBODY_FP32C", "NBODY_FP32", "NBODY_EXCLUDE_SELF",
    "NBODY_CHECK_FINITE", "NBODY_ACC_VALID",
]
