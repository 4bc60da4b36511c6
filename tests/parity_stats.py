"""Error statistics of the GPU parity tests (element-wise, gated on the max).

* row_rel: e_i = |a_i - ref_i| / |ref_i| per particle (the force's relative
  error; the paper validates each particle against a double-precision brute
  force, Sec. 4.1);
* cond_err: |a_i - ref_i| / scale_i with scale_i the sum of the magnitudes of
  row i's terms, from the oracle (term_scale_rows for the force,
  accel_vjp_scale_rows for the VJP): the error relative to the condition of
  the row's sum, meaningful also where the terms cancel (|ref_i| << scale_i),
  which random cotangents make common for the VJP;
* coord_err: |g - r| / max(|r|, 1e-3 max|r|) per coordinate, the gradient
  statistic of the 16384-body workload (r: the reference gradient of one kind,
  positions, velocities or masses).
"""
import numpy as np


def _norm_rows(a):
    a = np.asarray(a)
    return np.abs(a) if a.ndim == 1 else np.linalg.norm(a, axis=0)


def row_rel(a, ref):
    den = _norm_rows(ref)
    return _norm_rows(np.asarray(a) - np.asarray(ref)) / np.where(den > 0, den, 1.0)


def cond_err(a, ref, scale):
    scale = np.asarray(scale, dtype=np.float64)
    return _norm_rows(np.asarray(a) - np.asarray(ref)) / np.where(scale > 0, scale, 1.0)


def coord_err(g, ref):
    g, ref = np.asarray(g), np.asarray(ref)
    floor = 1e-3 * np.abs(ref).max()
    return np.abs(g - ref) / np.maximum(np.abs(ref), floor if floor > 0 else 1.0)
