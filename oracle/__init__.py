"""FP64 CPU oracle (ctypes wrapper over ``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It shares no code
with the GPU library; the two meet only in the seeded inputs of ``ics``.

Arrays follow the same SoA convention as the C code: positions, velocities and
accelerations are float64 arrays of shape (3, N); masses have shape (N,).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64


def build(force=False):
    """Compile ``liboracle.so`` with gcc (plain IEEE double, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_accel.argtypes = [_I64, _D, _D, ctypes.c_double, ctypes.c_double, _D]
        lib.oracle_accel_rows.argtypes = [_I64, _D, _D, ctypes.c_double, ctypes.c_double, _I64,
                                          ctypes.POINTER(ctypes.c_int64), _D]
        lib.oracle_term_scale_rows.argtypes = lib.oracle_accel_rows.argtypes
        lib.oracle_kdk.argtypes = [_I64, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, _I64, _D]
        lib.oracle_energy.argtypes = [_I64, _D, _D, _D, ctypes.c_double, ctypes.c_double, _D]
        lib.oracle_accel_vjp.argtypes = [_I64, _D, _D, _D, ctypes.c_double, ctypes.c_double, _D, _D]
        lib.oracle_accel_vjp_rows.argtypes = [_I64, _D, _D, _D, ctypes.c_double, ctypes.c_double, _I64,
                                              ctypes.POINTER(ctypes.c_int64), _D, _D]
        lib.oracle_accel_vjp_scale_rows.argtypes = lib.oracle_accel_vjp_rows.argtypes
        lib.oracle_accel_jvp.argtypes = [_I64, _D, _D, _D, _D, ctypes.c_double, ctypes.c_double, _D]
        lib.oracle_kdk_adjoint.argtypes = [_I64, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, _I64, _D, _D, _D, _D, _D]
        lib.oracle_accel_jerk.argtypes = [_I64, _D, _D, _D, ctypes.c_double, ctypes.c_double, _D, _D]
        lib.oracle_hermite4.argtypes = [_I64, _D, _D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double, _I64]
        lib.oracle_accel_jerk_snap.argtypes = [_I64, _D, _D, _D, _D, ctypes.c_double, ctypes.c_double, _D, _D, _D]
        lib.oracle_accel_jerk_snap_rows.argtypes = [_I64, _D, _D, _D, _D, ctypes.c_double, ctypes.c_double, _I64,
                                                    ctypes.POINTER(ctypes.c_int64), _D, _D, _D]
        lib.oracle_accel_jerk_rows.argtypes = [_I64, _D, _D, _D, ctypes.c_double, ctypes.c_double, _I64,
                                               ctypes.POINTER(ctypes.c_int64), _D, _D]
        lib.oracle_hermite6_crackle.argtypes = [_I64, ctypes.c_double, _D, _D, _D, _D, _D, _D, _D]
        lib.oracle_hermite6.argtypes = [_I64, _D, _D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double, _I64]
        lib.oracle_potential.argtypes = [_I64, _D, _D, ctypes.c_double, ctypes.c_double, _D]
        lib.oracle_msd_loss.argtypes = [_I64, _D, _D]
        lib.oracle_msd_loss.restype = ctypes.c_double
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_num_threads.restype = None
        _lib = lib
    return _lib


def _c(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


def _p(a):
    return a.ctypes.data_as(_D)


def num_threads():
    return _load().oracle_num_threads()


def set_num_threads(k):
    """Threads of the following oracle calls (OpenMP); for timing only."""
    _load().oracle_set_num_threads(int(k))


def accel(x, m, G=1.0, eps=0.0):
    """a_i = G sum_{j != i} m_j d_ij / (|d_ij|^2 + eps^2)^(3/2), d_ij = x_j - x_i."""
    m = _c(m)
    n = m.shape[0]
    x = _c(x, (3, n))
    a = np.empty((3, n))
    _load().oracle_accel(n, _p(x), _p(m), float(G), float(eps), _p(a))
    return a


def accel_rows(x, m, rows, G=1.0, eps=0.0):
    """The rows ``rows`` of ``accel`` only, shape (3, len(rows))."""
    m = _c(m)
    n = m.shape[0]
    x = _c(x, (3, n))
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= n):
        raise ValueError("row index out of range")
    out = np.empty((3, rows.size))
    _load().oracle_accel_rows(n, _p(x), _p(m), float(G), float(eps), rows.size,
                              rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(out))
    return out


def term_scale_rows(x, m, rows, G=1.0, eps=0.0):
    """|G| sum_{j != i} m_j / (|d_ij|^2 + eps^2) for each listed row i: an upper
    bound of the sum of the magnitudes of the row's terms (|d| <= |d|^2 + eps^2
    under the root), the scale of the condition-normalised force error."""
    m = _c(m)
    n = m.shape[0]
    x = _c(x, (3, n))
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(rows.size)
    _load().oracle_term_scale_rows(n, _p(x), _p(m), float(G), float(eps), rows.size,
                                   rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(out))
    return out


def accel_vjp_scale_rows(x, m, w, rows, G=1.0, eps=0.0):
    """Sums of the magnitudes of the terms of the listed rows of ``accel_vjp``:
    sx (len(rows),) of the 2-norms of the gx terms and sm (len(rows),) of the
    absolute gm terms; the scales of the condition-normalised VJP error."""
    m = _c(m)
    n = m.shape[0]
    x = _c(x, (3, n))
    w = _c(w, (3, n))
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= n):
        raise ValueError("row index out of range")
    sx = np.empty(rows.size)
    sm = np.empty(rows.size)
    _load().oracle_accel_vjp_scale_rows(n, _p(x), _p(m), _p(w), float(G), float(eps), rows.size,
                                        rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(sx), _p(sm))
    return sx, sm


def kdk(x, v, m, dt, nsteps, G=1.0, eps=0.0, trajectory=False):
    """Kick-drift-kick leapfrog; returns (x, v) or (x, v, traj (S+1, 3, N))."""
    m = _c(m)
    n = m.shape[0]
    x = _c(x, (3, n)).copy()
    v = _c(v, (3, n)).copy()
    traj = np.empty((int(nsteps) + 1, 3, n)) if trajectory else None
    _load().oracle_kdk(n, _p(x), _p(v), _p(m), float(G), float(eps), float(dt), int(nsteps),
                       _p(traj) if trajectory else ctypes.cast(None, _D))
    return (x, v, traj) if trajectory else (x, v)


ENERGY_FIELDS = ("K", "W", "E", "Px", "Py", "Pz", "Lx", "Ly", "Lz")


def energy(x, v, m, G=1.0, eps=0.0):
    """[K, W, E, Px, Py, Pz, Lx, Ly, Lz] with the self pair excluded from W."""
    m = _c(m)
    n = m.shape[0]
    x = _c(x, (3, n))
    v = _c(v, (3, n))
    out = np.empty(9)
    _load().oracle_energy(n, _p(x), _p(v), _p(m), float(G), float(eps), _p(out))
    return out


def accel_vjp(x, m, w, G=1.0, eps=0.0):
    """((da/dx)^T w, (da/dm)^T w) with shapes (3, N) and (N,)."""
    m = _c(m)
    n = m.shape[0]
    x = _c(x, (3, n))
    w = _c(w, (3, n))
    gx = np.empty((3, n))
    gm = np.empty(n)
    _load().oracle_accel_vjp(n, _p(x), _p(m), _p(w), float(G), float(eps), _p(gx), _p(gm))
    return gx, gm


def accel_vjp_rows(x, m, w, rows, G=1.0, eps=0.0):
    """The rows ``rows`` of ``accel_vjp`` only: gx (3, len(rows)), gm (len(rows),)."""
    m = _c(m)
    n = m.shape[0]
    x = _c(x, (3, n))
    w = _c(w, (3, n))
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= n):
        raise ValueError("row index out of range")
    gx = np.empty((3, rows.size))
    gm = np.empty(rows.size)
    _load().oracle_accel_vjp_rows(n, _p(x), _p(m), _p(w), float(G), float(eps), rows.size,
                                  rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(gx), _p(gm))
    return gx, gm


def accel_jvp(x, m, tx, tm, G=1.0, eps=0.0):
    """(da/dx) tx + (da/dm) tm, shape (3, N)."""
    m = _c(m)
    n = m.shape[0]
    x = _c(x, (3, n))
    tx = _c(tx, (3, n))
    tm = _c(tm, (n,))
    out = np.empty((3, n))
    _load().oracle_accel_jvp(n, _p(x), _p(m), _p(tx), _p(tm), float(G), float(eps), _p(out))
    return out


def kdk_adjoint(x0, v0, m, dt, nsteps, gxT, gvT, G=1.0, eps=0.0):
    """Cotangents (gx0, gv0, gm) of the initial state for final cotangents (gxT, gvT)."""
    m = _c(m)
    n = m.shape[0]
    x0 = _c(x0, (3, n))
    v0 = _c(v0, (3, n))
    gxT = _c(gxT, (3, n))
    gvT = _c(gvT, (3, n))
    gx0 = np.empty((3, n))
    gv0 = np.empty((3, n))
    gm = np.empty(n)
    _load().oracle_kdk_adjoint(n, _p(x0), _p(v0), _p(m), float(G), float(eps), float(dt),
                               int(nsteps), _p(gxT), _p(gvT), _p(gx0), _p(gv0), _p(gm))
    return gx0, gv0, gm


def accel_jerk(x, v, m, G=1.0, eps=0.0):
    """(a, jerk), each (3, N): App. A Algorithm 3 with softened r^2."""
    m = _c(m)
    n = m.shape[0]
    x = _c(x, (3, n))
    v = _c(v, (3, n))
    a = np.empty((3, n))
    jk = np.empty((3, n))
    _load().oracle_accel_jerk(n, _p(x), _p(v), _p(m), float(G), float(eps), _p(a), _p(jk))
    return a, jk


def accel_jerk_rows(x, v, m, rows, G=1.0, eps=0.0):
    """The listed rows of ``accel_jerk``, each (3, len(rows))."""
    m = _c(m)
    n = m.shape[0]
    x = _c(x, (3, n))
    v = _c(v, (3, n))
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    a = np.empty((3, rows.size))
    jk = np.empty((3, rows.size))
    _load().oracle_accel_jerk_rows(n, _p(x), _p(v), _p(m), float(G), float(eps), rows.size,
                                   rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(a), _p(jk))
    return a, jk


def hermite4(x, v, m, dt, nsteps, G=1.0, eps=0.0):
    """Fourth-order Hermite predictor-evaluator-corrector; returns (x, v)."""
    m = _c(m)
    n = m.shape[0]
    x = _c(x, (3, n)).copy()
    v = _c(v, (3, n)).copy()
    _load().oracle_hermite4(n, _p(x), _p(v), _p(m), float(G), float(eps), float(dt), int(nsteps))
    return x, v


def potential(x, m, G=1.0, eps=0.0):
    """phi_i = -G sum_{j != i} m_j / (|d_ij|^2 + eps^2)^(1/2), shape (N,)."""
    m = _c(m)
    n = m.shape[0]
    x = _c(x, (3, n))
    phi = np.empty(n)
    _load().oracle_potential(n, _p(x), _p(m), float(G), float(eps), _p(phi))
    return phi


def accel_jerk_snap(x, v, acc, m, G=1.0, eps=0.0):
    """(a, jerk, snap), each (3, N), along paths of constant acceleration acc."""
    m = _c(m)
    n = m.shape[0]
    x, v, acc = _c(x, (3, n)), _c(v, (3, n)), _c(acc, (3, n))
    a, jk, sn = np.empty((3, n)), np.empty((3, n)), np.empty((3, n))
    _load().oracle_accel_jerk_snap(n, _p(x), _p(v), _p(acc), _p(m), float(G), float(eps), _p(a), _p(jk), _p(sn))
    return a, jk, sn


def accel_jerk_snap_rows(x, v, acc, m, rows, G=1.0, eps=0.0):
    """The listed rows of ``accel_jerk_snap``, each (3, len(rows))."""
    m = _c(m)
    n = m.shape[0]
    x, v, acc = _c(x, (3, n)), _c(v, (3, n)), _c(acc, (3, n))
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= n):
        raise ValueError("row index out of range")
    a, jk, sn = (np.empty((3, rows.size)) for _ in range(3))
    _load().oracle_accel_jerk_snap_rows(n, _p(x), _p(v), _p(acc), _p(m), float(G), float(eps), rows.size,
                                        rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(a), _p(jk), _p(sn))
    return a, jk, sn


def hermite6_crackle(h, a0, j0, s0, a1, j1, s1):
    """Third derivative at t = h of the quintic through (a, jerk, snap) at 0 and h."""
    arrs = [_c(q) for q in (a0, j0, s0, a1, j1, s1)]
    out = np.empty_like(arrs[0])
    _load().oracle_hermite6_crackle(out.size, float(h), *[_p(q) for q in arrs], _p(out))
    return out


def hermite6(x, v, m, dt, nsteps, G=1.0, eps=0.0):
    """Sixth-order Hermite predictor-evaluator-corrector; returns (x, v)."""
    m = _c(m)
    n = m.shape[0]
    x = _c(x, (3, n)).copy()
    v = _c(v, (3, n)).copy()
    _load().oracle_hermite6(n, _p(x), _p(v), _p(m), float(G), float(eps), float(dt), int(nsteps))
    return x, v


def msd_loss(x, tgt):
    """(1/N) sum_i |x_i - tgt_i|^2."""
    x = _c(x)
    tgt = _c(tgt, x.shape)
    return _load().oracle_msd_loss(x.shape[1], _p(x), _p(tgt))


def loss_grad(x0, v0, m, tgt, dt, nsteps, G=1.0, eps=0.0):
    """Loss (1/N) sum |x_S - tgt|^2 after nsteps KDK steps and its gradient
    with respect to (x0, v0, m)."""
    n = np.asarray(m).shape[0]
    xS, _ = kdk(x0, v0, m, dt, nsteps, G=G, eps=eps)
    loss = msd_loss(xS, tgt)
    gxT = 2.0 * (xS - np.asarray(tgt)) / n
    gvT = np.zeros_like(gxT)
    return loss, kdk_adjoint(x0, v0, m, dt, nsteps, gxT, gvT, G=G, eps=eps)
