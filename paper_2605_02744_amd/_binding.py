"""ctypes binding of libnbody_accel.so (declared in include/nbody.h).

Argument marshalling only: every function checks its tensors (CUDA/HIP
device, float64, contiguous, expected shape), passes raw device pointers and
torch's current stream to the C entry point of the same name, and raises
NBodyError with the library's message on a non-zero status.  All arithmetic
runs in the library's HIP kernels; there is no fallback of any kind, and
importing a function fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnbody_accel.so")

NBODY_OK = 0
NBODY_EINVAL = -1
NBODY_EHIP = -2
NBODY_ENOMEM = -3
NBODY_ENONFINITE = -4
NBODY_EUNSUPPORTED = -5

NBODY_FP64 = 0
NBODY_FP32C = 1
NBODY_FP32 = 2
PRECISIONS = {"fp64": NBODY_FP64, "fp32c": NBODY_FP32C, "fp32": NBODY_FP32}

NBODY_EXCLUDE_SELF = 1
NBODY_CHECK_FINITE = 2
NBODY_ACC_VALID = 4


class NBodyError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("nbody status %d: %s" % (status, message))
        self.status = status


class nbody_params(ctypes.Structure):
    _fields_ = [("G", ctypes.c_double), ("eps", ctypes.c_double),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class nbody_config(ctypes.Structure):
    _fields_ = [("ipl", ctypes.c_int32), ("split", ctypes.c_int32),
                ("bsplit", ctypes.c_int32), ("bpass", ctypes.c_int32), ("bitem", ctypes.c_int32),
                ("pairs", ctypes.c_int32), ("rescue", ctypes.c_int32), ("sweep", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double


def load():
    """Loads the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libnbody_accel.so is not built at %s; run "
                          "`python -m paper_2605_02744_amd.build` (or __graft_entry__.build())" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    PP = ctypes.POINTER(nbody_params)
    lib.nbody_accel.argtypes = [_I64, _P, _P, _P, PP, _P]
    lib.nbody_accel_noalloc.argtypes = [_I64, _P, _P, _P, PP, _P]
    lib.nbody_step.argtypes = [_I64, _P, _P, _P, _P, _D, _I64, PP, _P]
    lib.nbody_energy.argtypes = [_I64, _P, _P, _P, PP, _P, _P]
    lib.nbody_accel_vjp.argtypes = [_I64, _P, _P, _P, _P, _P, PP, _P]
    lib.nbody_traj_grad.argtypes = [_I64, _P, _P, _I64, _I64, _P, _D, _P, _P, _P, _P, _P, PP, _P]
    lib.nbody_step_batched.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_double), _P, _P, _P, _P, _D, _I64, PP, _P]
    lib.nbody_accel_jerk.argtypes = [_I64, _P, _P, _P, _P, _P, PP, _P]
    lib.nbody_step_hermite.argtypes = [_I64, _P, _P, _P, _P, _P, _D, _I64, PP, _P]
    lib.nbody_potential.argtypes = [_I64, _P, _P, _P, PP, _P]
    lib.nbody_accel_jerk_snap.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, PP, _P]
    lib.nbody_step_hermite6.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _P, _D, _I64, PP, _P]
    lib.nbody_set_config.argtypes = [ctypes.POINTER(nbody_config)]
    lib.nbody_tune.argtypes = [_I64, ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(nbody_config)]
    lib.nbody_tune_batched.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                       _P, _P, _P, _D, _I64, ctypes.c_int32, PP, ctypes.POINTER(nbody_config)]
    lib.nbody_last_error.restype = ctypes.c_char_p
    lib.nbody_last_error.argtypes = []
    lib.nbody_finalize.argtypes = []
    lib.nbody_version.argtypes = []
    for f in ("nbody_accel", "nbody_accel_noalloc", "nbody_step", "nbody_energy", "nbody_accel_vjp", "nbody_traj_grad",
              "nbody_step_batched", "nbody_set_config", "nbody_tune", "nbody_finalize", "nbody_version",
              "nbody_accel_jerk", "nbody_step_hermite", "nbody_accel_jerk_snap", "nbody_step_hermite6",
              "nbody_potential", "nbody_tune_batched"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status):
    if status != NBODY_OK:
        raise NBodyError(status, load().nbody_last_error().decode(errors="replace"))


def _ptr(t, name, shape=None, dtype=torch.float64):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be on the GPU" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


def _params(G, eps, precision, flags):
    if isinstance(precision, str):
        precision = PRECISIONS[precision.lower()]
    return nbody_params(float(G), float(eps), int(precision), int(flags))


def _flags(exclude_self=False, check_finite=False, acc_valid=False):
    return ((NBODY_EXCLUDE_SELF if exclude_self else 0) | (NBODY_CHECK_FINITE if check_finite else 0)
            | (NBODY_ACC_VALID if acc_valid else 0))


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def nbody_accel(x, m, *, G=1.0, eps, precision="fp32c", exclude_self=False, check_finite=False, out=None):
    """Accelerations (3, N) of particles x (3, N) with masses m (N,)."""
    lib = load()
    n = m.shape[0]
    if out is None:
        out = torch.empty((3, n), dtype=torch.float64, device=x.device)
    p = _params(G, eps, precision, _flags(exclude_self, check_finite))
    with torch.cuda.device(x.device):
        _check(lib.nbody_accel(n, _ptr(x, "x", (3, n)), _ptr(m, "m", (n,)), _ptr(out, "a", (3, n)),
                               ctypes.byref(p), _stream(x.device)))
    return out


def nbody_accel_noalloc(x, m, *, G=1.0, eps, precision="fp32c", exclude_self=False, out=None):
    """nbody_accel with every scratch byte taken from the library's fixed
    per-GPU array (no allocation inside the call; N <= 2^21; calls on one GPU
    must not overlap).  Allocates `out` here only when it is not given."""
    lib = load()
    n = m.shape[0]
    if out is None:
        out = torch.empty((3, n), dtype=torch.float64, device=x.device)
    p = _params(G, eps, precision, _flags(exclude_self))
    with torch.cuda.device(x.device):
        _check(lib.nbody_accel_noalloc(n, _ptr(x, "x", (3, n)), _ptr(m, "m", (n,)), _ptr(out, "a", (3, n)),
                                       ctypes.byref(p), _stream(x.device)))
    return out


def nbody_step(x, v, a, m, dt, nsteps, *, G=1.0, eps, precision="fp32c", acc_valid=False,
               exclude_self=False, check_finite=False):
    """nsteps KDK steps in place on x, v, a (each (3, N)); a = a(x) on return."""
    lib = load()
    n = m.shape[0]
    p = _params(G, eps, precision, _flags(exclude_self, check_finite, acc_valid))
    with torch.cuda.device(x.device):
        _check(lib.nbody_step(n, _ptr(x, "x", (3, n)), _ptr(v, "v", (3, n)), _ptr(a, "a", (3, n)),
                              _ptr(m, "m", (n,)), float(dt), int(nsteps), ctypes.byref(p), _stream(x.device)))
    return x, v, a


ENERGY_FIELDS = ("K", "W", "E", "Px", "Py", "Pz", "Lx", "Ly", "Lz")


def nbody_energy(x, v, m, *, G=1.0, eps, check_finite=False, out=None):
    """Device tensor (9,) = [K, W, E, Px, Py, Pz, Lx, Ly, Lz] in FP64."""
    lib = load()
    n = m.shape[0]
    if out is None:
        out = torch.empty(9, dtype=torch.float64, device=x.device)
    p = _params(G, eps, NBODY_FP64, _flags(False, check_finite))
    with torch.cuda.device(x.device):
        _check(lib.nbody_energy(n, _ptr(x, "x", (3, n)), _ptr(v, "v", (3, n)), _ptr(m, "m", (n,)),
                                ctypes.byref(p), _ptr(out, "out9", (9,)), _stream(x.device)))
    return out


def nbody_accel_vjp(x, m, w, *, G=1.0, eps, precision="fp32c", exclude_self=False, check_finite=False):
    """((da/dx)^T w, (da/dm)^T w) for a cotangent w (3, N)."""
    lib = load()
    n = m.shape[0]
    gx = torch.empty((3, n), dtype=torch.float64, device=x.device)
    gm = torch.empty(n, dtype=torch.float64, device=x.device)
    p = _params(G, eps, precision, _flags(exclude_self, check_finite))
    with torch.cuda.device(x.device):
        _check(lib.nbody_accel_vjp(n, _ptr(x, "x", (3, n)), _ptr(m, "m", (n,)), _ptr(w, "w", (3, n)),
                                   _ptr(gx, "gx", (3, n)), _ptr(gm, "gm", (n,)), ctypes.byref(p),
                                   _stream(x.device)))
    return gx, gm


def nbody_traj_grad(ckpt_x, ckpt_v, every, nsteps, m, dt, gxT, gvT, *, G=1.0, eps, precision="fp32c",
                    exclude_self=False, check_finite=False):
    """Cotangents (gx0, gv0, gm) of the initial state of an nsteps KDK run from
    checkpoints ckpt_x, ckpt_v of shape (ceil(nsteps/every), 3, N)."""
    lib = load()
    n = m.shape[0]
    nck = max(1, -(-int(nsteps) // int(every)))
    gx0 = torch.empty((3, n), dtype=torch.float64, device=m.device)
    gv0 = torch.empty((3, n), dtype=torch.float64, device=m.device)
    gm = torch.empty(n, dtype=torch.float64, device=m.device)
    p = _params(G, eps, precision, _flags(exclude_self, check_finite))
    with torch.cuda.device(m.device):
        _check(lib.nbody_traj_grad(n, _ptr(ckpt_x, "ckpt_x", (nck, 3, n)), _ptr(ckpt_v, "ckpt_v", (nck, 3, n)),
                                   int(every), int(nsteps), _ptr(m, "m", (n,)), float(dt),
                                   _ptr(gxT, "gxT", (3, n)), _ptr(gvT, "gvT", (3, n)), _ptr(gx0, "gx0", (3, n)),
                                   _ptr(gv0, "gv0", (3, n)), _ptr(gm, "gm", (n,)), ctypes.byref(p),
                                   _stream(m.device)))
    return gx0, gv0, gm


def nbody_step_batched(off, eps, x, v, a, m, dt, nsteps, *, G=1.0, precision="fp32c", acc_valid=False,
                       exclude_self=False, check_finite=False):
    """nsteps KDK steps of every system of a concatenated ensemble, in place.
    off: host int64 sequence (ncl+1), eps: host float64 sequence (ncl)."""
    import numpy as np
    lib = load()
    off_h = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    eps_h = np.ascontiguousarray(np.asarray(eps, dtype=np.float64))
    ncl = eps_h.shape[0]
    if off_h.shape[0] != ncl + 1:
        raise ValueError("off must have ncl + 1 entries")
    total = int(off_h[-1])
    p = _params(G, 0.0, precision, _flags(exclude_self, check_finite, acc_valid))
    with torch.cuda.device(x.device):
        _check(lib.nbody_step_batched(ncl, off_h.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      eps_h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      _ptr(x, "x", (3, total)), _ptr(v, "v", (3, total)), _ptr(a, "a", (3, total)),
                                      _ptr(m, "m", (total,)), float(dt), int(nsteps), ctypes.byref(p),
                                      _stream(x.device)))
    return x, v, a


def nbody_tune_batched(off, eps, x, v, m, dt, nsteps, *, G=1.0, precision="fp32c", exclude_self=False,
                       allow_cooperative=True):
    """Times the batched kernels' configurations on copies of (x, v) for this
    layout, records the fastest for later nbody_step_batched calls, and
    returns it as {"bsplit", "bpass", "bitem"}.  allow_cooperative: False keeps
    to the modes that need no co-resident workgroups (0, 3, 4), True allows all,
    "persistent" keeps to the single-launch modes (0, 1, 2)."""
    import numpy as np
    lib = load()
    off_h = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    eps_h = np.ascontiguousarray(np.asarray(eps, dtype=np.float64))
    ncl = eps_h.shape[0]
    if off_h.shape[0] != ncl + 1:
        raise ValueError("off must have ncl + 1 entries")
    total = int(off_h[-1])
    p = _params(G, 0.0, precision, _flags(exclude_self, False))
    best = nbody_config()
    with torch.cuda.device(x.device):
        torch.cuda.current_stream(x.device).synchronize()
        _check(lib.nbody_tune_batched(ncl, off_h.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      eps_h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      _ptr(x, "x", (3, total)), _ptr(v, "v", (3, total)), _ptr(m, "m", (total,)),
                                      float(dt), int(nsteps),
                                      2 if allow_cooperative == "persistent" else (1 if allow_cooperative else 0),
                                      ctypes.byref(p),
                                      ctypes.byref(best)))
    return {"bsplit": best.bsplit, "bpass": best.bpass, "bitem": best.bitem}


def nbody_accel_jerk(x, v, m, *, G=1.0, eps, precision="fp32c", exclude_self=False, check_finite=False):
    """(a, jerk), each (3, N), of particles x, v (3, N) with masses m (N,)."""
    lib = load()
    n = m.shape[0]
    a = torch.empty((3, n), dtype=torch.float64, device=x.device)
    jk = torch.empty((3, n), dtype=torch.float64, device=x.device)
    p = _params(G, eps, precision, _flags(exclude_self, check_finite))
    with torch.cuda.device(x.device):
        _check(lib.nbody_accel_jerk(n, _ptr(x, "x", (3, n)), _ptr(v, "v", (3, n)), _ptr(m, "m", (n,)),
                                    _ptr(a, "a", (3, n)), _ptr(jk, "jk", (3, n)), ctypes.byref(p), _stream(x.device)))
    return a, jk


def nbody_step_hermite(x, v, a, jk, m, dt, nsteps, *, G=1.0, eps, precision="fp32c", acc_valid=False,
                       exclude_self=False, check_finite=False):
    """nsteps fourth-order Hermite steps in place on x, v, a, jk (each (3, N))."""
    lib = load()
    n = m.shape[0]
    p = _params(G, eps, precision, _flags(exclude_self, check_finite, acc_valid))
    with torch.cuda.device(x.device):
        _check(lib.nbody_step_hermite(n, _ptr(x, "x", (3, n)), _ptr(v, "v", (3, n)), _ptr(a, "a", (3, n)),
                                      _ptr(jk, "jk", (3, n)), _ptr(m, "m", (n,)), float(dt), int(nsteps),
                                      ctypes.byref(p), _stream(x.device)))
    return x, v, a, jk


def nbody_potential(x, m, *, G=1.0, eps, check_finite=False, out=None):
    """Device tensor (N,): phi_i = -G sum_{j != i} m_j / (|d_ij|^2 + eps^2)^(1/2), FP64."""
    lib = load()
    n = m.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=x.device)
    p = _params(G, eps, NBODY_FP64, _flags(False, check_finite))
    with torch.cuda.device(x.device):
        _check(lib.nbody_potential(n, _ptr(x, "x", (3, n)), _ptr(m, "m", (n,)), _ptr(out, "phi", (n,)),
                                   ctypes.byref(p), _stream(x.device)))
    return out


def nbody_accel_jerk_snap(x, v, acc, m, *, G=1.0, eps, precision="fp32c", exclude_self=False, check_finite=False):
    """(a, jerk, snap), each (3, N), of particles x, v moving with accelerations acc."""
    lib = load()
    n = m.shape[0]
    a, jk, sn = (torch.empty((3, n), dtype=torch.float64, device=x.device) for _ in range(3))
    p = _params(G, eps, precision, _flags(exclude_self, check_finite))
    with torch.cuda.device(x.device):
        _check(lib.nbody_accel_jerk_snap(n, _ptr(x, "x", (3, n)), _ptr(v, "v", (3, n)), _ptr(acc, "acc", (3, n)),
                                         _ptr(m, "m", (n,)), _ptr(a, "a", (3, n)), _ptr(jk, "jk", (3, n)),
                                         _ptr(sn, "sn", (3, n)), ctypes.byref(p), _stream(x.device)))
    return a, jk, sn


def nbody_step_hermite6(x, v, a, jk, sn, cr, m, dt, nsteps, *, G=1.0, eps, precision="fp32c", acc_valid=False,
                        exclude_self=False, check_finite=False):
    """nsteps sixth-order Hermite steps in place on x, v and the state a, jk, sn, cr (each (3, N))."""
    lib = load()
    n = m.shape[0]
    p = _params(G, eps, precision, _flags(exclude_self, check_finite, acc_valid))
    with torch.cuda.device(x.device):
        _check(lib.nbody_step_hermite6(n, _ptr(x, "x", (3, n)), _ptr(v, "v", (3, n)), _ptr(a, "a", (3, n)),
                                       _ptr(jk, "jk", (3, n)), _ptr(sn, "sn", (3, n)), _ptr(cr, "cr", (3, n)),
                                       _ptr(m, "m", (n,)), float(dt), int(nsteps), ctypes.byref(p),
                                       _stream(x.device)))


def nbody_set_config(ipl=0, split=0, bsplit=0, bpass=0, bitem=0, pairs=0, rescue=0, sweep=0):
    """Forces a tile configuration on this thread (all zeros = automatic).
    Ensemble (nbody_step_batched): bsplit=0 with bpass set runs one workgroup
    per system (its records resident in LDS), bsplit=1 as 0 with the largest
    systems split over up to 4 workgroups, bsplit=2 the streamed kernel
    (systems cut into items, one persistent launch), bsplit=3 its items of 64
    particles with two launches per step, bsplit=4 as 3 with each unordered pair
    of a system evaluated once (FP32C, FP32); all zero: the tuned choice for the
    layout, else mode 4 or 3.  bpass sets how many of a lane's i-particles the
    resident kernel evaluates per pass (1, 2, 4); bitem the streamed kernel's
    item size (64, the automatic choice: one wave per item; or 256, 512, 1024:
    one workgroup per item).  pairs: the form of the force kernels (1 ordered,
    2 symmetric: each unordered pair once; 0 automatic; the VJP follows in
    FP32C/FP32).  rescue: FP32C force rows flagged by the kernels' error
    estimate recomputed in FP64 (0 automatic = on, 1 on, 2 off).  sweep: the
    adjoint sweep of nbody_traj_grad (0 automatic: the next segment's
    trajectory recomputed on a second stream where that helps; 1 one stream;
    bitwise the same result)."""
    c = nbody_config(int(ipl), int(split), int(bsplit), int(bpass), int(bitem), int(pairs), int(rescue),
                     int(sweep))
    _check(load().nbody_set_config(ctypes.byref(c)))


def nbody_tune(n, precision="fp32c", cache_path=None):
    """Runs the force-kernel autotuner for (n, precision); returns the choice."""
    if isinstance(precision, str):
        precision = PRECISIONS[precision.lower()]
    best = nbody_config()
    path = cache_path.encode() if cache_path else None
    _check(load().nbody_tune(int(n), int(precision), path, ctypes.byref(best)))
    return {"ipl": best.ipl, "split": best.split, "pairs": best.pairs}


def nbody_last_error():
    return load().nbody_last_error().decode(errors="replace")


def nbody_finalize():
    _check(load().nbody_finalize())


def nbody_version():
    return load().nbody_version()
