"""Seeded synthetic initial conditions for direct-summation N-body runs.

This module only draws inputs; it holds none of the force, integrator, energy
or adjoint arithmetic, and it is shared by the FP64 oracle (``oracle/``) and
the GPU library alike.  Every array is float64; vectors are SoA with shape
(3, N) (row 0 = x, row 1 = y, row 2 = z), masses have shape (N,).

The paper states no initial-condition model (Sec. 4.2 gives only the particle
count), so the workloads use Plummer spheres in Henon units (G = M = 1), drawn
with the method of Aarseth, Henon & Wielen (1974, A&A 37, 183):

* radius from the cumulative mass fraction X1: r = a (X1^(-2/3) - 1)^(-1/2),
  with X1 > 0.999 rejected (r > 38.7 a) so the sample has no far outliers;
* isotropic direction from two more uniforms;
* speed q * v_esc, v_esc = sqrt(2 G M) (r^2 + a^2)^(-1/4), with q drawn by
  von Neumann rejection from g(q) = q^2 (1 - q^2)^(7/2) (0.1 bounds g);
* centre-of-mass position and velocity subtracted at the end.

Random streams are numpy ``Generator(PCG64(seed))``; ensembles spawn one
child ``SeedSequence`` per cluster.
"""
from __future__ import annotations

import math

import numpy as np

HENON_A = 3.0 * math.pi / 16.0   # Plummer scale radius giving E = -1/4 for G = M = 1
X1_MAX = 0.999                   # cumulative-mass cut for the radius draw


def _rng(seed):
    if isinstance(seed, np.random.SeedSequence):
        return np.random.Generator(np.random.PCG64(seed))
    return np.random.Generator(np.random.PCG64(int(seed)))


def _isotropic(rng, mag):
    """Unit vectors scaled by ``mag`` (shape (N,)), returned as (3, N)."""
    n = mag.shape[0]
    z = 1.0 - 2.0 * rng.random(n)
    phi = 2.0 * math.pi * rng.random(n)
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z]) * mag


def _plummer_radii(rng, n, a):
    r = np.empty(n)
    filled = 0
    while filled < n:
        x1 = rng.random(n - filled)
        x1 = x1[(x1 > 0.0) & (x1 <= X1_MAX)]
        take = x1[: n - filled]
        r[filled:filled + take.size] = a / np.sqrt(take ** (-2.0 / 3.0) - 1.0)
        filled += take.size
    return r


def _plummer_speed_fraction(rng, n):
    q = np.empty(n)
    filled = 0
    while filled < n:
        m = max(16, 2 * (n - filled))
        x4 = rng.random(m)
        x5 = rng.random(m)
        ok = 0.1 * x5 < x4 * x4 * (1.0 - x4 * x4) ** 3.5
        acc = x4[ok][: n - filled]
        q[filled:filled + acc.size] = acc
        filled += acc.size
    return q


def _remove_com(x, v, m):
    mt = m.sum()
    x -= (x * m).sum(axis=1, keepdims=True) / mt
    if v is not None:
        v -= (v * m).sum(axis=1, keepdims=True) / mt


def plummer(n, seed, a=HENON_A, total_mass=1.0, G=1.0, with_velocities=True):
    """Equal-mass Plummer sphere: returns (x (3,N), v (3,N), m (N,))."""
    n = int(n)
    if n <= 0:
        return np.zeros((3, 0)), np.zeros((3, 0)), np.zeros(0)
    rng = _rng(seed)
    r = _plummer_radii(rng, n, a)
    x = np.ascontiguousarray(_isotropic(rng, r))
    if with_velocities:
        vesc = math.sqrt(2.0 * G * total_mass) * (r * r + a * a) ** -0.25
        q = _plummer_speed_fraction(rng, n)
        v = np.ascontiguousarray(_isotropic(rng, q * vesc))
    else:
        v = np.zeros((3, n))
    m = np.full(n, total_mass / n)
    _remove_com(x, v, m)
    return x, v, m


def two_component(n, seed, core_frac=0.9, a_core=0.5, a_halo=3.0, mlo=0.1, mhi=10.0):
    """Two-component Plummer model used for the single large force evaluation.

    round(core_frac * n) particles follow a Plummer profile of radius a_core and
    the rest one of radius a_halo.  Masses are log-uniform in [mlo, mhi], then
    rescaled so the core holds core_frac of the unit total mass and the halo the
    rest.  Velocities are zero (only one force evaluation is made).
    """
    n = int(n)
    rng = _rng(seed)
    nc = int(round(core_frac * n))
    nh = n - nc
    r = np.concatenate([_plummer_radii(rng, nc, a_core), _plummer_radii(rng, nh, a_halo)])
    x = np.ascontiguousarray(_isotropic(rng, r))
    m = np.exp(rng.uniform(math.log(mlo), math.log(mhi), n))
    if nc:
        m[:nc] *= core_frac / m[:nc].sum()
    if nh:
        m[nc:] *= (1.0 - core_frac) / m[nc:].sum()
    v = np.zeros((3, n))
    _remove_com(x, None, m)
    return x, v, m


def ensemble_sizes(ncl, seed, nmin=64, nmax=4096):
    """Cluster sizes drawn uniformly from the integers [nmin, nmax]."""
    rng = _rng(seed)
    return rng.integers(nmin, nmax + 1, size=int(ncl)).astype(np.int64)


def ensemble_eps(sizes):
    """Per-cluster softening 0.04 / sqrt(N_c)."""
    return 0.04 / np.sqrt(np.asarray(sizes, dtype=np.float64))


def ensemble(ncl, seed, nmin=64, nmax=4096, sizes=None):
    """Independent Henon-unit Plummer clusters, concatenated.

    Returns (offsets (ncl+1,) int64, eps (ncl,), x (3,S), v (3,S), m (S,)), where
    cluster c occupies columns [offsets[c], offsets[c+1]).
    """
    if sizes is None:
        sizes = ensemble_sizes(ncl, seed, nmin, nmax)
    sizes = np.asarray(sizes, dtype=np.int64)
    off = np.zeros(sizes.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    children = np.random.SeedSequence(int(seed)).spawn(sizes.size)
    total = int(off[-1])
    x = np.empty((3, total))
    v = np.empty((3, total))
    m = np.empty(total)
    for c, nc in enumerate(sizes):
        xc, vc, mc = plummer(int(nc), children[c])
        s, e = off[c], off[c + 1]
        x[:, s:e] = xc
        v[:, s:e] = vc
        m[s:e] = mc
    return off, ensemble_eps(sizes), x, v, m


def perturb(x, v, sigma, seed):
    """Copies of (x, v) with i.i.d. N(0, sigma^2) added to every component."""
    rng = _rng(seed)
    return (x + sigma * rng.standard_normal(x.shape),
            v + sigma * rng.standard_normal(v.shape))


def random_cloud(n, seed, scale=1.0, mass_range=(0.5, 2.0)):
    """Small uniform-in-a-cube system with unequal masses, for unit tests."""
    rng = _rng(seed)
    x = scale * (2.0 * rng.random((3, int(n))) - 1.0)
    v = 0.3 * (2.0 * rng.random((3, int(n))) - 1.0)
    m = rng.uniform(mass_range[0], mass_range[1], int(n)) / max(int(n), 1)
    return np.ascontiguousarray(x), np.ascontiguousarray(v), m


# Named workloads (sizes, softening, steps) used by tests and the benchmark.
WORKLOADS = {
    "plummer1k_fp64": dict(n=1024, eps=0.01, steps=10, dt=1.0 / 128, seed=1),
    "plummer64k_fp32c": dict(n=65536, eps=0.005, steps=100, dt=1.0 / 256, seed=2),
    "twocomp1m_force": dict(n=1 << 20, eps=0.001, steps=0, dt=0.0, seed=3),
    "ensemble512": dict(ncl=512, nmin=64, nmax=4096, steps=1000, dt=1.0 / 512, seed=4),
    "grad16k": dict(n=16384, eps=0.01, steps=200, dt=1.0 / 256, seed=5, target_seed=55,
                    sigma=1e-3, every=20),
    # the paper's end-to-end run: N = 409600, three sixth-order Hermite steps,
    # softening 1e-7 (App. A); its initial conditions and step are not stated
    "hermite6_409600": dict(n=409600, eps=1e-7, steps=3, dt=1.0 / 1024, seed=7),
}


def plummer_mean_field(x, b=3.0 * np.pi / 16.0):
    """Acceleration of the smooth unit-mass Plummer potential, -x / (|x|^2 + b^2)^(3/2):
    a physically scaled acceleration field for snap evaluations."""
    r2 = (np.asarray(x) ** 2).sum(axis=0)
    return -np.asarray(x) / (r2 + b * b) ** 1.5
