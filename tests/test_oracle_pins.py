"""Pins of the FP64 oracle against facts it does not define itself.

Each test checks the oracle against something fixed by mathematics or physics
rather than by retyping the oracle's own formula:

* 50-digit mpmath brute force (tests/golden/tiny5_mp50.txt) for the
  acceleration, the pair potential and the vector-Jacobian product;
* the force as minus the gradient of the separately written potential W;
* Newton's third law (sum m_i a_i = 0);
* the analytic mean field of a Plummer sphere;
* the two-body Kepler solution and second-order convergence of KDK;
* conservation of momentum and angular momentum, time reversibility,
  O(dt^2) energy error, the virial theorem and E = -1/4 in Henon units;
* complex-step and central finite differences of an independent numpy
  forward model for the adjoint, and a forward/reverse dot-product test;
* for the sixth-order Hermite step: the 50-digit snap, central differences of
  the separately written jerk along the path, the crackle formula on exact
  quintics, sixth-order convergence on the Kepler problem and conservation.
"""
import math
import os

import numpy as np
import pytest

import ics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny5_mp50.txt")


def _read_golden():
    d = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *vals = line.split()
            d[k] = np.array([float(v) for v in vals])
    x = np.stack([d["x0"], d["x1"], d["x2"]])
    w = np.stack([d["w0"], d["w1"], d["w2"]])
    a = np.stack([d["a0"], d["a1"], d["a2"]])
    gx = np.stack([d["gx0"], d["gx1"], d["gx2"]])
    vel = np.stack([d["v0"], d["v1"], d["v2"]])
    jk = np.stack([d["j0"], d["j1"], d["j2"]])
    acc = np.stack([d["acc0"], d["acc1"], d["acc2"]])
    sn = np.stack([d["s0"], d["s1"], d["s2"]])
    return dict(x=x, m=d["m"], w=w, a=a, W=float(d["W"][0]), gx=gx, gm=d["gm"], v=vel, j=jk, acc=acc, s=sn,
                phi=d["phi"], G=float(d["G"][0]), eps=float(d["eps"][0]))


def test_golden_accel_mp50(oracle_mod):
    g = _read_golden()
    a = oracle_mod.accel(g["x"], g["m"], G=g["G"], eps=g["eps"])
    err = np.abs(a - g["a"]).max() / np.abs(g["a"]).max()
    assert err < 2e-16 * 8, err


def test_golden_potential_mp50(oracle_mod):
    g = _read_golden()
    e = oracle_mod.energy(g["x"], np.zeros_like(g["x"]), g["m"], G=g["G"], eps=g["eps"])
    assert abs(e[1] - g["W"]) <= 4e-16 * abs(g["W"])
    assert e[0] == 0.0 and e[2] == e[1]


def test_golden_vjp_mp50(oracle_mod):
    g = _read_golden()
    gx, gm = oracle_mod.accel_vjp(g["x"], g["m"], g["w"], G=g["G"], eps=g["eps"])
    assert np.abs(gx - g["gx"]).max() <= 1e-14 * np.abs(g["gx"]).max()
    assert np.abs(gm - g["gm"]).max() <= 1e-14 * np.abs(g["gm"]).max()


def test_mpmath_bruteforce_random(oracle_mod):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    x, _, m = ics.random_cloud(8, seed=11)
    eps = 0.05
    a = oracle_mod.accel(x, m, G=1.7, eps=eps)
    for i in range(8):
        acc = [mp.mpf(0)] * 3
        for j in range(8):
            if j == i:
                continue
            d = [mp.mpf(x[c, j]) - mp.mpf(x[c, i]) for c in range(3)]
            s = d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + mp.mpf(eps) ** 2
            for c in range(3):
                acc[c] += mp.mpf(1.7) * mp.mpf(m[j]) * d[c] / s ** mp.mpf(1.5)
        ref = np.array([float(v) for v in acc])
        assert np.abs(a[:, i] - ref).max() <= 4e-16 * np.abs(ref).max()


def test_accel_is_minus_grad_potential(oracle_mod):
    """m_i a_i = -dW/dx_i with W computed by the separately written potential."""
    x, v, m = ics.random_cloud(12, seed=3)
    eps, G = 0.1, 1.3
    a = oracle_mod.accel(x, m, G=G, eps=eps)
    h = 1e-5
    for c in range(3):
        for i in range(12):
            xp = x.copy(); xp[c, i] += h
            xm = x.copy(); xm[c, i] -= h
            dW = (oracle_mod.energy(xp, v, m, G, eps)[1] - oracle_mod.energy(xm, v, m, G, eps)[1]) / (2 * h)
            assert abs(m[i] * a[c, i] + dW) <= 1e-7 * (abs(dW) + 1e-3 * np.abs(m * a).max())


def test_newton_third_law(oracle_mod):
    x, _, m = ics.two_component(3000, seed=5)
    a = oracle_mod.accel(x, m, G=1.0, eps=0.001)
    tot = (a * m).sum(axis=1)
    scale = (np.abs(a) * m).sum()
    assert np.abs(tot).max() <= 1e-14 * scale


def test_two_body_closed_form(oracle_mod):
    """N = 2: |a_1| = G m_2 r / (r^2 + eps^2)^(3/2), directed towards body 2."""
    x = np.array([[0.3, -1.1], [0.2, 0.7], [-0.4, 0.1]])
    m = np.array([2.5, 0.75])
    eps, G = 0.3, 0.9
    a = oracle_mod.accel(x, m, G=G, eps=eps)
    d = x[:, 1] - x[:, 0]
    r = math.sqrt(float(d @ d))
    mag = G * m[1] * r / (r * r + eps * eps) ** 1.5
    np.testing.assert_allclose(np.linalg.norm(a[:, 0]), mag, rtol=1e-15)
    np.testing.assert_allclose(a[:, 0] / np.linalg.norm(a[:, 0]), d / r, rtol=1e-14)
    np.testing.assert_allclose(m[0] * a[:, 0], -m[1] * a[:, 1], rtol=1e-15)


def test_plummer_mean_field(oracle_mod):
    """Radial acceleration of a Plummer sample matches -G M r / (r^2 + a^2)^(3/2)."""
    n = 8192
    x, _, m = ics.plummer(n, seed=21)
    acc = oracle_mod.accel(x, m, G=1.0, eps=0.002)
    r = np.linalg.norm(x, axis=0)
    ar = (acc * x).sum(axis=0) / r
    a = ics.HENON_A
    model = -r / (r * r + a * a) ** 1.5
    edges = np.quantile(r, np.linspace(0.05, 0.9, 9))
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (r >= lo) & (r < hi)
        ratio = ar[sel].mean() / model[sel].mean()
        assert abs(ratio - 1.0) < 0.05, (lo, hi, ratio)


def _kepler_positions(m1, m2, a_sm, e, t, G=1.0):
    """Relative orbit from Kepler's equation, pericentre on +x at t = 0."""
    mu = G * (m1 + m2)
    n_mean = math.sqrt(mu / a_sm ** 3)
    M = n_mean * t
    E = M if e < 0.8 else math.pi
    for _ in range(60):
        E -= (E - e * math.sin(E) - M) / (1 - e * math.cos(E))
    rx = a_sm * (math.cos(E) - e)
    ry = a_sm * math.sqrt(1 - e * e) * math.sin(E)
    return np.array([rx, ry, 0.0])


def _kepler_ics(m1, m2, a_sm, e, G=1.0):
    mu = G * (m1 + m2)
    rp = a_sm * (1 - e)
    vp = math.sqrt(mu * (1 + e) / (a_sm * (1 - e)))
    rel_x = np.array([rp, 0.0, 0.0])
    rel_v = np.array([0.0, vp, 0.0])
    mt = m1 + m2
    x = np.stack([-m2 / mt * rel_x, m1 / mt * rel_x], axis=1)
    v = np.stack([-m2 / mt * rel_v, m1 / mt * rel_v], axis=1)
    return x, v, np.array([m1, m2])


def test_kepler_orbit_second_order(oracle_mod):
    m1, m2, a_sm, e = 0.7, 0.3, 1.0, 0.5
    x0, v0, m = _kepler_ics(m1, m2, a_sm, e)
    period = 2 * math.pi * math.sqrt(a_sm ** 3 / (m1 + m2))
    t_end = 0.8 * period
    errs = []
    for steps in (2000, 4000, 8000):
        dt = t_end / steps
        x, _ = oracle_mod.kdk(x0, v0, m, dt, steps, G=1.0, eps=0.0)
        rel = x[:, 1] - x[:, 0]
        errs.append(np.linalg.norm(rel - _kepler_positions(m1, m2, a_sm, e, t_end)))
    assert errs[-1] < 2e-4
    for coarse, fine in zip(errs[:-1], errs[1:]):
        assert 3.5 < coarse / fine < 4.5, errs


def test_momentum_and_angular_momentum_conserved(oracle_mod):
    x, v, m = ics.random_cloud(64, seed=8)
    e0 = oracle_mod.energy(x, v, m, 1.0, 0.05)
    x1, v1 = oracle_mod.kdk(x, v, m, 1e-3, 50, G=1.0, eps=0.05)
    e1 = oracle_mod.energy(x1, v1, m, 1.0, 0.05)
    pscale = (m * np.abs(v1).sum(axis=0)).sum()
    lscale = (m * np.linalg.norm(x1, axis=0) * np.linalg.norm(v1, axis=0)).sum()
    assert np.abs(e1[3:6] - e0[3:6]).max() <= 1e-14 * pscale
    assert np.abs(e1[6:9] - e0[6:9]).max() <= 1e-13 * lscale


def test_time_reversibility(oracle_mod):
    x, v, m = ics.plummer(128, seed=9)
    x1, v1 = oracle_mod.kdk(x, v, m, 1.0 / 256, 40, eps=0.05)
    x2, v2 = oracle_mod.kdk(x1, -v1, m, 1.0 / 256, 40, eps=0.05)
    assert np.abs(x2 - x).max() < 1e-12
    assert np.abs(v2 + v).max() < 1e-12


def test_energy_error_second_order(oracle_mod):
    """Leapfrog's energy error oscillates but its amplitude scales as dt^2: the
    largest error over common sample times drops about 4x when dt halves."""
    x, v, m = ics.plummer(256, seed=10)
    eps = 0.05
    e0 = oracle_mod.energy(x, v, m, 1.0, eps)[2]
    amps = []
    for dt in (1.0 / 64, 1.0 / 128):
        per = int(round((1.0 / 32) / dt))
        xs, vs, worst = x, v, 0.0
        for _ in range(16):
            xs, vs = oracle_mod.kdk(xs, vs, m, dt, per, eps=eps)
            worst = max(worst, abs(oracle_mod.energy(xs, vs, m, 1.0, eps)[2] - e0))
        amps.append(worst)
    assert 3.0 < amps[0] / amps[1] < 5.0, amps


def test_plummer_virial_and_energy(oracle_mod):
    x, v, m = ics.plummer(16384, seed=12)
    e = oracle_mod.energy(x, v, m, 1.0, 1e-4)
    assert abs(2 * e[0] / abs(e[1]) - 1.0) < 0.05
    assert abs(e[2] + 0.25) < 0.015


def test_accel_rows_match_full(oracle_mod):
    x, _, m = ics.plummer(700, seed=13)
    full = oracle_mod.accel(x, m, eps=0.01)
    rows = np.array([0, 5, 699, 350, 5])
    part = oracle_mod.accel_rows(x, m, rows, eps=0.01)
    assert np.array_equal(part, full[:, rows])


def test_exclude_self_eps_zero(oracle_mod):
    x, _, m = ics.random_cloud(10, seed=14)
    a = oracle_mod.accel(x, m, eps=0.0)
    assert np.isfinite(a).all()


def test_vjp_dot_product(oracle_mod):
    x, _, m = ics.random_cloud(24, seed=15)
    rng = np.random.default_rng(1)
    tx, tm, w = rng.standard_normal((3, 24)), rng.standard_normal(24), rng.standard_normal((3, 24))
    jv = oracle_mod.accel_jvp(x, m, tx, tm, G=1.1, eps=0.07)
    gx, gm = oracle_mod.accel_vjp(x, m, w, G=1.1, eps=0.07)
    lhs = float((jv * w).sum())
    rhs = float((tx * gx).sum() + (tm * gm).sum())
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + abs(rhs))


def test_vjp_rows_match_full(oracle_mod):
    """The sampled-row VJP is the same row computation as the full one."""
    x, _, m = ics.plummer(300, seed=18)
    w = np.random.default_rng(18).standard_normal((3, 300))
    gx, gm = oracle_mod.accel_vjp(x, m, w, G=0.9, eps=0.02)
    rows = np.array([0, 7, 150, 299, 42])
    rgx, rgm = oracle_mod.accel_vjp_rows(x, m, w, rows, G=0.9, eps=0.02)
    assert np.array_equal(rgx, gx[:, rows]) and np.array_equal(rgm, gm[rows])


def test_jvp_matches_central_difference(oracle_mod):
    x, _, m = ics.random_cloud(16, seed=16)
    rng = np.random.default_rng(2)
    tx, tm = rng.standard_normal((3, 16)), rng.standard_normal(16)
    h = 1e-6
    fd = (oracle_mod.accel(x + h * tx, m + h * tm, eps=0.1)
          - oracle_mod.accel(x - h * tx, m - h * tm, eps=0.1)) / (2 * h)
    jv = oracle_mod.accel_jvp(x, m, tx, tm, eps=0.1)
    assert np.abs(fd - jv).max() <= 1e-7 * np.abs(jv).max()


# ---- independent complex-capable numpy forward model for the adjoint pins ----

def _np_accel(x, m, eps, G):
    d = x[:, None, :] - x[:, :, None]              # d[c, i, j] = x_j - x_i
    s = (d * d).sum(axis=0) + eps * eps
    n = x.shape[1]
    s = s + np.eye(n)                               # keep the diagonal finite
    w = m[None, :] / (s * np.sqrt(s))
    w = w * (1 - np.eye(n))
    return G * (w[None] * d).sum(axis=2)


def _np_kdk_loss(x, v, m, tgt, dt, steps, eps, G):
    a = _np_accel(x, m, eps, G)
    for _ in range(steps):
        v = v + 0.5 * dt * a
        x = x + dt * v
        a = _np_accel(x, m, eps, G)
        v = v + 0.5 * dt * a
    d = x - tgt
    return (d * d).sum() / x.shape[1]


def test_kdk_adjoint_complex_step(oracle_mod):
    """Every component of the oracle's gradient against a complex-step derivative
    (Squire & Trapp 1998) of an independent numpy forward model."""
    n, steps, dt, eps, G = 6, 12, 1.0 / 64, 0.08, 1.0
    x, v, m = ics.random_cloud(n, seed=17)
    tgt = x + 0.05 * np.random.default_rng(3).standard_normal(x.shape)
    loss, (gx, gv, gm) = oracle_mod.loss_grad(x, v, m, tgt, dt, steps, G=G, eps=eps)
    assert abs(loss - _np_kdk_loss(x, v, m, tgt, dt, steps, eps, G)) <= 1e-13 * loss
    h = 1e-30
    for c in range(3):
        for i in range(n):
            xc = x.astype(complex); xc[c, i] += 1j * h
            vc = v.astype(complex); vc[c, i] += 1j * h
            np.testing.assert_allclose(gx[c, i], _np_kdk_loss(xc, v, m, tgt, dt, steps, eps, G).imag / h,
                                       rtol=1e-11, atol=1e-14)
            np.testing.assert_allclose(gv[c, i], _np_kdk_loss(x, vc, m, tgt, dt, steps, eps, G).imag / h,
                                       rtol=1e-11, atol=1e-14)
    for i in range(n):
        mc = m.astype(complex); mc[i] += 1j * h
        np.testing.assert_allclose(gm[i], _np_kdk_loss(x, v, mc, tgt, dt, steps, eps, G).imag / h,
                                   rtol=1e-11, atol=1e-14)


def test_kdk_adjoint_final_velocity_cotangent(oracle_mod):
    """A cotangent on the final velocities propagates like the complex step says."""
    n, steps, dt, eps = 5, 7, 1.0 / 32, 0.1
    x, v, m = ics.random_cloud(n, seed=18)
    wv = np.random.default_rng(4).standard_normal((3, n))
    _, gv0, gm = oracle_mod.kdk_adjoint(x, v, m, dt, steps, np.zeros((3, n)), wv, eps=eps)

    def final_v_dot(xc, vc, mc):
        a = _np_accel(xc, mc, eps, 1.0)
        for _ in range(steps):
            vc = vc + 0.5 * dt * a
            xc = xc + dt * vc
            a = _np_accel(xc, mc, eps, 1.0)
            vc = vc + 0.5 * dt * a
        return (vc * wv).sum()

    h = 1e-30
    for i in range(n):
        vc = v.astype(complex); vc[1, i] += 1j * h
        np.testing.assert_allclose(gv0[1, i], final_v_dot(x, vc, m).imag / h, rtol=1e-11, atol=1e-14)
        mc = m.astype(complex); mc[i] += 1j * h
        np.testing.assert_allclose(gm[i], final_v_dot(x, v, mc).imag / h, rtol=1e-11, atol=1e-14)


def test_kdk_adjoint_central_difference(oracle_mod):
    """A Plummer-sampled system, gradient against central differences h = 1e-6."""
    n, steps, dt, eps = 64, 20, 1.0 / 256, 0.01
    x, v, m = ics.plummer(n, seed=19)
    tgt, _ = ics.perturb(x, v, 1e-3, seed=20)
    _, (gx, gv, gm) = oracle_mod.loss_grad(x, v, m, tgt, dt, steps, eps=eps)
    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(6):
        c, i = int(rng.integers(3)), int(rng.integers(n))
        for arr, g in ((x, gx), (v, gv)):
            p = arr.copy(); p[c, i] += h
            q = arr.copy(); q[c, i] -= h
            if arr is x:
                lp = oracle_mod.msd_loss(oracle_mod.kdk(p, v, m, dt, steps, eps=eps)[0], tgt)
                lq = oracle_mod.msd_loss(oracle_mod.kdk(q, v, m, dt, steps, eps=eps)[0], tgt)
            else:
                lp = oracle_mod.msd_loss(oracle_mod.kdk(x, p, m, dt, steps, eps=eps)[0], tgt)
                lq = oracle_mod.msd_loss(oracle_mod.kdk(x, q, m, dt, steps, eps=eps)[0], tgt)
            fd = (lp - lq) / (2 * h)
            assert abs(fd - g[c, i]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max())


# ---- acceleration + jerk (App. A, Algorithm 3) and the Hermite integrator ----

def test_golden_jerk_mp50(oracle_mod):
    g = _read_golden()
    a, jk = oracle_mod.accel_jerk(g["x"], g["v"], g["m"], G=g["G"], eps=g["eps"])
    assert np.abs(a - g["a"]).max() <= 2e-15 * np.abs(g["a"]).max()
    assert np.abs(jk - g["j"]).max() <= 2e-15 * np.abs(g["j"]).max()


def test_jerk_is_time_derivative_of_accel(oracle_mod):
    """jerk_i = d/dt a_i(x + v t) at t = 0, by central differences of the
    separately written acceleration routine."""
    x, v, m = ics.plummer(200, seed=40)
    eps = 0.02
    _, jk = oracle_mod.accel_jerk(x, v, m, G=1.3, eps=eps)
    h = 1e-6
    fd = (oracle_mod.accel(x + h * v, m, G=1.3, eps=eps) - oracle_mod.accel(x - h * v, m, G=1.3, eps=eps)) / (2 * h)
    assert np.abs(fd - jk).max() <= 2e-8 * np.abs(jk).max()


def test_jerk_total_is_zero_momentum_rate(oracle_mod):
    """sum_i m_i jerk_i = d/dt sum_i m_i a_i = 0 (pairwise antisymmetry)."""
    x, v, m = ics.random_cloud(300, seed=41)
    _, jk = oracle_mod.accel_jerk(x, v, m, eps=0.05)
    assert np.abs((jk * m).sum(axis=1)).max() <= 1e-14 * (np.abs(jk) * m).sum()


def test_jerk_rows_equal_full_evaluation(oracle_mod):
    """The rows variant computes each listed row exactly as the pinned full
    evaluation does (bitwise), in any order and with repeats."""
    x, v, m = ics.random_cloud(257, seed=43)
    a, jk = oracle_mod.accel_jerk(x, v, m, G=0.8, eps=0.03)
    rows = np.array([256, 0, 17, 17, 131, 5])
    ar, jr = oracle_mod.accel_jerk_rows(x, v, m, rows, G=0.8, eps=0.03)
    assert np.array_equal(ar, a[:, rows]) and np.array_equal(jr, jk[:, rows])


def test_hermite4_kepler_fourth_order(oracle_mod):
    m1, m2, a_sm, e = 0.7, 0.3, 1.0, 0.5
    x0, v0, m = _kepler_ics(m1, m2, a_sm, e)
    period = 2 * math.pi * math.sqrt(a_sm ** 3 / (m1 + m2))
    t_end = 0.8 * period
    errs = []
    for steps in (400, 800, 1600):
        x, _ = oracle_mod.hermite4(x0, v0, m, t_end / steps, steps, eps=0.0)
        errs.append(np.linalg.norm(x[:, 1] - x[:, 0] - _kepler_positions(m1, m2, a_sm, e, t_end)))
    assert errs[-1] < 1e-6
    for coarse, fine in zip(errs[:-1], errs[1:]):
        assert 12.0 < coarse / fine < 20.0, errs


def test_hermite4_conserves_momentum_and_energy(oracle_mod):
    x, v, m = ics.plummer(128, seed=42)
    eps = 0.05
    e0 = oracle_mod.energy(x, v, m, 1.0, eps)
    x1, v1 = oracle_mod.hermite4(x, v, m, 1.0 / 256, 64, eps=eps)
    e1 = oracle_mod.energy(x1, v1, m, 1.0, eps)
    pscale = (m * np.abs(v1).sum(axis=0)).sum()
    assert np.abs(e1[3:6] - e0[3:6]).max() <= 1e-13 * pscale
    assert abs(e1[2] - e0[2]) <= 1e-7 * abs(e0[2])


def test_golden_snap_mp50(oracle_mod):
    g = _read_golden()
    a, jk, sn = oracle_mod.accel_jerk_snap(g["x"], g["v"], g["acc"], g["m"], G=g["G"], eps=g["eps"])
    assert np.abs(a - g["a"]).max() <= 2e-15 * np.abs(g["a"]).max()
    assert np.abs(jk - g["j"]).max() <= 1e-14 * np.abs(g["j"]).max()
    assert np.abs(sn - g["s"]).max() <= 1e-14 * np.abs(g["s"]).max()


def test_snap_is_time_derivative_of_jerk(oracle_mod):
    """snap_i = d/dt jerk_i along x + v t + acc t^2/2 (velocity v + acc t), by
    central differences of the separately written Algorithm-3 routine, for an
    arbitrary acceleration field acc."""
    x, v, m = ics.plummer(200, seed=43)
    eps = 0.02
    acc = np.random.default_rng(44).standard_normal((3, 200))
    _, _, sn = oracle_mod.accel_jerk_snap(x, v, acc, m, G=1.3, eps=eps)
    h = 2e-6

    def jerk_at(t):
        return oracle_mod.accel_jerk(x + v * t + acc * (t * t / 2), v + acc * t, m, G=1.3, eps=eps)[1]
    fd = (jerk_at(h) - jerk_at(-h)) / (2 * h)
    assert np.abs(fd - sn).max() <= 5e-8 * np.abs(sn).max()


def test_snap_total_is_zero(oracle_mod):
    """sum_i m_i snap_i = d^2/dt^2 sum_i m_i a_i = 0 (pairwise antisymmetry)."""
    x, v, m = ics.random_cloud(300, seed=45)
    acc = np.random.default_rng(46).standard_normal((3, 300))
    _, _, sn = oracle_mod.accel_jerk_snap(x, v, acc, m, eps=0.05)
    assert np.abs((sn * m).sum(axis=1)).max() <= 1e-14 * (np.abs(sn) * m).sum()


def test_hermite6_crackle_exact_on_quintics(oracle_mod):
    """The crackle estimate is the third derivative at t = h of the quintic
    matching value, first and second derivative at both ends: exact when the
    acceleration history is itself a quintic."""
    rng = np.random.default_rng(47)
    h = 0.37
    k = rng.standard_normal((6, 50))           # q(t) = sum_p k_p t^p, 50 independent series

    def der(t, order):
        out = np.zeros(50)
        for p in range(order, 6):
            out += k[p] * math.factorial(p) / math.factorial(p - order) * t ** (p - order)
        return out
    c1 = oracle_mod.hermite6_crackle(h, der(0, 0), der(0, 1), der(0, 2), der(h, 0), der(h, 1), der(h, 2))
    assert np.abs(c1 - der(h, 3)).max() <= 1e-11 * np.abs(der(h, 3)).max()


def test_hermite6_kepler_sixth_order(oracle_mod):
    m1, m2, a_sm, e = 0.7, 0.3, 1.0, 0.5
    x0, v0, m = _kepler_ics(m1, m2, a_sm, e)
    period = 2 * math.pi * math.sqrt(a_sm ** 3 / (m1 + m2))
    t_end = 0.8 * period
    errs = []
    for steps in (100, 200, 400):
        x, _ = oracle_mod.hermite6(x0, v0, m, t_end / steps, steps, eps=0.0)
        errs.append(np.linalg.norm(x[:, 1] - x[:, 0] - _kepler_positions(m1, m2, a_sm, e, t_end)))
    assert errs[-1] < 1e-8
    for coarse, fine in zip(errs[:-1], errs[1:]):
        assert 50.0 < coarse / fine < 80.0, errs


def test_hermite6_conserves_momentum_and_energy(oracle_mod):
    x, v, m = ics.plummer(128, seed=42)
    eps = 0.05
    e0 = oracle_mod.energy(x, v, m, 1.0, eps)
    x1, v1 = oracle_mod.hermite6(x, v, m, 1.0 / 256, 64, eps=eps)
    e1 = oracle_mod.energy(x1, v1, m, 1.0, eps)
    pscale = (m * np.abs(v1).sum(axis=0)).sum()
    assert np.abs(e1[3:6] - e0[3:6]).max() <= 1e-13 * pscale
    assert abs(e1[2] - e0[2]) <= 1e-9 * abs(e0[2])
    # the fourth-order scheme lands within its own (larger) error of the same point
    x4, _ = oracle_mod.hermite4(x, v, m, 1.0 / 256, 64, eps=eps)
    x4f, _ = oracle_mod.hermite4(x, v, m, 1.0 / 512, 128, eps=eps)
    assert np.abs(x1 - x4f).max() < np.abs(x4 - x4f).max()


def test_golden_potential_per_particle_mp50(oracle_mod):
    g = _read_golden()
    phi = oracle_mod.potential(g["x"], g["m"], G=g["G"], eps=g["eps"])
    assert np.abs(phi - g["phi"]).max() <= 4e-16 * np.abs(g["phi"]).max()


def test_potential_sums_to_twice_the_pair_energy(oracle_mod):
    """sum_i m_i phi_i counts every pair twice: 2 W of the separately written
    pair sum over i < j."""
    x, v, m = ics.random_cloud(400, seed=81)
    phi = oracle_mod.potential(x, m, G=1.2, eps=0.03)
    W = oracle_mod.energy(x, v, m, 1.2, 0.03)[1]
    assert abs((m * phi).sum() - 2 * W) <= 1e-13 * abs(W)


def test_potential_plummer_mean_field(oracle_mod):
    """For a Plummer sample, phi_i follows the smooth potential -1/(r^2 + b^2)^(1/2)
    (b = 3 pi / 16, unit mass) up to sampling noise."""
    x, _, m = ics.plummer(8192, seed=82)
    phi = oracle_mod.potential(x, m, eps=0.01)
    r2 = (x ** 2).sum(axis=0)
    ref = -1.0 / np.sqrt(r2 + (3 * np.pi / 16) ** 2)
    rel = np.abs(phi - ref) / np.abs(ref)
    assert np.median(rel) < 0.01 and np.quantile(rel, 0.99) < 0.05


def test_potential_gradient_is_minus_acceleration(oracle_mod):
    """grad_i phi_i with the other particles held fixed is -a_i (central differences)."""
    x, _, m = ics.random_cloud(50, seed=83)
    a = oracle_mod.accel(x, m, eps=0.05)
    h = 1e-6
    for i in (0, 17, 49):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[c, i] += h
            xm[c, i] -= h
            d = (oracle_mod.potential(xp, m, eps=0.05)[i] - oracle_mod.potential(xm, m, eps=0.05)[i]) / (2 * h)
            assert abs(d + a[c, i]) <= 1e-7 * np.abs(a[:, i]).max()


# ---- term scales (the denominators of the condition-normalised errors) -----

def test_term_scale_two_body_and_collinear(oracle_mod):
    """N = 2: |G| m_2 / (r^2 + eps^2) in closed form.  All partners on one ray
    from particle 0 with eps = 0: every term points the same way and has
    magnitude G m_j / r_j^2, so the separately pinned acceleration reaches
    the scale exactly; elsewhere it stays below it."""
    x = np.array([[0.1, 0.4], [0.2, -0.1], [-0.3, 0.5]])
    m = np.array([0.7, 1.9])
    r2 = ((x[:, 1] - x[:, 0]) ** 2).sum()
    s = oracle_mod.term_scale_rows(x, m, [0, 1], G=1.3, eps=0.1)
    assert np.allclose(s, [1.3 * 1.9 / (r2 + 0.01), 1.3 * 0.7 / (r2 + 0.01)], rtol=1e-15)
    rng = np.random.default_rng(3)
    r = np.concatenate([[0.0], rng.uniform(0.1, 3.0, 20)])
    xr = np.outer(np.array([2.0, -1.0, 0.5]) / np.linalg.norm([2.0, -1.0, 0.5]), r)
    mr = rng.uniform(0.5, 2.0, 21)
    a0 = oracle_mod.accel_rows(xr, mr, [0], G=0.9, eps=0.0)
    s0 = oracle_mod.term_scale_rows(xr, mr, [0], G=0.9, eps=0.0)[0]
    assert abs(np.linalg.norm(a0) - s0) <= 1e-14 * s0
    xp, _, mp = ics.plummer(300, seed=4)
    rows = np.arange(300)
    sp = oracle_mod.term_scale_rows(xp, mp, rows, eps=0.01)
    ap = oracle_mod.accel(xp, mp, eps=0.01)
    assert (np.linalg.norm(ap, axis=0) <= sp * (1 + 1e-14)).all()


def test_vjp_scale_two_body_aligned_and_bound(oracle_mod):
    """The VJP term scales against the separately pinned VJP: equal to |gx_k|
    and |gm_k| when a row has one term (N = 2) or when all its terms are
    parallel (partners on one ray with eps = 0, cotangents along that ray and
    none on the row itself), and never below them otherwise; linear in w and
    in a common scale of the masses (for gx)."""
    x = np.array([[0.1, 0.4], [0.2, -0.1], [-0.3, 0.5]])
    m = np.array([0.7, 1.9])
    w = np.array([[0.3, -1.2], [2.0, 0.4], [-0.5, 0.9]])
    gx, gm = oracle_mod.accel_vjp(x, m, w, G=-0.8, eps=0.05)
    sx, sm = oracle_mod.accel_vjp_scale_rows(x, m, w, [0, 1], G=-0.8, eps=0.05)
    assert np.allclose(sx, np.linalg.norm(gx, axis=0), rtol=1e-14)
    assert np.allclose(sm, np.abs(gm), rtol=1e-14)
    rng = np.random.default_rng(5)
    e = np.array([1.0, 2.0, -2.0]) / 3.0
    r = np.concatenate([[0.0], rng.uniform(0.2, 2.0, 15)])
    xr = np.outer(e, r)
    mr = rng.uniform(0.5, 2.0, 16)
    wr = np.outer(e, np.concatenate([[0.0], rng.uniform(0.1, 1.0, 15)]))
    gx, gm = oracle_mod.accel_vjp(xr, mr, wr, eps=0.0)
    sx, sm = oracle_mod.accel_vjp_scale_rows(xr, mr, wr, [0], eps=0.0)
    assert abs(np.linalg.norm(gx[:, 0]) - sx[0]) <= 1e-14 * sx[0]
    assert abs(abs(gm[0]) - sm[0]) <= 1e-14 * sm[0]
    xp, _, mp = ics.two_component(400, seed=6)
    wp = rng.standard_normal((3, 400))
    rows = np.arange(400)
    gx, gm = oracle_mod.accel_vjp(xp, mp, wp, G=0.7, eps=0.02)
    sx, sm = oracle_mod.accel_vjp_scale_rows(xp, mp, wp, rows, G=0.7, eps=0.02)
    assert (np.linalg.norm(gx, axis=0) <= sx * (1 + 1e-14)).all() and (np.abs(gm) <= sm * (1 + 1e-14)).all()
    sx2, sm2 = oracle_mod.accel_vjp_scale_rows(xp, 3.0 * mp, -2.0 * wp, rows, G=0.7, eps=0.02)
    assert np.allclose(sx2, 6.0 * sx, rtol=1e-13) and np.allclose(sm2, 2.0 * sm, rtol=1e-13)
