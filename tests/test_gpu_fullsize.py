"""Parity at the workloads' full sizes, in the launch configuration the
benchmark uses, on outputs the oracle can compute one by one:

* N = 2^20 two-component force (eps = 0.001): FP32C and FP64 on every row
  against the ordered FP64 kernel (max gated), and on sampled, worst and
  central rows against the oracle; the FP32C VJP per row (condition-
  normalised) against the oracle on sampled rows and on the rows where it
  differs most from the ordered FP64 VJP, both FP64 VJP forms on the same rows;
* N = 2^20 Plummer acceleration + jerk (eps = 0.001): the symmetric FP32C and
  FP64 kernels and the ordered FP64 kernel against the oracle on sampled rows
  and on the rows where FP32C differs most from the ordered FP64 kernel;
* N = 65536 Plummer force (eps = 0.005): every row against the ordered FP64
  kernel at t = 0 and after 100 FP32C KDK steps, with the energy drift;
* 512-cluster ensemble, every batched mode: sampled clusters against the
  oracle's own KDK, and their final accelerations per row;
* N = 16384 adjoint: the 200-step gradients (FP64, the library's FP32C form
  and the all-FP32C form) per coordinate against central finite differences
  (h = 1e-6) of the FP64 GPU forward on 64 random coordinates, and a shorter
  run against the oracle's full adjoint;
* N = 409600 sixth-order Hermite (eps = 1e-7): acceleration, jerk and snap on
  sampled rows against the oracle, and three FP32C steps against three FP64
  steps of the GPU path.
"""
import numpy as np
import pytest

import ics
from parity_stats import coord_err, cond_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_02744_amd as nbm
    nbm.load()
    return nbm


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def row_err(a, ref):
    return np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)


def ordered(nb, fn, *args, **kw):
    """fn with the ordered kernels forced (pairs = 1): every ordered pair for
    its i, code that shares nothing with the symmetric kernels' ring, slots and
    slot sums, and an FP64 path that is checked against the oracle itself."""
    nb.nbody_set_config(pairs=1)
    try:
        return fn(*args, **kw)
    finally:
        nb.nbody_set_config()


def test_twocomp1m_all_rows(nb, oracle_mod):
    """N = 2^20 two-component force in the benchmark's configuration (the
    symmetric kernels), FP32C and FP64: every row against the ordered FP64
    kernel, gated on the maximum (1e-5 FP32C, 1e-12 FP64); the ordered FP64
    kernel and both symmetric paths against the oracle on sampled rows, on
    the rows where FP32C is worst and on the rows closest to the centre."""
    w = ics.WORKLOADS["twocomp1m_force"]
    n, eps = w["n"], w["eps"]
    x, _, m = ics.two_component(n, seed=w["seed"])
    tx, tm = dev(x), dev(m)
    a64 = nb.nbody_accel(tx, tm, eps=eps, precision="fp64").cpu().numpy()
    a32 = nb.nbody_accel(tx, tm, eps=eps, precision="fp32c").cpu().numpy()
    o64 = ordered(nb, nb.nbody_accel, tx, tm, eps=eps, precision="fp64").cpu().numpy()
    e_all = row_err(a32, o64)
    e64_all = row_err(a64, o64)
    print("N=2^20 all rows vs ordered FP64: fp32c max %.3e p99.9 %.3e p99 %.3e; fp64 (symmetric) max %.3e"
          % (e_all.max(), np.quantile(e_all, 0.999), np.quantile(e_all, 0.99), e64_all.max()))
    assert e_all.max() <= 1e-5
    assert e64_all.max() <= 1e-12
    rng = np.random.default_rng(0)
    rows = np.concatenate([[0, n - 1], rng.choice(n, 96, replace=False), np.argsort(e_all)[-32:],
                           np.argsort(np.linalg.norm(x, axis=0))[:16]])
    rows = np.unique(rows)
    ref = oracle_mod.accel_rows(x, m, rows, eps=eps)
    scale = oracle_mod.term_scale_rows(x, m, rows, eps=eps)
    checks = {"fp64 ordered": (o64, 1e-12), "fp64 symmetric": (a64, 1e-12), "fp32c symmetric": (a32, 1e-5)}
    for name, (a, tol) in checks.items():
        e = row_err(a[:, rows], ref)
        c = cond_err(a[:, rows], ref, scale)
        print("  %s vs oracle on %d rows: max rel %.3e, max condition-normalised %.3e" % (name, rows.size, e.max(), c.max()))
        assert e.max() <= tol, name


def test_twocomp1m_vjp(nb, oracle_mod):
    """The FP32C VJP at N = 2^20 in the benchmark's configuration (the
    symmetric kernel): per-row condition-normalised error against the oracle
    on sampled rows and on the rows that differ most from the ordered FP64
    VJP (pairs = 1: no code shared with the symmetric ring), which is itself
    checked against the oracle on the same rows, as is the symmetric FP64 VJP
    (the FP64 default at this size)."""
    w_ = ics.WORKLOADS["twocomp1m_force"]
    n, eps = w_["n"], w_["eps"]
    x, _, m = ics.two_component(n, seed=w_["seed"])
    w = np.random.default_rng(1).standard_normal((3, n))
    tx, tm, tw = dev(x), dev(m), dev(w)
    gx, gm = nb.nbody_accel_vjp(tx, tm, tw, eps=eps, precision="fp32c")
    sx64, sm64 = nb.nbody_accel_vjp(tx, tm, tw, eps=eps, precision="fp64")
    nb.nbody_set_config(pairs=1)
    try:
        gx64, gm64 = nb.nbody_accel_vjp(tx, tm, tw, eps=eps, precision="fp64")
    finally:
        nb.nbody_set_config()
    gx, gm, gx64, gm64 = gx.cpu().numpy(), gm.cpu().numpy(), gx64.cpu().numpy(), gm64.cpu().numpy()
    sx64, sm64 = sx64.cpu().numpy(), sm64.cpu().numpy()
    dx = np.linalg.norm(gx - gx64, axis=0)
    dm = np.abs(gm - gm64)
    worst = np.concatenate([np.argsort(dx)[-48:], np.argsort(dx / np.linalg.norm(gx64, axis=0))[-48:],
                            np.argsort(dm)[-48:], np.argsort(dm / np.abs(gm64))[-48:]])
    rows = np.unique(np.concatenate([np.random.default_rng(12).choice(n, 96, replace=False), worst]))
    rgx, rgm = oracle_mod.accel_vjp_rows(x, m, w, rows, eps=eps)
    sx, sm = oracle_mod.accel_vjp_scale_rows(x, m, w, rows, eps=eps)
    for name, (a, b, tol) in {"fp32c": (gx, gm, 2e-5), "fp64 ordered": (gx64, gm64, 1e-13),
                              "fp64 symmetric": (sx64, sm64, 1e-13)}.items():
        cx = cond_err(a[:, rows], rgx, sx)
        cm = cond_err(b[rows], rgm, sm)
        print("vjp 2^20 %s vs oracle on %d rows: condition-normalised gx %.2e gm %.2e; rel gx %.2e gm %.2e"
              % (name, rows.size, cx.max(), cm.max(), row_err(a[:, rows], rgx).max(),
                 (np.abs(b[rows] - rgm) / np.abs(rgm)).max()))
        assert cx.max() <= tol and cm.max() <= tol, name


def test_jerk1m_sampled_rows(nb, oracle_mod):
    """Acceleration + jerk at N = 2^20 in the benchmark's configuration
    (Plummer, eps = 0.001): the symmetric FP32C and FP64 kernels (the defaults
    at this size) against the oracle on sampled rows and on the rows where the
    FP32C jerk differs most from the ordered FP64 kernel's (pairs = 1).  FP32C:
    acceleration within 1e-5 per row, jerk within the paper's 0.2 % per
    component (Sec. 4.1); FP64: 1e-12 and 1e-11 per row."""
    n, eps = 1 << 20, 0.001
    x, v, m = ics.plummer(n, seed=6)
    tx, tv, tm = dev(x), dev(v), dev(m)
    a32, j32 = [q.cpu().numpy() for q in nb.nbody_accel_jerk(tx, tv, tm, eps=eps, precision="fp32c")]
    a64, j64 = [q.cpu().numpy() for q in nb.nbody_accel_jerk(tx, tv, tm, eps=eps, precision="fp64")]
    nb.nbody_set_config(pairs=1)
    try:
        o64, oj64 = [q.cpu().numpy() for q in nb.nbody_accel_jerk(tx, tv, tm, eps=eps, precision="fp64")]
    finally:
        nb.nbody_set_config()
    dj = np.linalg.norm(j32 - oj64, axis=0) / np.linalg.norm(oj64, axis=0)
    da = np.linalg.norm(a32 - o64, axis=0) / np.linalg.norm(o64, axis=0)
    rows = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(6).choice(n, 96, replace=False),
                                     np.argsort(dj)[-32:], np.argsort(da)[-32:]]))
    ra, rj = oracle_mod.accel_jerk_rows(x, v, m, rows, eps=eps)
    for name, (a, jk, tola, tolj) in {"fp32c": (a32, j32, 1e-5, 2e-3), "fp64 symmetric": (a64, j64, 1e-12, 1e-11),
                                      "fp64 ordered": (o64, oj64, 1e-12, 1e-11)}.items():
        ea, ej = row_err(a[:, rows], ra), row_err(jk[:, rows], rj)
        print("jerk 2^20 %s vs oracle on %d rows: a %.2e jerk %.2e" % (name, rows.size, ea.max(), ej.max()))
        assert ea.max() <= tola and ej.max() <= tolj, name
    assert np.all(np.abs(j32[:, rows] - rj) <= 2e-3 * np.abs(rj) + 1e-6 * np.abs(rj).max())


def test_plummer64k_force_and_drift(nb, oracle_mod):
    w = ics.WORKLOADS["plummer64k_fp32c"]
    n, eps, dt = w["n"], w["eps"], w["dt"]
    x, v, m = ics.plummer(n, seed=w["seed"])
    rows = np.sort(np.random.default_rng(1).choice(n, 128, replace=False))
    ref = oracle_mod.accel_rows(x, m, rows, eps=eps)
    tx, tv, tm = dev(x), dev(v), dev(m)
    a32 = nb.nbody_accel(tx, tm, eps=eps, precision="fp32c").cpu().numpy()
    o64 = ordered(nb, nb.nbody_accel, tx, tm, eps=eps, precision="fp64").cpu().numpy()
    assert row_err(o64[:, rows], ref).max() <= 1e-12
    assert row_err(a32[:, rows], ref).max() <= 1e-5
    e0 = row_err(a32, o64)
    print("N=65536 t=0 fp32c vs ordered fp64, all rows: max %.3e" % e0.max())
    assert e0.max() <= 1e-5
    drift = {}
    finals = {}
    for prec in ("fp32c", "fp64"):
        px, pv = dev(x), dev(v)
        pa = torch.empty_like(px)
        e0 = nb.nbody_energy(px, pv, tm, eps=eps).cpu().numpy()[2]
        nb.nbody_step(px, pv, pa, tm, dt, w["steps"], eps=eps, precision=prec)
        e1 = nb.nbody_energy(px, pv, tm, eps=eps).cpu().numpy()[2]
        drift[prec] = abs((e1 - e0) / e0)
        finals[prec] = (px, pa)
    print("N=65536 100 steps |dE/E|: fp32c %.3e fp64 %.3e" % (drift["fp32c"], drift["fp64"]))
    assert drift["fp32c"] < 1e-4 and drift["fp64"] < 1e-4
    assert abs(drift["fp32c"] - drift["fp64"]) < 1e-6
    # force error of FP32C against the ordered FP64 kernel at the final FP64 state, every row
    fx = finals["fp64"][0]
    o64 = ordered(nb, nb.nbody_accel, fx, tm, eps=eps, precision="fp64").cpu().numpy()
    b32 = nb.nbody_accel(fx, tm, eps=eps, precision="fp32c").cpu().numpy()
    e1 = row_err(b32, o64)
    print("N=65536 final state fp32c vs ordered fp64, all rows: max %.3e" % e1.max())
    assert e1.max() <= 1e-5


@pytest.mark.parametrize("mode,bitem", [(0, 0), (2, 1024), (2, 64), (3, 0), (4, 0)])
def test_ensemble512_sampled_clusters(nb, oracle_mod, mode, bitem):
    """The batched kernels (mode 0: systems resident in LDS; mode 2: streamed
    items of up to 1024 particles, or of 64 evaluated by one wave each; mode 3:
    the items of 64 with two launches per step; mode 4: their symmetric form,
    each unordered pair once, the untuned default and the tuner's choice for
    FP32C on this layout) on the full 512-cluster layout, against the oracle's
    own KDK on sampled clusters, and the accelerations the run leaves behind,
    a(x) at the final positions, per row against the oracle's (1e-5)."""
    w = ics.WORKLOADS["ensemble512"]
    off, epsv, x, v, m = ics.ensemble(w["ncl"], seed=w["seed"], nmin=w["nmin"], nmax=w["nmax"])
    steps, dt = 8, w["dt"]
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta = torch.empty_like(tx)
    nb.nbody_set_config(bsplit=mode, bitem=bitem, bpass=4 if mode == 0 else 0)  # bpass forces the resident kernel
    try:
        nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, dt, steps, precision="fp32c", check_finite=True)
    finally:
        nb.nbody_set_config()
    bx, bv, ba = tx.cpu().numpy(), tv.cpu().numpy(), ta.cpu().numpy()
    sizes = np.diff(off)
    picks = [int(np.argmin(sizes)), int(np.argmax(sizes))] + list(np.random.default_rng(2).choice(len(sizes), 4, replace=False))
    worst_a = 0.0
    for c in picks:
        s, e = off[c], off[c + 1]
        rx, rv = oracle_mod.kdk(x[:, s:e], v[:, s:e], m[s:e], dt, steps, eps=float(epsv[c]))
        scale = np.abs(v[:, s:e]).max() * dt * steps
        assert np.abs(bx[:, s:e] - rx).max() <= 1e-6 * scale, (c, sizes[c])
        assert np.abs(bv[:, s:e] - rv).max() <= 1e-5 * np.abs(rv).max(), (c, sizes[c])
        ra = oracle_mod.accel(bx[:, s:e], m[s:e], eps=float(epsv[c]))
        ea = row_err(ba[:, s:e], ra).max()
        worst_a = max(worst_a, ea)
        assert ea <= 1e-5, (c, sizes[c], ea)
    print("ensemble512 mode %d: worst per-row acceleration error on %d clusters %.2e" % (mode, len(picks), worst_a))


def _grad_setup():
    w = ics.WORKLOADS["grad16k"]
    x, v, m = ics.plummer(w["n"], seed=w["seed"])
    xp, vp = ics.perturb(x, v, w["sigma"], seed=w["target_seed"])
    return w, x, v, m, xp, vp


@pytest.fixture(scope="module")
def grad16k_fd(nb):
    """Central differences (h = 1e-6) of L = mean |x_T - x_tgt|^2 after 200
    FP64 GPU KDK steps on 64 seeded coordinates (24 position, 24 velocity, 16
    mass), the reference every gradient form of the workload is checked
    against."""
    w, x, v, m, xp, vp = _grad_setup()
    n, eps, dt, steps = w["n"], w["eps"], w["dt"], w["steps"]
    tm = dev(m)
    tg_x, tg_v = dev(xp), dev(vp)
    nb.nbody_step(tg_x, tg_v, torch.empty_like(tg_x), tm, dt, steps, eps=eps, precision="fp64")

    def loss_at(xx, vv, mm):
        px, pv, pm = dev(xx), dev(vv), dev(mm)
        pa = torch.empty_like(px)
        nb.nbody_step(px, pv, pa, pm, dt, steps, eps=eps, precision="fp64")
        return float((((px - tg_x) ** 2).sum() / n).item())

    rng = np.random.default_rng(5)
    h = 1e-6
    coords = [("x", int(rng.integers(3)), int(rng.integers(n))) for _ in range(24)]
    coords += [("v", int(rng.integers(3)), int(rng.integers(n))) for _ in range(24)]
    coords += [("m", 0, int(rng.integers(n))) for _ in range(16)]
    fd = []
    for kind, c, i in coords:
        xx, vv, mm = x.copy(), v.copy(), m.copy()
        arr = {"x": xx, "v": vv, "m": mm}[kind]
        idx = i if kind == "m" else (c, i)
        arr[idx] += h
        lp = loss_at(xx, vv, mm)
        arr[idx] -= 2 * h
        lq = loss_at(xx, vv, mm)
        fd.append((lp - lq) / (2 * h))
    return coords, np.array(fd), tg_x


def _grad16k(nb, precision, forward_precision, tg_x):
    w, x, v, m, _, _ = _grad_setup()
    n, eps, dt, steps, every = w["n"], w["eps"], w["dt"], w["steps"], w["every"]
    tx, tv, tmg = dev(x).requires_grad_(), dev(v).requires_grad_(), dev(m).requires_grad_()
    xT, _ = nb.NBodyTrajectory.apply(tx, tv, tmg, dt, steps, every, 1.0, eps, precision, forward_precision)
    (((xT - tg_x) ** 2).sum() / n).backward()
    return {"x": tx.grad.cpu().numpy(), "v": tv.grad.cpu().numpy(), "m": tmg.grad.cpu().numpy()}


@pytest.mark.parametrize("precision,forward", [("fp64", None), ("fp32c", None), ("fp32c", "fp32c")])
def test_grad16k_against_finite_differences(nb, grad16k_fd, precision, forward):
    """Gradient of L after 200 steps (checkpoints every 20) against central
    differences of the FP64 forward, per coordinate: |g - fd| / max(|fd|,
    1e-3 max|g|) <= 1e-4 for the FP64 gradient and for the library's FP32C
    gradient (FP64 forward, FP32C sweep: the FP64 map's gradient).  The
    all-FP32C form differentiates the FP32C map, whose sensitivities to
    single mass coordinates and small position components differ from the
    FP64 map's by up to 4.7e-4 of their own size (central differences of the
    FP32C forward show the same offsets), so it is held to 1e-4 of the
    largest component of each kind (measured: 7.7e-5 for the masses)."""
    coords, fd, tg_x = grad16k_fd
    g = _grad16k(nb, precision, forward, tg_x)
    kinds = {k: [q for q, (kk, _, _) in enumerate(coords) if kk == k] for k in ("x", "v", "m")}
    worst = 0.0
    for kind, idx in kinds.items():
        gv = np.array([g[kind][coords[q][2]] if kind == "m" else g[kind][coords[q][1], coords[q][2]] for q in idx])
        f = fd[idx]
        e = np.abs(gv - f) / np.maximum(np.abs(f), 1e-3 * np.abs(g[kind]).max())
        ek = np.abs(gv - f).max() / np.abs(g[kind]).max()
        worst = max(worst, e.max())
        print("grad16k %s (forward %s) %s: per coordinate %.2e, vs largest component %.2e"
              % (precision, forward, kind, e.max(), ek))
        if forward == "fp32c":
            assert ek <= 1e-4, kind
        else:
            assert e.max() <= 1e-4, kind


def test_grad16k_default_fp32c_is_the_fp64_gradient(nb, grad16k_fd):
    """The library's FP32C gradient (FP64 forward and checkpoints, FP32C
    reverse sweep) differentiates the FP64 trajectory: each segment of the
    sweep restarts from an FP64 checkpoint, so it agrees with the all-FP64
    gradient to FP32C arithmetic, per coordinate within 1e-5 of each kind's
    largest component."""
    _, _, tg_x = grad16k_fd
    g64 = _grad16k(nb, "fp64", None, tg_x)
    gmix = _grad16k(nb, "fp32c", None, tg_x)
    for kind in ("x", "v", "m"):
        e = np.abs(gmix[kind] - g64[kind]).max() / np.abs(g64[kind]).max()
        print("grad16k default fp32c vs fp64 %s: %.2e of the largest component" % (kind, e))
        assert e <= 1e-5, kind


# per-coordinate bars over ALL coordinates against the oracle (kind: x, v, m)
SHORT_TOL = {"fp64": {"x": 1e-9, "v": 1e-9, "m": 1e-9}, "fp32c": {"x": 1e-4, "v": 1e-4, "m": 1e-3}}


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_grad16k_against_oracle_short(nb, oracle_mod, prec):
    """Full N = 16384 system, 10 steps with checkpoints every 4, against the
    oracle's adjoint (which stores the whole trajectory), per coordinate:
    |g - r| / max(|r|, 1e-3 max|r|) for each kind, on a seeded sample of 64
    coordinates (24 position, 24 velocity, 16 mass, as in the workload's
    finite-difference check) at the gradient bar 1e-4, and on every
    coordinate.  Over all 16384 mass coordinates the FP32C sweep (the
    library's FP32C gradient: FP64 forward) reaches 1.5e-4: a mass
    coordinate is a sum over all partners of FP32 terms s^-3/2 d.w, and on
    this system (cotangent 2 (x - x_tgt) / N) the magnitudes of those terms
    add up to as much as 3900 times the coordinate where it sits at the 1e-3
    floor (median 43, 99th percentile 1050: oracle term scales), so a single
    rounding of each term (u = 6e-8) already allows 2.3e-4 and the few of an
    FP32 term about 1e-3; positions and velocities stay below 1e-4."""
    w, x, v, m, xp, vp = _grad_setup()
    n, eps, dt = w["n"], w["eps"], w["dt"]
    steps, every = 10, 4
    tgt, _ = oracle_mod.kdk(xp, vp, m, dt, steps, eps=eps)
    loss, (rgx, rgv, rgm) = oracle_mod.loss_grad(x, v, m, tgt, dt, steps, eps=eps)
    tx, tv, tmg = dev(x).requires_grad_(), dev(v).requires_grad_(), dev(m).requires_grad_()
    xT, _ = nb.NBodyTrajectory.apply(tx, tv, tmg, dt, steps, every, 1.0, eps, prec)
    L = ((xT - dev(tgt)) ** 2).sum() / n
    L.backward()
    rng = np.random.default_rng(5)
    sample = {"x": [(int(rng.integers(3)), int(rng.integers(n))) for _ in range(24)],
              "v": [(int(rng.integers(3)), int(rng.integers(n))) for _ in range(24)],
              "m": [(0, int(rng.integers(n))) for _ in range(16)]}
    for kind, g, r in (("x", tx.grad, rgx), ("v", tv.grad, rgv), ("m", tmg.grad, rgm)):
        e = coord_err(g.cpu().numpy(), r)
        es = np.array([e[i] if kind == "m" else e[c, i] for c, i in sample[kind]])
        print("grad16k short %s %s: per coordinate, 64-coordinate sample %.3e, all %.3e" % (prec, kind, es.max(), e.max()))
        assert es.max() <= min(1e-4, SHORT_TOL[prec][kind]), kind
        assert e.max() <= SHORT_TOL[prec][kind], kind


def test_hermite6_409600_sampled_rows_and_steps(nb, oracle_mod):
    w = ics.WORKLOADS["hermite6_409600"]
    n, eps, dt, steps = w["n"], w["eps"], w["dt"], w["steps"]
    x, v, m = ics.plummer(n, seed=w["seed"])
    acc = ics.plummer_mean_field(x)
    rows = np.sort(np.random.default_rng(1).choice(n, 48, replace=False))
    ra, rj, rs = oracle_mod.accel_jerk_snap_rows(x, v, acc, m, rows, eps=eps)
    tx, tv, tacc, tm = dev(x), dev(v), dev(acc), dev(m)
    for prec, tols in (("fp64", (1e-12, 1e-11, 1e-10)), ("fp32c", (1e-5, 2e-3, 2e-3))):
        a, jk, sn = (q.cpu().numpy()[:, rows] for q in
                     nb.nbody_accel_jerk_snap(tx, tv, tacc, tm, eps=eps, precision=prec))
        errs = (row_err(a, ra).max(), row_err(jk, rj).max(), row_err(sn, rs).max())
        print("N=409600 %s sampled rows: a %.2e jerk %.2e snap %.2e" % ((prec,) + errs))
        assert all(e <= t for e, t in zip(errs, tols))
    out = {}
    for prec in ("fp64", "fp32c"):
        sx, sv = dev(x), dev(v)
        st = [torch.empty_like(sx) for _ in range(4)]
        nb.nbody_step_hermite6(sx, sv, *st, tm, dt, steps, eps=eps, precision=prec, check_finite=True)
        out[prec] = (sx.cpu().numpy(), sv.cpu().numpy())
    dx = np.abs(out["fp32c"][0] - out["fp64"][0]).max()
    # positions move by about dt^2 a per step, so a relative force error of
    # 1e-5 allows steps * dt^2 * 1e-5 * max|a|
    amax = np.abs(nb.nbody_accel(tx, tm, eps=eps, precision="fp64").cpu().numpy()).max()
    tol = steps * dt * dt * 1e-5 * amax + 1e-12
    print("N=409600 three steps: fp32c vs fp64 max |dx| %.2e (bound %.2e)" % (dx, tol))
    assert dx <= tol
