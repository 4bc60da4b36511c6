"""Parity at the workloads' full sizes, in the launch configuration the
benchmark uses, on outputs the oracle can compute one by one:

* N = 2^20 two-component force (eps = 0.001): FP32C and FP64 on sampled rows,
  and the FP32C VJP on sampled rows and against the FP64 VJP;
* N = 65536 Plummer force (eps = 0.005) on sampled rows, and 100 FP32C KDK
  steps against the FP64 GPU path (energy drift and force error reported);
* 512-cluster ensemble: sampled clusters against the oracle's own KDK;
* N = 16384 adjoint: the 200-step FP64 gradient against central finite
  differences (h = 1e-6) of the FP64 GPU forward on 64 random coordinates,
  and a shorter run against the oracle's full adjoint;
* N = 409600 sixth-order Hermite (eps = 1e-7): acceleration, jerk and snap on
  sampled rows against the oracle, and three FP32C steps against three FP64
  steps of the GPU path.
"""
import numpy as np
import pytest

import ics

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


def test_twocomp1m_sampled_rows(nb, oracle_mod):
    w = ics.WORKLOADS["twocomp1m_force"]
    n, eps = w["n"], w["eps"]
    x, _, m = ics.two_component(n, seed=w["seed"])
    rows = np.sort(np.random.default_rng(0).choice(n, 96, replace=False))
    rows = np.concatenate([[0, n - 1], rows])
    ref = oracle_mod.accel_rows(x, m, rows, eps=eps)
    tx, tm = dev(x), dev(m)
    a64 = nb.nbody_accel(tx, tm, eps=eps, precision="fp64").cpu().numpy()
    a32 = nb.nbody_accel(tx, tm, eps=eps, precision="fp32c").cpu().numpy()
    e64 = row_err(a64[:, rows], ref)
    e32 = row_err(a32[:, rows], ref)
    print("N=2^20 sampled rows: fp64 max %.3e, fp32c max %.3e" % (e64.max(), e32.max()))
    assert e64.max() <= 1e-12
    assert e32.max() <= 1e-5
    # every row of FP32C against the (oracle-checked) FP64 path
    e_all = row_err(a32, a64)
    print("N=2^20 fp32c vs fp64 all rows: max %.3e p99 %.3e" % (e_all.max(), np.quantile(e_all, 0.99)))
    assert np.quantile(e_all, 0.999) <= 1e-5


def test_twocomp1m_vjp_sampled_rows(nb, oracle_mod):
    """The FP32C VJP at N = 2^20 in the benchmark's configuration (the
    symmetric kernel at this size): sampled rows against the oracle and all
    rows against the FP64 GPU path, norm-wise as the smaller VJP tests."""
    w_ = ics.WORKLOADS["twocomp1m_force"]
    n, eps = w_["n"], w_["eps"]
    x, _, m = ics.two_component(n, seed=w_["seed"])
    w = np.random.default_rng(1).standard_normal((3, n))
    tx, tm, tw = dev(x), dev(m), dev(w)
    gx, gm = nb.nbody_accel_vjp(tx, tm, tw, eps=eps, precision="fp32c")
    gx64, gm64 = nb.nbody_accel_vjp(tx, tm, tw, eps=eps, precision="fp64")
    gx, gm, gx64, gm64 = gx.cpu().numpy(), gm.cpu().numpy(), gx64.cpu().numpy(), gm64.cpu().numpy()
    ex = np.linalg.norm(gx - gx64) / np.linalg.norm(gx64)
    em = np.linalg.norm(gm - gm64) / np.linalg.norm(gm64)
    rows = np.random.default_rng(12).choice(n, 192, replace=False)
    rgx, rgm = oracle_mod.accel_vjp_rows(x, m, w, rows, eps=eps)
    ox = np.linalg.norm(gx[:, rows] - rgx) / np.linalg.norm(rgx)
    om = np.linalg.norm(gm[rows] - rgm) / np.linalg.norm(rgm)
    o64 = np.linalg.norm(gx64[:, rows] - rgx) / np.linalg.norm(rgx)
    print("vjp 2^20: fp32c vs fp64 gx %.2e gm %.2e; vs oracle (192 rows) gx %.2e gm %.2e; fp64 vs oracle %.2e"
          % (ex, em, ox, om, o64))
    assert ex <= 2e-5 and em <= 2e-5
    assert ox <= 2e-5 and om <= 2e-5
    assert o64 <= 1e-11


def test_plummer64k_force_and_drift(nb, oracle_mod):
    w = ics.WORKLOADS["plummer64k_fp32c"]
    n, eps, dt = w["n"], w["eps"], w["dt"]
    x, v, m = ics.plummer(n, seed=w["seed"])
    rows = np.sort(np.random.default_rng(1).choice(n, 128, replace=False))
    ref = oracle_mod.accel_rows(x, m, rows, eps=eps)
    tx, tv, tm = dev(x), dev(v), dev(m)
    a32 = nb.nbody_accel(tx, tm, eps=eps, precision="fp32c").cpu().numpy()
    assert row_err(a32[:, rows], ref).max() <= 1e-5
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
    # force error of FP32C against FP64 at the final FP64 state
    fx = finals["fp64"][0]
    a64 = nb.nbody_accel(fx, tm, eps=eps, precision="fp64").cpu().numpy()
    b32 = nb.nbody_accel(fx, tm, eps=eps, precision="fp32c").cpu().numpy()
    assert np.quantile(row_err(b32, a64), 0.999) <= 1e-5


@pytest.mark.parametrize("mode,bitem", [(0, 0), (2, 1024), (2, 64), (3, 0)])
def test_ensemble512_sampled_clusters(nb, oracle_mod, mode, bitem):
    """The batched kernels (mode 0: systems resident in LDS; mode 2: streamed
    items of up to 1024 particles, or of 64 evaluated by one wave each; mode 3:
    the items of 64 with two launches per step, the default) against the
    oracle's own KDK on sampled clusters."""
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
    bx, bv = tx.cpu().numpy(), tv.cpu().numpy()
    sizes = np.diff(off)
    picks = [int(np.argmin(sizes)), int(np.argmax(sizes))] + list(np.random.default_rng(2).choice(len(sizes), 4, replace=False))
    for c in picks:
        s, e = off[c], off[c + 1]
        rx, rv = oracle_mod.kdk(x[:, s:e], v[:, s:e], m[s:e], dt, steps, eps=float(epsv[c]))
        scale = np.abs(v[:, s:e]).max() * dt * steps
        assert np.abs(bx[:, s:e] - rx).max() <= 1e-6 * scale, (c, sizes[c])
        assert np.abs(bv[:, s:e] - rv).max() <= 1e-5 * np.abs(rv).max(), (c, sizes[c])


def _grad_setup():
    w = ics.WORKLOADS["grad16k"]
    x, v, m = ics.plummer(w["n"], seed=w["seed"])
    xp, vp = ics.perturb(x, v, w["sigma"], seed=w["target_seed"])
    return w, x, v, m, xp, vp


def test_grad16k_against_finite_differences(nb):
    """Gradient of L = mean |x_T - x_tgt|^2 after 200 steps (checkpoints every
    20) against central differences of the FP64 GPU forward, 64 coordinates."""
    w, x, v, m, xp, vp = _grad_setup()
    n, eps, dt, steps, every = w["n"], w["eps"], w["dt"], w["steps"], w["every"]
    tm = dev(m)
    tg_x, tg_v = dev(xp), dev(vp)
    tg_a = torch.empty_like(tg_x)
    nb.nbody_step(tg_x, tg_v, tg_a, tm, dt, steps, eps=eps, precision="fp64")
    tx, tv, tmg = dev(x).requires_grad_(), dev(v).requires_grad_(), dev(m).requires_grad_()
    xT, _ = nb.NBodyTrajectory.apply(tx, tv, tmg, dt, steps, every, 1.0, eps, "fp64")
    L = ((xT - tg_x) ** 2).sum() / n
    L.backward()
    grads = {"x": tx.grad.cpu().numpy(), "v": tv.grad.cpu().numpy(), "m": tmg.grad.cpu().numpy()}

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
    worst = 0.0
    gnorm = {k: np.abs(g).max() for k, g in grads.items()}
    for kind, c, i in coords:
        xx, vv, mm = x.copy(), v.copy(), m.copy()
        arr = {"x": xx, "v": vv, "m": mm}[kind]
        if kind == "m":
            arr[i] += h; lp = loss_at(xx, vv, mm); arr[i] -= 2 * h; lq = loss_at(xx, vv, mm)
            g = grads["m"][i]
        else:
            arr[c, i] += h; lp = loss_at(xx, vv, mm); arr[c, i] -= 2 * h; lq = loss_at(xx, vv, mm)
            g = grads[kind][c, i]
        fd = (lp - lq) / (2 * h)
        err = abs(g - fd) / max(abs(fd), 1e-3 * gnorm[kind])
        worst = max(worst, err)
    print("grad16k FD check: worst normalised error %.3e over %d coordinates" % (worst, len(coords)))
    assert worst <= 1e-4


def test_grad16k_mixed_precision_adjoint(nb):
    """FP64 forward, FP32C reverse sweep: the gradient of the FP64 trajectory.
    Each segment of the sweep restarts from an FP64 checkpoint, so it must
    agree with the all-FP64 gradient to FP32C arithmetic (1e-5 of each
    gradient's largest component), unlike the all-FP32C gradient, which
    differentiates its own trajectory."""
    w, x, v, m, xp, vp = _grad_setup()
    n, eps, dt, steps, every = w["n"], w["eps"], w["dt"], w["steps"], w["every"]
    tm = dev(m)
    tg_x, tg_v = dev(xp), dev(vp)
    nb.nbody_step(tg_x, tg_v, torch.empty_like(tg_x), tm, dt, steps, eps=eps, precision="fp64")
    grads = {}
    for aprec in ("fp64", "fp32c"):
        tx, tv, tmg = dev(x).requires_grad_(), dev(v).requires_grad_(), dev(m).requires_grad_()
        xT, _ = nb.NBodyTrajectory.apply(tx, tv, tmg, dt, steps, every, 1.0, eps, "fp64", aprec)
        (((xT - tg_x) ** 2).sum() / n).backward()
        grads[aprec] = [tx.grad.cpu().numpy(), tv.grad.cpu().numpy(), tmg.grad.cpu().numpy()]
    for g64, gmix in zip(grads["fp64"], grads["fp32c"]):
        assert np.abs(gmix - g64).max() <= 1e-5 * np.abs(g64).max()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32c", 1e-4)])
def test_grad16k_against_oracle_short(nb, oracle_mod, prec, tol):
    """Full N = 16384 system, 10 steps with checkpoints every 4, against the
    oracle's adjoint (which stores the whole trajectory)."""
    w, x, v, m, xp, vp = _grad_setup()
    n, eps, dt = w["n"], w["eps"], w["dt"]
    steps, every = 10, 4
    tgt, _ = oracle_mod.kdk(xp, vp, m, dt, steps, eps=eps)
    loss, (rgx, rgv, rgm) = oracle_mod.loss_grad(x, v, m, tgt, dt, steps, eps=eps)
    tx, tv, tmg = dev(x).requires_grad_(), dev(v).requires_grad_(), dev(m).requires_grad_()
    xT, _ = nb.NBodyTrajectory.apply(tx, tv, tmg, dt, steps, every, 1.0, eps, prec)
    L = ((xT - dev(tgt)) ** 2).sum() / n
    L.backward()
    for g, r in ((tx.grad, rgx), (tv.grad, rgv), (tmg.grad, rgm)):
        rel = np.linalg.norm(g.cpu().numpy() - r) / np.linalg.norm(r)
        print("grad16k short %s rel err %.3e" % (prec, rel))
        assert rel <= tol


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
