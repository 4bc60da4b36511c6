"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Error statistic for accelerations: per particle e_i = |a_i - a_i^ref| / |a_i^ref|,
gated on the maximum over particles.  Tolerances: 1e-12 for the FP64 path and
1e-5 for FP32C (FP32 pair arithmetic on float-float positions with compensated
sums); FP32 (rounded positions) is held to 1e-4 on these well-separated inputs.

The VJP is gated per row on its condition-normalised error |g_k - ref_k| /
scale_k, scale_k the sum of the magnitudes of row k's terms (oracle): with
random cotangents a row's terms cancel, so |ref_k| alone says little about the
accuracy of its sum.  Bars (CTOL): 1e-13 for FP64; 2e-5 for FP32C, the rounding
bound of a pair just outside the near-field radius f |x_i| (f >= 0.02), whose
FP32 displacement is off by up to u (|x_i| + |x_j|) / |d| <= 101 u relative
and whose term (s^-3/2, s^-5/2 d d^T) moves by about three times that; 5e-4
for FP32 (rounded positions, no repair; these inputs hold no pair closer than
about 1e-3 of |x|).  Trajectory gradients are gated per coordinate with
|g - r| / max(|r|, 1e-3 max|r|) for each kind (positions, velocities, masses).
"""
import numpy as np
import pytest

import ics
from parity_stats import cond_err, coord_err, row_rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32c": 1e-5, "fp32": 1e-4}


@pytest.fixture(scope="module")
def nb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_02744_amd as nbm
    nbm.load()
    return nbm


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def rel_err(a, ref):
    num = np.linalg.norm(a - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    return (num / np.where(den > 0, den, 1.0)).max()


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 255, 256, 257, 511, 1000, 1025, 3001])
@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
def test_accel_ragged_sizes(nb, oracle_mod, n, prec):
    x, _, m = ics.plummer(n, seed=100 + n)
    eps = 0.01
    ref = oracle_mod.accel(x, m, G=1.0, eps=eps)
    a = nb.nbody_accel(dev(x), dev(m), eps=eps, precision=prec).cpu().numpy()
    if n == 1:
        assert np.all(a == 0.0)
        return
    print("accel n=%d %s max rel err %.3e" % (n, prec, rel_err(a, ref)))
    assert rel_err(a, ref) <= TOL[prec]


@pytest.mark.parametrize("n", [64, 300, 2049])
def test_accel_fp32c_small_systems_many_seeds(nb, oracle_mod, n):
    """Small systems have heavy particles: one pair just outside a fixed
    near-field radius can carry more than the particle's whole acceleration,
    so the repair radius grows as n^-1/3 (regression: a 2049-body Plummer
    sample reached 1.5e-5 with a radius of 0.02 |x| alone)."""
    worst = 0.0
    for seed in range(12):
        x, v, m = ics.plummer(n, seed=1000 * n + seed)
        ref = oracle_mod.accel(x, m, G=1.1, eps=0.01)
        a = nb.nbody_accel(dev(x), dev(m), G=1.1, eps=0.01, precision="fp32c").cpu().numpy()
        ra, rj = oracle_mod.accel_jerk(x, v, m, G=1.1, eps=0.01)
        aj, jk = nb.nbody_accel_jerk(dev(x), dev(v), dev(m), G=1.1, eps=0.01, precision="fp32c")
        worst = max(worst, rel_err(a, ref), rel_err(aj.cpu().numpy(), ra))
    print("n=%d worst fp32c accel error over 12 seeds %.2e" % (n, worst))
    assert worst <= 1e-5


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
@pytest.mark.parametrize("ipl,split", [(1, 1), (2, 1), (4, 1), (1, 3), (2, 7), (4, 16), (2, 0), (1, 64)])
def test_accel_tile_configs(nb, oracle_mod, prec, ipl, split):
    n = 4099
    x, _, m = ics.two_component(n, seed=7)
    G, eps = 1.3, 0.02
    ref = oracle_mod.accel(x, m, G=G, eps=eps)
    nb.nbody_set_config(ipl=ipl, split=split)
    try:
        a1 = nb.nbody_accel(dev(x), dev(m), G=G, eps=eps, precision=prec)
        a2 = nb.nbody_accel(dev(x), dev(m), G=G, eps=eps, precision=prec)
    finally:
        nb.nbody_set_config()
    assert torch.equal(a1, a2), "not deterministic"
    assert rel_err(a1.cpu().numpy(), ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_accel_exclude_self_eps_zero(nb, oracle_mod, prec):
    x, _, m = ics.random_cloud(700, seed=3)
    ref = oracle_mod.accel(x, m, eps=0.0)
    a = nb.nbody_accel(dev(x), dev(m), eps=0.0, precision=prec, exclude_self=True).cpu().numpy()
    assert np.isfinite(a).all()
    assert rel_err(a, ref) <= 10 * TOL[prec]


def _tight_pairs_far_away(n=3000, seed=30):
    """A Plummer cloud shifted to (3, -2, 5) with 200 particles given a partner
    at 1e-5 .. 1e-3 (well inside eps = 0.01): FP32-rounded positions resolve
    those separations to only a few per cent."""
    x, _, m = ics.plummer(n, seed=seed)
    x = x + np.array([[3.0], [-2.0], [5.0]])
    rng = np.random.default_rng(seed)
    a = rng.choice(n // 2, 200, replace=False)
    b = n // 2 + np.arange(200)
    off = rng.standard_normal((3, 200))
    off *= 10 ** rng.uniform(-5, -3, 200) / np.linalg.norm(off, axis=0)
    x[:, b] = x[:, a] + off
    return x, m


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32c", 1e-5)])
def test_accel_tight_pairs_near_field(nb, oracle_mod, prec, tol):
    x, m = _tight_pairs_far_away()
    ref = oracle_mod.accel(x, m, eps=0.01)
    a = nb.nbody_accel(dev(x), dev(m), eps=0.01, precision=prec).cpu().numpy()
    e = rel_err(a, ref)
    print("tight pairs %s max rel err %.3e" % (prec, e))
    assert e <= tol
    # rounded positions without the repair are far off for these pairs
    a32 = nb.nbody_accel(dev(x), dev(m), eps=0.01, precision="fp32").cpu().numpy()
    assert rel_err(a32, ref) > 10 * tol


def test_vjp_tight_pairs_near_field(nb, oracle_mod):
    x, m = _tight_pairs_far_away(2000, seed=31)
    w = np.random.default_rng(2).standard_normal(x.shape)
    gx, gm = nb.nbody_accel_vjp(dev(x), dev(m), dev(w), eps=0.01, precision="fp32c")
    cx, cm, _, _ = vjp_cond(oracle_mod, x, m, w, gx.cpu().numpy(), gm.cpu().numpy(), 1.0, 0.01)
    print("vjp tight pairs: cond gx %.2e gm %.2e" % (cx.max(), cm.max()))
    assert cx.max() <= CTOL["fp32c"] and cm.max() <= CTOL["fp32c"]


def test_accel_plummer1k_fp64(nb, oracle_mod):
    w = ics.WORKLOADS["plummer1k_fp64"]
    x, _, m = ics.plummer(w["n"], seed=w["seed"])
    ref = oracle_mod.accel(x, m, eps=w["eps"])
    a = nb.nbody_accel(dev(x), dev(m), eps=w["eps"], precision="fp64").cpu().numpy()
    assert rel_err(a, ref) <= 1e-12


def test_kdk_plummer1k_fp64_trajectory(nb, oracle_mod):
    """Ten KDK steps of the 1024-body Plummer sphere, FP64 path vs oracle."""
    w = ics.WORKLOADS["plummer1k_fp64"]
    x, v, m = ics.plummer(w["n"], seed=w["seed"])
    rx, rv = oracle_mod.kdk(x, v, m, w["dt"], w["steps"], eps=w["eps"])
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta = torch.empty_like(tx)
    nb.nbody_step(tx, tv, ta, tm, w["dt"], w["steps"], eps=w["eps"], precision="fp64")
    assert np.abs(tx.cpu().numpy() - rx).max() <= 1e-10
    assert np.abs(tv.cpu().numpy() - rv).max() <= 1e-10
    ra = oracle_mod.accel(rx, m, eps=w["eps"])
    assert rel_err(ta.cpu().numpy(), ra) <= 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_step_resumable_bitwise(nb, prec):
    x, v, m = ics.plummer(2000, seed=4)
    out = []
    for chunks in ((10,), (4, 6), (1, 1, 8)):
        tx, tv, tm = dev(x), dev(v), dev(m)
        ta = torch.empty_like(tx)
        valid = False
        for c in chunks:
            nb.nbody_step(tx, tv, ta, tm, 1.0 / 128, c, eps=0.01, precision=prec, acc_valid=valid)
            valid = True
        out.append((tx.cpu(), tv.cpu(), ta.cpu()))
    for o in out[1:]:
        for p, q in zip(out[0], o):
            assert torch.equal(p, q)


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
def test_pair_kernels_repeat_bitwise(nb, prec):
    """Repeated calls on the same inputs give bitwise-identical outputs: every
    j-sum (in-kernel folds, slice sums, group combines) has a fixed order, which
    the checkpointed adjoint relies on when it recomputes the forward pass."""
    x, v, m = ics.plummer(3001, seed=12)
    tx, tv, tm = dev(x), dev(v), dev(m)
    w = dev(np.random.default_rng(3).standard_normal((3, 3001)))
    acc = dev(ics.plummer_mean_field(x))
    nb.nbody_set_config(ipl=1, split=8)  # several j-slices, so the slice sum is exercised
    try:
        runs = []
        for _ in range(3):
            outs = [nb.nbody_accel(tx, tm, eps=0.01, precision=prec)]
            outs += list(nb.nbody_accel_vjp(tx, tm, w, eps=0.01, precision=prec))
            outs += list(nb.nbody_accel_jerk(tx, tv, tm, eps=0.01, precision=prec))
            outs += list(nb.nbody_accel_jerk_snap(tx, tv, acc, tm, eps=0.01, precision=prec))
            if prec == "fp64":
                outs.append(nb.nbody_potential(tx, tm, eps=0.01))
            runs.append([o.cpu() for o in outs])
    finally:
        nb.nbody_set_config()
    for r in runs[1:]:
        for p_, q_ in zip(runs[0], r):
            assert torch.equal(p_, q_)


def test_step_zero_steps_computes_acc(nb, oracle_mod):
    x, v, m = ics.plummer(300, seed=5)
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta = torch.zeros_like(tx)
    nb.nbody_step(tx, tv, ta, tm, 0.01, 0, eps=0.01, precision="fp64")
    assert torch.equal(tx.cpu(), torch.tensor(x)) and torch.equal(tv.cpu(), torch.tensor(v))
    assert rel_err(ta.cpu().numpy(), oracle_mod.accel(x, m, eps=0.01)) <= 1e-12


@pytest.mark.parametrize("n", [1, 2, 77, 1024, 5000])
def test_energy_matches_oracle(nb, oracle_mod, n):
    x, v, m = ics.plummer(n, seed=6 + n)
    ref = oracle_mod.energy(x, v, m, G=1.2, eps=0.01)
    e = nb.nbody_energy(dev(x), dev(v), dev(m), G=1.2, eps=0.01).cpu().numpy()
    for k in range(3):
        assert abs(e[k] - ref[k]) <= 1e-12 * max(abs(ref[k]), 1e-300), (k, e[k], ref[k])
    scale_p = (m * np.abs(v).sum(axis=0)).sum()
    scale_l = (m * np.linalg.norm(x, axis=0) * np.linalg.norm(v, axis=0)).sum()
    assert np.abs(e[3:6] - ref[3:6]).max() <= 1e-14 * scale_p + 1e-300
    assert np.abs(e[6:9] - ref[6:9]).max() <= 1e-14 * scale_l + 1e-300


def test_energy_eps_zero_excludes_self(nb, oracle_mod):
    x, v, m = ics.random_cloud(257, seed=9)
    ref = oracle_mod.energy(x, v, m, eps=0.0)
    e = nb.nbody_energy(dev(x), dev(v), dev(m), eps=0.0).cpu().numpy()
    assert np.isfinite(e).all()
    assert abs(e[1] - ref[1]) <= 1e-12 * abs(ref[1])


CTOL = {"fp64": 1e-13, "fp32c": 2e-5, "fp32": 5e-4}


def vjp_cond(oracle_mod, x, m, w, gx, gm, G, eps):
    """Per-row condition-normalised errors of (gx, gm) against the oracle."""
    rows = np.arange(m.shape[0])
    rgx, rgm = oracle_mod.accel_vjp(x, m, w, G=G, eps=eps)
    sx, sm = oracle_mod.accel_vjp_scale_rows(x, m, w, rows, G=G, eps=eps)
    return cond_err(gx, rgx, sx), cond_err(gm, rgm, sm), row_rel(gx, rgx), row_rel(gm, rgm)


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
@pytest.mark.parametrize("n", [2, 65, 1000, 2049])
def test_vjp_matches_oracle(nb, oracle_mod, prec, n):
    x, _, m = ics.two_component(n, seed=11)
    w = np.random.default_rng(n).standard_normal((3, n))
    gx, gm = nb.nbody_accel_vjp(dev(x), dev(m), dev(w), G=0.7, eps=0.02, precision=prec)
    cx, cm, rx, rm = vjp_cond(oracle_mod, x, m, w, gx.cpu().numpy(), gm.cpu().numpy(), 0.7, 0.02)
    print("vjp n=%d %s: cond gx %.2e gm %.2e; rel gx %.2e gm %.2e (max over rows)"
          % (n, prec, cx.max(), cm.max(), rx.max(), rm.max()))
    assert cx.max() <= CTOL[prec] and cm.max() <= CTOL[prec]


def test_vjp_split_configs_agree(nb, oracle_mod):
    n = 3000
    x, _, m = ics.plummer(n, seed=12)
    w = np.random.default_rng(1).standard_normal((3, n))
    for ipl, split in ((1, 1), (2, 5), (1, 11)):
        nb.nbody_set_config(ipl=ipl, split=split)
        try:
            gx, gm = nb.nbody_accel_vjp(dev(x), dev(m), dev(w), eps=0.01, precision="fp64")
        finally:
            nb.nbody_set_config()
        cx, cm, _, _ = vjp_cond(oracle_mod, x, m, w, gx.cpu().numpy(), gm.cpu().numpy(), 1.0, 0.01)
        assert cx.max() <= CTOL["fp64"] and cm.max() <= CTOL["fp64"], (ipl, split, cx.max(), cm.max())


@pytest.mark.parametrize("prec,fwd,tol", [("fp64", None, 1e-9), ("fp32c", None, 1e-4), ("fp32c", "fp32c", 1e-4)])
def test_traj_grad_matches_oracle(nb, oracle_mod, prec, fwd, tol):
    """Checkpointed trajectory gradient against the oracle's full adjoint, per
    coordinate.  ("fp32c", None) is the library's FP32C gradient (FP64
    forward, FP32C sweep); ("fp32c", "fp32c") differentiates the FP32C
    trajectory, a different map, and is held to the same bar relative to the
    largest component of each kind."""
    n, steps, every, dt, eps = 512, 23, 5, 1.0 / 256, 0.01
    x, v, m = ics.plummer(n, seed=13)
    tgt, _ = ics.perturb(x, v, 1e-3, seed=14)
    loss, (rgx, rgv, rgm) = oracle_mod.loss_grad(x, v, m, tgt, dt, steps, eps=eps)
    tx, tv, tm = dev(x).requires_grad_(), dev(v).requires_grad_(), dev(m).requires_grad_()
    xT, _ = nb.NBodyTrajectory.apply(tx, tv, tm, dt, steps, every, 1.0, eps, prec, fwd)
    L = ((xT - dev(tgt)) ** 2).sum() / n
    L.backward()
    assert abs(L.item() - loss) <= (1e-5 if fwd == "fp32c" else 1e-12) * loss
    for kind, g, r in (("x", tx.grad, rgx), ("v", tv.grad, rgv), ("m", tm.grad, rgm)):
        g = g.cpu().numpy()
        e = coord_err(g, r)
        ek = np.abs(g - r).max() / np.abs(r).max()
        print("traj grad %s (forward %s) %s: per coordinate %.2e, vs largest %.2e" % (prec, fwd, kind, e.max(), ek))
        if fwd == "fp32c":
            assert ek <= tol, kind
        else:
            assert e.max() <= tol, kind


def test_traj_grad_recompute_matches_forward(nb):
    """The forward with checkpoints and one uninterrupted nbody_step agree bitwise."""
    n, steps = 700, 13
    x, v, m = ics.plummer(n, seed=15)
    tx, tv, tm = dev(x), dev(v), dev(m)
    xT, vT = nb.trajectory(tx, tv, tm, 1.0 / 128, steps, 4, 1.0, 0.01, "fp32c", "fp32c")
    ax, av = dev(x), dev(v)
    aa = torch.empty_like(ax)
    nb.nbody_step(ax, av, aa, tm, 1.0 / 128, steps, eps=0.01, precision="fp32c")
    assert torch.equal(xT, ax) and torch.equal(vT, av)


def _sweep_inputs(nb, n, steps, every, seed):
    """Checkpoints of an FP64 KDK run (the states at steps 0, every, ...) and
    random final cotangents, for nbody_traj_grad."""
    x, v, m = ics.plummer(n, seed=seed)
    dt, eps = 1.0 / 256, 0.01
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta = torch.empty_like(tx)
    ckx, ckv = [], []
    for c in range(-(-steps // every)):
        ckx.append(tx.clone())
        ckv.append(tv.clone())
        nb.nbody_step(tx, tv, ta, tm, dt, min(every, steps - c * every), eps=eps, precision="fp64", acc_valid=c > 0)
    rng = np.random.default_rng(seed + 1)
    gxT, gvT = dev(rng.standard_normal((3, n))), dev(rng.standard_normal((3, n)))
    return torch.stack(ckx), torch.stack(ckv), tm, gxT, gvT, dt, eps


@pytest.mark.parametrize("prec,n,steps,every", [("fp32c", 2049, 47, 10), ("fp64", 1500, 30, 6), ("fp32", 999, 8, 3),
                                                ("fp32c", 16384, 9, 4), ("fp32c", 700, 13, 13)])
def test_traj_grad_two_streams_bitwise(nb, prec, n, steps, every):
    """The adjoint sweep with the next segment's trajectory recomputed on the
    library's second stream (sweep = 0, automatic: more than one segment and
    n <= 65536) and with everything on the caller's stream (sweep = 1) give
    bitwise the same cotangents, and repeated calls do too: shorter last
    segments, an odd and an even number of segments, the symmetric VJP
    (16384) and one segment (no second stream)."""
    ckx, ckv, tm, gxT, gvT, dt, eps = _sweep_inputs(nb, n, steps, every, 31)
    out = []
    for sweep in (0, 1, 0):
        nb.nbody_set_config(sweep=sweep)
        try:
            out.append(nb.nbody_traj_grad(ckx, ckv, every, steps, tm, dt, gxT, gvT, eps=eps, precision=prec))
        finally:
            nb.nbody_set_config()
    for k, (a, b, c) in enumerate(zip(*out)):
        assert torch.isfinite(a).all() and torch.equal(a, b) and torch.equal(a, c), k


def test_traj_grad_two_streams_graph_capture(nb):
    """The two-stream adjoint sweep captured into a HIP graph (after one eager
    call has sized the workspaces and made the second stream) replays bitwise
    like the eager call, with eager work and eager sweeps between replays."""
    n, steps, every = 1024, 12, 4
    ckx, ckv, tm, gxT, gvT, dt, eps = _sweep_inputs(nb, n, steps, every, 33)
    call = lambda: nb.nbody_traj_grad(ckx, ckv, every, steps, tm, dt, gxT, gvT, eps=eps, precision="fp32c")
    ref = call()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
        outs = call()
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = (outs[0].sum() + 1.0).item()  # eager work between replays
        assert all(torch.equal(a, b) for a, b in zip(outs, ref)), k
        assert all(torch.equal(a, b) for a, b in zip(call(), ref)), k


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
def test_batched_matches_single_system(nb, prec):
    """Every system of a batched run against nbody_step on that system alone:
    FP64 to 1e-12; the FP32 modes (same pair arithmetic, different summation
    blocking) against the FP64 single-system run, to FP32 accuracy of the
    motion over the run."""
    sizes = [1, 64, 100, 300, 513, 1024, 1500, 2500, 4096, 65]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=16, sizes=sizes)
    dt, steps = 1.0 / 512, 7
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta = torch.empty_like(tx)
    nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, dt, steps, precision=prec)
    bx, bv = tx.cpu().numpy(), tv.cpu().numpy()
    for c in range(len(sizes)):
        s, e = off[c], off[c + 1]
        cx, cv, cm = dev(x[:, s:e]), dev(v[:, s:e]), dev(m[s:e])
        ca = torch.empty_like(cx)
        nb.nbody_step(cx, cv, ca, cm, dt, steps, eps=float(epsv[c]), precision="fp64")
        rx, rv, ra = cx.cpu().numpy(), cv.cpu().numpy(), ca.cpu().numpy()
        dx = np.abs(bx[:, s:e] - rx).max()
        dv = np.abs(bv[:, s:e] - rv).max()
        if prec == "fp64":
            assert dx <= 1e-12 and dv <= 1e-12, (c, sizes[c], dx, dv)
        else:
            # relative accuracy of the velocity change dt*steps*a and the displacement
            tol_v = (1e-5 if prec == "fp32c" else 1e-3) * dt * steps * max(np.abs(ra).max(), 1e-30)
            assert dv <= tol_v and dx <= tol_v * dt * steps, (c, sizes[c], dx, dv, tol_v)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_batched_split_and_unsplit_agree(nb, prec):
    """Large systems split over workgroups give the same trajectories (to
    rounding) as one workgroup per system."""
    sizes = [4096, 3000, 2048, 700, 64, 1]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=21, sizes=sizes)
    out = []
    for bsplit in (1, 0):
        nb.nbody_set_config(bsplit=bsplit, bpass=4 if bsplit == 0 else 0)  # bpass forces the resident kernel
        try:
            tx, tv, tm = dev(x), dev(v), dev(m)
            ta = torch.empty_like(tx)
            nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, 1.0 / 512, 6, precision=prec, check_finite=True)
        finally:
            nb.nbody_set_config()
        out.append((tx.cpu().numpy(), tv.cpu().numpy()))
    assert np.abs(out[0][0] - out[1][0]).max() <= 1e-10
    assert np.abs(out[0][1] - out[1][1]).max() <= 1e-8


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_batched_pass_widths_agree(nb, prec):
    """Evaluating 1, 2 or 4 of a lane's i-particles per pass over the records
    changes only which j-blocks the near-field repair revisits."""
    sizes = [4096, 1500, 333, 64]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=22, sizes=sizes)
    out = []
    for bpass in (4, 1, 2):
        nb.nbody_set_config(bpass=bpass)
        try:
            tx, tv, tm = dev(x), dev(v), dev(m)
            ta = torch.empty_like(tx)
            nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, 1.0 / 512, 4, precision=prec, check_finite=True)
        finally:
            nb.nbody_set_config()
        out.append((tx.cpu().numpy(), tv.cpu().numpy()))
    for k in (1, 2):
        if prec == "fp64":
            assert np.array_equal(out[0][0], out[k][0]) and np.array_equal(out[0][1], out[k][1])
        else:
            assert np.abs(out[0][0] - out[k][0]).max() <= 1e-10
            assert np.abs(out[0][1] - out[k][1]).max() <= 1e-8


def _stream(nb, fn, bitem=0, mode=2):
    nb.nbody_set_config(bsplit=mode, bitem=bitem)
    try:
        return fn()
    finally:
        nb.nbody_set_config()


@pytest.mark.parametrize("mode,bitem", [(2, 1024), (2, 64), (3, 0), (4, 0)])
@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_stream_batched_matches_oracle(nb, oracle_mod, prec, mode, bitem):
    """Streamed ensemble kernels against the oracle's KDK: items of <= 1024
    particles (one item per system here), or of 64 particles evaluated by one
    wave each (several items per system above 64; the automatic choice)."""
    sizes = [5, 64, 65, 80, 129, 700, 1300]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=23, sizes=sizes)
    dt, steps = 1.0 / 512, 5
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta = torch.empty_like(tx)
    _stream(nb, lambda: nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, dt, steps, precision=prec,
                                              check_finite=True), bitem, mode)
    for c in range(len(sizes)):
        s, e = off[c], off[c + 1]
        rx, rv = oracle_mod.kdk(x[:, s:e], v[:, s:e], m[s:e], dt, steps, eps=float(epsv[c]))
        dx = np.abs(tx.cpu().numpy()[:, s:e] - rx).max()
        dv = np.abs(tv.cpu().numpy()[:, s:e] - rv).max()
        if prec == "fp64":
            assert dx <= 1e-12 and dv <= 1e-12, (c, dx, dv)
        else:
            ra = oracle_mod.accel(x[:, s:e], m[s:e], eps=float(epsv[c]))
            tol_v = 1e-5 * dt * steps * max(np.abs(ra).max(), 1e-30)
            assert dv <= tol_v and dx <= tol_v * dt * steps, (c, dx, dv, tol_v)


@pytest.mark.parametrize("prec,bitem", [("fp64", 1024), ("fp32c", 0), ("fp32c", 256), ("fp32c", 1024),
                                        ("fp64", 64), ("fp32c", 64)])
def test_stream_batched_agrees_with_resident_kernel(nb, prec, bitem):
    sizes = [4096, 3000, 2048, 700, 257, 64, 1]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=24, sizes=sizes)
    out = []
    for mode in (0, 2):
        nb.nbody_set_config(bsplit=mode, bitem=bitem if mode == 2 else 0, bpass=4 if mode == 0 else 0)
        try:
            tx, tv, tm = dev(x), dev(v), dev(m)
            ta = torch.empty_like(tx)
            nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, 1.0 / 512, 6, precision=prec, check_finite=True)
        finally:
            nb.nbody_set_config()
        out.append((tx.cpu().numpy(), tv.cpu().numpy()))
    assert np.abs(out[0][0] - out[1][0]).max() <= 1e-10
    assert np.abs(out[0][1] - out[1][1]).max() <= 1e-8


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_per_step_wave_items_equal_persistent(nb, prec):
    """Mode 3 (two launches per step) runs the same items and arithmetic as
    mode 2 with items of 64 (one persistent launch): bitwise the same state
    (with the FP32C rescue off, which only mode 3 carries)."""
    sizes = [4096, 3000, 2048, 700, 257, 64, 1]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=28, sizes=sizes)
    out = []
    for mode, bitem in ((2, 64), (3, 0)):
        nb.nbody_set_config(bsplit=mode, bitem=bitem, rescue=2)
        try:
            tx, tv, tm = dev(x), dev(v), dev(m)
            ta = torch.empty_like(tx)
            nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, 1.0 / 512, 5, precision=prec)
        finally:
            nb.nbody_set_config()
        out.append((tx.cpu(), tv.cpu(), ta.cpu()))
    for p_, q_ in zip(out[0], out[1]):
        assert torch.equal(p_, q_)


@pytest.mark.parametrize("mode,bitem", [(2, 1024), (2, 64), (3, 0)])
def test_stream_batched_resumable_and_eps0(nb, oracle_mod, mode, bitem):
    sizes = [300, 77, 1025]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=25, sizes=sizes)
    res = []
    for chunks in ((6,), (2, 4), (0, 3, 3)):
        tx, tv, tm = dev(x), dev(v), dev(m)
        ta = torch.empty_like(tx)
        valid = False
        for c in chunks:
            _stream(nb, lambda: nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, 1.0 / 256, c, precision="fp32c",
                                                      acc_valid=valid), bitem, mode)
            valid = True
        res.append((tx.cpu(), tv.cpu()))
    for r in res[1:]:
        assert torch.equal(res[0][0], r[0]) and torch.equal(res[0][1], r[1])
    # eps = 0 with the self pair masked by index
    eps0 = np.zeros(len(sizes))
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta = torch.empty_like(tx)
    _stream(nb, lambda: nb.nbody_step_batched(off, eps0, tx, tv, ta, tm, 1.0 / 1024, 2, precision="fp64",
                                              exclude_self=True, check_finite=True), bitem, mode)
    for c in range(len(sizes)):
        s, e = off[c], off[c + 1]
        rx, _ = oracle_mod.kdk(x[:, s:e], v[:, s:e], m[s:e], 1.0 / 1024, 2, eps=0.0)
        assert np.abs(tx.cpu().numpy()[:, s:e] - rx).max() <= 1e-11


@pytest.mark.parametrize("mode,bitem", [(2, 1024), (2, 64), (3, 0)])
def test_stream_batched_graph_capture(nb, mode, bitem):
    sizes = [64, 257, 1000]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=26, sizes=sizes)
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta = torch.empty_like(tx)
    nb.nbody_set_config(bsplit=mode, bitem=bitem)
    try:
        ex, ev, ea = tx.clone(), tv.clone(), ta.clone()
        nb.nbody_step_batched(off, epsv, ex, ev, ea, tm, 1.0 / 512, 2, precision="fp32c")
        ref = []
        for _ in range(3):
            nb.nbody_step_batched(off, epsv, ex, ev, ea, tm, 1.0 / 512, 2, precision="fp32c", acc_valid=True)
            ref.append((ex.clone(), ev.clone()))
        gx, gv, ga = tx.clone(), tv.clone(), ta.clone()
        nb.nbody_step_batched(off, epsv, gx, gv, ga, tm, 1.0 / 512, 2, precision="fp32c")
        s = torch.cuda.Stream()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
            nb.nbody_step_batched(off, epsv, gx, gv, ga, tm, 1.0 / 512, 2, precision="fp32c", acc_valid=True)
    finally:
        nb.nbody_set_config()
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = (gx.sum() + 1.0).item()
        assert torch.equal(gx, ref[k][0]) and torch.equal(gv, ref[k][1]), k


def test_tune_batched_records_and_applies_choice(nb):
    """The batched autotuner returns one of its candidates, leaves the caller's
    arrays untouched, and later calls on the same layout (no forced
    configuration) run exactly the chosen configuration."""
    sizes = [1500, 333, 2700, 64, 901]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=27, sizes=sizes)
    tx, tv, tm = dev(x), dev(v), dev(m)
    best = nb.nbody_tune_batched(off, epsv, tx, tv, tm, 1.0 / 512, 4, precision="fp32c")
    assert best["bsplit"] in (0, 1, 2, 3, 4) and best["bpass"] in (0, 1, 2, 4) and best["bitem"] in (0, 64, 256, 512, 1024)
    assert torch.equal(tx, dev(x)) and torch.equal(tv, dev(v))
    out = []
    for forced in (False, True):
        if forced:
            nb.nbody_set_config(bsplit=best["bsplit"], bpass=best["bpass"], bitem=best["bitem"])
        try:
            gx, gv = dev(x), dev(v)
            ga = torch.empty_like(gx)
            nb.nbody_step_batched(off, epsv, gx, gv, ga, tm, 1.0 / 512, 5, precision="fp32c", check_finite=True)
        finally:
            nb.nbody_set_config()
        out.append((gx.cpu(), gv.cpu()))
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    # the search without co-residency returns a configuration that needs none (resident kernel or per-step items)
    best0 = nb.nbody_tune_batched(off, epsv, tx, tv, tm, 1.0 / 512, 2, precision="fp64", allow_cooperative=False)
    assert best0["bsplit"] in (0, 3)
    best2 = nb.nbody_tune_batched(off, epsv, tx, tv, tm, 1.0 / 512, 2, precision="fp32c", allow_cooperative=False)
    assert best2["bsplit"] in (0, 3, 4)
    # the single-launch search returns a configuration that runs all steps in one launch
    best1 = nb.nbody_tune_batched(off, epsv, tx, tv, tm, 1.0 / 512, 2, precision="fp32c",
                                  allow_cooperative="persistent")
    assert best1["bsplit"] in (0, 1, 2)


def test_tune_batched_skips_candidates_that_cannot_serve_the_layout(nb, oracle_mod):
    """A layout with a system above 4096 particles: the resident kernel
    cannot hold it (NBODY_EUNSUPPORTED), so the tuner skips it and picks one
    of the per-step item modes, which then runs the layout to the oracle's
    accelerations (1e-5 per row)."""
    sizes = [8192, 100, 300]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=28, sizes=sizes)
    tx, tv, tm = dev(x), dev(v), dev(m)
    nb.nbody_set_config(bsplit=0, bpass=4)
    try:
        with pytest.raises(nb.NBodyError) as ei:
            nb.nbody_step_batched(off, epsv, tx.clone(), tv.clone(), torch.empty_like(tx), tm, 1.0 / 512, 1,
                                  precision="fp32c")
        assert ei.value.status == nb.NBODY_EUNSUPPORTED
    finally:
        nb.nbody_set_config()
    for prec, modes in (("fp32c", (3, 4)), ("fp64", (3,))):
        best = nb.nbody_tune_batched(off, epsv, tx, tv, tm, 1.0 / 512, 2, precision=prec, allow_cooperative=False)
        assert best["bsplit"] in modes, (prec, best)
    ta = torch.empty_like(tx)
    nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, 1.0 / 512, 0, precision="fp32c")
    a = ta.cpu().numpy()
    for c in range(len(sizes)):
        s_, e_ = off[c], off[c + 1]
        ref = oracle_mod.accel(x[:, s_:e_], m[s_:e_], eps=float(epsv[c]))
        assert row_rel(a[:, s_:e_], ref).max() <= 1e-5, c


def test_batched_matches_oracle_fp64(nb, oracle_mod):
    sizes = [5, 80, 700]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=17, sizes=sizes)
    dt, steps = 1.0 / 512, 5
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta = torch.empty_like(tx)
    nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, dt, steps, precision="fp64")
    for c in range(len(sizes)):
        s, e = off[c], off[c + 1]
        rx, rv = oracle_mod.kdk(x[:, s:e], v[:, s:e], m[s:e], dt, steps, eps=float(epsv[c]))
        assert np.abs(tx.cpu().numpy()[:, s:e] - rx).max() <= 1e-12
        assert np.abs(tv.cpu().numpy()[:, s:e] - rv).max() <= 1e-12


def test_batched_repeat_and_graph_capture(nb):
    sizes = [64, 257, 1000]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=18, sizes=sizes)
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta = torch.empty_like(tx)
    # eager reference: 3 calls of 2 steps
    ex, ev, ea = tx.clone(), tv.clone(), ta.clone()
    nb.nbody_step_batched(off, epsv, ex, ev, ea, tm, 1.0 / 512, 2, precision="fp32c")
    ref = []
    for _ in range(3):
        nb.nbody_step_batched(off, epsv, ex, ev, ea, tm, 1.0 / 512, 2, precision="fp32c", acc_valid=True)
        ref.append((ex.clone(), ev.clone()))
    # graph: the first call (plan build, a(x)) runs eagerly, then replays
    gx, gv, ga = tx.clone(), tv.clone(), ta.clone()
    nb.nbody_step_batched(off, epsv, gx, gv, ga, tm, 1.0 / 512, 2, precision="fp32c")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
        nb.nbody_step_batched(off, epsv, gx, gv, ga, tm, 1.0 / 512, 2, precision="fp32c", acc_valid=True)
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = (gx.sum() + 1.0).item()  # eager work between replays
        assert torch.equal(gx, ref[k][0]) and torch.equal(gv, ref[k][1]), k


@pytest.mark.parametrize("kind", ["kdk", "kdk_sym", "kdk_sym_one", "kdk_sym64", "hermite6", "hermite6_sym"])
def test_single_system_graph_capture(nb, kind):
    """nbody_step (ordered and symmetric force kernels: FP32C with two
    half-ring launches, whose block-diagonal kernel and slot sums run on the
    library's second stream, or with one, all on the caller's stream; FP64 with
    two) and nbody_step_hermite6 (ordered, and symmetric acceleration + jerk +
    snap with two launches) captured into a HIP graph (after one eager call
    has sized the library's workspace) replay bitwise like eager calls, with
    eager work and synchronisation between the replays."""
    x, v, m = ics.plummer(3001, seed=19)
    dt = 1.0 / 256
    tm = dev(m)

    def state():
        tx, tv = dev(x), dev(v)
        return [tx, tv] + [torch.empty_like(tx) for _ in range(4 if kind.startswith("hermite6") else 1)]

    def call(st, valid):
        if kind == "kdk":
            nb.nbody_step(st[0], st[1], st[2], tm, dt, 2, eps=0.01, precision="fp32c", acc_valid=valid)
        elif kind.startswith("kdk_sym"):
            # two half-ring launches per evaluation, or one
            nb.nbody_set_config(pairs=2, split=1 if kind == "kdk_sym_one" else 2)
            try:
                nb.nbody_step(st[0], st[1], st[2], tm, dt, 2, eps=0.01,
                              precision="fp64" if kind == "kdk_sym64" else "fp32c", acc_valid=valid)
            finally:
                nb.nbody_set_config()
        elif kind == "hermite6_sym":
            # the symmetric acceleration + jerk + snap, two half-ring launches per evaluation
            nb.nbody_set_config(pairs=2, split=2)
            try:
                nb.nbody_step_hermite6(st[0], st[1], *st[2:], tm, dt, 2, eps=0.01, precision="fp32c", acc_valid=valid)
            finally:
                nb.nbody_set_config()
        else:
            nb.nbody_step_hermite6(st[0], st[1], *st[2:], tm, dt, 2, eps=0.01, precision="fp32c", acc_valid=valid)

    eager = state()
    call(eager, False)
    ref = []
    for _ in range(3):
        call(eager, True)
        ref.append([q.clone() for q in eager[:2]])
    graph = state()
    call(graph, False)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
        call(graph, True)
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = (graph[0].sum() + 1.0).item()  # eager work between replays
        assert torch.equal(graph[0], ref[k][0]) and torch.equal(graph[1], ref[k][1]), k


def test_sym_vjp_graph_capture(nb):
    """The symmetric VJP with two half-ring launches (its block-diagonal kernel
    and slot sums on the library's second stream) captured into a HIP graph
    replays bitwise like the eager call, with eager work between replays."""
    x, _, m = ics.plummer(3001, seed=23)
    w = np.random.default_rng(3).standard_normal(x.shape)
    tx, tm, tw = dev(x), dev(m), dev(w)
    nb.nbody_set_config(pairs=2, split=2)
    try:
        rx, rm = nb.nbody_accel_vjp(tx, tm, tw, eps=0.01, precision="fp32c")
        s = torch.cuda.Stream()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
            gx, gm = nb.nbody_accel_vjp(tx, tm, tw, eps=0.01, precision="fp32c")
    finally:
        nb.nbody_set_config()
    for k in range(3):
        gx.zero_()
        gm.zero_()
        g.replay()
        torch.cuda.synchronize()
        _ = (tx.sum() + 1.0).item()  # eager work between replays
        assert torch.equal(gx, rx) and torch.equal(gm, rm), k


def test_abi_rejects_bad_pointers(nb):
    from paper_2605_02744_amd._binding import nbody_params
    import ctypes
    L = nb.load()
    p = nbody_params(1.0, 0.01, nb.NBODY_FP32C, 0)
    x = torch.zeros((3, 100), dtype=torch.float64, device="cuda:0")
    m = torch.ones(100, dtype=torch.float64, device="cuda:0")
    a = torch.empty_like(x)
    host = np.zeros(300)
    # host pointer where device memory is required
    st = L.nbody_accel(100, ctypes.c_void_p(host.ctypes.data), ctypes.c_void_p(m.data_ptr()),
                       ctypes.c_void_p(a.data_ptr()), ctypes.byref(p), None)
    assert st == nb.NBODY_EINVAL
    # misaligned pointer
    st = L.nbody_accel(100, ctypes.c_void_p(x.data_ptr() + 4), ctypes.c_void_p(m.data_ptr()),
                       ctypes.c_void_p(a.data_ptr()), ctypes.byref(p), None)
    assert st == nb.NBODY_EINVAL and b"aligned" in L.nbody_last_error()
    # null output
    st = L.nbody_accel(100, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(m.data_ptr()), None,
                       ctypes.byref(p), None)
    assert st == nb.NBODY_EINVAL
    # aliasing output
    st = L.nbody_accel(100, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(m.data_ptr()),
                       ctypes.c_void_p(x.data_ptr()), ctypes.byref(p), None)
    assert st == nb.NBODY_EINVAL
    # the binding refuses wrong dtype and CPU tensors before the C call
    with pytest.raises(TypeError):
        nb.nbody_accel(x.float(), m, eps=0.01)
    with pytest.raises(ValueError):
        nb.nbody_accel(x.cpu(), m, eps=0.01)


def test_check_finite_flag(nb):
    x, _, m = ics.plummer(200, seed=19)
    x[0, 5] = np.nan
    with pytest.raises(nb.NBodyError) as ei:
        nb.nbody_accel(dev(x), dev(m), eps=0.01, precision="fp64", check_finite=True)
    assert ei.value.status == nb.NBODY_ENONFINITE
    x[0, 5] = 0.1
    a = nb.nbody_accel(dev(x), dev(m), eps=0.01, precision="fp64", check_finite=True)
    assert torch.isfinite(a).all()


def test_tune_records_a_choice(nb, tmp_path, oracle_mod):
    n = 5000
    path = str(tmp_path / "tune.jsonl")
    best = nb.nbody_tune(n, "fp32c", path)
    assert best["ipl"] in (1, 2, 4) and best["split"] >= 1
    import json
    rec = json.loads(open(path).read().splitlines()[-1])
    assert rec["n"] == n and rec["arch"].startswith("gfx950") and rec["trials"]
    x, _, m = ics.plummer(n, seed=20)
    a = nb.nbody_accel(dev(x), dev(m), eps=0.01, precision="fp32c").cpu().numpy()
    assert rel_err(a, oracle_mod.accel(x, m, eps=0.01)) <= 1e-5


# ---- acceleration + jerk (Algorithm 3) and fourth-order Hermite -------------

@pytest.mark.parametrize("n", [2, 65, 1000, 2049])
@pytest.mark.parametrize("prec,tola,tolj", [("fp64", 1e-12, 1e-11), ("fp32c", 1e-5, 1e-4)])
def test_accel_jerk_matches_oracle(nb, oracle_mod, n, prec, tola, tolj):
    x, v, m = ics.plummer(n, seed=50 + n)
    ra, rj = oracle_mod.accel_jerk(x, v, m, G=1.1, eps=0.01)
    a, jk = nb.nbody_accel_jerk(dev(x), dev(v), dev(m), G=1.1, eps=0.01, precision=prec)
    assert rel_err(a.cpu().numpy(), ra) <= tola
    assert rel_err(jk.cpu().numpy(), rj) <= tolj
    # the paper's per-component criterion (0.05 % acceleration, 0.2 % jerk)
    assert np.all(np.abs(jk.cpu().numpy() - rj) <= 2e-3 * np.abs(rj) + 1e-6 * np.abs(rj).max())


def test_accel_jerk_split_configs(nb, oracle_mod):
    x, v, m = ics.plummer(3001, seed=60)
    ra, rj = oracle_mod.accel_jerk(x, v, m, eps=0.01)
    for ipl, split in ((1, 1), (2, 5), (1, 13)):
        nb.nbody_set_config(ipl=ipl, split=split)
        try:
            a, jk = nb.nbody_accel_jerk(dev(x), dev(v), dev(m), eps=0.01, precision="fp64")
        finally:
            nb.nbody_set_config()
        assert rel_err(a.cpu().numpy(), ra) <= 1e-12
        assert rel_err(jk.cpu().numpy(), rj) <= 1e-11


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32c", 1e-6)])
def test_hermite_matches_oracle(nb, oracle_mod, prec, tol):
    x, v, m = ics.plummer(1024, seed=61)
    dt, steps, eps = 1.0 / 256, 8, 0.01
    rx, rv = oracle_mod.hermite4(x, v, m, dt, steps, eps=eps)
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta, tj = torch.empty_like(tx), torch.empty_like(tx)
    nb.nbody_step_hermite(tx, tv, ta, tj, tm, dt, steps, eps=eps, precision=prec)
    assert np.abs(tx.cpu().numpy() - rx).max() <= tol
    assert np.abs(tv.cpu().numpy() - rv).max() <= 10 * tol


def test_hermite_resumable_bitwise(nb):
    x, v, m = ics.plummer(700, seed=62)
    out = []
    for chunks in ((6,), (2, 4)):
        tx, tv, tm = dev(x), dev(v), dev(m)
        ta, tj = torch.empty_like(tx), torch.empty_like(tx)
        valid = False
        for c in chunks:
            nb.nbody_step_hermite(tx, tv, ta, tj, tm, 1.0 / 128, c, eps=0.01, precision="fp32c", acc_valid=valid)
            valid = True
        out.append((tx.cpu(), tv.cpu()))
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
