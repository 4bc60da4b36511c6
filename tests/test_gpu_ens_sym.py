"""GPU parity of the symmetric per-step ensemble (nbody_config.bsplit = 4:
each unordered pair of a system evaluated once, by one wave per block of 64
particles) against the FP64 CPU oracle, through the C ABI.  Same statistic and
tolerances as the single-system kernels: max over particles of
|a_i - a_i^ref| / |a_i^ref|, 1e-5 for FP32C, 1e-4 for FP32.

System sizes cover the block structure: one block (the block with itself only),
two blocks (an even ring whose opposite block is visited from one side), odd
and even block counts, ragged last blocks, and the largest ensemble systems.
"""
import numpy as np
import pytest

import ics

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32c": 1e-5, "fp32": 1e-4}
SIZES = [1, 2, 63, 64, 65, 127, 128, 129, 191, 192, 256, 1000, 1025, 2048, 4096]


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


def run(nb, off, epsv, x, v, m, steps, mode=4, rescue=0, **kw):
    """nbody_step_batched with the batched mode forced; returns (x, v, a) on the host."""
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta = torch.empty_like(tx)
    nb.nbody_set_config(bsplit=mode, rescue=rescue)
    try:
        nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, 1.0 / 512, steps, **kw)
    finally:
        nb.nbody_set_config()
    return tx.cpu().numpy(), tv.cpu().numpy(), ta.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp32c", "fp32"])
def test_ens_sym_accel_matches_oracle(nb, oracle_mod, prec):
    """a(x) of every system (no step taken) against the oracle, G != 1."""
    off, epsv, x, v, m = ics.ensemble(len(SIZES), seed=41, sizes=SIZES)
    print("ens sym accel %s" % prec, flush=True)
    _, _, a = run(nb, off, epsv, x, v, m, 0, G=0.8, precision=prec, check_finite=True)
    for c in range(len(SIZES)):
        s, e = off[c], off[c + 1]
        ref = oracle_mod.accel(x[:, s:e], m[s:e], G=0.8, eps=float(epsv[c]))
        if e - s == 1:
            assert np.all(a[:, s:e] == 0.0)
            continue
        err = rel_err(a[:, s:e], ref)
        assert err <= TOL[prec], (SIZES[c], err)


def test_ens_sym_kdk_matches_oracle(nb, oracle_mod):
    """Five KDK steps against the oracle's KDK, at the bound the ordered modes meet."""
    sizes = [5, 64, 65, 80, 129, 700, 1300]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=23, sizes=sizes)
    dt, steps = 1.0 / 512, 5
    print("ens sym kdk", flush=True)
    tx, tv, _ = run(nb, off, epsv, x, v, m, steps, precision="fp32c", check_finite=True)
    for c in range(len(sizes)):
        s, e = off[c], off[c + 1]
        rx, rv = oracle_mod.kdk(x[:, s:e], v[:, s:e], m[s:e], dt, steps, eps=float(epsv[c]))
        ra = oracle_mod.accel(x[:, s:e], m[s:e], eps=float(epsv[c]))
        tol_v = 1e-5 * dt * steps * max(np.abs(ra).max(), 1e-30)
        dx = np.abs(tx[:, s:e] - rx).max()
        dv = np.abs(tv[:, s:e] - rv).max()
        assert dv <= tol_v and dx <= tol_v * dt * steps, (c, dx, dv, tol_v)


def test_ens_sym_agrees_with_ordered_items(nb, oracle_mod):
    """Mode 4 against the ordered per-step items (mode 3) over six steps.  The
    two sum in different orders, so each is held to the acceleration bound
    (1e-5 of max |a| per system) carried through the steps, twice over."""
    sizes = [4096, 3000, 2048, 700, 257, 64, 1]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=24, sizes=sizes)
    dt, steps = 1.0 / 512, 6
    print("ens sym vs ordered", flush=True)
    o3 = run(nb, off, epsv, x, v, m, steps, mode=3, precision="fp32c", check_finite=True)
    o4 = run(nb, off, epsv, x, v, m, steps, mode=4, precision="fp32c", check_finite=True)
    for c in range(len(sizes)):
        s, e = off[c], off[c + 1]
        ra = oracle_mod.accel(x[:, s:e], m[s:e], eps=float(epsv[c]))
        tol_v = 2e-5 * dt * steps * max(np.abs(ra).max(), 1e-30)
        dv = np.abs(o3[1][:, s:e] - o4[1][:, s:e]).max()
        dx = np.abs(o3[0][:, s:e] - o4[0][:, s:e]).max()
        assert dv <= tol_v and dx <= tol_v * dt * steps, (c, dx, dv, tol_v)


def test_ens_sym_tight_pairs_near_field(nb, oracle_mod):
    """Tight pairs far from the origin in one system of 3000 (separations
    1e-5 .. 1e-3 at |x| ~ 6), beside a small system: the repair must fix the
    term for both particles of each pair, in the ordered block and in block pairs."""
    xa, _, ma = ics.plummer(3000, seed=30)
    xa = xa + np.array([[3.0], [-2.0], [5.0]])
    rng = np.random.default_rng(30)
    same = 64 * np.arange(10) + 10  # partners in the same block of 64
    pool = np.setdiff1d(np.arange(1500), np.concatenate([same, same + 1]))
    pa = np.concatenate([rng.choice(pool, 200, replace=False), same])
    pb = np.concatenate([1500 + np.arange(200), same + 1])
    d = rng.standard_normal((3, pa.size))
    d *= 10 ** rng.uniform(-5, -3, pa.size) / np.linalg.norm(d, axis=0)
    xa[:, pb] = xa[:, pa] + d
    xb, _, mb = ics.plummer(100, seed=31)
    x = np.concatenate([xa, xb], axis=1)
    m = np.concatenate([ma, mb])
    v = np.zeros_like(x)
    off = np.array([0, 3000, 3100], dtype=np.int64)
    epsv = np.array([0.01, 0.004])
    print("ens sym tight pairs", flush=True)
    _, _, a = run(nb, off, epsv, x, v, m, 0, precision="fp32c")
    _, _, a32 = run(nb, off, epsv, x, v, m, 0, precision="fp32")
    ref = oracle_mod.accel(xa, ma, eps=0.01)
    e = rel_err(a[:, :3000], ref)
    print("ens sym tight pairs max rel err %.3e" % e)
    assert e <= TOL["fp32c"]
    assert rel_err(a32[:, :3000], ref) > 10 * TOL["fp32c"]
    assert rel_err(a[:, 3000:], oracle_mod.accel(xb, mb, eps=0.004)) <= TOL["fp32c"]


def test_ens_sym_exclude_self_eps_zero(nb, oracle_mod):
    sizes = [700, 77, 1025]
    off, _, x, v, m = ics.ensemble(len(sizes), seed=25, sizes=sizes)
    eps0 = np.zeros(len(sizes))
    print("ens sym eps0", flush=True)
    _, _, a = run(nb, off, eps0, x, v, m, 0, precision="fp32c", exclude_self=True, check_finite=True)
    for c in range(len(sizes)):
        s, e = off[c], off[c + 1]
        ref = oracle_mod.accel(x[:, s:e], m[s:e], eps=0.0)
        assert rel_err(a[:, s:e], ref) <= 10 * TOL["fp32c"], c


def test_ens_sym_unequal_masses(nb, oracle_mod):
    """The far-side term uses m_i: masses spread over four decades."""
    sizes = [900, 2100]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=44, sizes=sizes)
    m = m * 10 ** np.random.default_rng(44).uniform(-2, 2, m.shape)
    _, _, a = run(nb, off, epsv, x, v, m, 0, G=0.7, precision="fp32c")
    for c in range(len(sizes)):
        s, e = off[c], off[c + 1]
        ref = oracle_mod.accel(x[:, s:e], m[s:e], G=0.7, eps=float(epsv[c]))
        assert rel_err(a[:, s:e], ref) <= TOL["fp32c"], c


def test_ens_sym_repeat_resumable_and_graph(nb):
    """Fixed-order sums: the same state bitwise on a repeat, when the steps are
    split over calls, and on replays of a captured graph."""
    sizes = [300, 77, 1025, 64]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=45, sizes=sizes)
    res = []
    for chunks in ((6,), (6,), (2, 4), (0, 3, 3)):
        tx, tv, tm = dev(x), dev(v), dev(m)
        ta = torch.empty_like(tx)
        valid = False
        nb.nbody_set_config(bsplit=4)
        try:
            for c in chunks:
                nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, 1.0 / 256, c, precision="fp32c", acc_valid=valid)
                valid = True
        finally:
            nb.nbody_set_config()
        res.append((tx.cpu(), tv.cpu()))
    for r in res[1:]:
        assert torch.equal(res[0][0], r[0]) and torch.equal(res[0][1], r[1])
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta = torch.empty_like(tx)
    nb.nbody_set_config(bsplit=4)
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


def test_ens_sym_fp64_runs_ordered_items(nb):
    """FP64 has no symmetric ensemble form: mode 4 runs mode 3, bitwise."""
    sizes = [500, 129]
    off, epsv, x, v, m = ics.ensemble(len(sizes), seed=46, sizes=sizes)
    o3 = run(nb, off, epsv, x, v, m, 3, mode=3, precision="fp64")
    o4 = run(nb, off, epsv, x, v, m, 3, mode=4, precision="fp64")
    for p_, q_ in zip(o3, o4):
        assert np.array_equal(p_, q_)


def test_ens_sym_untuned_default(nb):
    """Without a forced or tuned choice, FP32C runs mode 4 on a layout whose
    systems span several blocks of 64 and mode 3 on one of single-block
    systems, with the FP64 rescue of ill-conditioned rows (the default) and
    without it (bitwise the forced modes' states)."""
    for rescue, sizes, mode in ((0, [4096, 3000, 700, 129], 4), (2, [4096, 3000, 700, 129], 4),
                                (0, [64, 40, 64, 17], 3), (2, [64, 40, 64, 17], 3)):
        off, epsv, x, v, m = ics.ensemble(len(sizes), seed=47, sizes=sizes)
        tx, tv, tm = dev(x), dev(v), dev(m)
        ta = torch.empty_like(tx)
        nb.nbody_set_config(rescue=rescue)
        try:
            nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, 1.0 / 512, 3, precision="fp32c")
        finally:
            nb.nbody_set_config()
        fx, fv, _ = run(nb, off, epsv, x, v, m, 3, mode=mode, rescue=rescue, precision="fp32c")
        assert np.array_equal(tx.cpu().numpy(), fx) and np.array_equal(tv.cpu().numpy(), fv), (rescue, sizes)
