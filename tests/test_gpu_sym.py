"""GPU parity of the symmetric FP32C/FP32 force kernel (each unordered pair
evaluated once and applied to both particles) against the FP64 CPU oracle,
through the C ABI.  Same error statistic and tolerances as the ordered kernel:
max over particles of |a_i - a_i^ref| / |a_i^ref|, 1e-5 for FP32C, 1e-4 for
FP32 (rounded positions, no repair) on inputs without tight pairs.

Sizes cover the block structure of the kernel: blocks of 512 particles, an odd
and an even number of blocks (the half ring of block pairs visits the opposite
block once when the count is even), ragged last blocks, a single block (only
the block with itself), and half rings cut into several launches.
"""
import numpy as np
import pytest

import ics
from parity_stats import cond_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32c": 1e-5, "fp32": 1e-4}


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


def sym_accel(nb, x, m, launches=0, **kw):
    nb.nbody_set_config(pairs=2, split=launches)
    try:
        return nb.nbody_accel(dev(x), dev(m), **kw).cpu().numpy()
    finally:
        nb.nbody_set_config()


@pytest.mark.parametrize("n", [1, 2, 3, 511, 512, 513, 1024, 1025, 1536, 2048, 2500, 4097, 6000])
@pytest.mark.parametrize("prec", ["fp32c", "fp32"])
def test_sym_accel_ragged_sizes(nb, oracle_mod, n, prec):
    x, _, m = ics.plummer(n, seed=300 + n)
    G, eps = 1.2, 0.01
    ref = oracle_mod.accel(x, m, G=G, eps=eps)
    print("sym accel n=%d %s" % (n, prec), flush=True)
    a = sym_accel(nb, x, m, G=G, eps=eps, precision=prec)
    if n == 1:
        assert np.all(a == 0.0)
        return
    e = rel_err(a, ref)
    print("  max rel err %.3e" % e)
    assert e <= TOL[prec]


@pytest.mark.parametrize("n,launches", [(5000, 1), (5000, 2), (5000, 5), (9000, 3), (9000, 9), (20000, 4)])
def test_sym_accel_launch_splits(nb, oracle_mod, n, launches):
    """The half ring cut into several launches (each with its own slot sums)
    gives the oracle's accelerations, and the same bits whatever the cut is
    not promised, but the same values to rounding."""
    x, _, m = ics.two_component(n, seed=41)
    G, eps = 1.0, 0.02
    ref = oracle_mod.accel(x, m, G=G, eps=eps)
    print("sym accel n=%d launches=%d" % (n, launches), flush=True)
    a = sym_accel(nb, x, m, launches=launches, G=G, eps=eps, precision="fp32c")
    e = rel_err(a, ref)
    print("  max rel err %.3e" % e)
    assert e <= TOL["fp32c"]


def test_sym_accel_tight_pairs_near_field(nb, oracle_mod):
    """Tight pairs far from the origin (separations 1e-5 .. 1e-3 at |x| ~ 6):
    the repair must fix the term for both particles of the pair, whichever of
    them is the lane's i and whichever the streamed j."""
    x, _, m = ics.plummer(3000, seed=30)
    x = x + np.array([[3.0], [-2.0], [5.0]])
    rng = np.random.default_rng(30)
    a_idx = rng.choice(1500, 200, replace=False)
    b_idx = 1500 + np.arange(200)
    off = rng.standard_normal((3, 200))
    off *= 10 ** rng.uniform(-5, -3, 200) / np.linalg.norm(off, axis=0)
    x[:, b_idx] = x[:, a_idx] + off
    ref = oracle_mod.accel(x, m, eps=0.01)
    a = sym_accel(nb, x, m, eps=0.01, precision="fp32c")
    e = rel_err(a, ref)
    print("sym tight pairs max rel err %.3e" % e)
    assert e <= TOL["fp32c"]
    a32 = sym_accel(nb, x, m, eps=0.01, precision="fp32")
    assert rel_err(a32, ref) > 10 * TOL["fp32c"]


@pytest.mark.parametrize("n", [700, 1500])
def test_sym_accel_exclude_self_eps_zero(nb, oracle_mod, n):
    x, _, m = ics.random_cloud(n, seed=3)
    ref = oracle_mod.accel(x, m, eps=0.0)
    a = sym_accel(nb, x, m, eps=0.0, precision="fp32c", exclude_self=True)
    assert np.isfinite(a).all()
    assert rel_err(a, ref) <= 10 * TOL["fp32c"]


def test_sym_accel_unequal_masses(nb, oracle_mod):
    """The j-side term uses m_i: masses spread over four decades."""
    x, _, m = ics.plummer(3001, seed=77)
    m = m * 10 ** np.random.default_rng(77).uniform(-2, 2, m.shape)
    ref = oracle_mod.accel(x, m, G=0.7, eps=0.02)
    a = sym_accel(nb, x, m, G=0.7, eps=0.02, precision="fp32c")
    assert rel_err(a, ref) <= TOL["fp32c"]


def test_sym_accel_repeat_bitwise(nb):
    x, _, m = ics.two_component(7000, seed=5)
    runs = [sym_accel(nb, x, m, launches=2, eps=0.01, precision="fp32c") for _ in range(3)]
    for r in runs[1:]:
        assert np.array_equal(r, runs[0])


def test_sym_and_ordered_agree(nb, oracle_mod):
    x, _, m = ics.plummer(50000, seed=8)
    rows = np.random.default_rng(8).choice(50000, 400, replace=False)
    ref = oracle_mod.accel_rows(x, m, rows, eps=0.01)
    nb.nbody_set_config(pairs=1)
    try:
        ao = nb.nbody_accel(dev(x), dev(m), eps=0.01, precision="fp32c").cpu().numpy()
    finally:
        nb.nbody_set_config()
    asym = sym_accel(nb, x, m, eps=0.01, precision="fp32c")
    # the automatic choice at this size (FP32C: from 49152 particles) is the symmetric kernel
    aauto = nb.nbody_accel(dev(x), dev(m), eps=0.01, precision="fp32c").cpu().numpy()
    assert np.array_equal(aauto, asym)
    a64 = nb.nbody_accel(dev(x), dev(m), eps=0.01, precision="fp64").cpu().numpy()
    assert rel_err(asym, a64) <= TOL["fp32c"]
    assert rel_err(ao, a64) <= TOL["fp32c"]
    assert rel_err(asym[:, rows], ref) <= TOL["fp32c"]


def test_sym_fp64_automatic_threshold(nb):
    """The FP64 force runs the symmetric kernel from 8192 particles on (the
    measured crossover) and the ordered one below: the automatic result equals
    the forced form's bitwise on each side."""
    for n, pairs in ((8192, 2), (8191, 1)):
        x, _, m = ics.plummer(n, seed=10)
        nb.nbody_set_config(pairs=pairs)
        try:
            forced = nb.nbody_accel(dev(x), dev(m), eps=0.01, precision="fp64").cpu().numpy()
        finally:
            nb.nbody_set_config()
        auto = nb.nbody_accel(dev(x), dev(m), eps=0.01, precision="fp64").cpu().numpy()
        assert np.array_equal(auto, forced), n


def test_sym_kdk_steps_match_ordered(nb):
    """nbody_step with the symmetric force: the trajectory stays within the
    FP32C force error of the ordered kernel's trajectory."""
    x, v, m = ics.plummer(6000, seed=9)
    out = {}
    for pairs in (1, 2):
        tx, tv = dev(x), dev(v)
        ta = torch.empty_like(tx)
        nb.nbody_set_config(pairs=pairs)
        try:
            nb.nbody_step(tx, tv, ta, dev(m), 1.0 / 256, 8, eps=0.01, precision="fp32c")
        finally:
            nb.nbody_set_config()
        out[pairs] = (tx.cpu().numpy(), tv.cpu().numpy())
    assert np.abs(out[1][0] - out[2][0]).max() <= 1e-9
    assert np.abs(out[1][1] - out[2][1]).max() <= 1e-7


def test_sym_tune_candidate(nb):
    best = nb.nbody_tune(40000, "fp32c")
    assert best["pairs"] in (1, 2)


# ---------------------------------------------------------------- VJP
# (da/dx)^T w and (da/dm)^T w from the symmetric kernel: the pair term changes
# sign under k <-> j (d and u = m_k w_j - m_j w_k both do), so each unordered
# pair serves both particles.  Gated per row on the condition-normalised error
# |g_k - ref_k| / scale_k (scale_k: the sum of the magnitudes of row k's terms,
# from the oracle), with the ordered VJP's bars: 2e-5 for FP32C (the rounding
# bound of a pair just outside the near-field radius), 5e-4 for FP32, 1e-13
# for FP64 (the symmetric FP64 kernel, from 8192 particles by default).

CTOL = {"fp32c": 2e-5, "fp32": 5e-4, "fp64": 1e-13}


def sym_vjp(nb, x, m, w, launches=0, **kw):
    nb.nbody_set_config(pairs=2, split=launches)
    try:
        gx, gm = nb.nbody_accel_vjp(dev(x), dev(m), dev(w), **kw)
        return gx.cpu().numpy(), gm.cpu().numpy()
    finally:
        nb.nbody_set_config()


def vjp_cond(oracle_mod, x, m, w, gx, gm, G=1.0, eps=0.0):
    """Largest per-row condition-normalised errors of gx and gm."""
    rgx, rgm = oracle_mod.accel_vjp(x, m, w, G=G, eps=eps)
    sx, sm = oracle_mod.accel_vjp_scale_rows(x, m, w, np.arange(m.shape[0]), G=G, eps=eps)
    return cond_err(gx, rgx, sx).max(), cond_err(gm, rgm, sm).max()


@pytest.mark.parametrize("n", [2, 511, 513, 1025, 2048, 3001])
@pytest.mark.parametrize("prec", ["fp32c", "fp32", "fp64"])
def test_sym_vjp_matches_oracle(nb, oracle_mod, n, prec):
    x, _, m = ics.two_component(n, seed=11)
    w = np.random.default_rng(n).standard_normal((3, n))
    print("sym vjp n=%d %s" % (n, prec), flush=True)
    gx, gm = sym_vjp(nb, x, m, w, G=0.7, eps=0.02, precision=prec)
    ex, em = vjp_cond(oracle_mod, x, m, w, gx, gm, G=0.7, eps=0.02)
    print("  cond gx %.3e gm %.3e" % (ex, em))
    assert ex <= CTOL[prec] and em <= CTOL[prec]


@pytest.mark.parametrize("n,launches", [(5000, 3), (9000, 9)])
@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_sym_vjp_launch_splits(nb, oracle_mod, n, launches, prec):
    x, _, m = ics.plummer(n, seed=42)
    w = np.random.default_rng(42).standard_normal((3, n))
    print("sym vjp n=%d launches=%d %s" % (n, launches, prec), flush=True)
    gx, gm = sym_vjp(nb, x, m, w, launches=launches, eps=0.01, precision=prec)
    ex, em = vjp_cond(oracle_mod, x, m, w, gx, gm, eps=0.01)
    print("  cond gx %.3e gm %.3e" % (ex, em))
    assert ex <= CTOL[prec] and em <= CTOL[prec]


def test_sym_vjp_tight_pairs_near_field(nb, oracle_mod):
    x, _, m = ics.plummer(2000, seed=31)
    x = x + np.array([[3.0], [-2.0], [5.0]])
    rng = np.random.default_rng(31)
    a_idx = rng.choice(1000, 200, replace=False)
    b_idx = 1000 + np.arange(200)
    off = rng.standard_normal((3, 200))
    off *= 10 ** rng.uniform(-5, -3, 200) / np.linalg.norm(off, axis=0)
    x[:, b_idx] = x[:, a_idx] + off
    w = np.random.default_rng(2).standard_normal(x.shape)
    gx, gm = sym_vjp(nb, x, m, w, eps=0.01, precision="fp32c")
    ex, em = vjp_cond(oracle_mod, x, m, w, gx, gm, eps=0.01)
    print("sym vjp tight pairs cond gx %.3e gm %.3e" % (ex, em))
    assert ex <= CTOL["fp32c"] and em <= CTOL["fp32c"]


def test_sym_vjp_exclude_self_eps_zero(nb, oracle_mod):
    """eps = 0 with the own pair excluded: the unsoftened terms of the closest
    pairs dominate their rows, so the FP32C bar is taken ten times looser."""
    x, _, m = ics.random_cloud(1500, seed=3)
    w = np.random.default_rng(5).standard_normal(x.shape)
    gx, gm = sym_vjp(nb, x, m, w, eps=0.0, precision="fp32c", exclude_self=True)
    assert np.isfinite(gx).all() and np.isfinite(gm).all()
    ex, em = vjp_cond(oracle_mod, x, m, w, gx, gm, eps=0.0)
    print("sym vjp eps=0 cond gx %.3e gm %.3e" % (ex, em))
    assert ex <= 10 * CTOL["fp32c"] and em <= 10 * CTOL["fp32c"]


def test_sym_vjp64_exclude_self_eps_zero(nb, oracle_mod):
    """The FP64 symmetric VJP with eps = 0 (the block-diagonal kernel leaves
    the own pair out): finite, and at the FP64 bar ten times looser for the
    unsoftened closest pairs."""
    x, _, m = ics.random_cloud(1500, seed=3)
    w = np.random.default_rng(5).standard_normal(x.shape)
    gx, gm = sym_vjp(nb, x, m, w, eps=0.0, precision="fp64", exclude_self=True)
    assert np.isfinite(gx).all() and np.isfinite(gm).all()
    ex, em = vjp_cond(oracle_mod, x, m, w, gx, gm, eps=0.0)
    print("sym vjp64 eps=0 cond gx %.3e gm %.3e" % (ex, em))
    assert ex <= 10 * CTOL["fp64"] and em <= 10 * CTOL["fp64"]


@pytest.mark.parametrize("n", [8192, 12289])
def test_sym_vjp64_default_matches_ordered_and_oracle(nb, oracle_mod, n):
    """From 8192 particles the FP64 VJP is the symmetric one by default: it
    repeats bitwise and both it and the ordered FP64 VJP meet the FP64 bar
    against the oracle on sampled rows."""
    x, _, m = ics.two_component(n, seed=8)
    w = np.random.default_rng(8).standard_normal((3, n))
    tx, tm, tw = dev(x), dev(m), dev(w)
    runs = [nb.nbody_accel_vjp(tx, tm, tw, eps=0.01, precision="fp64") for _ in range(2)]
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])
    nb.nbody_set_config(pairs=1)
    try:
        ogx, ogm = nb.nbody_accel_vjp(tx, tm, tw, eps=0.01, precision="fp64")
    finally:
        nb.nbody_set_config()
    rows = np.random.default_rng(n).choice(n, 96, replace=False)
    rows[:2] = [0, n - 1]
    rgx, rgm = oracle_mod.accel_vjp_rows(x, m, w, rows, eps=0.01)
    sx, sm = oracle_mod.accel_vjp_scale_rows(x, m, w, rows, eps=0.01)
    for gx, gm in ((runs[0][0], runs[0][1]), (ogx, ogm)):
        gx, gm = gx.cpu().numpy()[:, rows], gm.cpu().numpy()[rows]
        ex, em = cond_err(gx, rgx, sx).max(), cond_err(gm, rgm, sm).max()
        print("vjp64 n=%d cond gx %.3e gm %.3e" % (n, ex, em))
        assert ex <= CTOL["fp64"] and em <= CTOL["fp64"]


def test_sym_vjp_repeat_bitwise_and_agrees_with_ordered(nb, oracle_mod):
    x, _, m = ics.two_component(6000, seed=6)
    w = np.random.default_rng(6).standard_normal((3, 6000))
    runs = [sym_vjp(nb, x, m, w, launches=2, eps=0.01, precision="fp32c") for _ in range(2)]
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    nb.nbody_set_config(pairs=1)
    try:
        ogx, ogm = nb.nbody_accel_vjp(dev(x), dev(m), dev(w), eps=0.01, precision="fp32c")
    finally:
        nb.nbody_set_config()
    for gx, gm in (runs[0], (ogx.cpu().numpy(), ogm.cpu().numpy())):
        ex, em = vjp_cond(oracle_mod, x, m, w, gx, gm, eps=0.01)
        assert ex <= CTOL["fp32c"] and em <= CTOL["fp32c"]


def test_sym_traj_grad_matches_ordered(nb):
    """The checkpointed adjoint sweep with the symmetric force and VJP gives the
    ordered kernels' gradient to the FP32C tolerance."""
    n, steps, every, dt = 3000, 12, 4, 1.0 / 256
    x, v, m = ics.plummer(n, seed=14)
    tgt = x + 0.01
    out = {}
    for pairs in (1, 2):
        nb.nbody_set_config(pairs=pairs)
        try:
            tx = dev(x).requires_grad_(True)
            tv = dev(v).requires_grad_(True)
            tm = dev(m).requires_grad_(True)
            xT, _ = nb.NBodyTrajectory.apply(tx, tv, tm, dt, steps, every, 1.0, 0.01, "fp32c", "fp32c")
            ((xT - dev(tgt)) ** 2).sum().backward()
            out[pairs] = (tx.grad.cpu().numpy(), tv.grad.cpu().numpy(), tm.grad.cpu().numpy())
        finally:
            nb.nbody_set_config()
    for a, b in zip(out[1], out[2]):
        # per coordinate, relative to the largest component of each kind
        assert np.abs(a - b).max() <= 1e-5 * np.abs(a).max()


# ---------------------------------------------------------------- FP64
# The symmetric FP64 kernel (selected with pairs = 2): the plain FP64 path's
# 1e-12 bar against the oracle.

@pytest.mark.parametrize("n", [1, 2, 511, 513, 1025, 2048, 3001])
def test_sym_accel_fp64_matches_oracle(nb, oracle_mod, n):
    x, _, m = ics.two_component(n, seed=60 + n)
    ref = oracle_mod.accel(x, m, G=0.8, eps=0.01)
    print("sym fp64 n=%d" % n, flush=True)
    a = sym_accel(nb, x, m, G=0.8, eps=0.01, precision="fp64")
    if n == 1:
        assert np.all(a == 0.0)
        return
    e = rel_err(a, ref)
    print("  max rel err %.3e" % e)
    assert e <= 1e-12


@pytest.mark.parametrize("n,launches", [(5000, 3), (9000, 9)])
def test_sym_accel_fp64_launch_splits_and_repeat(nb, oracle_mod, n, launches):
    x, _, m = ics.plummer(n, seed=61)
    ref = oracle_mod.accel(x, m, eps=0.005)
    a1 = sym_accel(nb, x, m, launches=launches, eps=0.005, precision="fp64")
    a2 = sym_accel(nb, x, m, launches=launches, eps=0.005, precision="fp64")
    assert np.array_equal(a1, a2)
    assert rel_err(a1, ref) <= 1e-12


def test_sym_accel_fp64_exclude_self_eps_zero(nb, oracle_mod):
    x, _, m = ics.random_cloud(1500, seed=62)
    ref = oracle_mod.accel(x, m, eps=0.0)
    a = sym_accel(nb, x, m, eps=0.0, precision="fp64", exclude_self=True)
    assert np.isfinite(a).all()
    assert rel_err(a, ref) <= 1e-11


# ---- symmetric acceleration + jerk (Algorithm 3's pair term once per pair) ---

def sym_jerk(nb, x, v, m, launches=2, **kw):
    """nbody_accel_jerk through the symmetric kernel (pairs = 2), the half ring
    in at least `launches` launches where it is that long."""
    nb.nbody_set_config(pairs=2, split=launches)
    try:
        a, jk = nb.nbody_accel_jerk(dev(x), dev(v), dev(m), **kw)
    finally:
        nb.nbody_set_config()
    return a.cpu().numpy(), jk.cpu().numpy()


@pytest.mark.parametrize("n", [1, 2, 511, 513, 1500, 2049, 4113])
@pytest.mark.parametrize("prec,tola,tolj", [("fp32c", 1e-5, 1e-4), ("fp32", 1e-4, 1e-3), ("fp64", 1e-12, 1e-11)])
def test_sym_jerk_matches_oracle(nb, oracle_mod, n, prec, tola, tolj):
    """Per-row acceleration and jerk against the oracle at sizes that span one
    block, a two-block ring seen from one side, odd and even block counts and
    ragged last blocks, G != 1; FP32C also meets the paper's per-component
    jerk criterion (0.2 %, Sec. 4.1)."""
    x, v, m = ics.plummer(n, seed=70 + n)
    ra, rj = oracle_mod.accel_jerk(x, v, m, G=1.1, eps=0.01)
    print("sym jerk n=%d %s" % (n, prec), flush=True)
    a, jk = sym_jerk(nb, x, v, m, G=1.1, eps=0.01, precision=prec)
    assert rel_err(a, ra) <= tola
    assert rel_err(jk, rj) <= tolj
    if prec == "fp32c":
        assert np.all(np.abs(jk - rj) <= 2e-3 * np.abs(rj) + 1e-6 * np.abs(rj).max())


def test_sym_jerk64_exclude_self_eps_zero(nb, oracle_mod):
    """The FP64 symmetric acceleration + jerk without softening, the self pair
    left out (NBODY_EXCLUDE_SELF), at the FP64 bars ten times looser for the
    unsoftened closest pairs."""
    x, v, m = ics.plummer(3000, seed=77)
    ra, rj = oracle_mod.accel_jerk(x, v, m, eps=0.0)
    a, jk = sym_jerk(nb, x, v, m, eps=0.0, precision="fp64", exclude_self=True)
    assert np.isfinite(a).all() and np.isfinite(jk).all()
    assert rel_err(a, ra) <= 1e-11 and rel_err(jk, rj) <= 1e-10


@pytest.mark.parametrize("n", [8192, 10001])
def test_sym_jerk64_default_and_ordered_agree(nb, oracle_mod, n):
    """From 8192 particles the FP64 acceleration + jerk is the symmetric one by
    default: it repeats bitwise, and both it and the ordered FP64 kernel
    (pairs = 1) meet the FP64 bars against the oracle on sampled rows."""
    x, v, m = ics.plummer(n, seed=79)
    tx, tv, tm = dev(x), dev(v), dev(m)
    runs = [nb.nbody_accel_jerk(tx, tv, tm, eps=0.01, precision="fp64") for _ in range(2)]
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])
    nb.nbody_set_config(pairs=1)
    try:
        a1, j1 = nb.nbody_accel_jerk(tx, tv, tm, eps=0.01, precision="fp64")
    finally:
        nb.nbody_set_config()
    rows = np.random.default_rng(n).choice(n, 128, replace=False)
    rows[:2] = [0, n - 1]
    ra, rj = oracle_mod.accel_jerk_rows(x, v, m, rows, eps=0.01)
    for a, jk in ((runs[0][0], runs[0][1]), (a1, j1)):
        a, jk = a.cpu().numpy(), jk.cpu().numpy()
        assert rel_err(a[:, rows], ra) <= 1e-12 and rel_err(jk[:, rows], rj) <= 1e-11


def test_sym_jerk64_hermite_matches_oracle(nb, oracle_mod):
    """Eight FP64 fourth-order Hermite steps with the symmetric FP64
    acceleration + jerk (pairs = 2, two launches per evaluation) against the
    oracle's Hermite run, at the ordered FP64 path's bars."""
    x, v, m = ics.plummer(1024, seed=61)
    dt, steps, eps = 1.0 / 256, 8, 0.01
    rx, rv = oracle_mod.hermite4(x, v, m, dt, steps, eps=eps)
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta, tj = torch.empty_like(tx), torch.empty_like(tx)
    nb.nbody_set_config(pairs=2, split=2)
    try:
        nb.nbody_step_hermite(tx, tv, ta, tj, tm, dt, steps, eps=eps, precision="fp64")
    finally:
        nb.nbody_set_config()
    assert np.abs(tx.cpu().numpy() - rx).max() <= 1e-11
    assert np.abs(tv.cpu().numpy() - rv).max() <= 1e-10


def test_sym_jerk_exclude_self_eps_zero(nb, oracle_mod):
    """Without softening, the self pair left out (NBODY_EXCLUDE_SELF)."""
    x, v, m = ics.plummer(3000, seed=77)
    ra, rj = oracle_mod.accel_jerk(x, v, m, eps=0.0)
    a, jk = sym_jerk(nb, x, v, m, eps=0.0, precision="fp32c", exclude_self=True)
    assert np.isfinite(a).all() and np.isfinite(jk).all()
    assert rel_err(a, ra) <= 1e-5 and rel_err(jk, rj) <= 1e-4


def test_sym_jerk_default_and_ordered_agree(nb, oracle_mod):
    """From 16384 particles the symmetric kernel is the FP32C default: it and
    the ordered kernel (pairs = 1) agree, and both meet the oracle on sampled
    rows."""
    n = 20000
    x, v, m = ics.plummer(n, seed=78)
    tx, tv, tm = dev(x), dev(v), dev(m)
    a2, j2 = [q.cpu().numpy() for q in nb.nbody_accel_jerk(tx, tv, tm, eps=0.01, precision="fp32c")]
    nb.nbody_set_config(pairs=1)
    try:
        a1, j1 = [q.cpu().numpy() for q in nb.nbody_accel_jerk(tx, tv, tm, eps=0.01, precision="fp32c")]
    finally:
        nb.nbody_set_config()
    rows = np.random.default_rng(5).choice(n, 256, replace=False)
    ra, rj = oracle_mod.accel_jerk_rows(x, v, m, rows, eps=0.01)
    for a, jk in ((a2, j2), (a1, j1)):
        assert rel_err(a[:, rows], ra) <= 1e-5 and rel_err(jk[:, rows], rj) <= 1e-4
    assert rel_err(a2, a1) <= 2e-5 and rel_err(j2, j1) <= 2e-4


def test_sym_jerk_hermite_matches_oracle(nb, oracle_mod):
    """Eight fourth-order Hermite steps with the symmetric acceleration + jerk
    (pairs = 2, two launches per evaluation) against the oracle's Hermite run."""
    x, v, m = ics.plummer(1024, seed=61)
    dt, steps, eps = 1.0 / 256, 8, 0.01
    rx, rv = oracle_mod.hermite4(x, v, m, dt, steps, eps=eps)
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta, tj = torch.empty_like(tx), torch.empty_like(tx)
    nb.nbody_set_config(pairs=2, split=2)
    try:
        nb.nbody_step_hermite(tx, tv, ta, tj, tm, dt, steps, eps=eps, precision="fp32c")
    finally:
        nb.nbody_set_config()
    assert np.abs(tx.cpu().numpy() - rx).max() <= 1e-6
    assert np.abs(tv.cpu().numpy() - rv).max() <= 1e-5
