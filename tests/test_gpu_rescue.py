"""The FP64 rescue of ill-conditioned FP32C rows (nbody_config.rescue).

FP32C rows keep a rounding error of a few u (u = 2^-24) per term, and the
position rounding of strong pairs just outside the near-field radius; where a
row's terms cancel, that error grows against |a_i|.  Softened Plummer spheres
of 4096 bodies with eps = 0.04 / sqrt(4096) = 6.25e-4 -- the largest clusters
of the 512-cluster ensemble workload -- have such rows: without the rescue the
seeds below reach 1.1e-5 to 4.1e-5 (per-row relative error against FP64).  The
kernels' error estimate flags them and the rescue recomputes them in FP64, so
the force meets the FP32C bound of 1e-5 per row against the oracle, in the
ordered and the symmetric single-system kernels and in the batched per-step
wave items.
"""
import numpy as np
import pytest

import ics
from parity_stats import row_rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SEEDS = [5001, 5010, 5054, 5066, 5150]
EPS = 0.04 / 64.0


@pytest.fixture(scope="module")
def nb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_02744_amd as nbm
    nbm.load()
    return nbm


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def accel(nb, x, m, pairs, rescue):
    nb.nbody_set_config(pairs=pairs, rescue=rescue)
    try:
        return nb.nbody_accel(dev(x), dev(m), eps=EPS, precision="fp32c").cpu().numpy()
    finally:
        nb.nbody_set_config()


@pytest.mark.parametrize("pairs", [1, 2])
def test_rescue_small_softening_clusters(nb, oracle_mod, pairs):
    """Every row within 1e-5 of the oracle with the rescue (the default), in
    the ordered (pairs = 1) and the symmetric (pairs = 2) kernel; without it
    the ordered kernel exceeds 1e-5 on these inputs."""
    worst_on = worst_off = 0.0
    for seed in SEEDS:
        x, _, m = ics.plummer(4096, seed=seed)
        ref = oracle_mod.accel(x, m, eps=EPS)
        e_on = row_rel(accel(nb, x, m, pairs, 0), ref).max()
        e_off = row_rel(accel(nb, x, m, pairs, 2), ref).max()
        print("seed %d pairs %d: rescue %.2e, without %.2e" % (seed, pairs, e_on, e_off), flush=True)
        worst_on, worst_off = max(worst_on, e_on), max(worst_off, e_off)
    assert worst_on <= 1e-5
    if pairs == 1:
        assert worst_off > 1e-5


def test_rescue_repeat_bitwise(nb):
    """The flagged rows are listed in whatever order the flags arrive, but each
    row is recomputed on its own in a fixed order: repeated calls agree
    bitwise, and the rescue changed some rows."""
    x, _, m = ics.plummer(4096, seed=SEEDS[-1])
    a1 = accel(nb, x, m, 0, 0)
    a2 = accel(nb, x, m, 0, 0)
    a0 = accel(nb, x, m, 0, 2)
    assert np.array_equal(a1, a2)
    assert np.any(a1 != a0)


def _layout():
    xs, ms = [], []
    for seed in SEEDS:
        x, _, m = ics.plummer(4096, seed=seed)
        xs.append(x)
        ms.append(m)
    xs.append(ics.plummer(300, seed=3)[0])
    ms.append(ics.plummer(300, seed=3)[2])
    sizes = [q.shape[0] for q in ms]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    epsv = np.array([EPS] * len(SEEDS) + [0.04 / 300 ** 0.5])
    return off, epsv, np.concatenate(xs, axis=1), np.concatenate(ms)


@pytest.mark.parametrize("mode", [3, 4])
def test_rescue_batched_per_step_items(nb, oracle_mod, mode):
    """The batched per-step items, ordered (mode 3) and symmetric (mode 4, the
    FP32C default on this layout), with the rescue: a(x) of every system within
    1e-5 of the oracle, and some rows recomputed in FP64 (within 1e-12 of the
    oracle, which no FP32C row comes near); without the rescue no row is, and
    in mode 3 some row exceeds 1e-5."""
    off, epsv, x, m = _layout()
    worst, exact = {}, {}
    for rescue in (0, 2):
        tx, tv, tm = dev(x), dev(np.zeros_like(x)), dev(m)
        ta = torch.empty_like(tx)
        print("batched mode %d rescue %d" % (mode, rescue), flush=True)
        nb.nbody_set_config(bsplit=mode, rescue=rescue)
        try:
            nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, 1.0 / 512, 0, precision="fp32c", check_finite=True)
        finally:
            nb.nbody_set_config()
        a = ta.cpu().numpy()
        err = np.concatenate([row_rel(a[:, off[c]:off[c + 1]],
                                      oracle_mod.accel(x[:, off[c]:off[c + 1]], m[off[c]:off[c + 1]],
                                                       eps=float(epsv[c])))
                              for c in range(len(epsv))])
        worst[rescue], exact[rescue] = err.max(), int((err < 1e-12).sum())
    print("batched mode %d: rescue %.2e (%d rows in FP64), without %.2e" % (mode, worst[0], exact[0], worst[2]))
    assert worst[0] <= 1e-5
    assert exact[0] > 0 and exact[2] == 0
    if mode == 3:
        assert worst[2] > 1e-5


def test_rescue_batched_explicit_needs_per_step_items(nb):
    """rescue = 1 (asked for explicitly) with a batched mode that has no rescue
    (the resident kernel, mode 0) is refused; rescue = 0 (automatic) runs such a
    mode without it."""
    off, epsv, x, m = _layout()
    tx, tv, tm = dev(x), dev(np.zeros_like(x)), dev(m)
    ta = torch.empty_like(tx)
    nb.nbody_set_config(bsplit=0, bpass=4, rescue=1)  # bpass forces the resident kernel
    try:
        with pytest.raises(nb.NBodyError) as ei:
            nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, 1.0 / 512, 0, precision="fp32c")
        assert ei.value.status == nb.NBODY_EUNSUPPORTED
    finally:
        nb.nbody_set_config()
    nb.nbody_set_config(bsplit=0, bpass=4)
    try:
        nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, 1.0 / 512, 0, precision="fp32c", check_finite=True)
    finally:
        nb.nbody_set_config()


@pytest.mark.parametrize("mode", [3, 4])
def test_rescue_batched_graph_replays(nb, mode):
    """Two steps of the batched per-step items (ordered and symmetric) with the
    rescue captured in a HIP graph and replayed three times, with eager work
    between the replays: every replay equals the eager run from the same state
    (the flag counts are cleared by a kernel, not a memset)."""
    print("graph replays, batched mode %d" % mode, flush=True)
    nb.nbody_set_config(bsplit=mode)
    try:
        _graph_replays(nb)
    finally:
        nb.nbody_set_config()


def _graph_replays(nb):
    off, epsv, x, m = _layout()
    v = np.random.default_rng(1).standard_normal(x.shape) * 0.1
    tm = dev(m)
    ex, ev = dev(x), dev(v)
    ea = torch.empty_like(ex)
    nb.nbody_step_batched(off, epsv, ex, ev, ea, tm, 1.0 / 512, 0, precision="fp32c")
    gx, gv, ga = ex.clone(), ev.clone(), ea.clone()
    nb.nbody_step_batched(off, epsv, ex, ev, ea, tm, 1.0 / 512, 2, precision="fp32c", acc_valid=True)
    ref = (ex.cpu().numpy(), ev.cpu().numpy(), ea.cpu().numpy())
    sx, sv, sa = gx.clone(), gv.clone(), ga.clone()
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        nb.nbody_step_batched(off, epsv, gx, gv, ga, tm, 1.0 / 512, 2, precision="fp32c", acc_valid=True)
    for rep in range(3):
        gx.copy_(sx)
        gv.copy_(sv)
        ga.copy_(sa)
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(gx.cpu().numpy(), ref[0]) and np.array_equal(gv.cpu().numpy(), ref[1]), rep
        assert np.array_equal(ga.cpu().numpy(), ref[2]), rep
        # eager work between the replays
        nb.nbody_accel(dev(x[:, :4096]), dev(m[:4096]), eps=EPS, precision="fp32c")
        torch.cuda.synchronize()
