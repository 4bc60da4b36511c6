"""nbody_finalize releases the library's device state (workspaces, batched
plans, its second streams) after waiting for the work in flight; the calls
after it build that state again and reproduce their earlier results bitwise."""
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
    return torch.tensor(np.ascontiguousarray(a), device="cuda:0")


def _work(nb):
    """One call of each kind that keeps state: the symmetric force with two
    half-ring launches (second stream), the two-stream adjoint sweep, and the
    symmetric batched items (a cached plan)."""
    out = []
    x, v, m = ics.plummer(9000, seed=41)
    tx, tm = dev(x), dev(m)
    nb.nbody_set_config(pairs=2, split=2)
    try:
        out.append(nb.nbody_accel(tx, tm, eps=0.01))
    finally:
        nb.nbody_set_config()
    n, steps, every, dt = 1200, 9, 4, 1.0 / 256
    x, v, m = ics.plummer(n, seed=42)
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta = torch.empty_like(tx)
    ckx, ckv = [], []
    for c in range(-(-steps // every)):
        ckx.append(tx.clone())
        ckv.append(tv.clone())
        nb.nbody_step(tx, tv, ta, tm, dt, min(every, steps - c * every), eps=0.01, precision="fp64", acc_valid=c > 0)
    rng = np.random.default_rng(43)
    out.extend(nb.nbody_traj_grad(torch.stack(ckx), torch.stack(ckv), every, steps, tm, dt,
                                  dev(rng.standard_normal((3, n))), dev(rng.standard_normal((3, n))), eps=0.01))
    off, epsv, x, v, m = ics.ensemble(6, seed=44, sizes=[700, 129, 2000, 64, 1500, 300])
    tx, tv, tm = dev(x), dev(v), dev(m)
    ta = torch.empty_like(tx)
    nb.nbody_step_batched(off, epsv, tx, tv, ta, tm, 1.0 / 512, 5, precision="fp32c")
    out.extend([tx, tv, ta])
    return [o.clone() for o in out]


def test_finalize_then_rebuild(nb):
    ref = _work(nb)
    nb.nbody_finalize()
    nb.nbody_finalize()  # nothing left to release: still fine
    again = _work(nb)
    for k, (a, b) in enumerate(zip(ref, again)):
        assert torch.isfinite(a).all() and torch.equal(a, b), k
    # work enqueued right before the call is waited for, not cut short
    x, v, m = ics.plummer(20000, seed=45)
    tx, tm = dev(x), dev(m)
    a0 = nb.nbody_accel(tx, tm, eps=0.01)
    torch.cuda.synchronize()
    a1 = nb.nbody_accel(tx, tm, eps=0.01)
    nb.nbody_finalize()
    assert torch.equal(a0, a1)
