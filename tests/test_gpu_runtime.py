"""Runtime features on the MI355X: recovery iteration histograms, resume from
a saved state, per-kernel timing."""
import numpy as np
import pytest
import torch

from paper_2510_18968_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2510_18968_amd import rmhd
    assert torch.cuda.is_available(), "needs a HIP device"
    return rmhd


def setup(R, w):
    g = R.grid_for(w)
    if w.metric is not None:
        met = torch.from_numpy(w.metric).cuda()
        g.set_metric(met)
    sig = torch.from_numpy(w.sigma).cuda()
    P = torch.from_numpy(w.P).cuda()
    U = g.prim2con(P)
    return g, sig, U, P


@pytest.mark.parametrize("name", ["blob12", "box10", "batch"])
def test_recovery_histograms_count_every_cell(R, name):
    w = {"blob12": W.curved_blob(n=12), "box10": W.periodic_box(n=10),
         "batch": W.sheet_batch(nprob=3, n=96)}[name]
    g, sig, U, P = setup(R, w)
    g.step(w.dt, sig, U, P)
    g.recovery_stats(True)
    for _ in range(2):
        g.step(w.dt, sig, U, P)
    h = g.recovery_stats_read()
    g.recovery_stats(False)
    assert g.failures() == 0
    n = w.n_interior
    for key in ("stage1", "stage2", "final"):
        c = np.array(h[key])
        print(f"[hist] {name} {key}: " + " ".join(f"{i}:{v}" for i, v in enumerate(c) if v), flush=True)
        assert c.sum() == 2 * n
        assert c[31] == 0
    # read zeroes the bins; disabled stats count nothing
    g.step(w.dt, sig, U, P)
    assert sum(sum(v) for v in g.recovery_stats_read().values()) == 0


def test_resume_from_saved_state_is_bitwise(R):
    """N steps == N/2 steps, save (U, P), restore into fresh buffers, N/2 steps"""
    w = W.curved_blob(n=16)
    g, sig, U, P = setup(R, w)
    Ua, Pa = U.clone(), P.clone()
    for _ in range(6):
        g.step(w.dt, sig, Ua, Pa)
    Ub, Pb = U.clone(), P.clone()
    for _ in range(3):
        g.step(w.dt, sig, Ub, Pb)
    saved = (Ub.cpu().numpy().copy(), Pb.cpu().numpy().copy())
    del Ub, Pb
    Uc, Pc = torch.from_numpy(saved[0]).cuda(), torch.from_numpy(saved[1]).cuda()
    for _ in range(3):
        g.step(w.dt, sig, Uc, Pc)
    torch.cuda.synchronize()
    assert g.failures() == 0
    assert torch.equal(Ua, Uc) and torch.equal(Pa, Pc)


def test_timing_classes(R):
    w = W.curved_blob(n=16)
    g, sig, U, P = setup(R, w)
    g.timing(True)
    g.timing_read()
    g.step(w.dt, sig, U, P)
    t = g.timing_read()
    g.timing(False)
    assert t["flux_x"][1] == 2 and t["update_stage2"][1] == 1 and t["update_final"][1] == 1 and t["stage1"][1] == 1
    assert all(v[0] >= 0.0 for v in t.values())
