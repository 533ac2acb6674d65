"""rmhd_step_adjoint_static, the adjoint step for callers that cannot
allocate device memory (its scratch is the library's static per-device
array), against rmhd_step_adjoint with a caller workspace, through the C ABI:
two calls in a row on one device, the second on a smaller grid, so that it
runs over the first call's leftovers in the shared array."""
import numpy as np
import pytest
import torch

from paper_2510_18968_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12     # FP64 parity bar, per field (the two calls run the same kernels)


@pytest.fixture(scope="module")
def R():
    from paper_2510_18968_amd import rmhd
    assert torch.cuda.is_available(), "needs a HIP device"
    return rmhd


def setup(R, w, seed, warm=1):
    """a grid, its metric, and a generic state after `warm` GPU steps, with a
    random cotangent on the interior and a nonzero sigma-bar to add to"""
    g = R.grid_for(w)
    if w.metric is not None:
        g._met = torch.from_numpy(w.metric).cuda()
        g.set_metric(g._met)
    sig = torch.from_numpy(w.sigma).cuda()
    P = torch.from_numpy(w.P.copy()).cuda()
    U = g.prim2con(P)
    for _ in range(warm):
        g.step(w.dt, sig, U, P)
    torch.cuda.synchronize()
    assert g.failures() == 0
    rng = np.random.default_rng(seed)
    I = (slice(None),) + tuple(w.interior)
    Ub = np.zeros((14,) + tuple(w.padded))
    Ub[I] = rng.normal(size=Ub[I].shape)
    return g, sig, U, P, torch.from_numpy(Ub).cuda(), I


def rel(a, b, I):
    """per-field max |a - b| / max |b| over interior cells"""
    a, b = a.cpu().numpy(), b.cpu().numpy()
    if a.ndim == 3:
        a, b = a[None], b[None]
        I = (slice(None),) + tuple(I[1:])
    d = np.abs(a[I] - b[I]).reshape(a.shape[0], -1).max(1)
    s = np.abs(b[I]).reshape(a.shape[0], -1).max(1)
    return d / np.maximum(s, 1e-300)


def test_static_adjoint_matches_workspace_adjoint(R):
    big = W.sheet_batch()                        # 64 x 2048: the differentiable-form batch
    small = W.curved_blob(n=10, recon="weno5")   # then a smaller, curved grid
    cases = []
    for w, seed in ((big, 31), (small, 32)):
        g, sig, U, P, Ub, I = setup(R, w, seed)
        ref_U, ref_s = torch.zeros_like(Ub), torch.full_like(sig, 0.25)
        g.step_adjoint(w.dt, sig, U, P, Ub, ref_U, ref_s)
        torch.cuda.synchronize()
        assert g.failures() == 0
        cases.append((w, g, sig, U, P, Ub, I, ref_U, ref_s))
    # the two static calls back to back: big, then small
    outs = []
    for (w, g, sig, U, P, Ub, I, _, _) in cases:
        Un, sb = torch.zeros_like(Ub), torch.full_like(sig, 0.25)
        g.step_adjoint_static(w.dt, sig, U, P, Ub, Un, sb)
        outs.append((Un, sb))
    torch.cuda.synchronize()
    for (w, g, sig, U, P, Ub, I, ref_U, ref_s), (Un, sb) in zip(cases, outs):
        assert g.failures() == 0
        eU, es = rel(Un, ref_U, I), rel(sb, ref_s, I)
        bitwise = torch.equal(Un, ref_U) and torch.equal(sb, ref_s)
        print(f"[no-alloc] {w.name}: Ubar^n max rel {eU.max():.2e}, sigma-bar {es.max():.2e}, "
              f"bitwise {bitwise}", flush=True)
        assert (eU <= TOL).all() and (es <= TOL).all(), (eU, es)


def test_static_adjoint_rejects_what_it_cannot_hold(R):
    w = W.periodic_box(n=64, steps=1)            # 70^3 padded cells: 217 MB of adjoint scratch
    g = R.grid_for(w)
    sig = torch.from_numpy(w.sigma).cuda()
    P = torch.from_numpy(w.P).cuda()
    U = g.prim2con(P)
    Un, sb = torch.zeros_like(U), torch.zeros_like(sig)
    with pytest.raises(R.RMHDError, match="static scratch holds"):
        g.step_adjoint_static(w.dt, sig, U, P, U, Un, sb)
    w = W.curved_blob(n=10, recon="weno5")
    g = R.grid_for(w)
    met = torch.from_numpy(w.metric).cuda()
    g.set_metric(met)
    sig = torch.from_numpy(w.sigma).cuda()
    P = torch.from_numpy(w.P).cuda()
    U = g.prim2con(P)
    Un, sb = torch.zeros_like(U), torch.zeros_like(sig)
    g.timing(True)
    with pytest.raises(R.RMHDError, match="timing"):
        g.step_adjoint_static(w.dt, sig, U, P, U, Un, sb)
    g.timing(False)
    torch.cuda.synchronize()
