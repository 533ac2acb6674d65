"""Reverse mode of one IMEX step on the MI355X (rmhd_step_adjoint) against
the oracle's forward mode (dual numbers through its own step): sampled
components of U^n-bar and sigma-bar, a dot-product identity over whole
fields, the prim2con adjoint against central differences of the oracle, and
the differentiable rollout against central differences of the GPU forward."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def ogrid(orc, w, **kw):
    return orc.make_grid(w.n, w.active, w.dx, w.bc, w.gamma_ad, recon=kw.get("recon", w.recon), x0=w.x0,
                         kappa=w.kappa)


def cases():
    return {
        "batch2x48": W.sheet_batch(nprob=2, n=48),
        "shocktube_s1e3": W.shocktube(seed=101, sigma0=1e3, n=64),
        "box8": W.periodic_box(n=8),
        "blob10_weno5": W.curved_blob(n=10, recon="weno5"),
        "blob10_mc2": W.curved_blob(n=10, recon="mc2"),
        "blob10_minmod": W.curved_blob(n=10, recon="minmod"),
    }


def start_state(orc, w, og, warm):
    """The workload's data after `warm` oracle steps (a generic state: the
    seeded data has v = E = 0, where several limiter branches tie)."""
    P = w.P.copy()
    U = orc.prim2con(og, P, w.metric)
    for _ in range(warm):
        assert orc.step(og, w.dt, w.sigma, U, P, w.metric) == 0
    return U, P


def gpu_adjoint(R, w, U, P, Ub):
    g = R.grid_for(w)
    if w.metric is not None:
        met = dev(w.metric)
        g.set_metric(met)
        g._met = met
    sig = dev(w.sigma)
    Ud, Pd, Ubd = dev(U), dev(P), dev(Ub)
    Ubn = torch.zeros_like(Ubd)
    sb = torch.zeros_like(sig)
    g.step_adjoint(w.dt, sig, Ud, Pd, Ubd, Ubn, sb)
    torch.cuda.synchronize()
    assert g.failures() == 0
    return g, host(Ubn), host(sb)


def tangent_dot(orc, og, w, U, P, Ub, dU=None, dsig=None):
    """<Ub, dU^{n+1}> for the input direction (dU, dsig), oracle forward mode"""
    Ut, Pt = U.copy(), P.copy()
    dUt = np.zeros_like(U) if dU is None else dU.copy()
    nf, _ = orc.step_tangent(og, w.dt, w.sigma, Ut, dUt, Pt, dsigma=dsig, metric=w.metric)
    assert nf == 0
    I = (slice(None),) + orc.interior(og)
    return float((Ub[I] * dUt[I]).sum())


# Both sides differentiate the same discrete map in FP64; they differ by the
# rounding of the forward values the derivatives are taken at (parity 1e-12)
# and by the summation order of the adjoint gather.  The sampled comparison
# is relative to max |Ubar^n| over the field (entries can cancel to zero).
TOL = 1e-9


@pytest.mark.parametrize("name", list(cases()))
def test_adjoint_sampled_components(R, orc, name):
    w = cases()[name]
    og = ogrid(orc, w)
    U, P = start_state(orc, w, og, warm=1)
    rng = np.random.default_rng(11)
    I = (slice(None),) + orc.interior(og)
    Ub = np.zeros_like(U)
    Ub[I] = rng.normal(size=Ub[I].shape)
    g, Ubn, sb = gpu_adjoint(R, w, U, P, Ub)
    inter = np.argwhere(np.ones(Ub[0][I[1:]].shape, bool))
    lo = np.array([s.start for s in I[1:]])
    picks = [inter[0], inter[-1], inter[len(inter) // 2]] + [inter[i] for i in rng.integers(0, len(inter), 9)]
    fields = list(range(14))
    worst_u, worst_s = 0.0, 0.0
    scale_u = np.abs(Ubn[I]).max()
    scale_s = max(np.abs(sb[I[1:]]).max(), 1e-300)
    for c in picks:
        cell = tuple(int(v) for v in c + lo)
        for f in rng.choice(fields, 4, replace=False):
            dU = np.zeros_like(U)
            dU[(int(f),) + cell] = 1.0
            ref = tangent_dot(orc, og, w, U, P, Ub, dU=dU)
            err = abs(Ubn[(int(f),) + cell] - ref) / scale_u
            worst_u = max(worst_u, err)
            assert err <= TOL, (name, cell, int(f), Ubn[(int(f),) + cell], ref)
        ds = np.zeros_like(w.sigma)
        ds[cell] = 1.0
        ref = tangent_dot(orc, og, w, U, P, Ub, dsig=ds)
        err = abs(sb[cell] - ref) / scale_s
        worst_s = max(worst_s, err)
        assert err <= TOL, (name, cell, "sigma", sb[cell], ref)
    print(f"[adjoint] {name}: sampled Ubar max err {worst_u:.2e} (scale {scale_u:.2e}), "
          f"sigma-bar max err {worst_s:.2e} (scale {scale_s:.2e})", flush=True)


@pytest.mark.parametrize("name", ["batch2x48", "box8", "blob10_weno5"])
def test_adjoint_dot_product(R, orc, name):
    """<Ubar^{n+1}, J u> + ... = <J^T Ubar^{n+1}, u> + <sigma-bar, s> for
    random whole-field directions (u, s)"""
    w = cases()[name]
    og = ogrid(orc, w)
    U, P = start_state(orc, w, og, warm=1)
    rng = np.random.default_rng(12)
    I = (slice(None),) + orc.interior(og)
    Ub = np.zeros_like(U)
    Ub[I] = rng.normal(size=Ub[I].shape)
    _, Ubn, sb = gpu_adjoint(R, w, U, P, Ub)
    for trial in range(3):
        dU = np.zeros_like(U)
        dU[I] = rng.normal(size=dU[I].shape) * np.maximum(np.abs(U[I]), 1e-3)
        ds = np.zeros_like(w.sigma)
        ds[I[1:]] = rng.normal(size=ds[I[1:]].shape) * w.sigma[I[1:]]
        lhs = tangent_dot(orc, og, w, U, P, Ub, dU=dU, dsig=ds)
        terms = np.concatenate([(Ubn[I] * dU[I]).ravel(), (sb[I[1:]] * ds[I[1:]]).ravel()])
        rhs = float(terms.sum())
        rel = abs(lhs - rhs) / np.abs(terms).sum()
        print(f"[adjoint] {name} dot product {trial}: {lhs:.15e} vs {rhs:.15e} rel {rel:.2e}", flush=True)
        assert rel <= 1e-11


def test_adjoint_aliasing_and_accumulation(R, orc):
    """Ubar_n may alias Ubar_np1; sigma_bar accumulates"""
    w = cases()["blob10_weno5"]
    og = ogrid(orc, w)
    U, P = start_state(orc, w, og, warm=1)
    rng = np.random.default_rng(13)
    I = (slice(None),) + orc.interior(og)
    Ub = np.zeros_like(U)
    Ub[I] = rng.normal(size=Ub[I].shape)
    g, Ubn, sb = gpu_adjoint(R, w, U, P, Ub)
    sig = dev(w.sigma)
    Ud, Pd, Ubd = dev(U), dev(P), dev(Ub)
    sacc = torch.full_like(sig, 0.5)
    g.step_adjoint(w.dt, sig, Ud, Pd, Ubd, Ubd, sacc)
    got, gs = host(Ubd), host(sacc)
    assert np.array_equal(got[I], Ubn[I])
    assert np.array_equal(gs[I[1:]], sb[I[1:]] + 0.5)


@pytest.mark.parametrize("name", ["box8", "blob10_weno5"])
def test_prim2con_adjoint(R, orc, name):
    w = cases()[name]
    og = ogrid(orc, w)
    U, P = start_state(orc, w, og, warm=1)
    g = R.grid_for(w)
    if w.metric is not None:
        met = dev(w.metric)
        g.set_metric(met)
    rng = np.random.default_rng(14)
    I = (slice(None),) + orc.interior(og)
    Ub = np.zeros_like(U)
    Ub[I] = rng.normal(size=Ub[I].shape)
    Pb = host(g.prim2con_adjoint(dev(P), dev(Ub)))
    dP = np.zeros_like(P)
    dP[I] = rng.normal(size=dP[I].shape) * np.maximum(np.abs(P[I]), 1e-3)
    # central differences of the oracle's prim2con; truncation ~ h^2
    h = 1e-6
    Up = orc.prim2con(og, P + h * dP, w.metric)
    Um = orc.prim2con(og, P - h * dP, w.metric)
    lhs = float((Ub[I] * (Up[I] - Um[I])).sum() / (2 * h))
    terms = (Pb[I] * dP[I]).ravel()
    rel = abs(lhs - terms.sum()) / np.abs(terms).sum()
    print(f"[adjoint] prim2con {name}: rel {rel:.2e}", flush=True)
    assert rel <= 1e-8


def test_adjoint_rejects_mixed(R):
    w = W.periodic_box(n=8)
    g = R.grid_for(w, precision="mixed")
    sig = dev(w.sigma)
    P = dev(w.P)
    U = g.prim2con(P)
    with pytest.raises(RuntimeError):
        g.step_adjoint(w.dt, sig, U, P, U.clone(), U.clone(), torch.zeros_like(sig))


def inversion_fd_check(R, w, ckpt, ndir, h=1e-6, seed=21):
    """gradient of the sheet-inversion loss (autograd over the library's
    adjoint) against central differences of the GPU forward, along random
    directions in (B^y_0, log sigma)"""
    from paper_2510_18968_amd.autograd import SheetInversion
    g = R.grid_for(w)
    prob = SheetInversion(w, g, ckpt=ckpt)
    By0 = prob.P0[6].clone().requires_grad_(True)
    ls = torch.tensor(w.extra["sigma_problem"], device="cuda").log().requires_grad_(True)
    L = prob.loss(By0, ls)
    gB, gs = torch.autograd.grad(L, (By0, ls))
    rng = np.random.default_rng(seed)
    I = prob.I[1:]
    worst = 0.0
    with torch.no_grad():
        for k in range(ndir):
            dB = torch.zeros_like(By0)
            dB[I] = dev(rng.normal(size=tuple(dB[I].shape)) * 0.05)
            dls = dev(rng.normal(size=ls.shape))
            Lp = float(prob.loss(By0 + h * dB, ls + h * dls))
            Lm = float(prob.loss(By0 - h * dB, ls - h * dls))
            fd = (Lp - Lm) / (2 * h)
            ad = float((gB * dB).sum() + (gs * dls).sum())
            rel = abs(ad - fd) / max(abs(fd), 1e-300)
            worst = max(worst, rel)
            print(f"[rollout] {w.name} dir {k}: adjoint {ad:.12e} FD {fd:.12e} rel {rel:.2e}", flush=True)
    assert g.failures() == 0
    return worst, float(L), gB, gs


def test_rollout_gradient_matches_fd(R):
    w = W.sheet_batch(nprob=4, n=256, steps=30)
    worst, L, _, _ = inversion_fd_check(R, w, ckpt=7, ndir=3)
    assert L > 0
    assert worst <= 1e-6


def test_rollout_checkpoint_interval_is_exact(R):
    """recomputing segments from checkpoints gives the same gradient bit for
    bit whatever the interval (the forward is deterministic)"""
    from paper_2510_18968_amd.autograd import SheetInversion
    w = W.sheet_batch(nprob=2, n=128, steps=12)
    out = []
    for ckpt in (1, 5, 12):
        g = R.grid_for(w)
        prob = SheetInversion(w, g, ckpt=ckpt)
        By0 = prob.P0[6].clone().requires_grad_(True)
        ls = torch.tensor(w.extra["sigma_problem"], device="cuda").log().requires_grad_(True)
        gB, gs = torch.autograd.grad(prob.loss(By0, ls), (By0, ls))
        out.append((host(gB), host(gs)))
    for gB, gs in out[1:]:
        assert np.array_equal(gB, out[0][0]) and np.array_equal(gs, out[0][1])

