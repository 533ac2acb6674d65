"""The oracle's forward-mode tangent of one IMEX step (dual numbers through
every function, recovery roots included) against central finite
differences of the oracle step itself (CPU)."""
import numpy as np
import pytest

from paper_2510_18968_amd import workloads as W


def oracle_grid(orc, w):
    return orc.make_grid(w.n, w.active, w.dx, w.bc, w.gamma_ad, recon=w.recon, x0=w.x0, kappa=w.kappa)


@pytest.mark.parametrize("name", ["batch", "blob"])
def test_step_tangent_matches_central_differences(orc, name):
    w = {"batch": W.sheet_batch(nprob=3, n=64), "blob": W.curved_blob(n=8, recon="weno5")}[name]
    g = oracle_grid(orc, w)
    rng = np.random.default_rng(3)
    P0 = w.P.copy()
    U0 = orc.prim2con(g, P0, w.metric)
    I = (slice(None),) + orc.interior(g)
    dU = np.zeros_like(U0)
    dU[I] = rng.normal(size=dU[I].shape) * np.maximum(np.abs(U0[I]), 1e-3)
    dsig = np.zeros_like(w.sigma)
    dsig[I[1:]] = rng.normal(size=dsig[I[1:]].shape) * w.sigma[I[1:]]
    # tangent
    U, P, dUt = U0.copy(), P0.copy(), dU.copy()
    nf, _ = orc.step_tangent(g, w.dt, w.sigma, U, dUt, P, dsigma=dsig, metric=w.metric)
    assert nf == 0
    # central differences; their truncation error falls like h^2 (1e-4: 3e-2,
    # 1e-6: 7e-6, 1e-7: 7e-8 on the batch case), so h = 1e-7
    h = 1e-7
    outs = []
    for sgn in (1, -1):
        Uh, Ph = U0 + sgn * h * dU, P0.copy()
        assert orc.step(g, w.dt, w.sigma + sgn * h * dsig, Uh, Ph, w.metric) == 0
        outs.append(Uh)
    fd = (outs[0] - outs[1]) / (2 * h)
    scale = np.abs(fd[I]).max()
    err = np.abs(dUt[I] - fd[I]).max() / scale
    print(f"[tangent] {name}: max |tangent - FD| / max |FD| = {err:.2e}")
    assert err <= 1e-6
