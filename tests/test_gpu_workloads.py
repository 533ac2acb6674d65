"""The paper's 1D and 2D test problems run through the C-ABI library on the
MI355X and compared with the oracle: the circularly polarised Alfven wave
(Sec. IV.D) and the 2D cylindrical explosion (Sec. IV.B)."""
import math

import numpy as np
import pytest
import torch

from paper_2510_18968_amd import workloads as W
from parity_util import NAMES_P, NAMES_U, rel_errors, report, tolerances

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def R():
    from paper_2510_18968_amd import rmhd
    assert torch.cuda.is_available(), "needs a HIP device"
    return rmhd


def gpu_run(R, w, steps, x_align=0):
    g = R.grid_for(w, x_align=x_align)
    sig = g.to_layout(w.sigma)
    P = g.to_layout(w.P)
    U = g.prim2con(P)
    for _ in range(steps):
        g.step(w.dt, sig, U, P)
    torch.cuda.synchronize()
    nf = g.failures()
    return g.from_layout(U).cpu().numpy(), g.from_layout(P).cpu().numpy(), nf


def oracle_run(orc, w, steps):
    og = orc.make_grid(w.n, w.active, w.dx, w.bc, w.gamma_ad, recon=w.recon, x0=w.x0, kappa=w.kappa)
    P = w.P.copy()
    U = orc.prim2con(og, P)
    nf = 0
    for _ in range(steps):
        nf += orc.step(og, w.dt, w.sigma, U, P)
    return U, P, nf, og


def compare(tag, w, steps, gpu, ref, og):
    U, P, nf = gpu
    Uo, Po, nfo, _ = ref
    assert nf == 0 and nfo == 0, (nf, nfo)
    I = og if isinstance(og, tuple) else None
    eU, eP = rel_errors(U, Uo, I, kind="U"), rel_errors(P, Po, I, kind="P")
    report(f"{tag} U", eU, NAMES_U)
    report(f"{tag} P", eP, NAMES_P)
    tol = tolerances(14, TOL, float(w.sigma.max()), w.dt / min(w.dx), 2 * steps, t_total=steps * w.dt)
    assert (eU <= tol).all() and (eP <= tol).all(), (eU, eP, tol)


def test_cp_alfven_one_period(R, orc):
    """eqs. Bi, vyvz, Alf_vel: rho = p = eta_A = 1, B0 = 1.1547, sigma = 1e6,
    MC2, CFL 0.25, periodic.  After one period (t = L/v_A = 2) the GPU equals
    the oracle cell by cell, and the wave is back where it started with an
    error that falls at about second order (Delta x = 1/50, 1/100, 1/200)."""
    errs = []
    for n in (50, 100, 200):
        w = W.cp_alfven(n=n)
        assert abs(w.extra["v_A"] - 0.5) <= 5e-5
        gpu = gpu_run(R, w, w.steps, x_align=1)
        if n <= 100:
            ref = oracle_run(orc, w, w.steps)
            compare(f"cp_alfven {n} one period", w, w.steps, gpu, ref, tuple(w.interior))
        By = gpu[1][6, 0, 0, 3:-3]
        By0 = w.extra["By0"][3:-3]
        errs.append(np.abs(By - By0).sum() / np.abs(By0).sum())
    print(f"[alfven] L1 return error after one period: {errs}", flush=True)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[1] < 0.05 and rates[0] >= 1.4 and rates[1] >= 1.4, (errs, rates)


def test_cylindrical_explosion_200(R, orc):
    """Sec. IV.B at the paper's size: 200 x 200 cells on [-6, 6]^2, two
    active dimensions, minmod, CFL 0.25, sigma = 1e6, to t = 4 (267 steps):
    the GPU equals the oracle at every cell and no recovery fails."""
    w = W.cylindrical_explosion(n=200)
    gpu = gpu_run(R, w, w.steps, x_align=1)
    ref = oracle_run(orc, w, w.steps)
    compare(f"cylindrical explosion 200^2 t=4 ({w.steps} steps)", w, w.steps, gpu, ref, tuple(w.interior))
    P = gpu[1][(slice(None),) + tuple(w.interior)]
    # the blast has swept the centre out and compressed the field in a shell
    assert P[0].min() < 1e-3 and P[5].max() > 0.1


@pytest.mark.parametrize("sigma0", [1e4, 1e6])
def test_cylindrical_explosion_sigma(R, orc, sigma0):
    """Sec. IV.B also runs at sigma = 1e4: 60 steps of the 200^2 explosion at
    both conductivities match the oracle."""
    w = W.cylindrical_explosion(n=200, sigma0=sigma0, steps=60)
    gpu = gpu_run(R, w, w.steps)
    ref = oracle_run(orc, w, w.steps)
    compare(f"cylindrical explosion 200^2 sigma={sigma0:g} 60 steps", w, w.steps, gpu, ref, tuple(w.interior))
