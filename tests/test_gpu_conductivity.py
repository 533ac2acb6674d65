"""Conductivity models and the artificial atmosphere on the MI355X against the
oracle: eq. sigma_evol on the Sec. IV.A shocktube (sigma0 = 1e6, gamma = 6
and 12, the whole run to t = 0.4), eq. dynamo_sigma with the Sec. IV.E
atmosphere (rho_atmo = 1e-3, K = 100, Gamma = 2) on the curved blob, stage
by stage and over several steps, with the atmosphere cells counted."""
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


def ogrid(orc, w):
    return orc.make_grid(w.n, w.active, w.dx, w.bc, w.gamma_ad, recon=w.recon, x0=w.x0, kappa=w.kappa,
                         **w.extra.get("model", {}))


def sigma_max(w):
    m = w.extra.get("model", {})
    return float(m.get("sigma0", 0.0)) if m.get("sigma_model", 0) else float(w.sigma.max())


def gpu_grid(R, w, x_align=0, **kw):
    g = R.grid_for(w, x_align=x_align, **kw)
    met = None
    if w.metric is not None:
        met = g.to_layout(w.metric)
        g.set_metric(met)
    g._met = met
    return g


def run_both(R, orc, w, steps, x_align=0):
    """steps whole steps on both sides, with the atmosphere count of each
    step (GPU counter, oracle status 2)"""
    g = gpu_grid(R, w, x_align)
    P = g.to_layout(w.P)
    U = g.prim2con(P)
    og = ogrid(orc, w)
    Po = w.P.copy()
    Uo = orc.prim2con(og, Po, w.metric)
    st = np.zeros(Po.shape[1:], np.int32)
    I = orc.interior(og)
    counts = []
    for _ in range(steps):
        g.step(w.dt, None, U, P)          # the model sets sigma: no field passed
        assert orc.step(og, w.dt, None, Uo, Po, w.metric, st) == 0
        counts.append((g.atmosphere_cells(), int((st[I] == 2).sum())))
    assert g.failures() == 0
    torch.cuda.synchronize()
    return g.from_layout(U).cpu().numpy(), g.from_layout(P).cpu().numpy(), Uo, Po, I, counts


@pytest.mark.parametrize("gexp", [6.0, 12.0])
def test_shocktube_sigma_of_D_full_run(R, orc, gexp):
    """Sec. IV.A shocktube, sigma = 1e6 D^gamma, dx = 0.0025, 640 steps to
    t = 0.4: the whole run against the oracle"""
    w = W.brio_wu(sigma0=1e6, n=400, sigma_exp=gexp)
    U, P, Uo, Po, I, _ = run_both(R, orc, w, w.steps)
    eU, eP = rel_errors(U, Uo, I, kind="U"), rel_errors(P, Po, I, kind="P")
    report(f"{w.name} {w.steps} steps U", eU, NAMES_U)
    report(f"{w.name} {w.steps} steps P", eP, NAMES_P)
    tol = tolerances(14, TOL, sigma_max(w), w.dt / w.dx[0], 2 * w.steps, t_total=w.steps * w.dt)
    assert (eU <= tol).all() and (eP <= tol).all(), (eU, eP, tol)


def test_gamma_zero_model_equals_the_field(R):
    """sigma0 D^0 = sigma0: bitwise the run with the uniform field"""
    w = W.brio_wu(sigma0=1e6, n=400)
    wm = W.brio_wu(sigma0=1e6, n=400, sigma_exp=0.0)
    out = []
    for ww, sig in ((w, torch.from_numpy(w.sigma).cuda()), (wm, None)):
        g = R.grid_for(ww)
        P = torch.from_numpy(ww.P.copy()).cuda()
        U = g.prim2con(P)
        for _ in range(40):
            g.step(ww.dt, sig, U, P)
        torch.cuda.synchronize()
        assert g.failures() == 0
        out.append((U.clone(), P.clone()))
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])


@pytest.mark.parametrize("recon,x_align", [("weno5", 1), ("mc2", 0)])
def test_dynamo_atmosphere_blob_stagewise(R, orc, recon, x_align):
    """eq. dynamo_sigma + atmosphere on the curved blob: every stage of one
    step against the oracle (stage 1 and 2 solve with sigma of their stage
    state's D, the fluxes with sigma of the stage primitives)"""
    w = W.curved_blob(n=16, recon=recon, atmosphere=True)
    og = ogrid(orc, w)
    g = gpu_grid(R, w, x_align)
    Pn = g.to_layout(w.P)
    Un = g.prim2con(Pn)
    P1, R1 = g.empty(), g.empty(3)
    g.imex_stage(1, w.dt, None, Un, Pn, P1, R_out=R1)
    U2, P2, R2 = g.empty(), g.empty(), g.empty(3)
    g.imex_stage(2, w.dt, None, Un, P1, P2, R_out=R2, R1=R1, U_out=U2)
    U3, P3 = g.empty(), g.empty()
    st = torch.zeros(g.padded, dtype=torch.int32, device="cuda")
    g.imex_stage(3, w.dt, None, Un, P2, P3, R1=R1, R2=R2, U_s=U2, U_out=U3, status=st)
    torch.cuda.synchronize()
    assert g.failures() == 0
    gpu = {k: g.from_layout(v).cpu().numpy() for k, v in dict(P1=P1, R1=R1, U2=U2, P2=P2, R2=R2, U3=U3, P3=P3).items()}
    stg = g.from_layout(st[None])[0].cpu().numpy()
    U0 = orc.prim2con(og, w.P, w.metric)
    s1 = orc.stage1(og, w.dt, None, U0, w.P, w.metric)
    s2 = orc.stage2(og, w.dt, None, U0, s1["P1"], s1["R1"], w.metric)
    s3 = orc.final(og, w.dt, None, U0, s2["F1"], s2["P2"], s1["R1"], s2["R2"], w.metric)
    ref = dict(P1=s1["P1"], R1=s1["R1"], U2=s2["U2"], P2=s2["P2"], R2=s2["R2"], U3=s3["U"], P3=s3["P"])
    I = orc.interior(og)
    natmo = int((s3["status"][I] == 2).sum())
    assert natmo > 0, "the workload must reach the atmosphere"
    assert np.array_equal(stg[I] == 2, s3["status"][I] == 2)
    assert g.atmosphere_cells() == natmo
    escale = float(np.abs(U0[(slice(8, 11),) + I]).max()) / (orc.gamma_imex() * w.dt)
    for key in ("P1", "R1", "U2", "P2", "R2", "U3", "P3"):
        isR = key.startswith("R")
        e = rel_errors(gpu[key], ref[key], I, em=not isR, floor=escale if isR else 0.0,
                       kind=None if isR else key[0])
        report(f"{w.name} {key}", e, NAMES_P if key[0] == "P" else (NAMES_U if key[0] == "U" else None))
        nflux = {"U2": 1, "P2": 1, "R2": 1, "U3": 2, "P3": 2}.get(key, 1)
        tol = tolerances(len(e), TOL, sigma_max(w), w.dt / min(w.dx), nflux, t_total=w.dt)
        assert (e <= tol).all(), (key, e, tol)


def test_dynamo_atmosphere_blob_steps(R, orc):
    """four whole steps with the atmosphere counted in every step"""
    w = W.curved_blob(n=20, recon="weno5", atmosphere=True)
    steps = 4
    U, P, Uo, Po, I, counts = run_both(R, orc, w, steps, x_align=1)
    print(f"[conductivity] atmosphere cells per step (GPU, oracle): {counts}", flush=True)
    assert all(a == b for a, b in counts) and counts[-1][0] > 0
    eU, eP = rel_errors(U, Uo, I, kind="U"), rel_errors(P, Po, I, kind="P")
    report(f"{w.name} {steps} steps U", eU, NAMES_U)
    report(f"{w.name} {steps} steps P", eP, NAMES_P)
    tol = tolerances(14, TOL, sigma_max(w), w.dt / min(w.dx), 2 * steps, t_total=steps * w.dt)
    assert (eU <= tol).all() and (eP <= tol).all(), (eU, eP, tol)


def test_adjoint_rejects_models(R):
    w = W.brio_wu(sigma0=1e3, n=64, sigma_exp=2.0)
    g = R.grid_for(w)
    P = torch.from_numpy(w.P.copy()).cuda()
    U = g.prim2con(P)
    sb = torch.zeros(g.padded, dtype=torch.float64, device="cuda")
    with pytest.raises(R.RMHDError, match="static sigma field"):
        g.step_adjoint(w.dt, sb, U, P, U, torch.zeros_like(U), sb)
