"""GPU (HIP C-ABI library) against the CPU oracle, element by element, on
the same seeded inputs (requires an MI355X)."""
import numpy as np
import pytest
import torch

from paper_2510_18968_amd import workloads as W
from parity_util import NAMES_P, NAMES_U, rel_errors, report, tolerances

pytestmark = pytest.mark.gpu

TOL = 1e-12          # FP64 parity bar (relative, per field)


@pytest.fixture(scope="module")
def R():
    from paper_2510_18968_amd import rmhd
    assert torch.cuda.is_available(), "needs a HIP device"
    return rmhd


def ogrid(orc, w, **kw):
    return orc.make_grid(w.n, w.active, w.dx, w.bc, w.gamma_ad, recon=kw.get("recon", w.recon), x0=w.x0,
                         kappa=w.kappa, speed_mode=w.extra.get("speed_mode", 0))


def ggrid(R, w, x_align=0):
    return R.grid_for(w, x_align=x_align, speed_mode=w.extra.get("speed_mode", 0))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def small_workloads():
    mode1 = W.curved_blob(n=16, recon="mc2", steps=2, shift=0.05)
    mode1.extra["speed_mode"] = 1      # alpha sqrt(gamma^dd) -+ beta^d
    box_mc2 = W.periodic_box(n=12, steps=2)
    box_mc2.recon = W.RECON["mc2"]     # flat 3D MC2: the z sweep runs the stage-2 update
    box_mc2.name = "periodic_box_12^3_mc2"
    return {
        "box12_mc2": box_mc2,
        "shocktube_s1e6": W.shocktube(seed=103, sigma0=1e6),
        "shocktube_s1": W.shocktube(seed=101, sigma0=1.0),
        "box12": W.periodic_box(n=12, steps=2),
        "blob20_weno5": W.curved_blob(n=20, recon="weno5", steps=2),
        "blob20_mc2": W.curved_blob(n=20, recon="mc2", steps=2),
        "blob20_minmod": W.curved_blob(n=20, recon="minmod", steps=2),
        "batch4x128": W.sheet_batch(nprob=4, n=128, steps=3),
        "blob16_shift_weno5": W.curved_blob(n=16, recon="weno5", steps=2, shift=0.05),
        "blob16_shift_mode1": mode1,
        "slicing16_weno5": W.tilted_slicing(n=16, steps=2),
        "slicing32_2d_mc2": W.tilted_slicing(n=32, dims=2, recon="mc2", steps=3),
        "cylexp40_minmod": W.cylindrical_explosion(n=40, steps=3),
    }


@pytest.mark.parametrize("name", ["box12", "blob20_weno5", "blob16_shift_weno5"])
def test_prim2con_parity(R, orc, name):
    w = small_workloads()[name]
    g = R.grid_for(w)
    og = ogrid(orc, w)
    if w.metric is not None:
        met = dev(w.metric)
        g.set_metric(met)
    U = host(g.prim2con(dev(w.P)))
    Uo = orc.prim2con(og, w.P, w.metric)
    e = rel_errors(U, Uo, orc.interior(og), kind="U")
    report(f"prim2con {name}", e, NAMES_U)
    assert e.max() <= 1e-14


@pytest.mark.parametrize("name", ["box12", "blob20_weno5"])
def test_con2prim_round_trip_parity(R, orc, name):
    """Sec. III.B recovery: the GPU recovers the seeded primitives from the
    oracle's conserved variables and matches the oracle's own recovery."""
    w = small_workloads()[name]
    g = R.grid_for(w)
    og = ogrid(orc, w)
    if w.metric is not None:
        met = dev(w.metric)
        g.set_metric(met)
    Uo = orc.prim2con(og, w.P, w.metric)
    guess = w.P.copy()
    guess[1] *= 1.2
    guess[2:5] *= 0.8
    st = torch.zeros(g.padded, dtype=torch.int32, device="cuda")
    P = host(g.con2prim(dev(Uo), dev(guess), st))
    Po, sto, _, nf = orc.con2prim(og, Uo, guess, w.metric)
    I = orc.interior(og)
    assert nf == 0 and (host(st)[I] == 0).all()
    e = rel_errors(P, Po, I, kind="P")
    report(f"con2prim {name}", e, NAMES_P)
    assert e.max() <= TOL
    assert rel_errors(P, w.P, I, kind="P").max() <= TOL


def stage_chain_gpu(R, w, dt, sigma_np, P0, x_align=0):
    g = ggrid(R, w, x_align)
    met = None
    if w.metric is not None:
        met = g.to_layout(w.metric)
        g.set_metric(met)
    sig = g.to_layout(sigma_np)
    Pn = g.to_layout(P0)
    Un = g.prim2con(Pn)
    P1, R1, U1 = g.empty(), g.empty(3), g.empty()
    g.imex_stage(1, dt, sig, Un, Pn, P1, R_out=R1, U_out=U1)
    U2, P2, R2 = g.empty(), g.empty(), g.empty(3)
    g.imex_stage(2, dt, sig, Un, P1, P2, R_out=R2, R1=R1, U_out=U2)
    U3, P3 = g.empty(), g.empty()
    g.imex_stage(3, dt, sig, Un, P2, P3, R1=R1, R2=R2, U_s=U2, U_out=U3)
    out = {k: host(g.from_layout(v))
           for k, v in dict(U0=Un, P1=P1, R1=R1, U1=U1, U2=U2, P2=P2, R2=R2, U3=U3, P3=P3).items()}
    out["nfail"] = g.failures()
    return out


def stage_chain_oracle(orc, og, w, dt, sigma_np, P0):
    U0 = orc.prim2con(og, P0, w.metric)
    s1 = orc.stage1(og, dt, sigma_np, U0, P0, w.metric)
    s2 = orc.stage2(og, dt, sigma_np, U0, s1["P1"], s1["R1"], w.metric)
    s3 = orc.final(og, dt, sigma_np, U0, s2["F1"], s2["P2"], s1["R1"], s2["R2"], w.metric)
    return dict(U0=U0, P1=s1["P1"], R1=s1["R1"], U1=s1["U1"], U2=s2["U2"], P2=s2["P2"], R2=s2["R2"], U3=s3["U"],
                P3=s3["P"], nfail=s1["nfail"] + s2["nfail"] + s3["nfail"])


@pytest.mark.parametrize("x_align", [0, 1])
@pytest.mark.parametrize("name", list(small_workloads().keys()))
def test_one_step_stagewise_parity(R, orc, name, x_align):
    """Each stage of table imex / eq. IMEX3 (stage 1 implicit, stage 2
    explicit + implicit, final update + recovery) from the same seeded
    primitives: every intermediate matches the oracle, in both x paddings."""
    w = small_workloads()[name]
    og = ogrid(orc, w)
    gpu = stage_chain_gpu(R, w, w.dt, w.sigma, w.P, x_align)
    ref = stage_chain_oracle(orc, og, w, w.dt, w.sigma, w.P)
    assert gpu["nfail"] == 0 and ref["nfail"] == 0
    I = orc.interior(og)
    escale = float(np.abs(ref["U0"][(slice(8, 11),) + tuple(I)]).max()) / (orc.gamma_imex() * w.dt)
    for key in ("U0", "P1", "R1", "U2", "P2", "R2", "U3", "P3"):
        names = NAMES_P if key.startswith("P") else (NAMES_U if key.startswith("U") else ["x", "y", "z"])
        isR = key.startswith("R")
        e = rel_errors(gpu[key], ref[key], I, em=not isR, floor=escale if isR else 0.0, kind=None if isR else key[0])
        report(f"{name} {key}", e, names)
        nflux = {"U2": 1, "P2": 1, "R2": 1, "U3": 2, "P3": 2}.get(key, 1)
        tol = tolerances(len(e), TOL, float(w.sigma.max()), w.dt / min(w.dx), nflux, t_total=w.dt)
        assert (e <= tol).all(), (key, e, tol)


def run_gpu(R, w, steps, x_align=0):
    g = ggrid(R, w, x_align)
    if w.metric is not None:
        met = g.to_layout(w.metric)
        g.set_metric(met)
    sig = g.to_layout(w.sigma)
    P = g.to_layout(w.P)
    U = g.prim2con(P)
    for _ in range(steps):
        g.step(w.dt, sig, U, P)
    nf = g.failures()
    return host(g.from_layout(U)), host(g.from_layout(P)), nf


def run_oracle(orc, w, steps):
    og = ogrid(orc, w)
    P = w.P.copy()
    U = orc.prim2con(og, P, w.metric)
    nf = 0
    for _ in range(steps):
        nf += orc.step(og, w.dt, w.sigma, U, P, w.metric)
    return U, P, nf, og


@pytest.mark.parametrize("name,steps,x_align", [("box12", 2, 0), ("blob20_weno5", 2, 0), ("blob20_mc2", 2, 0),
                                                ("batch4x128", 3, 0), ("shocktube_s1", 20, 0),
                                                ("shocktube_s1e6", 20, 0), ("blob16_shift_weno5", 3, 0),
                                                ("box12", 2, 1), ("blob20_weno5", 2, 1), ("batch4x128", 3, 1),
                                                ("shocktube_s1e6", 20, 1), ("blob16_shift_weno5", 3, 1),
                                                ("blob16_shift_mode1", 3, 1), ("slicing16_weno5", 3, 1),
                                                ("slicing32_2d_mc2", 4, 0), ("cylexp40_minmod", 6, 1),
                                                ("box12_mc2", 3, 1), ("blob20_minmod", 3, 1), ("blob20_mc2", 3, 1),
                                                ("cylexp40_minmod", 6, 0), ("batch64x2048", 3, 1)])
def test_multi_step_parity(R, orc, name, steps, x_align):
    """Several whole steps against the oracle.  batch64x2048 is the full
    64 x 2048 batch: 2048 stage-kernel chunks and 2266 x-sweep segments for
    1024 persistent waves, so every wave walks two or more work items and
    its prefetch of the next one is compared too."""
    w = W.sheet_batch() if name == "batch64x2048" else small_workloads()[name]
    U, P, nf = run_gpu(R, w, steps, x_align)
    Uo, Po, nfo, og = run_oracle(orc, w, steps)
    assert nf == 0 and nfo == 0
    I = orc.interior(og)
    eU, eP = rel_errors(U, Uo, I, kind="U"), rel_errors(P, Po, I, kind="P")
    report(f"{name} {steps} steps U", eU, NAMES_U)
    report(f"{name} {steps} steps P", eP, NAMES_P)
    tol = tolerances(14, TOL, float(w.sigma.max()), w.dt / min(w.dx), 2 * steps, t_total=steps * w.dt)
    assert (eU <= tol).all() and (eP <= tol).all(), (eU, eP, tol)


@pytest.mark.parametrize("seed", [101, 102, 103])
@pytest.mark.parametrize("sigma0", [1.0, 1e3, 1e6])
def test_shocktube_full_run_parity(R, orc, seed, sigma0):
    """The 400-cell resistive Riemann problem (seeded analogue of Sec. IV.A),
    minmod, CFL 0.5, 320 steps to t = 0.4: GPU == oracle at every cell."""
    w = W.shocktube(seed=seed, sigma0=sigma0)
    U, P, nf = run_gpu(R, w, w.steps)
    Uo, Po, nfo, og = run_oracle(orc, w, w.steps)
    assert nf == 0 and nfo == 0
    I = orc.interior(og)
    eU, eP = rel_errors(U, Uo, I, kind="U"), rel_errors(P, Po, I, kind="P")
    report(f"shocktube seed={seed} sigma={sigma0:g} U", eU, NAMES_U)
    report(f"shocktube seed={seed} sigma={sigma0:g} P", eP, NAMES_P)
    tol = tolerances(14, TOL, sigma0, w.dt / w.dx[0], 2 * w.steps, t_total=w.steps * w.dt)
    assert (eU <= tol).all() and (eP <= tol).all(), (eU, eP, tol)


def test_max_signal_speed_parity(R, orc):
    w = W.curved_blob(n=20)
    g = R.grid_for(w)
    met = dev(w.metric)
    g.set_metric(met)
    s = g.max_signal_speed()
    so = orc.max_signal_speed(ogrid(orc, w), w.metric)
    assert abs(s - so) <= 1e-14 * so


def test_deterministic_bitwise(R):
    """No float atomics on the state: two runs are bitwise identical."""
    w = W.periodic_box(n=12, steps=2)
    a = run_gpu(R, w, 2)
    b = run_gpu(R, w, 2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_failure_flags_and_counter(R, orc):
    """Unphysical cells are flagged with the same status as the oracle and
    counted; they never abort the launch."""
    w = W.periodic_box(n=12, steps=1)
    og = ogrid(orc, w)
    Uo = orc.prim2con(og, w.P)
    I = orc.interior(og)
    bad = Uo.copy()
    cells = [(3, 3, 3), (5, 6, 7), (8, 4, 10)]
    bad[4][cells[0]] = -1.0            # tau < 0
    bad[0][cells[1]] = -0.5            # D < 0
    bad[1][cells[2]] = np.nan          # NaN momentum
    g = R.grid_for(w)
    st = torch.zeros(g.padded, dtype=torch.int32, device="cuda")
    g.con2prim(dev(bad), dev(w.P), st)
    nf = g.failures()
    Po, sto, _, nfo = orc.con2prim(og, bad, w.P)
    stg = host(st)
    assert nf == nfo == 3
    assert np.array_equal(stg[I], sto[I])


def test_set_stream_runs_on_the_given_stream(R):
    """rmhd_set_stream: a step launched on a side stream (ordered after the
    default stream's inputs, waited for before the read) gives the default
    stream's result bit for bit."""
    w = small_workloads()["blob20_weno5"]
    g = R.grid_for(w)
    g.set_metric(dev(w.metric))
    sig = dev(w.sigma)
    out = []
    for side in (False, True):
        P = dev(w.P)
        U = g.prim2con(P)
        if side:
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            g.set_stream(s)
            g.step(w.dt, sig, U, P)
            torch.cuda.current_stream().wait_stream(s)
            g.set_stream()
        else:
            g.step(w.dt, sig, U, P)
        out.append((host(U), host(P)))
    assert g.failures() == 0
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
