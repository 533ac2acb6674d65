"""rmhd_steps: n steps in one call, where each final update also runs the
next step's stage 1 (eq. 3D_NR on U^{n+1} guessed from P^{n+1}, Sec. III.B),
must give what n calls of rmhd_step give: the same recovery on the same
inputs.  The compiler may contract the fused kernel's arithmetic into FMAs
differently, so the bar is the parity bar (the recovery's result moves by
rounding only), the failure and atmosphere counts must be equal and the
recovery iteration histograms equal up to a few cells that sit at a
stopping threshold (at most 0.1%).  Covered: the flat and the diagonal and general curved metrics, the
three reconstructions, stiff 1D shocktubes with a field and a model sigma,
the atmosphere, two active dimensions, the mixed form, the 64x2048 batch
(more chunks than stage blocks, so waves walk several) and the 256^3 blob.
One case is also compared with the oracle directly."""
import numpy as np
import pytest
import torch

from paper_2510_18968_amd import workloads as W
from parity_util import NAMES_P, NAMES_U, rel_errors, report, tolerances

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2510_18968_amd import rmhd
    assert torch.cuda.is_available(), "needs a HIP device"
    return rmhd


def model_of(w):
    return w.extra.get("model", {})


def prepare(R, w, x_align, precision):
    g = R.grid_for(w, x_align=x_align, precision=precision)
    if w.metric is not None:
        g.set_metric(g.to_layout(w.metric))
    sig = None if model_of(w).get("sigma_model", 0) else g.to_layout(w.sigma)
    return g, sig


def run(R, w, steps, fused, x_align=0, precision="fp64"):
    g, sig = prepare(R, w, x_align, precision)
    P = g.to_layout(w.P)
    U = g.prim2con(P)
    g.recovery_stats(True)
    if fused:
        g.steps(w.dt, sig, U, P, steps)
    else:
        for _ in range(steps):
            g.step(w.dt, sig, U, P)
    torch.cuda.synchronize()
    h = g.recovery_stats_read()
    counts = (g.failures(), g.atmosphere_cells(), tuple(h["stage1"] + h["stage2"] + h["final"]))
    g.recovery_stats(False)
    return U, P, counts


CASES = {
    "blob20_weno5": (lambda: W.curved_blob(n=20, recon="weno5"), 4, 1, "fp64"),
    "blob16_shift_mc2": (lambda: W.curved_blob(n=16, recon="mc2", shift=0.05), 3, 0, "fp64"),
    "slicing16_weno5": (lambda: W.tilted_slicing(n=16), 3, 0, "fp64"),
    "brio_wu_s1e6": (lambda: W.brio_wu(sigma0=1e6, n=400), 40, 0, "fp64"),
    "brio_wu_power6": (lambda: W.brio_wu(sigma0=1e6, n=400, sigma_exp=6.0), 40, 0, "fp64"),
    "blob20_dynamo_atmo": (lambda: W.curved_blob(n=20, recon="weno5", atmosphere=True), 4, 1, "fp64"),
    "cylexp40_minmod": (lambda: W.cylindrical_explosion(n=40, steps=3), 5, 0, "fp64"),
    "blob20_mixed": (lambda: W.curved_blob(n=20, recon="weno5"), 4, 1, "mixed"),
    "batch64x2048": (lambda: W.sheet_batch(), 4, 0, "fp64"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_steps_equal_repeated_step(R, name):
    make, steps, x_align, prec = CASES[name]
    w = make()
    print(f"[steps] {name}: {steps} steps, x_align {x_align}, {prec}", flush=True)
    Ua, Pa, ca = run(R, w, steps, False, x_align, prec)
    Ub, Pb, cb = run(R, w, steps, True, x_align, prec)
    compare(name, w, steps, x_align, prec, (Ua, Pa, ca), (Ub, Pb, cb))
    if name == "blob20_dynamo_atmo":
        assert ca[1] > 0, "the workload must reach the atmosphere"


def compare(name, w, steps, x_align, prec, a, b):
    (Ua, Pa, ca), (Ub, Pb, cb) = a, b
    assert ca[0] == cb[0] == 0, (ca[0], cb[0])
    assert ca[1] == cb[1], ("atmosphere cells", ca[1], cb[1])
    ha, hb = np.array(ca[2]), np.array(cb[2])
    moved = int(np.abs(ha - hb).sum()) // 2
    print(f"[steps] {name}: bitwise U {torch.equal(Ua, Ub)}, P {torch.equal(Pa, Pb)}; recoveries with another "
          f"iteration count {moved} of {int(ha.sum())}", flush=True)
    if not (torch.equal(Ua, Ub) and torch.equal(Pa, Pb)):
        values(name, w, steps, x_align, prec, Ua, Pa, Ub, Pb)
    assert ha.sum() == hb.sum() and moved <= max(4, ha.sum() // 1000), (moved, ha, hb)


def values(name, w, steps, x_align, prec, Ua, Pa, Ub, Pb):
    g, _ = prepare(R_mod(), w, x_align, prec)
    I = tuple(w.interior)
    ua, ub = g.from_layout(Ua).cpu().numpy(), g.from_layout(Ub).cpu().numpy()
    pa, pb = g.from_layout(Pa).cpu().numpy(), g.from_layout(Pb).cpu().numpy()
    eU, eP = rel_errors(ub, ua, I, kind="U"), rel_errors(pb, pa, I, kind="P")
    report(f"{name} {steps} steps fused vs repeated U", eU, NAMES_U)
    report(f"{name} {steps} steps fused vs repeated P", eP, NAMES_P)
    m = model_of(w)
    smax = float(m.get("sigma0", 0.0)) if m.get("sigma_model", 0) else float(w.sigma.max())
    tol = tolerances(14, 1e-12, smax, w.dt / min(w.dx), 2 * steps, t_total=steps * w.dt)
    assert (eU <= tol).all() and (eP <= tol).all(), (eU, eP, tol)


def R_mod():
    from paper_2510_18968_amd import rmhd
    return rmhd


def test_steps_against_the_oracle(R, orc):
    """four fused steps of the curved blob against four oracle steps"""
    w = W.curved_blob(n=20, recon="weno5")
    steps = 4
    U, P, counts = run(R, w, steps, True, x_align=1)
    assert counts[0] == 0
    og = orc.make_grid(w.n, w.active, w.dx, w.bc, w.gamma_ad, recon=w.recon, x0=w.x0, kappa=w.kappa)
    Po = w.P.copy()
    Uo = orc.prim2con(og, Po, w.metric)
    for _ in range(steps):
        assert orc.step(og, w.dt, w.sigma, Uo, Po, w.metric) == 0
    g, _ = prepare(R, w, 1, "fp64")
    Ug, Pg = g.from_layout(U).cpu().numpy(), g.from_layout(P).cpu().numpy()
    I = orc.interior(og)
    eU, eP = rel_errors(Ug, Uo, I, kind="U"), rel_errors(Pg, Po, I, kind="P")
    report(f"{w.name} {steps} fused steps U", eU, NAMES_U)
    report(f"{w.name} {steps} fused steps P", eP, NAMES_P)
    tol = tolerances(14, 1e-12, float(w.sigma.max()), w.dt / min(w.dx), 2 * steps, t_total=steps * w.dt)
    assert (eU <= tol).all() and (eP <= tol).all(), (eU, eP, tol)


def test_steps_equal_repeated_step_256(R):
    """the 256^3 blob (aligned layout), two steps: the bench's size and launch
    configuration"""
    w = W.curved_blob(n=256, recon="weno5")
    print("[steps] blob256 weno5: 2 steps", flush=True)
    a = run(R, w, 2, False, 1)
    b = run(R, w, 2, True, 1)
    compare("blob256_weno5", w, 2, 1, "fp64", a, b)


def test_steps_argument_checks(R):
    w = W.brio_wu(sigma0=1e3, n=64)
    g, sig = prepare(R, w, 0, "fp64")
    P = g.to_layout(w.P)
    U = g.prim2con(P)
    U0, P0 = U.clone(), P.clone()
    g.steps(w.dt, sig, U, P, 0)
    torch.cuda.synchronize()
    assert torch.equal(U, U0) and torch.equal(P, P0)
    with pytest.raises(R.RMHDError, match="nsteps"):
        g.steps(w.dt, sig, U, P, -1)
    with pytest.raises(R.RMHDError, match="dt"):
        g.steps(0.0, sig, U, P, 2)
