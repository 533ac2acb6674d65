"""Full-size checks on the MI355X, at the sizes and launch configuration the
benchmark times: sampled outputs the oracle computes cell by cell, and
properties that hold at any size."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def bc_image(c, n, g, bc):
    """padded index along one axis -> padded index of its interior image"""
    if g <= c < g + n:
        return c
    if bc == 0:
        return c + n if c < g else c - n
    return g if c < g else g + n - 1


def sample_cells(n, rng, count=24):
    cells = {(n // 2, n // 2, n // 2), (0, 0, 0), (n - 1, n - 1, n - 1), (0, n // 2, n - 1), (n - 1, 1, n // 3),
             (2, n - 2, 1)}
    while len(cells) < count:
        cells.add(tuple(int(v) for v in rng.integers(0, n, 3)))
    return sorted(cells)


@pytest.mark.parametrize("recon", ["weno5", "mc2"])
def test_curved_256_stage2_sampled(R, orc, recon):
    """The 256^3 curved-background workload: stage 1 + stage 2 on the full
    grid on the GPU; the oracle recomputes stage 2 at sampled cells from the
    seeded data (pointwise stage 1 on each sample's cross-shaped stencil,
    then stage 2 on a 7^3 grid whose outer cells are given)."""
    w = W.curved_blob(n=256, recon=recon)
    n, gh = 256, 3
    # GPU: full grid, in the layout the benchmark uses (aligned x rows)
    g = R.grid_for(w, x_align=1)
    met = g.to_layout(w.metric)
    g.set_metric(met)
    sig = g.to_layout(w.sigma)
    P0 = g.to_layout(w.P)
    U0 = g.prim2con(P0)
    P1, R1 = g.empty(), g.empty(3)
    g.imex_stage(1, w.dt, sig, U0, P0, P1, R_out=R1)
    U2, P2, R2 = g.empty(), g.empty(), g.empty(3)
    g.imex_stage(2, w.dt, sig, U0, P1, P2, R_out=R2, R1=R1, U_out=U2)
    torch.cuda.synchronize()
    assert g.failures() == 0
    rng = np.random.default_rng(7)
    cells = sample_cells(n, rng)
    # oracle: pointwise stage 1 on every cell of every sample's cross stencil
    need, where = [], {}
    for (i, j, k) in cells:
        c = np.array([k + gh, j + gh, i + gh])             # (z, y, x) padded
        for ax in range(3):
            for s in range(-3, 4):
                q = c.copy()
                q[ax] += s
                img = tuple(bc_image(int(q[a]), n, gh, 1) for a in range(3))
                if img not in where:
                    where[img] = len(need)
                    need.append(img)
    L = len(need)
    idx = tuple(np.array(need).T)
    lg = orc.make_grid((L, 1, 1), 0, (1.0, 1.0, 1.0), (2, 2, 2), w.gamma_ad, recon=w.recon)
    Pl = np.ascontiguousarray(w.P[(slice(None),) + idx].reshape(14, 1, 1, L))
    Ml = np.ascontiguousarray(w.metric[(slice(None),) + idx].reshape(16, 1, 1, L))
    Sl = np.ascontiguousarray(w.sigma[idx].reshape(1, 1, L))
    Ul = orc.prim2con(lg, Pl, Ml)
    s1 = orc.stage1(lg, w.dt, Sl, Ul, Pl, Ml)
    assert s1["nfail"] == 0
    # oracle stage 2 on a 7^3 grid per sample
    mg = orc.make_grid((1, 1, 1), 7, w.dx, (2, 2, 2), w.gamma_ad, recon=w.recon)
    gpu_sel = [(slice(None), k + gh, j + gh, i + gh) for (i, j, k) in cells]
    U2h, P2h, R2h = (g.from_layout(t).cpu().numpy() for t in (U2, P2, R2))
    errs = {"U2": [], "P2": [], "R2": []}
    for (i, j, k), gs in zip(cells, gpu_sel):
        c = np.array([k + gh, j + gh, i + gh])
        Pm = np.zeros((14, 7, 7, 7))
        Mm = np.zeros((16, 7, 7, 7))
        Sm = np.ones((7, 7, 7))
        Um = np.zeros((14, 7, 7, 7))
        R1m = np.zeros((3, 7, 7, 7))
        Mm[...] = w.metric[(slice(None),) + tuple(c)][:, None, None, None]
        Pm[...] = s1["P1"][:, 0, 0, where[tuple(c)]][:, None, None, None]
        for ax in range(3):
            for s in range(-3, 4):
                q = c.copy()
                q[ax] += s
                img = tuple(bc_image(int(q[a]), n, gh, 1) for a in range(3))
                m = [3, 3, 3]
                m[ax] += s
                m = tuple(m)
                Pm[(slice(None),) + m] = s1["P1"][:, 0, 0, where[img]]
                Mm[(slice(None),) + m] = w.metric[(slice(None),) + tuple(q)]
                Sm[m] = w.sigma[img]
        ci = where[tuple(c)]
        Um[:, 3, 3, 3] = Ul[:, 0, 0, ci]
        R1m[:, 3, 3, 3] = s1["R1"][:, 0, 0, ci]
        s2 = orc.stage2(mg, w.dt, Sm, Um, Pm, R1m, Mm)
        assert s2["nfail"] == 0
        ref = {"U2": s2["U2"][:, 3, 3, 3], "P2": s2["P2"][:, 3, 3, 3], "R2": s2["R2"][:, 3, 3, 3]}
        got = {"U2": U2h[gs], "P2": P2h[gs], "R2": R2h[gs]}
        for key in errs:
            errs[key].append((got[key], ref[key]))
    # R arrays are measured against the size of the E change they encode (oracle values)
    escale = max(float(np.abs(b[8:11]).max()) for a, b in errs["U2"]) / (orc.gamma_imex() * w.dt)
    for key, names in (("U2", NAMES_U), ("P2", NAMES_P), ("R2", ["x", "y", "z"])):
        got = np.array([a for a, b in errs[key]]).T.reshape(-1, 1, 1, len(cells))
        ref = np.array([b for a, b in errs[key]]).T.reshape(-1, 1, 1, len(cells))
        isR = key == "R2"
        e = rel_errors(got, ref, (slice(None),) * 3, em=not isR, floor=escale if isR else 0.0,
                       kind=None if isR else key[0])
        report(f"256^3 {recon} stage 2 sampled {key} ({len(cells)} cells)", e, names)
        tol = tolerances(len(e), 1e-12, float(w.sigma.max()), w.dt / w.dx[0], 1, t_total=w.dt)
        assert (e <= tol).all(), (key, e)


# ------------------------------------------------ whole step at the timed state
RADIUS = 9          # sub-box half width: a step reaches 6 cells (stage 2 and the final stage, 3 each)


def subbox_axis(c, n, bc):
    """Padded indices (3-cell ghost layout) of one axis of the oracle sub-box
    around interior cell c, the sub-box's own boundary condition and the
    sample's index inside it.  Inside the domain the sub-box takes its ghost
    cells from the GPU state (given); near a copy boundary it is aligned to
    the boundary and fills its ghosts the same way the domain does; with
    periodic boundaries it wraps."""
    m = 2 * RADIUS + 1
    if bc == 0:                                   # periodic: wrap, ghosts given
        lo = c - RADIUS
        return np.array([(lo - 3 + t) % n + 3 for t in range(m + 6)]), 2, RADIUS
    if c < RADIUS + 3:                            # aligned to the low boundary
        return np.arange(0, m + 6), 1, c
    if c > n - 1 - RADIUS - 3:                    # aligned to the high boundary
        return np.arange(n - m, n + 6), 1, c - (n - m)
    return np.arange(c - RADIUS, c + RADIUS + 7), 2, RADIUS


def take_subbox(t, desc_off, iz, iy, ix):
    """t[..., iz, iy, ix] of a device tensor in the grid's layout, indices
    in the 3-cell ghost layout"""
    oz, oy, ox = desc_off
    z = torch.as_tensor(iz + oz, device=t.device)
    y = torch.as_tensor(iy + oy, device=t.device)
    x = torch.as_tensor(ix + ox, device=t.device)
    return t[..., z[:, None, None], y[None, :, None], x[None, None, :]].cpu().numpy()


def field_scales(R, g, t, interior):
    """per-field max |t| over interior cells (A25 normalisation; the EM,
    cleaning and charge fields by at least the largest |E| or |B|)"""
    I = (slice(None),) + tuple(interior)
    a = g.from_layout(t)[I].abs().reshape(t.shape[0], -1).amax(1).cpu().numpy()
    a[5:] = np.maximum(a[5:], a[5:11].max())
    return a


def seam_cells(n, rng, count):
    """corners, face centres, the centre, cells on both sides of the x
    sweep's 58-position segment seams and of the 64-cell chunk seams of the
    stage kernels, then random cells"""
    cells = set()
    for i in (0, n - 1):
        for j in (0, n - 1):
            for k in (0, n - 1):
                cells.add((i, j, k))
    h = n // 2
    cells.update({(0, h, h), (n - 1, h, h), (h, 0, h), (h, n - 1, h), (h, h, 0), (h, h, n - 1), (h, h, h)})
    for (j, k) in ((n // 3, n // 5), (n // 2 + 7, n // 4 + 3)):
        r = k * n + j                                     # row index in the x sweep's row sequence
        x = (-(r * (n + 6)) - 3) % 58                     # row-sequence position r (n + 6) + x + 3 = 0 mod 58
        for xx in (x, x + 58):
            for d in (-1, 0):
                if 0 <= xx + d < n:
                    cells.add((xx + d, j, k))
    for xx in (63, 64, 127, 128):
        if xx < n:
            cells.add((xx, n // 2 + 3, n // 3))
    while len(cells) < count:
        cells.add(tuple(int(v) for v in rng.integers(0, n, 3)))
    return sorted(cells)


def whole_step_sampled(R, orc, w, pre_steps, cells, tag):
    """pre_steps IMEX steps of w on the GPU in the benchmark's layout, then
    one more; the oracle repeats that last step on a sub-box around every
    sampled cell, from the GPU's state before it, and both U^{n+1} and
    P^{n+1} at the cell are compared"""
    n = w.n[0]
    g = R.grid_for(w, x_align=1)
    met = None
    if w.metric is not None:
        met = g.to_layout(w.metric)
        g.set_metric(met)
    sig = g.to_layout(w.sigma)
    P = g.to_layout(w.P)
    U = g.prim2con(P)
    for _ in range(pre_steps):
        g.step(w.dt, sig, U, P)
    torch.cuda.synchronize()
    assert g.failures() == 0
    off = R.std_offsets(g.desc)
    boxes = []
    for (i, j, k) in cells:
        ax = [subbox_axis(c, n, w.bc[d]) for d, c in enumerate((i, j, k))]
        ix, iy, iz = ax[0][0], ax[1][0], ax[2][0]
        boxes.append(dict(U=take_subbox(U, off, iz, iy, ix), P=take_subbox(P, off, iz, iy, ix),
                          S=take_subbox(sig, off, iz, iy, ix),
                          M=None if met is None else take_subbox(met, off, iz, iy, ix),
                          bc=tuple(a[1] for a in ax), at=tuple(a[2] for a in ax)))
    g.step(w.dt, sig, U, P)
    torch.cuda.synchronize()
    assert g.failures() == 0
    sU = field_scales(R, g, U, w.interior)
    sP = field_scales(R, g, P, w.interior)
    eU, eP = np.zeros(14), np.zeros(14)
    m = 2 * RADIUS + 1
    for (i, j, k), b in zip(cells, boxes):
        og = orc.make_grid((m, m, m), 7, w.dx, b["bc"], w.gamma_ad, recon=w.recon, kappa=w.kappa)
        Uo, Po = np.ascontiguousarray(b["U"]), np.ascontiguousarray(b["P"])
        M = None if b["M"] is None else np.ascontiguousarray(b["M"])
        assert orc.step(og, w.dt, np.ascontiguousarray(b["S"]), Uo, Po, M) == 0
        ai, aj, ak = b["at"]
        ci = np.array([k + 3, j + 3, i + 3]) + np.array(off)
        ug = U[:, ci[0], ci[1], ci[2]].cpu().numpy()
        pg = P[:, ci[0], ci[1], ci[2]].cpu().numpy()
        eU = np.maximum(eU, np.abs(ug - Uo[:, ak + 3, aj + 3, ai + 3]) / sU)
        eP = np.maximum(eP, np.abs(pg - Po[:, ak + 3, aj + 3, ai + 3]) / sP)
    report(f"{tag} U^(n+1) ({len(cells)} cells)", eU, NAMES_U)
    report(f"{tag} P^(n+1) ({len(cells)} cells)", eP, NAMES_P)
    tol = tolerances(14, 1e-12, float(w.sigma.max()), w.dt / min(w.dx), 2, t_total=w.dt)
    assert (eU <= tol).all() and (eP <= tol).all(), (eU, eP, tol)


@pytest.mark.parametrize("recon", ["weno5", "mc2"])
def test_curved_256_whole_step_at_timed_state(R, orc, recon):
    """The state the benchmark times (256^3 curved blob after 10 IMEX steps,
    aligned layout): one more full step (stage 1, stage 2, final update and
    recovery) on the GPU against the oracle's step of each sampled cell's
    sub-box, taken from the GPU state (eq. IMEX3, Sec. III.B)."""
    w = W.curved_blob(n=256, recon=recon)
    cells = seam_cells(256, np.random.default_rng(11), 32)
    whole_step_sampled(R, orc, w, 10, cells, f"256^3 {recon} step 11")


def test_periodic_box_128_whole_step(R, orc):
    """The 128^3 periodic box: its first IMEX step on the GPU against the
    oracle's step of wrapped sub-boxes around sampled cells, including the
    seams of the y/z sweep segments (32 rows at this size)."""
    w = W.periodic_box(n=128)
    cells = seam_cells(128, np.random.default_rng(12), 26)
    cells += [(40, 31, 70), (40, 32, 70), (90, 77, 63), (90, 77, 64)]
    whole_step_sampled(R, orc, w, 0, sorted(set(cells)), "128^3 periodic step 1")


def test_periodic_box_128_conservation(R):
    """The 128^3 periodic box, 10 IMEX steps: the totals of D, S_i, tau,
    B^i and Q (no sources in flat space, flux form) are conserved."""
    w = W.periodic_box(n=128)
    g = R.grid_for(w, x_align=1)
    sig = g.to_layout(w.sigma)
    P = g.to_layout(w.P)
    U = g.prim2con(P)
    I = (slice(None),) + tuple(w.interior)
    U0 = g.from_layout(U)[I].cpu().numpy().astype(np.float64)
    for _ in range(w.steps):
        g.step(w.dt, sig, U, P)
    torch.cuda.synchronize()
    assert g.failures() == 0
    U1 = g.from_layout(U)[I].cpu().numpy()
    for f in (0, 1, 2, 3, 4, 5, 6, 7, 13):
        a, b = U0[f].sum(), U1[f].sum()
        scale = np.abs(U0[f]).sum() + np.abs(U1[f]).sum()
        print(f"[conservation] {NAMES_U[f]}: {a:.17e} -> {b:.17e} rel {abs(a - b) / scale:.2e}", flush=True)
        assert abs(a - b) <= 1e-13 * scale


def test_curved_256_round_trip_after_evolution(R):
    """con2prim(prim2con(P)) = P at full size on the state after 5 steps,
    from a perturbed guess (Sec. III.B recovery, E fixed)."""
    w = W.curved_blob(n=256)
    g = R.grid_for(w, x_align=1)
    met = g.to_layout(w.metric)
    g.set_metric(met)
    sig = g.to_layout(w.sigma)
    P = g.to_layout(w.P)
    U = g.prim2con(P)
    for _ in range(5):
        g.step(w.dt, sig, U, P)
    Ut = g.prim2con(P)
    guess = P.clone()
    guess[1] *= 1.05
    guess[2:5] *= 0.9
    st = torch.zeros(g.padded, dtype=torch.int32, device="cuda")
    g.con2prim(Ut, guess, st)
    torch.cuda.synchronize()
    assert g.failures() == 0
    I = tuple(w.interior)
    assert int((g.from_layout(st)[I] != 0).sum()) == 0
    e = rel_errors(g.from_layout(guess).cpu().numpy(), g.from_layout(P).cpu().numpy(), I, kind="P")
    report("256^3 round trip after 5 steps", e, NAMES_P)
    assert e.max() <= 1e-12


@pytest.mark.parametrize("name", ["box16", "blob24"])
def test_mixed_precision_vs_oracle(R, orc, name):
    """Mixed form (FP32 reconstruction, HLLE and divergence; FP64 recovery
    and state) against the FP64 oracle: per-field L1 and Linf relative
    errors of rho, p, B, E at most 1e-5."""
    w = {"box16": W.periodic_box(n=16), "blob24": W.curved_blob(n=24)}[name]
    steps = 5
    g = R.grid_for(w, precision="mixed")
    if w.metric is not None:
        met = dev(w.metric)
        g.set_metric(met)
    sig = dev(w.sigma)
    P = dev(w.P)
    U = g.prim2con(P)
    for _ in range(steps):
        g.step(w.dt, sig, U, P)
    torch.cuda.synchronize()
    assert g.failures() == 0
    og = orc.make_grid(w.n, w.active, w.dx, w.bc, w.gamma_ad, recon=w.recon, x0=w.x0)
    Po = w.P.copy()
    Uo = orc.prim2con(og, Po, w.metric)
    for _ in range(steps):
        assert orc.step(og, w.dt, w.sigma, Uo, Po, w.metric) == 0
    I = orc.interior(og)
    Pg = P.cpu().numpy()
    worst = 0.0
    # E is normalised by the electromagnetic scale max(|E|, |B|): in the
    # stiff interior E is slaved to -v x B and can be orders below |B|
    em_max = max(np.abs(Po[5:11][(slice(None),) + I]).max(), 1e-300)
    em_sum = max(np.abs(Po[5:11][(slice(None),) + I]).sum(axis=(1, 2, 3)).max(), 1e-300)
    for f in (0, 1, 5, 6, 7, 8, 9, 10):
        a, b = Po[f][I], Pg[f][I]
        d = np.abs(a - b)
        l1 = d.sum() / max(np.abs(a).sum(), em_sum if f >= 8 else 1e-300)
        li = d.max() / max(np.abs(a).max(), em_max if f >= 8 else 1e-300)
        print(f"[mixed] {name} {NAMES_P[f]}: L1 {l1:.2e} Linf {li:.2e}", flush=True)
        worst = max(worst, l1, li)
    assert worst <= 1e-5


@pytest.mark.slow
def test_sheet_inversion_64x2048_gradient(R):
    """The 64 x 2048 batch of current sheets, 200 steps, checkpoints every
    20 steps: the loss gradient in (B^y_0, log sigma) from the adjoint
    against central differences (h = 1e-6) along 8 random directions."""
    from test_gpu_adjoint import inversion_fd_check
    w = W.sheet_batch()
    worst, L, gB, gs = inversion_fd_check(R, w, ckpt=20, ndir=8)
    print(f"[rollout] 64x2048 loss {L:.6e} worst rel {worst:.2e}", flush=True)
    assert worst <= 1e-6


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_curved_256_steps_bitwise_reproducible(R, precision):
    """Three full IMEX steps of the 256^3 workload in the benchmark's layout,
    twice from the same inputs: bitwise identical states (every ring read of
    the y/z sweeps waits for its row; no atomics touch the state)."""
    w = W.curved_blob(n=256)
    out = []
    for _ in range(2):
        g = R.grid_for(w, precision=precision, x_align=1)
        g.set_metric(g.to_layout(w.metric))
        sig = g.to_layout(w.sigma)
        P = g.to_layout(w.P)
        U = g.prim2con(P)
        for _ in range(3):
            g.step(w.dt, sig, U, P)
        torch.cuda.synchronize()
        assert g.failures() == 0
        out.append((g.from_layout(U).cpu(), g.from_layout(P).cpu()))
        del g, U, P, sig
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
