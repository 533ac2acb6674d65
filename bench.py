#!/usr/bin/env python3
"""Benchmark of the resistive GRMHD IMEX-SSP2(2,2,2) stage on one MI355X.

Metric: zone-updates/s per IMEX stage (interior cells x stage-2 applications
per second) on the 256^3 static curved background with a magnetised blob,
FP64, WENO5 + HLLE, after 10 steps of evolution (so that the stiff recovery
does real work).  One timed "step" is one application of IMEX stage 2: ghost
fill, reconstruction, HLLE fluxes, flux divergence + sources + RK combination
and the coupled implicit-E / primitive recovery, i.e. every row of the hot
path.  A full IMEX step (two such flux stages plus the pointwise stage 1) is
timed as well and reported beside it.

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "zone-updates/s per IMEX stage, FP64 vs mixed at 256^3; fwd+adjoint s/step"

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_VECTOR_TFLOPS = 78.6

# Per interior cell and launch of each kernel class on the 256^3 curved WENO5
# workload (zero shift and extrinsic curvature, so the metric read is alpha and
# gamma_ij, 7 words):
#  * algorithmic HBM bytes: each word the kernel must read or write, once;
#  * FP64 flops: executed, from the SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64
#    counters (FMA = 2 flops, 64 lanes per wave instruction);
#  * measured HBM traffic: FETCH_SIZE + WRITE_SIZE of the same launch, scaled by
#    what the counters read for a streaming kernel of known size.
# The flops and traffic figures belong to the kernels as profiled (the file
# names under profiles/ say which); they are re-measured when a kernel changes.
BYTES_PER_CELL = {
    # P 14 + sigma 1 + metric 7 read, rhs 14 written
    "flux_x": 8 * (14 + 1 + 7 + 14),
    # as x, plus the read half of the rhs read-modify-write
    "flux_y": 8 * (14 + 1 + 7 + 14 + 14),
    "flux_z": 8 * (14 + 1 + 7 + 14 + 14),
    # P(1) 7 (p, v and the cleaning fields: the guess and, without K, all the
    # local sources read), U^n 14, rhs 14, R1 3, sigma 1, metric 7 read;
    # U(2) 14, P(2) 14, R2 3 written
    "update_stage2": 8 * (7 + 14 + 14 + 3 + 1 + 7 + 14 + 14 + 3),
    # ghost layers only
    "ghost_fill": 0,
}
FLOPS_PER_CELL = {"flux_x": 2920.5, "flux_y": 2687.0, "flux_z": 2689.0, "update_stage2": 2091.1}
TRAFFIC_BYTES_PER_CELL = {"flux_x": 201.8 + 120.0, "flux_y": 292.9 + 112.0, "flux_z": 292.9 + 112.0,
                          "update_stage2": 368.3 + 248.0}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed stage-2 applications")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256, help="cells per dimension (default: the 256^3 workload)")
    ap.add_argument("--recon", default="weno5", choices=["weno5", "mc2", "minmod"])
    ap.add_argument("--evolve", type=int, default=10, help="IMEX steps before timing")
    ap.add_argument("--full-steps", type=int, default=3, help="timed full IMEX steps (reported beside)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", default="128,128,96", help="oracle sub-box (nx,ny,nz) for cpu_baseline")
    ap.add_argument("--cpu-reps", type=int, default=12, help="timed oracle stage-2 applications for cpu_baseline")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also launch a plain device copy of known size (for HBM counter calibration)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision (FP32 stencil) form")
    ap.add_argument("--mixed-steps", type=int, default=50, help="steps of the FP64-vs-mixed accuracy run")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the forward + adjoint rollout timing")
    ap.add_argument("--no-other-recon", action="store_true", help="skip timing the other reconstruction (MC2/WENO5)")
    ap.add_argument("--adjoint-steps", type=int, default=200, help="steps of the differentiated rollout")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(w, dt, sample, reps):
    """The oracle, as it stands, on a sub-box of the same workload: the
    central nx x ny x nz cells of the seeded initial data with their real
    neighbours as ghost cells (held fixed), advanced two oracle steps, then
    `reps` timed oracle stage-2 applications at that state."""
    import oracle

    oracle.build(force=False)
    nx, ny, nz = sample
    N = w.n[0]
    c = N // 2
    lo = [c - nx // 2, c - ny // 2, c - nz // 2]
    sl = (slice(lo[2], lo[2] + nz + 6), slice(lo[1], lo[1] + ny + 6), slice(lo[0], lo[0] + nx + 6))
    P = np.ascontiguousarray(w.P[(slice(None),) + sl])
    met = np.ascontiguousarray(w.metric[(slice(None),) + sl])
    sig = np.ascontiguousarray(w.sigma[sl])
    x0 = tuple(w.x0[d] + lo[d] * w.dx[d] for d in range(3))
    og = oracle.make_grid((nx, ny, nz), 7, w.dx, (oracle.BC_GIVEN,) * 3, w.gamma_ad, recon=w.recon, x0=x0)
    U = oracle.prim2con(og, P, met)
    for _ in range(2):
        oracle.step(og, dt, sig, U, P, met)
    s1 = oracle.stage1(og, dt, sig, U, P, met)
    t0 = time.perf_counter()
    for _ in range(reps):
        s2 = oracle.stage2(og, dt, sig, U, s1["P1"], s1["R1"], met)
    t = time.perf_counter() - t0
    cells = nx * ny * nz * reps
    return {"value": cells / t, "unit": "zone-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{reps} applications of IMEX stage 2 on the central {nx}x{ny}x{nz} cells of the 256^3 "
                      f"curved-blob workload (real neighbour ghosts, held fixed), after two oracle steps; "
                      f"{t:.2f} s timed, {int(s2['nfail'])} failed cells"}


def roofline(per_launch, kern, ncell):
    """Roofline of the kernel class with the largest total time: its binding
    ceiling is the larger of the HBM time of its algorithmic bytes and the FP64
    time of its flops; both fractions are reported."""
    dominant = max(per_launch, key=lambda k: kern[k][0])
    t = per_launch[dominant] * 1e-3
    nbytes = BYTES_PER_CELL.get(dominant, 0) * ncell
    flops = FLOPS_PER_CELL.get(dominant, 0.0) * ncell
    t_hbm = nbytes / (PEAK_HBM_GBS * 1e9)
    t_alu = flops / (PEAK_FP64_VECTOR_TFLOPS * 1e12)
    gbs = nbytes / t / 1e9
    tfs = flops / t / 1e12
    traffic = TRAFFIC_BYTES_PER_CELL.get(dominant)
    if t_alu > t_hbm:
        roof = {"bound": "alu", "achieved": tfs, "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": tfs / PEAK_FP64_VECTOR_TFLOPS}
    else:
        roof = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS}
    roof["traffic"] = None if traffic is None else traffic * ncell / 1e9
    roof.update({"traffic_unit": "GB per launch (FETCH_SIZE + WRITE_SIZE, calibrated)", "kernel": dominant,
                 "kernel_ms": t * 1e3, "algorithmic_GB": nbytes / 1e9, "hbm_frac": gbs / PEAK_HBM_GBS,
                 "fp64_TFLOP": flops / 1e12, "fp64_frac": tfs / PEAK_FP64_VECTOR_TFLOPS})
    return roof


def adjoint_leg(torch, rmhd, W, steps):
    """Forward + adjoint of the 64 x 2048 current-sheet batch inverse problem
    (200 steps, checkpoints every 20): one loss and gradient in (B^y_0,
    log sigma) per timed pass; reported as seconds per IMEX step."""
    from paper_2510_18968_amd.autograd import SheetInversion
    w = W.sheet_batch(steps=steps)
    g = rmhd.grid_for(w)
    prob = SheetInversion(w, g, ckpt=20)
    By0 = prob.P0[6].clone().requires_grad_(True)
    ls = torch.tensor(w.extra["sigma_problem"], device="cuda").log().requires_grad_(True)

    def fwd():
        with torch.no_grad():
            return prob.loss(By0, ls)

    def fwd_bwd():
        L = prob.loss(By0, ls)
        return torch.autograd.grad(L, (By0, ls))

    fwd_bwd()   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L = fwd()
    torch.cuda.synchronize()
    t_f = time.perf_counter() - t0
    t0 = time.perf_counter()
    gB, gs = fwd_bwd()
    torch.cuda.synchronize()
    t_fb = time.perf_counter() - t0
    if g.failures():
        raise SystemExit("recovery failures in the adjoint rollout")
    log(f"adjoint rollout {w.name}: forward {t_f:.3f} s, forward + adjoint {t_fb:.3f} s for {steps} steps")
    return {"workload": f"{w.name}: {steps} IMEX steps, WENO5, loss sum (B^y(T) - target)^2, gradient in "
                        f"(B^y_0, log sigma per problem), checkpoints every 20 steps",
            "fwd_adjoint_s_per_step": t_fb / steps, "fwd_s_per_step": t_f / steps,
            "adjoint_over_forward": (t_fb - t_f) / t_f, "loss": float(L),
            "grad_norm_By0": float(gB.norm()), "grad_norm_log_sigma": float(gs.norm())}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU domain decomposition "
              f"is a design note, not part of this build.", file=sys.stderr)
        return 2
    import torch

    from paper_2510_18968_amd import rmhd
    from paper_2510_18968_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        return 2
    rmhd.lib()   # fails loudly if the library is missing

    t0 = time.perf_counter()
    w = W.curved_blob(n=args.n, recon=args.recon)
    log(f"inputs generated in {time.perf_counter() - t0:.1f} s: {w.name}, padded {w.padded}")
    ncell = w.n_interior
    # interior x rows on 128-byte lines (16 cells of x padding)
    met = sig = None

    def setup(precision, recon=None):
        nonlocal met, sig
        g = rmhd.grid_for(w, precision=precision, x_align=1, **({"recon": recon} if recon else {}))
        if met is None:
            met = g.to_layout(w.metric)
            sig = g.to_layout(w.sigma)
        g.set_metric(met)
        P = g.to_layout(w.P)
        U = g.prim2con(P)
        return g, U, P

    g, U, P = setup("fp64")
    # CFL time step from the characteristic speeds (static metric: constant)
    smax = g.max_signal_speed()
    dt = 0.25 / smax
    log(f"max signal speed {smax:.6g} -> dt {dt:.6g} (CFL 0.25)")

    def evolve(g, U, P, steps, tag):
        t0 = time.perf_counter()
        for _ in range(steps):
            g.step(dt, sig, U, P)
        torch.cuda.synchronize()
        nfail = g.failures()
        log(f"{tag}: {steps} steps in {time.perf_counter() - t0:.2f} s, failed recoveries {nfail}")
        if nfail:
            raise SystemExit("recovery failures during evolution")

    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_stage2(g, U, P, steps, warmup):
        """K timed applications of IMEX stage 2 at the state (U, P)"""
        P1, R1 = g.empty(), g.empty(3)
        g.imex_stage(1, dt, sig, U, P, P1, R_out=R1)
        U2, P2, R2 = g.empty(), g.empty(), g.empty(3)

        def stage2():
            g.imex_stage(2, dt, sig, U, P1, P2, R_out=R2, R1=R1, U_out=U2)

        for _ in range(warmup):
            stage2()
        torch.cuda.synchronize()
        g.timing(True)
        g.timing_read()
        torch.cuda.synchronize()
        start.record()
        for _ in range(steps):
            stage2()
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop)
        kern = g.timing_read()
        g.timing(False)
        # one more application, untimed, for the recovery iteration histogram
        g.recovery_stats(True)
        stage2()
        hist = g.recovery_stats_read()["stage2"]
        g.recovery_stats(False)
        nfail = g.failures()
        if nfail:
            raise SystemExit(f"{nfail} failed recoveries in the timed stages")
        del P1, R1, U2, P2, R2
        return ms, kern, {str(i): c for i, c in enumerate(hist) if c}

    evolve(g, U, P, args.evolve, "fp64")
    ms, kern, hist = time_stage2(g, U, P, args.steps, args.warmup)
    value = ncell * args.steps / (ms * 1e-3)
    log(f"stage 2: {ms / args.steps:.3f} ms -> {value:.4g} zone-updates/s")

    # full IMEX steps (stage 1 + stage 2 + final), reported beside
    Uc, Pc = U.clone(), P.clone()
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.full_steps):
        g.step(dt, sig, Uc, Pc)
    stop.record()
    torch.cuda.synchronize()
    ms_step = start.elapsed_time(stop) / max(1, args.full_steps)
    if g.failures():
        raise SystemExit("failed recoveries in the full steps")

    if args.calibrate_copy:
        # a plain streaming kernel of known traffic for the HBM byte counters:
        # b = -a over 2^28 doubles reads 2 GiB and writes 2 GiB
        a = torch.zeros(1 << 28, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(2):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b

    # the other reconstruction of the same workload, on the same evolved state
    other = None
    if not args.no_other_recon:
        orec = "mc2" if args.recon == "weno5" else "weno5"
        go, _, _ = setup("fp64", orec)
        ms_o, kern_o, _ = time_stage2(go, U, P, args.steps, args.warmup)
        other = {"recon": orec, "value": ncell * args.steps / (ms_o * 1e-3), "unit": "zone-updates/s",
                 "ms_per_step": ms_o / args.steps,
                 "kernels_ms_per_launch": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kern_o.items()}}
        log(f"{orec} stage 2 on the same state: {ms_o / args.steps:.3f} ms")
        del go

    mixed = None
    if not args.no_mixed:
        gm, Um, Pm = setup("mixed")
        evolve(gm, Um, Pm, args.evolve, "mixed")
        ms_m, kern_m, _ = time_stage2(gm, Um, Pm, args.steps, args.warmup)
        val_m = ncell * args.steps / (ms_m * 1e-3)
        log(f"mixed stage 2: {ms_m / args.steps:.3f} ms -> {val_m:.4g} zone-updates/s")
        # accuracy: both forms from the same seed to the same step count
        rest = max(0, args.mixed_steps - args.evolve)
        evolve(g, U, P, rest, "fp64 accuracy run")
        evolve(gm, Um, Pm, rest, "mixed accuracy run")
        I = (slice(None),) + tuple(w.interior)
        P, Pm = g.from_layout(P), gm.from_layout(Pm)     # the 3-ghost layout of w.interior
        names = ["rho", "p", "vx", "vy", "vz", "Bx", "By", "Bz", "Ex", "Ey", "Ez", "phi", "psi", "q"]
        errs = {}
        # E (slaved to -v x B in the stiff interior) is measured against the
        # electromagnetic scale max(|E|, |B|), as are phi, psi and q
        em_max = float(P[5:11][I].abs().max())
        em_sum = max(float(P[f][I[1:]].abs().sum()) for f in range(5, 11))
        for f, nm in enumerate(names):
            a, b = P[f][I[1:]], Pm[f][I[1:]]
            d = (a - b).abs()
            s1, si = float(a.abs().sum()), float(a.abs().max())
            if f >= 8:
                s1, si = max(s1, em_sum), max(si, em_max)
            errs[nm] = {"L1": float(d.sum()) / max(s1, 1e-300), "Linf": float(d.max()) / max(si, 1e-300)}
        worst = max(max(errs[n]["L1"], errs[n]["Linf"]) for n in ["rho", "p", "Bx", "By", "Bz", "Ex", "Ey", "Ez"])
        mixed = {"value": val_m, "unit": "zone-updates/s", "ms_per_step": ms_m / args.steps,
                 "speedup_vs_fp64": ms / ms_m,
                 "kernels_ms_per_launch": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kern_m.items()},
                 "accuracy_steps": args.evolve + rest,
                 "max_rel_err_rho_p_B_E": worst, "per_field_vs_fp64": errs,
                 "reference": "the FP64 GPU path from the same seed (equal to the oracle by the parity tests)"}
        log(f"mixed: speedup {ms / ms_m:.3f}, max rel err (rho, p, B, E) after {args.evolve + rest} steps "
            f"{worst:.3e}")
        del gm, Um, Pm

    adjoint = None
    if not args.no_adjoint:
        adjoint = adjoint_leg(torch, rmhd, W, args.adjoint_steps)

    per_launch = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kern.items()}
    roof = roofline(per_launch, kern, ncell)
    stage_bytes = sum(BYTES_PER_CELL.get(k, 0) * kern[k][1] for k in kern) / max(1, args.steps) * ncell
    stage_flops = sum(FLOPS_PER_CELL.get(k, 0.0) * kern[k][1] for k in kern) / max(1, args.steps) * ncell
    roof["stage"] = {"ms": ms / args.steps, "algorithmic_GB": stage_bytes / 1e9,
                     "hbm_frac": stage_bytes / (ms / args.steps * 1e-3) / 1e9 / PEAK_HBM_GBS,
                     "fp64_TFLOP": stage_flops / 1e12,
                     "fp64_frac": stage_flops / (ms / args.steps * 1e-3) / 1e12 / PEAK_FP64_VECTOR_TFLOPS}

    cpu = None
    if not args.no_cpu_baseline:
        del U, P, Uc, Pc
        t0 = time.perf_counter()
        cpu = cpu_baseline(w, dt, tuple(int(x) for x in args.cpu_sample.split(",")), args.cpu_reps)
        log(f"cpu baseline {cpu['value']:.4g} zone-updates/s in {time.perf_counter() - t0:.1f} s")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"curved_blob {args.n}^3 {args.recon} FP64: IMEX-SSP2(2,2,2) stage 2 after "
                               f"{args.evolve} steps (static conformally flat metric, Gamma = 2, "
                               f"sigma = 1e6 rho/rho_max + 1, CFL 0.25, copy boundaries)",
                   "n": [args.n] * 3, "recon": args.recon, "dt": dt, "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels_ms_per_launch": per_launch,
        "stage2_recovery_iterations": hist,
        "full_step": {"ms": ms_step, "zone_updates_per_s_per_stage": 2 * ncell / (ms_step * 1e-3)},
        "other_recon": other,
        "mixed": mixed,
        "adjoint": adjoint,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
