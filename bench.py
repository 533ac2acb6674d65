#!/usr/bin/env python3
"""Benchmark of the resistive GRMHD IMEX-SSP2(2,2,2) stage on one MI355X.

Metric: zone-updates/s per IMEX stage (interior cells per stage-2 application
per second) on the 256^3 static curved background with a magnetised blob,
FP64, WENO5 + HLLE, after 10 steps of evolution (so that the stiff recovery
does real work).  One timed "step" is one application of IMEX stage 2: the
boundary values (read at the ghost cells' interior images), reconstruction,
HLLE fluxes, flux divergence + sources + RK combination and the coupled
implicit-E / primitive recovery, i.e. every row of the hot path.  Each application is bracketed by HIP events on the library's stream
with the library's own launch timers off; `value` is the interior cell count
over the median application time.  Per-kernel times come from a separate
pass with the launch timers on.

Beside the headline it reports the full IMEX step, MC2, the mixed form (with
its per-field error after 50 steps), the forward + adjoint rollout of the
64 x 2048 batch, GPU and oracle timings of the 400-cell shocktubes, the 128^3
periodic box and the 64 x 2048 batch, and the oracle (the plain FP64 CPU
implementation of the same method) timed on the GPU's timed state.

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "zone-updates/s per IMEX stage, FP64 vs mixed at 256^3; fwd+adjoint s/step"

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_VECTOR_TFLOPS = 78.6

# Algorithmic HBM bytes of one IMEX stage per interior zone, curved metric:
# every stage input and output word moved once (reads U^n 14, E(1) 3, the
# hydro primitives 5, R1 3, sigma 1, metric 10; writes U(2) 14, the hydro
# primitives 5, R2 3: 58 words).
STAGE_FLOOR_BYTES = 464

# Per interior cell and launch of each kernel class on the 256^3 curved WENO5
# workload (zero shift and extrinsic curvature and a diagonal 3-metric, so the
# metric read is alpha and the diagonal of gamma_ij, 4 words):
#  * BYTES_PER_CELL: each word the kernel as designed reads or writes, once
#    (this includes the 14-field flux-divergence accumulator between the
#    launches, which the stage floor above does not);
#  * FLOPS_PER_CELL: executed FP64 flops, from the
#    SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 counters (FMA = 2 flops, 64 lanes
#    per wave instruction);
#  * TRAFFIC_BYTES_PER_CELL: FETCH_SIZE + WRITE_SIZE of the same launch,
#    scaled by what the counters read for a streaming kernel of known size.
# The flops and traffic figures belong to the kernels as profiled
# (profiles/counters_curved256_weno5.md); they are re-measured when a kernel
# changes.
BYTES_PER_CELL = {
    # P 14 + sigma 1 + metric 4 read, rhs 14 written
    "flux_x": 8 * (14 + 1 + 4 + 14),
    # as x, plus the read half of the rhs read-modify-write
    "flux_y": 8 * (14 + 1 + 4 + 14 + 14),
    "flux_z": 8 * (14 + 1 + 4 + 14 + 14),
    # P(1) 4 (p and v: the guess and, without K, the local sources' velocity;
    # the cleaning fields come from U^n), U^n 14, rhs 14, R1 3, sigma 1,
    # metric 4 read; U(2) 14, P(2) 14, R2 3 written
    "update_stage2": 8 * (4 + 14 + 14 + 3 + 1 + 4 + 14 + 14 + 3),
}
FLOPS_PER_CELL = {"flux_x": 2576.1, "flux_y": 2339.5, "flux_z": 2341.6, "update_stage2": 1685.6}
TRAFFIC_BYTES_PER_CELL = {"flux_x": 158.2 + 118.5, "flux_y": 265.8 + 112.0, "flux_z": 266.0 + 112.0,
                          "update_stage2": 320.2 + 248.0}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed stage-2 applications")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256, help="cells per dimension (default: the 256^3 workload)")
    ap.add_argument("--recon", default="weno5", choices=["weno5", "mc2", "minmod"])
    ap.add_argument("--evolve", type=int, default=10, help="IMEX steps before timing")
    ap.add_argument("--full-steps", type=int, default=10, help="timed full IMEX steps (reported beside)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", default="128,128,96", help="oracle sub-box (nx,ny,nz) for cpu_baseline")
    ap.add_argument("--cpu-reps", type=int, default=12, help="timed oracle stage-2 applications for cpu_baseline")
    ap.add_argument("--cpu-single", default="48,48,32", help="oracle sub-box of the single-thread figure")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also launch a plain device copy of known size (for HBM counter calibration)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision (FP32 stencil) form")
    ap.add_argument("--mixed-steps", type=int, default=50, help="steps of the FP64-vs-mixed accuracy run")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the forward + adjoint rollout timing")
    ap.add_argument("--no-other-recon", action="store_true", help="skip timing the other reconstruction (MC2/WENO5)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the shocktube / periodic box / batch timings (GPU and oracle)")
    ap.add_argument("--no-breakdown", action="store_true", help="skip the per-kernel timing pass")
    ap.add_argument("--adjoint-steps", type=int, default=200, help="steps of the differentiated rollout")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def timed_calls(torch, fn, steps, warmup):
    """Per-call times (ms) of `steps` calls of fn, each bracketed by HIP
    events on the current stream (the stream the library launches on)."""
    for _ in range(warmup):
        fn()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i in range(steps):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)], ev[0].elapsed_time(ev[-1])


def stage_roofline(ms, ncell, kernels_ms):
    """Stage-level roofline: the stage floor bytes and the counted FP64 flops
    of the four launches over the median stage time, with the per-kernel
    figures as a breakdown."""
    t = ms * 1e-3
    nbytes = STAGE_FLOOR_BYTES * ncell
    flops = sum(FLOPS_PER_CELL.values()) * ncell
    traffic = sum(TRAFFIC_BYTES_PER_CELL.values()) * ncell
    t_hbm = nbytes / (PEAK_HBM_GBS * 1e9)
    t_alu = flops / (PEAK_FP64_VECTOR_TFLOPS * 1e12)
    gbs = nbytes / t / 1e9
    roof = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
            "traffic": traffic / 1e9,
            "scope": "one IMEX stage 2 (x/y/z flux sweeps, update + recovery) at the median time",
            "algorithmic_bytes_per_zone": STAGE_FLOOR_BYTES, "algorithmic_GB": nbytes / 1e9,
            "traffic_unit": "GB per stage (FETCH_SIZE + WRITE_SIZE of the four launches, calibrated)",
            "traffic_over_algorithmic": traffic / nbytes,
            "fp64": {"flops_per_zone_counted": sum(FLOPS_PER_CELL.values()), "TFLOP": flops / 1e12,
                     "achieved_TFLOPs": flops / t / 1e12, "peak_TFLOPs": PEAK_FP64_VECTOR_TFLOPS,
                     "frac": flops / t / 1e12 / PEAK_FP64_VECTOR_TFLOPS},
            "ceilings_ms": {"hbm": t_hbm * 1e3, "fp64": t_alu * 1e3},
            "min_roofline_frac": max(t_hbm, t_alu) / t}
    br = {}
    for k, kms in kernels_ms.items():
        if k not in FLOPS_PER_CELL or kms <= 0:
            continue
        tk = kms * 1e-3
        b = BYTES_PER_CELL[k] * ncell
        f = FLOPS_PER_CELL[k] * ncell
        tb = max(b / (PEAK_HBM_GBS * 1e9), f / (PEAK_FP64_VECTOR_TFLOPS * 1e12))
        br[k] = {"ms": kms, "design_GB": b / 1e9, "hbm_frac": b / tk / 1e9 / PEAK_HBM_GBS,
                 "fp64_frac": f / tk / 1e12 / PEAK_FP64_VECTOR_TFLOPS, "roofline_frac": tb / tk,
                 "traffic_GB": TRAFFIC_BYTES_PER_CELL[k] * ncell / 1e9}
    roof["kernels"] = br
    return roof


def subbox(t, off, lo, size):
    """host copy of t[..., box with 3 ghost cells] of a device tensor in a
    grid's layout; lo and size per axis (x, y, z) in interior cells"""
    oz, oy, ox = off
    sl = (slice(lo[2] + oz, lo[2] + oz + size[2] + 6), slice(lo[1] + oy, lo[1] + oy + size[1] + 6),
          slice(lo[0] + ox, lo[0] + ox + size[0] + 6))
    return np.ascontiguousarray(t[(Ellipsis,) + sl].cpu().numpy())


def oracle_on_state(oracle, w, dt, U, P, off, size, reps):
    """`reps` oracle stage-2 applications on the central box of the GPU's
    state (U, P in the grid's layout): the real neighbours as ghost cells,
    held fixed; stage 1 first, as on the GPU.  Returns (seconds, cells,
    failed cells)."""
    N = w.n[0]
    lo = [N // 2 - s // 2 for s in size]
    Us = subbox(U, off, lo, size)
    Ps = subbox(P, off, lo, size)
    sl = tuple(slice(lo[d], lo[d] + size[d] + 6) for d in (2, 1, 0))
    met = np.ascontiguousarray(w.metric[(slice(None),) + sl])
    sig = np.ascontiguousarray(w.sigma[sl])
    x0 = tuple(w.x0[d] + lo[d] * w.dx[d] for d in range(3))
    og = oracle.make_grid(tuple(size), 7, w.dx, (oracle.BC_GIVEN,) * 3, w.gamma_ad, recon=w.recon, x0=x0)
    s1 = oracle.stage1(og, dt, sig, Us, Ps, met)
    t0 = time.perf_counter()
    nf = 0
    for _ in range(reps):
        s2 = oracle.stage2(og, dt, sig, Us, s1["P1"], s1["R1"], met)
        nf += int(s2["nfail"])
    return time.perf_counter() - t0, size[0] * size[1] * size[2] * reps, nf


def cpu_baseline(oracle, w, dt, U, P, off, sample, reps, single):
    """The oracle, as it stands, on the state the GPU times: the central
    sample box of the 256^3 state after the evolution steps, all host
    threads, then one thread on a smaller central box."""
    t, cells, nf = oracle_on_state(oracle, w, dt, U, P, off, sample, reps)
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    t1, cells1, nf1 = oracle_on_state(oracle, w, dt, U, P, off, single, 1)
    oracle.set_num_threads(threads)
    return {"value": cells / t, "unit": "zone-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} applications of IMEX stage 2 on the central {'x'.join(map(str, sample))} cells "
                      f"of the GPU's timed state (256^3 curved blob after the evolution steps; real neighbours "
                      f"as ghost cells, held fixed): {t:.2f} s, {nf} failed cells",
            "cpu_model": cpu_model(), "threads": threads,
            "single_thread": {"value": cells1 / t1, "unit": "zone-updates/s",
                              "sample": f"one stage-2 application on the central {'x'.join(map(str, single))} "
                                        f"cells of the same state: {t1:.2f} s, {nf1} failed cells"}}


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


def other_configs(torch, rmhd, W, oracle):
    """GPU and oracle timings of the smaller workloads: the nine 400-cell
    shocktubes (320 steps each), the 128^3 periodic box (10 steps on the GPU,
    one on the oracle) and the 64 x 2048 batch forward (and the oracle's
    forward-mode tangent)."""
    out = {}
    # shocktubes: the GPU runs all nine, the oracle one seed per sigma
    t_gpu, zs = 0.0, 0
    runs = []
    for seed in (101, 102, 103):
        for s0 in (1.0, 1e3, 1e6):
            w = W.shocktube(seed=seed, sigma0=s0)
            g = rmhd.grid_for(w)
            sig = torch.from_numpy(w.sigma).cuda()
            P = torch.from_numpy(w.P).cuda()
            U = g.prim2con(P)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(w.steps):
                g.step(w.dt, sig, U, P)
            torch.cuda.synchronize()
            t_gpu += time.perf_counter() - t0
            zs += 2 * w.steps * w.n_interior
            if g.failures():
                raise SystemExit(f"recovery failures in the shocktube seed {seed} sigma {s0}")
            runs.append((seed, s0))
    t_orc, zo = 0.0, 0
    if oracle is not None:
        for s0 in (1.0, 1e3, 1e6):
            w = W.shocktube(seed=101, sigma0=s0)
            og = oracle.make_grid(w.n, w.active, w.dx, w.bc, w.gamma_ad, recon=w.recon, x0=w.x0)
            P = w.P.copy()
            U = oracle.prim2con(og, P)
            t0 = time.perf_counter()
            for _ in range(w.steps):
                oracle.step(og, w.dt, w.sigma, U, P)
            t_orc += time.perf_counter() - t0
            zo += 2 * w.steps * w.n_interior
    out["shocktube_400"] = {
        "workload": "nine 400-cell resistive shocktubes (seeds 101-103 x sigma 1, 1e3, 1e6), minmod, 320 steps "
                    "each to t = 0.4 (one launch sequence per step: latency-bound on the GPU)",
        "gpu": {"value": zs / t_gpu, "unit": "zone-updates/s per stage", "s_per_run": t_gpu / len(runs)},
        "oracle": None if oracle is None else {"value": zo / t_orc, "unit": "zone-updates/s per stage",
                                               "s_per_run": t_orc / 3, "runs": "seed 101, sigma 1, 1e3, 1e6"}}
    log(f"shocktubes: GPU {zs / t_gpu:.3g}, oracle {zo / max(t_orc, 1e-9):.3g} zone-updates/s per stage")

    # periodic box 128^3
    w = W.periodic_box(n=128)
    g = rmhd.grid_for(w, x_align=1)
    sig = g.to_layout(w.sigma)
    P = g.to_layout(w.P)
    U = g.prim2con(P)
    per, _ = timed_calls(torch, lambda: g.step(w.dt, sig, U, P), w.steps, 0)
    if g.failures():
        raise SystemExit("recovery failures in the periodic box")
    ms_step = statistics.median(per)
    box = {"workload": f"{w.name}: 128^3 flat periodic, WENO5, {w.steps} IMEX steps (median step)",
           "gpu": {"value": 2 * w.n_interior / (ms_step * 1e-3), "unit": "zone-updates/s per stage",
                   "ms_per_step": ms_step}}
    del g, U, P, sig
    if oracle is not None:
        og = oracle.make_grid(w.n, w.active, w.dx, w.bc, w.gamma_ad, recon=w.recon, x0=w.x0)
        Po = w.P.copy()
        Uo = oracle.prim2con(og, Po)
        t0 = time.perf_counter()
        oracle.step(og, w.dt, w.sigma, Uo, Po)
        t = time.perf_counter() - t0
        box["oracle"] = {"value": 2 * w.n_interior / t, "unit": "zone-updates/s per stage", "s_per_step": t,
                         "sample": "the first IMEX step"}
    out["periodic_box_128"] = box
    log(f"periodic box: GPU {box['gpu']['value']:.3g} zone-updates/s per stage")

    # 64 x 2048 batch forward
    w = W.sheet_batch()
    g = rmhd.grid_for(w)
    sig = torch.from_numpy(w.sigma).cuda()
    P = torch.from_numpy(w.P).cuda()
    U = g.prim2con(P)
    per, tot = timed_calls(torch, lambda: g.step(w.dt, sig, U, P), 40, 0)
    batch = {"workload": "64 x 2048 current-sheet batch, WENO5, forward steps",
             "gpu": {"s_per_step": statistics.median(per) * 1e-3,
                     "value": 2 * w.n_interior / (statistics.median(per) * 1e-3),
                     "unit": "zone-updates/s per stage"}}
    del g, U, P, sig
    if oracle is not None:
        og = oracle.make_grid(w.n, w.active, w.dx, w.bc, w.gamma_ad, recon=w.recon, x0=w.x0)
        Po = w.P.copy()
        Uo = oracle.prim2con(og, Po)
        nst = 10
        t0 = time.perf_counter()
        for _ in range(nst):
            oracle.step(og, w.dt, w.sigma, Uo, Po)
        t_f = (time.perf_counter() - t0) / nst
        rng = np.random.default_rng(7)
        dU = rng.standard_normal(Uo.shape)
        ds = rng.standard_normal(w.sigma.shape)
        ntan = 3
        t0 = time.perf_counter()
        for _ in range(ntan):
            oracle.step_tangent(og, w.dt, w.sigma, Uo, dU, Po, dsigma=ds)
        t_t = (time.perf_counter() - t0) / ntan
        batch["oracle"] = {"s_per_step": t_f, "tangent_s_per_step": t_t,
                           "value": 2 * w.n_interior / t_f, "unit": "zone-updates/s per stage",
                           "sample": f"{nst} forward steps, then {ntan} steps in dual numbers (forward-mode "
                                     f"tangent along a random (U, sigma) direction)"}
    out["sheet_batch_64x2048"] = batch
    log(f"batch: GPU {batch['gpu']['s_per_step'] * 1e3:.3f} ms per forward step")
    return out


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

    def time_stage2(g, U, P, steps, warmup, breakdown):
        """K applications of IMEX stage 2 at the state (U, P), each timed by
        events with the launch timers off; then (optionally) K more with the
        library's per-launch timers on for the per-kernel breakdown"""
        P1, R1 = g.empty(), g.empty(3)
        g.imex_stage(1, dt, sig, U, P, P1, R_out=R1)
        U2, P2, R2 = g.empty(), g.empty(), g.empty(3)

        def stage2():
            g.imex_stage(2, dt, sig, U, P1, P2, R_out=R2, R1=R1, U_out=U2)

        per, tot = timed_calls(torch, stage2, steps, warmup)
        kern = None
        if breakdown:
            g.timing(True)
            g.timing_read()
            for _ in range(steps):
                stage2()
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
        return per, tot, kern, {str(i): c for i, c in enumerate(hist) if c}

    evolve(g, U, P, args.evolve, "fp64")
    per, tot, kern, hist = time_stage2(g, U, P, args.steps, args.warmup, not args.no_breakdown)
    ms = statistics.median(per)
    value = ncell / (ms * 1e-3)
    log(f"stage 2: median {ms:.3f} ms (mean {tot / args.steps:.3f}, min {min(per):.3f}, max {max(per):.3f}) -> "
        f"{value:.4g} zone-updates/s")
    per_launch = {} if kern is None else {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kern.items()}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        t0 = time.perf_counter()
        cpu = cpu_baseline(oracle, w, dt, U, P, rmhd.std_offsets(g.desc),
                           tuple(int(x) for x in args.cpu_sample.split(",")), args.cpu_reps,
                           tuple(int(x) for x in args.cpu_single.split(",")))
        log(f"cpu baseline {cpu['value']:.4g} zone-updates/s ({cpu['threads']} threads), single thread "
            f"{cpu['single_thread']['value']:.4g}, in {time.perf_counter() - t0:.1f} s")

    # full IMEX steps (stage 1 + stage 2 + final), reported beside: one
    # rmhd_step per step, and all of them in one rmhd_steps call (each final
    # update runs the next step's stage 1)
    Uc, Pc = U.clone(), P.clone()
    per_step, _ = timed_calls(torch, lambda: g.step(dt, sig, Uc, Pc), args.full_steps, 0)
    ms_step = statistics.median(per_step)
    Uc.copy_(U)
    Pc.copy_(P)
    _, tot_f = timed_calls(torch, lambda: g.steps(dt, sig, Uc, Pc, args.full_steps), 1, 0)
    ms_fused = tot_f / args.full_steps
    if g.failures():
        raise SystemExit("failed recoveries in the full steps")
    log(f"full step: {ms_step:.3f} ms (rmhd_step, median of {args.full_steps}), {ms_fused:.3f} ms per step in one "
        f"rmhd_steps call of {args.full_steps}")
    del Uc, Pc

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
        per_o, _, _, _ = time_stage2(go, U, P, args.steps, args.warmup, False)
        ms_o = statistics.median(per_o)
        other = {"recon": orec, "value": ncell / (ms_o * 1e-3), "unit": "zone-updates/s", "ms_per_step": ms_o}
        log(f"{orec} stage 2 on the same state: {ms_o:.3f} ms")
        del go

    mixed = None
    if not args.no_mixed:
        gm, Um, Pm = setup("mixed")
        evolve(gm, Um, Pm, args.evolve, "mixed")
        per_m, _, kern_m, _ = time_stage2(gm, Um, Pm, args.steps, args.warmup, not args.no_breakdown)
        ms_m = statistics.median(per_m)
        val_m = ncell / (ms_m * 1e-3)
        log(f"mixed stage 2: {ms_m:.3f} ms -> {val_m:.4g} zone-updates/s")
        # accuracy: both forms from the same seed to the same step count
        rest = max(0, args.mixed_steps - args.evolve)
        Ua, Pa = U.clone(), P.clone()
        evolve(g, Ua, Pa, rest, "fp64 accuracy run")
        evolve(gm, Um, Pm, rest, "mixed accuracy run")
        I = (slice(None),) + tuple(w.interior)
        Pa, Pm = g.from_layout(Pa), gm.from_layout(Pm)     # the 3-ghost layout of w.interior
        names = ["rho", "p", "vx", "vy", "vz", "Bx", "By", "Bz", "Ex", "Ey", "Ez", "phi", "psi", "q"]
        errs = {}
        # E (slaved to -v x B in the stiff interior) is measured against the
        # electromagnetic scale max(|E|, |B|), as are phi, psi and q
        em_max = float(Pa[5:11][I].abs().max())
        em_sum = max(float(Pa[f][I[1:]].abs().sum()) for f in range(5, 11))
        for f, nm in enumerate(names):
            a, b = Pa[f][I[1:]], Pm[f][I[1:]]
            d = (a - b).abs()
            s1, si = float(a.abs().sum()), float(a.abs().max())
            if f >= 8:
                s1, si = max(s1, em_sum), max(si, em_max)
            errs[nm] = {"L1": float(d.sum()) / max(s1, 1e-300), "Linf": float(d.max()) / max(si, 1e-300)}
        worst = max(max(errs[n]["L1"], errs[n]["Linf"]) for n in ["rho", "p", "Bx", "By", "Bz", "Ex", "Ey", "Ez"])
        mixed = {"value": val_m, "unit": "zone-updates/s", "ms_per_step": ms_m,
                 "speedup_vs_fp64": ms / ms_m,
                 "kernels_ms_per_launch": None if kern_m is None else
                 {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kern_m.items()},
                 "accuracy_steps": args.evolve + rest,
                 "max_rel_err_rho_p_B_E": worst, "per_field_vs_fp64": errs,
                 "reference": "the FP64 GPU path from the same seed (equal to the oracle by the parity tests)"}
        log(f"mixed: speedup {ms / ms_m:.3f}, max rel err (rho, p, B, E) after {args.evolve + rest} steps "
            f"{worst:.3e}")
        del gm, Um, Pm, Ua, Pa

    del g, U, P
    met = sig = None
    torch.cuda.empty_cache()

    adjoint = None
    if not args.no_adjoint:
        adjoint = adjoint_leg(torch, rmhd, W, args.adjoint_steps)

    configs = None
    if not args.no_configs:
        orc = None
        if not args.no_cpu_baseline:
            import oracle as orc
        configs = other_configs(torch, rmhd, W, orc)

    roof = stage_roofline(ms, ncell, per_launch)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"curved_blob {args.n}^3 {args.recon} FP64: IMEX-SSP2(2,2,2) stage 2 after "
                               f"{args.evolve} steps (static conformally flat metric, Gamma = 2, "
                               f"sigma = 1e6 rho/rho_max + 1, CFL 0.25, copy boundaries)",
                   "n": [args.n] * 3, "recon": args.recon, "dt": dt, "parallelism": "single GPU"},
        "timing": {"statistic": "median of the per-application event times", "ms_median": ms,
                   "ms_mean": tot / args.steps, "ms_min": min(per), "ms_max": max(per)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels_ms_per_launch": per_launch,
        "stage2_recovery_iterations": hist,
        "full_step": {"ms": ms_step, "zone_updates_per_s_per_stage": 2 * ncell / (ms_step * 1e-3),
                      "fused_steps": {"steps": args.full_steps, "ms_per_step": ms_fused,
                                      "zone_updates_per_s_per_stage": 2 * ncell / (ms_fused * 1e-3),
                                      "speedup_vs_step": ms_step / ms_fused}},
        "other_recon": other,
        "mixed": mixed,
        "adjoint": adjoint,
        "configs": configs,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
