"""Host-side check of the kernels' index maps: every global address the x
sweep, the stage kernels, the y/z window sweeps and the adjoint x gather form
lies inside its array, for the benchmark's 256^3 aligned layout, the 64 x 2048
batch, a 2D grid and small grids (no device needed).

The formulas are those of the kernels (work item -> lane -> padded offset),
evaluated here for every work item and lane with numpy, with the launch
shapes the host code picks on a 256-CU device.
"""
import numpy as np
import pytest

TSEG, TSEGA, CHUNK = 58, 60, 64
CUS = 256


def layout(n, active, x_align):
    g = [(16 if (d == 0 and x_align) else 3) if (active >> d) & 1 else 0 for d in range(3)]
    npd = [n[d] + 2 * g[d] for d in range(3)]
    st = [1, npd[0], npd[0] * npd[1]]
    return g, npd, st, npd[0] * npd[1] * npd[2]


def bc_map(c, g, n):
    """ghost -> interior image (copy boundaries; periodic images are interior too)"""
    return np.clip(c, g, g + n - 1)


def check(name, off, lo, hi):
    off = np.asarray(off)
    if off.size == 0:
        return
    assert off.min() >= lo and off.max() < hi, (name, int(off.min()), int(off.max()), lo, hi)


def x_sweep(n, active, x_align):
    g, npd, st, Np = layout(n, active, x_align)
    W0 = n[0] + 6
    V = W0 * n[1] * n[2]
    assert V + 64 <= 2 ** 31 - 1                        # 32-bit positions (host check)
    items = (V + TSEG - 1) // TSEG
    lane = np.arange(64)
    for w0 in range(0, items, 20000):
        wid = np.arange(w0, min(items, w0 + 20000))[:, None]
        v = wid * TSEG - 3 + lane
        vc = np.clip(v, 0, V - 1)
        r = vc // W0
        x = vc - r * W0 - 3
        a1, a2 = r % n[1], r // n[1]
        cp = x + g[0]
        o = (a1 + g[1]) * st[1] + (a2 + g[2]) * st[2] + cp
        check("x sweep loads (P, metric)", o, 0, Np)
        check("x sweep sigma", o + (bc_map(cp, g[0], n[0]) - cp), 0, Np)
        c = np.where(v == vc, x, -4)
        cell = (lane >= 3) & (lane < 3 + TSEG) & (c >= 0) & (c < n[0])
        os = np.where(cell, o, o - (cp - (g[0] - 1)))
        check("x sweep rhs stores", os, 0, Np)
        # a lane without a cell writes an x ghost of rhs, never an interior cell
        xs = os % npd[0]
        assert ((xs >= g[0]) & (xs < g[0] + n[0]) | ~cell).all() and (xs[~cell] == g[0] - 1).all()


def stage_chunks(n, active, x_align):
    g, npd, st, Np = layout(n, active, x_align)
    nsx = (n[0] + CHUNK - 1) // CHUNK
    nchunk = nsx * n[1] * n[2]
    lane = np.arange(64)
    for q0 in range(0, nchunk, 50000):
        q = np.arange(q0, min(nchunk, q0 + 50000))[:, None]
        r = q // nsx
        seg = q - r * nsx
        j, k = r % n[1], r // n[1]
        orow = (k + g[2]) * st[2] + (j + g[1]) * st[1] + g[0]
        x0 = seg * CHUNK
        xp = np.minimum(x0 + 2 * (lane & 31), npd[0] - 2 - g[0])
        oo = orow + xp
        check("stage LDS pair loads", np.concatenate([oo, oo + 1]), 0, Np)
        # the pair stays inside the padded row
        assert ((oo + 1) // npd[0] == oo // npd[0]).all()
        ok = x0 + lane < n[0]
        lc = np.where(ok, lane, n[0] - 1 - x0)
        o = orow + x0 + lc
        check("stage cells", o, 0, Np)
        xo = o % npd[0]
        assert ((xo >= g[0]) & (xo < g[0] + n[0])).all()


def window(n, active, x_align, D):
    g, npd, st, Np = layout(n, active, x_align)
    E = 2 if D == 1 else 1
    nxb = (n[0] + 63) // 64
    cols = nxb * n[E]
    want = 4 * CUS
    nseg0 = min(max(1, (want + cols - 1) // cols), (n[D] + 7) // 8)
    seglen = (n[D] + nseg0 - 1) // nseg0
    nseg = (n[D] + seglen - 1) // seglen
    gD, nD, s = g[D], n[D], st[D]
    lane = np.arange(64)
    fhalf = lane >> 5
    waves = nxb * n[E] * nseg
    wid = np.arange(waves)[:, None]
    xb = wid % nxb
    r = wid // nxb
    e = r % n[E]
    seg = r // n[E]
    i = xb * 64 + lane
    c0 = seg * seglen
    c1 = np.minimum(c0 + seglen, nD)
    rowb = (e + g[E]) * st[E]
    base = rowb + np.minimum(i, n[0] - 1) + g[0]
    xpair = np.minimum(g[0] + xb * 64 + 2 * (lane & 31), npd[0] - 2)
    # rows touched: ring c0-3 .. nD+2 (clamped), staging c0+1 and the clamped
    # c+3 of every step, metric rows c0-4 .. c0 (those >= -gD), rhs rows c-1
    steps = np.arange(-1, seglen + 1)                       # c = c0 - 1 .. c0 + seglen (<= c1)
    cs = c0[..., None] + steps                              # [waves, 1, steps]
    live = cs <= c1[..., None]
    cnext = np.minimum(cs + 3, nD + 2)
    ring_rows = np.concatenate([c0[..., None] + np.arange(-3, 2), np.where(live, cnext, c0[..., None])], -1)
    for rr in ring_rows.reshape(waves, -1).T:
        off = rowb + (rr[:, None] + gD) * s + xpair
        for f in range(0, 14, 2):
            check("ring loads", np.stack([(fhalf + f) * Np + off, (fhalf + f) * Np + off + 1]), 0, 14 * Np)
    stage_rows = np.concatenate([c0[..., None] + 1, np.where(live, cnext, c0[..., None] + 1)], -1)
    for rr in stage_rows.reshape(waves, -1).T:
        ro = rowb + (rr[:, None] + gD) * s + xpair
        rs = rowb + bc_map(rr[:, None] + gD, gD, nD) * s + xpair
        check("staging sigma", np.stack([rs, rs + 1]), 0, Np)
        check("staging metric", np.stack([ro, ro + 1]), 0, Np)
    for k in range(5):
        c = c0 - 4 + k
        use = c >= -gD
        o = base + (c + gD) * s
        check("window metric rows", o[np.broadcast_to(use, o.shape)], 0, Np)
        sg = o + (bc_map(c + gD, gD, nD) - (c + gD)) * s
        check("window sigma rows", sg[np.broadcast_to(use, o.shape)], 0, Np)
    valid = i < n[0]
    odummy = rowb + g[0] - 1
    for t in range(len(steps)):
        c = cs[..., t]
        lv = np.broadcast_to(live[..., t], base.shape)
        om = base + (c - 1 + gD) * s
        check("rhs row reads", om[lv], 0, Np)
        fin = (c - 1) >= c0
        os = np.where(fin & valid, om, odummy + (c - 1 + gD) * s)
        check("rhs row stores", os[lv], 0, Np)
        # a store that is not a finished cell lands on the x ghost g0 - 1
        stray = lv & ~(fin & valid)
        assert (os[stray] % npd[0] == g[0] - 1).all()


def adjoint_x(n, active, x_align):
    g, npd, st, Np = layout(n, active, x_align)
    W0 = n[0] + 6
    V = W0 * n[1] * n[2]
    items = (V + TSEGA - 1) // TSEGA
    lane = np.arange(64)
    for w0 in range(0, items, 20000):
        w = np.arange(w0, min(items, w0 + 20000))[:, None]
        v = w * TSEGA - 2 + lane
        vc = np.clip(v, 0, V - 1)
        r = vc // W0
        x = vc - r * W0 - 3
        j, k = r % n[1], r // n[1]
        rowo = (k + g[2]) * st[2] + (j + g[1]) * st[1]
        o = rowo + g[0] + x
        isrec = (x >= -1) & (x <= n[0])
        check("adjoint stencil reads", np.concatenate([(o - 2)[isrec], (o + 2)[isrec]]), 0, Np)
        check("adjoint left-face flags", (o - 1)[x >= 0], 0, Np)
        check("adjoint right-face flags", o[x <= n[0] - 1], 0, Np)
        check("adjoint cell writes", o[(v == vc) & (lane >= 2) & (lane < 2 + TSEGA)], 0, Np)


CASES = {
    "curved256_aligned": ((256, 256, 256), 7, 1),
    "curved256_3ghost": ((256, 256, 256), 7, 0),
    "batch64x2048": ((2048, 64, 1), 1, 0),
    "batch64x2048_aligned": ((2048, 64, 1), 1, 1),
    "explosion200_2d": ((200, 200, 1), 3, 1),
    "box12": ((12, 12, 12), 7, 0),
    "ragged37x5x3": ((37, 5, 3), 7, 1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_x_sweep_and_stage_maps(name):
    n, act, xa = CASES[name]
    x_sweep(n, act, xa)
    stage_chunks(n, act, xa)
    adjoint_x(n, act, 0)


@pytest.mark.parametrize("name", [k for k, v in CASES.items() if v[1] != 1])
def test_window_maps(name):
    n, act, xa = CASES[name]
    for D in (1, 2):
        if (act >> D) & 1:
            window(n, act, xa, D)
