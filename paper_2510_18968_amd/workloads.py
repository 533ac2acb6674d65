"""Seeded synthetic inputs for the resistive GRMHD stage update.

This module only draws initial data: primitive fields, the fixed background
metric and the conductivity.  It holds none of the method's arithmetic (no
prim2con, no fluxes, no recovery), so both the HIP library and the CPU oracle
can take their inputs from it.  Every array is float64, field-major
``[nf, nz_p, ny_p, nx_p]`` with ghost cells, x fastest.

The workloads are seeded analogues of the paper's initial-value problems
(Sec. IV: 1D shocktube, smooth 3D MHD, a static curved background with a
magnetised blob, and a batch of 1D current-sheet-like problems); the paper's
figures carry no data, so no item of them is reproduced.

Primitive order: rho, p, v^x, v^y, v^z, B^x, B^y, B^z, E^x, E^y, E^z, phi, psi, q.
Metric order: alpha, beta^x, beta^y, beta^z, gamma_xx, gamma_xy, gamma_xz,
gamma_yy, gamma_yz, gamma_zz, K_xx, K_xy, K_xz, K_yy, K_yz, K_zz.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NG = 3
RECON = {"minmod": 0, "mc2": 1, "weno5": 2}
BC = {"periodic": 0, "copy": 1}


@dataclass
class Workload:
    name: str
    n: tuple            # interior cells (nx, ny, nz)
    active: int         # bit d set: fluxes and ghosts along d
    dx: tuple
    x0: tuple           # centre of the first interior cell
    bc: tuple
    gamma_ad: float
    recon: int
    dt: float
    steps: int
    P: np.ndarray       # [14, nz_p, ny_p, nx_p]
    sigma: np.ndarray   # [nz_p, ny_p, nx_p]
    metric: np.ndarray | None = None   # [16, ...] or None (flat)
    kappa: float = 1.0
    extra: dict = field(default_factory=dict)

    @property
    def ghosts(self):
        return tuple(NG if (self.active >> d) & 1 else 0 for d in range(3))

    @property
    def padded(self):
        g = self.ghosts
        return (self.n[2] + 2 * g[2], self.n[1] + 2 * g[1], self.n[0] + 2 * g[0])

    @property
    def interior(self):
        g = self.ghosts
        return tuple(slice(g[d], g[d] + self.n[d]) for d in (2, 1, 0))

    @property
    def n_interior(self):
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


def _coords(n, active, x0, dx):
    """Cell-centre coordinates of the padded grid, as broadcastable (z, y, x)."""
    out = []
    for d in range(3):
        g = NG if (active >> d) & 1 else 0
        idx = np.arange(-g, n[d] + g, dtype=np.float64)
        out.append(x0[d] + idx * dx[d])
    x, y, z = out
    return x[None, None, :], y[None, :, None], z[:, None, None]


def _pad(a, n, active, mode):
    """Embed an interior array (nz, ny, nx) into the padded shape."""
    widths = []
    for d in (2, 1, 0):
        g = NG if (active >> d) & 1 else 0
        widths.append((g, g))
    return np.pad(a, widths, mode=mode)


def _flat_metric_fields(shape):
    m = np.zeros((16,) + shape)
    m[0] = 1.0
    m[4] = m[7] = m[9] = 1.0
    return m


# ----------------------------------------------------------------- config 1
def shocktube(seed=101, sigma0=1e6, n=400, cfl=0.5, t_end=0.4) -> Workload:
    """1D resistive Riemann problem on x in [-0.5, 0.5], flat, Gamma = 2,
    minmod, copy boundaries; left/right states drawn from the seed (the
    paper's shocktube of Sec. IV.A with randomised states)."""
    rng = np.random.default_rng(seed)
    rhoL, rhoR, pL, pR = rng.uniform(0.1, 1.0, 4)
    ByL, BzL, ByR, BzR = rng.uniform(-1.0, 1.0, 4)
    dx = 1.0 / n
    nn = (n, 1, 1)
    x, _, _ = _coords(nn, 1, (-0.5 + 0.5 * dx, 0.0, 0.0), (dx, 1.0, 1.0))
    left = (x < 0.0)[None]
    shape = (1, 1, n + 2 * NG)
    P = np.zeros((14,) + shape)
    P[0] = np.where(left, rhoL, rhoR)
    P[1] = np.where(left, pL, pR)
    P[5] = 0.5
    P[6] = np.where(left, ByL, ByR)
    P[7] = np.where(left, BzL, BzR)
    sigma = np.full(shape, float(sigma0))
    dt = cfl * dx
    steps = int(round(t_end / dt))
    return Workload("shocktube_1d_400", nn, 1, (dx, 1.0, 1.0), (-0.5 + 0.5 * dx, 0.0, 0.0), (1, 1, 1), 2.0,
                    RECON["minmod"], t_end / steps, steps, P, sigma, None,
                    extra=dict(seed=seed, sigma0=sigma0, cfl=cfl))


# ----------------------------------------------------------------- config 2
_KSET = None


def _kset():
    global _KSET
    if _KSET is None:
        r = np.arange(-4, 5)
        k = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
        nrm = np.sqrt((k ** 2).sum(1))
        _KSET = k[(nrm > 0) & (nrm <= 4.0)]
    return _KSET


def _modes(rng, nmodes=8):
    ks = _kset()
    k = ks[rng.integers(0, len(ks), nmodes)]
    a = rng.uniform(-1.0, 1.0, nmodes)
    ph = rng.uniform(0.0, 2.0 * math.pi, nmodes)
    return k, a, ph


def _mode_sum(k, a, ph, x, y, z):
    s = 0.0
    for m in range(len(a)):
        s = s + a[m] * np.cos(2 * math.pi * (k[m, 0] * x + k[m, 1] * y + k[m, 2] * z) + ph[m])
    return s


def _mode_grad(k, a, ph, x, y, z):
    g = [0.0, 0.0, 0.0]
    for m in range(len(a)):
        s = -a[m] * 2 * math.pi * np.sin(2 * math.pi * (k[m, 0] * x + k[m, 1] * y + k[m, 2] * z) + ph[m])
        for d in range(3):
            g[d] = g[d] + k[m, d] * s
    return g


def periodic_box(n=128, seed=201, cfl=0.4, steps=10) -> Workload:
    """Smooth 3D periodic box [0,1)^3, flat, Gamma = 4/3, WENO5: density,
    pressure and velocity from random Fourier modes (|k| <= 4), B from the
    analytic curl of a random vector potential (rms |B| = 0.5), E = -v x B,
    and a smoothed log-uniform conductivity in [1, 1e6]."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    nn = (n, n, n)
    x, y, z = _coords(nn, 7, (0.5 * dx,) * 3, (dx,) * 3)
    shape = (n + 2 * NG,) * 3
    P = np.zeros((14,) + shape)

    def norm_modes():
        k, a, ph = _modes(rng)
        M = _mode_sum(k, a, ph, x, y, z)
        inner = M[NG:-NG, NG:-NG, NG:-NG]
        return M / np.abs(inner).max()

    P[0] = 1.0 + 0.3 * norm_modes()
    P[1] = 0.5 * (1.0 + 0.2 * norm_modes())
    for d in range(3):
        P[2 + d] = (0.5 / math.sqrt(3.0)) * norm_modes()
    grads = []
    for d in range(3):
        k, a, ph = _modes(rng)
        grads.append(_mode_grad(k, a, ph, x, y, z))
    # B = curl A, with grads[c][j] = d_j A_c
    Bx = grads[2][1] - grads[1][2]
    By = grads[0][2] - grads[2][0]
    Bz = grads[1][0] - grads[0][1]
    Bx, By, Bz = (np.broadcast_to(b, shape) for b in (Bx, By, Bz))
    inner = (slice(NG, -NG),) * 3
    rms = math.sqrt(float(np.mean(Bx[inner] ** 2 + By[inner] ** 2 + Bz[inner] ** 2)))
    P[5], P[6], P[7] = Bx * (0.5 / rms), By * (0.5 / rms), Bz * (0.5 / rms)
    vx, vy, vz = P[2], P[3], P[4]
    P[8] = -(vy * P[7] - vz * P[6])
    P[9] = -(vz * P[5] - vx * P[7])
    P[10] = -(vx * P[6] - vy * P[5])
    s = rng.standard_normal((n, n, n))
    for _ in range(3):
        for ax in range(3):
            s = 0.25 * np.roll(s, 1, ax) + 0.5 * s + 0.25 * np.roll(s, -1, ax)
    s = (s - s.min()) / (s.max() - s.min())
    sigma = _pad(10.0 ** (6.0 * s), nn, 7, "wrap")
    return Workload(f"periodic_box_{n}^3", nn, 7, (dx,) * 3, (0.5 * dx,) * 3, (0, 0, 0), 4.0 / 3.0,
                    RECON["weno5"], cfl * dx, steps, P, sigma, None, extra=dict(seed=seed, cfl=cfl))


# ----------------------------------------------------------------- config 3
def curved_blob(n=256, seed=301, recon="weno5", cfl=0.25, steps=20, shift=0.0, atmosphere=False) -> Workload:
    """Static conformally flat background on [-1,1]^3 (gamma_ij = psi^4
    delta_ij, psi = 1 + 0.1 exp(-r^2/0.25), alpha = 1 - 0.3 exp(-r^2/0.25),
    zero shift and extrinsic curvature), a seeded density blob
    rho = 1e-3 + exp(-r^2/0.09)(1 + 0.05 noise), p = 100 rho^2, v = E = 0,
    a poloidal B (max |B| = 1e-3) confined to r < 0.4 from the discrete curl
    of A = a(r) (-y, x, 0), and sigma = 1e6 rho/rho_max + 1; Gamma = 2.
    shift != 0 adds a smooth shift beta = shift b(r) (y, -x, z/2) and
    extrinsic curvature K_ij = shift b(r) k_ij (fixed symmetric k), b the bump,
    to exercise every metric term (input fields, not a solution of Einstein's
    equations).  atmosphere=True selects the stellar-exterior treatment of
    Sec. IV.E instead of the static sigma: sigma = 1e6 max(1 - D_atmo/D, 0)^2
    (eq. dynamo_sigma) with D_atmo = 1e-3, and the artificial atmosphere at
    rho_atmo = 1e-3 with the paper's polytrope K = 100 (Gamma = 2, which is
    also the blob's p = 100 rho^2)."""
    rng = np.random.default_rng(seed)
    dx = 2.0 / n
    nn = (n, n, n)
    x0 = -1.0 + 0.5 * dx
    x, y, z = _coords(nn, 7, (x0,) * 3, (dx,) * 3)
    shape = (n + 2 * NG,) * 3
    r2 = x * x + y * y + z * z
    met = np.zeros((16,) + shape)
    bump = np.exp(-r2 / 0.25)
    psi = 1.0 + 0.1 * bump
    met[0] = 1.0 - 0.3 * bump
    met[4] = met[7] = met[9] = psi ** 4
    if shift:
        met[1], met[2], met[3] = shift * bump * y, -shift * bump * x, 0.5 * shift * bump * z
        for a, kv in enumerate((1.0, 0.2, -0.1, 0.8, 0.3, 0.5)):
            met[10 + a] = shift * kv * bump
    noise = _pad(rng.uniform(-1.0, 1.0, (n, n, n)), nn, 7, "edge")
    P = np.zeros((14,) + shape)
    P[0] = 1e-3 + np.exp(-r2 / 0.09) * (1.0 + 0.05 * noise)
    P[1] = 100.0 * P[0] ** 2

    def a_of(xx, yy, zz):
        rr = xx * xx + yy * yy + zz * zz
        return np.where(rr < 0.16, (0.16 - rr) ** 2, 0.0)

    h = dx

    def A(xx, yy, zz):
        a = a_of(xx, yy, zz)
        return -a * yy, a * xx

    Ax_yp, Ay_yp = A(x, y + h, z)
    Ax_ym, Ay_ym = A(x, y - h, z)
    Ax_zp, Ay_zp = A(x, y, z + h)
    Ax_zm, Ay_zm = A(x, y, z - h)
    Ax_xp, Ay_xp = A(x + h, y, z)
    Ax_xm, Ay_xm = A(x - h, y, z)
    Bx = -(Ay_zp - Ay_zm) / (2 * h)
    By = (Ax_zp - Ax_zm) / (2 * h)
    Bz = (Ay_xp - Ay_xm) / (2 * h) - (Ax_yp - Ax_ym) / (2 * h)
    Bx, By, Bz = (np.broadcast_to(b, shape) for b in (Bx, By, Bz))
    inner = (slice(NG, -NG),) * 3
    bmax = float(np.sqrt(Bx[inner] ** 2 + By[inner] ** 2 + Bz[inner] ** 2).max())
    scale = 1e-3 / bmax
    P[5], P[6], P[7] = Bx * scale, By * scale, Bz * scale
    rho_max = float(P[0][inner].max())
    sigma = 1e6 * P[0] / rho_max + 1.0
    extra = dict(seed=seed, cfl=cfl)
    if atmosphere:
        extra["model"] = dict(sigma_model=2, sigma0=1e6, sigma_Datmo=1e-3, rho_atmo=1e-3, K_atmo=100.0)
    name = f"curved_blob_{n}^3_{recon}" + ("_shift" if shift else "") + ("_atmo" if atmosphere else "")
    return Workload(name, nn, 7, (dx,) * 3, (x0,) * 3, (1, 1, 1), 2.0, RECON[recon],
                    cfl * dx, steps, P, sigma, met, extra=extra)


# ----------------------------------------------------------------- config 5
def sheet_batch(nprob=64, n=2048, seed=501, target_seed=502, cfl=0.25, steps=200) -> Workload:
    """Batch of independent 1D flat problems on x in [-0.5, 0.5] (a batch
    of current sheets with smooth noise): B^y = tanh(x/w) + 0.05 noise,
    rho = 1, p ~ U[0.1, 1] per problem, v = E = 0, per-problem sigma =
    10^U[0,3]; Gamma = 4/3, WENO5, copy boundaries.  The batch index is the
    y dimension, which carries no flux."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    nn = (n, nprob, 1)
    x0 = -0.5 + 0.5 * dx
    x = x0 + dx * np.arange(-NG, n + NG)
    shape = (1, nprob, n + 2 * NG)
    P = np.zeros((14,) + shape)
    w = rng.uniform(0.02, 0.1, nprob)
    pb = rng.uniform(0.1, 1.0, nprob)
    sig = 10.0 ** rng.uniform(0.0, 3.0, nprob)
    for b in range(nprob):
        g = rng.standard_normal(8)
        ph = rng.uniform(0.0, 2 * math.pi, 8)
        nz = sum((g[m - 1] / m) * np.sin(2 * math.pi * m * (x + 0.5) + ph[m - 1]) for m in range(1, 9))
        nz = nz / np.abs(nz[NG:-NG]).max()
        P[6, 0, b] = np.tanh(x / w[b]) + 0.05 * nz
        P[1, 0, b] = pb[b]
    P[0] = 1.0
    sigma = np.broadcast_to(sig[None, :, None], shape).copy()
    trng = np.random.default_rng(target_seed)
    sig_t = 10.0 ** trng.uniform(0.0, 3.0, nprob)
    return Workload(f"sheet_batch_{nprob}x{n}", nn, 1, (dx, 1.0, 1.0), (x0, 0.0, 0.0), (1, 1, 1), 4.0 / 3.0,
                    RECON["weno5"], cfl * dx, steps, P, sigma, None,
                    extra=dict(seed=seed, sigma_problem=sig, sigma_target=sig_t))


# ------------------------------------------------- paper tests of Sec. IV
def brio_wu(sigma0=1e6, n=400, cfl=0.25, t_end=0.4, sigma_exp=None) -> Workload:
    """The shocktube of Sec. IV.A as printed: (rho, p, B^y) = (1, 1, 0.5) for
    x < 0 and (0.125, 0.1, -0.5) for x > 0, v = B^x = B^z = E = 0, Gamma = 2,
    minmod, copy boundaries, on [-0.5, 0.5] with Delta x = 1/n.  With
    sigma_exp (gamma of eq. sigma_evol) the conductivity is the model sigma0
    D^gamma; otherwise the static field sigma0."""
    dx = 1.0 / n
    nn = (n, 1, 1)
    x0 = -0.5 + 0.5 * dx
    x, _, _ = _coords(nn, 1, (x0, 0.0, 0.0), (dx, 1.0, 1.0))
    left = (x < 0.0)[None]
    shape = (1, 1, n + 2 * NG)
    P = np.zeros((14,) + shape)
    P[0] = np.where(left, 1.0, 0.125)
    P[1] = np.where(left, 1.0, 0.1)
    P[6] = np.where(left, 0.5, -0.5)
    sigma = np.full(shape, float(sigma0))
    steps = int(round(t_end / (cfl * dx)))
    extra = dict(sigma0=sigma0, sigma_exp=sigma_exp, cfl=cfl)
    if sigma_exp is not None:
        extra["model"] = dict(sigma_model=1, sigma0=sigma0, sigma_exp=float(sigma_exp))
    return Workload(f"brio_wu_{n}" + ("" if sigma_exp is None else f"_gamma{sigma_exp:g}"), nn, 1, (dx, 1.0, 1.0),
                    (x0, 0.0, 0.0), (1, 1, 1), 2.0, RECON["minmod"], t_end / steps, steps, P, sigma, None, extra=extra)


def alfven_speed(rho, p, eta_A, B0, gamma_ad):
    """eq. Alf_vel, with h the enthalpy density rho (1 + eps) + p of an ideal gas"""
    h = rho + gamma_ad / (gamma_ad - 1.0) * p
    a = 2.0 * B0 ** 2 / (h + B0 ** 2 * (1.0 + eta_A ** 2))
    b = 2.0 * eta_A * B0 ** 2 / (h + B0 ** 2 * (1.0 + eta_A ** 2))
    return math.sqrt(a / (1.0 + math.sqrt(1.0 - b * b)))


def cp_alfven(n=200, cfl=0.25, sigma0=1e6, rho=1.0, p=1.0, eta_A=1.0, B0=1.1547, periods=1.0) -> Workload:
    """The large-amplitude circularly polarised Alfven wave of Sec. IV.D
    (eqs. Bi, vyvz, Alf_vel, E = -v x B): periodic x in [-0.5, 0.5], k = 2 pi,
    Gamma = 2, MC2, uniform sigma; run for `periods` wave periods L/v_A."""
    G = 2.0
    vA = alfven_speed(rho, p, eta_A, B0, G)
    dx = 1.0 / n
    nn = (n, 1, 1)
    x0 = -0.5 + 0.5 * dx
    x = x0 + dx * np.arange(-NG, n + NG)
    k = 2.0 * math.pi
    shape = (1, 1, n + 2 * NG)
    P = np.zeros((14,) + shape)
    By, Bz = eta_A * B0 * np.cos(k * x), eta_A * B0 * np.sin(k * x)
    P[0], P[1], P[5] = rho, p, B0
    P[6, 0, 0], P[7, 0, 0] = By, Bz
    P[3, 0, 0], P[4, 0, 0] = -vA / B0 * By, -vA / B0 * Bz
    P[9, 0, 0], P[10, 0, 0] = vA * Bz, -vA * By
    T = periods / vA
    steps = int(math.ceil(T / (cfl * dx)))
    return Workload(f"cp_alfven_{n}", nn, 1, (dx, 1.0, 1.0), (x0, 0.0, 0.0), (0, 0, 0), G, RECON["mc2"],
                    T / steps, steps, P, np.full(shape, float(sigma0)), None,
                    extra=dict(v_A=vA, period=1.0 / vA, By0=By.copy()))


def cylindrical_explosion(n=200, cfl=0.25, sigma0=1e6, t_end=4.0, steps=None, recon="minmod") -> Workload:
    """The 2D cylindrical explosion of Sec. IV.B: [-6, 6]^2 with n x n cells,
    Gamma = 4/3, copy boundaries, uniform B^x = 0.05, v = E = 0, sigma0;
    rho = 0.01, p = 1 inside r = 0.8, rho = p = 0.001 outside r = 1, and in
    between log-linear in r from the inner to the outer value (the printed
    interpolation has the two logarithms swapped, which would jump at both
    radii; the continuous reading is used)."""
    L = 12.0
    dx = L / n
    nn = (n, n, 1)
    x0 = -6.0 + 0.5 * dx
    x, y, _ = _coords(nn, 3, (x0, x0, 0.0), (dx, dx, 1.0))
    r = np.sqrt(x * x + y * y)
    rin, rout = 0.8, 1.0

    def prof(vin, vout):
        t = np.clip((r - rin) / (rout - rin), 0.0, 1.0)
        mid = np.exp((1.0 - t) * math.log(vin) + t * math.log(vout))
        return np.where(r <= rin, vin, np.where(r >= rout, vout, mid))

    shape = (1, n + 2 * NG, n + 2 * NG)
    P = np.zeros((14,) + shape)
    P[0] = np.broadcast_to(prof(0.01, 0.001), shape)
    P[1] = np.broadcast_to(prof(1.0, 0.001), shape)
    P[5] = 0.05
    dt = cfl * dx
    if steps is None:
        steps = int(round(t_end / dt))
        dt = t_end / steps
    return Workload(f"cylindrical_explosion_{n}^2", nn, 3, (dx, dx, 1.0), (x0, x0, 0.0), (1, 1, 1), 4.0 / 3.0,
                    RECON[recon], dt, steps, P, np.full(shape, float(sigma0)), None, extra=dict(cfl=cfl))


# h(x) = sum_m a_m sin(2 pi n_m . x + c_m) of the tilted slicing (period 1 along each axis)
SLICING_MODES = [
    (0.034, (1.0, 0.0, 0.0), 0.3),
    (0.026, (0.0, 1.0, 0.0), 1.1),
    (0.022, (0.0, 0.0, 1.0), 2.0),
    (0.019, (1.0, 1.0, 0.0), 0.7),
    (0.015, (0.0, 1.0, -1.0), 2.9),
    (0.015, (1.0, 0.0, 1.0), 4.1),
]


def tilted_slicing_fields(x, y, z, dims=3, q0=0.0, psi0=0.0, phi0=0.0, B0=(0.31, -0.22, 0.17), rho0=1.0,
                          p0=0.6, xc=(0.07, -0.05, 0.03)):
    """Flat spacetime in the stationary slicing t = T + h(x) (T, X^i
    Minkowski; x^i = X^i), with a static Minkowski-frame state: fluid at
    rest, uniform B0, uniform charge q0 with E = q0 (X - xc)/dims and the
    pressure p0 + q0^2 |X - xc|^2/(2 dims) that balances q0 E, uniform psi0,
    phi0.  Returns (metric [16], primitives [14]) at the points, both closed
    form: gamma_ij = delta_ij - h_i h_j, alpha = (1 - |grad h|^2)^(-1/2),
    beta^i = alpha^2 h_i, K_ij = alpha h_ij; v^i = alpha h_i,
    E = alpha (E_flat - h x B0), B = alpha (B0 + h x E_flat), q = alpha q0.
    Modes with a component along an inactive dimension are dropped."""
    X = np.broadcast_arrays(x, y, z)
    shp = X[0].shape
    kk = 2.0 * math.pi
    hi = np.zeros((3,) + shp)
    hij = np.zeros((3, 3) + shp)
    for a, nv, c in SLICING_MODES:
        if any(nv[d] != 0.0 for d in range(dims, 3)):
            continue
        th = kk * (nv[0] * X[0] + nv[1] * X[1] + nv[2] * X[2]) + c
        cs, sn = np.cos(th), np.sin(th)
        for i in range(3):
            hi[i] += a * kk * nv[i] * cs
            for j in range(3):
                hij[i, j] -= a * kk * kk * nv[i] * nv[j] * sn
    alp = 1.0 / np.sqrt(1.0 - (hi * hi).sum(0))
    met = np.zeros((16,) + shp)
    met[0] = alp
    met[1:4] = alp * alp * hi
    for s, (i, j) in enumerate([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
        met[4 + s] = (1.0 if i == j else 0.0) - hi[i] * hi[j]
        met[10 + s] = alp * hij[i, j]
    R = np.array([X[d] - xc[d] if d < dims else np.zeros(shp) for d in range(3)])
    Ef = q0 * R / dims
    Bf = np.array([np.full(shp, b) for b in B0])
    P = np.zeros((14,) + shp)
    P[0] = rho0
    P[1] = p0 + q0 * q0 * (R * R).sum(0) / (2.0 * dims)
    P[2:5] = alp * hi
    P[5:8] = alp * (Bf + np.cross(hi, Ef, axis=0))
    P[8:11] = alp * (Ef - np.cross(hi, Bf, axis=0))
    P[11] = phi0
    P[12] = psi0
    P[13] = alp * q0
    return met, P


def tilted_slicing(n=16, dims=3, sigma0=100.0, psi0=0.2, phi0=-0.15, recon="weno5", cfl=0.25, steps=2) -> Workload:
    """A static, uncharged Minkowski state seen from a tilted stationary
    slicing (see tilted_slicing_fields) on the periodic unit box
    [-0.5, 0.5)^dims: every shift and extrinsic-curvature term is active and
    the exact solution is stationary; kappa = 0 keeps the uniform cleaning
    scalars stationary."""
    dx = 1.0 / n
    act = (1 << dims) - 1
    nn = tuple(n if d < dims else 1 for d in range(3))
    x0 = tuple(-0.5 + 0.5 * dx if d < dims else 0.0 for d in range(3))
    x, y, z = _coords(nn, act, x0, (dx,) * 3)
    met, P = tilted_slicing_fields(x, y, z, dims=dims, psi0=psi0, phi0=phi0)
    shape = P.shape[1:]
    return Workload(f"tilted_slicing_{n}_{dims}d", nn, act, (dx,) * 3, x0, (0, 0, 0), 4.0 / 3.0, RECON[recon],
                    cfl * dx, steps, P, np.full(shape, float(sigma0)), met, kappa=0.0)


def by_name(name: str, **kw) -> Workload:
    return {"shocktube": shocktube, "periodic_box": periodic_box, "curved_blob": curved_blob,
            "sheet_batch": sheet_batch, "brio_wu": brio_wu, "cp_alfven": cp_alfven,
            "cylindrical_explosion": cylindrical_explosion, "tilted_slicing": tilted_slicing}[name](**kw)
