"""Helpers for GPU-vs-oracle parity: per-field relative errors.

Normalisation: each field's max |gpu - oracle| over interior cells is divided
by the field's max |oracle|; the electromagnetic, cleaning and charge fields
(indices 5..13 of both P and U) are divided by at least the largest E or B
magnitude, since phi, psi and q start at zero and E can vanish.  The
components of the velocity (P indices 2..4) or of the momentum (U indices
1..3) are divided by at least the largest component of the same vector: a
component that vanishes in exact arithmetic (v^z of a flow in the x-y plane)
holds only rounding on both sides.
"""
import numpy as np

EM = set(range(5, 14))
NAMES_P = ["rho", "p", "vx", "vy", "vz", "Bx", "By", "Bz", "Ex", "Ey", "Ez", "phi", "psi", "q"]
NAMES_U = ["D", "Sx", "Sy", "Sz", "tau", "Bx", "By", "Bz", "Ex", "Ey", "Ez", "Phi", "Psi", "Q"]


EPS = 2.0 ** -53


VEC = {"P": (2, 5), "U": (1, 4)}


def rel_errors(gpu, ref, interior, em=True, floor=0.0, kind=None):
    """per-field max |gpu - ref| / scale; floor: lower bound of every scale
    (R arrays use |E|/(gamma dt), the size of the E change they encode);
    kind "P" or "U" names the array, for the vector normalisation"""
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    nf = ref.shape[0]
    sl = (slice(None),) + tuple(interior)
    g, r = gpu[sl], ref[sl]
    em_scale = float(np.abs(r[5:11]).max()) if (em and nf == 14) else 0.0
    lo, hi = VEC[kind] if (kind and nf == 14) else (0, 0)
    vec_scale = float(np.abs(r[lo:hi]).max()) if hi > lo else 0.0
    out = []
    for f in range(nf):
        d = float(np.abs(g[f] - r[f]).max())
        s = max(float(np.abs(r[f]).max()), floor)
        if em and nf == 14 and f in EM:
            s = max(s, em_scale)
        if lo <= f < hi:
            s = max(s, vec_scale)
        out.append(d / s if s > 0 else d)
    return np.array(out)


def tolerances(nf, base, sigma_max=0.0, dt_over_dx=0.0, n_flux=1, t_total=0.0):
    """Parity bar per field.  Every field gets `base` (1e-12 in FP64) except
    the charge (index 13), whose flux carries J = sigma W [E + v x B - (v.E) v]
    with the bracket a near-cancelling difference of O(|E|) terms: two correct
    FP64 evaluations differ by ~eps sigma |E| per face, i.e. by
    eps sigma (dt/dx) |E| per flux evaluation, growing like sqrt(n_flux); and
    the E-cleaning scalar Psi (index 12), whose only source coupling to the
    charge is + alpha Q (alpha <= 1): its deviation is at most the time
    integral of the charge's, t_total times the charge bar, on top of base."""
    tol = np.full(nf, base)
    if nf == 14:
        tol[13] = max(base, EPS * sigma_max * dt_over_dx * np.sqrt(n_flux))
        tol[12] = base + t_total * tol[13]
    return tol


def report(tag, errs, names=None):
    names = names or [str(i) for i in range(len(errs))]
    worst = int(np.argmax(errs))
    print(f"[parity] {tag}: max rel err {errs.max():.3e} ({names[worst]}) | " +
          " ".join(f"{n}={e:.1e}" for n, e in zip(names, errs)), flush=True)
