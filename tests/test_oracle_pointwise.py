"""Pins of the oracle's pointwise pieces against closed forms, library
routines, textbook special cases and brute force (CPU only).

Each test names the passage of arXiv:2510.18968 it checks.
"""
import json
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))


def conformal(psi, alpha=1.0):
    m = np.zeros(16)
    m[0] = alpha
    m[4] = m[7] = m[9] = psi ** 4
    return m


def random_metric(rng, with_shift=True):
    m = np.zeros(16)
    m[0] = rng.uniform(0.6, 1.0)
    if with_shift:
        m[1:4] = rng.uniform(-0.1, 0.1, 3)
    A = rng.normal(size=(3, 3)) * 0.15
    g = np.eye(3) * rng.uniform(0.9, 1.4) + A @ A.T
    m[4:10] = [g[0, 0], g[0, 1], g[0, 2], g[1, 1], g[1, 2], g[2, 2]]
    m[10:16] = rng.normal(size=6) * 0.05
    return m, g


def sym(m, off):
    a = m[off:off + 6]
    return np.array([[a[0], a[1], a[2]], [a[1], a[3], a[4]], [a[2], a[4], a[5]]])


def random_state(rng, g=None, vmax=0.9, bmax_over_p=10.0, near_ideal=False):
    g = np.eye(3) if g is None else g
    P = np.zeros(14)
    P[0] = rng.uniform(0.1, 2.0)
    P[1] = rng.uniform(0.05, 2.0)
    v = rng.normal(size=3)
    v *= rng.uniform(0.0, vmax) / math.sqrt(v @ g @ v)
    P[2:5] = v
    B = rng.normal(size=3)
    B *= math.sqrt(rng.uniform(0, bmax_over_p) * P[1] / (B @ g @ B))
    P[5:8] = B
    E = rng.normal(size=3)
    E *= math.sqrt(rng.uniform(0, bmax_over_p) * P[1] / (E @ g @ E))
    if near_ideal:
        # E = -v x B (flat components) plus a small resistive part
        E = -np.cross(v, B) + 0.05 * E
    P[8:11] = E
    P[11:14] = rng.uniform(-0.5, 0.5, 3)
    return P


# ---------------------------------------------------------------- metric
def test_metric_inverse_and_determinant(orc):
    """Sec. II.A: gamma^{ij} is the algebraic inverse of gamma_ij; sqrt(gamma)."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        m, g = random_metric(rng)
        gi, sg = orc.point_metric(m)
        assert np.allclose(gi, np.linalg.inv(g), rtol=1e-14, atol=1e-14)
        assert abs(sg - math.sqrt(np.linalg.det(g))) <= 1e-14 * sg


# ---------------------------------------------------------------- prim2con
def test_prim2con_flat_static_hand_values(orc):
    """eqs. conserved_dens/_tau/_S with v = 0, flat: D = rho, S = E x B,
    tau = rho eps + (E^2 + B^2)/2 with eps = p/((Gamma-1) rho)."""
    G = 2.0
    P = np.zeros(14)
    P[0], P[1] = 0.7, 0.3
    P[5:8] = [0.2, -0.4, 0.5]
    P[8:11] = [0.1, 0.3, -0.2]
    P[11:14] = [0.01, 0.02, 0.03]
    U = orc.point_prim2con(P, G)
    E, B = P[8:11], P[5:8]
    assert U[0] == pytest.approx(0.7, abs=1e-16)
    assert np.allclose(U[1:4], np.cross(E, B), atol=1e-16)
    assert U[4] == pytest.approx(0.3 / (G - 1) + 0.5 * (E @ E + B @ B), abs=1e-15)
    assert np.allclose(U[5:8], B) and np.allclose(U[8:11], E) and np.allclose(U[11:14], P[11:14])


def test_prim2con_textbook_hydro(orc):
    """E = B = 0, flat: D = rho W, S = rho h W^2 v, tau = rho h W^2 - p - D
    with specific enthalpy 1 + Gamma/(Gamma-1) p/rho (special relativistic
    hydro, the ideal-gas limit of eqs. conserved_*)."""
    G = 4.0 / 3.0
    P = np.zeros(14)
    P[0], P[1] = 1.3, 0.4
    P[2:5] = [0.3, -0.2, 0.5]
    W = 1.0 / math.sqrt(1 - P[2:5] @ P[2:5])
    hs = 1.0 + G / (G - 1) * P[1] / P[0]
    U = orc.point_prim2con(P, G)
    assert U[0] == pytest.approx(P[0] * W, rel=1e-15)
    assert np.allclose(U[1:4], P[0] * hs * W * W * P[2:5], rtol=1e-15)
    assert U[4] == pytest.approx(P[0] * hs * W * W - P[1] - P[0] * W, rel=1e-14)


def test_prim2con_conformal_scaling(orc):
    """gamma_ij = psi^4 delta_ij: sqrt(gamma) = psi^6, epsilon_ijk =
    psi^6 eta_ijk, E^2 = psi^4 |E|^2; v = 0 gives D = psi^6 rho,
    S_i = psi^12 (E x B)_i, tau = psi^6 (rho eps + psi^4 (|E|^2+|B|^2)/2)."""
    G, psi = 2.0, 1.07
    P = np.zeros(14)
    P[0], P[1] = 0.9, 0.2
    P[5:8] = [0.3, 0.1, -0.2]
    P[8:11] = [-0.1, 0.2, 0.25]
    P[13] = 0.05
    U = orc.point_prim2con(P, G, conformal(psi, 0.8))
    E, B = P[8:11], P[5:8]
    s6 = psi ** 6
    assert U[0] == pytest.approx(s6 * 0.9, rel=1e-15)
    assert np.allclose(U[1:4], psi ** 12 * np.cross(E, B), rtol=1e-14)
    assert U[4] == pytest.approx(s6 * (0.2 / (G - 1) + 0.5 * psi ** 4 * (E @ E + B @ B)), rel=1e-14)
    assert np.allclose(U[5:8], s6 * B) and np.allclose(U[8:11], s6 * E) and U[13] == pytest.approx(s6 * 0.05)


# ---------------------------------------------------------------- con2prim
@pytest.mark.parametrize("curved", [False, True])
def test_con2prim_round_trip(orc, curved):
    """Sec. III.B recovery (E fixed): con2prim(prim2con(x)) = x, v <= 0.9,
    B^2/p, E^2/p <= 10, flat and general curved metrics."""
    rng = np.random.default_rng(7 if curved else 3)
    worst = 0.0
    for t in range(300):
        if curved:
            m, g = random_metric(rng)
        else:
            m, g = None, np.eye(3)
        G = [2.0, 4.0 / 3.0][t % 2]
        P = random_state(rng, g)
        U = orc.point_prim2con(P, G, m)
        Pg = P.copy()
        Pg[1] *= rng.uniform(0.7, 1.4)
        Pg[2:5] *= rng.uniform(0.5, 1.0)
        Pr, E, st, it = orc.point_coupled(U, U[8:11], 0.0, 0.0, Pg, G, m)
        assert st == 0, (t, st, it)
        err = np.abs(Pr - P) / np.maximum(np.abs(P), 1e-3 * max(1.0, np.abs(P).max()))
        worst = max(worst, err.max())
    assert worst <= 1e-12, worst


def test_hydro_recovery_vs_bisection(orc):
    """E = B = 0 reduces Sec. III.B to ideal-gas hydro recovery; compare with
    a long-double bisection on f(p) = (Gamma-1) rho eps - p."""
    rng = np.random.default_rng(11)
    L = np.longdouble
    for _ in range(40):
        G = 2.0
        P = np.zeros(14)
        P[0], P[1] = rng.uniform(0.1, 1), rng.uniform(0.01, 1)
        P[2:5] = rng.uniform(-0.5, 0.5, 3)
        U = orc.point_prim2con(P, G)
        D, S, tau = L(U[0]), [L(x) for x in U[1:4]], L(U[4])
        S2 = sum(x * x for x in S)

        def f(p):
            den = tau + D + p
            v2 = S2 / (den * den)
            W = 1 / np.sqrt(L(1) - v2)
            rho = D / W
            eps = (tau - D * (W - 1) - p * (W * W - 1)) / (D * W)
            return (L(G) - 1) * rho * eps - p

        lo = max(L(1e-12), np.sqrt(S2) - tau - D + L(1e-15))
        hi = L(10.0)
        for _ in range(200):
            mid = (lo + hi) / 2
            if f(mid) > 0:
                lo = mid
            else:
                hi = mid
        pb = float((lo + hi) / 2)
        Pr, E, st, it = orc.point_coupled(U, U[8:11], 0.0, 0.0, P * 1.2, G)
        assert st == 0
        assert abs(Pr[1] - pb) <= 2e-13 * pb


# ---------------------------------------------------------------- implicit E
def test_implicit_E_matches_linear_solve(orc):
    """eq. 3D_NR at fixed v is linear in E: the Newton-Raphson result equals
    numpy.linalg.solve of ((1+c) I - c v v_l^T) E = E* - c eps^{ijk} v_j B_k."""
    rng = np.random.default_rng(5)
    for t in range(50):
        m, g = random_metric(rng)
        sg = math.sqrt(np.linalg.det(g))
        v = rng.normal(size=3)
        v *= rng.uniform(0, 0.9) / math.sqrt(v @ g @ v)
        Bc = rng.normal(size=3)
        Es = rng.normal(size=3)
        c = 10.0 ** rng.uniform(-3, 6)
        vl, Bl = g @ v, g @ Bc
        vxb = np.cross(vl, Bl) / sg
        A = (1 + c) * np.eye(3) - c * np.outer(v, vl)
        ref = np.linalg.solve(A, Es - c * vxb)
        E = orc.point_esolve(v, Bc, Es, c, m)
        assert np.allclose(E, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_implicit_E_limits(orc):
    """sigma -> 0 leaves E*; sigma -> infinity gives the ideal E = -v x B."""
    v = np.array([0.3, -0.2, 0.1])
    Bc = np.array([0.5, 0.7, -0.3])
    Es = np.array([0.1, 0.2, 0.3])
    assert np.array_equal(orc.point_esolve(v, Bc, Es, 0.0), Es)
    E = orc.point_esolve(v, Bc, Es, 1e14)
    assert np.allclose(E, -np.cross(v, Bc), atol=1e-12)


# ---------------------------------------------------------------- coupled root
def stage_residuals(orc, U, Estar, adt, sigma, P, E, G, m):
    """Residuals of the defining equations of the coupled stage solve."""
    Ur = orc.point_prim2con(P, G, m)
    sel = [0, 1, 2, 3, 4, 5, 6, 7, 11, 12, 13]
    r_cons = np.abs(Ur[sel] - U[sel]) / np.maximum(np.abs(U[sel]), 1.0)
    r_e = np.abs(Ur[8:11] - E).max()
    R = orc.point_stiff(P[2:5], E, Ur[5:8], sigma, m)
    # the equation E (1 + c) - ... = E* is scaled by 1 + c, c = a dt alpha W sigma,
    # so that the residual is measured against the rounding of its terms
    c = adt * sigma / math.sqrt(max(1e-300, 1.0 - min(0.999999, float(P[2:5] @ P[2:5]))))
    r_impl = np.abs(E - Estar - adt * R).max() / (max(1.0, np.abs(E).max(), np.abs(Estar).max()) * (1.0 + c))
    return r_cons.max(), r_e, r_impl


@pytest.mark.parametrize("curved", [False, True])
def test_coupled_root_residuals(orc, curved):
    """Sec. III.B with the stiff E (eq. 3D_NR): the output satisfies the
    implicit stage equation E = E* + a dt R_E(E, v) and reproduces the
    conserved variables, for sigma up to 1e8 and B^2/p up to 10."""
    rng = np.random.default_rng(21 if curved else 17)
    for t in range(200):
        m, g = (random_metric(rng) if curved else (None, np.eye(3)))
        G = [2.0, 4.0 / 3.0][t % 2]
        P = random_state(rng, g, vmax=0.8, near_ideal=True)
        sigma = 10.0 ** rng.uniform(0, 8)
        adt = rng.uniform(1e-4, 1e-2)
        # the stage input: conserved vars of a state whose E is then perturbed
        U = orc.point_prim2con(P, G, m)
        Estar = U[8:11] + rng.normal(size=3) * 0.01
        Pg = P.copy()
        Pg[1] *= 1.1
        Pr, E, st, it = orc.point_coupled(U, Estar, adt, sigma, Pg, G, m)
        assert st == 0, (t, st, it)
        rc, re, ri = stage_residuals(orc, U, Estar, adt, sigma, Pr, E, G, m)
        assert rc <= 1e-12 and re <= 1e-13 and ri <= 1e-14, (t, rc, re, ri)


def test_coupled_root_equals_paper_iteration(orc):
    """Where the paper's iteration (Picard in v, Newton in p) converges, it
    reaches the same root as the oracle's Newton solve."""
    rng = np.random.default_rng(23)
    n_cmp = 0
    for t in range(200):
        P = random_state(rng, vmax=0.6, bmax_over_p=1.0, near_ideal=True)
        G = 2.0
        U = orc.point_prim2con(P, G)
        Estar = U[8:11] + rng.normal(size=3) * 0.02
        sigma, adt = 10.0 ** rng.uniform(0, 6), 1e-3
        Pn, En, st, _ = orc.point_coupled(U, Estar, adt, sigma, P, G)
        Pp, Ep, sp, _ = orc.point_recover_paper(U, Estar, adt, sigma, P, G, maxit=2000)
        assert st == 0
        if sp == 0:
            n_cmp += 1
            assert np.allclose(Pn, Pp, rtol=1e-12, atol=1e-13), t
            assert np.allclose(En, Ep, rtol=1e-12, atol=1e-13), t
    assert n_cmp >= 150


def test_coupled_root_unique_from_many_guesses(orc):
    """Several correct answers would show up as different roots from
    different starting guesses: 20 random guesses per state, one root."""
    rng = np.random.default_rng(29)
    for t in range(20):
        P = random_state(rng, vmax=0.7, near_ideal=True)
        U = orc.point_prim2con(P, 2.0)
        Estar = U[8:11] + rng.normal(size=3) * 0.01
        roots = []
        for k in range(20):
            Pg = P.copy()
            Pg[1] *= rng.uniform(0.3, 3.0)
            Pg[2:5] = rng.uniform(-0.4, 0.4, 3)
            Pr, E, st, _ = orc.point_coupled(U, Estar, 2e-3, 1e5, Pg, 2.0)
            if st == 0:
                roots.append(np.concatenate([Pr, E]))
        assert len(roots) >= 15
        roots = np.array(roots)
        assert np.abs(roots - roots[0]).max() <= 1e-11 * max(1.0, np.abs(roots[0]).max())


def test_coupled_sigma_zero_is_plain_recovery(orc):
    rng = np.random.default_rng(31)
    P = random_state(rng)
    U = orc.point_prim2con(P, 2.0)
    Estar = U[8:11] * 0.9
    Pa, Ea, sa, _ = orc.point_coupled(U, Estar, 1e-3, 0.0, P, 2.0)
    assert sa == 0 and np.array_equal(Ea, Estar)


def test_recovery_failure_flags(orc):
    """Unphysical inputs are flagged, never repaired (status < 0 and the
    guess is returned): tau < 0, S^2 > (tau + D)^2, D <= 0, NaN, and an
    iteration cap of one."""
    G = 2.0
    P = np.zeros(14)
    P[0], P[1], P[2:5] = 1.0, 0.5, [0.3, 0.1, 0.0]
    U = orc.point_prim2con(P, G)
    cases = []
    u = U.copy(); u[4] = -0.1; cases.append(u)
    u = U.copy(); u[1] = 3.0 * (U[4] + U[0]); cases.append(u)
    u = U.copy(); u[0] = 0.0; cases.append(u)
    u = U.copy(); u[2] = np.nan; cases.append(u)
    for u in cases:
        Pr, E, st, it = orc.point_coupled(u, u[8:11], 0.0, 0.0, P * 1.1, G)
        assert st < 0
        assert np.array_equal(Pr, P * 1.1)
    Pr, E, st, it = orc.point_coupled(U, U[8:11], 0.0, 0.0, P * 1.5, G, maxit=1)
    assert st == orc.ST_NOCONV


# ---------------------------------------------------------------- reconstruction
def cell_avg_poly(coef, xl, xr):
    """exact cell average of sum_k coef[k] x^k over [xl, xr]"""
    F = lambda x: sum(c * x ** (k + 1) / (k + 1) for k, c in enumerate(coef))
    return (F(xr) - F(xl)) / (xr - xl)


def test_weno5_exact_for_quadratic_cell_averages(orc):
    """Every WENO5 candidate stencil (Shu 1998, cited in Sec. III) is exact
    for cell averages of a quadratic, hence so is any convex combination."""
    rng = np.random.default_rng(41)
    for _ in range(50):
        coef = rng.normal(size=3) * 10.0 ** rng.uniform(-2, 2, 3)
        h = 10.0 ** rng.uniform(-3, 0)
        f = np.array([cell_avg_poly(coef, (j - 0.5) * h, (j + 0.5) * h) for j in range(-2, 3)])
        fm, fp = orc.recon(orc.REC_WENO5, f)
        ex = lambda x: coef[0] + coef[1] * x + coef[2] * x * x
        scale = np.abs(f).max()
        assert abs(fp - ex(0.5 * h)) <= 1e-12 * scale
        assert abs(fm - ex(-0.5 * h)) <= 1e-12 * scale


def test_weno5_fifth_order_on_smooth_data(orc):
    """On smooth data the nonlinear weights approach the ideal ones and the
    face value converges at fifth order."""
    errs = []
    for h in (0.04, 0.02, 0.01):
        x0 = 0.3
        f = np.array([(math.cos(x0 + (j - 0.5) * h) - math.cos(x0 + (j + 0.5) * h)) / h for j in range(-2, 3)])
        fm, fp = orc.recon(orc.REC_WENO5, f)
        errs.append(abs(fp - math.sin(x0 + 0.5 * h)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) >= 4.5, rates


@pytest.mark.parametrize("method", [0, 1])
def test_tvd_exact_on_linear_data(orc, method):
    """minmod and MC2 (Sec. IV.A, IV.D) reproduce linear data exactly."""
    f = np.array([1.0, 1.5, 2.0, 2.5, 3.0])
    fm, fp = orc.recon(method, f)
    assert fm == pytest.approx(1.75, abs=1e-15) and fp == pytest.approx(2.25, abs=1e-15)
    fm, fp = orc.recon(method, f[::-1].copy())
    assert fm == pytest.approx(2.25, abs=1e-15) and fp == pytest.approx(1.75, abs=1e-15)


def test_tvd_limiters_at_extremum_and_slopes(orc):
    """At an extremum both TVD limiters give zero slope; MC2 takes
    min(2|dm|, 2|dp|, |dm+dp|/2) of common sign, minmod min(|dm|, |dp|)."""
    for m in (0, 1):
        assert orc.recon(m, np.array([0.0, 1.0, 2.0, 1.0, 0.0])) == (2.0, 2.0)
    fm, fp = orc.recon(0, np.array([0.0, 0.0, 1.0, 4.0, 0.0]))
    assert (fm, fp) == (0.5, 1.5)
    fm, fp = orc.recon(1, np.array([0.0, 0.0, 1.0, 4.0, 0.0]))
    assert (fm, fp) == (0.0, 2.0)            # min(2*1, 2*3, 2) = 2
    fm, fp = orc.recon(1, np.array([0.0, 0.0, 1.0, 1.2, 0.0]))
    assert fm == pytest.approx(0.8) and fp == pytest.approx(1.2)   # min(2, 0.4, 0.6) = 0.4


# ---------------------------------------------------------------- fluxes / HLLE
def test_flat_maxwell_fluxes_are_textbook_curls(orc):
    """Flat space, eq. GRRMHD_flux_form: dt B = -curl E and dt E = curl B - J
    in flux form, plus the cleaning couplings."""
    P = np.zeros(14)
    P[0], P[1] = 1.0, 1.0
    P[5:8] = [0.1, 0.2, 0.3]
    P[8:11] = [0.4, 0.5, 0.6]
    P[11], P[12] = 0.07, 0.09
    for d in range(3):
        F = orc.point_flux(P, 2.0, 0.0, d)
        E, B = P[8:11], P[5:8]
        e = np.zeros(3); e[d] = 1.0
        # dt B = -curl E = -d_d (e_d x E) and dt E = curl B = d_d (e_d x B), so
        # F^d(B^i) = (e_d x E)^i + delta^{id} phi and F^d(E^i) = -(e_d x B)^i + delta^{id} psi
        assert np.allclose(F[5:8], np.cross(e, E) + e * P[11], atol=1e-16)
        assert np.allclose(F[8:11], -np.cross(e, B) + e * P[12], atol=1e-16)
        assert F[11] == pytest.approx(B[d]) and F[12] == pytest.approx(E[d])


def test_flat_hydro_flux_textbook(orc):
    G = 2.0
    P = np.zeros(14)
    P[0], P[1], P[2:5] = 0.8, 0.6, [0.4, -0.1, 0.2]
    v = P[2:5]
    W = 1 / math.sqrt(1 - v @ v)
    h = P[0] + G / (G - 1) * P[1]
    F = orc.point_flux(P, G, 0.0, 0)
    assert F[0] == pytest.approx(P[0] * W * v[0], rel=1e-15)
    assert np.allclose(F[1:4], h * W * W * v * v[0] + np.array([P[1], 0, 0]), rtol=1e-14)
    assert F[4] == pytest.approx((h * W * W - P[0] * W) * v[0], rel=1e-14)


def test_hlle_consistency_and_flat_form(orc):
    """HLLE (Sec. III): F(U, U) = F(U); flat speeds are +-1 so
    F = (F_L + F_R)/2 - (U_R - U_L)/2."""
    rng = np.random.default_rng(43)
    for _ in range(20):
        PL, PR = random_state(rng, vmax=0.5), random_state(rng, vmax=0.5)
        d = int(rng.integers(0, 3))
        assert np.allclose(orc.point_hlle(PL, PL, 2.0, 5.0, d), orc.point_flux(PL, 2.0, 5.0, d), rtol=1e-14,
                           atol=1e-14)
        FL, FR = orc.point_flux(PL, 2.0, 5.0, d), orc.point_flux(PR, 2.0, 5.0, d)
        UL, UR = orc.point_prim2con(PL, 2.0), orc.point_prim2con(PR, 2.0)
        ref = 0.5 * (FL + FR) - 0.5 * (UR - UL)
        assert np.allclose(orc.point_hlle(PL, PR, 2.0, 5.0, d), ref, rtol=1e-13, atol=1e-13)


def test_hlle_speeds_curved_as_printed(orc):
    """lambda_+- = +-sqrt(gamma^dd) - beta^d/alpha (Sec. III), clipped to
    lambda+ >= 0 >= lambda-, in the HLLE combination."""
    rng = np.random.default_rng(47)
    for _ in range(10):
        m, g = random_metric(rng)
        gi = np.linalg.inv(g)
        PL, PR = random_state(rng, g, vmax=0.5), random_state(rng, g, vmax=0.5)
        for d in range(3):
            lp = max(0.0, math.sqrt(gi[d, d]) - m[1 + d] / m[0])
            lm = min(0.0, -math.sqrt(gi[d, d]) - m[1 + d] / m[0])
            FL, FR = orc.point_flux(PL, 2.0, 1.0, d, m), orc.point_flux(PR, 2.0, 1.0, d, m)
            UL, UR = orc.point_prim2con(PL, 2.0, m), orc.point_prim2con(PR, 2.0, m)
            ref = (lp * FL - lm * FR + lp * lm * (UR - UL)) / (lp - lm)
            assert np.allclose(orc.point_hlle(PL, PR, 2.0, 1.0, d, m), ref, rtol=1e-13, atol=1e-13)


def test_ohm_stiff_source_ideal_state_vanishes(orc):
    """eq. Ohm_law: for E = -v x B (ideal MHD) the conduction current is
    zero, so R_E = 0 at any sigma; for v = 0 it is -alpha sigma E."""
    v = np.array([0.2, -0.3, 0.1])
    B = np.array([0.4, 0.1, -0.6])
    E = -np.cross(v, B)
    assert np.abs(orc.point_stiff(v, E, B, 1e6)).max() <= 1e-9
    R = orc.point_stiff(np.zeros(3), E, B, 7.0, conformal(1.0, 0.5))
    assert np.allclose(R, -0.5 * 7.0 * E, rtol=1e-15)


# ---------------------------------------------------------------- tableau
def test_imex_tableau_constants(orc):
    """table imex: gamma = 1 - 1/sqrt(2); c_i = row sums of the implicit
    tableau = (gamma, 1 - gamma); explicit c~ = (0, 1); weights (1/2, 1/2)."""
    g = orc.gamma_imex()
    assert g == pytest.approx(1 - 1 / math.sqrt(2), rel=1e-16)
    A = np.array([[g, 0.0], [1 - 2 * g, g]])
    assert np.allclose(A.sum(1), [g, 1 - g], rtol=1e-15)
    tab = GOLD["imex_ssp2_222"]
    assert np.allclose(np.array(tab["explicit_A"]).sum(1), tab["explicit_c"])
    # L-stability of the implicit part: R(z) -> 0 for z -> infinity
    z = 1e12
    y1 = 1 / (1 + g * z)
    y2 = (1 - (1 - 2 * g) * z * y1) / (1 + g * z)
    assert abs(1 - 0.5 * z * (y1 + y2)) < 1e-10
