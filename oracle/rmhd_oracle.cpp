/*
 * Oracle: resistive GRMHD, one IMEX-SSP2(2,2,2) step on a uniform grid in a
 * fixed 3+1 metric (arXiv:2510.18968, "A resistive MHD module in the
 * GPU-accelerated GRMHD code GRaM-X").
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation
 * written straight from the paper's equations.  It exists so that the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark can check
 * the HIP library against something independent.  The product library never
 * links, loads or calls it, and the two share no source, header, table,
 * constant generator or helper.  Build: g++ -O2 -ffp-contract=off (no fused
 * multiply-add), OpenMP over cells only.
 *
 * What each part follows (sections / equations of the paper):
 *   metric algebra ........ Sec. II.A (3+1 line element, inverse metric)
 *   prim2con .............. Sec. II.C, eqs. conserved_dens/_tau/_S and the
 *                           densitised EM variables of Sec. II.D
 *   stress S_ij ........... eq. conserved_Sij
 *   fluxes and sources .... eq. GRRMHD_flux_form (Sec. II.D)
 *   Ohm's law ............. eq. Ohm_law
 *   HLLE speeds ........... Sec. III (speed-of-light characteristic speeds)
 *   reconstruction ........ Sec. III (TVD minmod / MC2, WENO5 of Shu 1998)
 *   IMEX-SSP2(2,2,2) ...... Sec. III.A, table imex and eq. IMEX3
 *   stiff split ........... Sec. III.A (F_E / R_E split)
 *   implicit E solve ...... eq. 3D_NR (3D Newton-Raphson)
 *   coupled recovery ...... Sec. III.B steps (i)-(v)
 *   conductivity models ... eq. sigma_evol (Sec. IV.A), eq. dynamo_sigma and
 *                           the artificial atmosphere (Sec. IV.E)
 *
 * Where the paper is silent or garbled the readings below are used (each is
 * listed with its reason in the design notes of the repository):
 *   - sqrt(gamma) counted once in the momentum flux and sources (S_ij is
 *     already densitised);
 *   - con2prim momentum numerator S_i - eta_ijk E^j B^k (densitised fields);
 *   - sound speed c_s^2 = Gamma (Gamma-1) eps / (1 + Gamma eps);
 *   - the current in the charge flux at a face is the mean of the two
 *     adjacent cell-centre currents (Ohm's law evaluated on reconstructed
 *     face states multiplies sigma by the reconstruction error and is
 *     unstable for sigma >= 1e5 at CFL 0.5);
 *   - metric at faces by 4th-order interpolation (-1,9,9,-1)/16, metric
 *     derivatives at centres by 4th-order central differences;
 *   - stiff terms of the final update recovered from the stage equations;
 *   - recovery stops when |dp| <= tol p and max|dv^i| <= tol;
 *   - a face state with rho<=0, p<=0 or v^2>=1 falls back to first order;
 *   - derivatives through a limiter or a fallback are those of the branch
 *     taken (at a tie or a zero slope the returned branch, not an average);
 *   - a conductivity model sigma(D) takes the conserved D of the state it
 *     acts on: in an implicit solve the D of the stage's explicit state (the
 *     solve does not change D); in the charge flux of F(U(s)) the D of the
 *     stage primitives at each cell centre (sqrt(gamma) rho W); a ghost cell
 *     holds a copy of its interior image and carries the image's sigma, as
 *     the given sigma field does;
 *   - the artificial atmosphere acts at the end of each step: a cell whose
 *     assembled D is below 1.01 sqrt(gamma) rho_atmo gets the hydro part
 *     (D, S_i, tau) of the atmosphere state (rho_atmo, p = K_atmo
 *     rho_atmo^Gamma, v = 0) with its own E and B, is recovered from it and
 *     flagged with status 2 (never silently).
 *
 * Parity status: every function here is pinned by tests in tests/ against
 * closed forms, library routines, invariants or brute force, except the
 * whole-grid shock profiles (the paper's figures carry no numbers), which
 * are "parity unpinned" beyond GPU == oracle.
 */
#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdlib>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

/* ------------------------------------------------------------------------ */
/* Scalar type.  double for the plain oracle; Dual (value + one tangent)    */
/* for exact directional derivatives used to check the adjoint.             */
/* ------------------------------------------------------------------------ */
inline double val(double x) { return x; }

struct Dual {
    double v, d;
    Dual() : v(0), d(0) {}
    Dual(double x) : v(x), d(0) {}
    Dual(double x, double dx) : v(x), d(dx) {}
};
inline double val(const Dual& x) { return x.v; }
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
    double q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
inline Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
inline Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
inline Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual operator/(double a, Dual b) { return Dual(a) / b; }
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
inline Dual sqrt(Dual a) {
    double s = std::sqrt(a.v);
    return Dual(s, a.d / (2.0 * s));
}
inline Dual fabs(Dual a) { return a.v < 0 ? -a : a; }
/* x^e for a constant exponent e: d(x^e) = e x^(e-1) dx */
inline double pw(double x, double e) { return std::pow(x, e); }
inline Dual pw(Dual x, double e) {
    return Dual(std::pow(x.v, e), e == 0.0 ? 0.0 : e * std::pow(x.v, e - 1.0) * x.d);
}

using std::sqrt;
using std::fabs;

template <class T> inline T sq(T x) { return x * x; }
template <class T> inline T tmax(T a, T b) { return val(a) >= val(b) ? a : b; }
template <class T> inline T tmin(T a, T b) { return val(a) <= val(b) ? a : b; }
template <class T> inline double sgn(T x) { return val(x) > 0 ? 1.0 : (val(x) < 0 ? -1.0 : 0.0); }

/* Levi-Civita symbol eta_{ijk}, eta_{012} = +1. */
inline double eta(int i, int j, int k) { return 0.5 * (i - j) * (j - k) * (k - i); }

/* ------------------------------------------------------------------------ */
/* Field layout                                                             */
/* ------------------------------------------------------------------------ */
/* primitives: rho, p, v^x..v^z, B^x..B^z, E^x..E^z, phi, psi, q            */
enum { P_RHO = 0, P_PRS = 1, P_V = 2, P_B = 5, P_E = 8, P_PHI = 11, P_PSI = 12, P_Q = 13 };
/* conserved: D, S_x..S_z, tau, B^x..B^z, E^x..E^z (densitised), Phi, Psi, Q */
enum { U_D = 0, U_S = 1, U_TAU = 4, U_B = 5, U_E = 8, U_PHI = 11, U_PSI = 12, U_Q = 13 };
enum { NF = 14 };
/* metric: alpha, beta^x..z, gamma_xx,xy,xz,yy,yz,zz, K_xx,xy,xz,yy,yz,zz     */
enum { M_ALP = 0, M_BET = 1, M_G = 4, M_K = 10, NM = 16 };
static const int SYM[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

template <class T> struct Metric {
    T alp, beta[3], g[3][3], gi[3][3], sqrtg, K[3][3];
};

/* 3-metric, its inverse (cofactors / determinant) and sqrt(det), Sec. II.A. */
template <class T> void metric_point(const T* f, Metric<T>& m) {
    m.alp = f[M_ALP];
    for (int i = 0; i < 3; ++i) m.beta[i] = f[M_BET + i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            m.g[i][j] = f[M_G + SYM[i][j]];
            m.K[i][j] = f[M_K + SYM[i][j]];
        }
    const T(&g)[3][3] = m.g;
    T c[3][3];
    c[0][0] = g[1][1] * g[2][2] - g[1][2] * g[2][1];
    c[0][1] = g[1][2] * g[2][0] - g[1][0] * g[2][2];
    c[0][2] = g[1][0] * g[2][1] - g[1][1] * g[2][0];
    c[1][0] = g[0][2] * g[2][1] - g[0][1] * g[2][2];
    c[1][1] = g[0][0] * g[2][2] - g[0][2] * g[2][0];
    c[1][2] = g[0][1] * g[2][0] - g[0][0] * g[2][1];
    c[2][0] = g[0][1] * g[1][2] - g[0][2] * g[1][1];
    c[2][1] = g[0][2] * g[1][0] - g[0][0] * g[1][2];
    c[2][2] = g[0][0] * g[1][1] - g[0][1] * g[1][0];
    T det = g[0][0] * c[0][0] + g[0][1] * c[0][1] + g[0][2] * c[0][2];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) m.gi[i][j] = c[j][i] / det;
    m.sqrtg = sqrt(det);
}

template <class T> void flat_fields(T* f) {
    for (int a = 0; a < NM; ++a) f[a] = T(0.0);
    f[M_ALP] = T(1.0);
    f[M_G + 0] = T(1.0);
    f[M_G + 3] = T(1.0);
    f[M_G + 5] = T(1.0);
}

template <class T> void lower(const Metric<T>& m, const T* up, T* lo) {
    for (int i = 0; i < 3; ++i) lo[i] = m.g[i][0] * up[0] + m.g[i][1] * up[1] + m.g[i][2] * up[2];
}
template <class T> void raise(const Metric<T>& m, const T* lo, T* up) {
    for (int i = 0; i < 3; ++i) up[i] = m.gi[i][0] * lo[0] + m.gi[i][1] * lo[1] + m.gi[i][2] * lo[2];
}
template <class T> T dot3(const T* a, const T* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* ------------------------------------------------------------------------ */
/* prim2con: eqs. conserved_dens, conserved_tau, conserved_S and the        */
/* densitised EM / cleaning / charge variables of Sec. II.D.                */
/* ------------------------------------------------------------------------ */
template <class T> void prim2con(const Metric<T>& m, double G, const T* P, T* U) {
    T rho = P[P_RHO], p = P[P_PRS];
    T v[3], E[3], B[3], vl[3], El[3], Bl[3];
    for (int i = 0; i < 3; ++i) { v[i] = P[P_V + i]; E[i] = P[P_E + i]; B[i] = P[P_B + i]; }
    lower(m, v, vl); lower(m, E, El); lower(m, B, Bl);
    T v2 = dot3(vl, v);
    T W = 1.0 / sqrt(1.0 - v2);
    T E2 = dot3(El, E), B2 = dot3(Bl, B);
    T eps = p / ((G - 1.0) * rho);
    T h = rho * (1.0 + eps) + p;               /* enthalpy density, Sec. II.C */
    U[U_D] = m.sqrtg * rho * W;
    for (int i = 0; i < 3; ++i) {
        /* epsilon_ijk E^j B^k with epsilon_ijk = sqrt(gamma) eta_ijk */
        T exb = T(0.0);
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                if (eta(i, j, k) != 0.0) exb = exb + eta(i, j, k) * m.sqrtg * E[j] * B[k];
        U[U_S + i] = m.sqrtg * (h * W * W * vl[i] + exb);
    }
    U[U_TAU] = m.sqrtg * (h * W * W - p + 0.5 * (E2 + B2)) - U[U_D];
    for (int i = 0; i < 3; ++i) {
        U[U_B + i] = m.sqrtg * B[i];
        U[U_E + i] = m.sqrtg * E[i];
    }
    U[U_PHI] = m.sqrtg * P[P_PHI];
    U[U_PSI] = m.sqrtg * P[P_PSI];
    U[U_Q] = m.sqrtg * P[P_Q];
}

/* epsilon^{ijk} v_j Bcal_k with epsilon^{ijk} = eta^{ijk}/sqrt(gamma).      */
template <class T> void eps_up_cross(const Metric<T>& m, const T* vl, const T* Bcl, T* out) {
    for (int i = 0; i < 3; ++i) {
        T s = T(0.0);
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                if (eta(i, j, k) != 0.0) s = s + eta(i, j, k) * vl[j] * Bcl[k];
        out[i] = s / m.sqrtg;
    }
}

/* Ohm's law, eq. Ohm_law (densitised current). */
template <class T>
void ohm_current(const Metric<T>& m, const T* v, const T* Ec, const T* Bc, T Q, T sigma, T* J) {
    T vl[3], Bcl[3], vxb[3];
    lower(m, v, vl);
    lower(m, Bc, Bcl);
    T W = 1.0 / sqrt(1.0 - dot3(vl, v));
    eps_up_cross(m, vl, Bcl, vxb);
    T vE = dot3(vl, Ec);
    for (int i = 0; i < 3; ++i) J[i] = Q * v[i] + W * sigma * (Ec[i] + vxb[i] - vE * v[i]);
}

/* Stiff part of the E source, R_E (Sec. III.A). */
template <class T>
void stiff_source(const Metric<T>& m, const T* v, const T* Ec, const T* Bc, T sigma, T* R) {
    T vl[3], Bcl[3], vxb[3];
    lower(m, v, vl);
    lower(m, Bc, Bcl);
    T W = 1.0 / sqrt(1.0 - dot3(vl, v));
    eps_up_cross(m, vl, Bcl, vxb);
    T vE = dot3(vl, Ec);
    for (int i = 0; i < 3; ++i) R[i] = -m.alp * W * sigma * (Ec[i] + vxb[i] - vE * v[i]);
}

/* ------------------------------------------------------------------------ */
/* Physical flux F^d of eq. GRRMHD_flux_form (sqrt(gamma) counted once).    */
/* ------------------------------------------------------------------------ */
/* Jd: the current J^d carried by the charge flux.  At cell faces it is the
 * mean of the two adjacent cell-centre currents (Ohm's law on each cell's
 * own state), see face_flux; pass nullptr to evaluate Ohm's law on P. */
template <class T>
void phys_flux(const Metric<T>& m, double G, const T* P, const T* U, T sigma, int d, T* F, const T* Jd = nullptr) {
    T rho = P[P_RHO], p = P[P_PRS];
    T v[3], E[3], B[3], vl[3], El[3], Bl[3];
    for (int i = 0; i < 3; ++i) { v[i] = P[P_V + i]; E[i] = P[P_E + i]; B[i] = P[P_B + i]; }
    lower(m, v, vl); lower(m, E, El); lower(m, B, Bl);
    T W = 1.0 / sqrt(1.0 - dot3(vl, v));
    T E2 = dot3(El, E), B2 = dot3(Bl, B);
    T eps = p / ((G - 1.0) * rho);
    T h = rho * (1.0 + eps) + p;
    /* densitised spatial stress S_ij, eq. conserved_Sij */
    T Sij[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            Sij[i][j] = m.sqrtg * (h * W * W * vl[i] * vl[j] + m.g[i][j] * p - El[i] * El[j] - Bl[i] * Bl[j] +
                                   0.5 * m.g[i][j] * (E2 + B2));
    T alp = m.alp, bd = m.beta[d];
    F[U_D] = (alp * v[d] - bd) * U[U_D];
    for (int i = 0; i < 3; ++i) {
        T Sdi = m.gi[d][0] * Sij[0][i] + m.gi[d][1] * Sij[1][i] + m.gi[d][2] * Sij[2][i];
        F[U_S + i] = alp * Sdi - bd * U[U_S + i];
    }
    T Sl[3] = {U[U_S], U[U_S + 1], U[U_S + 2]}, Su[3];
    raise(m, Sl, Su);
    F[U_TAU] = alp * (Su[d] - v[d] * U[U_D]) - bd * U[U_TAU];
    T Ec[3] = {U[U_E], U[U_E + 1], U[U_E + 2]}, Bc[3] = {U[U_B], U[U_B + 1], U[U_B + 2]};
    T Ecl[3], Bcl[3];
    lower(m, Ec, Ecl);
    lower(m, Bc, Bcl);
    for (int i = 0; i < 3; ++i) {
        T curlE = T(0.0), curlB = T(0.0);
        for (int j = 0; j < 3; ++j) {
            double e = eta(i, d, j);
            if (e != 0.0) {
                curlE = curlE + e * Ecl[j] / m.sqrtg;   /* epsilon^{idj} Ecal_j */
                curlB = curlB + e * Bcl[j] / m.sqrtg;   /* epsilon^{idj} Bcal_j */
            }
        }
        F[U_B + i] = alp * (curlE + m.gi[i][d] * U[U_PHI]) - bd * Bc[i];
        F[U_E + i] = -(alp * (curlB - m.gi[i][d] * U[U_PSI]) + bd * Ec[i]);
    }
    F[U_PHI] = alp * Bc[d] - bd * U[U_PHI];
    F[U_PSI] = alp * Ec[d] - bd * U[U_PSI];
    T J[3];
    if (Jd) {
        J[d] = *Jd;
    } else {
        ohm_current(m, v, Ec, Bc, U[U_Q], sigma, J);
    }
    F[U_Q] = alp * J[d] - bd * U[U_Q];
}

/* current at a cell centre from the cell's primitives (densitised) */
template <class T> void cell_current(const Metric<T>& m, double G, const T* P, T sigma, T* J) {
    T U[NF];
    prim2con(m, G, P, U);
    T v[3] = {P[P_V], P[P_V + 1], P[P_V + 2]};
    T Ec[3] = {U[U_E], U[U_E + 1], U[U_E + 2]}, Bc[3] = {U[U_B], U[U_B + 1], U[U_B + 2]};
    ohm_current(m, v, Ec, Bc, U[U_Q], sigma, J);
}

/* Explicit sources of eq. GRRMHD_flux_form at a cell centre; the E rows
 * carry only the non-stiff part F_E (Sec. III.A).  dalp[i] = d_i alpha,
 * dbet[i][j] = d_i beta^j, dg[i][j][k] = d_i gamma_jk. */
template <class T>
void explicit_source(const Metric<T>& m, const T* dalp, T dbet[3][3], T dg[3][3][3], double kappa, double G,
                     const T* P, const T* U, T* S) {
    (void)G;
    /* Christoffel symbols Gamma^i_jk and their contraction Gamma^i = gamma^jk Gamma^i_jk */
    T Chr[3][3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) {
                T s = T(0.0);
                for (int l = 0; l < 3; ++l) s = s + m.gi[i][l] * (dg[j][l][k] + dg[k][l][j] - dg[l][j][k]);
                Chr[i][j][k] = 0.5 * s;
            }
    T Gam[3];
    for (int i = 0; i < 3; ++i) {
        T s = T(0.0);
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) s = s + m.gi[j][k] * Chr[i][j][k];
        Gam[i] = s;
    }
    T Ktr = T(0.0);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Ktr = Ktr + m.gi[i][j] * m.K[i][j];
    /* densitised stress with both indices up */
    T rho = P[P_RHO], p = P[P_PRS];
    T v[3], E[3], B[3], vl[3], El[3], Bl[3];
    for (int i = 0; i < 3; ++i) { v[i] = P[P_V + i]; E[i] = P[P_E + i]; B[i] = P[P_B + i]; }
    lower(m, v, vl); lower(m, E, El); lower(m, B, Bl);
    T W = 1.0 / sqrt(1.0 - dot3(vl, v));
    T E2 = dot3(El, E), B2 = dot3(Bl, B);
    T eps = p / ((G - 1.0) * rho);
    T h = rho * (1.0 + eps) + p;
    T Sij[3][3], Sup[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            Sij[i][j] = m.sqrtg * (h * W * W * vl[i] * vl[j] + m.g[i][j] * p - El[i] * El[j] - Bl[i] * Bl[j] +
                                   0.5 * m.g[i][j] * (E2 + B2));
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
            T s = T(0.0);
            for (int l = 0; l < 3; ++l)
                for (int n = 0; n < 3; ++n) s = s + m.gi[j][l] * m.gi[k][n] * Sij[l][n];
            Sup[j][k] = s;
        }
    T alp = m.alp;
    T Sl[3] = {U[U_S], U[U_S + 1], U[U_S + 2]}, Su[3];
    raise(m, Sl, Su);
    T Bc[3] = {U[U_B], U[U_B + 1], U[U_B + 2]}, Ec[3] = {U[U_E], U[U_E + 1], U[U_E + 2]};
    S[U_D] = T(0.0);
    for (int i = 0; i < 3; ++i) {
        T a = T(0.0), b = T(0.0);
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) a = a + Sup[j][k] * dg[i][j][k];
        for (int j = 0; j < 3; ++j) b = b + Sl[j] * dbet[i][j];
        S[U_S + i] = 0.5 * alp * a + b - (U[U_TAU] + U[U_D]) * dalp[i];
    }
    {
        T a = T(0.0), b = T(0.0);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) a = a + Sup[i][j] * m.K[i][j];
        for (int j = 0; j < 3; ++j) b = b + Su[j] * dalp[j];
        S[U_TAU] = alp * a - b;
    }
    for (int i = 0; i < 3; ++i) {
        T gda = m.gi[i][0] * dalp[0] + m.gi[i][1] * dalp[1] + m.gi[i][2] * dalp[2];
        T bb = T(0.0), eb = T(0.0);
        for (int k = 0; k < 3; ++k) {
            bb = bb + Bc[k] * dbet[k][i];
            eb = eb + Ec[k] * dbet[k][i];
        }
        S[U_B + i] = -bb + U[U_PHI] * (gda - alp * Gam[i]);
        S[U_E + i] = -eb + U[U_PSI] * (gda - alp * Gam[i]) - alp * U[U_Q] * v[i];
    }
    T Bda = Bc[0] * dalp[0] + Bc[1] * dalp[1] + Bc[2] * dalp[2];
    T Eda = Ec[0] * dalp[0] + Ec[1] * dalp[1] + Ec[2] * dalp[2];
    S[U_PHI] = -alp * U[U_PHI] * Ktr + Bda - alp * kappa * U[U_PHI];
    S[U_PSI] = -alp * U[U_PSI] * Ktr + Eda + alp * U[U_Q] - alp * kappa * U[U_PSI];
    S[U_Q] = T(0.0);
}

/* ------------------------------------------------------------------------ */
/* HLLE with speed-of-light characteristic speeds (Sec. III).               */
/* ------------------------------------------------------------------------ */
template <class T> void char_speeds(const Metric<T>& m, int d, int mode, T& lp, T& lm) {
    T s = sqrt(m.gi[d][d]);
    if (mode == 0) {                     /* as printed: +-sqrt(gamma^dd) - beta^d/alpha */
        lp = s - m.beta[d] / m.alp;
        lm = -s - m.beta[d] / m.alp;
    } else {                             /* coordinate speeds of the alpha-carrying flux */
        lp = m.alp * s - m.beta[d];
        lm = -m.alp * s - m.beta[d];
    }
}

template <class T>
void hlle(const T* UL, const T* UR, const T* FL, const T* FR, T lp, T lm, T* Fh) {
    T lpp = tmax(T(0.0), lp), lmm = tmin(T(0.0), lm);
    for (int a = 0; a < NF; ++a)
        Fh[a] = (lpp * FL[a] - lmm * FR[a] + lpp * lmm * (UR[a] - UL[a])) / (lpp - lmm);
}

/* ------------------------------------------------------------------------ */
/* Reconstruction of one field from the 5-cell stencil f[0..4] = f_{i-2..i+2}*/
/* to the faces i-1/2 (fm) and i+1/2 (fp).                                   */
/* ------------------------------------------------------------------------ */
/* minmod: zero unless both slopes share a strict sign, else the one of
 * smaller magnitude (b on a tie).  Written as a branch so that a derivative
 * taken through it is that of the returned branch, also at a zero slope. */
template <class T> T minmod2(T a, T b) {
    if (!(sgn(a) * sgn(b) > 0)) return T(0.0);
    return std::fabs(val(a)) < std::fabs(val(b)) ? a : b;
}
template <class T> T minmod3(T a, T b, T c) {
    if (val(a) > 0 && val(b) > 0 && val(c) > 0) return tmin(a, tmin(b, c));
    if (val(a) < 0 && val(b) < 0 && val(c) < 0) return tmax(a, tmax(b, c));
    return T(0.0);
}
/* WENO5-JS value at the right face of the middle cell of s[0..4] */
template <class T> T weno5_right(const T* s) {
    const double epsw = 1e-6;
    T q0 = (2.0 * s[0] - 7.0 * s[1] + 11.0 * s[2]) / 6.0;
    T q1 = (-s[1] + 5.0 * s[2] + 2.0 * s[3]) / 6.0;
    T q2 = (2.0 * s[2] + 5.0 * s[3] - s[4]) / 6.0;
    T b0 = (13.0 / 12.0) * sq(s[0] - 2.0 * s[1] + s[2]) + 0.25 * sq(s[0] - 4.0 * s[1] + 3.0 * s[2]);
    T b1 = (13.0 / 12.0) * sq(s[1] - 2.0 * s[2] + s[3]) + 0.25 * sq(s[1] - s[3]);
    T b2 = (13.0 / 12.0) * sq(s[2] - 2.0 * s[3] + s[4]) + 0.25 * sq(3.0 * s[2] - 4.0 * s[3] + s[4]);
    T a0 = 0.1 / sq(epsw + b0);
    T a1 = 0.6 / sq(epsw + b1);
    T a2 = 0.3 / sq(epsw + b2);
    T as = a0 + a1 + a2;
    return (a0 / as) * q0 + (a1 / as) * q1 + (a2 / as) * q2;
}
enum { REC_MINMOD = 0, REC_MC2 = 1, REC_WENO5 = 2 };
template <class T> void recon_cell(int method, const T* f, T& fm, T& fp) {
    if (method == REC_WENO5) {
        T r[5] = {f[4], f[3], f[2], f[1], f[0]};   /* mirror image for the left face */
        fp = weno5_right(f);
        fm = weno5_right(r);
        return;
    }
    T dm = f[2] - f[1], dp = f[3] - f[2];
    T slope = (method == REC_MINMOD) ? minmod2(dm, dp) : minmod3(2.0 * dm, 2.0 * dp, 0.5 * (dm + dp));
    fm = f[2] - 0.5 * slope;
    fp = f[2] + 0.5 * slope;
}

/* ------------------------------------------------------------------------ */
/* Implicit E solve, eq. 3D_NR: Newton-Raphson on                            */
/*   f(E) = E - E* + c [E + eps^{ijk} v_j Bcal_k - (v_k E^k) v^i],           */
/* c = a_ii dt alpha W sigma, at fixed v.  f is linear in E, so the first    */
/* Newton step is exact up to rounding; the loop stops on round-off.         */
/* ------------------------------------------------------------------------ */
template <class T> void solve3(T A[3][3], T* b) {   /* Gaussian elimination, partial pivoting */
    int perm[3] = {0, 1, 2};
    for (int c = 0; c < 3; ++c) {
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (std::fabs(val(A[r][c])) > std::fabs(val(A[piv][c]))) piv = r;
        if (piv != c) {
            for (int k = 0; k < 3; ++k) std::swap(A[c][k], A[piv][k]);
            std::swap(b[c], b[piv]);
            std::swap(perm[c], perm[piv]);
        }
        for (int r = c + 1; r < 3; ++r) {
            T f = A[r][c] / A[c][c];
            for (int k = c; k < 3; ++k) A[r][k] = A[r][k] - f * A[c][k];
            b[r] = b[r] - f * b[c];
        }
    }
    for (int r = 2; r >= 0; --r) {
        T s = b[r];
        for (int k = r + 1; k < 3; ++k) s = s - A[r][k] * b[k];
        b[r] = s / A[r][r];
    }
}

template <class T>
void esolve_nr(const Metric<T>& m, const T* v, const T* Bc, const T* Estar, T c, T* E) {
    T vl[3], Bcl[3], vxb[3];
    lower(m, v, vl);
    lower(m, Bc, Bcl);
    eps_up_cross(m, vl, Bcl, vxb);
    for (int it = 0; it < 5; ++it) {
        T vE = dot3(vl, E);
        T f[3], J[3][3];
        for (int i = 0; i < 3; ++i) f[i] = E[i] - Estar[i] + c * (E[i] + vxb[i] - vE * v[i]);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) J[i][j] = (i == j ? 1.0 + c : T(0.0)) - c * v[i] * vl[j];
        solve3(J, f);
        double dmax = 0, emax = 0;
        for (int i = 0; i < 3; ++i) {
            E[i] = E[i] - f[i];
            dmax = std::max(dmax, std::fabs(val(f[i])));
            emax = std::max(emax, std::fabs(val(E[i])));
        }
        if (dmax <= 4e-16 * emax) break;
    }
}

/* ------------------------------------------------------------------------ */
/* Coupled implicit-E + 1D primitive recovery, Sec. III.B steps (i)-(v).     */
/* adt = a_ii * dt (0 gives the plain recovery with E fixed at Estar).       */
/* Returns status: 0 converged, 1 converged at the iteration cap within     */
/* 1e-12 (warning), -3 no convergence, -4 unphysical state.                 */
/* ------------------------------------------------------------------------ */
enum { ST_OK = 0, ST_WARN = 1, ST_NOCONV = -3, ST_UNPHYS = -4 };

template <class T>
int recover_paper(const Metric<T>& m, double G, const T* U, const T* Estar, T adt, T sigma, const T* Pg, double tol,
                  int maxit, T* P, T* Eout, int* iters) {
    const T D = U[U_D], tau = U[U_TAU];
    T Sl[3] = {U[U_S], U[U_S + 1], U[U_S + 2]};
    T Bc[3] = {U[U_B], U[U_B + 1], U[U_B + 2]};
    T Bcl[3];
    lower(m, Bc, Bcl);
    T B2c = dot3(Bcl, Bc);
    const T sg = m.sqrtg;
    /* (i) guess p and v from the previous state */
    T p = Pg[P_PRS];
    T v[3] = {Pg[P_V], Pg[P_V + 1], Pg[P_V + 2]};
    T E[3] = {Estar[0], Estar[1], Estar[2]};
    bool stiff = val(adt) != 0.0 && val(sigma) != 0.0;
    int status = ST_NOCONV;
    double last_dp_rel = 1e300;
    int it = 0;
    auto fail = [&](int st) {
        for (int a = 0; a < NF; ++a) P[a] = Pg[a];
        for (int i = 0; i < 3; ++i) Eout[i] = Estar[i];
        *iters = it;
        return st;
    };
    if (!(val(D) > 0) || !std::isfinite(val(tau)) || !(val(p) > 0)) return fail(ST_UNPHYS);
    for (it = 1; it <= maxit; ++it) {
        T vl[3];
        lower(m, v, vl);
        T v2 = dot3(vl, v);
        if (!(val(v2) < 1.0)) return fail(ST_UNPHYS);
        /* (ii) implicit E at the current velocity */
        if (stiff) {
            T W = 1.0 / sqrt(1.0 - v2);
            T c = adt * m.alp * W * sigma;
            esolve_nr(m, v, Bc, Estar, c, E);
        }
        /* (iii) velocity, Lorentz factor, density, specific internal energy */
        T El[3];
        lower(m, E, El);
        T E2c = dot3(El, E);
        T den = tau + D + sg * p - (E2c + B2c) / (2.0 * sg);
        T vnl[3], vn[3];
        for (int i = 0; i < 3; ++i) {
            T exb = T(0.0);
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k)
                    if (eta(i, j, k) != 0.0) exb = exb + eta(i, j, k) * E[j] * Bc[k];
            vnl[i] = (Sl[i] - exb) / den;
        }
        raise(m, vnl, vn);
        T vn2 = dot3(vnl, vn);
        if (!(val(vn2) < 1.0) || !std::isfinite(val(vn2))) return fail(ST_UNPHYS);
        T Wn = 1.0 / sqrt(1.0 - vn2);
        T rho = D / (sg * Wn);
        T eps = (tau - D * (Wn - 1.0) - sg * p * (Wn * Wn - 1.0) - (E2c + B2c) / (2.0 * sg)) / (D * Wn);
        /* (iv) Newton-Raphson step on the pressure */
        T f = (G - 1.0) * rho * eps - p;
        T cs2 = G * (G - 1.0) * eps / (1.0 + G * eps);
        T fp = vn2 * cs2 - 1.0;
        T pn = p - f / fp;
        if (!(val(pn) > 0) || !std::isfinite(val(pn))) return fail(ST_UNPHYS);
        double dv = 0;
        for (int i = 0; i < 3; ++i) dv = std::max(dv, std::fabs(val(vn[i]) - val(v[i])));
        double dp = std::fabs(val(pn) - val(p));
        p = pn;
        for (int i = 0; i < 3; ++i) v[i] = vn[i];
        last_dp_rel = dp / val(p);
        /* (v) repeat until the change falls below the tolerance */
        if (dp <= tol * val(p) && dv <= tol) {
            status = ST_OK;
            break;
        }
    }
    if (status != ST_OK) {
        it = maxit;
        if (last_dp_rel <= 1e-12) status = ST_WARN;
        else return fail(ST_NOCONV);
    }
    T vl[3];
    lower(m, v, vl);
    T W = 1.0 / sqrt(1.0 - dot3(vl, v));
    P[P_RHO] = D / (sg * W);
    P[P_PRS] = p;
    for (int i = 0; i < 3; ++i) {
        P[P_V + i] = v[i];
        P[P_B + i] = Bc[i] / sg;
        P[P_E + i] = E[i] / sg;
        Eout[i] = E[i];
    }
    P[P_PHI] = U[U_PHI] / sg;
    P[P_PSI] = U[U_PSI] / sg;
    P[P_Q] = U[U_Q] / sg;
    *iters = it;
    return status;
}

/* ------------------------------------------------------------------------ */
/* Stiff coupled solve as the root of the recovery map.                     */
/*                                                                          */
/* One pass of steps (ii)-(iv) maps (p, v^i) to (p', v'^i).  The recovered  */
/* stage state is the fixed point: E solves the implicit stage equation at  */
/* v, v is the momentum/energy velocity at (E, p) and p is the EOS pressure.*/
/* The plain repetition of the pass diverges in the stiff limit once        */
/* B^2 > h W^2 (its velocity Jacobian tends to -B^2/(h W^2)), so the root   */
/* is found by Newton's method on r(p, v) = (p_EOS - p, v' - v) with the    */
/* exact Jacobian (dual numbers) and a backtracking line search.  The root  */
/* is the same one the paper's iteration reaches where that converges.      */
/* ------------------------------------------------------------------------ */
template <class S> struct RecIn {
    Metric<S> m;
    double G;
    S D, tau, Sl[3], Bc[3], Estar[3], adt, sigma;
};

template <class T, class S> void rec_in_cast(const RecIn<T>& a, RecIn<S>& b) {
    b.G = a.G;
    b.m.alp = S(val(a.m.alp));
    b.m.sqrtg = S(val(a.m.sqrtg));
    for (int i = 0; i < 3; ++i) {
        b.m.beta[i] = S(val(a.m.beta[i]));
        for (int j = 0; j < 3; ++j) {
            b.m.g[i][j] = S(val(a.m.g[i][j]));
            b.m.gi[i][j] = S(val(a.m.gi[i][j]));
            b.m.K[i][j] = S(val(a.m.K[i][j]));
        }
        b.Sl[i] = S(val(a.Sl[i]));
        b.Bc[i] = S(val(a.Bc[i]));
        b.Estar[i] = S(val(a.Estar[i]));
    }
    b.D = S(val(a.D));
    b.tau = S(val(a.tau));
    b.adt = S(val(a.adt));
    b.sigma = S(val(a.sigma));
}

/* r[0] = (Gamma-1) rho eps - p, r[1..3] = v'^i - v^i; false if unphysical */
template <class S> bool rec_residual(const RecIn<S>& in, const S* x, S* r, S* Eout) {
    const Metric<S>& m = in.m;
    S p = x[0];
    S v[3] = {x[1], x[2], x[3]}, vl[3];
    lower(m, v, vl);
    S v2 = dot3(vl, v);
    if (!(val(v2) < 1.0) || !(val(p) > 0)) return false;
    S W = 1.0 / sqrt(1.0 - v2);
    S c = in.adt * m.alp * W * in.sigma;
    S E[3] = {in.Estar[0], in.Estar[1], in.Estar[2]};
    esolve_nr(m, v, in.Bc, in.Estar, c, E);                        /* step (ii) */
    S Bcl[3], El[3];
    lower(m, in.Bc, Bcl);
    lower(m, E, El);
    S E2c = dot3(El, E), B2c = dot3(Bcl, in.Bc);
    S den = in.tau + in.D + m.sqrtg * p - (E2c + B2c) / (2.0 * m.sqrtg);
    S vnl[3], vn[3];
    for (int i = 0; i < 3; ++i) {                                  /* step (iii) */
        S exb = S(0.0);
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                if (eta(i, j, k) != 0.0) exb = exb + eta(i, j, k) * E[j] * in.Bc[k];
        vnl[i] = (in.Sl[i] - exb) / den;
    }
    raise(m, vnl, vn);
    S vn2 = dot3(vnl, vn);
    if (!(val(vn2) < 1.0) || !std::isfinite(val(vn2))) return false;
    S Wn = 1.0 / sqrt(1.0 - vn2);
    S rho = in.D / (m.sqrtg * Wn);
    S eps = (in.tau - in.D * (Wn - 1.0) - m.sqrtg * p * (Wn * Wn - 1.0) - (E2c + B2c) / (2.0 * m.sqrtg)) /
            (in.D * Wn);
    r[0] = (in.G - 1.0) * rho * eps - p;                              /* step (iv) */
    for (int i = 0; i < 3; ++i) r[1 + i] = vn[i] - v[i];
    if (Eout)
        for (int i = 0; i < 3; ++i) Eout[i] = E[i];
    for (int a = 0; a < 4; ++a)
        if (!std::isfinite(val(r[a]))) return false;
    return true;
}

/* solve the 4x4 system A y = b (A double, b of any scalar type), in place */
template <class T> bool solve4(double A[4][4], T* b) {
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
            if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
        if (A[piv][c] == 0.0) return false;
        if (piv != c) {
            for (int k = 0; k < 4; ++k) std::swap(A[c][k], A[piv][k]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < 4; ++r) {
            double f = A[r][c] / A[c][c];
            for (int k = c; k < 4; ++k) A[r][k] -= f * A[c][k];
            b[r] = b[r] - f * b[c];
        }
    }
    for (int r = 3; r >= 0; --r) {
        T s = b[r];
        for (int k = r + 1; k < 4; ++k) s = s - A[r][k] * b[k];
        b[r] = s / A[r][r];
    }
    return true;
}

template <class T> double rec_merit(const T* r, double p) {
    double a = val(r[0]) / p, s = a * a;
    for (int i = 1; i < 4; ++i) s += val(r[i]) * val(r[i]);
    return s;
}

template <class T>
int recover_newton(const Metric<T>& m, double G, const T* U, const T* Estar, T adt, T sigma, const T* Pg, double tol,
                   int maxit, T* P, T* Eout, int* iters) {
    RecIn<T> in;
    in.m = m;
    in.G = G;
    in.D = U[U_D];
    in.tau = U[U_TAU];
    for (int i = 0; i < 3; ++i) {
        in.Sl[i] = U[U_S + i];
        in.Bc[i] = U[U_B + i];
        in.Estar[i] = Estar[i];
    }
    in.adt = adt;
    in.sigma = sigma;
    RecIn<Dual> ind;
    rec_in_cast(in, ind);
    T x[4] = {Pg[P_PRS], Pg[P_V], Pg[P_V + 1], Pg[P_V + 2]};
    T r[4];
    int it = 0;
    auto fail = [&](int st) {
        for (int a = 0; a < NF; ++a) P[a] = Pg[a];
        for (int i = 0; i < 3; ++i) Eout[i] = Estar[i];
        *iters = it;
        return st;
    };
    if (!(val(in.D) > 0) || !std::isfinite(val(in.tau)) || !(val(x[0]) > 0)) return fail(ST_UNPHYS);
    if (!rec_residual(in, x, r, (T*)nullptr)) {
        /* guess outside the physical domain: restart from rest with a larger pressure */
        bool ok = false;
        x[1] = x[2] = x[3] = T(0.0);
        for (int k = 0; k < 64 && !ok; ++k) {
            ok = rec_residual(in, x, r, (T*)nullptr);
            if (!ok) x[0] = 2.0 * x[0];
        }
        if (!ok) return fail(ST_UNPHYS);
    }
    int status = ST_NOCONV;
    double last_rel = 1e300;
    for (it = 1; it <= maxit; ++it) {
        /* exact Jacobian at the current iterate, one dual direction per unknown */
        double J[4][4];
        for (int j = 0; j < 4; ++j) {
            Dual xd[4], rd[4];
            for (int a = 0; a < 4; ++a) xd[a] = Dual(val(x[a]), a == j ? 1.0 : 0.0);
            if (!rec_residual(ind, xd, rd, (Dual*)nullptr)) return fail(ST_UNPHYS);
            for (int a = 0; a < 4; ++a) J[a][j] = rd[a].d;
        }
        T dx[4] = {-r[0], -r[1], -r[2], -r[3]};
        if (!solve4(J, dx)) return fail(ST_NOCONV);
        /* backtracking: keep the state physical and the residual decreasing */
        double m0 = rec_merit(r, val(x[0]));
        double t = 1.0;
        T xt[4], rt[4];
        bool accepted = false;
        for (int ls = 0; ls < 40; ++ls) {
            for (int a = 0; a < 4; ++a) xt[a] = x[a] + t * dx[a];
            if (rec_residual(in, xt, rt, (T*)nullptr)) {
                double stepmax = std::fabs(t * val(dx[0])) / std::fabs(val(xt[0]));
                for (int a = 1; a < 4; ++a) stepmax = std::max(stepmax, std::fabs(t * val(dx[a])));
                if (rec_merit(rt, val(xt[0])) <= m0 || stepmax <= tol) {
                    accepted = true;
                    break;
                }
            }
            t *= 0.5;
        }
        if (!accepted) return fail(ST_NOCONV);
        double dp = std::fabs(val(xt[0]) - val(x[0]));
        double dv = 0;
        for (int a = 1; a < 4; ++a) dv = std::max(dv, std::fabs(val(xt[a]) - val(x[a])));
        for (int a = 0; a < 4; ++a) {
            x[a] = xt[a];
            r[a] = rt[a];
        }
        last_rel = dp / val(x[0]);
        if (dp <= tol * val(x[0]) && dv <= tol) {
            status = ST_OK;
            break;
        }
    }
    if (status != ST_OK) {
        it = maxit;
        if (last_rel <= 1e-12) status = ST_WARN;
        else return fail(ST_NOCONV);
    }
    T E[3];
    rec_residual(in, x, r, E);
    T v[3] = {x[1], x[2], x[3]}, vl[3];
    lower(m, v, vl);
    T W = 1.0 / sqrt(1.0 - dot3(vl, v));
    const T sg = m.sqrtg;
    P[P_RHO] = U[U_D] / (sg * W);
    P[P_PRS] = x[0];
    for (int i = 0; i < 3; ++i) {
        P[P_V + i] = v[i];
        P[P_B + i] = U[U_B + i] / sg;
        P[P_E + i] = E[i] / sg;
        Eout[i] = E[i];
    }
    P[P_PHI] = U[U_PHI] / sg;
    P[P_PSI] = U[U_PSI] / sg;
    P[P_Q] = U[U_Q] / sg;
    *iters = it;
    return status;
}

/* the stage solve: paper's 1D iteration when nothing is stiff (E fixed),
 * Newton on the same root otherwise */
template <class T>
int coupled_solve(const Metric<T>& m, double G, const T* U, const T* Estar, T adt, T sigma, const T* Pg, double tol,
                  int maxit, T* P, T* Eout, int* iters) {
    if (val(adt) == 0.0 || val(sigma) == 0.0)
        return recover_paper(m, G, U, Estar, adt, sigma, Pg, tol, maxit, P, Eout, iters);
    return recover_newton(m, G, U, Estar, adt, sigma, Pg, tol, maxit, P, Eout, iters);
}

/* ------------------------------------------------------------------------ */
/* Grid                                                                     */
/* ------------------------------------------------------------------------ */
enum { BC_PERIODIC = 0, BC_COPY = 1, BC_GIVEN = 2 };

struct Grid {                 /* mirrors oracle.py's ctypes structure */
    int32_t n[3];
    int32_t active;
    int32_t ng;
    int32_t bc[3];
    int32_t recon;
    int32_t c2p_maxit;
    int32_t speed_mode;
    int32_t sigma_model;      /* 0: the given sigma field; 1: eq. sigma_evol; 2: eq. dynamo_sigma */
    double x0[3], dx[3];
    double gamma_ad, kappa, c2p_tol;
    double sigma0, sigma_exp, sigma_Datmo;   /* parameters of the conductivity models */
    double rho_atmo, K_atmo;                 /* artificial atmosphere (rho_atmo = 0: none) */
};

/* Conductivity of a cell from the conserved rest-mass density D of its state:
 * model 1 is eq. sigma_evol, sigma = sigma0 D^gamma (Sec. IV.A), model 2 is
 * eq. dynamo_sigma, sigma = sigma0 max(1 - D_atmo/D, 0)^2 (Sec. IV.E); model
 * 0 returns the given per-cell field. */
template <class T> T conductivity(const Grid& gr, T sig_field, T D) {
    if (gr.sigma_model == 1) return gr.sigma0 * pw(D, gr.sigma_exp);
    if (gr.sigma_model == 2) {
        T t = tmax(1.0 - gr.sigma_Datmo / D, T(0.0));
        return gr.sigma0 * t * t;
    }
    return sig_field;
}

/* cells whose D lies below ATMO_FACTOR sqrt(gamma) rho_atmo are atmosphere */
constexpr double ATMO_FACTOR = 1.01;

struct Geo {
    int g[3], np[3];
    long Np;
    Geo(const Grid& gr) {
        for (int d = 0; d < 3; ++d) {
            g[d] = ((gr.active >> d) & 1) ? gr.ng : 0;
            np[d] = gr.n[d] + 2 * g[d];
        }
        Np = (long)np[0] * np[1] * np[2];
    }
    long idx(int i, int j, int k) const { return ((long)k * np[1] + j) * np[0] + i; }
    long stride(int d) const { return d == 0 ? 1 : (d == 1 ? np[0] : (long)np[0] * np[1]); }
};

/* ghost fill of nf fields (faces, edges and corners; only faces are read) */
template <class T> void ghost_fill(const Grid& gr, const Geo& ge, T* a, int nf) {
    for (int d = 0; d < 3; ++d) {
        if (!((gr.active >> d) & 1) || gr.bc[d] == BC_GIVEN) continue;
        int g = ge.g[d], n = gr.n[d];
        long st = ge.stride(d);
        for (int f = 0; f < nf; ++f) {
            T* b = a + (long)f * ge.Np;
            for (int k = 0; k < ge.np[2]; ++k)
                for (int j = 0; j < ge.np[1]; ++j)
                    for (int i = 0; i < ge.np[0]; ++i) {
                        int c[3] = {i, j, k};
                        int x = c[d];
                        if (x >= g && x < n + g) continue;
                        int src;
                        if (gr.bc[d] == BC_PERIODIC) src = x < g ? x + n : x - n;
                        else src = x < g ? g : n + g - 1;
                        long o = ge.idx(i, j, k);
                        b[o] = b[o + (src - x) * st];
                    }
        }
    }
}

template <class T> void load_metric(const T* metric, long Np, long o, T* f) {
    if (!metric) { flat_fields(f); return; }
    for (int a = 0; a < NM; ++a) f[a] = metric[(long)a * Np + o];
}

/* metric derivatives at a cell centre: 4th-order central differences along
 * active dimensions, zero along the others */
template <class T>
void metric_derivs(const Grid& gr, const Geo& ge, const T* metric, long o, T* dalp, T dbet[3][3], T dg[3][3][3]) {
    for (int i = 0; i < 3; ++i) {
        dalp[i] = T(0.0);
        for (int j = 0; j < 3; ++j) {
            dbet[i][j] = T(0.0);
            for (int k = 0; k < 3; ++k) dg[i][j][k] = T(0.0);
        }
    }
    if (!metric) return;
    for (int i = 0; i < 3; ++i) {
        if (!((gr.active >> i) & 1)) continue;
        long st = ge.stride(i);
        double h = gr.dx[i];
        auto D4 = [&](int fld) {
            const T* b = metric + (long)fld * ge.Np;
            return (b[o - 2 * st] - 8.0 * b[o - st] + 8.0 * b[o + st] - b[o + 2 * st]) / (12.0 * h);
        };
        dalp[i] = D4(M_ALP);
        for (int j = 0; j < 3; ++j) dbet[i][j] = D4(M_BET + j);
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) dg[i][j][k] = D4(M_G + SYM[j][k]);
    }
}

/* face metric between cells o and o+st: 4th-order interpolation */
template <class T> void face_metric(const T* metric, long Np, long o, long st, T* f) {
    if (!metric) { flat_fields(f); return; }
    for (int a = 0; a < NM; ++a) {
        const T* b = metric + (long)a * Np;
        f[a] = (-b[o - st] + 9.0 * b[o] + 9.0 * b[o + st] - b[o + 2 * st]) / 16.0;
    }
}

/* Explicit right-hand side F(U) of the stage with primitives Pst (ghosts
 * already filled), at interior cells: minus the flux divergence plus the
 * non-stiff sources (E rows: F_E). */
template <class T>
void explicit_rhs(const Grid& gr, const Geo& ge, const T* metric, const T* Pst, const T* sig, T* L) {
    const long Np = ge.Np;
    const double G = gr.gamma_ad;
    /* conductivity of each cell: the given field, or the model at the D of
     * the cell's primitives; a ghost cell, a copy of its interior image,
     * carries the image's value (as the given field does) */
    const T* sg = sig;
    std::vector<T> smod;
    if (gr.sigma_model != 0) {
        smod.assign((size_t)Np, T(0.0));
#pragma omp parallel for schedule(static)
        for (long o = 0; o < Np; ++o) {
            T mf[NM], P[NF], U[NF];
            load_metric(metric, Np, o, mf);
            Metric<T> m;
            metric_point(mf, m);
            for (int a = 0; a < NF; ++a) P[a] = Pst[(long)a * Np + o];
            T v[3] = {P[P_V], P[P_V + 1], P[P_V + 2]}, vl[3];
            lower(m, v, vl);
            if (!(val(P[P_RHO]) > 0.0) || !(val(dot3(vl, v)) < 1.0)) continue;   /* cells no face reads */
            prim2con(m, G, P, U);
            smod[(size_t)o] = conductivity(gr, T(0.0), U[U_D]);
        }
        ghost_fill(gr, ge, smod.data(), 1);
        sg = smod.data();
    }
    /* sources */
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = ge.g[2]; k < ge.g[2] + gr.n[2]; ++k)
        for (int j = ge.g[1]; j < ge.g[1] + gr.n[1]; ++j)
            for (int i = ge.g[0]; i < ge.g[0] + gr.n[0]; ++i) {
                long o = ge.idx(i, j, k);
                T mf[NM], P[NF], U[NF], S[NF];
                load_metric(metric, Np, o, mf);
                Metric<T> m;
                metric_point(mf, m);
                for (int a = 0; a < NF; ++a) P[a] = Pst[(long)a * Np + o];
                prim2con(m, G, P, U);
                T dalp[3], dbet[3][3], dg[3][3][3];
                metric_derivs(gr, ge, metric, o, dalp, dbet, dg);
                explicit_source(m, dalp, dbet, dg, gr.kappa, G, P, U, S);
                for (int a = 0; a < NF; ++a) L[(long)a * Np + o] = S[a];
            }
    /* flux divergence, one active direction at a time */
    std::vector<T> Fh((size_t)NF * Np);
    for (int d = 0; d < 3; ++d) {
        if (!((gr.active >> d) & 1)) continue;
        long st = ge.stride(d);
        int lo[3], hi[3];
        for (int e = 0; e < 3; ++e) { lo[e] = ge.g[e]; hi[e] = ge.g[e] + gr.n[e]; }
        lo[d] -= 1;   /* faces: left cell from g-1 to n+g-1 */
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = lo[2]; k < hi[2]; ++k)
            for (int j = lo[1]; j < hi[1]; ++j)
                for (int i = lo[0]; i < hi[0]; ++i) {
                    long o = ge.idx(i, j, k);
                    T mf[NM];
                    face_metric(metric, Np, o, st, mf);
                    Metric<T> m;
                    metric_point(mf, m);
                    T PL[NF], PR[NF];
                    for (int a = 0; a < NF; ++a) {
                        const T* b = Pst + (long)a * Np;
                        T fl[5], fr[5], dum;
                        for (int s = 0; s < 5; ++s) {
                            fl[s] = b[o + (s - 2) * st];
                            fr[s] = b[o + (s - 1) * st];
                        }
                        recon_cell(gr.recon, fl, dum, PL[a]);
                        recon_cell(gr.recon, fr, PR[a], dum);
                    }
                    /* first-order fallback for an unphysical face state */
                    for (int side = 0; side < 2; ++side) {
                        T* Ps = side ? PR : PL;
                        long oc = side ? o + st : o;
                        T v[3] = {Ps[P_V], Ps[P_V + 1], Ps[P_V + 2]}, vl[3];
                        lower(m, v, vl);
                        T v2 = dot3(vl, v);
                        if (!(val(Ps[P_RHO]) > 0) || !(val(Ps[P_PRS]) > 0) || !(val(v2) < 1.0))
                            for (int a = 0; a < NF; ++a) Ps[a] = Pst[(long)a * Np + oc];
                    }
                    /* current for the charge flux: mean of the two cell-centre currents */
                    T Jf;
                    {
                        T Jc[2][3];
                        for (int side = 0; side < 2; ++side) {
                            long oc = side ? o + st : o;
                            T Pc[NF], mc[NM];
                            for (int a = 0; a < NF; ++a) Pc[a] = Pst[(long)a * Np + oc];
                            load_metric(metric, Np, oc, mc);
                            Metric<T> mm;
                            metric_point(mc, mm);
                            cell_current(mm, G, Pc, sg[oc], Jc[side]);
                        }
                        Jf = 0.5 * (Jc[0][d] + Jc[1][d]);
                    }
                    T UL[NF], UR[NF], FL[NF], FR[NF], lp, lm;
                    prim2con(m, G, PL, UL);
                    prim2con(m, G, PR, UR);
                    phys_flux(m, G, PL, UL, T(0.0), d, FL, &Jf);
                    phys_flux(m, G, PR, UR, T(0.0), d, FR, &Jf);
                    char_speeds(m, d, gr.speed_mode, lp, lm);
                    T F[NF];
                    hlle(UL, UR, FL, FR, lp, lm, F);
                    for (int a = 0; a < NF; ++a) Fh[(size_t)a * Np + o] = F[a];
                }
        double h = gr.dx[d];
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = ge.g[2]; k < ge.g[2] + gr.n[2]; ++k)
            for (int j = ge.g[1]; j < ge.g[1] + gr.n[1]; ++j)
                for (int i = ge.g[0]; i < ge.g[0] + gr.n[0]; ++i) {
                    long o = ge.idx(i, j, k);
                    for (int a = 0; a < NF; ++a)
                        L[(long)a * Np + o] = L[(long)a * Np + o] -
                                               (Fh[(size_t)a * Np + o] - Fh[(size_t)a * Np + o - st]) / h;
                }
    }
}

/* IMEX-SSP2(2,2,2) constant, table imex */
inline double gam_imex() { return 1.0 - 1.0 / std::sqrt(2.0); }

/* copy of the primitives with ghosts filled, and a ghost-filled copy of sigma */
template <class T> std::vector<T> filled_copy(const Grid& gr, const Geo& ge, const T* a, int nf) {
    if (!a) return std::vector<T>((size_t)nf * ge.Np, T(0.0));   /* no sigma field: the models set it */
    std::vector<T> c(a, a + (size_t)nf * ge.Np);
    ghost_fill(gr, ge, c.data(), nf);
    return c;
}

/* Coupled solve on every interior cell.  Uin: conserved (E rows ignored),
 * Estar: [3][Np], Pg: guess.  Writes P, E (into Eout [3][Np]) and status. */
template <class T>
long solve_all(const Grid& gr, const Geo& ge, const T* metric, const T* Uin, const T* Estar, double adt,
               const T* sig, const T* Pg, T* Pout, T* Eout, int32_t* status, int32_t* iters) {
    const long Np = ge.Np;
    long nfail = 0;
#pragma omp parallel for collapse(2) schedule(dynamic, 1) reduction(+ : nfail)
    for (int k = ge.g[2]; k < ge.g[2] + gr.n[2]; ++k)
        for (int j = ge.g[1]; j < ge.g[1] + gr.n[1]; ++j)
            for (int i = ge.g[0]; i < ge.g[0] + gr.n[0]; ++i) {
                long o = ge.idx(i, j, k);
                T mf[NM], U[NF], P[NF], Pgs[NF], Es[3], E[3];
                load_metric(metric, Np, o, mf);
                Metric<T> m;
                metric_point(mf, m);
                for (int a = 0; a < NF; ++a) {
                    U[a] = Uin[(long)a * Np + o];
                    Pgs[a] = Pg[(long)a * Np + o];
                }
                for (int c = 0; c < 3; ++c) Es[c] = Estar[(long)c * Np + o];
                int it = 0;
                const T sc = adt == 0.0 ? T(0.0) : conductivity(gr, sig ? sig[o] : T(0.0), U[U_D]);
                int st = coupled_solve(m, gr.gamma_ad, U, Es, T(adt), sc, Pgs, gr.c2p_tol, gr.c2p_maxit, P, E,
                                       &it);
                for (int a = 0; a < NF; ++a) Pout[(long)a * Np + o] = P[a];
                for (int c = 0; c < 3; ++c) Eout[(long)c * Np + o] = E[c];
                if (status) status[o] = st;
                if (iters) iters[o] = it;
                if (st < 0) nfail += 1;
            }
    return nfail;
}

template <class T> void for_interior(const Grid& gr, const Geo& ge, T fn) {
    for (int k = ge.g[2]; k < ge.g[2] + gr.n[2]; ++k)
        for (int j = ge.g[1]; j < ge.g[1] + gr.n[1]; ++j)
            for (int i = ge.g[0]; i < ge.g[0] + gr.n[0]; ++i) fn(ge.idx(i, j, k));
}

/* Stage 1: U(1) = U^n + dt gamma R[U(1)] (only E changes).
 * Outputs P1, R1 = (E(1) - E^n)/(gamma dt), U1 (U^n with E replaced). */
template <class T>
long stage1(const Grid& gr, const T* metric, double dt, const T* sig, const T* Un, const T* Pn, T* P1, T* R1, T* U1,
            int32_t* status, int32_t* iters) {
    Geo ge(gr);
    const long Np = ge.Np;
    const double g = gam_imex();
    std::vector<T> E1((size_t)3 * Np);
    long nf = solve_all(gr, ge, metric, Un, Un + (long)U_E * Np, g * dt, sig, Pn, P1, E1.data(), status, iters);
    for_interior(gr, ge, [&](long o) {
        for (int c = 0; c < 3; ++c) R1[(long)c * Np + o] = (E1[(size_t)c * Np + o] - Un[(long)(U_E + c) * Np + o]) / (g * dt);
        if (U1) {
            for (int a = 0; a < NF; ++a) U1[(long)a * Np + o] = Un[(long)a * Np + o];
            for (int c = 0; c < 3; ++c) U1[(long)(U_E + c) * Np + o] = E1[(size_t)c * Np + o];
        }
    });
    return nf;
}

/* Stage 2: U(2) = U^n + dt F[U(1)] + dt{(1-2 gamma) R1 + gamma R[U(2)]}.
 * Also returns F1 = F[U(1)] (needed by the final update in its printed form). */
template <class T>
long stage2(const Grid& gr, const T* metric, double dt, const T* sig, const T* Un, const T* P1, const T* R1, T* U2,
            T* P2, T* R2, T* F1, int32_t* status, int32_t* iters) {
    Geo ge(gr);
    const long Np = ge.Np;
    const double g = gam_imex();
    std::vector<T> Pf = filled_copy(gr, ge, P1, NF);
    std::vector<T> sf = filled_copy(gr, ge, sig, 1);
    std::vector<T> L((size_t)NF * Np, T(0.0));
    explicit_rhs(gr, ge, metric, Pf.data(), sf.data(), L.data());
    std::vector<T> Y((size_t)NF * Np, T(0.0)), Es((size_t)3 * Np, T(0.0)), E2((size_t)3 * Np, T(0.0));
    for_interior(gr, ge, [&](long o) {
        for (int a = 0; a < NF; ++a) Y[(size_t)a * Np + o] = Un[(long)a * Np + o] + dt * L[(size_t)a * Np + o];
        for (int c = 0; c < 3; ++c)
            Es[(size_t)c * Np + o] = Un[(long)(U_E + c) * Np + o] + dt * L[(size_t)(U_E + c) * Np + o] +
                                     dt * (1.0 - 2.0 * g) * R1[(long)c * Np + o];
    });
    long nf = solve_all(gr, ge, metric, Y.data(), Es.data(), g * dt, sig, P1, P2, E2.data(), status, iters);
    for_interior(gr, ge, [&](long o) {
        for (int a = 0; a < NF; ++a) U2[(long)a * Np + o] = Y[(size_t)a * Np + o];
        for (int c = 0; c < 3; ++c) {
            U2[(long)(U_E + c) * Np + o] = E2[(size_t)c * Np + o];
            R2[(long)c * Np + o] = (E2[(size_t)c * Np + o] - Es[(size_t)c * Np + o]) / (g * dt);
        }
        if (F1)
            for (int a = 0; a < NF; ++a) F1[(long)a * Np + o] = L[(size_t)a * Np + o];
    });
    return nf;
}

/* Final update, eq. IMEX3 as printed:
 *   U^{n+1} = U^n + dt/2 (F[U(1)] + F[U(2)]) + dt/2 (R[U(1)] + R[U(2)]),
 * followed by the plain recovery (E fixed) with P2 as guess. */
template <class T>
long final_update(const Grid& gr, const T* metric, double dt, const T* sig, const T* Un, const T* F1, const T* P2,
                  const T* R1, const T* R2, T* Unp1, T* Pnp1, int32_t* status, int32_t* iters) {
    Geo ge(gr);
    const long Np = ge.Np;
    std::vector<T> Pf = filled_copy(gr, ge, P2, NF);
    std::vector<T> sf = filled_copy(gr, ge, sig, 1);
    std::vector<T> L((size_t)NF * Np, T(0.0));
    explicit_rhs(gr, ge, metric, Pf.data(), sf.data(), L.data());
    for_interior(gr, ge, [&](long o) {
        for (int a = 0; a < NF; ++a)
            Unp1[(long)a * Np + o] = Un[(long)a * Np + o] + 0.5 * dt * (F1[(long)a * Np + o] + L[(size_t)a * Np + o]);
        for (int c = 0; c < 3; ++c)
            Unp1[(long)(U_E + c) * Np + o] =
                Unp1[(long)(U_E + c) * Np + o] + 0.5 * dt * (R1[(long)c * Np + o] + R2[(long)c * Np + o]);
    });
    /* artificial atmosphere (Sec. IV.E): the hydro part of a cell whose D is
     * below ATMO_FACTOR sqrt(gamma) rho_atmo becomes that of the atmosphere
     * state (rho_atmo, p = K_atmo rho_atmo^Gamma, v = 0) with the cell's own
     * E, B and cleaning fields; the recovery below then returns that state */
    std::vector<char> atmo;
    if (gr.rho_atmo > 0.0) {
        atmo.assign((size_t)Np, 0);
        for_interior(gr, ge, [&](long o) {
            T mf[NM];
            load_metric(metric, Np, o, mf);
            Metric<T> m;
            metric_point(mf, m);
            if (!(val(Unp1[(long)U_D * Np + o]) < ATMO_FACTOR * val(m.sqrtg) * gr.rho_atmo)) return;
            atmo[(size_t)o] = 1;
            T Pa[NF], Ua[NF];
            Pa[P_RHO] = T(gr.rho_atmo);
            Pa[P_PRS] = T(gr.K_atmo * std::pow(gr.rho_atmo, gr.gamma_ad));
            for (int i = 0; i < 3; ++i) Pa[P_V + i] = T(0.0);
            for (int a = P_B; a < NF; ++a) Pa[a] = Unp1[(long)a * Np + o] / m.sqrtg;
            prim2con(m, gr.gamma_ad, Pa, Ua);
            for (int a = U_D; a <= U_TAU; ++a) Unp1[(long)a * Np + o] = Ua[a];
        });
    }
    std::vector<T> Ef((size_t)3 * Np, T(0.0));
    std::vector<int32_t> st((size_t)Np, 0);
    long nf = solve_all(gr, ge, metric, Unp1, Unp1 + (long)U_E * Np, 0.0, sig, P2, Pnp1, Ef.data(), st.data(), iters);
    if (!atmo.empty())
        for_interior(gr, ge, [&](long o) {
            if (atmo[(size_t)o] && st[(size_t)o] >= 0) st[(size_t)o] = 2;
        });
    if (status)
        for_interior(gr, ge, [&](long o) { status[o] = st[(size_t)o]; });
    return nf;
}

}  // namespace orc

/* ======================================================================== */
/* C ABI of the oracle (double).  All arrays are host arrays, field-major,  */
/* padded with ghost cells, x fastest.  metric may be NULL (flat space).    */
/* ======================================================================== */
using namespace orc;

extern "C" {

double orc_gamma_imex(void) { return gam_imex(); }

/* -- pointwise functions (for pins) ------------------------------------- */
void orc_point_prim2con(const double* mf, double G, const double* P, double* U) {
    Metric<double> m;
    double f[NM];
    if (mf) std::memcpy(f, mf, sizeof f); else flat_fields(f);
    metric_point(f, m);
    prim2con(m, G, P, U);
}
void orc_point_metric(const double* mf, double* gi9, double* sqrtg) {
    Metric<double> m;
    metric_point(mf, m);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) gi9[3 * i + j] = m.gi[i][j];
    *sqrtg = m.sqrtg;
}
void orc_point_flux(const double* mf, double G, const double* P, double sigma, int d, double* F) {
    Metric<double> m;
    double f[NM], U[NF];
    if (mf) std::memcpy(f, mf, sizeof f); else flat_fields(f);
    metric_point(f, m);
    prim2con(m, G, P, U);
    phys_flux(m, G, P, U, sigma, d, F);
}
void orc_point_hlle(const double* mf, double G, const double* PL, const double* PR, double sigma, int d, int mode,
                    double* Fh) {
    Metric<double> m;
    double f[NM], UL[NF], UR[NF], FL[NF], FR[NF], lp, lm;
    if (mf) std::memcpy(f, mf, sizeof f); else flat_fields(f);
    metric_point(f, m);
    prim2con(m, G, PL, UL);
    prim2con(m, G, PR, UR);
    phys_flux(m, G, PL, UL, sigma, d, FL);
    phys_flux(m, G, PR, UR, sigma, d, FR);
    char_speeds(m, d, mode, lp, lm);
    hlle(UL, UR, FL, FR, lp, lm, Fh);
}
void orc_point_speeds(const double* mf, int d, int mode, double* lp, double* lm) {
    Metric<double> m;
    double f[NM];
    if (mf) std::memcpy(f, mf, sizeof f); else flat_fields(f);
    metric_point(f, m);
    char_speeds(m, d, mode, *lp, *lm);
}
void orc_point_stiff(const double* mf, const double* v, const double* Ec, const double* Bc, double sigma, double* R) {
    Metric<double> m;
    double f[NM];
    if (mf) std::memcpy(f, mf, sizeof f); else flat_fields(f);
    metric_point(f, m);
    stiff_source(m, v, Ec, Bc, sigma, R);
}
void orc_point_esolve(const double* mf, const double* v, const double* Bc, const double* Estar, double c, double* E) {
    Metric<double> m;
    double f[NM];
    if (mf) std::memcpy(f, mf, sizeof f); else flat_fields(f);
    metric_point(f, m);
    for (int i = 0; i < 3; ++i) E[i] = Estar[i];
    esolve_nr(m, v, Bc, Estar, c, E);
}
int orc_point_recover_paper(const double* mf, double G, const double* U, const double* Estar, double adt,
                            double sigma, const double* Pg, double tol, int maxit, double* P, double* E, int* iters) {
    Metric<double> m;
    double f[NM];
    if (mf) std::memcpy(f, mf, sizeof f); else flat_fields(f);
    metric_point(f, m);
    return recover_paper(m, G, U, Estar, adt, sigma, Pg, tol, maxit, P, E, iters);
}
int orc_point_coupled(const double* mf, double G, const double* U, const double* Estar, double adt, double sigma,
                      const double* Pg, double tol, int maxit, double* P, double* E, int* iters) {
    Metric<double> m;
    double f[NM];
    if (mf) std::memcpy(f, mf, sizeof f); else flat_fields(f);
    metric_point(f, m);
    return coupled_solve(m, G, U, Estar, adt, sigma, Pg, tol, maxit, P, E, iters);
}
void orc_recon(int method, const double* f5, double* fm, double* fp) { recon_cell(method, f5, *fm, *fp); }

/* -- grid functions ------------------------------------------------------ */
long orc_padded_cells(const Grid* gr) { return Geo(*gr).Np; }

void orc_ghost_fill(const Grid* gr, double* a, int nf) { ghost_fill(*gr, Geo(*gr), a, nf); }

void orc_prim2con(const Grid* gr, const double* metric, const double* P, double* U) {
    Geo ge(*gr);
    const long Np = ge.Np;
#pragma omp parallel for schedule(static)
    for (long o = 0; o < Np; ++o) {
        int i = o % ge.np[0], j = (o / ge.np[0]) % ge.np[1], k = o / ((long)ge.np[0] * ge.np[1]);
        if (i < ge.g[0] || i >= ge.g[0] + gr->n[0] || j < ge.g[1] || j >= ge.g[1] + gr->n[1] || k < ge.g[2] ||
            k >= ge.g[2] + gr->n[2])
            continue;
        double mf[NM], p[NF], u[NF];
        load_metric(metric, Np, o, mf);
        Metric<double> m;
        metric_point(mf, m);
        for (int a = 0; a < NF; ++a) p[a] = P[(long)a * Np + o];
        prim2con(m, gr->gamma_ad, p, u);
        for (int a = 0; a < NF; ++a) U[(long)a * Np + o] = u[a];
    }
}

long orc_con2prim(const Grid* gr, const double* metric, const double* U, const double* Pg, double* P,
                  int32_t* status, int32_t* iters) {
    Geo ge(*gr);
    std::vector<double> E((size_t)3 * ge.Np), sig(ge.Np, 0.0);
    return solve_all(*gr, ge, metric, U, U + (long)U_E * ge.Np, 0.0, sig.data(), Pg, P, E.data(), status, iters);
}

void orc_explicit_rhs(const Grid* gr, const double* metric, const double* P, const double* sig, double* L) {
    Geo ge(*gr);
    std::vector<double> Pf = filled_copy(*gr, ge, P, NF);
    std::vector<double> sf = filled_copy(*gr, ge, sig, 1);
    explicit_rhs(*gr, ge, metric, Pf.data(), sf.data(), L);
}

long orc_stage1(const Grid* gr, const double* metric, double dt, const double* sig, const double* Un,
                const double* Pn, double* P1, double* R1, double* U1, int32_t* status, int32_t* iters) {
    return stage1(*gr, metric, dt, sig, Un, Pn, P1, R1, U1, status, iters);
}
long orc_stage2(const Grid* gr, const double* metric, double dt, const double* sig, const double* Un,
                const double* P1, const double* R1, double* U2, double* P2, double* R2, double* F1,
                int32_t* status, int32_t* iters) {
    return stage2(*gr, metric, dt, sig, Un, P1, R1, U2, P2, R2, F1, status, iters);
}
long orc_final(const Grid* gr, const double* metric, double dt, const double* sig, const double* Un,
               const double* F1, const double* P2, const double* R1, const double* R2, double* Unp1, double* Pnp1,
               int32_t* status, int32_t* iters) {
    return final_update(*gr, metric, dt, sig, Un, F1, P2, R1, R2, Unp1, Pnp1, status, iters);
}

/* one full step in place on (U, P); returns the number of failed cells;
 * status (optional, [Np]): the final recovery's status (2: atmosphere) */
long orc_step(const Grid* gr, const double* metric, double dt, const double* sig, double* U, double* P,
              int32_t* status) {
    Geo ge(*gr);
    size_t n = (size_t)NF * ge.Np;
    std::vector<double> P1(P, P + n), U1(U, U + n), R1((size_t)3 * ge.Np, 0.0), U2(U, U + n), P2(P, P + n),
        R2((size_t)3 * ge.Np, 0.0), F1(n, 0.0);
    long nf = stage1(*gr, metric, dt, sig, U, P, P1.data(), R1.data(), U1.data(), (int32_t*)nullptr,
                     (int32_t*)nullptr);
    nf += stage2(*gr, metric, dt, sig, U, P1.data(), R1.data(), U2.data(), P2.data(), R2.data(), F1.data(),
                 (int32_t*)nullptr, (int32_t*)nullptr);
    std::vector<double> Un(U, U + n);
    nf += final_update(*gr, metric, dt, sig, Un.data(), F1.data(), P2.data(), R1.data(), R2.data(), U, P,
                       status, (int32_t*)nullptr);
    return nf;
}

/* Tangent of one step (forward-mode dual numbers through every function
 * above, recovery roots included): (U, P) advance in place, dU carries the
 * directional derivative for the input direction (dU, dsigma).  dP, the
 * derivative of the primitives, is written too. */
long orc_step_tangent(const Grid* gr, const double* metric, double dt, const double* sig, const double* dsig,
                      double* U, double* dU, double* P, double* dP) {
    Geo ge(*gr);
    const size_t n = (size_t)NF * ge.Np;
    std::vector<Dual> Ud(n), Pd(n), sd(ge.Np), md;
    for (size_t i = 0; i < n; ++i) {
        Ud[i] = Dual(U[i], dU[i]);
        Pd[i] = Dual(P[i], 0.0);
    }
    for (long i = 0; i < ge.Np; ++i) sd[i] = Dual(sig[i], dsig ? dsig[i] : 0.0);
    const Dual* mp = nullptr;
    if (metric) {
        md.resize((size_t)NM * ge.Np);
        for (size_t i = 0; i < md.size(); ++i) md[i] = Dual(metric[i]);
        mp = md.data();
    }
    std::vector<Dual> P1(Pd), U1(Ud), R1((size_t)3 * ge.Np, Dual(0.0)), U2(Ud), P2(Pd), R2((size_t)3 * ge.Np, Dual(0.0)),
        F1(n, Dual(0.0));
    long nf = stage1(*gr, mp, dt, sd.data(), Ud.data(), Pd.data(), P1.data(), R1.data(), U1.data(), (int32_t*)nullptr,
                     (int32_t*)nullptr);
    nf += stage2(*gr, mp, dt, sd.data(), Ud.data(), P1.data(), R1.data(), U2.data(), P2.data(), R2.data(), F1.data(),
                 (int32_t*)nullptr, (int32_t*)nullptr);
    std::vector<Dual> Un(Ud);
    nf += final_update(*gr, mp, dt, sd.data(), Un.data(), F1.data(), P2.data(), R1.data(), R2.data(), Ud.data(),
                       Pd.data(), (int32_t*)nullptr, (int32_t*)nullptr);
    for (size_t i = 0; i < n; ++i) {
        U[i] = Ud[i].v;
        dU[i] = Ud[i].d;
        P[i] = Pd[i].v;
        if (dP) dP[i] = Pd[i].d;
    }
    return nf;
}

/* max over interior cells and active d of max|lambda^d_+-| / dx_d */
double orc_max_signal_speed(const Grid* gr, const double* metric) {
    Geo ge(*gr);
    double best = 0.0;
    for_interior(*gr, ge, [&](long o) {
        double mf[NM];
        load_metric(metric, ge.Np, o, mf);
        Metric<double> m;
        metric_point(mf, m);
        for (int d = 0; d < 3; ++d) {
            if (!((gr->active >> d) & 1)) continue;
            double lp, lm;
            char_speeds(m, d, gr->speed_mode, lp, lm);
            best = std::max(best, std::max(std::fabs(lp), std::fabs(lm)) / gr->dx[d]);
        }
    });
    return best;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

// thread count of the later parallel loops (timing of the CPU baseline)
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

}  // extern "C"
