// Pointwise physics of resistive GRMHD for gfx950 (device code).
//
// Equations of arXiv:2510.18968: conserved variables (eqs. conserved_dens,
// conserved_tau, conserved_S and the densitised fields of Sec. II.D), fluxes
// and sources (eq. GRRMHD_flux_form), Ohm's law (eq. Ohm_law), the stiff E
// source and its implicit solve (Sec. III.A, eq. 3D_NR), the primitive
// recovery (Sec. III.B) and the reconstructions named in Sec. III.
//
// Field order.  Primitives: rho, p, v^x..z, B^x..z, E^x..z, phi, psi, q.
// Conserved: D, S_x..z, tau, Bcal^x..z, Ecal^x..z, Phi, Psi, Qcal.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

namespace rmhd {

using ::sqrt;
using ::fabs;
using ::fmin;
using ::fmax;

// FP64 reciprocal / reciprocal square root: hardware estimate refined by two
// Newton steps (about 1 ulp; no IEEE scaling or fix-up, so arguments must be
// finite and nonzero -- every call site divides by a positive quantity).
__device__ __forceinline__ double frcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ double frsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    return y * fma(-h * y, y, 1.5);
}
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsqrt(float x) { return __builtin_amdgcn_rsqf(x); }

constexpr int NF = 14;
enum : int { I_RHO = 0, I_P = 1, I_V = 2, I_B = 5, I_E = 8, I_PHI = 11, I_PSI = 12, I_Q = 13 };
enum : int { I_D = 0, I_S = 1, I_TAU = 4 };
enum : int { REC_MINMOD = 0, REC_MC2 = 1, REC_WENO5 = 2 };

// symmetric 3x3 packed as xx, xy, xz, yy, yz, zz
__host__ __device__ constexpr int sidx(int i, int j) {
    return (i == j) ? (i == 0 ? 0 : (i == 1 ? 3 : 5)) : ((i + j == 1) ? 1 : ((i + j == 2) ? 2 : 4));
}

// 3-metric at one point with the quantities derived from it (Sec. II.A).
// DG: the metric is diagonal (gamma_xy = gamma_xz = gamma_yz = 0, e.g.
// conformally flat); its off-diagonal entries are held as zero and the
// contractions below skip them.
template <class R, bool DG = false> struct Geo {
    static constexpr bool diag = DG;
    R alp, bet[3], g[6], gi[6], sg, isg;
};

// packed symmetric index a is an entry a diagonal metric holds as zero
template <bool DG> __host__ __device__ constexpr bool zero_entry(int a) { return DG && (a == 1 || a == 2 || a == 4); }

template <class R, bool DG> __device__ __forceinline__ void geo_flat(Geo<R, DG>& m) {
    m.alp = R(1);
    m.bet[0] = m.bet[1] = m.bet[2] = R(0);
    m.g[0] = m.g[3] = m.g[5] = R(1);
    m.g[1] = m.g[2] = m.g[4] = R(0);
    for (int a = 0; a < 6; ++a) m.gi[a] = m.g[a];
    m.sg = m.isg = R(1);
}

// inverse by cofactors and sqrt(det); m.g already set (its diagonal, for DG)
template <class R, bool DG> __device__ __forceinline__ void geo_finish(Geo<R, DG>& m) {
    if constexpr (DG) {
        const R gxx = m.g[0], gyy = m.g[3], gzz = m.g[5];
        m.g[1] = m.g[2] = m.g[4] = R(0);
        const R cxx = gyy * gzz;
        const R det = gxx * cxx;
        const R rs = frsqrt(det);
        const R id = rs * rs;
        m.gi[0] = cxx * id;
        m.gi[1] = m.gi[2] = m.gi[4] = R(0);
        m.gi[3] = (gxx * gzz) * id;
        m.gi[5] = (gxx * gyy) * id;
        m.sg = det * rs;
        m.isg = rs;
        return;
    }
    const R gxx = m.g[0], gxy = m.g[1], gxz = m.g[2], gyy = m.g[3], gyz = m.g[4], gzz = m.g[5];
    const R cxx = gyy * gzz - gyz * gyz;
    const R cxy = gxz * gyz - gxy * gzz;
    const R cxz = gxy * gyz - gxz * gyy;
    const R det = gxx * cxx + gxy * cxy + gxz * cxz;
    const R rs = frsqrt(det);
    const R id = rs * rs;
    m.gi[0] = cxx * id;
    m.gi[1] = cxy * id;
    m.gi[2] = cxz * id;
    m.gi[3] = (gxx * gzz - gxz * gxz) * id;
    m.gi[4] = (gxy * gxz - gxx * gyz) * id;
    m.gi[5] = (gxx * gyy - gxy * gxy) * id;
    m.sg = det * rs;
    m.isg = rs;
}

template <class M, class R> __device__ __forceinline__ void lower(const M* g, const R* u, R* l) {
    l[0] = g[0] * u[0] + g[1] * u[1] + g[2] * u[2];
    l[1] = g[1] * u[0] + g[3] * u[1] + g[4] * u[2];
    l[2] = g[2] * u[0] + g[4] * u[1] + g[5] * u[2];
}
// gamma_ij u^j
template <class M, bool DG, class R> __device__ __forceinline__ void lower(const Geo<M, DG>& m, const R* u, R* l) {
    if constexpr (DG) {
        l[0] = m.g[0] * u[0];
        l[1] = m.g[3] * u[1];
        l[2] = m.g[5] * u[2];
    } else {
        lower(m.g, u, l);
    }
}
// component D of gamma^ij l_j
template <int D, class M, bool DG, class R> __device__ __forceinline__ R raise1(const Geo<M, DG>& m, const R* l) {
    if constexpr (DG) return l[D] * m.gi[sidx(D, D)];
    else return l[0] * m.gi[sidx(D, 0)] + l[1] * m.gi[sidx(D, 1)] + l[2] * m.gi[sidx(D, 2)];
}
template <class R> __device__ __forceinline__ R dot3(const R* a, const R* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
// (a x b)^i = eta^{ijk} a_j b_k
template <class R> __device__ __forceinline__ void cross(const R* a, const R* b, R* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// ---------------------------------------------------------------- prim2con
template <class M, bool DG, class R>
__device__ __forceinline__ void prim2con(const Geo<M, DG>& m, R G, const R* P, R* U) {
    const R* v = P + I_V;
    const R* B = P + I_B;
    const R* E = P + I_E;
    R vl[3], Bl[3], El[3], c[3];
    lower(m, v, vl);
    lower(m, B, Bl);
    lower(m, E, El);
    const R W = frsqrt(R(1) - dot3(vl, v));
    const R W2 = W * W;
    const R hW2 = (P[I_RHO] + G / (G - R(1)) * P[I_P]) * W2;
    const R em = R(0.5) * (dot3(El, E) + dot3(Bl, B));
    cross(E, B, c);   // eta_ijk E^j B^k; epsilon_ijk = sqrt(gamma) eta_ijk
    const R D = P[I_RHO] * W * m.sg;
    U[I_D] = D;
    for (int i = 0; i < 3; ++i) U[I_S + i] = (hW2 * vl[i] + c[i] * m.sg) * m.sg;
    U[I_TAU] = (hW2 - P[I_P] + em) * m.sg - D;
    for (int a = I_B; a < NF; ++a) U[a] = P[a] * m.sg;
}

// densitised current of eq. Ohm_law at a point:
// J^i = Q v^i + W sigma [Ecal^i + (v_l x B_l)^i - (v_l . Ecal) v^i]
template <class M, bool DG, class R>
__device__ __forceinline__ void current(const Geo<M, DG>& m, const R* P, R sigma, R* J) {
    const R* v = P + I_V;
    R vl[3], Bl[3], vb[3];
    lower(m, v, vl);
    lower(m, P + I_B, Bl);
    cross(vl, Bl, vb);
    const R W = frsqrt(R(1) - dot3(vl, v));
    const R Ec[3] = {P[I_E] * m.sg, P[I_E + 1] * m.sg, P[I_E + 2] * m.sg};
    const R vE = dot3(vl, Ec);
    const R Q = P[I_Q] * m.sg;
    for (int i = 0; i < 3; ++i) J[i] = Q * v[i] + W * sigma * (Ec[i] + vb[i] - vE * v[i]);
}

// conserved variables and physical flux along D of one state (eqs.
// conserved_*, GRRMHD_flux_form with sqrt(gamma) counted once); Jd is the
// current carried by the charge flux at this face
template <int D, class M, bool DG, class R>
__device__ __forceinline__ void state_flux(const Geo<M, DG>& m, R G, const R* P, R Jd, R* U, R* F) {
    const R* v = P + I_V;
    const R* B = P + I_B;
    const R* E = P + I_E;
    R vl[3], Bl[3], El[3], c[3];
    lower(m, v, vl);
    lower(m, B, Bl);
    lower(m, E, El);
    const R W = frsqrt(R(1) - dot3(vl, v));
    const R hW2 = (P[I_RHO] + G / (G - R(1)) * P[I_P]) * (W * W);
    const R em = R(0.5) * (dot3(El, E) + dot3(Bl, B));
    const R pt = P[I_P] + em;
    cross(E, B, c);
    const M sg = m.sg;
    const R Dd = P[I_RHO] * W * sg;
    U[I_D] = Dd;
    for (int i = 0; i < 3; ++i) U[I_S + i] = (hW2 * vl[i] + c[i] * sg) * sg;
    U[I_TAU] = (hW2 - P[I_P] + em) * sg - Dd;
    for (int a = I_B; a < NF; ++a) U[a] = P[a] * sg;
    const M a = m.alp, bd = m.bet[D], as = m.alp * sg;
    const R vd = v[D], Ed = E[D], Bd = B[D];
    F[I_D] = (a * vd - bd) * Dd;
    for (int i = 0; i < 3; ++i)
        F[I_S + i] = as * (hW2 * vd * vl[i] - Ed * El[i] - Bd * Bl[i] + (i == D ? pt : R(0))) - bd * U[I_S + i];
    const R Sd = raise1<D>(m, U + I_S);
    F[I_TAU] = a * (Sd - vd * Dd) - bd * U[I_TAU];
    // (e_D x X)^i for covariant X
    R eE[3], eB[3];
    if (D == 0) { eE[0] = R(0); eE[1] = -El[2]; eE[2] = El[1]; eB[0] = R(0); eB[1] = -Bl[2]; eB[2] = Bl[1]; }
    if (D == 1) { eE[0] = El[2]; eE[1] = R(0); eE[2] = -El[0]; eB[0] = Bl[2]; eB[1] = R(0); eB[2] = -Bl[0]; }
    if (D == 2) { eE[0] = -El[1]; eE[1] = El[0]; eE[2] = R(0); eB[0] = -Bl[1]; eB[1] = Bl[0]; eB[2] = R(0); }
    for (int i = 0; i < 3; ++i) {
        if (zero_entry<DG>(sidx(i, D))) {
            F[I_B + i] = a * eE[i] - bd * U[I_B + i];
            F[I_E + i] = -a * eB[i] - bd * U[I_E + i];
        } else {
            const M gid = m.gi[sidx(i, D)];
            F[I_B + i] = a * (eE[i] + gid * U[I_PHI]) - bd * U[I_B + i];
            F[I_E + i] = -a * (eB[i] - gid * U[I_PSI]) - bd * U[I_E + i];
        }
    }
    F[I_PHI] = a * U[I_B + D] - bd * U[I_PHI];
    F[I_PSI] = a * U[I_E + D] - bd * U[I_PSI];
    F[I_Q] = a * Jd - bd * U[I_Q];
}

// Reverse of state_flux at one state (the face current Jd held fixed):
// Pb = (dF/dP)^T wF + (dU/dP)^T wU, by the chain rule through the same
// intermediates (lowered vectors, W, h, E x B) in reverse order.
template <int D>
__device__ __forceinline__ void state_flux_vjp(const Geo<double>& m, double G, const double* P, const double* wF,
                                               const double* wU, double* Pb) {
    const double* v = P + I_V;
    const double* B = P + I_B;
    const double* E = P + I_E;
    double vl[3], Bl[3], El[3], c[3];
    lower(m.g, v, vl);
    lower(m.g, B, Bl);
    lower(m.g, E, El);
    const double W = frsqrt(1.0 - dot3(vl, v));
    const double kap = G / (G - 1.0);
    const double h = P[I_RHO] + kap * P[I_P];
    const double hW2 = h * (W * W);
    cross(E, B, c);
    const double sg = m.sg, a = m.alp, bd = m.bet[D], as = m.alp * sg;
    const double Dd = P[I_RHO] * W * sg;
    const double vd = v[D], Ed = E[D], Bd = B[D];
    // adjoints of U (direct weights and through F's -beta U terms) and of the intermediates
    double Ub[NF];
    for (int f = 0; f < NF; ++f) Ub[f] = wU[f] - bd * wF[f];
    double vd_b = 0.0, Dd_b = 0.0, hW2_b = 0.0, Ed_b = 0.0, Bd_b = 0.0, pt_b = 0.0, em_b = 0.0;
    double vl_b[3] = {0.0, 0.0, 0.0}, El_b[3] = {0.0, 0.0, 0.0}, Bl_b[3] = {0.0, 0.0, 0.0};
    // F_D = a vd Dd - bd U_D (the second term is in Ub)
    vd_b += wF[I_D] * a * Dd;
    Dd_b += wF[I_D] * a * vd;
    // F_S_i = as (hW2 vd vl_i - Ed El_i - Bd Bl_i + delta_iD pt) - bd U_S_i
    for (int i = 0; i < 3; ++i) {
        const double w = wF[I_S + i] * as;
        hW2_b += w * vd * vl[i];
        vd_b += w * hW2 * vl[i];
        vl_b[i] += w * hW2 * vd;
        Ed_b -= w * El[i];
        El_b[i] -= w * Ed;
        Bd_b -= w * Bl[i];
        Bl_b[i] -= w * Bd;
    }
    pt_b += wF[I_S + D] * as;
    // F_tau = a (Sd - vd Dd) - bd U_tau, Sd = U_S_i gamma^{Di}
    {
        const double w = wF[I_TAU] * a;
        for (int i = 0; i < 3; ++i) Ub[I_S + i] += w * m.gi[sidx(D, i)];
        vd_b -= w * Dd;
        Dd_b -= w * vd;
    }
    // F_B_i = a ((e_D x E_l)_i + gamma^{iD} U_phi) - bd U_B_i, F_E_i = -a ((e_D x B_l)_i - gamma^{iD} U_psi) - bd U_E_i
    // with (e_D x X)_i = X_{D+2} for i = D+1 and -X_{D+1} for i = D+2 (indices mod 3)
    {
        const int i1 = (D + 1) % 3, i2 = (D + 2) % 3;
        El_b[i2] += -a * wF[I_B + i1];
        El_b[i1] += a * wF[I_B + i2];
        Bl_b[i2] -= -a * wF[I_E + i1];
        Bl_b[i1] -= a * wF[I_E + i2];
        for (int i = 0; i < 3; ++i) {
            Ub[I_PHI] += a * wF[I_B + i] * m.gi[sidx(i, D)];
            Ub[I_PSI] += a * wF[I_E + i] * m.gi[sidx(i, D)];
        }
        Ub[I_B + D] += a * wF[I_PHI];
        Ub[I_E + D] += a * wF[I_PSI];
    }
    // U -> intermediates
    Dd_b += Ub[I_D];
    double c_b[3];
    for (int i = 0; i < 3; ++i) {
        hW2_b += Ub[I_S + i] * sg * vl[i];
        vl_b[i] += Ub[I_S + i] * sg * hW2;
        c_b[i] = Ub[I_S + i] * sg * sg;
    }
    double p_b = 0.0;
    hW2_b += Ub[I_TAU] * sg;
    p_b -= Ub[I_TAU] * sg;
    em_b += Ub[I_TAU] * sg;
    Dd_b -= Ub[I_TAU];
    // pt = p + em
    p_b += pt_b;
    em_b += pt_b;
    double v_b[3], B_b[3], E_b[3];
    for (int i = 0; i < 3; ++i) {
        B_b[i] = Ub[I_B + i] * sg + em_b * Bl[i];
        E_b[i] = Ub[I_E + i] * sg + em_b * El[i];
    }
    // c = E x B: E_b += B x c_b, B_b += c_b x E
    E_b[0] += B[1] * c_b[2] - B[2] * c_b[1];
    E_b[1] += B[2] * c_b[0] - B[0] * c_b[2];
    E_b[2] += B[0] * c_b[1] - B[1] * c_b[0];
    B_b[0] += c_b[1] * E[2] - c_b[2] * E[1];
    B_b[1] += c_b[2] * E[0] - c_b[0] * E[2];
    B_b[2] += c_b[0] * E[1] - c_b[1] * E[0];
    E_b[D] += Ed_b;
    B_b[D] += Bd_b;
    // El = g E, Bl = g B (g symmetric)
    double t[3];
    lower(m.g, El_b, t);
    for (int i = 0; i < 3; ++i) E_b[i] += t[i];
    lower(m.g, Bl_b, t);
    for (int i = 0; i < 3; ++i) B_b[i] += t[i];
    // Dd = rho W sg, hW2 = h W^2, h = rho + kap p
    double rho_b = Dd_b * W * sg;
    double W_b = Dd_b * P[I_RHO] * sg + hW2_b * 2.0 * h * W;
    const double h_b = hW2_b * W * W;
    rho_b += h_b;
    p_b += kap * h_b;
    // W = (1 - vl.v)^(-1/2): dW/d(vl.v) = W^3 / 2; d(vl.v)/dv = 2 vl
    const double v2_b = W_b * 0.5 * W * W * W;
    lower(m.g, vl_b, t);
    for (int i = 0; i < 3; ++i) v_b[i] = 2.0 * v2_b * vl[i] + t[i];
    v_b[D] += vd_b;
    Pb[I_RHO] = rho_b;
    Pb[I_P] = p_b;
    for (int i = 0; i < 3; ++i) {
        Pb[I_V + i] = v_b[i];
        Pb[I_B + i] = B_b[i];
        Pb[I_E + i] = E_b[i];
    }
    Pb[I_PHI] = Ub[I_PHI] * sg;
    Pb[I_PSI] = Ub[I_PSI] * sg;
    Pb[I_Q] = Ub[I_Q] * sg;
}

// ---------------------------------------------------------------- reconstruction
template <class R> __device__ __forceinline__ R mm2(R a, R b) {
    // minmod: 0 unless a, b share a sign, else the one of smaller magnitude
    return (a * b <= R(0)) ? R(0) : (fabs(a) < fabs(b) ? a : b);
}

// face values of the middle cell of s[0..4]: fm at i-1/2, fp at i+1/2
template <int RECON, class R> __device__ __forceinline__ void recon(const R* s, R& fm, R& fp) {
    if constexpr (RECON == REC_WENO5) {
        // WENO5-JS weights a_k = d_k / (eps + beta_k)^2 over the common
        // denominator e0 e1 e2: two divisions per cell instead of five; the
        // smoothness indicators are shared by the two faces
        const R eps = R(1e-6);
        const R t0 = s[0] - R(2) * s[1] + s[2], u0 = s[0] - R(4) * s[1] + R(3) * s[2];
        const R t1 = s[1] - R(2) * s[2] + s[3], u1 = s[1] - s[3];
        const R t2 = s[2] - R(2) * s[3] + s[4], u2 = R(3) * s[2] - R(4) * s[3] + s[4];
        const R c13 = R(13) / R(12);
        const R e0 = eps + (c13 * t0 * t0 + R(0.25) * u0 * u0);
        const R e1 = eps + (c13 * t1 * t1 + R(0.25) * u1 * u1);
        const R e2 = eps + (c13 * t2 * t2 + R(0.25) * u2 * u2);
        const R s0 = e0 * e0, s1 = e1 * e1, s2 = e2 * e2;
        const R p12 = s1 * s2, p02 = s0 * s2, p01 = s0 * s1;
        // six times the candidate values
        const R q0 = R(2) * s[0] - R(7) * s[1] + R(11) * s[2];
        const R q1 = -s[1] + R(5) * s[2] + R(2) * s[3];
        const R q2 = R(2) * s[2] + R(5) * s[3] - s[4];
        const R r0 = R(2) * s[4] - R(7) * s[3] + R(11) * s[2];
        const R r1 = -s[3] + R(5) * s[2] + R(2) * s[1];
        const R r2 = R(2) * s[2] + R(5) * s[1] - s[0];
        const R ap0 = R(0.1) * p12, ap1 = R(0.6) * p02, ap2 = R(0.3) * p01;   // right face
        const R am0 = R(0.1) * p01, am1 = R(0.6) * p02, am2 = R(0.3) * p12;   // left face (mirror)
        fp = (ap0 * q0 + ap1 * q1 + ap2 * q2) * frcp(R(6) * (ap0 + ap1 + ap2));
        fm = (am0 * r0 + am1 * r1 + am2 * r2) * frcp(R(6) * (am0 + am1 + am2));
    } else {
        const R dm = s[2] - s[1], dp = s[3] - s[2];
        R sl;
        if constexpr (RECON == REC_MINMOD) {
            sl = mm2(dm, dp);
        } else {   // MC2: minmod(2 dm, 2 dp, (dm + dp)/2)
            const R c = R(0.5) * (dm + dp);
            sl = (dm * dp <= R(0)) ? R(0) : (c > R(0) ? fmin(fmin(R(2) * dm, R(2) * dp), c)
                                                        : fmax(fmax(R(2) * dm, R(2) * dp), c));
        }
        fm = s[2] - R(0.5) * sl;
        fp = s[2] + R(0.5) * sl;
    }
}

// Reverse of recon<RECON> at one cell: g[j] = bm dfm/ds[j] + bp dfp/ds[j]
// (FP64).  Through the TVD limiters the derivative is that of the branch
// taken, with the same comparisons as recon.
template <int RECON> __device__ __forceinline__ void recon_vjp(const double* s, double bm, double bp, double* g) {
    if constexpr (RECON == REC_WENO5) {
        const double eps = 1e-6;
        const double t0 = s[0] - 2.0 * s[1] + s[2], u0 = s[0] - 4.0 * s[1] + 3.0 * s[2];
        const double t1 = s[1] - 2.0 * s[2] + s[3], u1 = s[1] - s[3];
        const double t2 = s[2] - 2.0 * s[3] + s[4], u2 = 3.0 * s[2] - 4.0 * s[3] + s[4];
        const double c13 = 13.0 / 12.0;
        const double e0 = eps + (c13 * t0 * t0 + 0.25 * u0 * u0);
        const double e1 = eps + (c13 * t1 * t1 + 0.25 * u1 * u1);
        const double e2 = eps + (c13 * t2 * t2 + 0.25 * u2 * u2);
        const double S0 = e0 * e0, S1 = e1 * e1, S2 = e2 * e2;
        const double p12 = S1 * S2, p02 = S0 * S2, p01 = S0 * S1;
        const double q0 = 2.0 * s[0] - 7.0 * s[1] + 11.0 * s[2];
        const double q1 = -s[1] + 5.0 * s[2] + 2.0 * s[3];
        const double q2 = 2.0 * s[2] + 5.0 * s[3] - s[4];
        const double r0 = 2.0 * s[4] - 7.0 * s[3] + 11.0 * s[2];
        const double r1 = -s[3] + 5.0 * s[2] + 2.0 * s[1];
        const double r2 = 2.0 * s[2] + 5.0 * s[1] - s[0];
        const double ap0 = 0.1 * p12, ap1 = 0.6 * p02, ap2 = 0.3 * p01;
        const double am0 = 0.1 * p01, am1 = 0.6 * p02, am2 = 0.3 * p12;
        // fp = Np / Dp, Dp = 6 (ap0 + ap1 + ap2); fm likewise
        const double iDp = frcp(6.0 * (ap0 + ap1 + ap2)), iDm = frcp(6.0 * (am0 + am1 + am2));
        const double fp = (ap0 * q0 + ap1 * q1 + ap2 * q2) * iDp;
        const double fm = (am0 * r0 + am1 * r1 + am2 * r2) * iDm;
        const double bNp = bp * iDp, bDp6 = -6.0 * bp * fp * iDp;
        const double bNm = bm * iDm, bDm6 = -6.0 * bm * fm * iDm;
        // adjoints of the weights, then of the products of squared indicators
        const double bap0 = bNp * q0 + bDp6, bap1 = bNp * q1 + bDp6, bap2 = bNp * q2 + bDp6;
        const double bam0 = bNm * r0 + bDm6, bam1 = bNm * r1 + bDm6, bam2 = bNm * r2 + bDm6;
        const double bp12 = 0.1 * bap0 + 0.3 * bam2, bp02 = 0.6 * (bap1 + bam1), bp01 = 0.3 * bap2 + 0.1 * bam0;
        const double bS0 = bp02 * S2 + bp01 * S1, bS1 = bp12 * S2 + bp01 * S0, bS2 = bp12 * S1 + bp02 * S0;
        const double be0 = 2.0 * e0 * bS0, be1 = 2.0 * e1 * bS1, be2 = 2.0 * e2 * bS2;
        const double bt0 = 2.0 * c13 * t0 * be0, bu0 = 0.5 * u0 * be0;
        const double bt1 = 2.0 * c13 * t1 * be1, bu1 = 0.5 * u1 * be1;
        const double bt2 = 2.0 * c13 * t2 * be2, bu2 = 0.5 * u2 * be2;
        const double bq0 = bNp * ap0, bq1 = bNp * ap1, bq2 = bNp * ap2;
        const double br0 = bNm * am0, br1 = bNm * am1, br2 = bNm * am2;
        g[0] = bt0 + bu0 + 2.0 * bq0 - br2;
        g[1] = -2.0 * bt0 - 4.0 * bu0 + bt1 + bu1 - 7.0 * bq0 - bq1 + 2.0 * br1 + 5.0 * br2;
        g[2] = bt0 + 3.0 * bu0 - 2.0 * bt1 + bt2 + 3.0 * bu2 + 11.0 * bq0 + 5.0 * bq1 + 2.0 * bq2 + 11.0 * br0 +
               5.0 * br1 + 2.0 * br2;
        g[3] = bt1 - bu1 - 2.0 * bt2 - 4.0 * bu2 + 2.0 * bq1 + 5.0 * bq2 - 7.0 * br0 - br1;
        g[4] = bt2 + bu2 - bq2 + 2.0 * br0;
    } else {
        // fm = s2 - sl/2, fp = s2 + sl/2, sl = limiter(dm, dp), dm = s2 - s1, dp = s3 - s2
        const double dm = s[2] - s[1], dp = s[3] - s[2];
        double gdm = 0.0, gdp = 0.0;                      // d sl / d dm, d sl / d dp
        if constexpr (RECON == REC_MINMOD) {
            if (!(dm * dp <= 0.0)) {
                if (fabs(dm) < fabs(dp)) gdm = 1.0; else gdp = 1.0;
            }
        } else {   // MC2: minmod(2 dm, 2 dp, (dm + dp)/2) as recon takes it
            if (!(dm * dp <= 0.0)) {
                const double c = 0.5 * (dm + dp);
                const double a = 2.0 * dm, b = 2.0 * dp;
                int pick;                                 // 0: 2 dm, 1: 2 dp, 2: c
                if (c > 0.0) {
                    const int inner = a <= b ? 0 : 1;
                    pick = (inner == 0 ? a : b) <= c ? inner : 2;
                } else {
                    const int inner = a >= b ? 0 : 1;
                    pick = (inner == 0 ? a : b) >= c ? inner : 2;
                }
                if (pick == 0) gdm = 2.0;
                else if (pick == 1) gdp = 2.0;
                else { gdm = 0.5; gdp = 0.5; }
            }
        }
        const double h = 0.5 * (bp - bm);
        g[0] = 0.0;
        g[1] = -h * gdm;
        g[2] = (bm + bp) + h * (gdm - gdp);
        g[3] = h * gdp;
        g[4] = 0.0;
    }
}

// ---------------------------------------------------------------- recovery
// 3-direction dual number: value and derivatives with respect to (v^x, v^y,
// v^z), the velocity columns of the recovery Jacobian in one pass
struct D3 {
    double v, d[3];
};
__device__ __forceinline__ D3 operator+(const D3& a, const D3& b) {
    return D3{a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1], a.d[2] + b.d[2]}};
}
__device__ __forceinline__ D3 operator-(const D3& a, const D3& b) {
    return D3{a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1], a.d[2] - b.d[2]}};
}
__device__ __forceinline__ D3 operator*(const D3& a, const D3& b) {
    return D3{a.v * b.v, {fma(a.d[0], b.v, a.v * b.d[0]), fma(a.d[1], b.v, a.v * b.d[1]),
                          fma(a.d[2], b.v, a.v * b.d[2])}};
}
__device__ __forceinline__ D3 operator*(double a, const D3& b) { return D3{a * b.v, {a * b.d[0], a * b.d[1], a * b.d[2]}}; }
__device__ __forceinline__ D3 operator*(const D3& b, double a) { return a * b; }
__device__ __forceinline__ D3 operator+(const D3& a, double b) { return D3{a.v + b, {a.d[0], a.d[1], a.d[2]}}; }
__device__ __forceinline__ D3 operator+(double b, const D3& a) { return a + b; }
__device__ __forceinline__ D3 operator-(const D3& a, double b) { return D3{a.v - b, {a.d[0], a.d[1], a.d[2]}}; }
__device__ __forceinline__ D3 operator-(double b, const D3& a) { return D3{b - a.v, {-a.d[0], -a.d[1], -a.d[2]}}; }
__device__ __forceinline__ D3 inv(const D3& a) {
    const double r = frcp(a.v), r2 = -r * r;
    return D3{r, {a.d[0] * r2, a.d[1] * r2, a.d[2] * r2}};
}
__device__ __forceinline__ D3 rsq(const D3& a) {
    const double r = frsqrt(a.v), h = -0.5 * r * r * r;
    return D3{r, {a.d[0] * h, a.d[1] * h, a.d[2] * h}};
}
__device__ __forceinline__ double val(const D3& x) { return x.v; }
__device__ __forceinline__ double rsq(double a) { return frsqrt(a); }
__device__ __forceinline__ double inv(double a) { return frcp(a); }
__device__ __forceinline__ double val(double x) { return x; }

// one-direction dual number (value, derivative): Jacobian columns one at a
// time keep 2 doubles per intermediate instead of 5; also the scalar type of
// the tangent passes of the adjoint
struct D1 {
    double v, d;
    D1() = default;
    __host__ __device__ constexpr explicit D1(double x) : v(x), d(0.0) {}
    __host__ __device__ constexpr D1(double x, double dx) : v(x), d(dx) {}
};
__device__ __forceinline__ D1 operator+(const D1& a, const D1& b) { return D1{a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ D1 operator-(const D1& a, const D1& b) { return D1{a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ D1 operator*(const D1& a, const D1& b) { return D1{a.v * b.v, fma(a.d, b.v, a.v * b.d)}; }
__device__ __forceinline__ D1 operator*(double a, const D1& b) { return D1{a * b.v, a * b.d}; }
__device__ __forceinline__ D1 operator*(const D1& b, double a) { return D1{a * b.v, a * b.d}; }
__device__ __forceinline__ D1 operator+(const D1& a, double b) { return D1{a.v + b, a.d}; }
__device__ __forceinline__ D1 operator+(double b, const D1& a) { return D1{a.v + b, a.d}; }
__device__ __forceinline__ D1 operator-(const D1& a, double b) { return D1{a.v - b, a.d}; }
__device__ __forceinline__ D1 operator-(double b, const D1& a) { return D1{b - a.v, -a.d}; }
__device__ __forceinline__ D1 operator-(const D1& a) { return D1{-a.v, -a.d}; }
__device__ __forceinline__ D1& operator+=(D1& a, const D1& b) { a = a + b; return a; }
__device__ __forceinline__ D1& operator-=(D1& a, const D1& b) { a = a - b; return a; }
__device__ __forceinline__ D1& operator*=(D1& a, const D1& b) { a = a * b; return a; }
__device__ __forceinline__ D1 inv(const D1& a) {
    const double r = frcp(a.v);
    return D1{r, -a.d * r * r};
}
__device__ __forceinline__ D1 rsq(const D1& a) {
    const double r = frsqrt(a.v);
    return D1{r, -0.5 * a.d * r * r * r};
}
__device__ __forceinline__ D1 frcp(const D1& a) { return inv(a); }
__device__ __forceinline__ D1 frsqrt(const D1& a) { return rsq(a); }
__device__ __forceinline__ D1 operator/(const D1& a, const D1& b) { return a * inv(b); }
__device__ __forceinline__ D1 operator/(double a, const D1& b) { return a * inv(b); }
__device__ __forceinline__ D1 operator/(const D1& a, double b) { return a * (1.0 / b); }
__device__ __forceinline__ double val(const D1& x) { return x.v; }
__device__ __forceinline__ bool operator<(const D1& a, const D1& b) { return a.v < b.v; }
__device__ __forceinline__ bool operator>(const D1& a, const D1& b) { return a.v > b.v; }
__device__ __forceinline__ bool operator<=(const D1& a, const D1& b) { return a.v <= b.v; }
__device__ __forceinline__ bool operator>=(const D1& a, const D1& b) { return a.v >= b.v; }
__device__ __forceinline__ D1 fabs(const D1& a) { return a.v < 0.0 ? -a : a; }
__device__ __forceinline__ D1 fmin(const D1& a, const D1& b) { return a.v <= b.v ? a : b; }
__device__ __forceinline__ D1 fmax(const D1& a, const D1& b) { return a.v >= b.v ? a : b; }

// inputs of one recovery (T = double, or a dual type when the adjoint
// differentiates the recovered state with respect to them)
template <class T, bool DG = false> struct RecInT {
    static constexpr bool diag = DG;                 // a diagonal 3-metric (zero entries skipped)
    double G;
    T D, tau, S[3], Bc[3], Bl[3], Es[3], cfac;   // cfac = a dt alpha sigma; Bl = lowered B / sqrt(gamma)
    T iD;                                        // 1 / D
    double sg, isg, g[6], gi[6];
};
using RecIn = RecInT<double>;

// Residual of the recovery map at x = (p, v): r0 = (Gamma-1) rho eps - p,
// r_i = v'^i - v^i, where E solves the implicit stage equation at v
// (closed form of eq. 3D_NR), v' is the velocity of Sec. III.B step (iii) at
// (E, p), and rho, eps follow it.  Returns false if unphysical.  With S =
// double and drdp given, also the column dr/dp: at fixed v the field E and
// the electromagnetic energy do not depend on p, so the column follows from
// the chain den -> w -> W' -> (rho, eps) by hand.
template <class S, class K>
__device__ __forceinline__ bool rec_residual(const K& k, const S* x, S* r, S* Eout, double* drdp = nullptr) {
    const S p = x[0];
    const S v[3] = {x[1], x[2], x[3]};
    S vl[3];
    for (int i = 0; i < 3; ++i) {
        if constexpr (K::diag) vl[i] = k.g[sidx(i, i)] * v[i];
        else vl[i] = k.g[sidx(i, 0)] * v[0] + k.g[sidx(i, 1)] * v[1] + k.g[sidx(i, 2)] * v[2];
    }
    const S v2 = vl[0] * v[0] + vl[1] * v[1] + vl[2] * v[2];
    if (!(val(v2) < 1.0) || !(val(p) > 0.0)) return false;
    const S W = rsq(1.0 - v2);
    const S c = k.cfac * W;
    // b = E* - c (v_l x B_l); (1 + c) E - c (v_l . E) v = b
    S b[3];
    b[0] = k.Es[0] - c * (vl[1] * k.Bl[2] - vl[2] * k.Bl[1]);
    b[1] = k.Es[1] - c * (vl[2] * k.Bl[0] - vl[0] * k.Bl[2]);
    b[2] = k.Es[2] - c * (vl[0] * k.Bl[1] - vl[1] * k.Bl[0]);
    // both denominators from one reciprocal
    const S a1 = 1.0 + c * (1.0 - v2);
    const S a2 = 1.0 + c;
    const S ia = inv(a1 * a2);
    const S vE = (vl[0] * b[0] + vl[1] * b[1] + vl[2] * b[2]) * (a2 * ia);
    const S i1c = a1 * ia;
    S E[3];
    for (int i = 0; i < 3; ++i) E[i] = (b[i] + c * vE * v[i]) * i1c;
    S El[3];
    for (int i = 0; i < 3; ++i) {
        if constexpr (K::diag) El[i] = k.g[sidx(i, i)] * E[i];
        else El[i] = k.g[sidx(i, 0)] * E[0] + k.g[sidx(i, 1)] * E[1] + k.g[sidx(i, 2)] * E[2];
    }
    const S em = (El[0] * E[0] + El[1] * E[1] + El[2] * E[2] +
                  (k.Bl[0] * k.Bc[0] + k.Bl[1] * k.Bc[1] + k.Bl[2] * k.Bc[2]) * k.sg) * (0.5 * k.isg);
    const S den = k.tau + k.D + k.sg * p - em;
    const S iden = inv(den);
    S wl[3];
    wl[0] = (k.S[0] - (E[1] * k.Bc[2] - E[2] * k.Bc[1])) * iden;
    wl[1] = (k.S[1] - (E[2] * k.Bc[0] - E[0] * k.Bc[2])) * iden;
    wl[2] = (k.S[2] - (E[0] * k.Bc[1] - E[1] * k.Bc[0])) * iden;
    S w[3];
    for (int i = 0; i < 3; ++i) {
        if constexpr (K::diag) w[i] = k.gi[sidx(i, i)] * wl[i];
        else w[i] = k.gi[sidx(i, 0)] * wl[0] + k.gi[sidx(i, 1)] * wl[1] + k.gi[sidx(i, 2)] * wl[2];
    }
    const S w2 = wl[0] * w[0] + wl[1] * w[1] + wl[2] * w[2];
    if (!(val(w2) < 1.0)) return false;
    const S omw = 1.0 - w2;
    const S Wn = rsq(omw);
    const S iW = omw * Wn;                       // 1 / W'
    const S Wn2 = Wn * Wn;
    const S rho = k.D * k.isg * iW;
    const S num = k.tau - k.D * (Wn - 1.0) - k.sg * p * (Wn2 - 1.0) - em;
    const S eps = num * (iW * k.iD);
    r[0] = (k.G - 1.0) * rho * eps - p;
    for (int i = 0; i < 3; ++i) r[1 + i] = w[i] - v[i];
    if (Eout)
        for (int i = 0; i < 3; ++i) Eout[i] = E[i];
    if constexpr (std::is_same<S, double>::value) {
        if (drdp) {
            // d(den)/dp = sqrt(gamma): every w_i and w2 scale with 1/den
            const double s = k.sg * iden;
            const double w2p = -2.0 * s * w2;
            const double Wnp = 0.5 * Wn * Wn2 * w2p;
            const double iWp = -Wnp * iW * iW;
            const double rhop = k.D * k.isg * iWp;
            const double nump = -k.D * Wnp - k.sg * (Wn2 - 1.0) - 2.0 * k.sg * p * Wn * Wnp;
            const double epsp = (nump * iW + num * iWp) * k.iD;
            drdp[0] = (k.G - 1.0) * (rhop * eps + rho * epsp) - 1.0;
            for (int i = 0; i < 3; ++i) drdp[1 + i] = -s * w[i];
        }
    }
    return isfinite(val(r[0])) && isfinite(val(r[1])) && isfinite(val(r[2])) && isfinite(val(r[3]));
}

__device__ __forceinline__ double rec_merit(const double* r, double p) {
    const double a = r[0] / p;
    return a * a + r[1] * r[1] + r[2] * r[2] + r[3] * r[3];
}

// LU factorisation of a 4x4 matrix with partial pivoting, in place
__device__ __forceinline__ bool lu4(double A[4][4], int* piv) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        int pv = c;
        double best = fabs(A[c][c]);
#pragma unroll
        for (int r = c + 1; r < 4; ++r)
            if (fabs(A[r][c]) > best) { best = fabs(A[r][c]); pv = r; }
        piv[c] = pv;
        if (best == 0.0) return false;
        if (pv != c) {
#pragma unroll
            for (int k = 0; k < 4; ++k) { const double t = A[c][k]; A[c][k] = A[pv][k]; A[pv][k] = t; }
        }
        const double ic = 1.0 / A[c][c];
        A[c][c] = ic;                              // keep the reciprocal pivot
#pragma unroll
        for (int r = c + 1; r < 4; ++r) {
            const double f = A[r][c] * ic;
            A[r][c] = f;
#pragma unroll
            for (int k = c + 1; k < 4; ++k) A[r][k] -= f * A[c][k];
        }
    }
    return true;
}
// solve with the factors of lu4: the factorisation swaps whole rows, so the
// complete permutation is applied to b before the forward substitution
__device__ __forceinline__ void lu4_solve(const double A[4][4], const int* piv, double* b) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
        if (piv[c] != c) { const double t = b[c]; b[c] = b[piv[c]]; b[piv[c]] = t; }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int r = c + 1; r < 4; ++r) b[r] -= A[r][c] * b[c];
    }
#pragma unroll
    for (int r = 3; r >= 0; --r) {
        double t = b[r];
#pragma unroll
        for (int k = r + 1; k < 4; ++k) t -= A[r][k] * b[k];
        b[r] = t * A[r][r];
    }
}

// inverse of a 4x4 matrix by its adjugate over the determinant (Laplace
// expansion in the 2x2 minors of rows 0-1 and rows 2-3): no pivot search, so
// no data-dependent register indexing; false if the determinant is 0 or not
// finite.  (The forward recovery only needs an approximate inverse for its
// chord steps; the adjoint keeps the pivoted LU.)
__device__ __forceinline__ bool inv4(const double A[4][4], double X[4][4]) {
    const double s0 = A[0][0] * A[1][1] - A[1][0] * A[0][1];
    const double s1 = A[0][0] * A[1][2] - A[1][0] * A[0][2];
    const double s2 = A[0][0] * A[1][3] - A[1][0] * A[0][3];
    const double s3 = A[0][1] * A[1][2] - A[1][1] * A[0][2];
    const double s4 = A[0][1] * A[1][3] - A[1][1] * A[0][3];
    const double s5 = A[0][2] * A[1][3] - A[1][2] * A[0][3];
    const double c5 = A[2][2] * A[3][3] - A[3][2] * A[2][3];
    const double c4 = A[2][1] * A[3][3] - A[3][1] * A[2][3];
    const double c3 = A[2][1] * A[3][2] - A[3][1] * A[2][2];
    const double c2 = A[2][0] * A[3][3] - A[3][0] * A[2][3];
    const double c1 = A[2][0] * A[3][2] - A[3][0] * A[2][2];
    const double c0 = A[2][0] * A[3][1] - A[3][0] * A[2][1];
    const double det = s0 * c5 - s1 * c4 + s2 * c3 + s3 * c2 - s4 * c1 + s5 * c0;
    if (!(fabs(det) > 0.0) || !isfinite(det)) return false;
    const double id = 1.0 / det;
    X[0][0] = (A[1][1] * c5 - A[1][2] * c4 + A[1][3] * c3) * id;
    X[0][1] = (-A[0][1] * c5 + A[0][2] * c4 - A[0][3] * c3) * id;
    X[0][2] = (A[3][1] * s5 - A[3][2] * s4 + A[3][3] * s3) * id;
    X[0][3] = (-A[2][1] * s5 + A[2][2] * s4 - A[2][3] * s3) * id;
    X[1][0] = (-A[1][0] * c5 + A[1][2] * c2 - A[1][3] * c1) * id;
    X[1][1] = (A[0][0] * c5 - A[0][2] * c2 + A[0][3] * c1) * id;
    X[1][2] = (-A[3][0] * s5 + A[3][2] * s2 - A[3][3] * s1) * id;
    X[1][3] = (A[2][0] * s5 - A[2][2] * s2 + A[2][3] * s1) * id;
    X[2][0] = (A[1][0] * c4 - A[1][1] * c2 + A[1][3] * c0) * id;
    X[2][1] = (-A[0][0] * c4 + A[0][1] * c2 - A[0][3] * c0) * id;
    X[2][2] = (A[3][0] * s4 - A[3][1] * s2 + A[3][3] * s0) * id;
    X[2][3] = (-A[2][0] * s4 + A[2][1] * s2 - A[2][3] * s0) * id;
    X[3][0] = (-A[1][0] * c3 + A[1][1] * c1 - A[1][2] * c0) * id;
    X[3][1] = (A[0][0] * c3 - A[0][1] * c1 + A[0][2] * c0) * id;
    X[3][2] = (-A[3][0] * s3 + A[3][1] * s1 - A[3][2] * s0) * id;
    X[3][3] = (A[2][0] * s3 - A[2][1] * s1 + A[2][2] * s0) * id;
    return true;
}

enum : int { ST_OK = 0, ST_WARN = 1, ST_NOCONV = -3, ST_UNPHYS = -4 };

// residual r and the inverse Ji of the exact Jacobian at x (the p column by
// hand, the v columns by one 3-direction dual pass): JAC_OK, or JAC_UNPHYS (x
// outside the physical domain), or JAC_SINGULAR
enum { JAC_OK = 0, JAC_UNPHYS = 1, JAC_SINGULAR = 2 };
template <bool DG>
__device__ __forceinline__ int rec_jacobian(const RecInT<double, DG>& k, const double* x, double Ji[4][4], double* r) {
    double J[4][4];
    double c0[4];
    if (!rec_residual<double>(k, x, r, (double*)nullptr, c0)) return JAC_UNPHYS;
#pragma unroll
    for (int a = 0; a < 4; ++a) J[a][0] = c0[a];
    D3 xd[4], rd[4];
    xd[0] = D3{x[0], {0.0, 0.0, 0.0}};
    xd[1] = D3{x[1], {1.0, 0.0, 0.0}};
    xd[2] = D3{x[2], {0.0, 1.0, 0.0}};
    xd[3] = D3{x[3], {0.0, 0.0, 1.0}};
    if (!rec_residual<D3>(k, xd, rd, (D3*)nullptr)) return JAC_UNPHYS;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) J[a][1 + b] = rd[a].d[b];
    return inv4(J, Ji) ? JAC_OK : JAC_SINGULAR;
}

// Stiff coupled solve: the root of the recovery map r(p, v) (the fixed point
// the paper's iteration converges to where it converges), by Newton's method
// with the exact Jacobian, kept between iterations while the steps contract
// fast (chord steps) and refreshed otherwise; backtracking keeps the state
// physical and the residual decreasing.  x in/out: guess -> (p, v^i);
// E out: densitised E at the root.  tolq = 0.0075 tol (the early stop).
template <bool DG>
__device__ int recover_stiff(const RecInT<double, DG>& k, double* x, double* E, double tol, double tolq, int maxit,
                             int* iters) {
    if (!(k.D > 0.0) || !isfinite(k.tau) || !(x[0] > 0.0)) { *iters = 0; return ST_UNPHYS; }
    double r[4], Ji[4][4];
    int it = 0, restart = 0;
    bool need = true, fresh = false, have_prev = false;
    // (flags and inline constants rather than a 1e300 sentinel: the compiler
    // keeps such a literal in two registers across the whole kernel)
    double last_rel = 1.0, prev_step = 0.0;
    // one call site each for the Jacobian and the residual keeps the code of
    // the stage kernels within the instruction cache
    for (;;) {
        if (need) {
            const int jst = rec_jacobian(k, x, Ji, r);
            if (jst == JAC_UNPHYS && it == 0 && restart < 64) {
                // guess outside the physical domain: restart at rest, then
                // double the pressure until the state is physical
                if (restart == 0) x[1] = x[2] = x[3] = 0.0;
                else x[0] *= 2.0;
                ++restart;
                continue;
            }
            if (jst != JAC_OK) { *iters = it; return (jst == JAC_UNPHYS && it == 0) ? ST_UNPHYS : ST_NOCONV; }
            need = false;
            fresh = true;
        }
        if (++it > maxit) break;
        double dx[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) dx[a] = -(Ji[a][0] * r[0] + Ji[a][1] * r[1] + Ji[a][2] * r[2] + Ji[a][3] * r[3]);
        const double m0 = rec_merit(r, x[0]);
        double t = 1.0, xt[4], rt[4];
        bool acc = false;
        for (int ls = 0; ls < 40; ++ls) {
#pragma unroll
            for (int a = 0; a < 4; ++a) xt[a] = x[a] + t * dx[a];
            if (rec_residual<double>(k, xt, rt, E)) {
                double smax = fabs(t * dx[0]) / fabs(xt[0]);
                for (int a = 1; a < 4; ++a) smax = fmax(smax, fabs(t * dx[a]));
                if (rec_merit(rt, xt[0]) <= m0 || smax <= tol) { acc = true; break; }
            }
            t *= 0.5;
        }
        if (!acc) {
            // a chord step that does not descend: refresh the Jacobian once
            if (fresh) { *iters = it; return ST_NOCONV; }
            need = true;
            continue;
        }
        const double dp = fabs(xt[0] - x[0]);
        const double dv = fmax(fabs(xt[1] - x[1]), fmax(fabs(xt[2] - x[2]), fabs(xt[3] - x[3])));
#pragma unroll
        for (int a = 0; a < 4; ++a) { x[a] = xt[a]; r[a] = rt[a]; }
        last_rel = dp / x[0];
        if (dp <= tol * x[0] && dv <= tol) { *iters = it; return ST_OK; }
        const double step = fmax(last_rel, dv);
        // a full step that contracted by q < 1/4 leaves an error of at most
        // about q step / (1 - q): once that is below tol / 100 the next step
        // would only confirm convergence, so stop here
        if (t == 1.0 && have_prev && step <= 0.25 * prev_step && step * step <= tolq * prev_step) {
            *iters = it;
            return ST_OK;
        }
        if (t < 1.0 || (have_prev && step > 0.25 * prev_step)) need = true;
        else fresh = false;
        prev_step = step;
        have_prev = isfinite(step);
    }
    *iters = maxit;
    return last_rel <= 1e-12 ? ST_WARN : ST_NOCONV;
}

// Plain recovery with E fixed (Sec. III.B): the velocity follows from p
// alone, and p is updated by the Newton step with f' = v^2 c_s^2 - 1,
// c_s^2 = Gamma (Gamma-1) eps / (1 + Gamma eps).  x in/out = (p, v).
template <bool DG>
__device__ int recover_plain(const RecInT<double, DG>& k, const double* Ec, double* x, double tol, int maxit,
                             int* iters) {
    if (!(k.D > 0.0) || !isfinite(k.tau) || !(x[0] > 0.0)) { *iters = 0; return ST_UNPHYS; }
    double El[3];
    if constexpr (DG) {
        for (int i = 0; i < 3; ++i) El[i] = k.g[sidx(i, i)] * Ec[i];
    } else {
        lower(k.g, Ec, El);
    }
    const double em = (dot3(El, Ec) + dot3(k.Bl, k.Bc) * k.sg) * (0.5 * k.isg);
    const double base = k.tau + k.D - em;
    double sm[3] = {k.S[0] - (Ec[1] * k.Bc[2] - Ec[2] * k.Bc[1]), k.S[1] - (Ec[2] * k.Bc[0] - Ec[0] * k.Bc[2]),
                    k.S[2] - (Ec[0] * k.Bc[1] - Ec[1] * k.Bc[0])};
    double smu[3];
    for (int i = 0; i < 3; ++i) {
        if constexpr (DG) smu[i] = k.gi[sidx(i, i)] * sm[i];
        else smu[i] = k.gi[sidx(i, 0)] * sm[0] + k.gi[sidx(i, 1)] * sm[1] + k.gi[sidx(i, 2)] * sm[2];
    }
    const double s2 = dot3(sm, smu);
    double p = x[0];
    double last_rel = 1.0;                       // (set by every iteration)
    const double G = k.G;
    const double iD = 1.0 / k.D;
    for (int it = 1; it <= maxit; ++it) {
        const double den = base + k.sg * p;
        if (!(den > 0.0)) { *iters = it; return ST_UNPHYS; }
        const double iden = frcp(den);
        const double w2 = s2 * iden * iden;
        if (!(w2 < 1.0) || !isfinite(w2)) { *iters = it; return ST_UNPHYS; }
        const double Wn = frsqrt(1.0 - w2);
        const double Wn2 = Wn * Wn;
        const double iW = frcp(Wn);
        const double rho = k.D * k.isg * iW;
        const double eps = (k.tau - k.D * (Wn - 1.0) - k.sg * p * (Wn2 - 1.0) - em) * (iW * iD);
        const double f = (G - 1.0) * rho * eps - p;
        const double cs2 = G * (G - 1.0) * eps / (1.0 + G * eps);
        const double pn = p - f / (w2 * cs2 - 1.0);
        if (!(pn > 0.0) || !isfinite(pn)) { *iters = it; return ST_UNPHYS; }
        double dv = 0.0;
        for (int i = 0; i < 3; ++i) {
            const double w = smu[i] * iden;
            dv = fmax(dv, fabs(w - x[1 + i]));
            x[1 + i] = w;
        }
        const double dp = fabs(pn - p);
        p = pn;
        x[0] = p;
        last_rel = dp / p;
        if (dp <= tol * p && dv <= tol) { *iters = it; return ST_OK; }
    }
    *iters = maxit;
    return last_rel <= 1e-12 ? ST_WARN : ST_NOCONV;
}

}  // namespace rmhd
