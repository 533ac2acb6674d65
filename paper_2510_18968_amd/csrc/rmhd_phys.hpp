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

namespace rmhd {

using ::sqrt;

constexpr int NF = 14;
enum : int { I_RHO = 0, I_P = 1, I_V = 2, I_B = 5, I_E = 8, I_PHI = 11, I_PSI = 12, I_Q = 13 };
enum : int { I_D = 0, I_S = 1, I_TAU = 4 };
enum : int { REC_MINMOD = 0, REC_MC2 = 1, REC_WENO5 = 2 };

// symmetric 3x3 packed as xx, xy, xz, yy, yz, zz
__host__ __device__ constexpr int sidx(int i, int j) {
    return (i == j) ? (i == 0 ? 0 : (i == 1 ? 3 : 5)) : ((i + j == 1) ? 1 : ((i + j == 2) ? 2 : 4));
}

// 3-metric at one point with the quantities derived from it (Sec. II.A)
template <class R> struct Geo {
    R alp, bet[3], g[6], gi[6], sg, isg;
};

template <class R> __device__ __forceinline__ void geo_flat(Geo<R>& m) {
    m.alp = R(1);
    m.bet[0] = m.bet[1] = m.bet[2] = R(0);
    m.g[0] = m.g[3] = m.g[5] = R(1);
    m.g[1] = m.g[2] = m.g[4] = R(0);
    for (int a = 0; a < 6; ++a) m.gi[a] = m.g[a];
    m.sg = m.isg = R(1);
}

// inverse by cofactors and sqrt(det); m.g already set
template <class R> __device__ __forceinline__ void geo_finish(Geo<R>& m) {
    const R gxx = m.g[0], gxy = m.g[1], gxz = m.g[2], gyy = m.g[3], gyz = m.g[4], gzz = m.g[5];
    const R cxx = gyy * gzz - gyz * gyz;
    const R cxy = gxz * gyz - gxy * gzz;
    const R cxz = gxy * gyz - gxz * gyy;
    const R det = gxx * cxx + gxy * cxy + gxz * cxz;
    const R id = R(1) / det;
    m.gi[0] = cxx * id;
    m.gi[1] = cxy * id;
    m.gi[2] = cxz * id;
    m.gi[3] = (gxx * gzz - gxz * gxz) * id;
    m.gi[4] = (gxy * gxz - gxx * gyz) * id;
    m.gi[5] = (gxx * gyy - gxy * gxy) * id;
    m.sg = sqrt(det);
    m.isg = R(1) / m.sg;
}

template <class R> __device__ __forceinline__ void lower(const R* g, const R* u, R* l) {
    l[0] = g[0] * u[0] + g[1] * u[1] + g[2] * u[2];
    l[1] = g[1] * u[0] + g[3] * u[1] + g[4] * u[2];
    l[2] = g[2] * u[0] + g[4] * u[1] + g[5] * u[2];
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
template <class R> __device__ __forceinline__ void prim2con(const Geo<R>& m, R G, const R* P, R* U) {
    const R* v = P + I_V;
    const R* B = P + I_B;
    const R* E = P + I_E;
    R vl[3], Bl[3], El[3], c[3];
    lower(m.g, v, vl);
    lower(m.g, B, Bl);
    lower(m.g, E, El);
    const R W2 = R(1) / (R(1) - dot3(vl, v));
    const R W = sqrt(W2);
    const R hW2 = (P[I_RHO] + G / (G - R(1)) * P[I_P]) * W2;
    const R em = R(0.5) * (dot3(El, E) + dot3(Bl, B));
    cross(E, B, c);   // eta_ijk E^j B^k; epsilon_ijk = sqrt(gamma) eta_ijk
    const R D = m.sg * P[I_RHO] * W;
    U[I_D] = D;
    for (int i = 0; i < 3; ++i) U[I_S + i] = m.sg * (hW2 * vl[i] + m.sg * c[i]);
    U[I_TAU] = m.sg * (hW2 - P[I_P] + em) - D;
    for (int a = I_B; a < NF; ++a) U[a] = m.sg * P[a];
}

// densitised current of eq. Ohm_law at a point:
// J^i = Q v^i + W sigma [Ecal^i + (v_l x B_l)^i - (v_l . Ecal) v^i]
template <class R> __device__ __forceinline__ void current(const Geo<R>& m, const R* P, R sigma, R* J) {
    const R* v = P + I_V;
    R vl[3], Bl[3], vb[3];
    lower(m.g, v, vl);
    lower(m.g, P + I_B, Bl);
    cross(vl, Bl, vb);
    const R W = R(1) / sqrt(R(1) - dot3(vl, v));
    const R Ec[3] = {m.sg * P[I_E], m.sg * P[I_E + 1], m.sg * P[I_E + 2]};
    const R vE = dot3(vl, Ec);
    const R Q = m.sg * P[I_Q];
    for (int i = 0; i < 3; ++i) J[i] = Q * v[i] + W * sigma * (Ec[i] + vb[i] - vE * v[i]);
}

// physical flux along D (eq. GRRMHD_flux_form, sqrt(gamma) once); Jd is the
// current carried by the charge flux at this face
template <int D, class R>
__device__ __forceinline__ void phys_flux(const Geo<R>& m, R G, const R* P, const R* U, R Jd, R* F) {
    const R* v = P + I_V;
    const R* B = P + I_B;
    const R* E = P + I_E;
    R vl[3], Bl[3], El[3];
    lower(m.g, v, vl);
    lower(m.g, B, Bl);
    lower(m.g, E, El);
    const R W2 = R(1) / (R(1) - dot3(vl, v));
    const R hW2 = (P[I_RHO] + G / (G - R(1)) * P[I_P]) * W2;
    const R pt = P[I_P] + R(0.5) * (dot3(El, E) + dot3(Bl, B));
    const R a = m.alp, bd = m.bet[D], as = m.alp * m.sg;
    const R vd = v[D], Ed = E[D], Bd = B[D];
    F[I_D] = (a * vd - bd) * U[I_D];
    for (int i = 0; i < 3; ++i)
        F[I_S + i] = as * (hW2 * vd * vl[i] - Ed * El[i] - Bd * Bl[i] + (i == D ? pt : R(0))) - bd * U[I_S + i];
    const R Sd = m.gi[sidx(D, 0)] * U[I_S] + m.gi[sidx(D, 1)] * U[I_S + 1] + m.gi[sidx(D, 2)] * U[I_S + 2];
    F[I_TAU] = a * (Sd - vd * U[I_D]) - bd * U[I_TAU];
    // (e_D x X)^i for covariant X
    R eE[3], eB[3];
    if (D == 0) { eE[0] = R(0); eE[1] = -El[2]; eE[2] = El[1]; eB[0] = R(0); eB[1] = -Bl[2]; eB[2] = Bl[1]; }
    if (D == 1) { eE[0] = El[2]; eE[1] = R(0); eE[2] = -El[0]; eB[0] = Bl[2]; eB[1] = R(0); eB[2] = -Bl[0]; }
    if (D == 2) { eE[0] = -El[1]; eE[1] = El[0]; eE[2] = R(0); eB[0] = -Bl[1]; eB[1] = Bl[0]; eB[2] = R(0); }
    for (int i = 0; i < 3; ++i) {
        const R gid = m.gi[sidx(i, D)];
        F[I_B + i] = a * (eE[i] + gid * U[I_PHI]) - bd * U[I_B + i];
        F[I_E + i] = -a * (eB[i] - gid * U[I_PSI]) - bd * U[I_E + i];
    }
    F[I_PHI] = a * U[I_B + D] - bd * U[I_PHI];
    F[I_PSI] = a * U[I_E + D] - bd * U[I_PSI];
    F[I_Q] = a * Jd - bd * U[I_Q];
}

// ---------------------------------------------------------------- reconstruction
template <class R> __device__ __forceinline__ R mm2(R a, R b) {
    // minmod: 0 unless a, b share a sign, else the one of smaller magnitude
    return (a * b <= R(0)) ? R(0) : (fabs(a) < fabs(b) ? a : b);
}

// face values of the middle cell of s[0..4]: fm at i-1/2, fp at i+1/2
template <int RECON, class R> __device__ __forceinline__ void recon(const R* s, R& fm, R& fp) {
    if constexpr (RECON == REC_WENO5) {
        const R eps = R(1e-6);
        const R t0 = s[0] - R(2) * s[1] + s[2], u0 = s[0] - R(4) * s[1] + R(3) * s[2];
        const R t1 = s[1] - R(2) * s[2] + s[3], u1 = s[1] - s[3];
        const R t2 = s[2] - R(2) * s[3] + s[4], u2 = R(3) * s[2] - R(4) * s[3] + s[4];
        const R c13 = R(13) / R(12);
        const R b0 = c13 * t0 * t0 + R(0.25) * u0 * u0;
        const R b1 = c13 * t1 * t1 + R(0.25) * u1 * u1;
        const R b2 = c13 * t2 * t2 + R(0.25) * u2 * u2;
        const R e0 = eps + b0, e1 = eps + b1, e2 = eps + b2;
        const R w0 = R(1) / (e0 * e0), w1 = R(1) / (e1 * e1), w2 = R(1) / (e2 * e2);
        const R i6 = R(1) / R(6);
        // right face: stencils {i-2..i}, {i-1..i+1}, {i..i+2}, ideal weights 1/10, 6/10, 3/10
        {
            const R q0 = (R(2) * s[0] - R(7) * s[1] + R(11) * s[2]) * i6;
            const R q1 = (-s[1] + R(5) * s[2] + R(2) * s[3]) * i6;
            const R q2 = (R(2) * s[2] + R(5) * s[3] - s[4]) * i6;
            const R a0 = R(0.1) * w0, a1 = R(0.6) * w1, a2 = R(0.3) * w2;
            fp = (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
        }
        // left face: mirror image, same smoothness indicators
        {
            const R q0 = (R(2) * s[4] - R(7) * s[3] + R(11) * s[2]) * i6;
            const R q1 = (-s[3] + R(5) * s[2] + R(2) * s[1]) * i6;
            const R q2 = (R(2) * s[2] + R(5) * s[1] - s[0]) * i6;
            const R a0 = R(0.1) * w2, a1 = R(0.6) * w1, a2 = R(0.3) * w0;
            fm = (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
        }
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

// ---------------------------------------------------------------- recovery
// 4-direction dual number: value and derivatives w.r.t. (p, v^x, v^y, v^z)
struct D4 {
    double v, d[4];
};
__device__ __forceinline__ D4 mk(double v) { return D4{v, {0.0, 0.0, 0.0, 0.0}}; }
__device__ __forceinline__ D4 operator+(const D4& a, const D4& b) {
    return D4{a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1], a.d[2] + b.d[2], a.d[3] + b.d[3]}};
}
__device__ __forceinline__ D4 operator-(const D4& a, const D4& b) {
    return D4{a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1], a.d[2] - b.d[2], a.d[3] - b.d[3]}};
}
__device__ __forceinline__ D4 operator*(const D4& a, const D4& b) {
    return D4{a.v * b.v, {a.d[0] * b.v + a.v * b.d[0], a.d[1] * b.v + a.v * b.d[1], a.d[2] * b.v + a.v * b.d[2],
                          a.d[3] * b.v + a.v * b.d[3]}};
}
__device__ __forceinline__ D4 operator*(double a, const D4& b) {
    return D4{a * b.v, {a * b.d[0], a * b.d[1], a * b.d[2], a * b.d[3]}};
}
__device__ __forceinline__ D4 operator*(const D4& b, double a) { return a * b; }
__device__ __forceinline__ D4 operator+(const D4& a, double b) { return D4{a.v + b, {a.d[0], a.d[1], a.d[2], a.d[3]}}; }
__device__ __forceinline__ D4 operator+(double b, const D4& a) { return a + b; }
__device__ __forceinline__ D4 operator-(const D4& a, double b) { return D4{a.v - b, {a.d[0], a.d[1], a.d[2], a.d[3]}}; }
__device__ __forceinline__ D4 operator-(double b, const D4& a) {
    return D4{b - a.v, {-a.d[0], -a.d[1], -a.d[2], -a.d[3]}};
}
__device__ __forceinline__ D4 recip(const D4& a) {
    const double r = 1.0 / a.v, r2 = -r * r;
    return D4{r, {a.d[0] * r2, a.d[1] * r2, a.d[2] * r2, a.d[3] * r2}};
}
__device__ __forceinline__ D4 operator/(const D4& a, const D4& b) { return a * recip(b); }
__device__ __forceinline__ D4 operator/(const D4& a, double b) { return a * (1.0 / b); }
__device__ __forceinline__ D4 operator/(double a, const D4& b) { return a * recip(b); }
__device__ __forceinline__ D4 sqrt(const D4& a) {
    const double s = ::sqrt(a.v), h = 0.5 / s;
    return D4{s, {a.d[0] * h, a.d[1] * h, a.d[2] * h, a.d[3] * h}};
}
__device__ __forceinline__ double val(double x) { return x; }
__device__ __forceinline__ double val(const D4& x) { return x.v; }

// constant inputs of one recovery
struct RecIn {
    double G, D, tau, S[3], Bc[3], Bl[3], Es[3], cfac;   // cfac = a dt alpha sigma
    double sg, isg, g[6], gi[6];
    double ExBs[3];   // not used by the stiff residual
};

// Residual of the recovery map at x = (p, v): r0 = (Gamma-1) rho eps - p,
// r_i = v'^i - v^i, where E solves the implicit stage equation at v
// (closed form of eq. 3D_NR), v' is the velocity of Sec. III.B step (iii) at
// (E, p), and rho, eps follow it.  Returns false if unphysical.
template <class S>
__device__ __forceinline__ bool rec_residual(const RecIn& k, const S* x, S* r, double* Eout) {
    const S p = x[0];
    const S v[3] = {x[1], x[2], x[3]};
    S vl[3];
    for (int i = 0; i < 3; ++i) vl[i] = k.g[sidx(i, 0)] * v[0] + k.g[sidx(i, 1)] * v[1] + k.g[sidx(i, 2)] * v[2];
    const S v2 = vl[0] * v[0] + vl[1] * v[1] + vl[2] * v[2];
    if (!(val(v2) < 1.0) || !(val(p) > 0.0)) return false;
    const S W = 1.0 / sqrt(1.0 - v2);
    const S c = k.cfac * W;
    // b = E* - c (v_l x B_l); (1 + c) E - c (v_l . E) v = b
    S b[3];
    b[0] = k.Es[0] - c * (vl[1] * k.Bl[2] - vl[2] * k.Bl[1]);
    b[1] = k.Es[1] - c * (vl[2] * k.Bl[0] - vl[0] * k.Bl[2]);
    b[2] = k.Es[2] - c * (vl[0] * k.Bl[1] - vl[1] * k.Bl[0]);
    const S vE = (vl[0] * b[0] + vl[1] * b[1] + vl[2] * b[2]) / (1.0 + c * (1.0 - v2));
    const S i1c = 1.0 / (1.0 + c);
    S E[3];
    for (int i = 0; i < 3; ++i) E[i] = (b[i] + c * vE * v[i]) * i1c;
    S El[3];
    for (int i = 0; i < 3; ++i) El[i] = k.g[sidx(i, 0)] * E[0] + k.g[sidx(i, 1)] * E[1] + k.g[sidx(i, 2)] * E[2];
    const S em = (El[0] * E[0] + El[1] * E[1] + El[2] * E[2] +
                  (k.Bl[0] * k.Bc[0] + k.Bl[1] * k.Bc[1] + k.Bl[2] * k.Bc[2]) * k.sg) * (0.5 * k.isg);
    const S den = k.tau + k.D + k.sg * p - em;
    const S iden = 1.0 / den;
    S wl[3];
    wl[0] = (k.S[0] - (E[1] * k.Bc[2] - E[2] * k.Bc[1])) * iden;
    wl[1] = (k.S[1] - (E[2] * k.Bc[0] - E[0] * k.Bc[2])) * iden;
    wl[2] = (k.S[2] - (E[0] * k.Bc[1] - E[1] * k.Bc[0])) * iden;
    S w[3];
    for (int i = 0; i < 3; ++i) w[i] = k.gi[sidx(i, 0)] * wl[0] + k.gi[sidx(i, 1)] * wl[1] + k.gi[sidx(i, 2)] * wl[2];
    const S w2 = wl[0] * w[0] + wl[1] * w[1] + wl[2] * w[2];
    if (!(val(w2) < 1.0)) return false;
    const S Wn2 = 1.0 / (1.0 - w2);
    const S Wn = sqrt(Wn2);
    const S DW = k.D * Wn;
    const S rho = k.D * k.isg / Wn;
    const S eps = (k.tau - k.D * (Wn - 1.0) - k.sg * p * (Wn2 - 1.0) - em) / DW;
    r[0] = (k.G - 1.0) * rho * eps - p;
    for (int i = 0; i < 3; ++i) r[1 + i] = w[i] - v[i];
    if (Eout)
        for (int i = 0; i < 3; ++i) Eout[i] = val(E[i]);
    return isfinite(val(r[0])) && isfinite(val(r[1])) && isfinite(val(r[2])) && isfinite(val(r[3]));
}

__device__ __forceinline__ double rec_merit(const double* r, double p) {
    const double a = r[0] / p;
    return a * a + r[1] * r[1] + r[2] * r[2] + r[3] * r[3];
}

// 4x4 Gaussian elimination with partial pivoting, in place; false if singular
__device__ __forceinline__ bool solve4(double A[4][4], double* b) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        double best = fabs(A[c][c]);
#pragma unroll
        for (int r = c + 1; r < 4; ++r)
            if (fabs(A[r][c]) > best) { best = fabs(A[r][c]); piv = r; }
        if (best == 0.0) return false;
        if (piv != c) {
#pragma unroll
            for (int k = 0; k < 4; ++k) { double t = A[c][k]; A[c][k] = A[piv][k]; A[piv][k] = t; }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        const double ic = 1.0 / A[c][c];
#pragma unroll
        for (int r = c + 1; r < 4; ++r) {
            const double f = A[r][c] * ic;
#pragma unroll
            for (int k = c; k < 4; ++k) A[r][k] -= f * A[c][k];
            b[r] -= f * b[c];
        }
    }
#pragma unroll
    for (int r = 3; r >= 0; --r) {
        double s = b[r];
#pragma unroll
        for (int k = r + 1; k < 4; ++k) s -= A[r][k] * b[k];
        b[r] = s / A[r][r];
    }
    return true;
}

enum : int { ST_OK = 0, ST_WARN = 1, ST_NOCONV = -3, ST_UNPHYS = -4 };

// Stiff coupled solve: Newton with the exact Jacobian (dual numbers) on the
// recovery map; converges to the root the paper's iteration converges to
// and stays convergent where that iteration does not (B^2 > h W^2).
// x in/out: guess -> root (p, v^i); E out: densitised E at the root.
__device__ int recover_stiff(const RecIn& k, double* x, double* E, double tol, int maxit, int* iters) {
    double r[4];
    if (!(k.D > 0.0) || !isfinite(k.tau) || !(x[0] > 0.0)) { *iters = 0; return ST_UNPHYS; }
    if (!rec_residual<double>(k, x, r, nullptr)) {
        // outside the physical domain: restart at rest with a larger pressure
        x[1] = x[2] = x[3] = 0.0;
        bool ok = false;
        for (int i = 0; i < 64 && !ok; ++i) {
            ok = rec_residual<double>(k, x, r, nullptr);
            if (!ok) x[0] *= 2.0;
        }
        if (!ok) { *iters = 0; return ST_UNPHYS; }
    }
    double last_rel = 1e300;
    for (int it = 1; it <= maxit; ++it) {
        D4 xd[4], rd[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            xd[a] = mk(x[a]);
            xd[a].d[a] = 1.0;
        }
        if (!rec_residual<D4>(k, xd, rd, nullptr)) { *iters = it; return ST_UNPHYS; }
        double J[4][4], dx[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            dx[a] = -rd[a].v;
#pragma unroll
            for (int b = 0; b < 4; ++b) J[a][b] = rd[a].d[b];
        }
        if (!solve4(J, dx)) { *iters = it; return ST_NOCONV; }
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
        if (!acc) { *iters = it; return ST_NOCONV; }
        const double dp = fabs(xt[0] - x[0]);
        const double dv = fmax(fabs(xt[1] - x[1]), fmax(fabs(xt[2] - x[2]), fabs(xt[3] - x[3])));
#pragma unroll
        for (int a = 0; a < 4; ++a) { x[a] = xt[a]; r[a] = rt[a]; }
        last_rel = dp / x[0];
        if (dp <= tol * x[0] && dv <= tol) { *iters = it; return ST_OK; }
    }
    *iters = maxit;
    return last_rel <= 1e-12 ? ST_WARN : ST_NOCONV;
}

// Plain recovery with E fixed (Sec. III.B): the velocity follows from p
// alone, and p is updated by the Newton step with f' = v^2 c_s^2 - 1,
// c_s^2 = Gamma (Gamma-1) eps / (1 + Gamma eps).  x in/out = (p, v).
__device__ int recover_plain(const RecIn& k, const double* Ec, double* x, double tol, int maxit, int* iters) {
    if (!(k.D > 0.0) || !isfinite(k.tau) || !(x[0] > 0.0)) { *iters = 0; return ST_UNPHYS; }
    double El[3];
    lower(k.g, Ec, El);
    const double em = (dot3(El, Ec) + dot3(k.Bl, k.Bc) * k.sg) * (0.5 * k.isg);
    const double base = k.tau + k.D - em;
    double sm[3] = {k.S[0] - (Ec[1] * k.Bc[2] - Ec[2] * k.Bc[1]), k.S[1] - (Ec[2] * k.Bc[0] - Ec[0] * k.Bc[2]),
                    k.S[2] - (Ec[0] * k.Bc[1] - Ec[1] * k.Bc[0])};
    double smu[3];
    for (int i = 0; i < 3; ++i) smu[i] = k.gi[sidx(i, 0)] * sm[0] + k.gi[sidx(i, 1)] * sm[1] + k.gi[sidx(i, 2)] * sm[2];
    const double s2 = dot3(sm, smu);
    double p = x[0];
    double last_rel = 1e300;
    const double G = k.G;
    for (int it = 1; it <= maxit; ++it) {
        const double den = base + k.sg * p;
        const double iden = 1.0 / den;
        const double w2 = s2 * iden * iden;
        if (!(w2 < 1.0) || !isfinite(w2)) { *iters = it; return ST_UNPHYS; }
        const double Wn2 = 1.0 / (1.0 - w2);
        const double Wn = sqrt(Wn2);
        const double rho = k.D * k.isg / Wn;
        const double eps = (k.tau - k.D * (Wn - 1.0) - k.sg * p * (Wn2 - 1.0) - em) / (k.D * Wn);
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
