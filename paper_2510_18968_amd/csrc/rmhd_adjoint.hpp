// Adjoint of one IMEX-SSP2(2,2,2) step (reverse mode, FP64).
//
// The step maps U^n (and sigma) to U^{n+1}; the primitives only seed the
// recoveries, whose roots do not depend on the guess, so the adjoint state is
// Ubar alone.  Reverse sweep (eq. IMEX3 read backwards):
//   final update   U^{n+1} = (U^n + U(2))/2 + dt/2 L(P(2)) + dt/2 (2 g R1 + (1-g) R2)_E
//   L(P(2))        flux divergence + sources, adjoint as a deterministic gather
//   stage 2        pointwise map (Y, E*, sigma) -> (U(2), P(2), R2) through the
//                  recovery root, differentiated with the implicit-function
//                  theorem: xbar = dOmega/dx, J^T lambda = xbar,
//                  thetabar = dOmega/dtheta - (dr/dtheta)^T lambda
//   L(P(1))        as above
//   stage 1        the same pointwise map on (U^n, E^n, sigma)
// Local Jacobian-vector products come from one-direction dual numbers (D1)
// through the same device functions the forward kernels use.
#pragma once
#include "rmhd_kernels.hpp"

namespace rmhd {

// ------------------------------------------------------------------ helpers
template <class M, class R> __device__ __forceinline__ void geo_zero_seed(const Geo<M>& a, Geo<M>& b) { b = a; }

// metric of a cell centre without the lapse / shift (for the current)
template <bool CURVED> __device__ __forceinline__ void cell_geo_g(const Params& p, long o, Geo<double>& m) {
    if (CURVED) {
        m.alp = 1.0;
        m.bet[0] = m.bet[1] = m.bet[2] = 0.0;
        for (int a = 0; a < 6; ++a) m.g[a] = p.gam[a * p.Np + o];
        geo_finish(m);
    } else {
        geo_flat(m);
    }
}

__global__ void k_fill(double* a, long n, double v) {
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) a[t] = v;
}

// -------------------------------------------------------- final update (reverse)
// Ub1 and Ubn may be the same array (in-place adjoint): no __restrict__ on them
__global__ __launch_bounds__(256) void k_adj_final(const Params p, double dt, const double* Ub1,
                                                   double* Ubn, double* __restrict__ Ub2,
                                                   double* __restrict__ Lb, double* __restrict__ R1b,
                                                   double* __restrict__ R2b) {
    long o;
    if (!interior_cell(p, (long)blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    const long Np = p.Np;
    const double g = GAM_IMEX();
    double u[NF];
    for (int f = 0; f < NF; ++f) u[f] = Ub1[f * Np + o];
    for (int f = 0; f < NF; ++f) {
        Ubn[f * Np + o] = 0.5 * u[f];
        Ub2[f * Np + o] = 0.5 * u[f];
        Lb[f * Np + o] = 0.5 * dt * u[f];
    }
    for (int i = 0; i < 3; ++i) {
        R1b[i * Np + o] = g * dt * u[I_E + i];
        R2b[i * Np + o] = 0.5 * dt * (1.0 - g) * u[I_E + i];
    }
}

// ------------------------------------------------ sources (pointwise, reverse)
// Pb_c += (dS/dP_c)^T Lb_c at interior cells
template <bool CURVED>
__global__ __launch_bounds__(256) void k_adj_sources(const Params p, const double* __restrict__ P,
                                                     const double* __restrict__ Lb, double* __restrict__ Pb) {
    long o;
    if (!interior_cell(p, (long)blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    const long Np = p.Np;
    Geo<double> m;
    cell_geo<CURVED>(p, o, m);
    MetricDerivs md;
    metric_derivs<CURVED>(p, o, md);
    double Pc[NF], lb[NF];
    for (int f = 0; f < NF; ++f) {
        Pc[f] = P[f * Np + o];
        lb[f] = Lb[f * Np + o];
    }
    for (int a = 0; a < NF; ++a) {
        D1 Pd[NF], Ud[NF], Sd[NF];
        for (int f = 0; f < NF; ++f) Pd[f] = D1(Pc[f], f == a ? 1.0 : 0.0);
        prim2con(m, D1(p.G), Pd, Ud);
        sources_t<CURVED, D1>(p, m, md, Pd, Ud, Sd);
        double acc = 0.0;
        for (int f = 0; f < NF; ++f) acc += lb[f] * Sd[f].d;
        Pb[a * Np + o] += acc;
    }
}

// ---------------------------------------------------- face pass (reverse)
// Per face of direction D (indexed by its left cell): Fbar = (Lb_R - Lb_L)/dx,
// then the sensitivities of the face flux to the two reconstructed face
// states (PLb, PRb) and to the face current (Jb); flags mark first-order
// fallback states.  fb layout: [0..13] PLb, [14..27] PRb, [28] Jb, [29] flags.
template <int D, int RECON, bool CURVED>
__global__ __launch_bounds__(128) void k_adj_face(const Params p, const double* __restrict__ P,
                                                  const double* __restrict__ sig, const double* __restrict__ Lb,
                                                  double* __restrict__ fb) {
    constexpr int E1 = (D == 0) ? 1 : 0, E2 = (D == 2) ? 1 : 2;
    const long nD = p.n[D] + 1, n1 = p.n[E1], n2 = p.n[E2];
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    // consecutive threads along x
    long c, a1, a2;
    if (D == 0) {
        if (t >= nD * n1 * n2) return;
        c = t % nD; t /= nD; a1 = t % n1; a2 = t / n1;
    } else {
        if (t >= nD * n1 * n2) return;
        a1 = t % n1; t /= n1; c = t % nD; a2 = t / nD;
    }
    const long s = p.st[D];
    const long cl = c + p.g[D] - 1;   // padded index of the left cell along D
    const long o = (a1 + p.g[E1]) * p.st[E1] + (a2 + p.g[E2]) * p.st[E2] + cl * s;   // left cell
    const long Np = p.Np;
    const double ih = p.idx[D];
    // Fbar: L_i holds -F_{i+1/2}/dx and L_{i+1} holds +F_{i+1/2}/dx
    const bool inL = cl >= p.g[D] && cl < p.g[D] + p.n[D];
    const bool inR = cl + 1 >= p.g[D] && cl + 1 < p.g[D] + p.n[D];
    double Fb[NF];
    for (int f = 0; f < NF; ++f)
        Fb[f] = ((inR ? Lb[f * Np + o + s] : 0.0) - (inL ? Lb[f * Np + o] : 0.0)) * ih;
    // recompute the face states
    double PL[NF], PR[NF], Pl[NF], Pr[NF];
    for (int f = 0; f < NF; ++f) {
        const double* a = P + f * Np + o;
        const double sl[5] = {a[-2 * s], a[-s], a[0], a[s], a[2 * s]};
        const double sr[5] = {a[-s], a[0], a[s], a[2 * s], a[3 * s]};
        double dm;
        recon<RECON>(sl, dm, PL[f]);
        recon<RECON>(sr, PR[f], dm);
        Pl[f] = sl[2];
        Pr[f] = sr[2];
    }
    Geo<double> m;
    if (CURVED) face_geo(p, o, s, m); else geo_flat(m);
    int flags = 0;
    if (bad_state(m, PL)) { for (int f = 0; f < NF; ++f) PL[f] = Pl[f]; flags |= 1; }
    if (bad_state(m, PR)) { for (int f = 0; f < NF; ++f) PR[f] = Pr[f]; flags |= 2; }
    double lp, lm;
    speeds<D>(p, m, lp, lm);
    const double id = frcp(lp - lm);
    const double cL = lp * id, cR = -lm * id, cU = lp * lm * id;
    // Fh = cL F(PL) - cU U(PL) + cR F(PR) + cU U(PR); the face current enters
    // only the charge flux (F_Q = alpha J - beta Q), its adjoint is fb[28]
    for (int side = 0; side < 2; ++side) {
        const double* Ps = side ? PR : PL;
        const double cF = side ? cR : cL, cS = side ? cU : -cU;
        double wF[NF], wU[NF], Pb[NF];
        for (int f = 0; f < NF; ++f) {
            wF[f] = Fb[f] * cF;
            wU[f] = Fb[f] * cS;
        }
        state_flux_vjp<D>(m, p.G, Ps, wF, wU, Pb);
        for (int a = 0; a < NF; ++a) fb[(side * NF + a) * Np + o] = Pb[a];
    }
    fb[28 * Np + o] = m.alp * Fb[I_Q];
    fb[29 * Np + o] = (double)flags;
}

// ---------------------------------------------------- cell pass (reverse)
// Per cell along D over the padded range: gather from the faces whose
// reconstruction stencils or currents use this cell.  Pb += ..., sb += ...
template <int D, int RECON, bool CURVED>
__global__ __launch_bounds__(128) void k_adj_cell(const Params p, const double* __restrict__ P,
                                                  const double* __restrict__ sig, const double* __restrict__ fb,
                                                  double* __restrict__ Pb, double* __restrict__ sb) {
    constexpr int E1 = (D == 0) ? 1 : 0, E2 = (D == 2) ? 1 : 2;
    const long nD = p.np[D], n1 = p.n[E1], n2 = p.n[E2];
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long c, a1, a2;
    if (D == 0) {
        if (t >= nD * n1 * n2) return;
        c = t % nD; t /= nD; a1 = t % n1; a2 = t / n1;
    } else {
        if (t >= nD * n1 * n2) return;
        a1 = t % n1; t /= n1; c = t % nD; a2 = t / nD;
    }
    const long s = p.st[D];
    const long Np = p.Np;
    const long base = (a1 + p.g[E1]) * p.st[E1] + (a2 + p.g[E2]) * p.st[E2];
    const long o = base + c * s;
    const long gD = p.g[D], lastD = p.g[D] + p.n[D];   // faces: left cells gD-1 .. lastD-1
    double acc[NF];
    for (int f = 0; f < NF; ++f) acc[f] = 0.0;
    // reconstruction of the cells m = c + k whose stencils contain c
    for (int k = -2; k <= 2; ++k) {
        const long mcell = c + k;
        if (mcell < gD - 1 || mcell > lastD) continue;              // not reconstructed
        const long om = base + mcell * s;
        const bool hasR = mcell >= gD;                              // face mcell-1/2 (left cell mcell-1)
        const bool hasL = mcell <= lastD - 1;                       // face mcell+1/2 (left cell mcell)
        const int flR = hasR ? (int)fb[29 * Np + om - s] : 0;
        const int flL = hasL ? (int)fb[29 * Np + om] : 0;
        const bool useR = hasR && !(flR & 2);
        const bool useL = hasL && !(flL & 1);
        if (!useR && !useL) continue;
        const int q = 2 - k;                                        // position of c in m's stencil
        for (int f = 0; f < NF; ++f) {
            const double bm = useR ? fb[(NF + f) * Np + om - s] : 0.0;
            const double bp = useL ? fb[f * Np + om] : 0.0;
            if (bm == 0.0 && bp == 0.0) continue;
            const double* a = P + f * Np + om;
            D1 st[5];
            for (int r = 0; r < 5; ++r) st[r] = D1(a[(r - 2) * s], r == q ? 1.0 : 0.0);
            D1 fm, fp;
            recon<RECON>(st, fm, fp);
            acc[f] += bm * fm.d + bp * fp.d;
        }
    }
    // first-order fallback states are the cell values themselves
    if (c >= gD - 1 && c <= lastD - 1 && ((int)fb[29 * Np + o] & 1))
        for (int f = 0; f < NF; ++f) acc[f] += fb[f * Np + o];
    if (c >= gD && c <= lastD && ((int)fb[29 * Np + o - s] & 2))
        for (int f = 0; f < NF; ++f) acc[f] += fb[(NF + f) * Np + o - s];
    // cell-centre current: J_face = (J_left + J_right)/2
    double sgb = 0.0;
    if (c >= gD - 1 && c <= lastD) {
        double Jb = 0.0;
        if (c >= gD) Jb += 0.5 * fb[28 * Np + o - s];
        if (c <= lastD - 1) Jb += 0.5 * fb[28 * Np + o];
        if (Jb != 0.0) {
            Geo<double> mc;
            cell_geo_g<CURVED>(p, o, mc);
            double Pc[NF];
            for (int f = 0; f < NF; ++f) Pc[f] = P[f * Np + o];
            const long os = o + (long)(bc_map(p, D, (int)c) - c) * s;
            const double sg = sig[os];
            // the current depends on v, B, E, q and sigma
            const int dep[10] = {I_V, I_V + 1, I_V + 2, I_B, I_B + 1, I_B + 2, I_E, I_E + 1, I_E + 2, I_Q};
            for (int a = 0; a < 10; ++a) {
                D1 Pd[NF], J[3];
                for (int f = 0; f < NF; ++f) Pd[f] = D1(Pc[f], f == dep[a] ? 1.0 : 0.0);
                current(mc, Pd, D1(sg), J);
                acc[dep[a]] += Jb * J[D].d;
            }
            D1 Pd[NF], J[3];
            for (int f = 0; f < NF; ++f) Pd[f] = D1(Pc[f]);
            current(mc, Pd, D1(sg, 1.0), J);
            sgb = Jb * J[D].d;
        }
    }
    for (int f = 0; f < NF; ++f)
        if (acc[f] != 0.0) Pb[f * Np + o] += acc[f];
    if (sgb != 0.0) sb[o] += sgb;
}

// x direction, one lane per position of the sequence of rows with their
// ghost cells (as the forward x sweep): a lane forms the whole gradient of its
// own cell's reconstruction (recon_vjp, one reverse sweep) and cell c gathers
// the components of the reconstructions c-2 .. c+2 from the neighbouring
// lanes; 60 of a wave's 64 lanes gather.  The fallback and current parts are
// those of k_adj_cell.
constexpr int TSEGA = 60;
template <int RECON, bool CURVED>
__global__ __launch_bounds__(128) void k_adj_cell_x(const Params p, const double* __restrict__ P,
                                                    const double* __restrict__ sig, const double* __restrict__ fb,
                                                    double* __restrict__ Pb, double* __restrict__ sb, long nitems) {
    const int lane = threadIdx.x & 63;
    const long w = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w >= nitems) return;                                     // uniform per wave
    const int n0 = p.n[0], gD = p.g[0];
    const int W0 = n0 + 6;
    const int V = W0 * p.n[1] * p.n[2];
    const int v = (int)w * TSEGA - 2 + lane;
    const int vc = v < 0 ? 0 : (v < V ? v : V - 1);
    const unsigned r = (unsigned)vc / (unsigned)W0;
    const int x = vc - (int)r * W0 - 3;                          // interior x: -3 .. n0 + 2
    const unsigned j = r % (unsigned)p.n[1], k = r / (unsigned)p.n[1];
    const long rowo = ((long)k + p.g[2]) * p.st[2] + ((long)j + p.g[1]) * p.st[1];
    const long Np = p.Np;
    const long o = rowo + gD + x;
    const bool gather = lane >= 2 && lane < 2 + TSEGA && v == vc;
    // the lane's cell m = c as a reconstruction: faces m - 1/2 (x >= 0) and m + 1/2 (x <= n0 - 1)
    const bool isrec = x >= -1 && x <= n0;
    const long oL = x >= 0 ? o - 1 : o;                          // left cell of face m - 1/2 (in range)
    const int flR = x >= 0 ? (int)fb[29 * Np + oL] : 0;
    const int flL = x <= n0 - 1 ? (int)fb[29 * Np + o] : 0;
    const bool useR = isrec && x >= 0 && !(flR & 2);
    const bool useL = isrec && x <= n0 - 1 && !(flL & 1);
    double acc[NF];
#pragma unroll 2
    for (int f = 0; f < NF; ++f) {
        double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (useR || useL) {
            const double bm = useR ? fb[(NF + f) * Np + oL] : 0.0;
            const double bp = useL ? fb[f * Np + o] : 0.0;
            const double* a = P + f * Np + o;
            const double st[5] = {a[-2], a[-1], a[0], a[1], a[2]};
            recon_vjp<RECON>(st, bm, bp, g);
        }
        // cell c: g of c + 2 at 0, c + 1 at 1, c at 2, c - 1 at 3, c - 2 at 4
        acc[f] = g[2] + (down<1>(g[1]) + down<2>(g[0])) + (up<1>(g[3]) + up<2>(g[4]));
    }
    if (!gather) return;
    const long cpad = gD + x, lastD = gD + n0;
    // first-order fallback states are the cell values themselves
    if (cpad >= gD - 1 && cpad <= lastD - 1 && (flL & 1))
        for (int f = 0; f < NF; ++f) acc[f] += fb[f * Np + o];
    if (cpad >= gD && cpad <= lastD && (flR & 2))
        for (int f = 0; f < NF; ++f) acc[f] += fb[(NF + f) * Np + oL];
    // cell-centre current: J_face = (J_left + J_right)/2
    double sgb = 0.0;
    if (cpad >= gD - 1 && cpad <= lastD) {
        double Jb = 0.0;
        if (cpad >= gD) Jb += 0.5 * fb[28 * Np + oL];
        if (cpad <= lastD - 1) Jb += 0.5 * fb[28 * Np + o];
        if (Jb != 0.0) {
            Geo<double> mc;
            cell_geo_g<CURVED>(p, o, mc);
            double Pc[NF];
            for (int f = 0; f < NF; ++f) Pc[f] = P[f * Np + o];
            const long os = o + (long)(bc_map(p, 0, (int)cpad) - cpad);
            const double sg = sig[os];
            const int dep[10] = {I_V, I_V + 1, I_V + 2, I_B, I_B + 1, I_B + 2, I_E, I_E + 1, I_E + 2, I_Q};
            for (int a = 0; a < 10; ++a) {
                D1 Pd[NF], J[3];
                for (int f = 0; f < NF; ++f) Pd[f] = D1(Pc[f], f == dep[a] ? 1.0 : 0.0);
                current(mc, Pd, D1(sg), J);
                acc[dep[a]] += Jb * J[0].d;
            }
            D1 Pd[NF], J[3];
            for (int f = 0; f < NF; ++f) Pd[f] = D1(Pc[f]);
            current(mc, Pd, D1(sg, 1.0), J);
            sgb = Jb * J[0].d;
        }
    }
    for (int f = 0; f < NF; ++f)
        if (acc[f] != 0.0) Pb[f * Np + o] += acc[f];
    if (sgb != 0.0) sb[o] += sgb;
}

// --------------------------------------------------- ghost fill (reverse)
// the ghost cells along d are copies of interior cells: add their adjoints to
// the images and clear them (one thread owns one image row, deterministic);
// the nf fields of a and then the one field of b
// (one thread per image row, side and field; the layers of one row fold in
// order, as the copies of a copy boundary share their image)
__global__ void k_adj_fold(const Params p, double* __restrict__ a, int nf, double* __restrict__ b1, int d) {
    const int e1 = (d == 0) ? 1 : 0, e2 = (d == 2) ? 1 : 2;
    const long n1 = p.n[e1], n2 = p.n[e2];
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2L * n1 * n2 * (nf + 1)) return;
    const int f = (int)(t / (2L * n1 * n2));
    t -= (long)f * 2L * n1 * n2;
    const int side = (int)(t % 2);
    t /= 2;
    const long a1 = t % n1 + p.g[e1], a2 = t / n1 + p.g[e2];
    const long ob = a1 * p.st[e1] + a2 * p.st[e2];
    const int g = p.g[d], n = p.n[d];
    {
        double* b = (f < nf ? a + f * p.Np : b1) + ob;
        for (int l = 0; l < p.ng; ++l) {
            const int c = side ? n + g + l : g - p.ng + l;
            const int src = bc_map(p, d, c);
            const double v = b[(long)c * p.st[d]];
            b[(long)c * p.st[d]] = 0.0;
            b[(long)src * p.st[d]] += v;
        }
    }
}

// ------------------------------------------------ pointwise stage (reverse)
// Omega = Pb . P(x, theta) + UbE . E(x, theta) + Rb . (E - E*)/(gamma dt);
// theta = (D, S_1..3, tau, Bcal^1..3, Phi, Psi, Q, E*_1..3, sigma)
constexpr int NTH = 15;

template <class S>
__device__ __forceinline__ bool stage_omega(const Params& p, const Geo<double>& m, double gdt, const S* th,
                                            const S* x, const double* Pb, const double* UbE, const double* Rb,
                                            S& Om, S* r) {
    RecInT<S> k;
    k.G = p.G;
    k.D = th[0];
    k.iD = inv(k.D);
    k.S[0] = th[1]; k.S[1] = th[2]; k.S[2] = th[3];
    k.tau = th[4];
    for (int i = 0; i < 3; ++i) {
        k.Bc[i] = th[5 + i];
        k.Es[i] = th[11 + i];
    }
    for (int a = 0; a < 6; ++a) { k.g[a] = m.g[a]; k.gi[a] = m.gi[a]; }
    k.sg = m.sg;
    k.isg = m.isg;
    lower(m.g, k.Bc, k.Bl);
    for (int i = 0; i < 3; ++i) k.Bl[i] = k.Bl[i] * m.isg;
    k.cfac = th[14] * (gdt * m.alp);
    S E[3];
    if (!rec_residual<S>(k, x, r, E)) return false;
    const S* v = x + 1;
    S vl[3];
    lower(m.g, v, vl);
    const S W = rsq(1.0 - dot3(vl, v));
    S Pv[NF];
    Pv[I_RHO] = k.D * m.isg * inv(W);
    Pv[I_P] = x[0];
    for (int i = 0; i < 3; ++i) {
        Pv[I_V + i] = v[i];
        Pv[I_B + i] = k.Bc[i] * m.isg;
        Pv[I_E + i] = E[i] * m.isg;
    }
    Pv[I_PHI] = th[8] * m.isg;
    Pv[I_PSI] = th[9] * m.isg;
    Pv[I_Q] = th[10] * m.isg;
    S o = S(0.0);
    for (int f = 0; f < NF; ++f) o += Pv[f] * Pb[f];
    for (int i = 0; i < 3; ++i) o += E[i] * (UbE[i] + Rb[i] / gdt) - k.Es[i] * (Rb[i] / gdt);
    Om = o;
    return true;
}

// STAGE 2: theta from (U(2) non-E rows, E* = U(2)_E - gamma dt R2), x = P(2);
//          adjoint in (Ub2, Pb, R2b); writes Ubn += Ybar, Lb = dt Ybar, R1b += ..., sb +=
// STAGE 1: theta from (U^n non-E rows, E* = U^n_E), x = P(1); adjoint in (Pb, R1b);
//          writes Ubn += thetabar, sb +=
template <int STAGE, bool CURVED>
__global__ __launch_bounds__(128) void k_adj_point(const Params p, double dt, const double* __restrict__ sig,
                                                   const double* __restrict__ Us, const double* __restrict__ Rs,
                                                   const double* __restrict__ Ps, const double* __restrict__ Ubs,
                                                   const double* __restrict__ Pb, const double* __restrict__ Rb,
                                                   double* __restrict__ Ubn, double* __restrict__ Lb,
                                                   double* __restrict__ R1b, double* __restrict__ sb,
                                                   unsigned long long* __restrict__ nfail) {
    long o;
    if (!interior_cell(p, (long)blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    const long Np = p.Np;
    const double g = GAM_IMEX();
    const double gdt = g * dt;
    Geo<double> m;
    cell_geo<CURVED>(p, o, m);
    double th[NTH], x[4], pb[NF], ubE[3] = {0.0, 0.0, 0.0}, rb[3];
    const int rows[11] = {0, 1, 2, 3, 4, 5, 6, 7, 11, 12, 13};
    for (int a = 0; a < 11; ++a) th[a] = Us[rows[a] * Np + o];
    for (int i = 0; i < 3; ++i)
        th[11 + i] = (STAGE == 2) ? Us[(I_E + i) * Np + o] - gdt * Rs[i * Np + o] : Us[(I_E + i) * Np + o];
    th[14] = sig[o];
    x[0] = Ps[I_P * Np + o];
    for (int i = 0; i < 3; ++i) x[1 + i] = Ps[(I_V + i) * Np + o];
    for (int f = 0; f < NF; ++f) pb[f] = Pb[f * Np + o];
    if (STAGE == 2)
        for (int i = 0; i < 3; ++i) ubE[i] = Ubs[(I_E + i) * Np + o];
    for (int i = 0; i < 3; ++i) rb[i] = Rb[i * Np + o];
    // xbar and the Jacobian of the residual at the root
    double J[4][4], xb[4];
    for (int b = 0; b < 4; ++b) {
        D1 xd[4], thd[NTH], rd[4], Om;
        for (int a = 0; a < 4; ++a) xd[a] = D1(x[a], a == b ? 1.0 : 0.0);
        for (int a = 0; a < NTH; ++a) thd[a] = D1(th[a]);
        stage_omega<D1>(p, m, gdt, thd, xd, pb, ubE, rb, Om, rd);
        xb[b] = Om.d;
        for (int a = 0; a < 4; ++a) J[b][a] = rd[a].d;   // transposed: J^T[b][a] = dr_a/dx_b
    }
    int piv[4];
    double lam[4] = {xb[0], xb[1], xb[2], xb[3]};
    if (lu4(J, piv)) {
        lu4_solve(J, piv, lam);
    } else {
        // a singular Jacobian at the root has no implicit-function derivative:
        // the cell is counted as failed (rmhd_failures), its lambda set to zero
        lam[0] = lam[1] = lam[2] = lam[3] = 0.0;
        atomicAdd(nfail, 1ull);
    }
    double thb[NTH];
    for (int b = 0; b < NTH; ++b) {
        D1 xd[4], thd[NTH], rd[4], Om;
        for (int a = 0; a < 4; ++a) xd[a] = D1(x[a]);
        for (int a = 0; a < NTH; ++a) thd[a] = D1(th[a], a == b ? 1.0 : 0.0);
        stage_omega<D1>(p, m, gdt, thd, xd, pb, ubE, rb, Om, rd);
        thb[b] = Om.d - (lam[0] * rd[0].d + lam[1] * rd[1].d + lam[2] * rd[2].d + lam[3] * rd[3].d);
    }
    // theta = (non-E rows, E*, sigma)
    double Yb[NF];
    for (int a = 0; a < 11; ++a) Yb[rows[a]] = thb[a];
    for (int i = 0; i < 3; ++i) Yb[I_E + i] = thb[11 + i];
    if (STAGE == 2) {
        // U(2) non-E rows are Y itself
        for (int a = 0; a < 11; ++a) Yb[rows[a]] += Ubs[rows[a] * Np + o];
        // Y = U^n + dt L1; E* = U^n_E + dt L1_E + dt (1 - 2 gamma) R1
        for (int f = 0; f < NF; ++f) {
            Ubn[f * Np + o] += Yb[f];
            Lb[f * Np + o] = dt * Yb[f];
        }
        for (int i = 0; i < 3; ++i) R1b[i * Np + o] += dt * (1.0 - 2.0 * g) * Yb[I_E + i];
    } else {
        for (int f = 0; f < NF; ++f) Ubn[f * Np + o] += Yb[f];
    }
    sb[o] += thb[14];
    // a non-finite sensitivity (from this cell or carried in by Pb, e.g. at a
    // state so close to the light cone that its derivatives overflow) is
    // counted with the failures, never passed on silently
    bool finite = isfinite(thb[14]);
    for (int f = 0; f < NF; ++f) finite = finite && isfinite(Yb[f]);
    if (!finite) atomicAdd(nfail, 1ull);
}

__global__ __launch_bounds__(256) void k_adj_sigma_out(const Params p, const double* __restrict__ sb,
                                                       double* __restrict__ out) {
    long o;
    if (!interior_cell(p, (long)blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    out[o] += sb[o];
}

// ------------------------------------------------ prim2con (reverse)
// Pb_c = (dU/dP_c)^T Ub_c at interior cells
template <bool CURVED>
__global__ __launch_bounds__(256) void k_adj_prim2con(const Params p, const double* __restrict__ P,
                                                      const double* __restrict__ Ub, double* __restrict__ Pb) {
    long o;
    if (!interior_cell(p, (long)blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    const long Np = p.Np;
    Geo<double> m;
    cell_geo<CURVED>(p, o, m);
    double Pc[NF], ub[NF];
    for (int f = 0; f < NF; ++f) {
        Pc[f] = P[f * Np + o];
        ub[f] = Ub[f * Np + o];
    }
    for (int a = 0; a < NF; ++a) {
        D1 Pd[NF], Ud[NF];
        for (int f = 0; f < NF; ++f) Pd[f] = D1(Pc[f], f == a ? 1.0 : 0.0);
        prim2con(m, D1(p.G), Pd, Ud);
        double acc = 0.0;
        for (int f = 0; f < NF; ++f) acc += ub[f] * Ud[f].d;
        Pb[a * Np + o] = acc;
    }
}

}  // namespace rmhd
