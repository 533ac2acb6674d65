// gfx950 kernels of the IMEX-SSP2(2,2,2) stage of resistive GRMHD.
//
// Data: float64 SoA over the padded grid (x fastest), one field per plane.
// The flux divergence is split by direction:
//   x: one wave64 per row segment of 62 cells; every lane reconstructs its
//      own cell to both faces (shared WENO smoothness indicators), the right
//      neighbour's left-face state and the left neighbour's face flux arrive
//      by cross-lane shuffles, so each face flux is computed once;
//   y, z: lanes run along x (coalesced loads) and each lane marches along the
//      flux direction, carrying the previous face state and flux in
//      registers.
// The pointwise kernels add the non-stiff sources, assemble the IMEX stage
// and run the stiff recovery, one cell per lane.
#pragma once
#include "rmhd_phys.hpp"

namespace rmhd {

struct Params {
    int n[3], g[3], np[3], active, bc[3], maxit, speed_mode;
    long st[3], Np;
    double dx[3], idx[3], G, kappa, tol;
    // metric (nullptr alp/gam: flat), beta/K may be nullptr
    const double* alp;
    const double* bet;
    const double* gam;
    const double* K;
};

__host__ __device__ __forceinline__ bool is_active(const Params& p, int d) { return (p.active >> d) & 1; }

// padded index along d of the interior cell that a ghost index maps to
__device__ __forceinline__ int bc_map(const Params& p, int d, int c) {
    const int g = p.g[d], n = p.n[d];
    if (c >= g && c < g + n) return c;
    if (p.bc[d] == 0) return c < g ? c + n : c - n;
    return c < g ? g : g + n - 1;
}

template <class R> __device__ __forceinline__ void load_geo(const Params& p, long o, Geo<R>& m) {
    m.alp = R(p.alp[o]);
    for (int a = 0; a < 3; ++a) m.bet[a] = p.bet ? R(p.bet[a * p.Np + o]) : R(0);
    for (int a = 0; a < 6; ++a) m.g[a] = R(p.gam[a * p.Np + o]);
    geo_finish(m);
}

// metric at the face between o and o + s (4th-order interpolation)
template <class R> __device__ __forceinline__ void face_geo(const Params& p, long o, long s, Geo<R>& m) {
    auto I4 = [&](const double* f) {
        return (-f[o - s] + 9.0 * f[o] + 9.0 * f[o + s] - f[o + 2 * s]) * 0.0625;
    };
    m.alp = R(I4(p.alp));
    for (int a = 0; a < 3; ++a) m.bet[a] = p.bet ? R(I4(p.bet + a * p.Np)) : R(0);
    for (int a = 0; a < 6; ++a) m.g[a] = R(I4(p.gam + a * p.Np));
    geo_finish(m);
}

template <int D, class R> __device__ __forceinline__ void speeds(const Params& p, const Geo<R>& m, R& lp, R& lm) {
    const R gdd = m.gi[sidx(D, D)];
    const R s = gdd * frsqrt(gdd);
    if (p.speed_mode == 0) {
        const R b = m.bet[D] * frcp(m.alp);
        lp = s - b;
        lm = -s - b;
    } else {
        lp = m.alp * s - m.bet[D];
        lm = -m.alp * s - m.bet[D];
    }
    lp = fmax(lp, R(0));
    lm = fmin(lm, R(0));
}

// a face state is unusable if rho <= 0, p <= 0 or v^2 >= 1
template <class R> __device__ __forceinline__ bool bad_state(const Geo<R>& m, const R* P) {
    R vl[3];
    lower(m.g, P + I_V, vl);
    const R v2 = dot3(vl, P + I_V);
    return !(P[I_RHO] > R(0)) || !(P[I_P] > R(0)) || !(v2 < R(1));
}

// HLLE flux of direction D at a face with metric m (Sec. III)
template <int D, class R>
__device__ __forceinline__ void face_flux(const Params& p, const Geo<R>& m, const R* PL, const R* PR, R Jd, R* Fh) {
    R lp, lm;
    speeds<D>(p, m, lp, lm);
    const R id = frcp(lp - lm);
    const R cL = lp * id, cR = -lm * id, cU = lp * lm * id;
    const R G = R(p.G);
    R U[NF], F[NF];
    state_flux<D>(m, G, PL, Jd, U, F);
#pragma unroll
    for (int a = 0; a < NF; ++a) Fh[a] = cL * F[a] - cU * U[a];
    __builtin_amdgcn_sched_barrier(0);
    state_flux<D>(m, G, PR, Jd, U, F);
#pragma unroll
    for (int a = 0; a < NF; ++a) Fh[a] += cR * F[a] + cU * U[a];
}

// Reconstruct the 14 fields of the cell at `o` along stride `s` to both faces.
// Loads are software-pipelined one field ahead and a scheduling barrier per
// field stops the compiler from hoisting all 70 stencil loads (which would
// need ~140 extra VGPRs and cut occupancy to one wave per SIMD).  The cell
// values are kept in FP64 for the cell-centre current.
template <int RECON, class R>
__device__ __forceinline__ void recon_cell14(const double* __restrict__ P, long Np, long o, long s, R* fm, R* fp,
                                             double* Pc) {
    double cur[5], nxt[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) cur[q] = P[o + (q - 2) * s];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        if (f + 1 < NF) {
#pragma unroll
            for (int q = 0; q < 5; ++q) nxt[q] = P[(f + 1) * Np + o + (q - 2) * s];
        }
        const R st[5] = {R(cur[0]), R(cur[1]), R(cur[2]), R(cur[3]), R(cur[4])};
        recon<RECON>(st, fm[f], fp[f]);
        Pc[f] = cur[2];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < 5; ++q) cur[q] = nxt[q];
    }
}

// ------------------------------------------------------------------ x fluxes
constexpr int XSEG = 62;

// R: arithmetic of reconstruction, HLLE and divergence (double, or float in
// the mixed-precision form); state and rhs stay double.
template <int RECON, bool CURVED, class R>
__global__ __launch_bounds__(256) void k_flux_x(const Params p, const double* __restrict__ P,
                                                const double* __restrict__ sig, double* __restrict__ rhs) {
    const int lane = threadIdx.x & 63;
    const long wid = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int nseg = (p.n[0] + XSEG - 1) / XSEG;
    const long nrows = (long)p.n[1] * p.n[2];
    if (wid >= nrows * nseg) return;
    const int seg = (int)(wid % nseg);
    const long row = wid / nseg;
    const int j = (int)(row % p.n[1]) + p.g[1];
    const int k = (int)(row / p.n[1]) + p.g[2];
    const int ilast = p.g[0] + p.n[0];                 // right ghost next to the last cell
    const int i = p.g[0] - 1 + seg * XSEG + lane;     // this lane's cell (padded index)
    const int ic = i <= ilast ? i : ilast;
    const long o = ((long)k * p.np[1] + j) * p.np[0] + ic;
    const long Np = p.Np;

    R fm[NF], fp[NF];
    double Pc[NF];
    recon_cell14<RECON>(P, Np, o, 1, fm, fp, Pc);
    // cell-centre current, x component (charge flux at faces = mean of the two
    // cells); FP64 in every form: sigma multiplies a near-cancelling bracket
    Geo<double> mc;
    if (CURVED) {
        mc.alp = 1.0;
        mc.bet[0] = mc.bet[1] = mc.bet[2] = 0.0;
        for (int a = 0; a < 6; ++a) mc.g[a] = p.gam[a * Np + o];
        geo_finish(mc);
    } else {
        geo_flat(mc);
    }
    const long os = o - ic + bc_map(p, 0, ic);
    double J[3];
    current(mc, Pc, sig[os], J);
    const double JR = __shfl_down(J[0], 1);
    R PR[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) PR[f] = __shfl_down(fm[f], 1);

    // face i + 1/2
    Geo<R> m;
    if (CURVED) face_geo(p, o, 1, m); else geo_flat(m);
    if (bad_state(m, fp))
        for (int f = 0; f < NF; ++f) fp[f] = R(P[f * Np + o]);
    if (bad_state(m, PR))
        for (int f = 0; f < NF; ++f) PR[f] = R(P[f * Np + o + 1]);
    R Fh[NF];
    face_flux<0>(p, m, fp, PR, R(0.5 * (J[0] + JR)), Fh);

    const bool cell = lane >= 1 && lane <= XSEG && i >= p.g[0] && i < ilast;
    const R ih = R(p.idx[0]);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const R Fl = __shfl_up(Fh[f], 1);
        if (cell) rhs[f * Np + o] = double(-(Fh[f] - Fl) * ih);
    }
}

// -------------------------------------------------------------- y / z fluxes
template <int D, int RECON, bool CURVED, class R>
__global__ __launch_bounds__(64) void k_flux_march(const Params p, const double* __restrict__ P,
                                                   const double* __restrict__ sig, double* __restrict__ rhs,
                                                   int seglen) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i >= p.n[0]) return;
    constexpr int E = (D == 1) ? 2 : 1;               // the other transverse dimension
    const int e = blockIdx.y + p.g[E];
    const int c0 = blockIdx.z * seglen;               // first cell (interior index) of the segment
    const int c1 = min(c0 + seglen, p.n[D]);
    const long s = p.st[D];
    const long Np = p.Np;
    const long base = (long)(i + p.g[0]) + (long)e * p.st[E];
    const R ih = R(p.idx[D]);

    R PLc[NF], Fprev[NF];
    double Jprev = 0.0;
#pragma unroll 1
    for (int c = c0 - 1; c <= c1; ++c) {
        const int cp = c + p.g[D];
        const long o = base + (long)cp * s;
        R fm[NF], fp[NF];
        double Pc[NF];
        recon_cell14<RECON>(P, Np, o, s, fm, fp, Pc);
        Geo<double> mc;
        if (CURVED) {
            mc.alp = 1.0;
            mc.bet[0] = mc.bet[1] = mc.bet[2] = 0.0;
            for (int a = 0; a < 6; ++a) mc.g[a] = p.gam[a * Np + o];
            geo_finish(mc);
        } else {
            geo_flat(mc);
        }
        const long os = o + (long)(bc_map(p, D, cp) - cp) * s;
        double J[3];
        current(mc, Pc, sig[os], J);
        if (c >= c0) {
            // face between c - 1 and c
            Geo<R> m;
            if (CURVED) face_geo(p, o - s, s, m); else geo_flat(m);
            if (bad_state(m, PLc))
                for (int f = 0; f < NF; ++f) PLc[f] = R(P[f * Np + o - s]);
            if (bad_state(m, fm))
                for (int f = 0; f < NF; ++f) fm[f] = R(P[f * Np + o]);
            R Fh[NF];
            face_flux<D>(p, m, PLc, fm, R(0.5 * (Jprev + J[D])), Fh);
            if (c > c0) {
                const long oc = o - s;
#pragma unroll
                for (int f = 0; f < NF; ++f) rhs[f * Np + oc] -= double((Fh[f] - Fprev[f]) * ih);
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) Fprev[f] = Fh[f];
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) PLc[f] = fp[f];
        Jprev = J[D];
    }
}

// ---------------------------------------------------------------- ghost fill
// faces only: ghost layers along each active d, interior extents elsewhere
__global__ void k_ghost(const Params p, double* __restrict__ a, int nf, int d) {
    const int e1 = (d == 0) ? 1 : 0, e2 = (d == 2) ? 1 : 2;
    const long n1 = p.n[e1], n2 = p.n[e2];
    const long tot = 2L * p.g[d] * n1 * n2;
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= tot) return;
    const int a1 = (int)(t % n1) + p.g[e1];
    t /= n1;
    const int a2 = (int)(t % n2) + p.g[e2];
    t /= n2;
    const int layer = (int)t;   // 0..2g-1
    const int c = layer < p.g[d] ? layer : p.n[d] + layer;
    const int src = bc_map(p, d, c);
    const long ob = (long)a1 * p.st[e1] + (long)a2 * p.st[e2];
    const long od = ob + (long)c * p.st[d], os = ob + (long)src * p.st[d];
    for (int f = 0; f < nf; ++f) a[f * p.Np + od] = a[f * p.Np + os];
}

// ------------------------------------------------------------- interior map
__device__ __forceinline__ bool interior_cell(const Params& p, long t, long& o) {
    const long n0 = p.n[0], n1 = p.n[1];
    if (t >= n0 * n1 * p.n[2]) return false;
    const int i = (int)(t % n0) + p.g[0];
    const int j = (int)((t / n0) % n1) + p.g[1];
    const int k = (int)(t / (n0 * n1)) + p.g[2];
    o = ((long)k * p.np[1] + j) * p.np[0] + i;
    return true;
}

template <bool CURVED> __device__ __forceinline__ void cell_geo(const Params& p, long o, Geo<double>& m) {
    if (CURVED) load_geo(p, o, m); else geo_flat(m);
}

template <bool CURVED>
__global__ __launch_bounds__(256) void k_prim2con(const Params p, const double* __restrict__ P,
                                                  double* __restrict__ U) {
    long o;
    if (!interior_cell(p, (long)blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    Geo<double> m;
    cell_geo<CURVED>(p, o, m);
    double Pc[NF], Uc[NF];
    for (int f = 0; f < NF; ++f) Pc[f] = P[f * p.Np + o];
    prim2con(m, p.G, Pc, Uc);
    for (int f = 0; f < NF; ++f) U[f * p.Np + o] = Uc[f];
}

__device__ __forceinline__ void rec_setup(const Params& p, const Geo<double>& m, const double* U, RecIn& k) {
    k.G = p.G;
    k.D = U[I_D];
    k.tau = U[I_TAU];
    for (int i = 0; i < 3; ++i) {
        k.S[i] = U[I_S + i];
        k.Bc[i] = U[I_B + i];
    }
    for (int a = 0; a < 6; ++a) { k.g[a] = m.g[a]; k.gi[a] = m.gi[a]; }
    k.sg = m.sg;
    k.isg = m.isg;
    lower(m.g, k.Bc, k.Bl);
    for (int i = 0; i < 3; ++i) k.Bl[i] *= m.isg;     // undensitised, lowered B
}

__device__ __forceinline__ void write_prims(const Params& p, long o, const Geo<double>& m, const double* U,
                                            const double* x, const double* Ec, double* P) {
    const double* v = x + 1;
    double vl[3];
    lower(m.g, v, vl);
    const double W = 1.0 / sqrt(1.0 - dot3(vl, v));
    P[I_RHO * p.Np + o] = U[I_D] * m.isg / W;
    P[I_P * p.Np + o] = x[0];
    for (int i = 0; i < 3; ++i) {
        P[(I_V + i) * p.Np + o] = v[i];
        P[(I_B + i) * p.Np + o] = U[I_B + i] * m.isg;
        P[(I_E + i) * p.Np + o] = Ec[i] * m.isg;
    }
    for (int f = I_PHI; f < NF; ++f) P[f * p.Np + o] = U[f] * m.isg;
}

// primitives at a recovered root from RecIn (D, Bcal) and the cleaning and
// charge rows of the conserved array U (global)
__device__ __forceinline__ void write_prims_k(const Params& p, long o, const Geo<double>& m, const RecIn& k,
                                              const double* U, const double* x, const double* Ec, double* P) {
    const double* v = x + 1;
    double vl[3];
    lower(m.g, v, vl);
    const double W = frsqrt(1.0 - dot3(vl, v));
    P[I_RHO * p.Np + o] = k.D * m.isg / W;
    P[I_P * p.Np + o] = x[0];
    for (int i = 0; i < 3; ++i) {
        P[(I_V + i) * p.Np + o] = v[i];
        P[(I_B + i) * p.Np + o] = k.Bc[i] * m.isg;
        P[(I_E + i) * p.Np + o] = Ec[i] * m.isg;
    }
    for (int f = I_PHI; f < NF; ++f) P[f * p.Np + o] = U[f * p.Np + o] * m.isg;
}

__device__ __forceinline__ void copy_prims(const Params& p, long o, const double* Pg, double* P) {
    for (int f = 0; f < NF; ++f) P[f * p.Np + o] = Pg[f];
}

// plain recovery (E fixed)
template <bool CURVED>
__global__ __launch_bounds__(256) void k_con2prim(const Params p, const double* __restrict__ U,
                                                  double* __restrict__ P, int* __restrict__ status,
                                                  unsigned long long* nfail) {
    long o;
    if (!interior_cell(p, (long)blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    Geo<double> m;
    cell_geo<CURVED>(p, o, m);
    double Uc[NF], Pg[NF];
    for (int f = 0; f < NF; ++f) { Uc[f] = U[f * p.Np + o]; Pg[f] = P[f * p.Np + o]; }
    RecIn k;
    rec_setup(p, m, Uc, k);
    double x[4] = {Pg[I_P], Pg[I_V], Pg[I_V + 1], Pg[I_V + 2]};
    int it;
    const double Ec[3] = {Uc[I_E], Uc[I_E + 1], Uc[I_E + 2]};
    const int st = recover_plain(k, Ec, x, p.tol, p.maxit, &it);
    if (st >= 0) write_prims(p, o, m, Uc, x, Ec, P);
    else atomicAdd(nfail, 1ull);
    if (status) status[o] = st;
}

// ------------------------------------------------------- explicit sources
// metric derivatives at a cell centre: 4th-order central differences along
// active dimensions (zero along the others), and K_ij
struct MetricDerivs {
    double da[3], db[3][3], dg[3][6], K[6];
};

template <bool CURVED>
__device__ __forceinline__ void metric_derivs(const Params& p, long o, MetricDerivs& md) {
    for (int d = 0; d < 3; ++d) {
        md.da[d] = 0.0;
        for (int a = 0; a < 3; ++a) md.db[d][a] = 0.0;
        for (int a = 0; a < 6; ++a) md.dg[d][a] = 0.0;
    }
    for (int a = 0; a < 6; ++a) md.K[a] = 0.0;
    if (!CURVED) return;
    for (int d = 0; d < 3; ++d) {
        if (!is_active(p, d)) continue;
        const long s = p.st[d];
        const double c = p.idx[d] / 12.0;
        auto D4 = [&](const double* f) { return (f[o - 2 * s] - 8.0 * f[o - s] + 8.0 * f[o + s] - f[o + 2 * s]) * c; };
        md.da[d] = D4(p.alp);
        if (p.bet)
            for (int a = 0; a < 3; ++a) md.db[d][a] = D4(p.bet + a * p.Np);
        for (int a = 0; a < 6; ++a) md.dg[d][a] = D4(p.gam + a * p.Np);
    }
    if (p.K)
        for (int a = 0; a < 6; ++a) md.K[a] = p.K[a * p.Np + o];
}

// eq. GRRMHD_flux_form sources at a cell centre, E rows without R_E.
// R: double, or the dual type of the adjoint's tangent passes (the metric
// is fixed input and enters as double)
template <bool CURVED, class R>
__device__ __forceinline__ void sources_t(const Params& p, const Geo<double>& m, const MetricDerivs& md,
                                          const R* Pc, const R* Uc, R* S) {
    const R* v = Pc + I_V;
    const double kap = p.kappa;
    if (!CURVED) {
        for (int f = 0; f < NF; ++f) S[f] = R(0.0);
        for (int i = 0; i < 3; ++i) S[I_E + i] = -(Uc[I_Q] * v[i]);
        S[I_PHI] = -(Uc[I_PHI] * kap);
        S[I_PSI] = Uc[I_Q] - Uc[I_PSI] * kap;
        return;
    }
    const double a = m.alp;
    // Gamma^i = gamma^il (gamma^jk d_j gamma_lk - 1/2 gamma^jk d_l gamma_jk)
    double A[3], Gm[3], gda[3];
    for (int l = 0; l < 3; ++l) {
        double s1 = 0.0, s2 = 0.0;
        for (int j = 0; j < 3; ++j)
            for (int kk = 0; kk < 3; ++kk) {
                s1 += m.gi[sidx(j, kk)] * md.dg[j][sidx(l, kk)];
                s2 += m.gi[sidx(j, kk)] * md.dg[l][sidx(j, kk)];
            }
        A[l] = s1 - 0.5 * s2;
    }
    for (int i = 0; i < 3; ++i) {
        Gm[i] = m.gi[sidx(i, 0)] * A[0] + m.gi[sidx(i, 1)] * A[1] + m.gi[sidx(i, 2)] * A[2];
        gda[i] = m.gi[sidx(i, 0)] * md.da[0] + m.gi[sidx(i, 1)] * md.da[1] + m.gi[sidx(i, 2)] * md.da[2];
    }
    // densitised stress with both indices up
    const R* B = Pc + I_B;
    const R* E = Pc + I_E;
    R vl[3], Bl[3], El[3];
    lower(m.g, v, vl);
    lower(m.g, B, Bl);
    lower(m.g, E, El);
    const R W = frsqrt(R(1.0) - dot3(vl, v));
    const R hW2 = (Pc[I_RHO] + Pc[I_P] * (p.G / (p.G - 1.0))) * (W * W);
    const R pt = Pc[I_P] + (dot3(El, E) + dot3(Bl, B)) * 0.5;
    R Su[6];
    for (int j = 0; j < 3; ++j)
        for (int kk = j; kk < 3; ++kk)
            Su[sidx(j, kk)] = (hW2 * v[j] * v[kk] - E[j] * E[kk] - B[j] * B[kk] + pt * m.gi[sidx(j, kk)]) * m.sg;
    const R* Sl = Uc + I_S;
    R Sup[3];
    for (int i = 0; i < 3; ++i) Sup[i] = Sl[0] * m.gi[sidx(i, 0)] + Sl[1] * m.gi[sidx(i, 1)] + Sl[2] * m.gi[sidx(i, 2)];
    double Ktr = 0.0;
    R SK = R(0.0);
    if (p.K) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const double kij = md.K[sidx(i, j)];
                Ktr += m.gi[sidx(i, j)] * kij;
                SK += Su[sidx(i, j)] * kij;
            }
    }
    S[I_D] = R(0.0);
    for (int i = 0; i < 3; ++i) {
        R t = R(0.0);
        for (int j = 0; j < 3; ++j)
            for (int kk = 0; kk < 3; ++kk) t += Su[sidx(j, kk)] * md.dg[i][sidx(j, kk)];
        S[I_S + i] = t * (0.5 * a) + (Sl[0] * md.db[i][0] + Sl[1] * md.db[i][1] + Sl[2] * md.db[i][2]) -
                     (Uc[I_TAU] + Uc[I_D]) * md.da[i];
    }
    S[I_TAU] = SK * a - (Sup[0] * md.da[0] + Sup[1] * md.da[1] + Sup[2] * md.da[2]);
    for (int i = 0; i < 3; ++i) {
        const R bb = Uc[I_B] * md.db[0][i] + Uc[I_B + 1] * md.db[1][i] + Uc[I_B + 2] * md.db[2][i];
        const R eb = Uc[I_E] * md.db[0][i] + Uc[I_E + 1] * md.db[1][i] + Uc[I_E + 2] * md.db[2][i];
        const double gg = gda[i] - a * Gm[i];
        S[I_B + i] = Uc[I_PHI] * gg - bb;
        S[I_E + i] = Uc[I_PSI] * gg - eb - Uc[I_Q] * v[i] * a;
    }
    S[I_PHI] = -(Uc[I_PHI] * (a * Ktr)) + (Uc[I_B] * md.da[0] + Uc[I_B + 1] * md.da[1] + Uc[I_B + 2] * md.da[2]) -
               Uc[I_PHI] * (a * kap);
    S[I_PSI] = -(Uc[I_PSI] * (a * Ktr)) + (Uc[I_E] * md.da[0] + Uc[I_E + 1] * md.da[1] + Uc[I_E + 2] * md.da[2]) +
               Uc[I_Q] * a - Uc[I_PSI] * (a * kap);
    S[I_Q] = R(0.0);
}

template <bool CURVED>
__device__ __forceinline__ void sources(const Params& p, long o, const Geo<double>& m, const double* Pc,
                                        const double* Uc, double* S) {
    MetricDerivs md;
    metric_derivs<CURVED>(p, o, md);
    sources_t<CURVED, double>(p, m, md, Pc, Uc, S);
}

// --------------------------------------------------------------- stages
// gamma of table imex
__host__ __device__ constexpr double GAM_IMEX() { return 0.29289321881345247560; }

// stage 1: E(1) = E^n + gamma dt R_E(U(1)), everything else unchanged
template <bool CURVED>
__global__ __launch_bounds__(256) void k_stage1(const Params p, double dt, const double* __restrict__ sig,
                                                const double* __restrict__ Un, const double* __restrict__ Pg_,
                                                double* __restrict__ P1, double* __restrict__ R1,
                                                double* __restrict__ U1, int* __restrict__ status,
                                                unsigned long long* nfail) {
    long o;
    if (!interior_cell(p, (long)blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    const long Np = p.Np;
    Geo<double> m;
    cell_geo<CURVED>(p, o, m);
    RecIn k;
    {
        double Uc[NF];
        for (int f = 0; f < NF; ++f) Uc[f] = Un[f * Np + o];
        rec_setup(p, m, Uc, k);
        for (int i = 0; i < 3; ++i) k.Es[i] = Uc[I_E + i];
        if (U1)
            for (int f = 0; f < NF; ++f)
                if (f < I_E || f >= I_E + 3) U1[f * Np + o] = Uc[f];
    }
    const double gdt = GAM_IMEX() * dt;
    k.cfac = gdt * m.alp * sig[o];
    double x[4] = {Pg_[I_P * Np + o], Pg_[I_V * Np + o], Pg_[(I_V + 1) * Np + o], Pg_[(I_V + 2) * Np + o]};
    double E[3] = {k.Es[0], k.Es[1], k.Es[2]};
    int it, st;
    __builtin_amdgcn_sched_barrier(0);
    if (k.cfac != 0.0) st = recover_stiff(k, x, E, p.tol, p.maxit, &it);
    else st = recover_plain(k, E, x, p.tol, p.maxit, &it);
    __builtin_amdgcn_sched_barrier(0);
    if (st >= 0) {
        write_prims_k(p, o, m, k, Un, x, E, P1);
    } else {
        for (int f = 0; f < NF; ++f) P1[f * Np + o] = Pg_[f * Np + o];
        for (int i = 0; i < 3; ++i) E[i] = k.Es[i];
        atomicAdd(nfail, 1ull);
    }
    for (int i = 0; i < 3; ++i) R1[i * Np + o] = (E[i] - k.Es[i]) / gdt;
    if (U1)
        for (int i = 0; i < 3; ++i) U1[(I_E + i) * Np + o] = E[i];
    if (status) status[o] = st;
}

// stage 2 (STAGE = 2) and the final update (STAGE = 3), after the flux
// divergence of P_s has been accumulated into rhs.  Output rows are written
// as soon as they are known so that little stays live across the recovery.
template <int STAGE, bool CURVED>
__global__ __launch_bounds__(256) void k_update(const Params p, double dt, const double* __restrict__ sig,
                                                const double* __restrict__ Un, const double* __restrict__ Us,
                                                const double* __restrict__ Ps, const double* __restrict__ R1,
                                                const double* __restrict__ R2, const double* __restrict__ rhs,
                                                double* __restrict__ Uo, double* __restrict__ Po,
                                                double* __restrict__ Ro, int* __restrict__ status,
                                                unsigned long long* nfail) {
    long o;
    if (!interior_cell(p, (long)blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    const long Np = p.Np;
    Geo<double> m;
    cell_geo<CURVED>(p, o, m);
    const double g = GAM_IMEX();
    RecIn k;
    double x[4];
    {
        double Y[NF];
        {
            double Pc[NF], Uc[NF], S[NF];
            for (int f = 0; f < NF; ++f) Pc[f] = Ps[f * Np + o];
            prim2con(m, p.G, Pc, Uc);
            sources<CURVED>(p, o, m, Pc, Uc, S);
            x[0] = Pc[I_P];
            x[1] = Pc[I_V];
            x[2] = Pc[I_V + 1];
            x[3] = Pc[I_V + 2];
            if (STAGE == 2) {
                for (int f = 0; f < NF; ++f) Y[f] = Un[f * Np + o] + dt * (rhs[f * Np + o] + S[f]);
            } else {
                // U^{n+1} = (U^n + U(2))/2 + dt/2 F(U(2)) + dt/2 (2 gamma R1 + (1 - gamma) R2) on E
                for (int f = 0; f < NF; ++f)
                    Y[f] = 0.5 * (Un[f * Np + o] + Us[f * Np + o]) + 0.5 * dt * (rhs[f * Np + o] + S[f]);
                for (int i = 0; i < 3; ++i)
                    Y[I_E + i] += 0.5 * dt * (2.0 * g * R1[i * Np + o] + (1.0 - g) * R2[i * Np + o]);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        for (int f = 0; f < NF; ++f)
            if (STAGE == 3 || f < I_E || f >= I_E + 3) Uo[f * Np + o] = Y[f];
        rec_setup(p, m, Y, k);
        if (STAGE == 2)
            for (int i = 0; i < 3; ++i) k.Es[i] = Y[I_E + i] + dt * (1.0 - 2.0 * g) * R1[i * Np + o];
        else
            for (int i = 0; i < 3; ++i) k.Es[i] = Y[I_E + i];
    }
    __builtin_amdgcn_sched_barrier(0);
    double E[3] = {k.Es[0], k.Es[1], k.Es[2]};
    int it, st;
    if (STAGE == 2) {
        k.cfac = g * dt * m.alp * sig[o];
        if (k.cfac != 0.0) st = recover_stiff(k, x, E, p.tol, p.maxit, &it);
        else st = recover_plain(k, E, x, p.tol, p.maxit, &it);
    } else {
        st = recover_plain(k, E, x, p.tol, p.maxit, &it);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (st >= 0) {
        write_prims_k(p, o, m, k, Uo, x, E, Po);
    } else {
        for (int f = 0; f < NF; ++f) Po[f * Np + o] = Ps[f * Np + o];
        for (int i = 0; i < 3; ++i) E[i] = k.Es[i];
        atomicAdd(nfail, 1ull);
    }
    if (STAGE == 2) {
        for (int i = 0; i < 3; ++i) {
            Uo[(I_E + i) * Np + o] = E[i];
            Ro[i * Np + o] = (E[i] - k.Es[i]) / (g * dt);
        }
    }
    if (status) status[o] = st;
}

// ---------------------------------------------------- max signal speed (CFL)
template <bool CURVED>
__global__ __launch_bounds__(256) void k_max_speed(const Params p, unsigned long long* out) {
    long o;
    double best = 0.0;
    const long ncell = (long)p.n[0] * p.n[1] * p.n[2];
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < ncell; t += (long)gridDim.x * blockDim.x) {
        interior_cell(p, t, o);
        Geo<double> m;
        cell_geo<CURVED>(p, o, m);
        double lp, lm;
        if (is_active(p, 0)) { speeds<0>(p, m, lp, lm); best = fmax(best, fmax(lp, -lm) * p.idx[0]); }
        if (is_active(p, 1)) { speeds<1>(p, m, lp, lm); best = fmax(best, fmax(lp, -lm) * p.idx[1]); }
        if (is_active(p, 2)) { speeds<2>(p, m, lp, lm); best = fmax(best, fmax(lp, -lm) * p.idx[2]); }
    }
    // wavefront reduction, then one atomic per wave on the ordered bit pattern
    for (int off = 32; off > 0; off >>= 1) best = fmax(best, __shfl_xor(best, off));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(best));
}

__global__ void k_zero_u64(unsigned long long* a, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = 0ull;
}

}  // namespace rmhd
