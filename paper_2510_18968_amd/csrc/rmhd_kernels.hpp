// gfx950 kernels of the IMEX-SSP2(2,2,2) stage of resistive GRMHD.
//
// Data: float64 SoA over the padded grid (x fastest), one field per plane.
// The flux divergence is split by direction:
//   x: the rows with their ghost cells form one sequence, cut into segments
//      of 58 positions; a wave64 holds one segment plus 3 halo lanes on each
//      side, every lane reconstructs its own cell to both faces (shared WENO
//      smoothness indicators), and the right neighbour's left-face state and
//      the left neighbour's face flux arrive by DPP lane moves, so each face
//      flux is computed once;
//   y, z: lanes run along x (coalesced loads) and each wave marches a
//      segment along the flux direction through a ring of the last five rows
//      of P in LDS, carrying the previous face state and flux in registers.
// The pointwise kernels add the non-stiff sources, assemble the IMEX stage
// and run the stiff recovery, one cell per lane.
#pragma once
#include "rmhd_phys.hpp"

namespace rmhd {

// g[d]: padded index of the first interior cell along d (the ghost width ng,
// or more padding along x for aligned rows); np[d] = n[d] + 2 g[d]
struct Params {
    int n[3], g[3], np[3], ng, active, bc[3], maxit, speed_mode;
    long st[3], Np;
    double dx[3], idx[3], G, kappa, tol;
    double cdiff[3];            // idx / 12: the 4th-order centred difference's factor
    double tolq;                // 0.0075 tol: the stiff recovery's early stop (kernel arguments
                                // live in scalar registers; a product formed on the device
                                // would hold two vector registers in every kernel that inlines it)
    // metric (nullptr alp/gam: flat), beta/K may be nullptr
    const double* alp;
    const double* bet;
    const double* gam;
    const double* K;
    // opt-in histograms of recovery iterations (3 x RMHD_HIST_BINS), nullptr = off
    unsigned long long* hist;
    // conductivity model (0: the sigma field) and the artificial atmosphere
    // (rho_atmo = 0: off; p_atmo = K_atmo rho_atmo^Gamma)
    int sig_model;
    double sig0, sig_exp, sig_Datmo, rho_atmo, p_atmo;
};

// conductivity from the conserved rest-mass density D (Sec. IV.A eq.
// sigma_evol: sigma0 D^gamma; Sec. IV.E eq. dynamo_sigma: sigma0 max(1 -
// D_atmo/D, 0)^2); only called when a model is selected
__device__ __forceinline__ double sigma_of_D(const Params& p, double D) {
    if (p.sig_model == 1) return p.sig0 * pow(D, p.sig_exp);
    const double t = fmax(1.0 - p.sig_Datmo / D, 0.0);
    return p.sig0 * t * t;
}
constexpr double ATMO_FACTOR = 1.01;

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

template <int D, class R, bool DG> __device__ __forceinline__ void speeds(const Params& p, const Geo<R, DG>& m, R& lp, R& lm) {
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
template <class R, bool DG> __device__ __forceinline__ bool bad_state(const Geo<R, DG>& m, const R* P) {
    R vl[3];
    lower(m, P + I_V, vl);
    const R v2 = dot3(vl, P + I_V);
    return !(P[I_RHO] > R(0)) || !(P[I_P] > R(0)) || !(v2 < R(1));
}

// HLLE flux of direction D at a face with metric m (Sec. III)
template <int D, class R, bool DG>
__device__ __forceinline__ void face_flux(const Params& p, const Geo<R, DG>& m, const R* PL, const R* PR, R Jd, R* Fh) {
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

// the metric-derivative sources of one direction (defined with the stage kernels)
template <int d, class R, bool DG>
__device__ __forceinline__ void sources_dir(const Params& p, const Geo<double, DG>& m, double da, const double* db,
                                            const double* dg, const R* Pc, const R* Uc, R* S);

// ----------------------------------------------------- fluxes, lanes along D
// One wave per segment of TSEG cells along D; lane l holds the cell
// seg*TSEG - 3 + l, so every lane loads its own 14 primitives and its metric
// once and takes the stencil neighbours, the right face state and the left
// face flux from the neighbouring lanes.  Lanes 2..61 reconstruct, faces lie
// between lanes 2..61, lanes 3..3+TSEG-1 write their divergence.  For D = 1, 2
// a lane's loads are strided by the row or plane; consecutive waves take
// consecutive x so that one 128-byte line serves 16 waves, and workgroups are
// renumbered so that those waves run on one XCD (one L2).
constexpr int TSEG = 58;

// workgroups go round-robin to the 8 XCDs: renumber so that consecutive
// logical workgroups share an XCD (gridDim.x is a multiple of 8)
__device__ __forceinline__ long xcd_block() {
    const unsigned nb = gridDim.x, b = blockIdx.x;
    return (long)(b & 7u) * (long)(nb >> 3) + (long)(b >> 3);
}

// s_waitcnt with vmcnt(N) and the other counters at their maxima
template <int N> __device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt has six bits");
    __builtin_amdgcn_s_waitcnt(0x0F70 | (N & 15) | ((N >> 4) << 14));
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" ::: "memory");
}
// s_waitcnt lgkmcnt(0) (LDS reads landed), the other counters at their maxima
__device__ __forceinline__ void wait_lgkm0() {
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" ::: "memory");
}

// v, with a data dependency on dep: keeps the compiler from hoisting the lane
// shuffles of v above the work that produced dep (which would keep every
// field's stencil live at once)
template <class R, class T> __device__ __forceinline__ R after(R v, T dep) {
    asm volatile("" : "+v"(v) : "v"(dep));
    return v;
}

// Whole-wave lane shifts by DPP (VALU moves, no LDS round trip):
// up<N>(v) on lane i is v of lane i - N, down<N>(v) is v of lane i + N; lanes
// whose source is off the wave get 0 (they carry no used result).
// Every lane of the wave must be active.
// (bound_ctrl: a lane whose source is off the wave reads 0, so no copy of
// the old value has to be made first)
__device__ __forceinline__ int dpp_up1(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_dn1(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
template <bool UP> __device__ __forceinline__ float shift1(float v) {
    const int b = __float_as_int(v);
    return __int_as_float(UP ? dpp_up1(b) : dpp_dn1(b));
}
template <bool UP> __device__ __forceinline__ double shift1(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(UP ? dpp_up1(hi) : dpp_dn1(hi), UP ? dpp_up1(lo) : dpp_dn1(lo));
}
template <int N, class R> __device__ __forceinline__ R up(R v) {
    for (int k = 0; k < N; ++k) v = shift1<true>(v);
    return v;
}
template <int N, class R> __device__ __forceinline__ R down(R v) {
    for (int k = 0; k < N; ++k) v = shift1<false>(v);
    return v;
}

template <class R> __device__ __forceinline__ R face4(R a) {
    // value at the face between this lane's cell and the next one, 4th order
    const R am = up<1>(a), ap = down<1>(a), app = down<2>(a);
    return (-am + 9.0 * a + 9.0 * ap - app) * 0.0625;
}

// inputs of one lane for one segment: its cell's primitives, metric and sigma
struct FluxIn {
    double P[NF], g[6], a, b[3], s;
};

// wave item -> segment and transverse position; o = this lane's padded offset
template <int D> struct FluxItem {
    int seg, c, cp;
    long o;
};

// x sweep: the rows, each with its 3 ghost cells on both sides (n_x + 6
// positions), are taken as one sequence; segment wid holds positions
// 58 wid - 3 .. 58 wid + 60 of it.  Ghost cells are the halo at a row's ends,
// so a segment may run across rows (a face between two rows is computed and
// never used) and no lanes idle at a row's end.  it.c: interior x of the
// lane's cell (outside 0..n_x-1 on ghost positions and past the end).
template <int D>
__device__ __forceinline__ FluxItem<D> flux_item(const Params& p, long wid, int nseg, int lane) {
    constexpr int E1 = (D == 0) ? 1 : 0, E2 = (D == 2) ? 1 : 2;
    const long n1 = p.n[E1];
    FluxItem<D> it;
    long a1, a2;
    if (D == 0) {
        // 32-bit: the sequence has fewer than 2^31 positions (checked on the host)
        const int W0 = p.n[0] + 6;
        const int V = W0 * p.n[E1] * p.n[E2];
        const int v = (int)wid * TSEG - 3 + lane;
        const int vc = v < 0 ? 0 : (v < V ? v : V - 1);
        const unsigned r = (unsigned)vc / (unsigned)W0;
        const int x = vc - (int)r * W0 - 3;
        a1 = r % (unsigned)p.n[E1];
        a2 = r / (unsigned)p.n[E1];
        it.seg = (int)wid;
        it.c = v == vc ? x : -4;
        it.cp = x + p.g[0];
        it.o = (a1 + p.g[E1]) * p.st[E1] + (a2 + p.g[E2]) * p.st[E2] + (long)it.cp;
        return it;
    } else {
        a1 = wid % n1;
        const long r = wid / n1;
        it.seg = (int)(r % nseg);
        a2 = r / nseg;
    }
    const int nD = p.n[D], gD = p.g[D];
    it.c = it.seg * TSEG - 3 + lane;                                // interior index of the lane's cell
    it.cp = min(max(it.c + gD, 0), nD + 2 * gD - 1);                // padded; clamped on unused edge lanes
    it.o = (a1 + p.g[E1]) * p.st[E1] + (a2 + p.g[E2]) * p.st[E2] + (long)it.cp * p.st[D];
    return it;
}

template <int D, bool CURVED, bool DG>
__device__ __forceinline__ void flux_load(const Params& p, const double* __restrict__ P,
                                          const double* __restrict__ sig, const FluxItem<D>& it, FluxIn& in) {
    const long Np = p.Np, o = it.o;
    // a ghost cell's primitives and sigma from its interior image (boundary
    // conditions; the metric is given at ghost cells)
    const long oi = o + (long)(bc_map(p, D, it.cp) - it.cp) * p.st[D];
#pragma unroll
    for (int f = 0; f < NF; ++f) in.P[f] = P[f * Np + oi];
    if (CURVED) {
#pragma unroll
        for (int a = 0; a < 6; ++a)
            in.g[a] = zero_entry<DG>(a) ? 0.0 : p.gam[a * Np + o];
        in.a = p.alp[o];
        if (p.bet) {
#pragma unroll
            for (int a = 0; a < 3; ++a) in.b[a] = p.bet[a * Np + o];
        }
    }
    in.s = sig[oi];
}

// minus the D-flux divergence of one segment into rhs (= or +=)
template <int D, int RECON, bool CURVED, class R, bool ACC, bool DG>
__device__ __forceinline__ void flux_compute(const Params& p, const double* __restrict__ P,
                                             double* __restrict__ rhs, const FluxItem<D>& it, const FluxIn& in,
                                             int lane) {
    const long s = p.st[D], Np = p.Np, o = it.o;
    const int nD = p.n[D], gD = p.g[D];
    const bool cell = lane >= 3 && lane < 3 + TSEG && it.c >= 0 && it.c < nD;
    double acc[NF];
    if (ACC) {
        // the read half of the read-modify-write, issued before the arithmetic
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f] = cell ? rhs[f * Np + o] : 0.0;
    } else {
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f] = 0.0;
    }
    Geo<double, DG> mc;   // the lane's cell
    if (CURVED) {
        mc.alp = in.a;
        for (int a = 0; a < 3; ++a) mc.bet[a] = p.bet ? in.b[a] : 0.0;
        for (int a = 0; a < 6; ++a)
            if (!zero_entry<DG>(a)) mc.g[a] = in.g[a];
        geo_finish(mc);
    } else {
        geo_flat(mc);
    }
    __builtin_amdgcn_sched_barrier(0);
    // cell-centre current (FP64 in every form), face value = mean of the two cells
    double JD;
    {
        double J[3];
        current(mc, in.P, in.s, J);
        JD = J[D];
    }
    const R Jf = R(0.5 * (JD + down<1>(JD)));
    __builtin_amdgcn_sched_barrier(0);
    R fm[NF], fp[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        // two fields in flight: the shuffles of f wait for field f - 2
        const R v = f >= 2 ? after(R(in.P[f]), fp[f - 2]) : R(in.P[f]);
        const R v1 = up<1>(v), w1 = down<1>(v);
        const R st[5] = {up<1>(v1), v1, v, w1, down<1>(w1)};
        recon<RECON>(st, fm[f], fp[f]);
    }
    // face between this lane's cell and the next
    Geo<R, DG> m;
    if (CURVED) {
        m.alp = R(face4(in.a));
        for (int a = 0; a < 3; ++a) m.bet[a] = p.bet ? R(face4(in.b[a])) : R(0);
        m.g[0] = R(face4(in.g[0]));
        if (DG) {
            m.g[3] = R(face4(after(in.g[3], m.g[0])));
            m.g[5] = R(face4(after(in.g[5], m.g[3])));
        } else {
            for (int a = 1; a < 6; ++a) m.g[a] = R(face4(after(in.g[a], m.g[a - 1])));
        }
        geo_finish(m);
    } else {
        geo_flat(m);
    }
    R PR[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) PR[f] = down<1>(fm[f]);
    __builtin_amdgcn_sched_barrier(0);
    // first-order fallback: the cell values of this lane and of the next one
    // (taken from the neighbouring lane, not reloaded: a load here would make
    // every later wait also wait for the next segment's prefetch)
    R Pn[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) Pn[f] = R(down<1>(in.P[f]));
    if (bad_state(m, fp))
        for (int f = 0; f < NF; ++f) fp[f] = R(in.P[f]);
    if (bad_state(m, PR))
        for (int f = 0; f < NF; ++f) PR[f] = Pn[f];
    R Fh[NF];
    face_flux<D>(p, m, fp, PR, Jf, Fh);

    if (CURVED) {
        // source terms with the metric derivatives along D, 4th-order centred
        // differences from the neighbouring lanes
        const double cd = p.idx[D] / 12.0;
        auto dD = [&](double f) {
            const double m1 = up<1>(f), p1 = down<1>(f), m2 = up<1>(m1), p2 = down<1>(p1);
            return (m2 - 8.0 * m1 + 8.0 * p1 - p2) * cd;
        };
        double dg[6], db[3] = {0.0, 0.0, 0.0};
        const double da = dD(in.a);
        if (p.bet)
            for (int a = 0; a < 3; ++a) db[a] = dD(in.b[a]);
        for (int a = 0; a < 6; ++a) dg[a] = zero_entry<DG>(a) ? 0.0 : dD(in.g[a]);
        double Uc[NF];
        prim2con(mc, p.G, in.P, Uc);
        sources_dir<D>(p, mc, da, db, dg, in.P, Uc, acc);
    }
    const R ih = R(p.idx[D]);
    // every lane stores (no branch: the wait for the next segment's loads can
    // then leave these stores in flight); a lane without a cell of its own
    // writes the line's last left ghost cell, which nothing reads in rhs
    const long os = cell ? o : o - (long)(it.cp - (gD - 1)) * s;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const R Fl = up<1>(Fh[f]);
        rhs[f * Np + os] = acc[f] + double(-(Fh[f] - Fl) * ih);
    }
}

// one segment per wave
template <int D, int RECON, bool CURVED, class R, bool ACC, bool DG>
__global__ __launch_bounds__(256) void k_flux_t(const Params p, const double* __restrict__ P,
                                                const double* __restrict__ sig, double* __restrict__ rhs,
                                                int nseg, long nitems) {
    const int lane = threadIdx.x & 63;
    const long wid = xcd_block() * 4 + (threadIdx.x >> 6);
    if (wid >= nitems) return;                       // uniform per wave
    const FluxItem<D> it = flux_item<D>(p, wid, nseg, lane);
    FluxIn in;
    flux_load<D, CURVED, DG>(p, P, sig, it, in);
    flux_compute<D, RECON, CURVED, R, ACC, DG>(p, P, rhs, it, in, lane);
}

// persistent: one wave per SIMD walks the segments wid, wid + W, ..., loading
// the next segment's inputs while it computes the current one
template <int D, int RECON, bool CURVED, class R, bool ACC, bool DG>
__global__ __launch_bounds__(256) void k_flux_p(const Params p, const double* __restrict__ P,
                                                const double* __restrict__ sig, double* __restrict__ rhs,
                                                int nseg, long nitems) {
    const int lane = threadIdx.x & 63;
    const long W = (long)gridDim.x * 4;
    long wid = xcd_block() * 4 + (threadIdx.x >> 6);
    if (wid >= nitems) return;                       // uniform per wave
    FluxItem<D> it = flux_item<D>(p, wid, nseg, lane);
    FluxIn in;
    flux_load<D, CURVED, DG>(p, P, sig, it, in);
    // the loop begins with every input loaded on both ways into it, so the
    // wait-count pass needs no wait on them inside
    if (!ACC) wait_vm<0>();
    for (;;) {
        const long nxt = wid + W;
        // unconditional (the last pass reloads a valid item): a branch around
        // the loads leaves the wait-count pass unsure of what is in flight and
        // it then waits for the prefetch right after issuing it
        const FluxItem<D> it2 = flux_item<D>(p, nxt < nitems ? nxt : wid, nseg, lane);
        FluxIn in2;
        flux_load<D, CURVED, DG>(p, P, sig, it2, in2);
        flux_compute<D, RECON, CURVED, R, ACC, DG>(p, P, rhs, it, in, lane);
        // the next segment's loads were followed by the NF stores of this one
        // only: wait for the loads, leave the stores in flight
        if (!ACC) wait_vm<NF>();
        if (nxt >= nitems) break;
        wid = nxt;
        it = it2;
        in = in2;
    }
}

// gamma of table imex
__host__ __device__ constexpr double GAM_IMEX() { return 0.29289321881345247560; }

// per-block tallies of the stage kernels in LDS (recovery iteration
// histogram, failed cells), added to the global counters once per block at
// the end: inside the chunk loop no global atomic sits between the next
// chunk's loads and the wait for them
struct StageTally {
    unsigned int hist[32];
    unsigned int fail, atmo;
};
__device__ __forceinline__ void tally_cell(StageTally& t, bool hist, bool counted, int st, int it) {
    if (!counted) return;
    if (hist) atomicAdd(&t.hist[it < 0 ? 0 : (it > 31 ? 31 : it)], 1u);
    if (st < 0) atomicAdd(&t.fail, 1u);
}

// the inputs of one cell's stage update
struct StageIn {
    long o;
    bool ok;
    double P[NF], Un[NF], rh[NF], Us[NF], R1[3], R2[3], sg, a, g[6], K[6];
};

// stage 2 / final update of one cell (defined with the stage kernels; the z
// window runs stage 2 on the rows it finishes).  MODEL = false: sigma is the
// given field (no conductivity-model code in the caller)
template <int STAGE, bool CURVED, bool HASK, bool DG, bool MODEL = true>
__device__ __forceinline__ void update_cell(const Params& p, double dt, const StageIn& in, double* __restrict__ Uo,
                                            double* __restrict__ Po, double* __restrict__ Ro,
                                            double* __restrict__ P1o, int* __restrict__ status, long st_stride,
                                            StageTally& tal, StageTally& tal1);

// ------------------------------------------- y / z fluxes: rolling window
// Lanes along x, one wave marches a segment of cells along D.  Every row of P
// is loaded once, straight from HBM into a ring of the last five rows in LDS
// (global_load_lds_dwordx4: lane m brings two consecutive doubles of one of
// two fields, so one instruction fills two 64-wide field rows; 35.8 KB per
// wave); the metric and sigma rows c-3 .. c+1 stay in registers, and row
// c+2, which step c does not use, waits in an LDS staging row, loaded the
// same way one step ahead.  Step c: rhs row c-1 is read, its sources are formed
// (derivatives from rows c-3..c+1), the current and the reconstruction of c
// are taken; then row c+3 is requested into the ring slot that row c-2 has
// just left, and while it arrives the face c-1/2 is computed and rhs row c-1
// written.  Lanes exchange data only through the ring.  Every ring read is
// preceded by a wait for the loads of its row (the first step included).
constexpr int WRING = 5;

// all counters but vmcnt at their maxima: wait for every outstanding vector
// memory operation, including the ring loads into LDS
__device__ __forceinline__ void wait_ring() {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" ::: "memory");
}

// packed index of the j-th stored metric component (DG: the diagonal only)
template <bool DG> __host__ __device__ constexpr int gcomp(int j) { return DG ? (j == 0 ? 0 : (j == 1 ? 3 : 5)) : j; }

// The stage-2 update run by the last window sweep on each row it finishes
// (FUSE): its inputs besides the ring row and the window's metric and sigma,
// and its outputs (status: st_stride 0 writes one dummy word)
struct FuseArgs {
    const double* Un;
    const double* R1;
    double* U2;
    double* P2;
    double* R2;
    int* status;
    long st_stride;
    double dt;
    unsigned long long* nfail;
    int* dummy;              // a word nothing reads
};

// SHIFT: the metric has a shift (beta rows in the window); without one the
// window holds alpha, gamma_ij and sigma only.  DG: a diagonal metric, whose
// window and staging row hold the three diagonal entries of gamma_ij.
// FUSE (D = 2, no extrinsic curvature, a sigma field): instead of storing rhs
// row c - 1, the step runs stage 2 on its cells (update_cell on U^n and R1
// loaded for the row, P(1) from the ring, metric and sigma from the window),
// so the 14-word rhs, P(1), metric and sigma of the stage update make no HBM
// round trip.
// A step with no finished row (the first of a segment) sends its 32 stores
// to an x ghost cell of rhs, which nothing reads; lanes past x's end write
// the x ghost cell next to the interior of U2, P2, R2 (and status).
template <int D, int RECON, bool CURVED, class R, bool SHIFT, bool DG, bool FUSE = false>
__global__ __launch_bounds__(64) void k_flux_w(const Params p, const double* __restrict__ P,
                                               const double* __restrict__ sig, double* __restrict__ rhs,
                                               int seglen, int nxb, int nseg, const FuseArgs fz = FuseArgs{}) {
    static_assert(!FUSE || D == 2, "the stage update follows the last sweep");
    constexpr int E = (D == 1) ? 2 : 1;                 // the other transverse dimension
    constexpr int NG = DG ? 3 : 6;                      // stored gamma_ij components
    // staging streams: sigma; alpha, gamma_ij (curved); beta^i (shift); an even count
    constexpr int NMS = CURVED ? ((2 + NG + (SHIFT ? 3 : 0) + 1) / 2 * 2) : 2;
    // one LDS object for the ring and the staging row: with two objects
    // filled by direct loads the wait-count pass makes every ring read wait
    // for all outstanding memory operations
    // (FUSE: the stage update's tally at the end of the same object)
    constexpr int NTAL = FUSE ? (int)((sizeof(StageTally) + 7) / 8) : 0;
    __shared__ double ring[WRING * NF * 64 + NMS * 64 + NTAL];
    double* const mst = ring + WRING * NF * 64;
    StageTally& tal = *reinterpret_cast<StageTally*>(ring + WRING * NF * 64 + NMS * 64);
    const int lane = threadIdx.x;
    const long wid = xcd_block();
    if (wid >= (long)nxb * p.n[E] * nseg) return;      // uniform per wave
    if (FUSE) {
        if (lane < 32) tal.hist[lane] = 0u;
        if (lane == 0) tal.fail = tal.atmo = 0u;
    }
    // stores of one step: rhs row c - 1, or the stage update's (update_cell)
    constexpr int NST = FUSE ? 32 : NF;
    // FUSE: U^n and R1 of row c - 1, loaded with rhs row c - 1
    constexpr int NUPD = FUSE ? NF + 3 : 0;
    const int xb = (int)(wid % nxb);
    const long r = wid / nxb;
    const int e = (int)(r % p.n[E]);
    const int seg = (int)(r / p.n[E]);
    const int i = xb * 64 + lane;
    const bool valid = i < p.n[0];                      // every lane takes part in the ring loads
    const int nD = p.n[D], gD = p.g[D];
    const int c0 = seg * seglen, c1 = min(c0 + seglen, nD);
    const long s = p.st[D], Np = p.Np;
    const long rowb = (long)(e + p.g[E]) * p.st[E];    // row offset without x and D
    const long base = rowb + (i < p.n[0] ? i : p.n[0] - 1) + p.g[0];
    // ring loads: lane m carries x pair 2(m mod 32) of field f + m / 32, clamped into the padded row
    const long xpair = min((long)p.g[0] + (long)xb * 64 + 2 * (lane & 31), (long)p.np[0] - 2);
    const int fhalf = lane >> 5;
    const R ih = R(p.idx[D]);
    const double cd = p.cdiff[D];
    auto slot = [&](int c) { return (c + gD) % WRING; };
    auto ringP = [&](int c, int f) -> double { return ring[(slot(c) * NF + f) * 64 + lane]; };
    // row c into its ring slot; r: the padded row it is read from (a ghost
    // row's interior image, the boundary conditions)
    auto load_ring = [&](int c, int r) {
        const double* src = P + (long)fhalf * Np + rowb + (long)r * s + xpair;
        double* dst = ring + slot(c) * NF * 64;
#pragma unroll
        for (int f = 0; f < NF; f += 2)
            __builtin_amdgcn_global_load_lds((const void*)(src + (long)f * Np),
                                             (__attribute__((address_space(3))) void*)(dst + f * 64), 16, 0, 0);
    };

    // metric and sigma window, index k <-> row c - 3 + k (k = 0..4).  Row c + 2
    // is loaded one step ahead into the LDS staging row (same lane layout as
    // the ring) and enters the window at the end of the next step, after the
    // wait that covers it.  (Loaded into registers, the row would be copied
    // into the window's registers right after its loads were issued, and the
    // copy would wait for every memory operation issued before it.)
    double wa[5], wb[SHIFT ? 5 : 1][3], wg[5][NG], ws[5];
    auto load_stage = [&](int c) {
        const long ro = rowb + (long)(c + gD) * s + xpair;
        const long rs = rowb + (long)bc_map(p, D, c + gD) * s + xpair;
        auto addr = [&](int k0) -> unsigned long long {
            // streams past the last one (an even count) repeat it
            constexpr int nvalid = 2 + NG + (SHIFT ? 3 : 0);
            const int k = k0 < nvalid ? k0 : nvalid - 1;
            const double* b = (!CURVED || k == 0) ? sig + rs
                            : k == 1 ? p.alp + ro
                            : k < 2 + NG ? p.gam + (long)gcomp<DG>(k - 2) * Np + ro
                                    : p.bet + (long)(k - 2 - NG) * Np + ro;
            return (unsigned long long)b;
        };
#pragma unroll
        for (int q = 0; q < NMS / 2; ++q) {
            // the lane's stream as an integer select (see the stage kernels)
            const unsigned long long a = addr(2 * q), b = addr(2 * q + 1);
            __builtin_amdgcn_global_load_lds((const void*)(fhalf ? b : a),
                                             (__attribute__((address_space(3))) void*)(mst + 2 * q * 64), 16, 0, 0);
        }
    };
    auto read_stage = [&](double& ar, double* br, double* gr, double& sr) {
        sr = mst[lane];
        if (CURVED) {
            ar = mst[64 + lane];
#pragma unroll
            for (int a = 0; a < NG; ++a) gr[a] = mst[(2 + a) * 64 + lane];
            if (SHIFT)
#pragma unroll
                for (int a = 0; a < 3; ++a) br[a] = mst[(2 + NG + a) * 64 + lane];
        }
    };
    auto bw = [&](int k, int a) { return SHIFT ? wb[SHIFT ? k : 0][a] : 0.0; };
    auto load_metric = [&](int c, double& ar, double* br, double* gr, double& sr) {
        const long o = base + (long)(c + gD) * s;
        sr = sig[o + (long)(bc_map(p, D, c + gD) - (c + gD)) * s];
        if (CURVED) {
            ar = p.alp[o];
            if (SHIFT)
                for (int a = 0; a < 3; ++a) br[a] = p.bet[a * Np + o];
#pragma unroll
            for (int a = 0; a < NG; ++a) gr[a] = p.gam[gcomp<DG>(a) * Np + o];
        }
    };
    // window of the first step (c = c0 - 1): P rows c0-3 .. c0+1, metric rows
    // c0-4 .. c0 (row c0-4 is outside the padding when c0 = 0 and unused),
    // staging row c0 + 1
    for (int c = c0 - 3; c <= c0 + 1; ++c) load_ring(c, bc_map(p, D, c + gD));
    load_stage(c0 + 1);
    for (int k = 0; k < 5; ++k) {
        const int c = c0 - 4 + k;
        wa[k] = 0.0;
        ws[k] = 0.0;
        double bdummy[3];
        double* bk = SHIFT ? wb[SHIFT ? k : 0] : bdummy;
        for (int a = 0; a < 3; ++a) bk[a] = 0.0;
        for (int a = 0; a < NG; ++a) wg[k][a] = 0.0;
        if (c >= -gD) load_metric(c, wa[k], bk, wg[k], ws[k]);
    }

    // every step issues the same memory operations in the same order (rhs
    // row c - 1 read; ring row c + 3; rhs row c - 1 written; staging row
    // c + 3), clamped or sent to a ghost cell where a step has nothing to do,
    // so the wait for a ring row can leave everything issued after it in flight
    constexpr int NMET = NMS / 2;
    const long odummy = rowb + p.g[0] - 1;               // an x ghost of rhs: written, never read
    // part: row c - 1 without its upper face, i.e. the lower face's flux over
    // dx (left by the previous step) plus the sources of c - 1
    R PLc[NF];
    double part[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) { PLc[f] = R(0); part[f] = 0.0; }
    double Jprev = 0.0;
    // everything of the first window has landed before the loop: on both ways
    // into the loop head the wait-count pass then sees the same loads pending
    wait_ring();
#pragma unroll 1
    for (int c = c0 - 1; c <= c1; ++c) {
        const int cnext = min(c + 3, nD + 2);           // row c + 3, clamped inside the padding
        const int rnext = bc_map(p, D, cnext + gD);     // the row it is read from
        const bool fin = c - 1 >= c0;                   // rhs of c - 1 is finished this step
        const long om = base + (long)(c - 1 + gD) * s;
        double acc[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f] = rhs[f * Np + om];
        // FUSE: the stage update's inputs of row c - 1 (U^n, R1) with them
        double un[FUSE ? NF : 1], r1v[FUSE ? 3 : 1];
        if constexpr (FUSE) {
#pragma unroll
            for (int f = 0; f < NF; ++f) un[f] = fz.Un[f * Np + om];
            for (int a = 0; a < 3; ++a) r1v[a] = fz.R1[a * Np + om];
        }
        // the sources go to the partial sum: acc is first used at the store,
        // so its loads have the whole step to land
        if (fin && CURVED) {
            // sources of c - 1: metric rows c-3 .. c+1 (window 0..4), P row c - 1
            Geo<double, DG> ms;
            ms.alp = wa[2];
            for (int a = 0; a < 3; ++a) ms.bet[a] = bw(2, a);
            for (int a = 0; a < NG; ++a) ms.g[gcomp<DG>(a)] = wg[2][a];
            geo_finish(ms);
            auto d4 = [&](double a0, double a1, double a3, double a4) { return (a0 - 8.0 * a1 + 8.0 * a3 - a4) * cd; };
            const double da = d4(wa[0], wa[1], wa[3], wa[4]);
            double db[3], dg[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            // (no shift: zero, not 0 * cd, which the compiler must keep)
            for (int a = 0; a < 3; ++a) db[a] = SHIFT ? d4(bw(0, a), bw(1, a), bw(3, a), bw(4, a)) : 0.0;
            for (int a = 0; a < NG; ++a) dg[gcomp<DG>(a)] = d4(wg[0][a], wg[1][a], wg[3][a], wg[4][a]);
            double Pm[NF], Um[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) Pm[f] = ringP(c - 1, f);
            prim2con(ms, p.G, Pm, Um);
            sources_dir<D>(p, ms, da, db, dg, Pm, Um, part);
        }
        __builtin_amdgcn_sched_barrier(0);
        // current of c (metric and sigma row c: window 3)
        double Jc;
        {
            Geo<double, DG> mc;
            if (CURVED) {
                mc.alp = wa[3];
                for (int a = 0; a < 3; ++a) mc.bet[a] = bw(3, a);
                for (int a = 0; a < NG; ++a) mc.g[gcomp<DG>(a)] = wg[3][a];
                geo_finish(mc);
            } else {
                geo_flat(mc);
            }
            double Pc[NF], J[3];
#pragma unroll
            for (int f = 0; f < NF; ++f) Pc[f] = ringP(c, f);
            current(mc, Pc, ws[3], J);
            Jc = J[D];
        }
        // ring row c + 2 (requested last step) must have landed; issued after
        // it: the last step's stores, staging row c + 2, rhs row c - 1 read
        // and the update's loads (at most 63 can be left in flight: waiting
        // for fewer is waiting longer)
        wait_vm<(NUPD + NST + NMET + NF < 63 ? NUPD + NST + NMET + NF : 63)>();
        // reconstruction of c
        R fm[NF], fp[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            // two fields in flight: the ring reads of f wait for field f - 2
            const int sl = f >= 2 ? after(0, fp[f - 2]) : 0;
            const R st[5] = {R(ringP(c - 2, f + sl)), R(ringP(c - 1, f + sl)), R(ringP(c, f + sl)),
                             R(ringP(c + 1, f + sl)), R(ringP(c + 2, f + sl))};
            recon<RECON>(st, fm[f], fp[f]);
        }
        // row c - 2 is consumed: request row c + 3 into its slot
        __builtin_amdgcn_sched_barrier(0);
        asm volatile("" ::: "memory");
        load_ring(cnext, rnext);
        {
            // (the first step's face is not needed: computed, and stored to the ghost cell)
            // face c - 1/2: metric at the face from rows c-2 .. c+1 (window 1..4)
            Geo<R, DG> m;
            if (CURVED) {
                auto f4 = [](double a0, double a1, double a2, double a3) {
                    return (-a0 + 9.0 * a1 + 9.0 * a2 - a3) * 0.0625;
                };
                m.alp = R(f4(wa[1], wa[2], wa[3], wa[4]));
                for (int a = 0; a < 3; ++a) m.bet[a] = R(f4(bw(1, a), bw(2, a), bw(3, a), bw(4, a)));
                for (int a = 0; a < NG; ++a) m.g[gcomp<DG>(a)] = R(f4(wg[1][a], wg[2][a], wg[3][a], wg[4][a]));
                geo_finish(m);
            } else {
                geo_flat(m);
            }
            // first-order fallback from the ring (rows c-1 and c are not the slot in flight)
            if (bad_state(m, PLc))
                for (int f = 0; f < NF; ++f) PLc[f] = R(ringP(c - 1, f));
            R PR[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) PR[f] = fm[f];
            if (bad_state(m, PR))
                for (int f = 0; f < NF; ++f) PR[f] = R(ringP(c, f));
            R Fh[NF];
            face_flux<D>(p, m, PLc, PR, R(0.5 * (Jprev + Jc)), Fh);
            // rhs row c - 1 (read at the top of the step, with the update's
            // loads) has landed once no more than the ring row c + 3 is in
            // flight behind it
            wait_vm<NF / 2>();
            const long os = (fin && valid) ? om : odummy + (long)(c - 1 + gD) * s;
            if constexpr (FUSE) {
                StageIn in;
                in.ok = fin && valid;
                in.o = os;
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const double fo = double(Fh[f] * ih);
                    in.rh[f] = acc[f] + (part[f] - fo);
                    part[f] = fo;
                    in.Un[f] = un[f];
                    in.P[f] = ringP(c - 1, f);
                }
                for (int a = 0; a < 3; ++a) in.R1[a] = r1v[a];
                in.sg = ws[2];
                in.a = wa[2];
                for (int a = 0; a < NG; ++a) in.g[gcomp<DG>(a)] = wg[2][a];
                // a step without a finished row stores to rhs's x ghost cell of
                // the row (its status to the dummy word); lanes past x's end
                // to the outputs' x ghost cell (the bases stay uniform)
                double* const Uo = fin ? fz.U2 : rhs;
                double* const Po = fin ? fz.P2 : rhs;
                double* const Ro = fin ? fz.R2 : rhs;
                int* const so = fin ? fz.status : fz.dummy;
                update_cell<2, CURVED, false, DG, false>(p, fz.dt, in, Uo, Po, Ro, nullptr, so,
                                                         fin ? fz.st_stride : 0L, tal, tal);
            } else {
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const double fo = double(Fh[f] * ih);
                    rhs[f * Np + os] = acc[f] + (part[f] - fo);
                    part[f] = fo;
                }
            }
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) PLc[f] = fp[f];
        Jprev = Jc;
        // advance the window by one row: the staging row (row c + 2, asked
        // for last step) has landed, since the wait before the stores above
        // left only the ring row c + 3 in flight; once it is read, row c + 3
        // is asked for in its place
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            ws[k] = ws[k + 1];
            if (CURVED) {
                wa[k] = wa[k + 1];
                if (SHIFT)
                    for (int a = 0; a < 3; ++a) wb[SHIFT ? k : 0][a] = wb[SHIFT ? k + 1 : 0][a];
                for (int a = 0; a < NG; ++a) wg[k][a] = wg[k + 1][a];
            }
        }
        {
            double bdummy[3];
            read_stage(wa[4], SHIFT ? wb[SHIFT ? 4 : 0] : bdummy, wg[4], ws[4]);
        }
        wait_lgkm0();                                   // the staging row is read before it is refilled
        load_stage(cnext);
    }
    // no ring load may be in flight when the wave ends
    wait_ring();
    if (FUSE) {
        // stage 2's histogram bins 32..63 and the failure count
        if (p.hist && lane < 32 && tal.hist[lane]) atomicAdd(p.hist + 32 + lane, (unsigned long long)tal.hist[lane]);
        if (lane == 0 && tal.fail) atomicAdd(fz.nfail, (unsigned long long)tal.fail);
    }
}

// ------------------------------------------------ metric set-up (one-time)
// flag := 1 if any of a[0..n) is non-zero (wave vote, one atomic per wave)
__global__ void k_any_nonzero(const double* __restrict__ a, long n, unsigned long long* flag) {
    bool nz = false;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
        nz = nz || a[t] != 0.0;
    if (__any(nz) && (threadIdx.x & 63) == 0) atomicOr(flag, 1ull);
}

// ---------------------------------------------------------------- ghost fill
// faces only: the ng ghost layers next to the interior along each active d,
// interior extents elsewhere; all active directions in one launch (the
// faces do not overlap: each copies interior-extent cells of its own d)
// (one thread per ghost cell and field: the copies are independent)
__host__ __device__ inline long ghost_count(const Params& p, int d) {
    if (!((p.active >> d) & 1)) return 0;
    const int e1 = (d == 0) ? 1 : 0, e2 = (d == 2) ? 1 : 2;
    return 2L * p.ng * p.n[e1] * p.n[e2];
}
// I: the index type of the decomposition (32-bit when the thread count fits:
// 64-bit division is a long instruction sequence on the GPU)
template <class I>
__global__ void k_ghost(const Params p, double* __restrict__ a, int nf) {
    I t = (I)((long)blockIdx.x * blockDim.x + threadIdx.x);
    int d = 0;
    I tot = (I)ghost_count(p, 0) * (I)nf;
    if (t >= tot) {
        t -= tot;
        d = 1;
        tot = (I)ghost_count(p, 1) * (I)nf;
        if (t >= tot) {
            t -= tot;
            d = 2;
            tot = (I)ghost_count(p, 2) * (I)nf;
            if (t >= tot) return;
        }
    }
    tot /= (I)nf;
    const int e1 = (d == 0) ? 1 : 0, e2 = (d == 2) ? 1 : 2;
    const I n1 = (I)p.n[e1], n2 = (I)p.n[e2];
    int f, a1, a2, layer;       // layer 0..2ng-1
    if (d == 0) {
        // x faces: the layers of one row next to each other (x is contiguous)
        const I nl = (I)(2 * p.ng);
        layer = (int)(t % nl);
        t /= nl;
        a1 = (int)(t % n1) + p.g[e1];
        t /= n1;
        a2 = (int)(t % n2) + p.g[e2];
        f = (int)(t / n2);
    } else {
        // y, z faces: x runs along the threads
        f = (int)(t / tot);
        t -= (I)f * tot;
        a1 = (int)(t % n1) + p.g[e1];
        t /= n1;
        a2 = (int)(t % n2) + p.g[e2];
        layer = (int)(t / n2);
    }
    const int c = layer < p.ng ? p.g[d] - p.ng + layer : p.g[d] + p.n[d] + layer - p.ng;
    const int src = bc_map(p, d, c);
    const long ob = (long)a1 * p.st[e1] + (long)a2 * p.st[e2];
    const long od = ob + (long)c * p.st[d], os = ob + (long)src * p.st[d];
    a[f * p.Np + od] = a[f * p.Np + os];
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

template <bool DG>
__device__ __forceinline__ void rec_setup(const Params& p, const Geo<double, DG>& m, const double* U,
                                          RecInT<double, DG>& k) {
    k.G = p.G;
    k.D = U[I_D];
    k.iD = frcp(k.D);          // used only when D > 0
    k.tau = U[I_TAU];
    for (int i = 0; i < 3; ++i) {
        k.S[i] = U[I_S + i];
        k.Bc[i] = U[I_B + i];
    }
    for (int a = 0; a < 6; ++a) { k.g[a] = m.g[a]; k.gi[a] = m.gi[a]; }
    k.sg = m.sg;
    k.isg = m.isg;
    lower(m, k.Bc, k.Bl);
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

// primitives at a recovered root from RecIn (D, Bcal) and the conserved
// cleaning and charge values cl = (Phi, Psi, Q) of the cell
template <bool DG>
__device__ __forceinline__ void write_prims_k(const Params& p, long o, const Geo<double, DG>& m,
                                              const RecInT<double, DG>& k,
                                              const double* cl, const double* x, const double* Ec, double* P) {
    const double* v = x + 1;
    double vl[3];
    lower(m, v, vl);
    const double W = frsqrt(1.0 - dot3(vl, v));
    P[I_RHO * p.Np + o] = k.D * m.isg / W;
    P[I_P * p.Np + o] = x[0];
    for (int i = 0; i < 3; ++i) {
        P[(I_V + i) * p.Np + o] = v[i];
        P[(I_B + i) * p.Np + o] = k.Bc[i] * m.isg;
        P[(I_E + i) * p.Np + o] = Ec[i] * m.isg;
    }
    for (int f = I_PHI; f < NF; ++f) P[f * p.Np + o] = cl[f - I_PHI] * m.isg;
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

// eq. GRRMHD_flux_form sources at a cell centre, E rows without R_E, split
// into the terms without metric derivatives (sources_local) and, for each
// direction d, the terms linear in d_d alpha, d_d beta^i, d_d gamma_ij
// (sources_dir<d>).  Every derivative term carries one derivative, so the sum
// over d of sources_dir plus sources_local is the whole source.  The flux
// kernel of direction d adds sources_dir<d> (its lanes hold the metric along
// d, so the derivative costs four lane shuffles per field); the stage kernels
// add sources_local.  R: double, or the dual type of the adjoint's passes.

// component i of gamma^ij A_j (i from an unrolled loop)
template <bool DG> __device__ __forceinline__ double raise1i(const Geo<double, DG>& m, int i, const double* A) {
    if constexpr (DG) return m.gi[sidx(i, i)] * A[i];
    else return m.gi[sidx(i, 0)] * A[0] + m.gi[sidx(i, 1)] * A[1] + m.gi[sidx(i, 2)] * A[2];
}

// densitised stress S^{jk} (both indices up) of a cell state
template <class R, bool DG>
__device__ __forceinline__ void stress_up(const Params& p, const Geo<double, DG>& m, const R* Pc, R* Su) {
    const R* v = Pc + I_V;
    const R* B = Pc + I_B;
    const R* E = Pc + I_E;
    R vl[3], Bl[3], El[3];
    lower(m, v, vl);
    lower(m, B, Bl);
    lower(m, E, El);
    const R W = frsqrt(R(1.0) - dot3(vl, v));
    const R hW2 = (Pc[I_RHO] + Pc[I_P] * (p.G / (p.G - 1.0))) * (W * W);
    const R pt = Pc[I_P] + (dot3(El, E) + dot3(Bl, B)) * 0.5;
    for (int j = 0; j < 3; ++j)
        for (int kk = j; kk < 3; ++kk) {
            if (zero_entry<DG>(sidx(j, kk)))
                Su[sidx(j, kk)] = (hW2 * v[j] * v[kk] - E[j] * E[kk] - B[j] * B[kk]) * m.sg;
            else
                Su[sidx(j, kk)] = (hW2 * v[j] * v[kk] - E[j] * E[kk] - B[j] * B[kk] + pt * m.gi[sidx(j, kk)]) * m.sg;
        }
}

// S = the terms without metric derivatives (K: extrinsic curvature, used if hasK)
template <bool CURVED, class R, bool DG>
__device__ __forceinline__ void sources_local(const Params& p, const Geo<double, DG>& m, const double (&K)[6], bool hasK,
                                              const R* Pc, const R* Uc, R* S) {
    const R* v = Pc + I_V;
    const double kap = p.kappa;
    for (int f = 0; f < NF; ++f) S[f] = R(0.0);
    if (!CURVED) {
        for (int i = 0; i < 3; ++i) S[I_E + i] = -(Uc[I_Q] * v[i]);
        S[I_PHI] = -(Uc[I_PHI] * kap);
        S[I_PSI] = Uc[I_Q] - Uc[I_PSI] * kap;
        return;
    }
    const double a = m.alp;
    double Ktr = 0.0;
    R SK = R(0.0);
    if (hasK) {
        R Su[6];
        stress_up(p, m, Pc, Su);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const double kij = K[sidx(i, j)];
                if (!zero_entry<DG>(sidx(i, j))) Ktr += m.gi[sidx(i, j)] * kij;
                SK += Su[sidx(i, j)] * kij;
            }
    }
    S[I_TAU] = SK * a;
    for (int i = 0; i < 3; ++i) S[I_E + i] = -(Uc[I_Q] * v[i] * a);
    S[I_PHI] = -(Uc[I_PHI] * (a * Ktr)) - Uc[I_PHI] * (a * kap);
    S[I_PSI] = -(Uc[I_PSI] * (a * Ktr)) + Uc[I_Q] * a - Uc[I_PSI] * (a * kap);
}

// S += the terms with the derivatives along d: da = d_d alpha, db[i] =
// d_d beta^i, dg[jk] = d_d gamma_jk.  Gamma^i = gamma^il A_l with
// A_l = gamma^jk d_j gamma_lk - 1/2 gamma^jk d_l gamma_jk.
// (DG: dg and the inverse metric are diagonal, their zero entries are skipped)
template <int d, class R, bool DG>
__device__ __forceinline__ void sources_dir(const Params& p, const Geo<double, DG>& m, double da, const double* db,
                                            const double* dg, const R* Pc, const R* Uc, R* S) {
    const double a = m.alp;
    R Su[6];
    stress_up(p, m, Pc, Su);
    // A_l restricted to the d-derivatives: gamma^dk dg[lk] - 1/2 delta_ld gamma^jk dg[jk]
    double A[3];
    double tr = 0.0;
    for (int j = 0; j < 3; ++j)
        for (int kk = 0; kk < 3; ++kk)
            if (!zero_entry<DG>(sidx(j, kk))) tr += m.gi[sidx(j, kk)] * dg[sidx(j, kk)];
    for (int l = 0; l < 3; ++l) {
        double s1 = 0.0;
        for (int kk = 0; kk < 3; ++kk)
            if (!zero_entry<DG>(sidx(d, kk)) && !zero_entry<DG>(sidx(l, kk))) s1 += m.gi[sidx(d, kk)] * dg[sidx(l, kk)];
        A[l] = s1 - (l == d ? 0.5 * tr : 0.0);
    }
    const R* Sl = Uc + I_S;
    R t = R(0.0);
    for (int j = 0; j < 3; ++j)
        for (int kk = 0; kk < 3; ++kk)
            if (!zero_entry<DG>(sidx(j, kk))) t += Su[sidx(j, kk)] * dg[sidx(j, kk)];
    S[I_S + d] += t * (0.5 * a) + (Sl[0] * db[0] + Sl[1] * db[1] + Sl[2] * db[2]) - (Uc[I_TAU] + Uc[I_D]) * da;
    const R Supd = raise1<d>(m, Sl);
    S[I_TAU] += -(Supd * da);
    for (int i = 0; i < 3; ++i) {
        const double Gm = raise1i(m, i, A);
        const double gg = zero_entry<DG>(sidx(i, d)) ? -(a * Gm) : m.gi[sidx(i, d)] * da - a * Gm;
        S[I_B + i] += Uc[I_PHI] * gg - Uc[I_B + d] * db[i];
        S[I_E + i] += Uc[I_PSI] * gg - Uc[I_E + d] * db[i];
    }
    S[I_PHI] += Uc[I_B + d] * da;
    S[I_PSI] += Uc[I_E + d] * da;
}

// whole source at a cell centre from its metric derivatives
template <bool CURVED, class R>
__device__ __forceinline__ void sources_t(const Params& p, const Geo<double>& m, const MetricDerivs& md,
                                          const R* Pc, const R* Uc, R* S) {
    sources_local<CURVED>(p, m, md.K, p.K != nullptr, Pc, Uc, S);
    if (!CURVED) return;
    sources_dir<0>(p, m, md.da[0], md.db[0], md.dg[0], Pc, Uc, S);
    sources_dir<1>(p, m, md.da[1], md.db[1], md.dg[1], Pc, Uc, S);
    sources_dir<2>(p, m, md.da[2], md.db[2], md.dg[2], Pc, Uc, S);
}

// --------------------------------------------------------------- stages
// ---------------------------------------------------------- stage kernels
// Persistent: one wave per SIMD (the recovery's register footprint allows no
// more) walks 64-cell chunks q, q + W, ...; the loads of the next chunk are
// in flight while the current chunk's recovery runs.

// Inputs of a stage kernel as a list of streams (array, field), each one
// [Np] row of doubles.  STAGE 1: U^n, the (p, v) guess, sigma, metric;
// 2: + P(1), rhs, R1, K; 3: P(2), U^n, U(2), rhs, R1, R2, metric, K;
// 4 (the final update followed by the next step's stage 1): 3 + sigma.
// Without K the local sources need only v and the densitised cleaning fields
// of the stage state, which are U^n's (stage 2: stage 1 leaves them as they
// are) or U(2)'s (final update), and the guess p and v: of P_s only p and v
// are loaded.
enum : int { SA_UN, SA_US, SA_PS, SA_R1, SA_R2, SA_RHS, SA_SIG, SA_ALP, SA_GAM, SA_K };
struct StreamList {
    int n;
    int s[80];                                   // array * 32 + field
};
template <int STAGE, bool CURVED, bool HASK, bool DG> __host__ __device__ constexpr StreamList stage_streams() {
    StreamList L{0, {}};
    auto add = [&L](int a, int f) { L.s[L.n++] = a * 32 + f; };
    for (int f = 0; f < NF; ++f) add(SA_UN, f);
    if (STAGE == 1) {
        for (int f = I_P; f < I_V + 3; ++f) add(SA_PS, f);
    } else {
        if (HASK) {
            for (int f = 0; f < NF; ++f) add(SA_PS, f);
        } else {
            for (int f = I_P; f < I_V + 3; ++f) add(SA_PS, f);
        }
        for (int f = 0; f < NF; ++f) add(SA_RHS, f);
        for (int i = 0; i < 3; ++i) add(SA_R1, i);
    }
    if (STAGE >= 3) {
        for (int f = 0; f < NF; ++f) add(SA_US, f);
        for (int i = 0; i < 3; ++i) add(SA_R2, i);
    }
    if (STAGE != 3) add(SA_SIG, 0);
    if (CURVED) {
        add(SA_ALP, 0);
        for (int a = 0; a < 6; ++a)
            if (!zero_entry<DG>(a)) add(SA_GAM, a);
        if (STAGE != 1 && HASK)
            for (int a = 0; a < 6; ++a) add(SA_K, a);
    }
    if (L.n & 1) add(L.s[L.n - 1] / 32, L.s[L.n - 1] % 32);   // even: two streams per load instruction
    return L;
}
// position of stream (a, f) in the list (-1: not there)
template <int STAGE, bool CURVED, bool HASK, bool DG> __device__ constexpr int stream_pos(int a, int f) {
    constexpr StreamList L = stage_streams<STAGE, CURVED, HASK, DG>();
    for (int i = 0; i < L.n; ++i)
        if (L.s[i] == a * 32 + f) return i;
    return -1;
}

struct StageArrays {
    const double *Un, *Us, *Ps, *R1, *R2, *rhs, *sig;
};
__device__ __forceinline__ const double* stream_ptr(const Params& p, const StageArrays& A, int s) {
    const int a = s / 32, f = s % 32;
    const double* b = a == SA_UN ? A.Un : a == SA_US ? A.Us : a == SA_PS ? A.Ps : a == SA_R1 ? A.R1
                    : a == SA_R2 ? A.R2 : a == SA_RHS ? A.rhs : a == SA_SIG ? A.sig : a == SA_ALP ? p.alp
                    : a == SA_GAM ? p.gam : p.K;
    return b + (long)f * p.Np;
}


// A chunk is 64 consecutive cells of one interior x row: chunk q is segment
// q mod nsx of row q / nsx (rows y fastest, then z).
struct Chunk {
    long orow;     // padded offset of the row's first interior cell
    int x0;        // interior x of the chunk's first cell
};
__device__ __forceinline__ Chunk chunk_at(const Params& p, long q, int nsx) {
    // 32-bit: fewer than 2^31 chunks (the x-sweep bound on the descriptor covers it)
    const unsigned uq = (unsigned)q, r = uq / (unsigned)nsx;
    const int seg = (int)(uq - r * (unsigned)nsx);
    const unsigned j = r % (unsigned)p.n[1], k = r / (unsigned)p.n[1];
    return Chunk{((long)k + p.g[2]) * p.st[2] + ((long)j + p.g[1]) * p.st[1] + p.g[0], seg * 64};
}

// Ask for chunk c's streams straight into the wave's LDS buffer
// (global_load_lds_dwordx4: lane m brings cells 2(m mod 32), +1 of stream
// 2i + m / 32; the pair is clamped inside the padded row, a pair past the
// row's end is never read).
template <int STAGE, bool CURVED, bool HASK, bool DG>
__device__ __forceinline__ void stage_issue(const Params& p, const StageArrays& A, const Chunk& c, double* buf,
                                            int lane) {
    constexpr StreamList L = stage_streams<STAGE, CURVED, HASK, DG>();
    const long xp = min((long)(c.x0 + 2 * (lane & 31)), (long)(p.np[0] - 2 - p.g[0]));
    const long oo = c.orow + xp;
    const bool hi = lane >= 32;
#pragma unroll
    for (int i = 0; i < L.n / 2; ++i) {
        // select the lane's stream as an integer (a select of two pointers
        // may be lowered through a stack slot)
        const unsigned long long a = (unsigned long long)stream_ptr(p, A, L.s[2 * i]);
        const unsigned long long b = (unsigned long long)stream_ptr(p, A, L.s[2 * i + 1]);
        const double* src = (const double*)(hi ? b : a) + oo;
        __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)(buf + 2 * i * 64),
                                         16, 0, 0);
    }
}

// The lane's inputs from the LDS buffer.  A lane past the row's end reads the
// row's last cell (ok = false): it repeats that cell's arithmetic and stores.
template <int STAGE, bool CURVED, bool HASK, bool DG>
__device__ __forceinline__ void stage_read(const Params& p, const Chunk& c, const double* buf, int lane, StageIn& in) {
    in.ok = c.x0 + lane < p.n[0];
    const int lc = in.ok ? lane : p.n[0] - 1 - c.x0;
    in.o = c.orow + c.x0 + lc;
    auto rd = [&](int a, int f) -> double {
        const int i = stream_pos<STAGE, CURVED, HASK, DG>(a, f);
        return i < 0 ? 0.0 : buf[i * 64 + lc];
    };
#pragma unroll
    for (int f = 0; f < NF; ++f) in.Un[f] = rd(SA_UN, f);
#pragma unroll
    for (int f = 0; f < NF; ++f) in.P[f] = rd(SA_PS, f);
    if (STAGE != 1) {
#pragma unroll
        for (int f = 0; f < NF; ++f) in.rh[f] = rd(SA_RHS, f);
        for (int i = 0; i < 3; ++i) in.R1[i] = rd(SA_R1, i);
    }
    if (STAGE >= 3) {
#pragma unroll
        for (int f = 0; f < NF; ++f) in.Us[f] = rd(SA_US, f);
        for (int i = 0; i < 3; ++i) in.R2[i] = rd(SA_R2, i);
    }
    if (STAGE != 3) in.sg = rd(SA_SIG, 0);
    if (CURVED) {
        in.a = rd(SA_ALP, 0);
        for (int a = 0; a < 6; ++a) in.g[a] = rd(SA_GAM, a);
        if (STAGE != 1 && HASK)
            for (int a = 0; a < 6; ++a) in.K[a] = rd(SA_K, a);
    }
}

// (the shift enters the stage kernels nowhere: the flux kernels carry it)
template <bool CURVED, bool DG> __device__ __forceinline__ void stage_geo(const StageIn& in, Geo<double, DG>& m) {
    if (CURVED) {
        m.alp = in.a;
        for (int a = 0; a < 3; ++a) m.bet[a] = 0.0;
        for (int a = 0; a < 6; ++a)
            if (!zero_entry<DG>(a)) m.g[a] = in.g[a];
        geo_finish(m);
    } else {
        geo_flat(m);
    }
}

// stage 1: E(1) = E^n + gamma dt R_E(U(1)), everything else unchanged.  A
// failed cell (flagged in status and the failure count) is written as the
// primitives of U^n at the guess's p and v with E = E^n.
template <bool CURVED, bool DG>
__device__ __forceinline__ void stage1_cell(const Params& p, double dt, const StageIn& in, double* __restrict__ P1,
                                            double* __restrict__ R1, double* __restrict__ U1,
                                            int* __restrict__ status, long st_stride, StageTally& tal) {
    const long Np = p.Np, o = in.o;
    Geo<double, DG> m;
    stage_geo<CURVED>(in, m);
    RecInT<double, DG> k;
    rec_setup(p, m, in.Un, k);
    for (int i = 0; i < 3; ++i) k.Es[i] = in.Un[I_E + i];
    if (U1)
        for (int f = 0; f < NF; ++f)
            if (f < I_E || f >= I_E + 3) U1[f * Np + o] = in.Un[f];
    const double gdt = GAM_IMEX() * dt;
    k.cfac = gdt * m.alp * (p.sig_model ? sigma_of_D(p, in.Un[I_D]) : in.sg);
    double x[4] = {in.P[I_P], in.P[I_V], in.P[I_V + 1], in.P[I_V + 2]};
    double E[3] = {k.Es[0], k.Es[1], k.Es[2]};
    int it, st;
    __builtin_amdgcn_sched_barrier(0);
    if (k.cfac != 0.0) st = recover_stiff(k, x, E, p.tol, p.tolq, p.maxit, &it);
    else st = recover_plain(k, E, x, p.tol, p.maxit, &it);
    __builtin_amdgcn_sched_barrier(0);
    tally_cell(tal, p.hist != nullptr, in.ok, st, it);
    if (st < 0) {
        x[0] = in.P[I_P];
        for (int i = 0; i < 3; ++i) { x[1 + i] = in.P[I_V + i]; E[i] = k.Es[i]; }
    }
    write_prims_k(p, o, m, k, in.Un + I_PHI, x, E, P1);
    for (int i = 0; i < 3; ++i) R1[i * Np + o] = (E[i] - k.Es[i]) / gdt;
    if (U1)
        for (int i = 0; i < 3; ++i) U1[(I_E + i) * Np + o] = E[i];
    status[st_stride * o] = st;
}

// stage 2 (STAGE = 2) and the final update (STAGE = 3), after the flux
// divergence (with the metric-derivative sources) of P_s is in rhs.
// STAGE = 4: the final update, then the next step's stage 1 on U^{n+1}
// guessed from P^{n+1} into P1o and Ro (to rounding, the results of stage1_cell on the
// stored U^{n+1} and P^{n+1}: the same recovery on the same inputs, which the
// plain recovery's setup already holds), tallied in tal1.
template <int STAGE, bool CURVED, bool HASK, bool DG, bool MODEL>
__device__ __forceinline__ void update_cell(const Params& p, double dt, const StageIn& in, double* __restrict__ Uo,
                                            double* __restrict__ Po, double* __restrict__ Ro,
                                            double* __restrict__ P1o, int* __restrict__ status, long st_stride,
                                            StageTally& tal, StageTally& tal1) {
    const long Np = p.Np, o = in.o;
    Geo<double, DG> m;
    stage_geo<CURVED>(in, m);
    const double g = GAM_IMEX();
    RecInT<double, DG> k;
    double x[4] = {in.P[I_P], in.P[I_V], in.P[I_V + 1], in.P[I_V + 2]};
    double cl[3];
    double YD;
    bool atmo = false;
    {
        double Y[NF];
        {
            double Uc[NF], S[NF];
            if (HASK) {
                prim2con(m, p.G, in.P, Uc);
            } else {
                // the densitised cleaning fields of the stage state, all the
                // local sources read besides v: U^n's in stage 2 (U(1) differs
                // from U^n in E only), U(2)'s in the final update
                for (int f = I_PHI; f < NF; ++f) Uc[f] = STAGE == 2 ? in.Un[f] : in.Us[f];
            }
            sources_local<CURVED>(p, m, in.K, CURVED && HASK, in.P, Uc, S);
            if (STAGE == 2) {
                for (int f = 0; f < NF; ++f) Y[f] = in.Un[f] + dt * (in.rh[f] + S[f]);
            } else {
                // U^{n+1} = (U^n + U(2))/2 + dt/2 F(U(2)) + dt/2 (2 gamma R1 + (1 - gamma) R2) on E
                for (int f = 0; f < NF; ++f) Y[f] = 0.5 * (in.Un[f] + in.Us[f]) + 0.5 * dt * (in.rh[f] + S[f]);
                for (int i = 0; i < 3; ++i) Y[I_E + i] += 0.5 * dt * (2.0 * g * in.R1[i] + (1.0 - g) * in.R2[i]);
            }
        }
        if (STAGE >= 3 && p.rho_atmo > 0.0 && Y[I_D] < ATMO_FACTOR * m.sg * p.rho_atmo) {
            // artificial atmosphere (Sec. IV.E): the hydro part of the state
            // rho_atmo, v = 0, p_atmo with the cell's own fields
            double Pa[NF], Ua[NF];
            Pa[I_RHO] = p.rho_atmo;
            Pa[I_P] = p.p_atmo;
            for (int i = 0; i < 3; ++i) Pa[I_V + i] = 0.0;
            for (int f = I_B; f < NF; ++f) Pa[f] = Y[f] * m.isg;
            prim2con(m, p.G, Pa, Ua);
            for (int f = I_D; f <= I_TAU; ++f) Y[f] = Ua[f];
            atmo = true;
        }
        YD = Y[I_D];
        __builtin_amdgcn_sched_barrier(0);
        for (int f = 0; f < NF; ++f)
            if (STAGE >= 3 || f < I_E || f >= I_E + 3) Uo[f * Np + o] = Y[f];
        rec_setup(p, m, Y, k);
        for (int i = 0; i < 3; ++i) cl[i] = Y[I_PHI + i];
        if (STAGE == 2)
            for (int i = 0; i < 3; ++i) k.Es[i] = Y[I_E + i] + dt * (1.0 - 2.0 * g) * in.R1[i];
        else
            for (int i = 0; i < 3; ++i) k.Es[i] = Y[I_E + i];
    }
    __builtin_amdgcn_sched_barrier(0);
    double E[3] = {k.Es[0], k.Es[1], k.Es[2]};
    int it, st;
    if (STAGE == 2) {
        k.cfac = g * dt * m.alp * ((MODEL && p.sig_model) ? sigma_of_D(p, YD) : in.sg);
        if (k.cfac != 0.0) st = recover_stiff(k, x, E, p.tol, p.tolq, p.maxit, &it);
        else st = recover_plain(k, E, x, p.tol, p.maxit, &it);
    } else {
        st = recover_plain(k, E, x, p.tol, p.maxit, &it);
    }
    __builtin_amdgcn_sched_barrier(0);
    tally_cell(tal, p.hist != nullptr, in.ok, st, it);
    if (STAGE >= 3 && atmo && st >= 0) {
        st = 2;                                           // flagged: atmosphere
        if (in.ok) atomicAdd(&tal.atmo, 1u);
    }
    if (st < 0) {
        // failed (flagged): the primitives of the stage state at the guess's
        // p and v with E = E*; every store below is taken on every path
        x[0] = in.P[I_P];
        for (int i = 0; i < 3; ++i) { x[1 + i] = in.P[I_V + i]; E[i] = k.Es[i]; }
    }
    write_prims_k(p, o, m, k, cl, x, E, Po);
    if (STAGE == 2) {
        for (int i = 0; i < 3; ++i) {
            Uo[(I_E + i) * Np + o] = E[i];
            Ro[i * Np + o] = (E[i] - k.Es[i]) / (g * dt);
        }
    }
    if (STAGE != 4) status[st_stride * o] = st;
    if (STAGE == 4) {
        // stage 1 of the next step: E(1) = E^{n+1} + gamma dt R_E(U(1)); a
        // failed cell keeps the guess and E^{n+1}, as in stage1_cell
        __builtin_amdgcn_sched_barrier(0);
        const double gdt = g * dt;
        k.cfac = gdt * m.alp * ((MODEL && p.sig_model) ? sigma_of_D(p, YD) : in.sg);
        const double xg[4] = {x[0], x[1], x[2], x[3]};
        double E1[3] = {k.Es[0], k.Es[1], k.Es[2]};
        int it1, st1;
        if (k.cfac != 0.0) st1 = recover_stiff(k, x, E1, p.tol, p.tolq, p.maxit, &it1);
        else st1 = recover_plain(k, E1, x, p.tol, p.maxit, &it1);
        __builtin_amdgcn_sched_barrier(0);
        tally_cell(tal1, p.hist != nullptr, in.ok, st1, it1);
        if (st1 < 0)
            for (int i = 0; i < 4; ++i) x[i] = xg[i];
        if (st1 < 0)
            for (int i = 0; i < 3; ++i) E1[i] = k.Es[i];
        write_prims_k(p, o, m, k, cl, x, E1, P1o);
        for (int i = 0; i < 3; ++i) Ro[i * Np + o] = (E1[i] - k.Es[i]) / gdt;
        status[st_stride * o] = st1;
    }
}

// stores of one chunk per lane: every one is taken on every path
template <int STAGE> constexpr int stage_stores() {
    return STAGE == 1 ? 18 : (STAGE == 2 ? 32 : (STAGE == 3 ? 29 : 28 + 18));
}

// STAGE 1: stage1_cell (Us, R2, rhs unused; Ps = the guess, Uo = U1, Ro = R1)
// STAGE 2, 3: update_cell.  STAGE 4: update_cell's final update with the next
// step's stage 1 (Ro = R1 of the next step, which may be the R1 read here:
// each cell's inputs are in LDS before its stores; P1o = its P(1)).  HASK:
// nonzero extrinsic curvature.  status is written at status[st_stride * o]
// (st_stride 0: one dummy word; STAGE 4 writes only its stage 1's status).
// Persistent, one wave per block (and per SIMD: the recovery's registers
// allow no more), walking chunks q, q + W, ...  The next chunk's inputs are
// loaded into the wave's LDS buffer while the current chunk (read from it
// into registers first) is computed and stored; the wait for them leaves the
// current chunk's stores in flight (stage 1 stores 18 or 32 per chunk, so
// waiting for 18 is safe in both cases).  Uo may be Un (the final update in
// place) and Ro may be R1 (STAGE 4), so those four are not restrict.
template <int STAGE, bool CURVED, bool HASK, bool DG>
__global__ __launch_bounds__(64) void k_stage(const Params p, double dt, const double* __restrict__ sig,
                                              const double* Un, const double* __restrict__ Us,
                                              const double* __restrict__ Ps, const double* R1,
                                              const double* __restrict__ R2, const double* __restrict__ rhs,
                                              double* Uo, double* __restrict__ Po,
                                              double* Ro, double* __restrict__ P1o, int* __restrict__ status,
                                              long st_stride, unsigned long long* nfail) {
    constexpr int NS = stage_streams<STAGE, CURVED, HASK, DG>().n;
    static_assert(NS <= 80 && NS % 2 == 0, "stream list");
    __shared__ double buf[NS * 64];
    __shared__ StageTally tal, tal1;
    const int lane = threadIdx.x;
    if (lane < 32) tal.hist[lane] = tal1.hist[lane] = 0u;
    if (lane == 0) tal.fail = tal.atmo = tal1.fail = tal1.atmo = 0u;
    const int nsx = (p.n[0] + 63) / 64;
    const long nchunk = (long)nsx * p.n[1] * p.n[2];
    const long W = gridDim.x;
    const StageArrays A{Un, Us, Ps, R1, R2, rhs, sig};
    // consecutive chunks on one XCD (shared cache lines at chunk ends)
    long q = xcd_block();
    if (q < nchunk) {                                          // uniform per wave
        Chunk c = chunk_at(p, q, nsx);
        stage_issue<STAGE, CURVED, HASK, DG>(p, A, c, buf, lane);
        wait_vm<0>();
        for (;;) {
            StageIn in;
            stage_read<STAGE, CURVED, HASK, DG>(p, c, buf, lane, in);
            wait_lgkm0();                                      // the buffer is free again
            const long qn = q + W;
            const Chunk cn = chunk_at(p, qn < nchunk ? qn : q, nsx);
            // unconditional (the last pass reloads its own chunk)
            stage_issue<STAGE, CURVED, HASK, DG>(p, A, cn, buf, lane);
            if (STAGE == 1) stage1_cell<CURVED, DG>(p, dt, in, Po, Ro, Uo, status, st_stride, tal);
            else update_cell<STAGE, CURVED, HASK, DG>(p, dt, in, Uo, Po, Ro, P1o, status, st_stride, tal, tal1);
            // the loads above were followed by this chunk's stores only
            wait_vm<stage_stores<STAGE>()>();
            if (qn >= nchunk) break;
            q = qn;
            c = cn;
        }
        wait_vm<0>();                                          // no load into LDS in flight at the end
    }
    __syncthreads();
    // histogram bins: stage 1 0..31, stage 2 32..63, final 64..95
    if (p.hist && lane < 32 && tal.hist[lane])
        atomicAdd(p.hist + 32 * (STAGE == 4 ? 2 : STAGE - 1) + lane, (unsigned long long)tal.hist[lane]);
    if (STAGE == 4 && p.hist && lane < 32 && tal1.hist[lane])
        atomicAdd(p.hist + lane, (unsigned long long)tal1.hist[lane]);
    if (lane == 0 && tal.fail + tal1.fail) atomicAdd(nfail, (unsigned long long)(tal.fail + tal1.fail));
    // nfail[4]: cells set to the atmosphere (the context's counter block)
    if (STAGE >= 3 && lane == 0 && tal.atmo) atomicAdd(nfail + 4, (unsigned long long)tal.atmo);
}

// conductivity model at the interior cells from the primitives P (D =
// sqrt(gamma) rho W), for the charge flux of the stage operator
template <bool CURVED>
__global__ __launch_bounds__(256) void k_sigma_field(const Params p, const double* __restrict__ P,
                                                     double* __restrict__ out) {
    long o;
    if (!interior_cell(p, (long)blockIdx.x * blockDim.x + threadIdx.x, o)) return;
    Geo<double> m;
    cell_geo<CURVED>(p, o, m);
    const double v[3] = {P[I_V * p.Np + o], P[(I_V + 1) * p.Np + o], P[(I_V + 2) * p.Np + o]};
    double vl[3];
    lower(m.g, v, vl);
    const double W = frsqrt(1.0 - dot3(vl, v));
    out[o] = sigma_of_D(p, P[I_RHO * p.Np + o] * W * m.sg);
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
