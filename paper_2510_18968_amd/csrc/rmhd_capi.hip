// Host side of the C ABI declared in include/rmhd.h: argument checks,
// workspace carving and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "rmhd.h"
#include "rmhd_adjoint.hpp"

using namespace rmhd;

struct rmhd_ctx {
    rmhd_grid_desc desc;
    Params p;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    double *rhs, *P1, *R1, *U2, *P2, *R2;
    double* sigf;                   // conductivity-model field of the stage primitives (models only)
    unsigned long long* counters;   // [0] failed recoveries, [1] max signal speed bits, [2] metric scan flag,
                                    // [3] dummy status word, [4] atmosphere cells;
                                    // [32..127] recovery iteration histograms
    bool curved;
    bool diag = false;              // curved with gamma_xy = gamma_xz = gamma_yz = 0 everywhere
    int device = 0;                 // the device current at rmhd_init_grid
    void* scratch = nullptr;        // that device's copy of the static adjoint scratch (or null)
    std::string scratch_err;        // why it could not be resolved
    long persist_blocks = 256;   // persistent flux grid: one 4-wave block per CU, multiple of 8
    // opt-in launch timing: event pairs per kernel class, reused after a read
    bool timing = false;
    bool timing_err = false;   // an event could not be created or recorded since the last read
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[RMHD_TIMING_CLASSES];
    size_t used[RMHD_TIMING_CLASSES] = {};
};

// Scratch of rmhd_step_adjoint_static: the adjoint workspace for callers that
// cannot allocate device memory.  One copy per device, held until the process
// ends; every call on a device shares it.
__device__ __align__(256) char scratch[RMHD_STATIC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return fail(RMHD_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define LAUNCH_CHECK()                                                                             \
    do {                                                                                           \
        hipError_t e_ = hipGetLastError();                                                         \
        if (e_ != hipSuccess) return fail(RMHD_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t ALIGN = 256;
size_t up(size_t b) { return (b + ALIGN - 1) / ALIGN * ALIGN; }

// Device addresses of the static adjoint scratch, one per device (each device
// holds its own copy of the array, at its own address).  In host code the
// array's name is only a host-side stand-in, so kernels get these addresses.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[MAX_DEVICES] = {};

// the address of `scratch` on device dev, which must be the current device
int resolve_scratch(int dev, void** out, std::string& why);

// padding on each side of dimension k: the ghost width on active dimensions,
// X_ALIGN_PAD along an active x with x_align (interior rows on 128-byte lines)
constexpr int X_ALIGN_PAD = 16;
int pad_lo(const rmhd_grid_desc* d, int k) {
    if (!((d->active_mask >> k) & 1)) return 0;
    return (k == 0 && d->x_align) ? X_ALIGN_PAD : d->ng;
}

bool check_desc(const rmhd_grid_desc* d, std::string& why) {
    if (!d) { why = "null descriptor"; return false; }
    if (d->ng != 3) { why = "ng must be 3"; return false; }
    if (d->active_mask < 1 || d->active_mask > 7 || !(d->active_mask & 1)) {
        why = "active_mask must include x (bit 0) and lie in 1..7";
        return false;
    }
    for (int k = 0; k < 3; ++k) {
        const bool act = (d->active_mask >> k) & 1;
        if (d->n[k] < 1) { why = "n[d] must be >= 1"; return false; }
        if (act && d->n[k] < 3) { why = "active dimensions need n[d] >= 3"; return false; }
        if (act && !(d->dx[k] > 0.0)) { why = "dx[d] must be > 0 on active dimensions"; return false; }
        if (act && d->bc[k] != RMHD_BC_PERIODIC && d->bc[k] != RMHD_BC_COPY) { why = "bad bc"; return false; }
        if (d->n[k] > (1 << 20)) { why = "n[d] too large"; return false; }
    }
    if (d->recon < RMHD_RECON_MINMOD || d->recon > RMHD_RECON_WENO5) { why = "bad recon"; return false; }
    if (d->precision != RMHD_PREC_FP64 && d->precision != RMHD_PREC_MIXED) { why = "bad precision"; return false; }
    if (!(d->gamma_ad > 1.0)) { why = "gamma_ad must be > 1"; return false; }
    if (!(d->kappa >= 0.0)) { why = "kappa must be >= 0"; return false; }
    if (!(d->c2p_tol > 0.0) || d->c2p_maxit < 1) { why = "bad recovery tolerance or cap"; return false; }
    if (d->speed_mode != 0 && d->speed_mode != 1) { why = "bad speed_mode"; return false; }
    if (d->x_align != 0 && d->x_align != 1) { why = "x_align must be 0 or 1"; return false; }
    if (d->sigma_model < RMHD_SIGMA_FIELD || d->sigma_model > RMHD_SIGMA_DYNAMO) { why = "bad sigma_model"; return false; }
    if (d->sigma_model != RMHD_SIGMA_FIELD &&
        !(d->sigma0 >= 0.0 && d->sigma0 < 1e300 && d->sigma_exp > -1e300 && d->sigma_exp < 1e300 &&
          d->sigma_Datmo >= 0.0 && d->sigma_Datmo < 1e300)) {
        why = "conductivity model: sigma0 and sigma_Datmo must be >= 0 and finite, sigma_exp finite";
        return false;
    }
    if (!(d->rho_atmo >= 0.0 && d->rho_atmo < 1e300) || !(d->K_atmo >= 0.0 && d->K_atmo < 1e300)) {
        why = "rho_atmo and K_atmo must be >= 0 and finite";
        return false;
    }
    long np = 1;
    for (int k = 0; k < 3; ++k) np *= d->n[k] + 2 * pad_lo(d, k);
    if (np > (1L << 36)) { why = "grid too large"; return false; }
    // the x sweep indexes the rows with their ghost cells in 32 bits
    if ((long)(d->n[0] + 6) * d->n[1] * d->n[2] + 64 > (1L << 31) - 1) { why = "grid too large"; return false; }
    return true;
}

long padded_cells(const rmhd_grid_desc* d) {
    long np = 1;
    for (int k = 0; k < 3; ++k) np *= d->n[k] + 2 * pad_lo(d, k);
    return np;
}

size_t ws_layout(const rmhd_grid_desc* d, size_t off[8]) {
    const size_t Np = (size_t)padded_cells(d);
    const size_t f14 = up(14 * Np * sizeof(double)), f3 = up(3 * Np * sizeof(double));
    size_t o = 0;
    off[0] = o; o += f14;   // rhs
    off[1] = o; o += f14;   // P1
    off[2] = o; o += f3;    // R1
    off[3] = o; o += f14;   // U2
    off[4] = o; o += f14;   // P2
    off[5] = o; o += f3;    // R2
    off[6] = o; o += d->sigma_model != RMHD_SIGMA_FIELD ? up(Np * sizeof(double)) : 0;   // model sigma field
    off[7] = o; o += 4 * ALIGN; // counters: 32 words, then the 96 histogram bins
    return o;
}

long ncells(const Params& p) { return (long)p.n[0] * p.n[1] * p.n[2]; }

enum { T_GHOST = 0, T_FX = 1, T_FY = 2, T_FZ = 3, T_UPD2 = 4, T_UPD3 = 5, T_STAGE1 = 6, T_OTHER = 7, T_FZU = 8 };

// brackets one launch with events when timing is on
struct Timed {
    rmhd_ctx* c;
    int cls;
    hipEvent_t stop = nullptr;
    Timed(rmhd_ctx* c_, int cls_) : c(c_), cls(cls_) {
        if (!c->timing) return;
        auto& v = c->ev[cls];
        if (c->used[cls] == v.size()) {
            hipEvent_t a = nullptr, b = nullptr;
            if (hipEventCreate(&a) != hipSuccess) { c->timing_err = true; return; }
            if (hipEventCreate(&b) != hipSuccess) {
                (void)hipEventDestroy(a);
                c->timing_err = true;
                return;
            }
            v.emplace_back(a, b);
        }
        auto& pr = v[c->used[cls]];
        if (hipEventRecord(pr.first, c->stream) != hipSuccess) { c->timing_err = true; return; }
        ++c->used[cls];
        stop = pr.second;
    }
    ~Timed() {
        if (stop && hipEventRecord(stop, c->stream) != hipSuccess) c->timing_err = true;
    }
};
unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

int ghost_fill(rmhd_ctx* c, double* a, int nf) {
    const Params& p = c->p;
    const long tot = (ghost_count(p, 0) + ghost_count(p, 1) + ghost_count(p, 2)) * nf;
    if (tot == 0) return RMHD_OK;
    Timed t(c, T_GHOST);
    if (tot < (1L << 31)) k_ghost<unsigned><<<nblk(tot, 256), 256, 0, c->stream>>>(p, a, nf);
    else k_ghost<unsigned long><<<nblk(tot, 256), 256, 0, c->stream>>>(p, a, nf);
    LAUNCH_CHECK();
    return RMHD_OK;
}

// x fluxes: in FP64 the persistent kernel (one wave per SIMD walking the
// segments with the next segment's loads in flight) is faster; in FP32 the
// one-segment-per-wave kernel is (measured on the 256^3 curved workload)
template <int D, int RECON, bool CURVED, class R, bool ACC, bool DG> void flux_t(rmhd_ctx* c, const double* P,
                                                                     const double* sig) {
    const Params& p = c->p;
    constexpr int E1 = (D == 0) ? 1 : 0, E2 = (D == 2) ? 1 : 2;
    static_assert(D == 0, "the lane-per-cell sweep runs along x");
    // the rows with their ghost cells as one sequence of 58-cell segments
    const int nseg = 0;
    const long items = ((long)(p.n[0] + 6) * p.n[E1] * p.n[E2] + TSEG - 1) / TSEG;
    const long need = (nblk(items, 4) + 7) / 8 * 8;   // multiple of 8 for the XCD renumbering
    if constexpr (std::is_same<R, float>::value) {
        k_flux_t<D, RECON, CURVED, R, ACC, DG><<<need, 256, 0, c->stream>>>(p, P, sig, c->rhs, nseg, items);
    } else {
        const long blocks = std::min<long>(need, c->persist_blocks);
        k_flux_p<D, RECON, CURVED, R, ACC, DG><<<blocks, 256, 0, c->stream>>>(p, P, sig, c->rhs, nseg, items);
    }
}

template <int D, int RECON, bool CURVED, class R, bool DG, bool FUSE = false>
void flux_w(rmhd_ctx* c, const double* P, const double* sig, const FuseArgs& fz = FuseArgs{}) {
    const Params& p = c->p;
    constexpr int E = (D == 1) ? 2 : 1;
    // segments as long as possible (each re-loads 3 halo rows at both ends
    // and starts a window) while the columns x segments still give one wave
    // per SIMD; at least 8 rows each
    const int nxb = (p.n[0] + 63) / 64;
    const long cols = (long)nxb * p.n[E];
    const long want = 4L * c->persist_blocks;
    const int nseg0 = (int)std::min<long>(std::max<long>(1, (want + cols - 1) / cols), (p.n[D] + 7) / 8);
    const int seglen = (p.n[D] + nseg0 - 1) / nseg0;
    const int nseg = (p.n[D] + seglen - 1) / seglen;
    const long waves = (long)nxb * p.n[E] * nseg;
    const long blocks = (waves + 7) / 8 * 8;          // one wave per block; multiple of 8 for the XCD renumbering
    // (the fused form runs without a shift only)
    if (!FUSE && CURVED && p.bet)
        k_flux_w<D, RECON, CURVED, R, !FUSE, DG, FUSE><<<blocks, 64, 0, c->stream>>>(p, P, sig, c->rhs, seglen, nxb,
                                                                                      nseg, fz);
    else
        k_flux_w<D, RECON, CURVED, R, false, DG, FUSE><<<blocks, 64, 0, c->stream>>>(p, P, sig, c->rhs, seglen, nxb,
                                                                                      nseg, fz);
}

// fz: the z sweep also runs stage 2 on the rows it finishes (z active)
template <int RECON, bool CURVED, class R, bool DG>
int flux_div_t(rmhd_ctx* c, const double* P, const double* sig, const FuseArgs* fz) {
    const Params& p = c->p;
    {
        Timed t(c, T_FX);
        flux_t<0, RECON, CURVED, R, false, DG>(c, P, sig);
    }
    LAUNCH_CHECK();
    if (is_active(p, 1)) {
        Timed t(c, T_FY);
        flux_w<1, RECON, CURVED, R, DG>(c, P, sig);
        LAUNCH_CHECK();
    }
    if (is_active(p, 2)) {
        Timed t(c, fz ? T_FZU : T_FZ);
        // the fused instances that stage 2 launches (FP64, MC2 or minmod,
        // flat or diagonal metric)
        constexpr bool FUSABLE = std::is_same<R, double>::value && RECON != REC_WENO5 && (!CURVED || DG);
        if constexpr (FUSABLE) {
            if (fz) flux_w<2, RECON, CURVED, R, DG, true>(c, P, sig, *fz);
            else flux_w<2, RECON, CURVED, R, DG>(c, P, sig);
        } else {
            if (fz) return fail(RMHD_EINVAL, "no fused z sweep for this configuration");
            flux_w<2, RECON, CURVED, R, DG>(c, P, sig);
        }
        LAUNCH_CHECK();
    }
    return RMHD_OK;
}

template <class R> int flux_div_r(rmhd_ctx* c, const double* P, const double* sig, const FuseArgs* fz) {
    const int r = c->desc.recon;
    if (c->curved && c->diag) {
        if (r == RMHD_RECON_MINMOD) return flux_div_t<REC_MINMOD, true, R, true>(c, P, sig, fz);
        if (r == RMHD_RECON_MC2) return flux_div_t<REC_MC2, true, R, true>(c, P, sig, fz);
        return flux_div_t<REC_WENO5, true, R, true>(c, P, sig, fz);
    }
    if (c->curved) {
        if (r == RMHD_RECON_MINMOD) return flux_div_t<REC_MINMOD, true, R, false>(c, P, sig, fz);
        if (r == RMHD_RECON_MC2) return flux_div_t<REC_MC2, true, R, false>(c, P, sig, fz);
        return flux_div_t<REC_WENO5, true, R, false>(c, P, sig, fz);
    }
    if (r == RMHD_RECON_MINMOD) return flux_div_t<REC_MINMOD, false, R, false>(c, P, sig, fz);
    if (r == RMHD_RECON_MC2) return flux_div_t<REC_MC2, false, R, false>(c, P, sig, fz);
    return flux_div_t<REC_WENO5, false, R, false>(c, P, sig, fz);
}

// minus the flux divergence of the (ghost-filled) primitives P into c->rhs;
// FP32 reconstruction / HLLE / divergence in the mixed-precision form
int flux_div(rmhd_ctx* c, const double* P, const double* sig, const FuseArgs* fz = nullptr) {
    if (c->desc.precision == RMHD_PREC_MIXED) return flux_div_r<float>(c, P, sig, fz);
    return flux_div_r<double>(c, P, sig, fz);
}

// persistent stage kernels: one one-wave block per SIMD (4 per CU)
template <int STAGE>
int launch_stage(rmhd_ctx* c, double dt, const double* sig, const double* Un, const double* Us, const double* Ps,
                 const double* R1, const double* R2, double* Uo, double* Po, double* Ro, int32_t* st,
                 double* P1o = nullptr) {
    const Params& p = c->p;
    const long nchunk = (long)((p.n[0] + 63) / 64) * p.n[1] * p.n[2];
    // a multiple of 8, so that the XCD renumbering of the blocks is a bijection
    const long blocks = std::min<long>(4 * c->persist_blocks, (nchunk + 7) / 8 * 8);
    // without a status array every cell writes one dummy word (counters[3])
    int32_t* sp = st ? st : reinterpret_cast<int32_t*>(c->counters + 3);
    const long ss = st ? 1 : 0;
    auto go = [&](auto kern) {
        kern<<<blocks, 64, 0, c->stream>>>(c->p, dt, sig, Un, Us, Ps, R1, R2, c->rhs, Uo, Po, Ro, P1o, sp, ss,
                                           c->counters);
    };
    if (c->curved && c->p.K) {
        if (c->diag) go(k_stage<STAGE, true, true, true>);
        else go(k_stage<STAGE, true, true, false>);
    } else if (c->curved) {
        if (c->diag) go(k_stage<STAGE, true, false, true>);
        else go(k_stage<STAGE, true, false, false>);
    } else {
        go(k_stage<STAGE, false, false, false>);
    }
    LAUNCH_CHECK();
    return RMHD_OK;
}

int stage1(rmhd_ctx* c, double dt, const double* sig, const double* Un, const double* Pg, double* P1, double* R1,
           double* U1, int32_t* st) {
    // with a conductivity model the kernel takes sigma from D^n; the sigma
    // stream it loads is then a placeholder (the model's own buffer)
    if (c->desc.sigma_model != RMHD_SIGMA_FIELD) sig = c->sigf;
    Timed t(c, T_STAGE1);
    return launch_stage<1>(c, dt, sig, Un, nullptr, Pg, nullptr, nullptr, U1, P1, R1, st);
}

template <int STAGE>
int update(rmhd_ctx* c, double dt, const double* sig, const double* Un, const double* Us, const double* Ps,
           const double* R1, const double* R2, double* Uo, double* Po, double* Ro, int32_t* st) {
    Timed t(c, STAGE == 2 ? T_UPD2 : T_UPD3);
    return launch_stage<STAGE>(c, dt, sig, Un, Us, Ps, R1, R2, Uo, Po, Ro, st);
}

// the sigma the flux sweeps read: the caller's field, or with a conductivity
// model the model at the stage primitives P (interior cells; the sweeps take
// ghost cells from their interior images)
int flux_sigma(rmhd_ctx* c, const double* P, const double* sig, const double** out) {
    if (c->desc.sigma_model == RMHD_SIGMA_FIELD) {
        *out = sig;
        return RMHD_OK;
    }
    const long n = ncells(c->p);
    Timed t(c, T_OTHER);
    if (c->curved) k_sigma_field<true><<<nblk(n, 256), 256, 0, c->stream>>>(c->p, P, c->sigf);
    else k_sigma_field<false><<<nblk(n, 256), 256, 0, c->stream>>>(c->p, P, c->sigf);
    LAUNCH_CHECK();
    *out = c->sigf;
    return RMHD_OK;
}

int stage2(rmhd_ctx* c, double dt, const double* sig, const double* Un, double* P1, const double* R1, double* U2,
           double* P2, double* R2, int32_t* st) {
    int r;
    // (no ghost fill: the sweeps read a ghost cell's primitives at its
    // interior image, as they do sigma)
    const double* fs = nullptr;
    if ((r = flux_sigma(c, P1, sig, &fs)) != RMHD_OK) return r;
    // The z sweep with the update in one kernel measured faster for FP64
    // MC2 and minmod on flat or diagonal metrics (256^3 blob, MC2: 3.40 ->
    // 2.86 ms for z sweep + update); with WENO5 (FP64 or mixed) or in the
    // mixed form the window and the recovery do not share the registers well
    // and it measured slower, so those keep the separate update.
    const bool fuse = is_active(c->p, 2) && c->desc.precision == RMHD_PREC_FP64 &&
                      c->desc.recon != RMHD_RECON_WENO5 && (!c->curved || c->diag) && !c->p.bet && !c->p.K &&
                      c->desc.sigma_model == RMHD_SIGMA_FIELD;
    if (fuse) {
        // the z sweep runs the update on each row it finishes
        int32_t* dummy = reinterpret_cast<int32_t*>(c->counters + 3);
        FuseArgs fz{Un, R1, U2, P2, R2, st ? st : dummy, st ? 1L : 0L, dt, c->counters, dummy};
        return flux_div(c, P1, fs, &fz);
    }
    if ((r = flux_div(c, P1, fs)) != RMHD_OK) return r;
    // (with a model the stage kernel takes sigma from D of its stage state;
    // the sigma stream it loads is then a placeholder)
    return update<2>(c, dt, fs, Un, nullptr, P1, R1, nullptr, U2, P2, R2, st);
}

int stage3(rmhd_ctx* c, double dt, const double* sig, const double* Un, const double* U2, double* P2,
           const double* R1, const double* R2, double* Uo, double* Po, int32_t* st) {
    int r;
    const double* fs = nullptr;
    if ((r = flux_sigma(c, P2, sig, &fs)) != RMHD_OK) return r;
    if ((r = flux_div(c, P2, fs)) != RMHD_OK) return r;
    return update<3>(c, dt, fs, Un, U2, P2, R1, R2, Uo, Po, nullptr, st);
}

// the final update of a step in place on (U, P), fused with the next step's
// stage 1 into the workspace's P(1) and R1 (R1 read and rewritten per cell)
int stage3_then_stage1(rmhd_ctx* c, double dt, const double* sig, double* U, double* P) {
    int r;
    const double* fs = nullptr;
    if ((r = flux_sigma(c, c->P2, sig, &fs)) != RMHD_OK) return r;
    if ((r = flux_div(c, c->P2, fs)) != RMHD_OK) return r;
    // the sigma stream feeds the stage-1 part only: the caller's field, or a
    // placeholder with a conductivity model (stage 1 takes sigma from D^{n+1})
    const double* s1 = c->desc.sigma_model != RMHD_SIGMA_FIELD ? c->sigf : sig;
    Timed t(c, T_UPD3);
    return launch_stage<4>(c, dt, s1, U, c->U2, c->P2, c->R1, c->R2, U, P, c->R1, nullptr, c->P1);
}

constexpr int ADJ_FIELDS = 79;   // Ub2 14, Pb 14, Lb 14, R1b 3, R2b 3, sb 1, fb 30

template <bool CURVED, int RECON> int adj_L_t(rmhd_ctx* c, const double* P, const double* sig, double* Lb,
                                              double* Pb, double* sb, double* fb) {
    const Params& p = c->p;
    const long n = ncells(p);
    k_adj_sources<CURVED><<<nblk(n, 256), 256, 0, c->stream>>>(p, P, Lb, Pb);
    LAUNCH_CHECK();
    for (int d = 0; d < 3; ++d) {
        if (!is_active(p, d)) continue;
        const int e1 = (d == 0) ? 1 : 0, e2 = (d == 2) ? 1 : 2;
        const long nf = (long)(p.n[d] + 1) * p.n[e1] * p.n[e2];
        const long nc = (long)p.np[d] * p.n[e1] * p.n[e2];
        if (d == 0) {
            k_adj_face<0, RECON, CURVED><<<nblk(nf, 128), 128, 0, c->stream>>>(p, P, sig, Lb, fb);
            LAUNCH_CHECK();
            const long items = ((long)(p.n[0] + 6) * p.n[1] * p.n[2] + TSEGA - 1) / TSEGA;   // 2 per block
            k_adj_cell_x<RECON, CURVED><<<(unsigned)((items + 1) / 2), 128, 0, c->stream>>>(p, P, sig, fb, Pb, sb,
                                                                                             items);
            (void)nc;
        } else if (d == 1) {
            k_adj_face<1, RECON, CURVED><<<nblk(nf, 128), 128, 0, c->stream>>>(p, P, sig, Lb, fb);
            LAUNCH_CHECK();
            k_adj_cell<1, RECON, CURVED><<<nblk(nc, 128), 128, 0, c->stream>>>(p, P, sig, fb, Pb, sb);
        } else {
            k_adj_face<2, RECON, CURVED><<<nblk(nf, 128), 128, 0, c->stream>>>(p, P, sig, Lb, fb);
            LAUNCH_CHECK();
            k_adj_cell<2, RECON, CURVED><<<nblk(nc, 128), 128, 0, c->stream>>>(p, P, sig, fb, Pb, sb);
        }
        LAUNCH_CHECK();
    }
    for (int d = 0; d < 3; ++d) {
        if (!is_active(p, d)) continue;
        const int e1 = (d == 0) ? 1 : 0, e2 = (d == 2) ? 1 : 2;
        const long nt = 2L * p.n[e1] * p.n[e2] * (NF + 1);
        k_adj_fold<<<nblk(nt, 256), 256, 0, c->stream>>>(p, Pb, NF, sb, d);
        LAUNCH_CHECK();
    }
    return RMHD_OK;
}

// adjoint of L(P) = -div F(P) + S(P): Pb += (dL/dP)^T Lb, sb += (dL/dsigma)^T Lb
int adj_L(rmhd_ctx* c, const double* P, const double* sig, double* Lb, double* Pb, double* sb, double* fb) {
    const int r = c->desc.recon;
    if (c->curved) {
        if (r == RMHD_RECON_MINMOD) return adj_L_t<true, REC_MINMOD>(c, P, sig, Lb, Pb, sb, fb);
        if (r == RMHD_RECON_MC2) return adj_L_t<true, REC_MC2>(c, P, sig, Lb, Pb, sb, fb);
        return adj_L_t<true, REC_WENO5>(c, P, sig, Lb, Pb, sb, fb);
    }
    if (r == RMHD_RECON_MINMOD) return adj_L_t<false, REC_MINMOD>(c, P, sig, Lb, Pb, sb, fb);
    if (r == RMHD_RECON_MC2) return adj_L_t<false, REC_MC2>(c, P, sig, Lb, Pb, sb, fb);
    return adj_L_t<false, REC_WENO5>(c, P, sig, Lb, Pb, sb, fb);
}

template <int STAGE>
int adj_point(rmhd_ctx* c, double dt, const double* sig, const double* Us, const double* Rs, const double* Ps,
              const double* Ubs, const double* Pb, const double* Rb, double* Ubn, double* Lb, double* R1b,
              double* sb) {
    const long n = ncells(c->p);
    if (c->curved)
        k_adj_point<STAGE, true><<<nblk(n, 128), 128, 0, c->stream>>>(c->p, dt, sig, Us, Rs, Ps, Ubs, Pb, Rb, Ubn,
                                                                      Lb, R1b, sb, c->counters);
    else
        k_adj_point<STAGE, false><<<nblk(n, 128), 128, 0, c->stream>>>(c->p, dt, sig, Us, Rs, Ps, Ubs, Pb, Rb, Ubn,
                                                                       Lb, R1b, sb, c->counters);
    LAUNCH_CHECK();
    return RMHD_OK;
}

int fill(rmhd_ctx* c, double* a, long n) {
    k_fill<<<(unsigned)std::min<long>(nblk(n, 256), 8192), 256, 0, c->stream>>>(a, n, 0.0);
    LAUNCH_CHECK();
    return RMHD_OK;
}

int resolve_scratch(int dev, void** out, std::string& why) {
    *out = nullptr;
    if (dev < 0 || dev >= MAX_DEVICES) {
        why = "device ordinal " + std::to_string(dev) + " beyond the static scratch table";
        return RMHD_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* a = nullptr;
        const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !a) {
            why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return RMHD_EHIP;
        }
        g_scratch_addr[dev] = a;
    }
    *out = g_scratch_addr[dev];
    return RMHD_OK;
}

}  // namespace

extern "C" {

size_t rmhd_adjoint_workspace_bytes(const rmhd_grid_desc* desc) {
    std::string why;
    if (!check_desc(desc, why)) {
        g_err = why;
        return 0;
    }
    return up((size_t)ADJ_FIELDS * (size_t)padded_cells(desc) * sizeof(double)) + ALIGN;
}

int rmhd_step_adjoint(rmhd_ctx* c, double dt, const double* sigma, const double* U_n, const double* P_n,
                      const double* Ubar_np1, double* Ubar_n, double* sigma_bar, void* adj_ws, size_t adj_bytes) {
    if (!c || !sigma || !U_n || !P_n || !Ubar_np1 || !Ubar_n || !sigma_bar || !adj_ws)
        return fail(RMHD_EINVAL, "null argument");
    if (!(dt > 0.0)) return fail(RMHD_EINVAL, "dt must be > 0");
    if (c->desc.precision != RMHD_PREC_FP64) return fail(RMHD_EINVAL, "the adjoint differentiates the FP64 form");
    if (c->desc.sigma_model != RMHD_SIGMA_FIELD || c->desc.rho_atmo > 0.0)
        return fail(RMHD_EINVAL, "the adjoint differentiates the static sigma field without an atmosphere");
    if (adj_bytes < rmhd_adjoint_workspace_bytes(&c->desc)) return fail(RMHD_EINVAL, "adjoint workspace too small");
    if ((reinterpret_cast<uintptr_t>(adj_ws) % ALIGN) != 0) return fail(RMHD_EINVAL, "adjoint workspace not aligned");
    const long Np = c->p.Np;
    double* base = static_cast<double*>(adj_ws);
    double* Ub2 = base;
    double* Pb = Ub2 + 14 * Np;
    double* Lb = Pb + 14 * Np;
    double* R1b = Lb + 14 * Np;
    double* R2b = R1b + 3 * Np;
    double* sb = R2b + 3 * Np;
    double* fb = sb + Np;
    int r;
    // forward recompute of the stages
    if ((r = stage1(c, dt, sigma, U_n, P_n, c->P1, c->R1, nullptr, nullptr)) != RMHD_OK) return r;
    if ((r = stage2(c, dt, sigma, U_n, c->P1, c->R1, c->U2, c->P2, c->R2, nullptr)) != RMHD_OK) return r;
    // the adjoint's face kernels read the stage primitives at ghost cells
    if ((r = ghost_fill(c, c->P1, NF)) != RMHD_OK) return r;
    if ((r = ghost_fill(c, c->P2, NF)) != RMHD_OK) return r;
    // reverse sweep
    const long n = ncells(c->p);
    k_adj_final<<<nblk(n, 256), 256, 0, c->stream>>>(c->p, dt, Ubar_np1, Ubar_n, Ub2, Lb, R1b, R2b);
    LAUNCH_CHECK();
    if ((r = fill(c, Pb, 14 * Np)) != RMHD_OK) return r;
    if ((r = fill(c, sb, Np)) != RMHD_OK) return r;
    if ((r = adj_L(c, c->P2, sigma, Lb, Pb, sb, fb)) != RMHD_OK) return r;
    if ((r = adj_point<2>(c, dt, sigma, c->U2, c->R2, c->P2, Ub2, Pb, R2b, Ubar_n, Lb, R1b, sb)) != RMHD_OK) return r;
    if ((r = fill(c, Pb, 14 * Np)) != RMHD_OK) return r;
    if ((r = adj_L(c, c->P1, sigma, Lb, Pb, sb, fb)) != RMHD_OK) return r;
    if ((r = adj_point<1>(c, dt, sigma, U_n, nullptr, c->P1, nullptr, Pb, R1b, Ubar_n, nullptr, nullptr, sb)) !=
        RMHD_OK)
        return r;
    k_adj_sigma_out<<<nblk(n, 256), 256, 0, c->stream>>>(c->p, sb, sigma_bar);
    LAUNCH_CHECK();
    return RMHD_OK;
}

int rmhd_step_adjoint_static(rmhd_ctx* c, double dt, const double* sigma, const double* U_n, const double* P_n,
                             const double* Ubar_np1, double* Ubar_n, double* sigma_bar) {
    if (!c) return fail(RMHD_EINVAL, "null context");
    // the launch timers create events, which allocate
    if (c->timing) return fail(RMHD_EINVAL, "rmhd_step_adjoint_static: switch the launch timing off first");
    const size_t need = rmhd_adjoint_workspace_bytes(&c->desc);
    if (need == 0) return fail(RMHD_EINVAL, "invalid grid");
    if (need > (size_t)RMHD_STATIC_SCRATCH_BYTES)
        return fail(RMHD_EINVAL, "rmhd_step_adjoint_static: this grid needs " + std::to_string(need) +
                                     " bytes of adjoint scratch; the static scratch holds " +
                                     std::to_string((size_t)RMHD_STATIC_SCRATCH_BYTES));
    if (!c->scratch)
        return fail(RMHD_EHIP, "rmhd_step_adjoint_static: no static scratch on this device: " + c->scratch_err);
    // the kernels take the device address resolved at rmhd_init_grid; the
    // buffers that must start at zero are cleared by fill kernels inside
    return rmhd_step_adjoint(c, dt, sigma, U_n, P_n, Ubar_np1, Ubar_n, sigma_bar, c->scratch, need);
}

int rmhd_prim2con_adjoint(rmhd_ctx* c, const double* P, const double* Ubar, double* Pbar) {
    if (!c || !P || !Ubar || !Pbar) return fail(RMHD_EINVAL, "null argument");
    const long n = ncells(c->p);
    if (c->curved) k_adj_prim2con<true><<<nblk(n, 256), 256, 0, c->stream>>>(c->p, P, Ubar, Pbar);
    else k_adj_prim2con<false><<<nblk(n, 256), 256, 0, c->stream>>>(c->p, P, Ubar, Pbar);
    LAUNCH_CHECK();
    return RMHD_OK;
}


const char* rmhd_last_error(void) { return g_err.c_str(); }

size_t rmhd_workspace_bytes(const rmhd_grid_desc* desc) {
    std::string why;
    if (!check_desc(desc, why)) {
        g_err = why;
        return 0;
    }
    size_t off[8];
    return ws_layout(desc, off);
}

int rmhd_padded_extent(const rmhd_grid_desc* desc, int32_t* host_out) {
    std::string why;
    if (!check_desc(desc, why)) return fail(RMHD_EINVAL, why);
    if (!host_out) return fail(RMHD_EINVAL, "host_out is NULL");
    for (int k = 0; k < 3; ++k) host_out[k] = desc->n[k] + 2 * pad_lo(desc, k);
    return RMHD_OK;
}

int rmhd_init_grid(const rmhd_grid_desc* desc, void* workspace, size_t ws_bytes, void* hip_stream, rmhd_ctx** out) {
    std::string why;
    if (!out) return fail(RMHD_EINVAL, "out is null");
    *out = nullptr;
    if (!check_desc(desc, why)) return fail(RMHD_EINVAL, why);
    size_t off[8];
    const size_t need = ws_layout(desc, off);
    if (!workspace || ws_bytes < need)
        return fail(RMHD_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
    if ((reinterpret_cast<uintptr_t>(workspace) % ALIGN) != 0) return fail(RMHD_EINVAL, "workspace not 256-byte aligned");
    rmhd_ctx* c = new rmhd_ctx;
    c->desc = *desc;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->ws = static_cast<char*>(workspace);
    c->ws_bytes = ws_bytes;
    c->rhs = reinterpret_cast<double*>(c->ws + off[0]);
    c->P1 = reinterpret_cast<double*>(c->ws + off[1]);
    c->R1 = reinterpret_cast<double*>(c->ws + off[2]);
    c->U2 = reinterpret_cast<double*>(c->ws + off[3]);
    c->P2 = reinterpret_cast<double*>(c->ws + off[4]);
    c->R2 = reinterpret_cast<double*>(c->ws + off[5]);
    c->sigf = desc->sigma_model != RMHD_SIGMA_FIELD ? reinterpret_cast<double*>(c->ws + off[6]) : nullptr;
    c->counters = reinterpret_cast<unsigned long long*>(c->ws + off[7]);
    Params& p = c->p;
    std::memset(&p, 0, sizeof p);
    for (int d = 0; d < 3; ++d) {
        p.n[d] = desc->n[d];
        p.g[d] = pad_lo(desc, d);
        p.np[d] = p.n[d] + 2 * p.g[d];
        p.bc[d] = desc->bc[d];
        p.dx[d] = desc->dx[d];
        p.idx[d] = ((desc->active_mask >> d) & 1) ? 1.0 / desc->dx[d] : 0.0;
        p.cdiff[d] = p.idx[d] / 12.0;
    }
    p.st[0] = 1;
    p.st[1] = p.np[0];
    p.st[2] = (long)p.np[0] * p.np[1];
    p.Np = (long)p.np[0] * p.np[1] * p.np[2];
    p.ng = desc->ng;
    p.active = desc->active_mask;
    p.maxit = desc->c2p_maxit;
    p.speed_mode = desc->speed_mode;
    p.G = desc->gamma_ad;
    p.kappa = desc->kappa;
    p.tol = desc->c2p_tol;
    p.tolq = 0.0075 * p.tol;
    p.sig_model = desc->sigma_model;
    p.sig0 = desc->sigma0;
    p.sig_exp = desc->sigma_exp;
    p.sig_Datmo = desc->sigma_Datmo;
    p.rho_atmo = desc->rho_atmo;
    p.p_atmo = desc->rho_atmo > 0.0 ? desc->K_atmo * std::pow(desc->rho_atmo, desc->gamma_ad) : 0.0;
    c->curved = false;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            c->device = dev;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
                c->persist_blocks = ((long)cus + 7) / 8 * 8;
            // the static adjoint scratch of this device (once per device); a
            // failure only disables rmhd_step_adjoint_static on this context
            if (resolve_scratch(dev, &c->scratch, c->scratch_err) != RMHD_OK) c->scratch = nullptr;
        } else {
            c->scratch_err = "hipGetDevice failed at rmhd_init_grid";
        }
    }
    k_zero_u64<<<1, 64, 0, c->stream>>>(c->counters, 5);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        delete c;
        return fail(RMHD_EHIP, std::string("init: ") + hipGetErrorString(e));
    }
    *out = c;
    return RMHD_OK;
}

int rmhd_set_metric(rmhd_ctx* c, const double* alpha, const double* beta, const double* gamma, const double* K) {
    if (!c) return fail(RMHD_EINVAL, "null context");
    if ((alpha == nullptr) != (gamma == nullptr)) return fail(RMHD_EINVAL, "alpha and gamma must both be set or both null");
    if (!alpha && (beta || K)) return fail(RMHD_EINVAL, "beta/K need alpha and gamma");
    // a shift or extrinsic curvature that is zero everywhere is dropped, which
    // selects the kernels without those terms (fewer registers and loads)
    auto all_zero = [&](const double* a, long n, bool& zero) -> int {
        k_zero_u64<<<1, 64, 0, c->stream>>>(c->counters + 2, 1);
        k_any_nonzero<<<(unsigned)std::min<long>(nblk(n, 256), 4096), 256, 0, c->stream>>>(a, n, c->counters + 2);
        LAUNCH_CHECK();
        unsigned long long h = 0;
        HIP_TRY(hipMemcpyAsync(&h, c->counters + 2, sizeof h, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        zero = h == 0;
        return RMHD_OK;
    };
    bool zb = false, zk = false, zxy = false, zyz = false;
    int r;
    if (beta && (r = all_zero(beta, 3 * c->p.Np, zb)) != RMHD_OK) return r;
    if (K && (r = all_zero(K, 6 * c->p.Np, zk)) != RMHD_OK) return r;
    // a diagonal gamma_ij (xy, xz: rows 1-2; yz: row 4) selects the kernels
    // that skip its zero entries
    if (gamma && (r = all_zero(gamma + c->p.Np, 2 * c->p.Np, zxy)) != RMHD_OK) return r;
    if (gamma && zxy && (r = all_zero(gamma + 4 * c->p.Np, c->p.Np, zyz)) != RMHD_OK) return r;
    c->diag = gamma && zxy && zyz;
    c->p.alp = alpha;
    c->p.gam = gamma;
    c->p.bet = (beta && !zb) ? beta : nullptr;
    c->p.K = (K && !zk) ? K : nullptr;
    c->curved = alpha != nullptr;
    return RMHD_OK;
}

int rmhd_prim2con(rmhd_ctx* c, const double* P, double* U) {
    if (!c || !P || !U) return fail(RMHD_EINVAL, "null argument");
    const long n = ncells(c->p);
    if (c->curved) k_prim2con<true><<<nblk(n, 256), 256, 0, c->stream>>>(c->p, P, U);
    else k_prim2con<false><<<nblk(n, 256), 256, 0, c->stream>>>(c->p, P, U);
    LAUNCH_CHECK();
    return RMHD_OK;
}

int rmhd_con2prim(rmhd_ctx* c, const double* U, double* P, int32_t* status) {
    if (!c || !P || !U) return fail(RMHD_EINVAL, "null argument");
    const long n = ncells(c->p);
    if (c->curved) k_con2prim<true><<<nblk(n, 256), 256, 0, c->stream>>>(c->p, U, P, status, c->counters);
    else k_con2prim<false><<<nblk(n, 256), 256, 0, c->stream>>>(c->p, U, P, status, c->counters);
    LAUNCH_CHECK();
    return RMHD_OK;
}

int rmhd_imex_stage(rmhd_ctx* c, int stage, double dt, const double* sigma, const rmhd_stage_bufs* b) {
    if (!c || !b || (!sigma && c->desc.sigma_model == RMHD_SIGMA_FIELD)) return fail(RMHD_EINVAL, "null argument");
    if (!(dt > 0.0)) return fail(RMHD_EINVAL, "dt must be > 0");
    if (!b->U_n || !b->P_in || !b->P_out) return fail(RMHD_EINVAL, "U_n, P_in and P_out are required");
    switch (stage) {
        case 1:
            if (!b->R_out) return fail(RMHD_EINVAL, "stage 1 needs R_out");
            if (b->P_out == b->P_in) return fail(RMHD_EINVAL, "stage 1: P_out must not alias P_in");
            return stage1(c, dt, sigma, b->U_n, b->P_in, b->P_out, b->R_out, b->U_out, b->status);
        case 2:
            if (!b->R1 || !b->U_out || !b->R_out) return fail(RMHD_EINVAL, "stage 2 needs R1, U_out and R_out");
            if (b->P_out == b->P_in || (const double*)b->U_out == b->U_n)
                return fail(RMHD_EINVAL, "stage 2 outputs must not alias its inputs");
            return stage2(c, dt, sigma, b->U_n, b->P_in, b->R1, b->U_out, b->P_out, b->R_out, b->status);
        case 3:
            if (!b->U_s || !b->R1 || !b->R2 || !b->U_out) return fail(RMHD_EINVAL, "stage 3 needs U_s, R1, R2, U_out");
            if (b->P_out == b->P_in) return fail(RMHD_EINVAL, "stage 3: P_out must not alias P_in");
            return stage3(c, dt, sigma, b->U_n, b->U_s, b->P_in, b->R1, b->R2, b->U_out, b->P_out, b->status);
        default:
            return fail(RMHD_EINVAL, "stage must be 1, 2 or 3");
    }
}

int rmhd_step(rmhd_ctx* c, double dt, const double* sigma, double* U, double* P) {
    if (!c || !U || !P || (!sigma && c->desc.sigma_model == RMHD_SIGMA_FIELD))
        return fail(RMHD_EINVAL, "null argument");
    if (!(dt > 0.0)) return fail(RMHD_EINVAL, "dt must be > 0");
    int r;
    if ((r = stage1(c, dt, sigma, U, P, c->P1, c->R1, nullptr, nullptr)) != RMHD_OK) return r;
    if ((r = stage2(c, dt, sigma, U, c->P1, c->R1, c->U2, c->P2, c->R2, nullptr)) != RMHD_OK) return r;
    return stage3(c, dt, sigma, U, c->U2, c->P2, c->R1, c->R2, U, P, nullptr);
}

int rmhd_steps(rmhd_ctx* c, double dt, const double* sigma, double* U, double* P, int nsteps) {
    if (!c || !U || !P || (!sigma && c->desc.sigma_model == RMHD_SIGMA_FIELD))
        return fail(RMHD_EINVAL, "null argument");
    if (!(dt > 0.0)) return fail(RMHD_EINVAL, "dt must be > 0");
    if (nsteps < 0) return fail(RMHD_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return RMHD_OK;
    int r;
    if ((r = stage1(c, dt, sigma, U, P, c->P1, c->R1, nullptr, nullptr)) != RMHD_OK) return r;
    for (int s = 0; s < nsteps; ++s) {
        if ((r = stage2(c, dt, sigma, U, c->P1, c->R1, c->U2, c->P2, c->R2, nullptr)) != RMHD_OK) return r;
        if (s + 1 < nsteps) r = stage3_then_stage1(c, dt, sigma, U, P);
        else r = stage3(c, dt, sigma, U, c->U2, c->P2, c->R1, c->R2, U, P, nullptr);
        if (r != RMHD_OK) return r;
    }
    return RMHD_OK;
}

int rmhd_max_signal_speed(rmhd_ctx* c, double* host_out) {
    if (!c || !host_out) return fail(RMHD_EINVAL, "null argument");
    k_zero_u64<<<1, 64, 0, c->stream>>>(c->counters + 1, 1);
    LAUNCH_CHECK();
    const long n = ncells(c->p);
    const unsigned blocks = (unsigned)std::min<long>(nblk(n, 256), 4096);
    if (c->curved) k_max_speed<true><<<blocks, 256, 0, c->stream>>>(c->p, c->counters + 1);
    else k_max_speed<false><<<blocks, 256, 0, c->stream>>>(c->p, c->counters + 1);
    LAUNCH_CHECK();
    unsigned long long bits = 0;
    HIP_TRY(hipMemcpyAsync(&bits, c->counters + 1, sizeof bits, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    double v;
    std::memcpy(&v, &bits, sizeof v);
    *host_out = v;
    return RMHD_OK;
}

int rmhd_failures(rmhd_ctx* c, int64_t* host_out) {
    if (!c || !host_out) return fail(RMHD_EINVAL, "null argument");
    unsigned long long n = 0;
    HIP_TRY(hipMemcpyAsync(&n, c->counters, sizeof n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    k_zero_u64<<<1, 64, 0, c->stream>>>(c->counters, 1);
    LAUNCH_CHECK();
    *host_out = (int64_t)n;
    return RMHD_OK;
}

int rmhd_atmosphere_cells(rmhd_ctx* c, int64_t* host_out) {
    if (!c || !host_out) return fail(RMHD_EINVAL, "null argument");
    unsigned long long n = 0;
    HIP_TRY(hipMemcpyAsync(&n, c->counters + 4, sizeof n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    k_zero_u64<<<1, 64, 0, c->stream>>>(c->counters + 4, 1);
    LAUNCH_CHECK();
    *host_out = (int64_t)n;
    return RMHD_OK;
}

int rmhd_recovery_stats(rmhd_ctx* c, int enable) {
    if (!c) return fail(RMHD_EINVAL, "null context");
    if (enable) {
        k_zero_u64<<<1, 128, 0, c->stream>>>(c->counters + 32, 3 * RMHD_HIST_BINS);
        LAUNCH_CHECK();
        c->p.hist = c->counters + 32;
    } else {
        c->p.hist = nullptr;
    }
    return RMHD_OK;
}

int rmhd_recovery_stats_read(rmhd_ctx* c, int64_t* bins_out) {
    if (!c || !bins_out) return fail(RMHD_EINVAL, "null argument");
    unsigned long long h[3 * RMHD_HIST_BINS];
    HIP_TRY(hipMemcpyAsync(h, c->counters + 32, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int i = 0; i < 3 * RMHD_HIST_BINS; ++i) bins_out[i] = (int64_t)h[i];
    k_zero_u64<<<1, 128, 0, c->stream>>>(c->counters + 32, 3 * RMHD_HIST_BINS);
    LAUNCH_CHECK();
    return RMHD_OK;
}

int rmhd_timing(rmhd_ctx* c, int enable) {
    if (!c) return fail(RMHD_EINVAL, "null context");
    c->timing = enable != 0;
    return RMHD_OK;
}

int rmhd_timing_read(rmhd_ctx* c, double* ms_out, int64_t* launches_out) {
    if (!c || !ms_out || !launches_out) return fail(RMHD_EINVAL, "null argument");
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->timing_err) {
        // some launch went untimed or half-timed: report it rather than a partial sum
        c->timing_err = false;
        for (int k = 0; k < RMHD_TIMING_CLASSES; ++k) c->used[k] = 0;
        return fail(RMHD_EHIP, "a timing event could not be created or recorded");
    }
    for (int k = 0; k < RMHD_TIMING_CLASSES; ++k) {
        double tot = 0.0;
        for (size_t i = 0; i < c->used[k]; ++i) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, c->ev[k][i].first, c->ev[k][i].second));
            tot += ms;
        }
        ms_out[k] = tot;
        launches_out[k] = (int64_t)c->used[k];
        c->used[k] = 0;
    }
    return RMHD_OK;
}

int rmhd_set_stream(rmhd_ctx* c, void* hip_stream) {
    if (!c) return fail(RMHD_EINVAL, "null context");
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return RMHD_OK;
}

int rmhd_destroy(rmhd_ctx* c) {
    if (!c) return RMHD_OK;
    // teardown: a failure to destroy an event leaves nothing to recover
    for (auto& v : c->ev)
        for (auto& pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    delete c;
    return RMHD_OK;
}

}  // extern "C"
