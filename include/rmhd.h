/*
 * rmhd.h -- C ABI of the MI355X (gfx950) resistive GRMHD stage library.
 *
 * The library advances the 14 conserved variables of resistive general-
 * relativistic MHD on a uniform grid in a fixed 3+1 metric with the
 * IMEX-SSP2(2,2,2) Runge-Kutta scheme of arXiv:2510.18968 (Sec. III.A,
 * table imex, eq. IMEX3): reconstruction of the primitives (minmod, MC2,
 * WENO5), HLLE fluxes with speed-of-light characteristic speeds (Sec. III),
 * flux divergence plus non-stiff sources (eq. GRRMHD_flux_form), and a
 * per-cell implicit solve of the stiff Ohm's-law term (eq. 3D_NR) coupled to
 * the primitive recovery (Sec. III.B).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array pointers are DEVICE pointers (HIP global memory) unless the
 *    name ends in host_out.  The caller owns every array; the library owns
 *    only the opaque context.  Scratch memory comes from a caller-provided
 *    workspace, so the library never allocates device memory itself.
 *  - Layout: float64, structure of arrays, field-major
 *    a[f][k][j][i] with i (x) fastest, over the PADDED grid: along every
 *    active dimension d there are pad_d cells on each side of the interior,
 *    inactive dimensions carry none.  pad_d = ng = 3, except along x with
 *    x_align = 1, where pad_x = 16: the 3 cells next to the interior are the
 *    ghost cells, the other 13 are never read or written.  With n[0] a
 *    multiple of 16 and a 128-byte aligned base pointer every interior x row
 *    then starts on a 128-byte line, which the streaming kernels read and
 *    write as whole lines.  Np = prod_d (n[d] + 2 pad_d);
 *    rmhd_padded_extent() returns the three extents.
 *  - Primitive vector P (14): rho, p, v^x, v^y, v^z, B^x, B^y, B^z,
 *    E^x, E^y, E^z, phi, psi, q (contravariant, not densitised; v is the
 *    Eulerian 3-velocity of Sec. II.A).
 *  - Conserved vector U (14): D, S_x, S_y, S_z, tau, Bcal^x..z, Ecal^x..z,
 *    Phi, Psi, Qcal (eqs. conserved_dens/_tau/_S and the densitised fields of
 *    Sec. II.D).  Index f of an EM / cleaning / charge field is the same in P
 *    and U.
 *  - Metric fields (Sec. II.A): alpha [Np], beta^i [3][Np], gamma_ij
 *    [6][Np] in the order xx, xy, xz, yy, yz, zz, K_ij [6][Np] likewise, all
 *    at cell centres INCLUDING ghost cells (the caller evaluates them there).
 *  - Every call is asynchronous on the context's HIP stream, except those
 *    documented as synchronising.  Only interior cells of outputs are
 *    written (stage 2's exception: rmhd_stage_bufs); ghost cells of U and
 *    of the primitives are never read (the flux sweeps take a ghost cell's
 *    primitives and sigma at its interior image, the boundary conditions).
 *  - Return codes: RMHD_OK or a negative RMHD_E* code.  Argument checks
 *    happen on the host before any device work (RMHD_EINVAL).  Per-cell
 *    recovery failures never abort a launch: they set a per-cell status and
 *    bump a device counter read by rmhd_failures().  rmhd_last_error() gives
 *    a thread-local message for the last failing call.
 *  - A context is not thread-safe; separate contexts are independent.
 */
#ifndef RMHD_H
#define RMHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rmhd_ctx rmhd_ctx;

enum rmhd_status {
    RMHD_OK = 0,
    RMHD_EINVAL = -1,   /* invalid argument (checked on the host)             */
    RMHD_EHIP = -2,     /* a HIP runtime call failed                           */
    RMHD_ENOCONV = -3,  /* per-cell: recovery did not converge                 */
    RMHD_EUNPHYS = -4   /* per-cell: unphysical state (rho<=0, v^2>=1, NaN ..) */
};
/* per-cell status values written by the recovery: 0 ok, 1 converged at the
 * iteration cap within 1e-12 (warning), 2 (RMHD_ST_ATMO) atmosphere state
 * set at the end of the step, RMHD_ENOCONV, RMHD_EUNPHYS */

enum rmhd_recon { RMHD_RECON_MINMOD = 0, RMHD_RECON_MC2 = 1, RMHD_RECON_WENO5 = 2 };
enum rmhd_bc { RMHD_BC_PERIODIC = 0, RMHD_BC_COPY = 1 };
enum rmhd_precision { RMHD_PREC_FP64 = 0, RMHD_PREC_MIXED = 1 };

typedef struct {
    int32_t n[3];        /* interior cells per dimension; a batch of 1D problems
                            is n = {cells, problems, 1} with only x active     */
    int32_t active_mask; /* bit d set: fluxes and ghost cells along d          */
    int32_t ng;          /* ghost width; must be 3                             */
    int32_t bc[3];       /* per dimension: RMHD_BC_PERIODIC or RMHD_BC_COPY    */
    int32_t recon;       /* enum rmhd_recon                                    */
    int32_t precision;   /* enum rmhd_precision (MIXED: FP32 stencil, FP64
                            recovery and state)                                */
    int32_t c2p_maxit;   /* recovery iteration cap (default 500)               */
    int32_t speed_mode;  /* 0: +-sqrt(gamma^dd) - beta^d/alpha as printed in
                            Sec. III; 1: alpha sqrt(gamma^dd) -+ beta^d        */
    int32_t x_align;     /* 0: 3 cells of padding along x, as along y and z;
                            1: 16 (aligned interior rows, see Layout)          */
    double x0[3];        /* centre of the first interior cell                  */
    double dx[3];        /* cell widths                                        */
    double gamma_ad;     /* ideal-gas adiabatic index Gamma (Sec. III.B)        */
    double kappa;        /* divergence-cleaning damping (1 in the paper, Sec. IV)*/
    double c2p_tol;      /* recovery tolerance on |dp|/p and |dv| (1e-14)       */
    /* conductivity (Sec. IV.A, IV.E): RMHD_SIGMA_FIELD takes the caller's
       per-cell sigma array; the models set sigma from the conserved D of the
       state each use acts on -- the stage's explicit state in an implicit
       solve (the solve leaves D unchanged), sqrt(gamma) rho W of the stage
       primitives at every cell centre in the charge flux -- and the sigma
       argument of the stage calls is then ignored (may be NULL)           */
    int32_t sigma_model; /* enum rmhd_sigma_model                              */
    int32_t reserved_;   /* set to 0                                           */
    double sigma0;       /* sigma_0 of both models                              */
    double sigma_exp;    /* gamma of eq. sigma_evol                             */
    double sigma_Datmo;  /* D_atmo of eq. dynamo_sigma                          */
    /* artificial atmosphere (Sec. IV.E), off when rho_atmo = 0: at the end of
       each step (the final update) a cell whose assembled D is below
       RMHD_ATMO_FACTOR sqrt(gamma) rho_atmo gets the D, S_i and tau of the
       state rho = rho_atmo, v = 0, p = K_atmo rho_atmo^Gamma with its own E,
       B and cleaning fields, is recovered from it and flagged with status
       RMHD_ST_ATMO (counted by rmhd_atmosphere_cells, not a failure)      */
    double rho_atmo;
    double K_atmo;
} rmhd_grid_desc;

/* sigma = field | sigma0 D^sigma_exp (eq. sigma_evol) |
 * sigma0 max(1 - sigma_Datmo / D, 0)^2 (eq. dynamo_sigma) */
enum rmhd_sigma_model { RMHD_SIGMA_FIELD = 0, RMHD_SIGMA_POWER = 1, RMHD_SIGMA_DYNAMO = 2 };
#define RMHD_ATMO_FACTOR 1.01
#define RMHD_ST_ATMO 2

/* Buffers of one IMEX stage (Sec. III.A, eq. IMEX3).  [3][Np] arrays hold the
 * stiff E source R_E of a stage, recovered from the stage equation as
 * (Ecal(s) - Ecal*)/(gamma dt); [14][Np] arrays are U or P.
 *   stage 1 (implicit only):   in U_n, P_in = P^n (guess)
 *                              out P_out = P(1), R_out = R1, U_out = U(1) (optional)
 *   stage 2 (explicit + impl.): in U_n, P_in = P(1), R1
 *                              out U_out = U(2), P_out = P(2), R_out = R2
 *   stage 3 (final update):    in U_n, U_s = U(2), P_in = P(2), R1, R2
 *                              out U_out = U^{n+1}, P_out = P^{n+1}
 * Stage 2's local sources take the densitised cleaning fields (phi, psi, q)
 * of U(1) from U_n (stage 1 changes only E), the final update those of U(2)
 * from U_s: only p and v of P_in are read at the cell (with zero extrinsic
 * curvature).  Stages 2 and 3 read no ghost cell of P_in: the flux sweeps take
 * a ghost cell's primitives at its interior image (the boundary conditions
 * of the descriptor), and P_in is not written.  Stage 2 may
 * also overwrite the x ghost cell next to the interior of each row of U_out,
 * P_out, R_out and status (when n_x is not a multiple of 64).  For stage 3,
 * U_out may alias U_n and P_out may alias nothing else.  status is optional
 * ([Np] int32, interior cells written).  A cell whose recovery fails (status
 * < 0, counted by rmhd_failures) gets the primitives of its stage state at
 * the guess's p and v with E = Ecal* (R = 0): a flagged non-solution, never
 * a silently repaired one. */
typedef struct {
    const double* U_n;
    const double* U_s;
    double* P_in;
    const double* R1;
    const double* R2;
    double* U_out;
    double* P_out;
    double* R_out;
    int32_t* status;
} rmhd_stage_bufs;

/* Bytes of device workspace a context needs for this grid (>= 0; 0 on an
 * invalid descriptor, see rmhd_last_error). */
size_t rmhd_workspace_bytes(const rmhd_grid_desc* desc);

/* Padded extents {x, y, z} of the arrays of this grid (see Layout) into
 * host_out[3]; host only, no device work.  RMHD_EINVAL on an invalid
 * descriptor or a NULL host_out. */
int rmhd_padded_extent(const rmhd_grid_desc* desc, int32_t* host_out);

/* Create a context.  workspace: device memory of at least
 * rmhd_workspace_bytes(desc) bytes, 256-byte aligned, owned by the caller and
 * kept alive until rmhd_destroy.  hip_stream: a hipStream_t (NULL = default
 * stream).  The metric defaults to flat space (alpha = 1, beta = 0,
 * gamma_ij = delta_ij, K_ij = 0).  Returns RMHD_EINVAL on a bad descriptor. */
int rmhd_init_grid(const rmhd_grid_desc* desc, void* workspace, size_t ws_bytes, void* hip_stream, rmhd_ctx** out);

/* Fixed background metric, Sec. II.A (alpha, beta^i, gamma_ij, K_ij at cell
 * centres including ghosts, layouts above).  beta == NULL means zero shift,
 * K == NULL zero extrinsic curvature; alpha == NULL and gamma == NULL restore
 * flat space.  The arrays are referenced, not copied: keep them alive and
 * unchanged while the context uses them.  A beta or K that is zero in every
 * cell is treated as NULL (checked here on the device; the call synchronises
 * the stream when beta or K is given). */
int rmhd_set_metric(rmhd_ctx* ctx, const double* alpha, const double* beta, const double* gamma, const double* K);

/* Conserved from primitive variables, eqs. conserved_dens, conserved_tau,
 * conserved_S and the densitised fields of Sec. II.D, at interior cells. */
int rmhd_prim2con(rmhd_ctx* ctx, const double* P, double* U);

/* Primitive recovery with E fixed, Sec. III.B steps (i)-(v): P is the guess
 * on input and the result on output (interior cells).  status optional. */
int rmhd_con2prim(rmhd_ctx* ctx, const double* U, double* P, int32_t* status);

/* One stage of IMEX-SSP2(2,2,2) (table imex, eq. IMEX3), see rmhd_stage_bufs.
 * sigma: conductivity [Np] (ghost cells are not read; ignored, may be NULL,
 * when the descriptor selects a conductivity model). */
int rmhd_imex_stage(rmhd_ctx* ctx, int stage, double dt, const double* sigma, const rmhd_stage_bufs* bufs);

/* One full IMEX-SSP2(2,2,2) step in place: (U, P) at t -> t + dt.  Stage
 * buffers live in the workspace. */
int rmhd_step(rmhd_ctx* ctx, double dt, const double* sigma, double* U, double* P);

/* nsteps IMEX-SSP2(2,2,2) steps in place (table imex, eq. IMEX3), the results
 * of nsteps calls of rmhd_step up to rounding (the fused kernel's arithmetic
 * may be contracted into FMAs differently): stage 1 of every step after the first
 * is the pointwise solve of eq. 3D_NR on U^{n+1} guessed from P^{n+1} (Sec.
 * III.B), which the final update of the step before runs in its own kernel on
 * the cell it has just recovered.  This saves one pass over U, P, sigma and
 * the metric and one launch per step.  nsteps = 0 does nothing; nsteps < 0,
 * dt <= 0 or a null argument (sigma may be NULL with a conductivity model) is
 * RMHD_EINVAL with nothing launched.  Failed cells of every stage count in
 * rmhd_failures; the recovery histogram sees the same stages as rmhd_step. */
int rmhd_steps(rmhd_ctx* ctx, double dt, const double* sigma, double* U, double* P, int nsteps);

/* Bytes of caller-provided device scratch rmhd_step_adjoint needs (79 padded
 * fields: adjoint buffers and per-face sensitivities). */
size_t rmhd_adjoint_workspace_bytes(const rmhd_grid_desc* desc);

/* Adjoint (reverse mode) of rmhd_step: given Ubar_np1 = dL/dU^{n+1}, writes
 * Ubar_n = dL/dU^n (interior cells) and ADDS dL/dsigma to sigma_bar [Np]
 * (interior cells).  U_n, P_n: the state the forward step started from (P_n
 * is only the recovery guess; the recovered roots do not depend on it).  The
 * forward stages are recomputed inside.  Differentiates the FP64 form: the
 * recovery roots by the implicit-function theorem (Sec. III.B, eq. 3D_NR),
 * the flux divergence and sources (eq. GRRMHD_flux_form) and reconstruction by
 * their local Jacobians, the stage combination of eq. IMEX3 exactly; limiter
 * kinks and first-order fallbacks take the derivative of the branch taken.
 * Ubar_n may alias Ubar_np1.  adj_ws: >= rmhd_adjoint_workspace_bytes bytes,
 * 256-byte aligned.  Returns RMHD_EINVAL for the mixed-precision form and
 * for a conductivity model or an atmosphere (it differentiates the static
 * sigma field without floors).  A
 * cell whose recovery Jacobian is singular at the root has no implicit-
 * function derivative: its multiplier is set to zero and the cell is counted
 * by rmhd_failures() (as are failed recoveries of the recomputed forward
 * stages and cells whose sensitivities come out non-finite), so a caller
 * that finds a nonzero count must not trust the gradient. */
int rmhd_step_adjoint(rmhd_ctx* ctx, double dt, const double* sigma, const double* U_n, const double* P_n,
                      const double* Ubar_np1, double* Ubar_n, double* sigma_bar, void* adj_ws, size_t adj_bytes);

/* rmhd_step_adjoint without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, kernels and results as
 * rmhd_step_adjoint; its 79-field scratch is instead a static device array of
 * RMHD_STATIC_SCRATCH_BYTES (one copy per device, reserved when the library
 * loads on that device and held until the process ends; its address is
 * resolved once per device by rmhd_init_grid).  Allocates nothing.  Returns
 * RMHD_EINVAL if the grid needs more than RMHD_STATIC_SCRATCH_BYTES (that is
 * rmhd_adjoint_workspace_bytes(desc) > RMHD_STATIC_SCRATCH_BYTES: about
 * 212,000 padded cells, e.g. the 64 x 2048 batch) or if launch timing is on
 * (its events allocate); RMHD_EHIP if the array's address could not be
 * resolved.  Every call on one device shares the array and leaves its
 * contents behind (the parts that must start at zero are cleared inside each
 * call): calls that overlap on one device, on any streams or contexts, race
 * and must be ordered by the caller. */
#define RMHD_STATIC_SCRATCH_BYTES (128u * 1024u * 1024u)
int rmhd_step_adjoint_static(rmhd_ctx* ctx, double dt, const double* sigma, const double* U_n,
                             const double* P_n, const double* Ubar_np1, double* Ubar_n, double* sigma_bar);

/* Adjoint of rmhd_prim2con at the primitives P: Pbar = (dU/dP)^T Ubar at
 * interior cells (eqs. conserved_dens, conserved_tau, conserved_S). */
int rmhd_prim2con_adjoint(rmhd_ctx* ctx, const double* P, const double* Ubar, double* Pbar);

/* max over interior cells and active d of max|lambda^d_+-| / dx_d with the
 * characteristic speeds of Sec. III; a stable step is dt = CFL / value.
 * Synchronises the stream and writes *host_out. */
int rmhd_max_signal_speed(rmhd_ctx* ctx, double* host_out);

/* Number of failed per-cell recoveries since the last call (then reset).
 * Synchronises the stream. */
int rmhd_failures(rmhd_ctx* ctx, int64_t* host_out);

/* Number of cells set to the atmosphere state (rho_atmo > 0, Sec. IV.E) by
 * the final updates since the last call (then reset).  Synchronises the
 * stream. */
int rmhd_atmosphere_cells(rmhd_ctx* ctx, int64_t* host_out);

/* Opt-in histograms of recovery iterations (diagnostic, off by default; the
 * cost of a recovery follows its iteration count, Sec. III.B).  With enable
 * != 0 the stage kernels count, per recovered cell, the iterations its
 * recovery took: bins [0, 32) stage 1, [32, 64) stage 2, [64, 96) the final
 * update, bin b of each = b iterations (the last bin: 31 or more).
 * rmhd_recovery_stats zeroes the bins when enabling; rmhd_recovery_stats_read
 * synchronises the stream, writes the 3 * RMHD_HIST_BINS counts and zeroes
 * them. */
#define RMHD_HIST_BINS 32
int rmhd_recovery_stats(rmhd_ctx* ctx, int enable);
int rmhd_recovery_stats_read(rmhd_ctx* ctx, int64_t* bins_out);

/* Opt-in per-kernel timing (profiling aid, off by default): with enable != 0
 * the library brackets every launch with HIP events on the context's stream,
 * grouped by kernel class: 0 ghost fill (the adjoint's), 1 x fluxes, 2 y
 * fluxes, 3 z fluxes, 4 stage-2 update + stiff recovery, 5 final update +
 * recovery, 6 stage 1, 7 other pointwise kernels, 8 z fluxes with the
 * stage-2 update of each finished row (stage 2 on 3D grids in FP64 with MC2
 * or minmod, a flat or diagonal metric without shift or K and a sigma field,
 * which then has no class-4 launch).  rmhd_timing_read synchronises the stream,
 * writes the summed milliseconds and launch counts of each class since the
 * last read (arrays of RMHD_TIMING_CLASSES entries) and resets them.  If an
 * event could not be created or recorded since the last read, it resets the
 * counts, writes nothing and returns RMHD_EHIP (the launches themselves ran). */
#define RMHD_TIMING_CLASSES 9
int rmhd_timing(rmhd_ctx* ctx, int enable);
int rmhd_timing_read(rmhd_ctx* ctx, double* ms_out, int64_t* launches_out);

/* Make hip_stream (a hipStream_t; NULL = the default stream) the stream of
 * every later call on this context.  Work already queued stays on the
 * previous stream: order the two streams yourself.  (rmhd_step,
 * rmhd_imex_stage, rmhd_step_adjoint and rmhd_prim2con only launch kernels
 * when timing is off; the calls that return counters to the host
 * synchronise the stream.) */
int rmhd_set_stream(rmhd_ctx* ctx, void* hip_stream);

/* Release the context (not the workspace). */
int rmhd_destroy(rmhd_ctx* ctx);

/* Message of the last failing call on this thread ("" if none). */
const char* rmhd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RMHD_H */
