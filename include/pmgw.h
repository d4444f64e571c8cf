/*
 * pmgw.h -- C ABI of the MI355X p-multigrid pressure Poisson library.
 *
 * The library solves the pressure Poisson problem of a sigma-transformed free-surface
 * Navier-Stokes wave model with a Fourier basis in x and a Chebyshev basis in sigma
 * (Melander, Bitsch, Chen, Engsig-Karup, "A High-Order Hybrid-Spectral Incompressible
 * Navier-Stokes Model For Nonlinear Water Waves"). It does so for one tank or for a batch
 * of independent tanks of uneven size.
 *
 * Conventions (all entry points)
 *   - A field of tank t is a float64 array [Nz_t][Nx_t], row-major, x fastest. Row j holds
 *     sigma_j = (1 + cos(j pi / M)) / 2 with M = Nz - 1: row 0 is the free surface
 *     (sigma = 1), row M the bed (sigma = 0). Column i holds x_i = i L_t / Nx_t.
 *     Tanks are packed back to back: tank t starts at element off2d[t] (see
 *     pmgw_field_offsets). One-dimensional fields (h, eta) are packed the same way with off1d.
 *   - Every field pointer is a DEVICE pointer owned by the caller, 8-byte aligned, on the
 *     device that was current at pmgw_plan_create. The library never allocates device
 *     memory: it reports a workspace size and the caller binds a device buffer of that size.
 *   - Every call enqueues work on the plan's stream and returns without waiting, except when
 *     a non-NULL HOST info pointer is given: then it waits for the stream before returning.
 *   - Return codes: 0 = OK; > 0 = soft failure, outputs valid (PMGW_NOCONV); < 0 = hard
 *     error, outputs unspecified. pmgw_last_error() describes the last failure of the
 *     calling thread. No C++ exception crosses this interface.
 *   - Sizes: Nx a power of two with 8 <= Nx <= 2048; Nz = M + 1 with M in {2, 4, 8, 16, 32}
 *     and Nx >= 2 M; L > 0; 1 <= ntanks <= 65536.
 *   - Calls on one plan must not overlap (the workspace is shared); plans are independent.
 */
#ifndef PMGW_H
#define PMGW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PMGW_OK = 0,
    PMGW_NOCONV = 1,       /* maxit reached; best iterate returned, relres in info          */
    PMGW_EINVAL = -1,      /* bad argument: NULL, size, precision, rtol, unbound workspace  */
    PMGW_EGEOM = -2,       /* water depth d = h + eta <= 0 (or not finite) somewhere        */
    PMGW_ENAN = -3,        /* NaN/Inf met in the right-hand side or the Krylov scalars     */
    PMGW_EWORKSPACE = -4,  /* workspace missing, too small or misaligned                    */
    PMGW_EDEVICE = -5      /* a HIP runtime call failed                                     */
};

enum { PMGW_FP64 = 0, PMGW_MIXED = 1 };

/* Preconditioner of poisson_solve: one V-cycle (paper Alg. 1) or one full-multigrid cycle
 * (paper Alg. 2) per FGMRES iteration. */
enum { PMGW_CYCLE_V = 0, PMGW_CYCLE_FMG = 1 };

/* Solver and model options. pmgw_default_opts fills the defaults given in brackets. */
typedef struct {
    int32_t nu1;            /* pre-smoothing pairs per level [1]                              */
    int32_t nu2;            /* post-smoothing pairs per level [1]                             */
    int32_t coarse_pairs;   /* smoothing pairs on the coarsest level (order 2) [1]            */
    int32_t restart;        /* FGMRES restart length, 1..32 [30]                              */
    double omega_c;         /* damping of the column-block step [1.0]                         */
    double omega_m;         /* damping of the flat-mode step [1.0]                            */
    double rho;             /* density [1000]                                                 */
    double g;               /* gravity magnitude [9.81]                                       */
    double nu_visc;         /* kinematic viscosity [1e-6]                                     */
    double filt_alpha;      /* filter strength alpha [36]                                     */
    double filt_s;          /* filter order s [2]                                             */
    double filt_fx;         /* x cut-off fraction of Nx/2 [0.5]                               */
    double filt_fz;         /* sigma cut-off fraction of M [0.9]                              */
    int32_t threads;        /* threads per solve workgroup: 64, 128, 256 or 512; 0 = 256 [0]
                               (512 applies to global-memory cycles of forward solves; LDS-
                               resident cycles and adjoint solves use at most 256)           */
    int32_t adapt_omega_m;  /* 1: scale omega_m per tank by the depth-variation rule below [1]   */
    int32_t cycle;          /* FGMRES preconditioner: PMGW_CYCLE_V or PMGW_CYCLE_FMG [V]       */
    int32_t coarse_exact;   /* coarsest level (order 2): 0 = coarse_pairs smoothing pairs,
                               1 = direct solve in float64 (paper Alg. 1), Nx <= 512 [0]    */
    int32_t resident;       /* PMGW_MIXED V-cycles: 1 = keep the cycle's level fields in LDS
                               for the tanks where they fit (Nz <= 17, 64 <= Nx <= 512, e.g.
                               256 x 17 and 512 x 5), 0 = always in global memory. Same
                               arithmetic either way [1]                                    */
    int32_t class_threads[5];  /* per finest-level class (3, 5, 9, 17, 33 rows): threads per
                               solve workgroup for that class's tanks, same values and limits
                               as threads; 0 = use threads [0]                              */
    int32_t class_resident[5]; /* per class: 0 = as resident, 1 = LDS-resident cycle where it
                               fits, 2 = global-memory cycle [0]                            */
    int32_t bed_line;       /* 1 = end every smoothing pair with the bed-line step below
                               (Nx <= 1024; the V-cycle then runs in global memory) [0]     */
    int32_t linear;         /* rk4_stage model: 1 = the linearised equations of the paper's
                               small-amplitude analysis (eq. NSElin, eq. linFS): no advection,
                               eta_t = w at the surface, sigma-map held on the still-water
                               domain (the plan's geometry is set with eta = 0) [0]          */
    int32_t no_slip;        /* rk4_stage bed: 1 = no-slip bed u = w = 0 (paper Sec. 5,
                               oscillatory wave boundary layer), see rk4_stage [0]           */
    int32_t guess_steps;    /* rk4_stage initial guess: 0 = the solve starts from p as passed
                               (the previous stage's pressure); m in 2..5 = from the
                               extrapolation of the same stage's pressure over the previous m
                               steps, see rk4_stage [0]                                     */
    int32_t guess_correct;  /* with guess_steps: 1 = add the previous stage's extrapolation
                               error to the extrapolation, see rk4_stage [0]                 */
} pmgw_opts;

/* Per-tank outcome of a solve. status is one of the codes above for that tank. */
typedef struct {
    int32_t iters;          /* FGMRES iterations (preconditioner applications)                */
    int32_t status;
    double relres;          /* ||b - A p||_2 / ||b||_2 of the returned p (0 when b = 0)       */
} pmgw_info;

typedef struct pmgw_plan_s* pmgw_plan;

/* The depth-variation rule of adapt_omega_m: with c = 1/(d_old d_new) over the tank's columns
 * and r = max c / min c, omega_m is multiplied by min(1, 2 / (1 + (r/2)^0.4)); it is 1 for flat
 * and mildly varying depth (r <= 2) and about 0.56 at a depth ratio of 4.6. */

/* The bed-line step (bed_line = 1), a line relaxation along x of the bed row (paper Sec. 4.3's
 * block smoother idea applied to the bed condition): the bed row couples the columns through
 * h_x D_x, which the column blocks and the x-averaged mode blocks leave out, and on steep,
 * finely resolved beds (max|h_x| kappa_max / M^2 above ~0.3) the cycle without it amplifies
 * the error. The step solves the bed row's own Nx x Nx block L_b of A exactly with the other
 * rows held, x_M <- L_b^-1 (f_M + (h_x sigma_x[M] + 1/d) sum_{l<M} (D_sigma)_Ml x_l) on the old
 * geometry. pmgw_set_geometry inverts L_b per level on the device (Gauss-Jordan with partial
 * pivoting, float64, Nx^3 multiply-adds per level; 12 Nx^2 bytes of workspace per level). */

/* The direct coarsest-level solve (coarse_exact = 1): pmgw_set_geometry forms, per tank, the
 * order-2 operator with its Dirichlet surface row eliminated (2 Nx unknowns, every x column
 * coupled through D_x) and inverts it on the device by Gauss-Jordan elimination with partial
 * pivoting, in float64 (about 12 Nx^3 multiply-adds per tank and geometry, 96 Nx^2 bytes of
 * workspace); each V-cycle then applies the stored inverse in float64, in mixed plans too. */

/* Fill *opts with the defaults. */
void pmgw_default_opts(pmgw_opts* opts);

/*
 * Create a plan for ntanks tanks with host arrays nx[ntanks], nz[ntanks], L[ntanks].
 * precision: PMGW_FP64 (everything in float64) or PMGW_MIXED (V-cycle smoothing, transfers
 * and block inverses in float32; operator residuals, Krylov work, metrics and the solution
 * in float64). opts may be NULL for the defaults. stream is a hipStream_t (NULL = default).
 * On success *out receives the plan; the caller destroys it with pmgw_plan_destroy.
 */
int pmgw_plan_create(pmgw_plan* out, int32_t ntanks, const int32_t* nx, const int32_t* nz,
                     const double* L, int32_t precision, const pmgw_opts* opts, void* stream);

/* Bytes of device workspace the plan needs (256-byte aligned buffer). */
size_t pmgw_workspace_bytes(pmgw_plan plan);

/*
 * Bind a device buffer of at least pmgw_workspace_bytes bytes, 256-byte aligned, owned by
 * the caller and kept alive while the plan is used. Copies the plan's constant tables into
 * it (synchronous). Must precede every compute call.
 */
int pmgw_bind_workspace(pmgw_plan plan, void* dev_ptr, size_t bytes);

/* Host outputs: off2d[ntanks+1] element offsets of 2D fields, off1d[ntanks+1] of 1D fields. */
int pmgw_field_offsets(pmgw_plan plan, int64_t* off2d, int64_t* off1d);

/*
 * Set the two geometries of the mixed-stage operator (paper eq. poissonp): h is the still-
 * water depth, eta_old the surface of stage k-1 (it carries the gradient and the bed
 * condition), eta_new the surface of stage k (it carries the divergence). eta_new may equal
 * eta_old (single-geometry problem). Computes the sigma-metrics (eq. 1_Scoef) and the
 * smoother's block inverses on the device. A tank with d <= 0 is marked: its later solves
 * report PMGW_EGEOM in info. All three are device arrays packed with off1d.
 */
int pmgw_set_geometry(pmgw_plan plan, const double* h, const double* eta_old,
                      const double* eta_new);

/*
 * Ap = A p (paper eq. poissonp with eq. bcpd and eq. bcpdneu): interior rows
 * Div^new(Grad^old p); row 0 = p (surface Dirichlet row); row M = -(h_x G_x + G_z) with
 * (G_x, G_z) = Grad^old p (bed impermeability row, un-normalised outward normal).
 * p and Ap are device fields; they must not overlap. Always float64.
 */
int laplacian_apply(pmgw_plan plan, const double* p, double* Ap);

/*
 * z = one p-multigrid V-cycle applied to r from a zero initial guess (paper Alg. 1, with
 * the coarsening of Sec. 4.1 and the modal transfers of Sec. 4.2). In PMGW_MIXED plans the
 * cycle runs in float32 (r is rounded on entry, z widened on exit). r and z are device
 * fields and must not overlap.
 */
int pmg_vcycle(pmgw_plan plan, const double* r, double* z);

/*
 * z = one full-multigrid cycle applied to r (paper Alg. 2): the right-hand side restricted to
 * every level; on the coarsest level the coarse cycle from zero; on each finer level the
 * prolongated result u of the level below, improved by one V-cycle of that level started from
 * u (evaluated as u + V_0(f - A u), V_0 the cycle from zero). Same conventions as pmg_vcycle.
 */
int pmgw_fmg(pmgw_plan plan, const double* r, double* z);

/*
 * Solve A p = b for every tank with flexible GMRES right-preconditioned by one V-cycle per
 * iteration (paper Sec. 4.4). p holds the initial guess on entry and the solution on exit.
 * Stops a tank when its true relative residual ||b - A p||_2/||b||_2 <= rtol or after maxit
 * iterations (PMGW_NOCONV). rtol > 0, maxit >= 1. info_dev (device, ntanks entries) and
 * info_host (host, ntanks entries; makes the call synchronous) are optional. The return
 * value is the worst tank status (hard errors first) when info_host is given, else the
 * launch status.
 */
int poisson_solve(pmgw_plan plan, const double* b, double* p, double rtol, int32_t maxit,
                  pmgw_info* info_host, pmgw_info* info_dev);

/*
 * One stage k (1..5) of the 5-stage 2N low-storage Runge-Kutta scheme (paper eq. LSERK,
 * Sec. 3.2 and 3.3) with the Carpenter-Kennedy (5,4) coefficients, for every tank:
 * kinematic surface update and filter, metrics of the old and new surface, forcing at the
 * old stage, provisional velocity, pressure right-hand side, poisson_solve (warm-started
 * from p), projection and velocity update, filter of u and w. u, w, Ku, Kw, p are device
 * fields; h, eta, Keta device 1D fields; all are updated in place except h. On exit p holds
 * the stage's dynamic pressure p_D^(k-1). The K registers need no reset between steps
 * (stage 1 multiplies them by alpha_1 = 0) but must hold finite values. The workspace keeps
 * the stage's intermediate fields; the plan's geometry is left at (eta^(k-1), eta^(k)), or at
 * the still-water geometry (eta = 0) with opts.linear.
 * With opts.no_slip the bed rows of u, w, Ku and Kw are set to zero after the update and the
 * filter; the bed row of the pressure problem keeps its form (with zero bed velocity at the
 * stage start its datum is the normal component of the momentum forcing, viscous stress
 * included), and the viscous term is left out on the surface row, for which the paper gives no
 * stress condition (the surface row moves by the inviscid momentum equation). Pass a state whose
 * bed rows of u, w, Ku, Kw are zero.
 * With opts.guess_steps = m >= 2 the plan records, at the start of each call, the pressure in p
 * (the previous call's result) as that stage's value for the current step, and starts the solve
 * from the polynomial extrapolation, in the step index, of stage k's pressure over its last
 * c = min(m, recorded) steps: p0 = sum_{i=1..c} (-1)^(i+1) C(c, i) p_k[n - i] (degree c - 1
 * through equally spaced steps). With c < 2 the solve starts from p as passed. The record
 * restarts when a call's k does not follow the previous call's k cyclically (1..5, 1..) or
 * dt changes, and on pmgw_history_reset. The stopping rule is unchanged: every solve still
 * reaches rtol; only its starting point differs. Workspace: 5 m n2d doubles more. The record's
 * slots are chosen on the host at each call, so a stage captured into a HIP graph replays the
 * slots of its capture: capture stages only of plans without guess_steps.
 * With opts.guess_correct = 1 as well, a call whose previous call (in order) started from an
 * extrapolation E' and returned p' starts from E + (p' - E') instead of E: the extrapolation
 * error of one stage is close to that of the next, whose pressure moves along with it. Without
 * such a previous call (first calls, after a restart of the record) it starts from E. The
 * extrapolations are kept in n2d doubles more of workspace.
 */
int rk4_stage(pmgw_plan plan, int32_t k, double dt, const double* h, double* u, double* w,
              double* eta, double* Ku, double* Kw, double* Keta, double* p, double rtol,
              int32_t maxit, pmgw_info* info_dev);

/*
 * Wave-flume relaxation zones (paper Sec. 5, harmonic generation over a submerged bar: waves
 * generated and absorbed by relaxation toward a target in zones at the ends of the flume).
 *
 * pmgw_stream_target writes the target fields of every tank at time t: a steady
 * stream-function wave (Fourier approximation) with coefficients coef (DEVICE array, per tank
 * 2 nmodes + 6 doubles: k, c, ubar, h0, x0, E_0..E_nmodes, B_1..B_nmodes), scaled by a * S(x)
 * (window S: device 1D field). With X = x - x0 - c t, s = a S:
 *   eta_t = s sum_q E_q cos(q k X); on the target's sigma grid zeta_j = sigma_j (h0 + eta_t),
 *   u_t = s ((c - ubar) + sum_q q k B_q cosh(q k zeta)/cosh(q k h0) cos(q k X)),
 *   w_t = s sum_q q k B_q sinh(q k zeta)/cosh(q k h0) sin(q k X).
 * nmodes in [1, 64]. Outputs are device fields (2D u_t, w_t, 1D eta_t).
 *
 * pmgw_relax blends the state toward the targets: q <- q + r (q_t - q) for u, w (every row) and
 * eta, with the relaxation strength r per column (device 1D field, values in [0, 1]). Meant once
 * per time step after the five rk4_stage calls (the next step's first stage multiplies the K
 * registers by zero, so they need no blend). Both calls enqueue on the plan's stream and need a
 * bound workspace.
 */
int pmgw_stream_target(pmgw_plan plan, const double* coef, int32_t nmodes, double t, double a,
                       const double* window, double* u_t, double* w_t, double* eta_t);
int pmgw_relax(pmgw_plan plan, const double* r, const double* u_t, const double* w_t,
               const double* eta_t, double* u, double* w, double* eta);

/* Forget the pressures recorded for opts.guess_steps and the last extrapolation kept for
 * opts.guess_correct (e.g. before stepping a new initial state with the same plan); the next
 * rk4_stage calls start from p as passed until two steps are recorded again. No-op for plans
 * without guess_steps. */
int pmgw_history_reset(pmgw_plan plan);

/*
 * out = A^T lambda for the operator of laplacian_apply (its exact transpose: D_x^T = -D_x,
 * explicit D_sigma^T, transposed boundary rows). Needed by the discrete adjoint of the
 * pressure solve. lambda and out are device fields and must not overlap. Always float64.
 */
int pmgw_adjoint_apply(pmgw_plan plan, const double* lambda, double* out);

/*
 * z = M^T r, the transpose of the linear map r -> pmg_vcycle(r): the V-cycle on A^T with
 * every smoothing step transposed and taken in reverse order, restriction by P^T and
 * prolongation by R^T. In PMGW_FP64 plans <pmg_vcycle(a), b> = <a, pmgw_adjoint_vcycle(b)> to
 * rounding. r and z must not overlap.
 */
int pmgw_adjoint_vcycle(pmgw_plan plan, const double* r, double* z);

/*
 * lambda = A^-T g: flexible GMRES on the transposed operator, right-preconditioned by M^T
 * (pmgw_adjoint_vcycle), in float64 (the cycle in the plan's precision). lambda holds the
 * initial guess on entry. Same conventions, stopping rule and return values as poisson_solve.
 */
int pmgw_adjoint_solve(pmgw_plan plan, const double* g, double* lambda, double rtol,
                       int32_t maxit, pmgw_info* info_host, pmgw_info* info_dev);

/*
 * Reverse of rk4_stage (its discrete adjoint), for gradients through time stepping.
 * u, w, eta, Ku, Kw, Keta: the stage's INPUT state (as passed to rk4_stage; unchanged here).
 * ub, wb, etab, Kub, Kwb, Ketab: on entry the adjoints of the stage's outputs, on exit the
 * adjoints of its inputs (in place). hbar: adjoint of the depth h, ACCUMULATED (+=).
 * The call recomputes the stage's intermediates (including its pressure solve, to rtol) in the
 * workspace, then solves one adjoint system A^T lambda = pbar (pmgw_adjoint_solve, to rtol).
 * info_dev (device, nullable) holds 2 x ntanks records: entries [0, ntanks) receive the forward
 * recompute solve's outcome per tank, entries [ntanks, 2 ntanks) the adjoint solve's. The forward
 * solve is differentiated as exact.
 * The plan's geometry is left at the stage's (eta^(k-1), eta^(k)). Plans created with
 * opts.linear or opts.no_slip are refused (PMGW_EINVAL): the adjoint covers the default model.
 */
int rk4_stage_adjoint(pmgw_plan plan, int32_t k, double dt, const double* h, const double* u,
                      const double* w, const double* eta, const double* Ku, const double* Kw,
                      const double* Keta, double* ub, double* wb, double* etab, double* Kub,
                      double* Kwb, double* Ketab, double* hbar, double rtol, int32_t maxit,
                      pmgw_info* info_dev);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): pmgw_set_geometry followed by poisson_solve, run in
 * the library's static scratch array instead of a bound workspace. The plan needs no workspace
 * (one bound to it is neither used nor changed) and must have been created on the current
 * device. The array holds 48 MiB per device (every single tank up to 1024 x 33 in either
 * precision fits); a plan whose pmgw_workspace_bytes exceeds it is refused with
 * PMGW_EWORKSPACE before anything is launched. The call allocates nothing: the array is a
 * file-scope device array, present on each device the library runs on until the process ends.
 * Each device has one such array, shared by every call on that device, and it keeps the last
 * call's contents: the first call of a plan (and the first after another plan used the array)
 * copies the plan's constant tables into it from host memory, later calls of the same plan only
 * launch kernels (every other value the call reads, it first writes). Calls that overlap on one
 * device -- on different streams, plans or threads -- race on the array and must not be made.
 * The Nz classes of a batch run one after another on the plan's stream. Arguments, outputs,
 * info and return values as for pmgw_set_geometry and poisson_solve.
 */
int poisson_solve_noalloc(pmgw_plan plan, const double* h, const double* eta_old,
                          const double* eta_new, const double* b, double* p, double rtol,
                          int32_t maxit, pmgw_info* info_host, pmgw_info* info_dev);

/* Release the plan (not the workspace, which the caller owns). NULL is ignored. */
void pmgw_plan_destroy(pmgw_plan plan);

/* Launch timing of the solve kernels, for measurement. capacity > 0 starts recording: every
 * following poisson_solve call (also the one inside rk4_stage) records a pair of HIP events on
 * the plan's stream around its kernel launches, for the first `capacity` calls; the previous
 * record is cleared. capacity = 0 stops recording. Events are created on the host here, never
 * device memory. Returns PMGW_EINVAL for capacity outside [0, 2^20]. */
int pmgw_profile(pmgw_plan plan, int32_t capacity);

/* Waits for the recorded events and returns the number of timed solve calls, their summed and
 * their largest duration in milliseconds (host pointers). */
int pmgw_profile_read(pmgw_plan plan, int32_t* launches, double* total_ms, double* max_ms);

/* Message of the last failing call on this thread ("" if none). Valid until the next call. */
const char* pmgw_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PMGW_H */
