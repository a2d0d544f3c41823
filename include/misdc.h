/*
 * misdc.h - C ABI of the MI355X multi-implicit spectral deferred correction
 * library (Hamon, Day & Minion, "Concurrent implicit spectral deferred
 * correction scheme for low-Mach number combustion with detailed chemistry",
 * arXiv:1801.01201).
 *
 * One time step advances phi = (Y_1..Y_N, h) of a constant-density reacting
 * flow, phi_t = FA(phi) + FD(phi) + FR(phi), on M+1 Gauss-Lobatto nodes with
 * K correction sweeps (section 3.1).  Three sweep schemes are provided:
 *   MISDC_SCHEME_MISDC   serial node-to-node MISDC
 *                        (eqs. update_equation_misdc_discrete_form_D/R);
 *   MISDC_SCHEME_MISDCQ  serial MISDCQ with LU-trick implicit weights
 *                        (eqs. update_equation_misdcq_discrete_form_D/R);
 *   MISDC_SCHEME_CISDCQ  the concurrent scheme CISDCQ-nu: the diffusion step
 *                        at node m+1 runs on one HIP stream while the
 *                        reaction step at node m runs on another
 *                        (eqs. update_equation_amisdcq_discrete_form_D and
 *                        _R_alt, lag initialisation initial_lagged_values_*,
 *                        nu nested iterations, algorithm steps S1-S7);
 *   MISDC_SCHEME_IMEXQ   the comparison scheme IMEXQ (section 3.2.2, the
 *                        scheme whose amplification factor R'_nu the
 *                        concurrent scheme is measured against): advection
 *                        explicit, diffusion (coefficients lagged at sweep
 *                        k) and reaction implicit together in one coupled
 *                        solve of the whole grid per node (Newton's method,
 *                        BiCGStab with each cell's own block as
 *                        preconditioner).  Single grids of 9 species only.
 *
 * Conventions
 *  - Every function returns an int status: MISDC_OK (0) or a negative code.
 *    misdc_last_error() returns a thread-local message for the last failure.
 *    No exception crosses the ABI.
 *  - Fields are stored structure-of-arrays, field-major: element (f, i) of a
 *    field array is at [f * n_cells + i]; in 2-D the cell index is
 *    i = iy * nx + ix (x fastest).  A state holds N+1 fields: the N mass
 *    fractions, then the enthalpy per unit mass h (erg/g).  Units are CGS.
 *  - Pointers named dev_* are device pointers owned by the caller (for
 *    example torch tensor storage); they must stay valid until the work
 *    enqueued on the given/bound stream has completed.  Host pointers are
 *    read during the call only.  Handles own their device workspace.
 *  - Calls that take a stream (hipStream_t passed as void*, NULL = the
 *    default stream) enqueue work and return without synchronising, except
 *    where stated.  Argument errors are detected on the host before any
 *    work is enqueued (these checks need no GPU).
 *  - Only FP64 arithmetic is used unless a mixed-precision option says
 *    otherwise.
 */
#ifndef MISDC_H
#define MISDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MISDC_OK = 0,
    MISDC_EINVAL = -1,      /* invalid argument (shape, range, null pointer) */
    MISDC_ENOMEM = -2,      /* device or host allocation failed */
    MISDC_EDEVICE = -3,     /* HIP runtime error */
    MISDC_ENOTCONV = -4,    /* a solver did not converge (see the stats) */
    MISDC_EUNSUPPORTED = -5, /* valid request outside what is built */
    MISDC_ESTATE = -6       /* call out of order (a sweep without an open step, ...) */
};

enum { MISDC_SCHEME_MISDC = 0, MISDC_SCHEME_MISDCQ = 1, MISDC_SCHEME_CISDCQ = 2,
       MISDC_SCHEME_IMEXQ = 3 };
enum { MISDC_QE_CUMULATIVE = 0, MISDC_QE_LITERAL = 1 };
enum { MISDC_QI_LU = 0, MISDC_QI_BE = 1 };

typedef struct misdc_mech_s* misdc_mech_t;
typedef struct misdc_grid_s* misdc_grid_t;
typedef struct misdc_integ_s* misdc_integ_t;

/* ---------------------------------------------------------------------- */
/* Library                                                                 */
/* ---------------------------------------------------------------------- */

/* Thread-local message describing the last non-zero status of this thread. */
const char* misdc_last_error(void);

/* Library version string. */
const char* misdc_version(void);

/* ---------------------------------------------------------------------- */
/* SDC coefficients (host only, no GPU needed)                             */
/* ---------------------------------------------------------------------- */

/* Section 3.1: n_nodes Gauss-Lobatto nodes on [0, 1] (M = n_nodes - 1),
 * the integration matrix Q (M x (M+1), q_{m+1,j} = integral from 0 to
 * tau_{m+1} of the Lagrange polynomial L_j), the implicit weights QI (M x M;
 * qi_kind MISDC_QI_LU: transpose of the upper factor of the Doolittle LU
 * decomposition of transpose(Q~), Q~ = Q without its first column;
 * MISDC_QI_BE: cumulative backward Euler), the explicit weights QE (M x M;
 * MISDC_QE_CUMULATIVE: forward Euler from every earlier node,
 * MISDC_QE_LITERAL: only the (m+1, m) entry) and the node-to-node weights
 * S (M x (M+1), s_{m+1,j} = integral over [tau_m, tau_{m+1}] of L_j).
 * All weights are divided by dt.  Row-major host arrays of the stated
 * sizes; any output pointer may be NULL.  2 <= n_nodes <= 9. */
int misdc_sdc_tables(int n_nodes, int qi_kind, int qe_mode, double* tau,
                     double* Q, double* QI, double* QE, double* S);

/* ---------------------------------------------------------------------- */
/* Mechanism                                                               */
/* ---------------------------------------------------------------------- */

/* Reversible mass-action mechanism (eq. species_equation source term).
 * All arrays are host arrays, copied by misdc_mech_create.
 *   react/prod: (R x 2) species index per slot or -1; a repeated index is a
 *               stoichiometric coefficient of 2.  At most 2 + 2 slots.
 *   A, beta, Ea: kf = A T^beta exp(-Ea / (R_c T)), Ea in cal/mol.
 *   cp, hf, s0: constant molar heat capacity (erg/mol/K), enthalpy of
 *               formation at 298.15 K (erg/mol), entropy at 298.15 K and
 *               p_atm (erg/mol/K).  kr = kf / Kc with Kc from the Gibbs
 *               energies (thermodynamic consistency).
 *   D0: species diffusivities at 300 K (cm^2/s); alpha0: enthalpy
 *       diffusivity at 300 K; both scale as (T/300)^1.7.
 *   bath: the dominant species i0 whose diffusion flux closes the sum
 *         (section 2); it must not react.
 *   rho0: constant density (g/cm^3). */
typedef struct {
    int32_t n_species;
    int32_t n_reactions;
    int32_t bath;
    const double* W;
    const int32_t* react;
    const int32_t* prod;
    const double* A;
    const double* beta;
    const double* Ea;
    const double* cp;
    const double* hf;
    const double* s0;
    const double* D0;
    double alpha0;
    double rho0;
    double p_atm;
    double R_u;
    double R_c;
} misdc_mech_desc;

/* Validates and copies the mechanism to the current HIP device (2 to 256
 * species).  What each part supports:
 *   - enthalpy, temperature and the explicit transport operators: any
 *     count;
 *   - the reaction source and the reaction solve: up to 63 species (one
 *     64-lane wavefront per cell, FP64 or FP32-MFMA LU); for exactly 9
 *     species also one thread per cell (MISDC_NEWTON_THREAD); for at most 12
 *     species a one-thread-per-cell kernel generated for the mechanism
 *     (MISDC_NEWTON_SPECIALIZED, the default wherever it is loaded);
 *   - the implicit diffusion solve: up to 64 diffused fields (N - 1 species
 *     plus h);
 *   - the integrator: up to 63 species (MISDC_EUNSUPPORTED beyond). */
int misdc_mech_create(const misdc_mech_desc* desc, misdc_mech_t* out);
int misdc_mech_destroy(misdc_mech_t mech);
/* Species count of a mechanism (host, no GPU work). */
int misdc_mech_species(misdc_mech_t mech, int32_t* n_species);
/* The reaction solve generated for this mechanism (MISDC_NEWTON_SPECIALIZED):
 * misdc_mech_create writes the source of a one-thread-per-cell Newton kernel
 * (section 3.3, step S5) in which every rate constant and species index is a
 * literal, compiles it with hiprtc for the current device (once per process,
 * device and mechanism) and loads it.  Mechanisms of at most 12 species.
 * *available is 1 if it is loaded, else 0 and the generic kernels serve;
 * *status (may be NULL) points to a message owned by the mechanism saying
 * which (for instance why it was not generated).  Host only. */
int misdc_mech_specialized(misdc_mech_t mech, int32_t* available, const char** status);
/* The source text that misdc_mech_create generates for a mechanism
 * descriptor, without a device: validates the descriptor, writes the text
 * (NUL-terminated) into buf when *len is large enough and sets *len to the
 * bytes needed (buf NULL: size query).  With compile != 0 the text is also
 * compiled with hiprtc for gfx950 (no GPU needed): MISDC_EDEVICE with the
 * compiler's log in misdc_last_error if that fails.  MISDC_EUNSUPPORTED
 * above 12 species. */
int misdc_mech_generate(const misdc_mech_desc* desc, int compile, char* buf, size_t* len);

/* h = sum_k Y_k h_k(T) / W_k for n cells.  dev_Y: N x n, dev_T, dev_h: n. */
int misdc_enthalpy(misdc_mech_t mech, int64_t n, const double* dev_Y,
                   const double* dev_T, double* dev_h, void* stream);
/* Closed-form inverse: T from (Y, h). */
int misdc_temperature(misdc_mech_t mech, int64_t n, const double* dev_Y,
                      const double* dev_h, double* dev_T, void* stream);
/* FR_k = W_k omega_k(Y, T(Y, h)) / rho0 for n cells; dev_FR: N x n. */
int misdc_reaction_source(misdc_mech_t mech, int64_t n, const double* dev_Y,
                          const double* dev_h, double* dev_FR, void* stream);

enum {
    MISDC_NEWTON_AUTO = 0,       /* the generated kernel where it exists (FP64 LU),
                                    else one thread per cell for 9 species, else
                                    one wavefront per cell */
    MISDC_NEWTON_THREAD = 1,     /* one thread per cell (9 species only) */
    MISDC_NEWTON_WAVE = 2,       /* one 64-lane wavefront per cell (<= 63 species) */
    MISDC_NEWTON_SPECIALIZED = 3 /* one thread per cell, source generated for the
                                    mechanism (see misdc_mech_specialized) */
};
enum {
    MISDC_LU_FP64 = 0,           /* LU with partial pivoting in FP64 */
    MISDC_LU_FP32_MFMA = 1       /* FP32 LU (matrix cores) refined in FP64 */
};

/* Reaction step S5 (eq. reaction_step_numerical_methodology) for n
 * independent cells: solve, at constant enthalpy h,
 *     Y - c FR(Y, T) = bY,   sum_k Y_k h_k(T) / W_k = h
 * for x = (Y, T) by Newton's method with the analytic Jacobian (LU with
 * partial pivoting), globalised by pseudo-transient continuation:
 *   start from (Y_guess, T(Y_guess, h)) with an infinite pseudo-step; a trial
 *   x - delta that is not finite, has T <= 0 or some Y_k < min(bY_k, 0) -
 *   neg_slack is rejected and the pseudo-step shrinks (1/dtau: 0 -> 1/dtau0,
 *   else x4); accepted steps grow it by max(2, |G_old|/|G|) until it passes
 *   dtau_max and becomes infinite again; converged when a plain Newton step
 *   has max|delta_Y| <= tol and |delta_T| <= tol T.
 * dev_bY, dev_Y (in: guess, out: solution): N x n; dev_h, dev_c: n.
 * dev_T_out (n), dev_FR_out (N x n, FR at (Y, T(Y, h))) may be NULL.
 * dev_iters_out (n int32): linear solves per cell, -1 if not converged.
 * Parameters <= 0 take the defaults tol 1e-12, maxit 200, dtau0 1,
 * dtau_max 1e10, neg_slack 1e-6. */
typedef struct {
    double tol;
    int32_t maxit;
    double dtau0;
    double dtau_max;
    double neg_slack;
    int32_t kernel;      /* MISDC_NEWTON_*: 0 auto (one thread per cell for 9
                            species, else one wavefront per cell) */
    int32_t lu;          /* MISDC_LU_*: precision of the Newton linear solves
                            (wavefront kernel only) */
} misdc_newton_opts;

int misdc_reaction_solve_batch(misdc_mech_t mech, int64_t n, const double* dev_bY,
                               const double* dev_h, const double* dev_c,
                               double* dev_Y, double* dev_T_out, double* dev_FR_out,
                               int32_t* dev_iters_out, const misdc_newton_opts* opts,
                               void* stream);

/* ---------------------------------------------------------------------- */
/* Grid and transport                                                      */
/* ---------------------------------------------------------------------- */

/* Uniform periodic grid, dim 1 or 2; n[d], dx[d], u[d] for d = x, y.
 * u is the prescribed uniform velocity (cm/s). */
int misdc_grid_create(int dim, const int64_t* n, const double* dx,
                      const double* u, misdc_grid_t* out);
/* Ensemble of n_flames independent periodic 1-D grids of lengths[f] cells,
 * spacing dx[f] and velocity u[f]; cells are concatenated flame by flame. */
int misdc_grid_create_ensemble(int n_flames, const int64_t* lengths,
                               const double* dx, const double* u, misdc_grid_t* out);
int misdc_grid_destroy(misdc_grid_t grid);
int misdc_grid_cells(misdc_grid_t grid, int64_t* n_cells);

/* Explicit operators at a state (N+1 fields): FA = -u . grad(phi) with the
 * fourth-order face value (7(phi_i+phi_{i+1}) - (phi_{i-1}+phi_{i+2}))/12;
 * FD = div(kappa_f(T) grad phi_f) in second-order flux form with face
 * coefficient the mean of the cell values, kappa = D0_k or alpha0 times
 * (T/300)^1.7, T = T(Y, h); the bath row is minus the sum of the other
 * species rows.  dev_FA / dev_FD may be NULL. */
int misdc_transport_operators(misdc_mech_t mech, misdc_grid_t grid,
                              const double* dev_state, double* dev_FA,
                              double* dev_FD, void* stream);

/* Implicit diffusion (steps S3/S4): for every field except the bath solve
 * (I - c kappa0_f L_theta) y_f = r_f, theta = (T_lag/300)^1.7, then
 * y_bath = r_bath - sum_{k != bath} (y_k - r_k).  1-D grids: direct cyclic
 * tridiagonal solve; 2-D grids: preconditioned conjugate gradients on all
 * fields at once (diagonal preconditioner, or, on grids of at most 128 tiles
 * of 32 x 16 cells, Jacobi sweeps on each tile's own operator) until
 * |r_f|_2 <= rtol |b_f|_2 (rtol <= 0: 1e-13,
 * maxit <= 0: 500).  dev_rhs, dev_y: N+1 fields; dev_T_lag: cells;
 * dev_iters_out (int32, may be NULL) receives the iteration count.  The
 * initial guess is dev_y's content if guess_in_y is non-zero, else rhs. */
int misdc_diffusion_solve(misdc_mech_t mech, misdc_grid_t grid, double c,
                          const double* dev_T_lag, const double* dev_rhs,
                          double* dev_y, int guess_in_y, double rtol, int maxit,
                          int32_t* dev_iters_out, void* stream);

/* misdc_diffusion_solve without any allocation, for callers that cannot
 * allocate device memory: code being captured into a HIP graph, serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, kernels and
 * results (bit for bit) as misdc_diffusion_solve, but its work buffers (CG
 * vectors, face coefficients, partial sums, barrier counters) live in one
 * fixed device array of MISDC_NOALLOC_SCRATCH_MIB MiB that the library holds
 * on each device it runs on until the process ends, and the call returns
 * without synchronising (misdc_diffusion_solve waits for its solve to free
 * its buffers).  No hipMalloc, hipFree or other allocating call is made;
 * the parts that must start at zero are cleared by kernels on ``stream``.
 * Every call on a device shares that device's array: calls that may overlap
 * on one device (on different streams, or from several threads) race and
 * must be ordered by the caller.  A grid whose workspace exceeds the array
 * (about 150,000 cells at 9 species) returns MISDC_EINVAL before any work
 * is enqueued. */
#define MISDC_NOALLOC_SCRATCH_MIB 32
int misdc_diffusion_solve_noalloc(misdc_mech_t mech, misdc_grid_t grid, double c,
                                  const double* dev_T_lag, const double* dev_rhs,
                                  double* dev_y, int guess_in_y, double rtol, int maxit,
                                  int32_t* dev_iters_out, void* stream);

/* ---------------------------------------------------------------------- */
/* Integrator                                                              */
/* ---------------------------------------------------------------------- */

typedef struct {
    int32_t n_nodes;     /* M + 1 Gauss-Lobatto nodes, 2..9 */
    int32_t n_sweeps;    /* K correction sweeps per step */
    int32_t nu;          /* nested iterations per sweep (CISDCQ) */
    int32_t scheme;      /* MISDC_SCHEME_* */
    int32_t qe_mode;     /* MISDC_QE_* */
    int32_t serialize;   /* 1: run the two tasks on one stream (same DAG) */
    misdc_newton_opts newton;
    double cg_rtol;      /* 2-D diffusion CG tolerance |r| <= cg_rtol |b| (<= 0: 1e-13) */
    int32_t cg_maxit;    /* (<= 0: 500) */
    int32_t profile;     /* 1: time every diffusion-solve and Newton kernel with
                            HIP events on the stream it runs on (see stats);
                            ignored while use_graph is set */
    int32_t use_graph;   /* 1: capture a whole step (both streams and their
                            event dependencies) into one HIP graph on its first
                            call and replay it while dev_state, dt and dev_dt
                            are unchanged; a change re-captures */
    double nu_tol;       /* > 0: adaptive nested iterations (CISDCQ, nu >= 3;
                            the paper's future-work item of sections 4.1-4.3).
                            nu is then the largest number of passes.  With
                            delta_l the change of the node-M state made by
                            pass l (max over fields of max_i |new - old| /
                            max_i |new|; pass 1 against sweep k), the sweep
                            stops after pass l >= 2 if delta_l <= nu_tol *
                            delta_1.  The host waits for each delta_l, so
                            use_graph must be 0 (MISDC_EINVAL otherwise).
                            <= 0: nu passes in every sweep */
    int32_t pipeline;    /* 1: pipelined nested iterations (section 3.2.2 and
                            Fig. 2; CISDCQ with nu >= 2, no nu_tol, two
                            streams): the tasks of pass l start as soon as
                            the equations allow instead of after pass l-1,
                            so up to 2 diffusion and nu reaction tasks run
                            at once.  The diffusion tasks of pass l run on
                            one of two streams confined to the two halves of
                            every XCD's CUs (l mod 2), so two persistent
                            diffusion solves never wait for each other's
                            CUs; the reaction tasks of pass l on a stream of
                            their own; each stream has its own work buffers.
                            Results are meant to be bitwise those of
                            pipeline = 0.  Not combined with use_graph (a
                            captured graph drops the lanes' CU masks),
                            misdc_set_streams, a CU split, the stagger or a
                            learned guess (MISDC_EINVAL / MISDC_EUNSUPPORTED);
                            the diffusion solve must fit half the CUs */
    /* MISDC_SCHEME_IMEXQ's coupled solve of node m+1,
     *   phi - c (FD_lag(phi) + FR(phi)) = rhs,
     * from phi^{m+1,(k)}: Newton's method stops once every mass fraction's
     * update is at most imexq_tol and the enthalpy's at most imexq_tol times
     * its largest magnitude (<= 0: 1e-13), at most imexq_maxit iterations
     * (<= 0: 30); each Newton system
     * is solved by BiCGStab on the field-scaled unknowns to a relative
     * residual of imexq_krylov_rtol (<= 0: 1e-9), at most
     * imexq_krylov_maxit iterations (<= 0: 400).  The host reads every
     * scalar of these iterations, so a step synchronises its streams many
     * times and use_graph must be 0 (MISDC_EINVAL). */
    double imexq_tol;
    int32_t imexq_maxit;
    double imexq_krylov_rtol;
    int32_t imexq_krylov_maxit;
} misdc_opts;

/* Fills the defaults: 5 nodes, 6 sweeps, nu 1, CISDCQ, cumulative QE. */
void misdc_opts_default(misdc_opts* opts);

/* Creates an integrator for a mechanism and grid; allocates its device
 * workspace and two streams (diffusion, reaction) of default priority. */
int misdc_integ_create(misdc_mech_t mech, misdc_grid_t grid, const misdc_opts* opts,
                       misdc_integ_t* out);
/* Destroys the integrator after its streams have drained; frees its device
 * workspace and the streams it created (never a caller's). */
int misdc_integ_destroy(misdc_integ_t integ);

/* The two streams the tasks of a sweep run on (section 3.2.2: the
 * diffusion steps S3-S4 on one, the reaction steps S5-S6 on the other):
 * hipStream_t values passed as void*, for example two torch streams, used
 * in place of the integrator's own; NULL selects the integrator's own
 * stream again (so the null/default stream itself cannot be passed).  The
 * caller keeps ownership and must keep the streams alive while the
 * integrator uses them (until misdc_integ_destroy or another call of this).
 * Both streams must have the default priority.  Synchronises the streams
 * in use before the switch.  A step captured as a graph is captured again.
 * A caller's reaction stream replaces a CU-masked one (misdc_tune.cu_split
 * falls to 0 and cannot be set while it is in use).  Results do not depend
 * on the streams.  Errors: MISDC_EINVAL (equal non-NULL streams: use
 * misdc_tune.serialize for one stream), MISDC_ESTATE (a step opened by
 * misdc_step_begin is not ended). */
int misdc_set_streams(misdc_integ_t integ, void* diffusion_stream, void* reaction_stream);

/* One time step of size dt (dev_dt: NULL for a scalar dt; for an ensemble
 * grid a device array of one dt per flame, in which case dt is ignored):
 * I1-I2 spread the state to every node, I4 evaluates FA, FD, FR at it, K
 * sweeps, and the state at node M is written back to dev_state in place.
 * With per-flame step sizes every term of the sweep that carries dt (the
 * quadrature and correction terms, the implicit factors of the diffusion and
 * reaction solves) takes the dt of the cell's flame, so each flame advances
 * exactly as it would alone.  dev_dt is read by the device during the step
 * and must stay valid until the step has completed on ``stream``.
 * Ordered after prior work on ``stream`` and before later work on it.
 * Errors: MISDC_EINVAL (NULL state, dt <= 0 without dev_dt, dev_dt on a grid
 * that is not an ensemble). */
int misdc_step(misdc_integ_t integ, double* dev_state, double dt,
               const double* dev_dt, void* stream);

/* The same step one sweep at a time (section 3, steps S1-S7 per call of
 * misdc_sweep), for callers that choose the number of sweeps as they go,
 * e.g. until the sweep increment of misdc_get_stats falls below a tolerance:
 * misdc_step_begin does I1-I4 (ordered after prior work on ``stream``),
 * each misdc_sweep issues one more correction sweep (at most 64 per step;
 * ordered after prior work on its ``stream``), and misdc_step_end writes
 * node M of the last sweep into dev_state (later work on ``stream`` is
 * ordered after it), then synchronises with the integrator's streams and
 * returns MISDC_ENOTCONV if any cell-node Newton solve of the step did not
 * converge or any diffusion solve stopped at its iteration limit (the state
 * is written either way; misdc_get_stats has the counts).  misdc_get_stats
 * between sweeps synchronises and reports the sweeps done so far.  Sweeps
 * run eagerly (no graph replay).  Begin and end with the same arguments and
 * K sweeps give misdc_step with n_sweeps = K bit for bit.  Errors: as
 * misdc_step; MISDC_ESTATE for begin while a step is open, a sweep or end
 * without one, or misdc_step, misdc_autotune, misdc_set_tune,
 * misdc_set_streams, misdc_integ_set_guess or misdc_integ_record while one
 * is open. */
int misdc_step_begin(misdc_integ_t integ, double* dev_state, double dt, const double* dev_dt,
                     void* stream);
int misdc_sweep(misdc_integ_t integ, void* stream);
int misdc_step_end(misdc_integ_t integ, void* stream);

/* Launch configuration of an integrator, chosen by misdc_autotune or set by
 * the caller.  Results agree to the solvers' tolerances across choices;
 * the choice only changes speed. */
typedef struct {
    int32_t cg_variant;   /* 2-D diffusion: 0 vectors in global memory, 1/2/4
                             cells per thread held in registers, 101..103 one
                             32x16 tile per workgroup with a block-local
                             preconditioner of 1..3 Jacobi sweeps (needs
                             cg_blocks = the number of tiles) */
    int32_t cg_blocks;    /* workgroups of the 2-D diffusion solve (<= CUs) */
    int32_t cyclic;       /* 1-D diffusion: 0 one thread per periodic system,
                             1 one wavefront per system (partition method) */
    int32_t serialize;    /* 1: both tasks on one stream */
    int32_t cu_split;     /* two streams only: 0 both streams on every CU;
                             1..3 the reaction stream limited to that many
                             quarters of each XCD's CUs (a CU-masked stream),
                             the diffusion stream on all CUs */
    int32_t stagger;      /* two streams, CISDCQ only: 1 the Newton solve of
                             node m waits until the diffusion solve of node
                             m+1 is next on its stream, so that the persistent
                             CG takes its CUs first (a start-order dependency:
                             results are unchanged); the default with two
                             streams */
    double step_ms;       /* measured by misdc_autotune: mean time of one step */
    int32_t fused;        /* ensembles of 1-D flames, CISDCQ, 9 species: 1 each
                             stage of a pass (the diffusion solve at node m+1
                             and the reaction solve at node m) as one
                             persistent launch whose wavefronts take the
                             flames' tridiagonal systems (longest flames
                             first) and 64-cell chunks of Newton solves from
                             one atomic work queue; the wavefront finishing a
                             flame's last system or cell does that flame's
                             closure or explicit operators.  Needs
                             serialize = 1 (one stream), cu_split = stagger
                             = 0, the FP64 one-thread-per-cell reaction solve
                             (newton.kernel AUTO or THREAD), no learned guess
                             or recording, flames of >= 16 cells */
} misdc_tune;

/* Times candidate launch configurations on the caller's workload (reps steps
 * each, after one warm-up step, on a private copy of dev_state, which is not
 * modified), keeps the fastest one in the integrator and returns it in
 * *best.  Candidates: for 2-D grids every register-resident CG variant that
 * fits, the tiled variants when the grid has at most 128 tiles, and the
 * global-memory variant with 1/4, 1/2 and all of the CUs; for
 * 1-D grids and ensembles both cyclic solvers; each with one stream, and
 * with two streams with the reaction stream on all, 3/4 or 1/2 of the CUs
 * (staggered or not on all and on 3/4).
 * Synchronises; allocates a state copy.  Errors as misdc_step. */
int misdc_autotune(misdc_integ_t integ, const double* dev_state, double dt,
                   const double* dev_dt, int reps, misdc_tune* best, void* stream);
/* Reads / sets the launch configuration (set: MISDC_EINVAL if the CG
 * variant cannot hold the grid, the block count exceeds the CUs or cu_split
 * is outside [0, 3], stagger is not 0 or 1, or the CU count is not a multiple of 32; MISDC_EDEVICE if
 * the runtime does not apply the CU mask). */
int misdc_get_tune(misdc_integ_t integ, misdc_tune* tune);
int misdc_set_tune(misdc_integ_t integ, const misdc_tune* tune);

/* Statistics of the last step (synchronises with the integrator's streams).
 * sweep_increment[k] = max over fields of max_i |phi^{M,(k+1)} - phi^{M,(k)}|
 * normalised by max_i |phi^{M,(k+1)}| of that field.
 * misdc_step is asynchronous and returns before its solves finish, so this
 * call reports their outcome: it fills *stats and returns MISDC_ENOTCONV if
 * newton_failed or cg_failed is above zero (cells whose Newton iteration
 * reached newton.maxit or stalled; diffusion solves that reached cg_maxit,
 * whose workgroups timed out waiting for each other, or, with the tiled 2-D
 * CG, whose result's own residual |b - A y|, taken over the cells whose four
 * neighbours lie in the same 32 x 16 tile, exceeded 10 cg_rtol |b| in some
 * field although the iteration's recurrence residual met the tolerance),
 * else MISDC_OK. */
typedef struct {
    int64_t newton_solves;      /* cell-node Newton solves */
    int64_t newton_iters;       /* total linear solves */
    int32_t newton_max;
    int64_t newton_failed;
    int64_t cg_solves;
    int64_t cg_iters;           /* sum over 2-D diffusion solves */
    int32_t cg_max;
    int32_t cg_failed;
    int32_t n_sweeps;
    double sweep_increment[64];
    /* with opts.profile: summed device durations (ms) and launch counts of
     * the implicit-diffusion solve kernels and of the Newton kernels since
     * the integrator was created or the last misdc_reset_profile() */
    double diffusion_kernel_ms;
    int64_t diffusion_kernel_launches;
    double newton_kernel_ms;
    int64_t newton_kernel_launches;
    /* with newton.lu = MISDC_LU_FP32_MFMA (last step): FP32 solves done by
     * the refinement, and Newton iterations that fell back to the FP64 LU
     * because the refinement did not contract */
    int64_t newton_lu_solves;
    int64_t newton_lu_fallbacks;
    /* with a learned guess (misdc_integ_set_guess, last step): cell-node
     * solves that started from the network's guess */
    int64_t newton_guess_learned;
    /* nested iterations done in each sweep of the last step (nu, or fewer
     * with opts.nu_tol) */
    int32_t nested_passes[64];
    /* generated reaction solve (MISDC_NEWTON_SPECIALIZED, last step): Newton
     * iterations whose diagonal pivots failed the threshold test and were
     * factored again with partial pivoting */
    int64_t newton_pivot_retries;
    /* MISDC_SCHEME_IMEXQ (last step): coupled solves, their Newton
     * iterations, solves that reached imexq_maxit (counted in newton_failed
     * too, so that the step reports MISDC_ENOTCONV), BiCGStab iterations
     * (sum and largest per Newton system) and Newton systems whose
     * BiCGStab stopped short of imexq_krylov_rtol */
    int64_t imexq_solves;
    int64_t imexq_newton_iters;
    int64_t imexq_failed;
    int64_t imexq_krylov_iters;
    int64_t imexq_krylov_max;
    int64_t imexq_krylov_failed;
} misdc_stats;

/* Outcomes of the last step's cell-node Newton solves in sweep k (0 <= k <
 * n_sweeps of that step; MISDC_EINVAL otherwise), for the per-sweep
 * iteration statistics of the reaction step S5: counts[0] = solves that did
 * not converge, counts[v] = solves that converged after v linear solves
 * (1 <= v <= 62), counts[63] = after 63 or more.  counts is a host array of
 * 64 entries owned by the caller.  Synchronises with the integrator's
 * streams.  The counts of a sweep add up to cells x M x (the sweep's
 * nested passes: nu, or fewer with opts.nu_tol). */
int misdc_get_newton_histogram(misdc_integ_t integ, int sweep, int64_t* counts);

/* Clears the accumulated kernel timings of opts.profile. */
int misdc_reset_profile(misdc_integ_t integ);

int misdc_get_stats(misdc_integ_t integ, misdc_stats* stats);

/* ---------------------------------------------------------------------- */
/* Learned Newton initial guess                                            */
/* ---------------------------------------------------------------------- */
/* An extension of the reaction step S5 (eq. reaction_step_numerical_
 * methodology), where the paper starts Newton from the previous iterate: a
 * dense network n_in -> n_hidden -> n_hidden -> n_out with ReLU hidden
 * layers, n_in = N + 2 inputs (b_Y, T_b = T(b_Y, h), ln c, each normalised
 * as (v - mu) / sd) and n_out = N + 1 outputs (Y* - b_Y, T* - T_b, each
 * divided by its sd).  Products on the matrix cores with BF16 operands and
 * FP32 accumulation (MISDC_MLP_BF16), or FP32 operands (MISDC_MLP_FP32).
 * Parameters are FP32, packed as W1 (n_in x n_hidden, row-major), b1, W2,
 * b2, W3, b3.  Device arrays of features and targets are FP32, row-major
 * (batch x n_in, batch x n_out).  A network handle holds work buffers sized
 * for the largest batch seen; calls on one handle must not overlap. */
typedef struct misdc_mlp_s* misdc_mlp_t;
enum { MISDC_MLP_BF16 = 0, MISDC_MLP_FP32 = 1 };

/* Creates a network with zero parameters and identity normalisation
 * (widths in [1, 512]; MISDC_EINVAL otherwise). */
int misdc_mlp_create(int n_in, int n_hidden, int n_out, int precision, misdc_mlp_t* out);
int misdc_mlp_destroy(misdc_mlp_t mlp);
int misdc_mlp_param_count(misdc_mlp_t mlp, int64_t* count);
/* Host FP32 arrays of param_count values; setting resets the Adam state. */
int misdc_mlp_set_params(misdc_mlp_t mlp, const float* host_params);
int misdc_mlp_get_params(misdc_mlp_t mlp, float* host_params);
/* Host arrays: in_mu, in_sd (n_in), out_sd (n_out); scales must be > 0. */
int misdc_mlp_set_normalization(misdc_mlp_t mlp, const float* in_mu, const float* in_sd,
                                const float* out_sd);
/* y = network(x) for batch rows. */
int misdc_mlp_forward(misdc_mlp_t mlp, int64_t batch, const float* dev_x, float* dev_y,
                      void* stream);
/* Gradient (packed like the parameters) of the loss mean((y - t)^2) over
 * the batch rows and the outputs; dev_loss (1 float, may be NULL) gets the
 * loss.  Deterministic (fixed-order reductions, no atomics). */
int misdc_mlp_gradients(misdc_mlp_t mlp, int64_t batch, const float* dev_x, const float* dev_t,
                        float* dev_grad, float* dev_loss, void* stream);
/* One Adam step (bias-corrected moments) with the given gradient. */
int misdc_mlp_adam_step(misdc_mlp_t mlp, const float* dev_grad, float lr, float beta1,
                        float beta2, float eps, void* stream);
/* epochs passes over floor(n / batch) consecutive minibatches of the
 * training set (the caller shuffles it), each forward + gradient + Adam
 * (0.9, 0.999, 1e-8); dev_loss (epochs floats, may be NULL) gets the loss
 * of each epoch's last minibatch. */
int misdc_mlp_train(misdc_mlp_t mlp, int64_t n, const float* dev_x, const float* dev_t,
                    int64_t batch, int epochs, float lr, float* dev_loss, void* stream);
/* Normalised features of n reaction problems (dev_bY: N x n, dev_h, dev_c:
 * n) and normalised targets from their solutions dev_Y (N x n). */
int misdc_mlp_features(misdc_mech_t mech, misdc_mlp_t mlp, int64_t n, const double* dev_bY,
                       const double* dev_h, const double* dev_c, float* dev_x, void* stream);
int misdc_mlp_targets(misdc_mech_t mech, misdc_mlp_t mlp, int64_t n, const double* dev_bY,
                      const double* dev_h, const double* dev_Y, float* dev_t, void* stream);
/* Training set of n reaction problems (dev_bY: N x n, dev_h, dev_c: n) and
 * their solutions dev_Y (N x n), 2 <= n <= 2^31: sets the network's
 * normalisation from the data and writes the normalised features (dev_x,
 * n x (N+2)) and targets (dev_t, n x (N+1)) in shuffled row order, ready for
 * misdc_mlp_train.  The statistics are FP64 column sums in a fixed order:
 * in_mu = mean of each raw feature, in_sd = its sample standard deviation
 * floored at max(1e-3 |in_mu|, 1e-6), out_sd = the sample standard
 * deviation of each raw target floored at 1e-30.  Problem i goes to row
 * (a i + b) mod n, with a coprime to n and b drawn from ``seed``
 * (SplitMix64).  Work buffers are allocated and freed on the stream. */
int misdc_mlp_prepare_training(misdc_mech_t mech, misdc_mlp_t mlp, int64_t n, const double* dev_bY,
                               const double* dev_h, const double* dev_c, const double* dev_Y,
                               uint64_t seed, float* dev_x, float* dev_t, void* stream);
/* Initial guess of misdc_reaction_solve_batch: dev_Y (N x n) holds the plain
 * guess on entry; each cell takes the network's guess (b_Y + predicted
 * increment) instead if
 * its residual |Y - c FR(Y, T(Y, h)) - b_Y|_2 is smaller (the network's
 * guess is first raised to min(b_Y, 0) where it falls below, the floor of
 * the Newton iteration's trial acceptance).  dev_choice (n
 * int32, may be NULL) records 1 where the learned guess was taken. */
int misdc_reaction_guess_mlp(misdc_mech_t mech, misdc_mlp_t mlp, int64_t n, const double* dev_bY,
                             const double* dev_h, const double* dev_c, double* dev_Y,
                             int32_t* dev_choice, void* stream);
/* Every reaction task of the first ``sweeps`` sweeps of later steps (0:
 * every sweep) starts from the learned guess where it has the smaller
 * residual (mlp NULL: the plain guess, the previous iterate, everywhere).
 * Allocates the network's buffers for the grid; the network must outlive
 * its use.  Synchronises.  MISDC_ESTATE while a step opened by
 * misdc_step_begin is not ended (as for misdc_integ_record). */
int misdc_integ_set_guess(misdc_integ_t integ, misdc_mlp_t mlp, int sweeps);
/* Records the reaction problems of later steps: task t (in issue order, up
 * to max_tasks) writes (b_Y: N x n, h: n, c: n, Y: N x n) doubles at
 * dev_buf + t (2N + 2) n.  max_tasks = 0 stops recording.  Steps are not
 * replayed as graphs while recording.  Synchronises. */
int misdc_integ_record(misdc_integ_t integ, double* dev_buf, int64_t max_tasks);
int misdc_integ_recorded(misdc_integ_t integ, int64_t* tasks);

#ifdef __cplusplus
}
#endif

#endif /* MISDC_H */
