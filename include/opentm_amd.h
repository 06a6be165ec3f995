/*
 * opentm_amd.h -- C ABI of the MI355X (gfx950) periodic thermal
 * homogenization library.
 *
 * The library computes one design iteration of the density-based thermal
 * microstructure method of Quan, Zhai and Fu ("OpenTM", arXiv 2405.19991):
 *
 *   density filter (Sec. 2.3, filter equation)
 *     -> SIMP conductivity k_e = kmin + rho~_e^p (k0 - kmin)   (Sec. 2.2)
 *     -> macro loads f^(i) for the three unit gradients        (Sec. 2.4, enforceMacroLoad)
 *     -> matrix-free hex-8 conduction operator [KT]_v inside Jacobi-preconditioned
 *        conjugate gradients, three load cases                 (Sec. 2.4, FEM; eq. K T^(i) = f^(i))
 *     -> homogenized tensor kappa^H                             (Sec. 2.2, discrete homogenization formula)
 *     -> objective and sensitivities, filter transpose          (Sec. 2.3 chain rule and sensitivity equation)
 *     -> adaptive volume bound V*                               (Algorithm 1)
 *     -> Optimality Criteria update                             (Sec. 3.3, OCOptimizer; Sec. 3.4 step 6)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  Grid     : periodic cube of n^3 voxel elements and n^3 nodes; node (i,j,k)
 *             is the lower corner of element (i,j,k); flat index
 *             i + n*(j + n*k) (x fastest).  4 <= n <= 1024.
 *  Fields   : float64, flat, in that order.  Three-load fields (macro loads,
 *             fluctuations chi) are load-major: [load][n^3].  chi is in voxel
 *             units and has zero mean per load.
 *  Tensor   : 6-vector [k11, k22, k33, k12, k23, k13] (Sec. 2.2 correspondence).
 *  Ownership: a context owns all device memory it allocates.  Host pointers
 *             are owned by the caller, read or written only during the call
 *             and never retained.  Device pointers passed in are read or
 *             written only during the call, on the context's (or the given)
 *             HIP stream; the call returns after that work has completed.
 *  Errors   : every int-returning function returns an OTM_* status.  Nothing
 *             throws or aborts across this boundary.  otm_last_error() gives a
 *             per-context message for the most recent failure.
 *  Threads  : a context must not be used from two threads at once.
 */
#ifndef OPENTM_AMD_H
#define OPENTM_AMD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define OTM_OK 0
#define OTM_NOT_CONVERGED 1 /* warning: outputs are filled; stats say how far the solve got */
#define OTM_EINVAL (-1)     /* invalid argument (null pointer, size mismatch, bad parameter) */
#define OTM_ENOMEM (-2)     /* device or host allocation failed */
#define OTM_EDEVICE (-3)    /* a HIP runtime call failed, or no usable gfx950 device */
#define OTM_ENONFINITE (-4) /* NaN or Inf in an input or a result */
#define OTM_EUNSUPPORTED (-5)
#define OTM_ESTATE (-6) /* call order violated (e.g. sensitivity before homogenize) */
#define OTM_EIO (-7)    /* a file could not be opened, read or written, or is malformed */

/* ---- enumerations -------------------------------------------------------- */
#define OTM_FP64 0  /* every vector and the operator in float64 */
#define OTM_MIXED 1 /* float32 operator and Krylov vectors; float64 solution, dots,
                       residual recomputation and tensor assembly */

/* Warm starts (PREVIOUS, USER, LEARNED) are scaled per load by
 * s = b.x / x.A x, the factor minimising the quadratic energy along the guess,
 * so the start is never farther from the solution in the energy norm than
 * chi = 0; a load with b.x <= 0 starts from zero. */
#define OTM_GUESS_ZERO 0     /* PCG starts from chi = 0 */
#define OTM_GUESS_PREVIOUS 1 /* PCG starts from the previous design iteration's chi */
#define OTM_GUESS_USER 2     /* PCG starts from the field set by otm_set_guess */
#define OTM_GUESS_LEARNED 3  /* PCG starts from the attached network's prediction
                                (otm_set_network; n a multiple of 16, else zero) */

/* Preconditioners of the conjugate-gradient solve. */
#define OTM_PRECOND_JACOBI 0 /* diagonal (Jacobi) preconditioner, Sec. 2.4 relaxation diagonal S_v */
#define OTM_PRECOND_MG 1     /* one geometric multigrid V-cycle per iteration (Sec. 2.4, Algorithm 3):
                                relaxation on S_v (damped Jacobi or 8-colour Gauss-Seidel,
                                mg_smoother), restriction of the residual,
                                direct solve on the coarsest level, interpolation and correction.
                                The V-cycle runs in float32; with OTM_FP64 the Krylov vectors,
                                dots and convergence test stay float64.  n = m 2^j with
                                m in {3, 4} and n >= 6, else OTM_EINVAL */

/* Relaxation of the multigrid V-cycle (OTM_PRECOND_MG). */
#define OTM_MG_JACOBI 0 /* damped Jacobi, weight 0.9 (default) */
#define OTM_MG_GS8 1    /* 8-colour Gauss-Seidel (Sec. 2.4): S_v T_v = f_v - M_v for the nodes of
                           one parity class (i mod 2, j mod 2, k mod 2) at a time, colours 0..7
                           before the coarse correction and 7..0 after it (a symmetric cycle);
                           mg_sweeps / mg_coarse_sweeps count full sweeps of 8 colours */

#define OTM_OBJ_MSE 0 /* g = sum_c (kappa_c - target_c)^2, Sec. 4.4 (MSE objective) */
#define OTM_OBJ_REL 1 /* g = sum_c (kappa_c / target_c - 1)^2, Sec. 4.4 (relative objective);
                         every target component must be nonzero, else OTM_EINVAL */
#define OTM_OBJ_L1 2  /* g = sum_c |kappa_c - target_c|, Sec. 4.4 (l1 objective), with the
                         derivative of |a| taken as 0 at a = 0 */

/* Initial density fields (Sec. 4.3, density initialization), otm_init_density. */
#define OTM_INIT_P 0    /* Schwarz P:  cos X + cos Y + cos Z */
#define OTM_INIT_D 1    /* Schwarz D:  cos X cos Y cos Z - sin X sin Y sin Z */
#define OTM_INIT_G 2    /* gyroid:     sin X cos Y + sin Y cos Z + sin Z cos X */
#define OTM_INIT_IWP 3  /* Schoen IWP: 2 (cos X cos Y + cos Y cos Z + cos Z cos X)
                                       - (cos 2X + cos 2Y + cos 2Z) */
#define OTM_INIT_BALL 4 /* centre ball: a solid cube with a spherical void at its centre */

/* Symmetry constraints on the design (Sec. 4.3, customized microstructures). */
#define OTM_SYM_NONE 0
#define OTM_SYM_CENTRAL 1 /* central symmetry: element (i,j,k) and its image (n-1-i, n-1-j, n-1-k)
                             (flat indices e and n^3-1-e) both take the mean of their densities
                             at the start of every evaluation and the mean of their
                             sensitivities after it */

/* Fields readable with otm_get_field (count = n^3, or 3 n^3 where noted). */
#define OTM_FIELD_RHO 0      /* design density rho (current) */
#define OTM_FIELD_RHOF 1     /* filtered density rho~ */
#define OTM_FIELD_K 2        /* element conductivity k_e */
#define OTM_FIELD_B 3        /* macro loads b^i, 3 n^3, projected to zero mean */
#define OTM_FIELD_DIAG 4     /* Jacobi diagonal d_v = (1/3) sum of the 8 incident k_e */
#define OTM_FIELD_CHI 5      /* fluctuation fields chi^i, 3 n^3, zero mean */
#define OTM_FIELD_SENS_ELEM 6 /* dg/drho~_e before the filter transpose */
#define OTM_FIELD_SENS 7     /* dg/drho_e after the filter transpose */

/* ---- initial densities ---------------------------------------------------- */
/* Writes an n^3 density field (host, float64, flat x-fastest) for the
 * initialization `kind` (OTM_INIT_*): the level set is evaluated at element
 * centres, X = 2 pi (i + 1/2) / n (Y, Z likewise; one period per cell), and
 * exactly round(vf n^3) elements with the smallest values are solid (1), the
 * rest void (0), ties broken by flat index.  For OTM_INIT_BALL the value is
 * minus the distance from the cell centre, so the solid is the cube minus a
 * central ball.  Host-only; needs no device and no context.
 * Errors: OTM_EINVAL (null pointer, n outside 4..1024, vf outside (0, 1],
 * unknown kind). */
int otm_init_density(int32_t n, int32_t kind, double vf, double* rho_out);

/* ---- parameter blocks ---------------------------------------------------- */
typedef struct {
    int32_t n;            /* elements per axis (cubic periodic cell), 4..1024 */
    double k0;            /* solid conductivity, > kmin */
    double kmin;          /* void conductivity, > 0 */
    double penal;         /* SIMP exponent p >= 1 */
    double filter_radius; /* hat-filter radius in voxels; < 1 disables the filter */
    double target[6];     /* target tensor, [11,22,33,12,23,13] */
    double vf;            /* initial volume bound V*_0 in (0, 1] */
    int32_t objective;    /* OTM_OBJ_MSE, OTM_OBJ_REL or OTM_OBJ_L1 */
    int32_t symmetry;     /* OTM_SYM_NONE or OTM_SYM_CENTRAL (single contexts only; a batch
                             returns OTM_EUNSUPPORTED for OTM_SYM_CENTRAL) */
} otm_problem;

typedef struct {
    int32_t precision;   /* OTM_FP64 or OTM_MIXED */
    int32_t guess;       /* OTM_GUESS_* */
    double tol;          /* stop when ||b - A chi||_2 <= tol ||b||_2 for every load */
    int32_t max_iter;    /* PCG iteration cap per solve */
    int32_t check_every; /* host convergence check interval (iterations), >= 1; with
                            OTM_PRECOND_MG at most 2 is used */
    double reliable_delta; /* OTM_MIXED: refresh the float64 residual when the float32
                              recursive residual has dropped by this factor (default
                              1e-2; 1e-3 suits OTM_PRECOND_MG, whose iterations each cut
                              the residual several-fold) */
    int32_t kernel_variant; /* 0: streaming z-march kernels (default; two nodes per
                               thread when n is even; with autotune on and automatic
                               tiles the fused iteration of 4 is chosen when it is
                               faster); 1: direct-gather kernels; 2: LDS-ring tiled
                               kernels; 3: z-march with one node per thread (same
                               arithmetic, kept as cross-checks); 4: fused PCG
                               iteration, one z-march pass and one reduction per
                               iteration (even n only, else OTM_EINVAL); 5: as 4,
                               with the passes of a check interval chained (each
                               block reduces its predecessor's sums itself; same
                               sums in the same order, so the iterates equal 4's).
                               All give Jacobi-PCG iterates that agree in exact
                               arithmetic. */
    int32_t tile_tz;        /* planes per z-march of the operator kernel; 0 = automatic */
    int32_t tile_tx;        /* tile width in x in nodes: 16, 32 or 64 (32 or 64 for the
                               two-node kernel); 0 = automatic */
    int32_t autotune;       /* 1: with kernel_variant 0 and automatic tiles, time the
                               candidate kernels and tile shapes once per (n, precision)
                               and process at otm_create and keep the fastest (a
                               candidate must be 2 % faster to displace an earlier one).
                               When the environment variable OTM_TUNE_CACHE names a
                               file, a choice stored there for this device architecture
                               and (n, precision) is used without timing, and a new
                               choice is appended to it (text, one line per choice:
                               architecture, key, values; the last line wins; lines a
                               context could not have chosen are ignored).  Batches do
                               the same per mix of n. */
    int32_t preconditioner; /* OTM_PRECOND_JACOBI (default) or OTM_PRECOND_MG; with
                               OTM_PRECOND_MG kernel_variant must be 0 and no autotuning
                               is done */
    int32_t mg_sweeps;      /* OTM_PRECOND_MG: relaxation steps before and after each
                               coarse correction on the finest level, 1..8 (default 1) */
    int32_t mg_coarse_sweeps; /* the same on the coarser levels, 0..8; 0 = mg_sweeps
                                 (default 2) */
    int32_t stall_window;   /* stagnation: a solve stops when no active load's best
                               recursive residual norm has halved within this many
                               of its iterations (or a residual is not finite);
                               0 = automatic, 200 + 10 n.  A stalled OTM_MIXED solve
                               continues in float64 (two-pass Jacobi-PCG) from its
                               solution, or from zero after a non-finite residual;
                               a stalled float64 solve returns OTM_NOT_CONVERGED */
    int32_t mg_smoother;    /* OTM_PRECOND_MG: OTM_MG_JACOBI (default) or OTM_MG_GS8 */
} otm_solver_opts;

typedef struct {
    double move;    /* OC move limit m */
    double eta;     /* OC damping exponent */
    double rho_min; /* lower density bound */
    double move_min; /* 0 (default): every design iteration (otm_step, otm_batch_step)
                        moves by at most `move`.  In (0, move]: the limit adapts
                        per design: halved after a design iteration whose objective
                        rose, grown by a tenth after one whose objective fell, kept
                        in [move_min, move].  otm_oc_update and
                        otm_oc_update_noalloc always use `move`. */
} otm_oc_opts;

/* Adaptive volume bound (Sec. 2.3, model 3; Algorithm 1).  Each design
 * iteration: an objective g <= bound shrinks V* by the fraction Df of the gap
 * to mean(rho~^p), and Df <- decay Df; otherwise an iteration with
 * |dg| < dg_small and |mean(rho) - V*| < dv_small is a stall, and the
 * patience-th consecutive stall raises V* by rebound * gap * Df.  V* stays in
 * [rho_min, 1].  Thresholds finite and >= 0, decay in [0, 1], patience and
 * stall_iters >= 1, else otm_create returns OTM_EINVAL. */
typedef struct {
    double bound;     /* objective considered small enough to shrink V* */
    double dg_small;  /* |g_prev - g| below this counts as little progress */
    double dv_small;  /* |V - V*| below this counts as sitting on the bound */
    double decay;     /* Df <- decay * Df after each reduction */
    double rebound;   /* V* <- V* + rebound * gap * Df after `patience` stalls */
    double g_tol;     /* termination: |g_prev - g| below this ... */
    int32_t patience;
    int32_t stall_iters; /* ... for this many consecutive iterations */
} otm_governor_opts;

typedef struct {
    int32_t iterations[3];  /* PCG iterations per load (float32 iterations in OTM_MIXED) */
    double rel_residual[3]; /* true ||b - A chi|| / ||b|| per load, float64 */
    int32_t converged;      /* 1 when every load met tol */
    int32_t refreshes;      /* OTM_MIXED: float64 residual refreshes */
    double ms_solve;        /* wall time of the three solves, milliseconds */
    int32_t stalled;        /* 0; 1 the (last) solve stagnated, 2 its residual was not finite */
    int32_t fallback;       /* 1 when a mixed-precision solve finished in float64 */
} otm_solve_stats;

typedef struct {
    int32_t iter;
    double g;
    double kappa[6];
    double volume;    /* mean(rho) before the update */
    double low_bound; /* mean(rho~^p) */
    double vstar;     /* V* used by this iteration's OC update */
    double lambda;    /* OC multiplier */
    int32_t pcg_iters[3];
    double rel_residual[3];
    double ms_total;
    double ms_solve;
    int32_t stop; /* 1 when the stall test of the governor fired */
    double move;  /* OC move limit this iteration's update used */
    int32_t stalled; /* the solve of this iteration: 0; 1 it stagnated (no 4x residual drop
                        within stall_window iterations), 2 its residual was not finite */
} otm_iter_record;

typedef struct otm_ctx otm_ctx;

/* Fill the three option blocks with the defaults: FP64, zero guess, tol 1e-8,
 * move 0.05, eta 0.5, rho_min 1e-3 (Sec. 4 parameters), governor bound 1e-4,
 * decay 0.8, rebound 0.3, patience 5 (Algorithm 1).  Any pointer may be NULL. */
void otm_default_options(otm_solver_opts* solver, otm_oc_opts* oc, otm_governor_opts* gov);

/* Create a context on the current HIP device.  `stream` is a hipStream_t or
 * NULL (the context then creates its own stream).  Options may be NULL for
 * defaults.  All device buffers for n^3 are allocated here.
 * Errors: OTM_EINVAL (bad parameters), OTM_EDEVICE (no gfx950 device),
 * OTM_ENOMEM.  On error *out is NULL. */
int otm_create(const otm_problem* problem, const otm_solver_opts* solver, const otm_oc_opts* oc,
               const otm_governor_opts* gov, void* stream, otm_ctx** out);
void otm_destroy(otm_ctx* ctx);

/* Design density: `count` must be n^3; values must be finite and are clamped
 * to [rho_min, 1] on entry (the return value is OTM_OK either way).
 * The _device variant reads a float64 device buffer of n^3 values. */
int otm_set_density(otm_ctx* ctx, const double* rho_host, int64_t count);
int otm_set_density_device(otm_ctx* ctx, const void* rho_device, int64_t count);

/* Filter, SIMP, macro loads, three PCG solves and the tensor (Sec. 2.2, 2.4).
 * kappa6 (host, 6 doubles) receives kappa^H; stats may be NULL.
 * Returns OTM_NOT_CONVERGED if a solve hit max_iter (kappa still filled). */
int otm_homogenize(otm_ctx* ctx, double kappa6[6], otm_solve_stats* stats);

/* Sensitivities for a given dg/dkappa (6 doubles, host), from the state of the
 * last otm_homogenize (Sec. 2.3).  dg_drho_host (n^3, may be NULL) receives
 * dg/drho after the filter transpose.  OTM_ESTATE without a prior homogenize. */
int otm_sensitivity(otm_ctx* ctx, const double dg_dkappa6[6], double* dg_drho_host);

/* Optimality Criteria update with volume bound `vstar` from the last
 * sensitivities: bisection on the multiplier (bracket [0, 1e9], relative width
 * 1e-13, at most 200 halvings).  rho_out_host (n^3) and lambda_out may be NULL.
 * The context's density is replaced by the update. */
int otm_oc_update(otm_ctx* ctx, double vstar, double* rho_out_host, double* lambda_out);

/* Optimality Criteria update that allocates nothing, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It computes what otm_oc_update computes
 * from caller device buffers, with no context:
 *   rho_dev   n^3 float64 design densities (device; expected in [rho_min, 1])
 *   sens_dev  n^3 float64 dg/drho (device)
 *   vstar     volume bound, 0 < vstar <= 1
 *   oc        move, eta, rho_min as for otm_create (host struct, read in-call)
 *   rho_out_dev  n^3 float64 updated densities (device); may be rho_dev itself
 *   lambda_dev   one float64 (device) receiving the multiplier; may be NULL
 *   stream    hipStream_t or NULL
 * The bisection's scratch (partial sums and device scalars, 132 KiB, the
 * same for every n) is a static device array that each GPU holds until the
 * process ends; q_e is recomputed from (rho_e, s_e), so no n^3 buffer is used.
 * The call only enqueues kernels on `stream` (no synchronisation, no host
 * read-back: every possible bisection pass is launched and those after the
 * stop return at once) and returns.  Calls on one GPU share the scratch:
 * calls that overlap on one GPU (other streams or threads) race, so the
 * caller serialises them.  With the same inputs and options it gives the
 * same rho and lambda as otm_oc_update.
 * Errors: OTM_EINVAL (null rho/sens/rho_out/oc, n outside 4..1024, vstar
 * outside (0, 1], invalid oc options, rho_out or lambda aliasing sens,
 * lambda aliasing a field), OTM_EDEVICE (no device, the scratch address
 * lookup or a launch failed), OTM_EUNSUPPORTED (device index >= 64). */
int otm_oc_update_noalloc(int32_t n, const void* rho_dev, const void* sens_dev, double vstar,
                          const otm_oc_opts* oc, void* rho_out_dev, void* lambda_dev, void* stream);

/* One full design iteration (Algorithm 2 body with the Algorithm 1 governor):
 * homogenize -> objective -> sensitivities -> V* update -> OC update. */
int otm_step(otm_ctx* ctx, otm_iter_record* rec);

/* Up to max_iter design iterations; stops early when the governor's stall test
 * fires.  log (may be NULL) receives up to log_cap records; rho_out_host (n^3,
 * may be NULL) the final density; iters_done (may be NULL) the count run. */
int otm_optimize(otm_ctx* ctx, int32_t max_iter, double* rho_out_host, otm_iter_record* log,
                 int32_t log_cap, int32_t* iters_done);

/* Copy a field (OTM_FIELD_*) to the host; count must equal its size. */
int otm_get_field(otm_ctx* ctx, int32_t field, double* host_out, int64_t count);

/* Overwrite a field from the host, for step-by-step use from externally
 * computed inputs: OTM_FIELD_RHO (n^3; same as otm_set_density),
 * OTM_FIELD_CHI (3 n^3; needs a prior otm_prepare or otm_homogenize of the
 * same density; the next otm_sensitivity uses it) or OTM_FIELD_SENS (n^3; the
 * next otm_oc_update uses it).  Other fields: OTM_EINVAL. */
int otm_set_field(otm_ctx* ctx, int32_t field, const double* host_in, int64_t count);

/* Initial guess for OTM_GUESS_USER: 3 n^3 float64 values (voxel units). */
int otm_set_guess(otm_ctx* ctx, const double* chi_host, int64_t count);

/* Adaptive volume bound (Algorithm 1) as 8 doubles: [V*, decrease factor Df,
 * consecutive stalls (the algorithm's count), gap, previous objective,
 * consecutive iterations with |dg| < g_tol, design iterations done, OC move
 * limit of the last design iteration (0 before the first)].
 * set restores a state returned by get (checkpoint/resume). */
int otm_get_governor(const otm_ctx* ctx, double state8[8]);
int otm_set_governor(otm_ctx* ctx, const double state8[8]);

/* Checkpoint / resume of a design run (the optimization loop of Sec. 3.4
 * interrupted between design iterations): the design density rho, the last
 * solution chi (the warm start of OTM_GUESS_PREVIOUS; present once a solve
 * has run) and the adaptive volume bound's state (Algorithm 1, as
 * otm_get_governor) go to one binary file that this library writes and reads:
 *   "OTMSTATE" | u32 version 2 | i32 n | u32 flags (bit 0: chi present) |
 *   u32 0 | f64[11] k0, kmin, penal, filter radius, target[6], objective |
 *   f64[8] governor state | f64 the objective's last change (memory of the
 *   adaptive OC step) | f64 rho[n^3] | f64 chi[3 n^3] if bit 0 |
 *   u64 FNV-1a hash of every preceding byte; little-endian.  Version 1 files
 *   (no last change; read as 0) load as well.
 * save writes path.tmp and renames it over path.  load restores all three
 * into a context created for the same n and problem constants, after which
 * otm_step continues the interrupted run exactly (same iterates, bit for bit).
 * Errors: OTM_EINVAL (null or empty path, another n or problem),
 * OTM_ESTATE (save without a density), OTM_EIO (open/read/write failure,
 * wrong magic, version, size or checksum), OTM_ENONFINITE, OTM_EDEVICE. */
int otm_save_state(otm_ctx* ctx, const char* path);
int otm_load_state(otm_ctx* ctx, const char* path);

/* Matrix-free operator y^i = A x^i for the three loads with the context's
 * current k (needs a prior otm_homogenize or otm_prepare), in the given
 * precision (OTM_FP64 or OTM_MIXED = float32 operator).  x and y are host
 * arrays of 3 n^3 float64 values.  This is [KT]_v of Sec. 2.4. */
int otm_apply(otm_ctx* ctx, int32_t precision, const double* x_host, double* y_host);

/* Filter + SIMP + macro loads + diagonal only (first half of otm_homogenize). */
int otm_prepare(otm_ctx* ctx);

/* Stateless operator on caller device memory: y^i = A x^i for the three loads
 * of an n^3 cell ([KT]_v of Sec. 2.4).  k_dev: n^3 element conductivities;
 * x_dev, y_dev: 3 n^3 node values, load-major, not aliased.  precision
 * OTM_FP64 -> all pointers are double*; OTM_MIXED -> all are float*.
 * variant: 0 = streaming z-march (two nodes per thread for even n),
 * 1 = direct gather, 2 = LDS-ring tiled, 3 = z-march, one node per thread.
 * stream: hipStream_t or NULL.  Asynchronous on `stream`. */
int otm_apply_device(int32_t n, int32_t precision, int32_t variant, const void* k_dev, const void* x_dev,
                     void* y_dev, void* stream);

/* As otm_apply_device with an explicit tile (tile_tx, tile_tz as for
 * otm_time_apply_device; 0 = automatic): one launch on `stream`, no
 * synchronisation.  Errors as otm_apply_device. */
int otm_apply_device_tiled(int32_t n, int32_t precision, int32_t variant, int32_t tile_tx, int32_t tile_tz,
                           const void* k_dev, const void* x_dev, void* y_dev, void* stream);

/* Timing of the stateless operator: runs `reps` launches of the operator on
 * `stream` and returns the mean kernel duration in microseconds, measured
 * with HIP events on that stream.  tile_tx / tile_tz: tile shape of the
 * z-march and ring kernels (0 = automatic). */
int otm_time_apply_device(int32_t n, int32_t precision, int32_t variant, int32_t tile_tx, int32_t tile_tz,
                          const void* k_dev, const void* x_dev, void* y_dev, void* stream, int32_t reps,
                          double* us_per_launch);

/* Operator kernel in use: [variant (0 pair z-march, 1 gather, 2 ring, 3 z-march,
 * 4 fused PCG iteration, 5 fused with chained passes), tile width, planes per
 * march, blocks per launch]. */
int otm_get_tile(const otm_ctx* ctx, int32_t tile4[4]);

/* Live timing of the solver's dominant kernel (the fused pass, or the
 * direction+operator pass of the two-pass iteration with the two-node
 * z-march), accumulated over the solves since the last reset: one launch per
 * host check interval is timed with HIP events that the launch itself records
 * at the kernel's start and end on the context stream (hipExtLaunchKernelGGL),
 * when every load takes a full step.  out4 = [sampled launches, mean
 * microseconds per launch, algorithmic bytes per launch, kernel (4 fused,
 * 0 direction+operator)].  reset != 0 clears the accumulators after reading.
 * Other kernel variants are not sampled (count 0). */
int otm_pass_timing(otm_ctx* ctx, int32_t reset, double out4[4]);

/* Per-phase timings of the last otm_step, milliseconds, HIP events on the
 * context stream: [filter+setup, solve, tensor, sensitivity, oc, total,
 * 1 if the last solve started from the network's prediction, PCG
 * iterations launched in the last solve]. */
int otm_get_timings(const otm_ctx* ctx, double t8[8]);

/* Device memory the context holds (every buffer it allocated, the multigrid
 * levels included; not the caller's tensors or a network), in bytes.  It is
 * fixed at creation (otm_apply's temporaries, freed before it returns, are
 * not counted). */
int otm_device_bytes(const otm_ctx* ctx, int64_t* bytes);

/* ---- batches of designs (uneven n) -----------------------------------------
 * Many independent cells in one set of device arenas; every phase of a design
 * iteration is one launch over all designs (per-design scalars and
 * reductions), and a chunk of PCG iterations is captured once as a hipGraph
 * and replayed until every design has converged.  Every n must be even
 * (4..1024).  Problems may differ in n, target, vf and material constants;
 * solver / OC / governor options are shared.  Precision OTM_FP64, or
 * OTM_MIXED (float32 operator and Krylov vectors, float64 solution, dots and
 * residual refreshes, as for contexts; fused iteration only, kernel_variant 0
 * or 4); Jacobi preconditioner only (else OTM_EUNSUPPORTED).  A batch's
 * solve skips the work of designs whose three loads have stopped.  autotune
 * (solver options) times whole PCG iterations of the fused single-pass
 * iteration and of the two-pass iteration over tile widths and march lengths
 * at creation and keeps the fastest (kernel_variant 4 or OTM_MIXED: the fused
 * iteration only; other variants, or autotune off with kernel_variant 0: the
 * two-pass iteration).  The fused iteration needs at most 4096 (design, tile)
 * work items (OTM_MIXED without such a tile: OTM_EUNSUPPORTED).  Errors as
 * for contexts; otm_batch_last_error gives details. */
typedef struct otm_batch otm_batch;
int otm_batch_create(const otm_problem* problems, int32_t count, const otm_solver_opts* solver,
                     const otm_oc_opts* oc, const otm_governor_opts* gov, void* stream, otm_batch** out);
void otm_batch_destroy(otm_batch* batch);
/* design index d in [0, count); count = n_d^3 host values */
int otm_batch_set_density(otm_batch* batch, int32_t d, const double* rho_host, int64_t count);
/* OTM_FIELD_RHO, _RHOF, _K, _CHI (3 n_d^3), _SENS, _SENS_ELEM of design d */
int otm_batch_get_field(otm_batch* batch, int32_t d, int32_t field, double* host_out, int64_t count);
/* One design iteration for every design; recs (may be NULL) receives count
 * records.  A design whose solve stagnates (the stall_window rule of a
 * context's solve) stops there, its record says so (stalled), and the others
 * go on.  OTM_NOT_CONVERGED if some solve hit max_iter or stalled. */
int otm_batch_step(otm_batch* batch, otm_iter_record* recs);
/* 1 (default): replay the captured PCG chunk; 0: launch it eagerly. */
int otm_batch_set_graph(otm_batch* batch, int32_t use_graph);
/* [designs, total cells, operator work items, tile width, march length of
 *  design 0, tuned PCG iteration us, last solve ms, last step ms, 1 if the
 *  fused single-pass iteration is in use (else 0), float64 residual
 *  refreshes of the last solve (OTM_MIXED; else 0)] */
int otm_batch_info(const otm_batch* batch, double info10[10]);
/* Adaptive volume bound state of design d (Algorithm 1), the 8 doubles of
 * otm_get_governor; the iteration count is the batch's. */
int otm_batch_get_governor(const otm_batch* batch, int32_t d, double state8[8]);
/* Checkpoint / resume of a batch run: every design's density, its previous
 * solution (when a step has run) and its adaptive volume bound state
 * (Algorithm 1, with the adaptive OC step's memory), plus the batch's
 * iteration count, in one binary file that this library writes and reads:
 *   "OTMBATCH" | u32 version 1 | i32 count | u32 flags (bit 0: solutions) |
 *   i32 iterations done | per design: i32 n | u32 0 | f64[11] k0, kmin,
 *   penal, filter radius, target[6], objective | f64[8] V*, Df, stalls, gap,
 *   previous objective, flat count, OC step, last objective change |
 *   f64 rho of every design in order | f64 chi (3 n^3 each) if bit 0 |
 *   u64 FNV-1a hash of every preceding byte; little-endian.
 * save writes path.tmp and renames it over path.  load restores the state
 * into a batch created for the same designs (count, n and problem constants
 * in the same order), after which otm_batch_step continues the interrupted
 * run exactly.  Errors: OTM_EINVAL (null or empty path, other designs),
 * OTM_ESTATE (save before every design has a density), OTM_EIO (open, read
 * or write failure; wrong magic, version, size or checksum),
 * OTM_ENONFINITE, OTM_EDEVICE. */
int otm_batch_save_state(otm_batch* batch, const char* path);
int otm_batch_load_state(otm_batch* batch, const char* path);
/* Device memory the batch holds (its arenas, tables and graph buffers), bytes. */
int otm_batch_device_bytes(const otm_batch* batch, int64_t* bytes);
const char* otm_batch_last_error(const otm_batch* batch);

/* ---- learned warm start ------------------------------------------------------
 * A fully convolutional network (5 periodic 3x3x3 layers, channels
 * 1-16-16-16-16-3, ReLU after the first four, output mean removed) maps the
 * filtered density to the three fluctuation fields.  Convolutions run as bf16
 * MFMA implicit GEMMs with float32 accumulation; parameters are float32 with
 * Adam.  Grids must have n a multiple of 16, 16 <= n <= n_max.
 * Parameter layout (compact, float32): for each layer, W[cout][cin][27] with
 * tap 9(dz+1)+3(dy+1)+(dx+1) of the correlation y[v] = b + sum W x[v+d], then
 * b[cout]. */
typedef struct otm_nn otm_nn;
int otm_nn_create(int32_t n_max, uint64_t seed, void* stream, otm_nn** out);
void otm_nn_destroy(otm_nn* net);
int32_t otm_nn_param_count(void);
int otm_nn_get_params(otm_nn* net, float* host, int64_t count);
int otm_nn_set_params(otm_nn* net, const float* host, int64_t count);
/* accumulated gradients, same layout */
int otm_nn_get_grads(otm_nn* net, float* host, int64_t count);
/* device pointers: rhof n^3 float64 -> chi0 3 n^3 float64 (mean removed) */
int otm_nn_forward(otm_nn* net, int32_t n, const void* rhof_dev, void* chi0_dev);
/* forward + backward of the mean-squared error against chi (3 n^3 float64,
 * device; mean removed inside), gradients added to the accumulator; loss_out
 * (host, may be NULL) receives the loss. */
int otm_nn_accumulate(otm_nn* net, int32_t n, const void* rhof_dev, const void* chi_dev, double* loss_out);
/* Adam step with the accumulated gradients divided by batch; clears them. */
int otm_nn_adam(otm_nn* net, double lr, int32_t batch);
int otm_nn_zero_grads(otm_nn* net);
const char* otm_nn_last_error(const otm_nn* net);
/* Network weights as a file: the compact parameter vector (layout above) as
 * a NumPy .npy array, dtype '<f4', shape (otm_nn_param_count(),), C order
 * (format 1.0 written; 1.0-3.0 read).  load replaces the parameters and
 * resets Adam's step count.  Errors: OTM_EINVAL (null or empty path),
 * OTM_EIO (open/read/write failure, not .npy, another dtype, order, shape or
 * size), OTM_ENONFINITE (a non-finite weight), OTM_EDEVICE. */
int otm_nn_save(otm_nn* net, const char* path);
int otm_nn_load(otm_nn* net, const char* path);
/* Attach a network to a context for OTM_GUESS_LEARNED (NULL detaches).  The
 * context does not own it. */
int otm_set_network(otm_ctx* ctx, otm_nn* net);

const char* otm_strerror(int status);
const char* otm_last_error(const otm_ctx* ctx);
/* Library version string. */
const char* otm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* OPENTM_AMD_H */
