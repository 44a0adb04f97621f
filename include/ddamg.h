/*
 * ddamg.h -- C-ABI of the MI355X DD-alpha-AMG solver for the clover-improved
 * Wilson Dirac system D z = b on a periodic 4D lattice.
 *
 * Method: Frommer, Kahl, Krieg, Leder, Rottmann, "Adaptive aggregation based
 * domain decomposition multigrid for the lattice Wilson Dirac operator"
 * (arXiv:1303.1377).  The problem statement is eq. (discreteDirac) with D of
 * eq. (lattice_WD) in the explicit site form of Sec. 2.2; the solver is FGMRES
 * right-preconditioned by the V-cycle C^(nu) of Sec. 4.2 (eq. iterationmatrix)
 * whose smoother is red-black SAP (Sec. 2.3) and whose coarse operator is
 * D_c = P^H D P for the standard aggregation (Sec. 3.2); the hierarchy is built
 * by the setup of Algorithm 2.  Default parameters are those of Table 1.
 *
 * Conventions shared by every entry point
 *   - All array pointers are DEVICE pointers (HIP, e.g. torch tensors'
 *     data_ptr()) unless stated otherwise.  Complex numbers are interleaved
 *     (re, im) doubles (complex128).
 *   - Lattice dims are {N0, N1, N2, N3}; x0 is time.  Canonical site index
 *     ((x0*N1 + x1)*N2 + x2)*N3 + x3.  Boundary conditions are periodic.
 *   - Fine spinor: [site][spin 0..3][colour 0..2] (colour fastest, Sec. 2.1).
 *   - Gauge field: [site][mu 0..3][row][col], U_mu(x) on the link x -> x+mu.
 *   - Coarse vectors of level l >= 1: [coarse site][2N] with index h*N + k,
 *     h = 0 for the aggregate of spins {0,1} (Gamma5^c = +1), h = 1 for spins
 *     {2,3}; coarse sites in canonical order of the coarse lattice.
 *   - The caller keeps ownership of every pointer it passes; the context copies
 *     what it needs.  A context is bound to the HIP stream given at creation and
 *     is not thread-safe; distinct contexts are independent.
 *   - Calls are synchronous with respect to the host: they return after the
 *     work they enqueued on the context's stream has completed.
 *   - On error the call returns a negative dd_status and dd_last_error() holds
 *     a message; the context stays usable unless the status is DD_EDEVICE.
 */
#ifndef DDAMG_H
#define DDAMG_H

#ifdef __cplusplus
extern "C" {
#endif

#define DD_MAXLEV 4

typedef struct dd_ctx dd_ctx;

typedef enum {
    DD_OK = 0,
    DD_EINVAL = -1,    /* invalid argument (dims, blocks, sizes, NULL pointer)      */
    DD_ENOMEM = -2,    /* device allocation failed                                  */
    DD_ENOCONV = -3,   /* iteration limit reached; x holds the last iterate         */
    DD_EDEVICE = -4,   /* HIP runtime error                                         */
    DD_ESTATE = -5,    /* call out of order (e.g. solve before setup)               */
    DD_ENUMERIC = -6   /* NaN/Inf, singular block, rank-deficient aggregate         */
} dd_status;

/* Solver parameters (defaults: Table 1 of the paper; see dd_default_params). */
typedef struct {
    int levels;                  /* number of levels, 2 .. DD_MAXLEV                       */
    int n_tv[DD_MAXLEV];         /* test vectors N of the transfer level l -> l+1          */
    int agg[DD_MAXLEV][4];       /* aggregate lattice-block dims on level l (Def. standard
                                    aggregation, Sec. 3.2)                                 */
    int sap[DD_MAXLEV][4];       /* SAP lattice-block dims on level l (Sec. 2.3)           */
    int mr_steps[DD_MAXLEV];     /* MR steps of the SAP block solver on level l (Sec. 5)   */
    int nu;                      /* SAP post-smoothing iterations per V-cycle              */
    int n_inv;                   /* setup iterations of Algorithm 2                        */
    double coarse_tol;           /* coarsest-level relative residual (5e-2)                */
    int coarse_restart;          /* restart length of the coarsest GMRES (30)              */
    int coarse_maxit;            /* iteration cap of one coarsest solve                    */
    int coarse_fixed;            /* >0: run exactly this many coarsest iterations          */
    double mid_tol;              /* intermediate-level FGMRES relative residual (3+ levels)*/
    int mid_restart;
    int mid_maxit;
    int mid_fixed;               /* >0: exactly this many intermediate iterations          */
    int outer_restart;           /* FGMRES restart length n_kv                             */
    int outer_maxit;             /* outer iteration cap                                    */
    int precision;               /* 64: FP64 preconditioner; 32: FP32 preconditioner;
                                    16: FP32 arithmetic on FP16-stored operators (links,
                                    clover blocks, P, D_c, self-block inverses; vectors
                                    FP32).  The outer FGMRES and its D are always FP64.  */
    int given_vectors;           /* 1: the setup starts from vectors installed with
                                    dd_set_test_vectors instead of drawing them            */
    unsigned long long seed;     /* counter-based RNG key for the initial test vectors     */
    int max_rhs;                 /* right-hand sides one dd_solve_batch call can carry in
                                    one batch (1..16); sizes the Krylov workspace          */
    int id_setup;                /* 1: the setup of inexact deflation (Sec. 4.3): in the
                                    n_inv rounds v_j <- C^(nu) v_j (V-cycle from a zero
                                    start) replaces v_j <- v_j + C^(nu)(v_j - D v_j)       */
} dd_params;

typedef struct {
    int outer_iters;             /* FGMRES iterations (sum over restarts)                  */
    int restarts;
    long coarse_iters[DD_MAXLEV];/* summed iterations of the level-l solver               */
    double true_relres;          /* ||b - D x|| / ||b|| in FP64 at exit                    */
    double setup_s, solve_s;     /* wall time of the last dd_setup / dd_solve              */
    int converged;
} dd_stats;

/* Fill *p with the Table 1 defaults (2 levels, N = 20, 4^4 aggregates and SAP
 * blocks, 4 MR steps, nu = 2, n_inv = 6, coarse GMRES(30) to 5e-2,
 * FGMRES(25), FP64). */
void dd_default_params(dd_params *p);

/* Create a solver context for D(U, m0, csw) (Sec. 2.2).
 *   dims     lattice extents, each even and >= 2
 *   gauge    device, complex128 [vol][4][3][3]; SU(3) links
 *   clover   device, complex128 [vol][2][6][6] or NULL.  If given: the two
 *            chiral 6x6 blocks of the clover term T(x) (without (m0+4)),
 *            spins {0,1} then {2,3}, index spin*3 + colour within a block.
 *            If NULL the term is computed on the device from the four-leaf
 *            Q_{mu nu} of eq. (lattice_WD).
 *   m0, csw  mass and Sheikholeslami-Wohlert coefficient
 *   hip_stream  hipStream_t the context enqueues on (NULL: default stream)
 * Errors: DD_EINVAL (dims, NULL gauge), DD_ENOMEM, DD_ENUMERIC (singular
 * clover block), DD_EDEVICE. */
dd_status dd_create(dd_ctx **out, const int dims[4], const double *gauge, const double *clover,
                    double m0, double csw, void *hip_stream);

/* Release every device buffer of the context.  NULL is ignored. */
void dd_destroy(dd_ctx *ctx);

/* Message of the last failing call on ctx (owned by ctx, valid until the next
 * call).  With ctx == NULL: the last dd_create failure. */
const char *dd_last_error(const dd_ctx *ctx);

/* Adaptive setup, Algorithm 2 (DD-alpha-AMG-setup(n_inv, nu)) level by level.
 *   n_tv, block, levels  override n_tv[0], agg[0] (= sap[0]) and levels of *p
 *                        when > 0 / non-NULL
 *   p                    parameters (NULL: defaults)
 * Requirements: block dims divide the lattice dims; the number of blocks per
 * dim is even or 1 (two colours, Sec. 2.3); every coarse lattice has even
 * extents.  Errors: DD_EINVAL, DD_ENOMEM, DD_ENUMERIC (rank-deficient
 * aggregate or singular coarse self block). */
dd_status dd_setup(dd_ctx *ctx, int n_tv, const int block[4], int levels, const dd_params *p);

/* Solve D x = b by FGMRES right-preconditioned by the V-cycle, x0 = 0, until
 * ||b - D x|| <= tol ||b|| (true residual, FP64).
 *   b, x  device complex128 fine spinors [vol][4][3]; x is output only
 * Errors: DD_ESTATE before setup, DD_ENOCONV at outer_maxit (x = last iterate),
 * DD_ENUMERIC on NaN/Inf in b or breakdown. */
dd_status dd_solve(dd_ctx *ctx, const double *b, double *x, double tol, dd_stats *stats);

/* k right-hand sides solved together on the resident setup: k independent
 * FGMRES processes advance in lockstep and share every V-cycle launch (the SAP
 * kernel loads each block operator once for all of them); a right-hand side
 * leaves the batch when its own true residual reaches tol.  Batches larger
 * than max_rhs are split.  The result of each right-hand side is the one a
 * single solve computes, up to the summation order of the reductions.
 *   b, x  device complex128 [k][vol][4][3]
 *   stats array of k records or NULL */
dd_status dd_solve_batch(dd_ctx *ctx, int k, const double *b, double *x, double tol, dd_stats *stats);

/* Comparison solver of Sec. 6 (Table 3 and its footnote): FGMRES(outer_restart)
 * in FP64 right-preconditioned by `steps` BiCGStab steps (zero start) on the
 * odd-even reduced system S x_o = b_o - D_oe A_ee^{-1} b_e,
 * S = A_oo - D_oe A_ee^{-1} D_eo, and the even-site back-substitution, in
 * `precision` 32 (the paper's mixed-precision form) or 64.  Needs
 * dd_configure (the outer Krylov workspace; no multigrid setup is used).
 *   b, x  device complex128 fine spinors; x output only (x0 = 0)
 * stats: outer_iters, restarts, true_relres, converged; coarse_iters[0] counts
 * the BiCGStab steps.  Errors as dd_solve (DD_ESTATE without dd_configure). */
dd_status dd_solve_bicgstab(dd_ctx *ctx, const double *b, double *x, double tol, int steps, int precision,
                            dd_stats *stats);

/* Comparison solver of Sec. 4.1 (inexact deflation, Tables 8 and 9), in FP64 on
 * a two-level setup (levels = 2, precision 64; dd_setup with id_setup = 1 gives
 * the setup of Sec. 4.3, any other setup is accepted too):
 *   chi' = P D_c^{-1} P^H b,
 *   FGMRES(outer_restart) on D pi_R chi = pi_L b = b - D chi', right-
 *   preconditioned by `nu` SAP iterations M_SAP^(nu) from zero,
 *   x = pi_R chi + chi',   pi_R = I - P D_c^{-1} P^H D.
 * Every D_c^{-1} is the coarsest odd-even GMRES run to relative residual
 * `coarse_tol` (the method needs it near the solve tolerance, Sec. 4.2; the
 * paper's comparison uses 1e-12).  tol applies to the deflated system; the
 * returned true_relres is ||b - D x|| / ||b|| of the final x.
 *   b, x  device complex128 fine spinors; x output only
 * stats: outer_iters, restarts, coarse_iters[1] = summed coarse GMRES
 * iterations, true_relres, converged.  Errors: DD_ESTATE before dd_setup or on
 * a setup that is not FP64 two-level, DD_EINVAL on nu < 1 or tolerances <= 0,
 * otherwise as dd_solve. */
dd_status dd_solve_id(dd_ctx *ctx, const double *b, double *x, double tol, int nu, double coarse_tol,
                      dd_stats *stats);

/* Continuous batching on the resident setup.  The max_rhs right-hand-side
 * slots of the outer FGMRES are filled, advanced and emptied independently:
 * a slot whose solve has finished is read out and refilled with a new
 * right-hand side between two restart cycles while the other slots keep their
 * Krylov state (the FGMRES of Sec. 4.2 with its restart length n_kv).  Each
 * slot's iterates are those of a single dd_solve of its right-hand side.
 *
 * dd_stream_load: put b (device complex128 [vol][4][3]) with tolerance tol
 *   into a free slot (x0 = 0).  DD_ESTATE before dd_setup or if the slot is in
 *   use; DD_EINVAL for a bad slot, tol or NULL b; DD_ENUMERIC for NaN/Inf in b.
 * dd_stream_cycle: run one restart cycle of every running slot (at most
 *   n_kv Arnoldi steps and the true-residual check).  state (may be NULL):
 *   max_rhs DD_SLOT_* values afterwards; st (may be NULL): max_rhs records.
 * dd_stream_take: copy the solution of a finished slot to x (device
 *   complex128 [vol][4][3]) and free the slot; st may be NULL.  DD_ESTATE if
 *   the slot is not finished; DD_ENOCONV (x still written) if it stopped at
 *   outer_maxit.
 * While any slot is in use dd_solve / dd_solve_batch return DD_ESTATE, and
 * dd_set_mass does while a slot runs; dd_setup / dd_configure free all slots. */
enum { DD_SLOT_FREE = 0, DD_SLOT_RUNNING = 1, DD_SLOT_CONVERGED = 2, DD_SLOT_STOPPED = 3 };
dd_status dd_stream_load(dd_ctx *ctx, int slot, const double *b, double tol);
dd_status dd_stream_cycle(dd_ctx *ctx, int *state, dd_stats *st);
dd_status dd_stream_take(dd_ctx *ctx, int slot, double *x, dd_stats *st);

/* Change m0 on a context that keeps its setup: A(x) -> A(x) + (m0' - m0) I and,
 * because P^H P = I, D_c -> D_c + (m0' - m0) I on every coarse level
 * (Sec. 6, mass scaling with one setup). */
dd_status dd_set_mass(dd_ctx *ctx, double m0);

/* ---------------------------------------------------------------------------
 * Component access.  The calls below expose single steps of the method on
 * the context's current hierarchy; they are used by the parity tests and by
 * the benchmark's kernel measurements.  Arrays use the canonical layouts
 * above and complex128.
 * ------------------------------------------------------------------------- */

/* Allocate the hierarchy geometry for parameters *p without running the
 * setup (the operators of coarse levels are filled by dd_build_level). */
dd_status dd_configure(dd_ctx *ctx, const dd_params *p);

/* Install n test vectors of the transfer level -> level+1:
 * v device complex128 [n][vol_level][nd_level], n = n_tv[level]. */
dd_status dd_set_test_vectors(dd_ctx *ctx, int level, int n, const double *v);
dd_status dd_get_test_vectors(dd_ctx *ctx, int level, double *v);

/* Build P (local Gram-Schmidt of the test vectors per aggregate, eq.
 * aggInterpolation) and D_c = P^H D P with its self-block inverses from the
 * installed test vectors, without setup iterations. */
dd_status dd_build_level(dd_ctx *ctx, int level);

/* Mark a hierarchy assembled piecewise (dd_build_level) as complete. */
dd_status dd_mark_setup(dd_ctx *ctx);

/* Read back P of the transfer level -> level+1: [N][vol_level][nd_level]. */
dd_status dd_get_P(dd_ctx *ctx, int level, double *out);

/* Read back the coarse operator of level (>= 1): M [volc][9][nd][nd] with
 * slot 0 the self block, slot 1+mu the coupling to x+mu, slot 5+mu the
 * coupling to x-mu (row-major blocks), and Minv [volc][nd][nd] the inverses
 * of the self blocks.  Either pointer may be NULL. */
dd_status dd_get_coarse(dd_ctx *ctx, int level, double *M, double *Minv);

/* Read back the clover blocks A(x) = (m0+4) I + T(x) and their inverses,
 * [vol][2][6][6] each (full matrices).  Either pointer may be NULL. */
dd_status dd_get_clover(dd_ctx *ctx, double *A, double *Ainv);

typedef enum {
    DD_OP_D = 0,            /* out = D in on `level` (level 0 in FP64)                 */
    DD_OP_D_PREC = 1,       /* level-0 D in the preconditioner precision               */
    DD_OP_SAP = 2,          /* out = M_SAP^(arg) in on `level` (zero initial guess)    */
    DD_OP_VCYCLE = 3,       /* out = C^(nu) in on `level` (coarsest = levels-1)        */
    DD_OP_RESTRICT = 4,     /* out (level+1) = P^H in (level)                          */
    DD_OP_PROLONG = 5,      /* out (level) = P in (level+1)                            */
    DD_OP_COARSE_SOLVE = 6, /* out = coarsest-level odd-even GMRES solution for in     */
    DD_OP_SCHUR = 7,        /* out = S in, S = A_oo - D_oe A_ee^-1 D_eo on `level`;
                               in and out are full vectors, zero on even sites        */
    DD_OP_FGMRES = 8,       /* intermediate-level FGMRES (3+ levels) on `level`         */
    DD_OP_BICGSTAB = 9,     /* level 0: `arg` BiCGStab steps on the odd-even reduced
                               system from zero, then the even-site back-substitution
                               (the preconditioner of dd_solve_bicgstab), in the
                               preconditioner precision                              */
    DD_OP_DEFLATED = 10     /* level 0, FP64 two-level setup: out = D pi_R in, the
                               operator of dd_solve_id, with the coarse system
                               solved to the parameters' coarse_tol                   */
} dd_op;

/* Apply one component.  in/out are device complex128 vectors of the level in
 * the canonical layout (sizes given by dd_level_info).  `arg` is the number
 * of SAP iterations for DD_OP_SAP and unused otherwise.  Returns the
 * iteration count of solver components in *iters when iters != NULL. */
dd_status dd_apply(dd_ctx *ctx, int op, int level, int arg, const double *in, double *out, long *iters);

/* dd_apply on k vectors at once (1 <= k <= max_rhs), run as one batch: the
 * batched kernels of the level (for the coarse stencil with k >= 2 in FP32
 * arithmetic, the matrix-core form).  in/out: device complex128
 * [k][vol_level][nd_level]; iters: NULL or k counts. */
dd_status dd_apply_batch(dd_ctx *ctx, int op, int level, int arg, int k, const double *in, double *out,
                         long *iters);

/* Allocation-free form of dd_apply(ctx, DD_OP_D, 0, 0, in, out, NULL): out = D in
 * on the fine level in FP64, computed by the same kernels, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The call allocates nothing: the two
 * internal-layout staging spinors live in a fixed 24 MiB device array that
 * each GPU the library runs on holds until the process ends.
 *   in, out  device complex128 fine spinors [vol][4][3] (the caller allocates)
 * Limit: vol <= 65,536 sites (a 16^4 lattice); larger lattices -> DD_EINVAL.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (two threads, or two contexts on different streams) race and must be
 * serialised by the caller.  Works on configured and unconfigured contexts.
 * Errors: DD_EINVAL (NULL pointer, lattice above the limit), DD_EDEVICE. */
dd_status dd_apply_D_noalloc(dd_ctx *ctx, const double *in, double *out);

/* Lattice dims and unknowns per site of a level (level 0: the fine lattice). */
dd_status dd_level_info(const dd_ctx *ctx, int level, int dims[4], int *nd);

/* ---------------------------------------------------------------------------
 * Live kernel timing.  With profiling enabled every launch of the kernel
 * classes below is bracketed by HIP events on the context stream; durations
 * are accumulated per class when the host next synchronises.
 * ------------------------------------------------------------------------- */
typedef enum {
    DD_K_DIRAC64 = 0,      /* fine stencil, FP64 (outer operator)              */
    DD_K_DIRAC_PREC = 1,   /* fine stencil, preconditioner precision           */
    DD_K_SAP = 2,          /* fine SAP half sweep (one colour)                 */
    DD_K_RESTRICT = 3,     /* P^H (any level)                                  */
    DD_K_PROLONG = 4,      /* P (any level)                                    */
    DD_K_COARSE = 5,       /* coarse stencil / Schur pieces                     */
    DD_K_COARSE_SAP = 6,   /* coarse-level SAP half sweep                       */
    DD_K_REDUCE = 7,       /* multi-dot and update+norm reductions             */
    DD_K_BLAS = 8,         /* other vector kernels (axpy, scale, conversions)  */
    DD_K_COARSE_STEP = 9,  /* coarsest-level Arnoldi steps: one graph launch of a
                              chunk of steps, or one cooperative restart cycle
                              (Schur complement + reductions + Givens + scale) */
    DD_K_NCLASS = 10
} dd_kernel_class;

/* enable != 0 starts (and resets) profiling of every kernel class; 0 stops
 * it.  Each timed launch (or launch group) is bracketed by two HIP events
 * on the context's stream. */
dd_status dd_profile(dd_ctx *ctx, int enable);

/* As dd_profile, but only the classes whose bit (1u << class) is set in
 * class_mask are timed; the others run without events.  class_mask = 0 stops
 * profiling.  DD_EINVAL for a bit at or above DD_K_NCLASS. */
dd_status dd_profile_classes(dd_ctx *ctx, unsigned class_mask);

/* Launch count, summed duration (ms) and summed algorithmic bytes (every
 * datum a launch must read or write, counted once) of one kernel class since
 * the last dd_profile(ctx, 1).  Any output pointer may be NULL. */
dd_status dd_profile_read(dd_ctx *ctx, int kernel_class, long *launches, double *total_ms, double *total_bytes);

/* Time `reps` back-to-back launches of one kernel class on the fine level
 * (DD_K_DIRAC64, DD_K_DIRAC_PREC or DD_K_SAP = one full SAP sweep, both
 * colours, preconditioner precision, mr_steps of level 0) on internal random
 * data between two HIP events; *avg_ms = mean duration of one launch.
 * DD_K_BLAS times a plain copy kernel of one FP64 fine spinor (16 bytes read
 * and 16 written per complex entry): the reference for achievable bandwidth
 * and for scaling memory counters.  DD_K_COARSE (after dd_setup) times D_c of
 * level 1 applied to max_rhs random vectors as one batch.  Needs dd_configure (for DD_K_DIRAC_PREC /
 * DD_K_SAP). */
dd_status dd_time_kernel(dd_ctx *ctx, int kernel_class, int reps, double *avg_ms);

/* Device bytes currently allocated by the context. */
long long dd_device_bytes(const dd_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Launch schedules and autotuning.  The fine stencil and SAP kernels have
 * schedule variants that compute identical results:
 *   DD_SCHED_FUSED  a stencil workgroup covers both parities of its layout
 *                   blocks (links and spinors reused on chip)
 *   DD_SCHED_XCD    workgroups renumbered so that each of the eight XCDs
 *                   (separate L2 caches) works on a contiguous lattice region
 *   DD_SCHED_LDS    stencil: one workgroup per layout block with its spinors
 *                   staged in LDS and each internal link applied twice per
 *                   load (needs 32..128 sites per block and parity; other
 *                   layouts fall back to the FUSED schedule's kernel)
 *   DD_SCHED_NO_MFMA  the coarse stencil with 2..16 right-hand sides in FP32
 *                   arithmetic runs on the vector units (one workgroup per
 *                   site and RHS) instead of the matrix cores (one workgroup
 *                   per site for all RHS); results agree to rounding
 *   DD_SCHED_GRAPH  the Arnoldi steps of the coarsest-level GMRES (Schur
 *                   complement, reductions, Givens update, scaling: six
 *                   kernels per step) that the host enqueues between two
 *                   reads of the stop flags are captured once as one HIP
 *                   graph per (level, first step, step count, batch size)
 *                   and replayed with one launch
 *   DD_SCHED_COOP   each restart cycle of the coarsest-level GMRES runs as one
 *                   persistent cooperative launch (workgroups meet at grid
 *                   barriers between the phases of an Arnoldi step); falls
 *                   back to DD_SCHED_GRAPH / single launches when the device
 *                   does not admit the grid.  Results agree to rounding.
 *   DD_SCHED_COOP_ABORT  for tests of the fallback: every cooperative cycle
 *                   starts with its abort flag raised, so its first grid
 *                   barrier gives up, all workgroups leave, and the coarse
 *                   solve reruns with step launches (the results of a
 *                   schedule without DD_SCHED_COOP)
 * The default is DD_SCHED_LDS | DD_SCHED_XCD | DD_SCHED_GRAPH with the matrix
 * cores on; dd_autotune_coarse decides about DD_SCHED_GRAPH, DD_SCHED_COOP and
 * the cooperative grid.
 * ------------------------------------------------------------------------- */
enum { DD_SCHED_FUSED = 1, DD_SCHED_XCD = 2, DD_SCHED_LDS = 4, DD_SCHED_NO_MFMA = 8, DD_SCHED_GRAPH = 16,
       DD_SCHED_COOP = 32, DD_SCHED_COOP_ABORT = 64 };

/* Select a schedule (a combination of DD_SCHED_* flags). DD_EINVAL otherwise. */
dd_status dd_set_schedule(dd_ctx *ctx, int sched);
/* Current schedule, -1 for ctx == NULL. */
int dd_get_schedule(const dd_ctx *ctx);

/* Time every schedule of the fine kernels (flag sets 0..7; the NO_MFMA, GRAPH
 * and COOP bits are kept as set) on the context's own fields (the FP64 stencil plus nu SAP
 * sweeps once configured, each the mean of `reps` launches) and keep the
 * fastest.  chosen (may be NULL) receives it; times_ms (may be NULL) holds 8
 * doubles, the cost of each schedule (flag set 0..7) in ms. */
dd_status dd_autotune(dd_ctx *ctx, int reps, int *chosen, double *times_ms);

/* Coarse-solver autotuner (after dd_setup): times `reps` coarsest-level solves
 * of a fixed random right-hand side with step-by-step single launches, with
 * graph replay (DD_SCHED_GRAPH) and with the cooperative cycle (DD_SCHED_COOP)
 * at 16, 32, 64 and 128 workgroups.  When a step-by-step form is the fastest,
 * single launches and graph replay are compared again by `reps` whole outer
 * solves (random right-hand side, tolerance 1e-10).  The winner is kept (the
 * call sets or clears DD_SCHED_GRAPH and DD_SCHED_COOP).  chosen_grid (may be
 * NULL): 0 for step-by-step launches, else the workgroup count; times_ms (may
 * be NULL): 8 doubles, ms per coarsest-level solve in the order above, then ms
 * per outer solve with single launches and with graph replay (0 when a
 * cooperative form won). */
dd_status dd_autotune_coarse(dd_ctx *ctx, int reps, int *chosen_grid, double *times_ms);

/* Persistent autotuning (after dd_setup).  `path` names a text file with one
 * line per tuned problem shape: a key (device architecture and compute-unit
 * count, lattice, precision, max_rhs, levels, and per level the test vectors,
 * aggregate and SAP block dims and MR steps, plus nu), a tab, the schedule
 * flags and the cooperative workgroup count.  On a hit the stored schedule is
 * applied without timing; on a miss dd_autotune and dd_autotune_coarse run
 * with `reps` and their choice is appended.  The choices are launch forms
 * whose results agree to rounding, so one entry serves every field and mass of
 * its shape.  sched, grid, hit (each may be NULL) receive the schedule in use,
 * the cooperative workgroups (0: step-by-step) and 1 for a cache hit.
 * Errors: DD_EINVAL for a NULL path, reps < 1 or a file that cannot be
 * appended to (the tuned forms stay in use); DD_ESTATE before dd_setup. */
dd_status dd_autotune_cached(dd_ctx *ctx, const char *path, int reps, int *sched, int *grid, int *hit);

#ifdef __cplusplus
}
#endif
#endif /* DDAMG_H */
