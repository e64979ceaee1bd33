/*
 * pintoc -- parallel-in-time all-at-once solver for unsteady Stokes / Oseen
 * distributed optimal control on MI355X (gfx950).
 *
 * Method: Heinzelreiter & Pearson, "Diagonalization-Based Parallel-in-Time
 * Preconditioners for Instationary Fluid Flow Control Problems".
 *
 * C ABI.  Plain pointers and sizes only; no C++ types cross this boundary.
 * Every device pointer argument names memory the caller owns (for example a
 * torch tensor's data pointer).  ``stream`` is a hipStream_t passed as void*
 * (NULL = the null stream).  All entry points return PINTOC_OK (0) on success
 * or a negative PINTOC_E* code; pintoc_last_error() then gives a message
 * (thread-local).  A problem handle is not thread-safe; distinct handles are.
 *
 * Vector layout at the boundary ("canonical"): real FP64, length
 *     n_all = 2 * nt * (2 (2N+1)^2 + (N+1)^2),
 * ordered [b][t][v_x (2N+1)^2, v_y (2N+1)^2, p (N+1)^2] with
 *   b = 0: unknowns (v, p) / rows of the adjoint equations,
 *   b = 1: unknowns (lambda, mu) / rows of the state equations,
 *   t = 1..nt (time level t*tau),
 * each grid row-major with x fastest.  This is the unknown ordering of the
 * permuted all-at-once system, eq. (FinalA) (section 2.2).  Entries on the
 * Dirichlet boundary of the velocity grids and the pinned pressure node (0,0)
 * (section 2.2: the pressure is fixed at one point) must be zero on input and
 * are zero on output.
 */
#ifndef PINTOC_H
#define PINTOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PINTOC_OK = 0,
  PINTOC_NOT_CONVERGED = 1, /* pintoc_solve: tolerance not reached, x = last iterate */
  PINTOC_PAUSED = 2,        /* pintoc_solve: stopped at a restart boundary after the
                               caller's cycle budget; resume it (stats.resume)   */
  PINTOC_EINVAL = -1,       /* invalid argument (sizes, parameters, NULL pointers)   */
  PINTOC_ENOMEM = -2,       /* workspace too small                                   */
  PINTOC_EHIP = -3,         /* a HIP runtime call failed (message has its string)    */
  PINTOC_ESTATE = -4        /* call order violated (e.g. no workspace bound)         */
};

/* Opaque problem handle (owned by the library). */
typedef struct pintoc_problem pintoc_problem;

enum { PINTOC_STOKES = 0, PINTOC_OSEEN = 1 };

/* Inner treatment of the frequency blocks.
 *  LINEAR: one application of the block preconditioner per frequency
 *          (Algorithm 1 for Stokes; P~_j^(UZ) of Algorithm 3 for Oseen).
 *  GMRES:  the blocks are solved by right-preconditioned GMRES to a relative
 *          tolerance (Algorithm 2 for Stokes; its Oseen analogue, section 4).
 *  MINRES: Stokes only (EINVAL for Oseen): the real symmetric blocks Z_j of
 *          section 3.2 are solved by preconditioned MINRES with the Hermitian
 *          positive definite P~_j, stopping when the P~_j-norm of the
 *          residual is below inner_tol times that of the right-hand side (at
 *          most inner_maxit steps; inner_restart is not used).  A short
 *          recurrence replaces the Arnoldi basis: seven block vectors instead
 *          of inner_restart + 1. */
enum { PINTOC_INNER_LINEAR = 0, PINTOC_INNER_GMRES = 1, PINTOC_INNER_MINRES = 2 };

/* Arithmetic of the per-frequency block solves.  The outer Krylov method,
 * residual recomputation, FFTs and the all-at-once matrix stay FP64. */
enum { PINTOC_PREC_FP64 = 0, PINTOC_PREC_FP32_INNER = 1 };

/* Multigrid smoother (section 3.4 names successive over-relaxation).
 *  TILED:  multicolour Gauss-Seidel inside square tiles of 48 (Q2 grids) or
 *          32 (Q1 grids) node indices held in LDS, block Jacobi between tiles
 *          -- a GPU-side variant of the sweep (one launch per sweep).
 *  GLOBAL: multicolour Gauss-Seidel (SOR, relaxation factor 1) over whole
 *          grids, 9 colours (ix mod 3, iy mod 3) on Q2 and 4 on Q1 grids,
 *          forward colour order before and backward after the coarse
 *          correction -- the reading of the paper's smoother (one launch per
 *          colour).
 * Grids of at most 48 (Q2) / 32 (Q1) nodes per side are one tile, where both
 * are the same sweep. */
enum { PINTOC_SMOOTHER_TILED = 0, PINTOC_SMOOTHER_GLOBAL = 1 };

/* Outer Krylov method.  FGMRES (section 3.4) takes any preconditioner.
 * MINRES applies to the Stokes problem with the linear preconditioner
 * (Algorithm 1): the all-at-once matrix of eq. (FinalA) is symmetric and the
 * preconditioner symmetric positive definite (section 3.3), so a short
 * recurrence replaces the Arnoldi basis.
 * FGMRES_FREQ runs FGMRES in the frequency domain (section 3.1, Theorem 1):
 * with A = P_C + U (U the rank-2 n_v corner term coupling the first and last
 * time steps), the Fourier-transformed matrix is diag(G_j) plus that corner
 * term, which needs two time samples of the velocity spread over all
 * frequencies; the Krylov vectors are the kept spectra scaled by
 * sqrt(w_j / nt) (w = 1 at j = 0 and nt/2, 2 otherwise), so their Euclidean
 * inner product is the time-domain one.  b is transformed once and x back
 * once: the iterations run no FFT.  Single problems on the unit square only,
 * FP64 inner solves for Oseen (EINVAL otherwise). */
enum { PINTOC_OUTER_FGMRES = 0, PINTOC_OUTER_MINRES = 1, PINTOC_OUTER_FGMRES_FREQ = 2 };

/* Problem of section 2 (eq. OseenOptimization / OseenFlow) on a square
 * domain [x0, x1] x [y0, y1] (all four zero: the unit square; section 5 uses
 * [-1, 1]^2), Q2-Q1 Taylor-Hood elements on N x N uniform quadrilaterals
 * (section 2.2), backward Euler with nt steps of tau = T / nt.  A square of
 * side l is solved as the unit square's problem with viscosity nu / l^2 and
 * wind w / l (its matrices M, K, B, N scale as l^2, 1, l, l), with momentum
 * rows scaled by l^2, divergence rows by l and the pressure by l at the
 * boundary, so every entry point takes and returns the physical vectors.
 * The inner GMRES of the nonlinear preconditioner then measures the
 * residual of the unit-square blocks. */
typedef struct {
  int32_t N;            /* quads per side, a power of two >= 2               */
  int32_t nt;           /* time steps = FFT length, >= 2, at most 1024       */
  double T;             /* final time > 0                                    */
  double nu;            /* viscosity > 0                                     */
  double beta;          /* control cost (regularisation) > 0                 */
  int32_t flow;         /* PINTOC_STOKES or PINTOC_OSEEN                     */
  const double* wind;   /* host, [2][(2N+1)^2] Q2 nodal values of the
                           divergence-free wind (x component first); NULL
                           for Stokes.  Copied; the caller may free it.      */
  double x0, y0, x1, y1; /* domain corners; x1 - x0 = y1 - y0 > 0 required
                           (square elements); all zero = [0, 1]^2.  The wind
                           is sampled at the physical Q2 nodes
                           (x0 + ix (x1 - x0) / (2N), y0 + iy (...) / (2N)). */
} pintoc_problem_desc;

/* Solver parameters.  Defaults (pintoc_default_options) follow section 5:
 * 4 V-cycles per multigrid solve, 10 Chebyshev steps, 6 Uzawa steps with
 * mu = 3/4 (section 4), inner tolerance 1e-2, outer FGMRES restart 10. */
typedef struct {
  int32_t inner;          /* PINTOC_INNER_LINEAR, _GMRES or _MINRES            */
  int32_t precision;      /* PINTOC_PREC_*                                   */
  int32_t restart;        /* outer FGMRES restart length                     */
  int32_t max_outer;      /* outer iteration cap                             */
  double tol;             /* outer: ||b - A x||_2 <= tol ||b||_2 (true res.) */
  double inner_tol;       /* inner GMRES relative tolerance (epsilon)        */
  int32_t inner_restart;  /* inner GMRES restart length                      */
  int32_t inner_maxit;    /* inner GMRES iteration cap                       */
  int32_t n_vcycles;      /* V-cycles per multigrid application             */
  int32_t n_cheb;         /* Chebyshev semi-iteration steps                  */
  int32_t n_uzawa;        /* Uzawa steps (Oseen)                             */
  double mu_uzawa;        /* Uzawa damping parameter (Oseen)                 */
  int32_t stall_guard;    /* 1 (default): give up early where the iteration
                             stagnates -- an inner GMRES frequency whose
                             residual estimate is still above half its start
                             after a restart cycle, and the outer solve when
                             its residual estimate is above half the initial
                             residual after its first restart cycle, and at
                             least 10 iterations (NOT_CONVERGED).  A
                             safeguard outside the paper's method for blocks
                             whose multigrid diverges; 0 turns it off.       */
  int32_t outer;          /* PINTOC_OUTER_FGMRES (default) or
                             PINTOC_OUTER_MINRES (Stokes with the linear
                             preconditioner only, restart >= 4: its vectors
                             reuse the FGMRES basis; EINVAL otherwise).
                             MINRES stops on the true residual, formed every
                             5 steps once its preconditioned residual
                             estimate is below 100 tol times its start;
                             outer_iterations counts MINRES steps, capped by
                             max_outer.                                      */
  int32_t smoother;       /* PINTOC_SMOOTHER_TILED (default) or _GLOBAL      */
  int32_t pressure_stream; /* Stokes: 1 = run the pressure part of P~_j (the
                             K_p multigrid and the M_p Chebyshev steps) on a
                             second stream of the handle beside the velocity
                             multigrid (they touch disjoint buffers; fork and
                             join by events; same results); 0 (default) = one
                             stream.  The overlap shortens an application but
                             the velocity kernels then share HBM with the
                             pressure kernels.                               */
  int32_t graphs;          /* 1 = capture the launch sequence of a block
                             preconditioner application (V-cycles, Chebyshev
                             and Uzawa steps of all frequencies, section 3.4)
                             once per set of buffers into a HIP graph and
                             replay it (same kernels and arguments: same
                             results); eager launches while the timing probe
                             records, for the global smoother and on the
                             legacy null stream.  0 (default) = eager.       */
  int32_t z_fp32;          /* 1 = keep the outer FGMRES basis Z of
                             preconditioned vectors (section 3.4) in FP32.
                             They come from the FP32 inner solves, so FP32
                             storage drops nothing they carry; the solution
                             update x += Z y reads them and the true residual
                             taken at every restart corrects the rest (the
                             outer loop acts as iterative refinement).  The
                             outer method's vectors shrink from 2 restart + 3
                             to 1.5 restart + 3 canonical FP64 vectors (at
                             restart 10 and N = 128, nt = 256: 3.0 GB less).
                             Needs PINTOC_PREC_FP32_INNER and
                             PINTOC_OUTER_FGMRES (EINVAL otherwise).
                             0 (default) = FP64.                             */
} pintoc_options;

/* Phases of a solve whose device time pintoc_solve_stats reports. */
enum {
  PINTOC_PHASE_FFT = 0,      /* forward time FFT (+ T_l^{-1}), section 3.1     */
  PINTOC_PHASE_BLOCKS = 1,   /* per-frequency block solves (sections 3.2-4)    */
  PINTOC_PHASE_IFFT = 2,     /* inverse time FFT (+ T_r^{-1})                  */
  PINTOC_PHASE_MATVEC = 3,   /* all-at-once products A x of eq. (FinalA)       */
  PINTOC_PHASE_ORTH = 4,     /* outer orthogonalisation, dots, vector updates  */
  PINTOC_NPHASES = 5
};

/* Statistics of one pintoc_solve call (host memory).  Fields marked "in" are
 * read by the library (set them before the call; zero/NULL = unused), the
 * rest are written. */
typedef struct {
  int32_t outer_iterations;
  int32_t converged;             /* 1 if the tolerance was met              */
  double rel_residual;           /* final true ||b - A x|| / ||b||          */
  double inner_iterations_mean;  /* mean inner GMRES count per block solve  */
  int32_t inner_iterations_max;
  int32_t precond_applications;
  double seconds;                /* host wall time of the call              */
  double model_bytes;            /* modelled compulsory HBM bytes of the
                                    whole solve: every preconditioner
                                    application (FFT pair, the multigrid,
                                    Chebyshev and Uzawa passes of each block
                                    application, the inner GMRES block
                                    products and orthogonalisation as
                                    executed), the all-at-once products and
                                    the outer orthogonalisation             */
  double precond_model_bytes;    /* the same model for ONE application of the
                                    linear block preconditioner (Algorithm 1
                                    / Algorithm 3) to all kept frequencies,
                                    FFT pair included                       */
  double phase_seconds[PINTOC_NPHASES]; /* device time per phase (HIP events
                                    on the solve's stream)                  */
  double* residual_history;      /* in: host array or NULL; out: relative
                                    residual after each outer iteration
                                    (FGMRES: the Arnoldi estimate |g_k+1| /
                                    ||b||; MINRES: the preconditioned-norm
                                    estimate over its start)                */
  int32_t history_capacity;      /* in: entries of residual_history         */
  int32_t history_length;        /* out: entries written (<= capacity)      */
  int32_t* inner_counts;         /* in: host array or NULL; out: inner GMRES
                                    iterations per kept frequency j =
                                    0..nt/2, summed over the solve          */
  int32_t inner_counts_capacity; /* in: entries of inner_counts             */
  int32_t cycle_budget;          /* in: > 0: FGMRES only -- return
                                    PINTOC_PAUSED after this many restart
                                    cycles of this call if not converged
                                    (x = the iterate at the restart boundary,
                                    the state of the solve kept in the
                                    handle); 0: run to the end              */
  int32_t resume;                /* in: 1 = continue the handle's paused
                                    solve (same b and x pointers, x
                                    untouched since); the iteration count,
                                    initial residual, history, statistics
                                    and the cap max_outer carry over, so the
                                    iterates equal those of one uninterrupted
                                    call bit for bit                        */
} pintoc_solve_stats;

/* Fill *o with the defaults above.  Never fails for a non-NULL pointer. */
int pintoc_default_options(pintoc_options* o);

/* Validate d and o, compute the per-frequency constants (section 3.1-3.2,
 * section 4), the multigrid hierarchy and the coarsest-grid inverses, and
 * plan the workspace.  Host only; no device memory is touched.
 * Errors: PINTOC_EINVAL for N not a power of two >= 2, nt < 2 or > 1024,
 * T, nu or beta <= 0, an unknown flow/inner/precision/smoother, Oseen
 * without wind, or a domain that is not a square.
 * On success *out owns the handle; release it with pintoc_problem_destroy. */
int pintoc_problem_create(const pintoc_problem_desc* d, const pintoc_options* o,
                          pintoc_problem** out);

/* Device bytes the problem needs (all buffers, tables and Krylov bases). */
size_t pintoc_workspace_bytes(const pintoc_problem* p);

/* Bind caller-owned device memory of at least pintoc_workspace_bytes(p) bytes
 * (256-byte aligned) and upload the tables on ``stream``.  The memory must
 * stay valid until the handle is destroyed or another workspace is bound.
 * Errors: PINTOC_ENOMEM if bytes is too small, PINTOC_EINVAL for NULL or a
 * misaligned pointer, PINTOC_EHIP if an upload fails. */
int pintoc_bind_workspace(pintoc_problem* p, void* dev, size_t bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): bind the
 * problem to a device array of the library itself instead of caller memory,
 * as pintoc_bind_workspace would bind a caller workspace (carve, clear, upload
 * the tables on ``stream``).  Allocates nothing: the array is a static device
 * array of 128 MiB that each device the library runs on holds until the
 * process ends; it is taken on the current device, which must be the
 * stream's.  After the call every entry point of the problem runs on it.
 * At most one problem per device is bound to the array at a time: binding
 * another problem takes it over, and the earlier one then fails with
 * PINTOC_ESTATE until it is bound again (its results are lost).  Calls on two
 * handles that overlap in time on one device race on the array.
 * pintoc_bind_workspace or pintoc_problem_destroy release the array.
 * Errors: PINTOC_ENOMEM if pintoc_workspace_bytes(p) exceeds 128 MiB (for
 * example a Stokes problem with N = 16, nt = 16 in GMRES mode needs 53 MiB,
 * N = 32, nt = 32 needs 393 MiB), PINTOC_EINVAL for NULL, PINTOC_EHIP if the
 * array's address or an upload fails. */
int pintoc_bind_scratch(pintoc_problem* p, void* stream);

/* Right-hand side for v_0 = f = h = 0 (section 2.2): b = tau M v_d(t_k) on the
 * adjoint momentum rows (b = 0 velocity entries), zero elsewhere.
 * vd: device, [nt][2][(2N+1)^2] Q2 nodal desired state at t_k = k tau,
 * k = 1..nt (boundary values are ignored).  b: device, canonical layout.
 * Asynchronous on ``stream``. */
int pintoc_assemble_rhs(pintoc_problem* p, const double* vd, double* b, void* stream);

/* Right-hand side for general data (section 2.2: the vectors g and h that
 * carry forcing, boundary and initial conditions).  With v_k = v_k^I + h_k^B
 * (unknown interior part, known Dirichlet values), the known terms of the
 * discrete state and adjoint equations move to the right:
 *   adjoint momentum rows  tau M (v_d(t_k) - h_k^B)
 *   state momentum rows    tau M f(t_k) - (M + tau L) h_k^B + M w_{k-1},
 *                          w_0 = v_0 (interior values) + h_0^B, w_{k-1} = h_{k-1}^B
 *   state divergence rows  -tau B h_k^B
 *   adjoint divergence rows 0
 * with the full-grid matrices (boundary columns included) on interior rows.
 * All inputs are device arrays of Q2 nodal values on the full grid, NULL
 * meaning zero:
 *   vd, f: [nt][2][(2N+1)^2] at t_k = k tau, k = 1..nt (x component first);
 *   h:     [nt+1][2][(2N+1)^2] at t_k, k = 0..nt (only boundary entries read);
 *   v0:    [2][(2N+1)^2] (only interior entries read).
 * b: device, canonical layout.  With every input but vd NULL this equals
 * pintoc_assemble_rhs except that boundary values of vd enter through the
 * mass matrix.  Asynchronous on ``stream``. */
int pintoc_assemble_rhs_data(pintoc_problem* p, const double* vd, const double* f, const double* h,
                             const double* v0, double* b, void* stream);

/* y = A x with A the all-at-once matrix of eq. (FinalA) (FP64).  x, y: device,
 * canonical layout, must not alias.  Asynchronous on ``stream``. */
int pintoc_kkt_apply(pintoc_problem* p, const double* x, double* y, void* stream);

/* z = P^{-1} r, the block-circulant preconditioner of section 3 / section 4:
 * time FFT, per-frequency block solves (per options.inner: Algorithm 1/2 for
 * Stokes, Algorithm 3 or its GMRES wrapper for Oseen), inverse FFT.
 * r, z: device, canonical layout, must not alias.  LINEAR mode is
 * asynchronous on ``stream``; GMRES mode synchronises the stream once per
 * inner iteration (convergence flags are read back). */
int pintoc_precond_apply(pintoc_problem* p, const double* r, double* z, void* stream);

/* Solve A x = b with restarted flexible GMRES (section 3.4) preconditioned by
 * pintoc_precond_apply.  A solve can run in slices of whole restart cycles
 * (stats.cycle_budget / stats.resume): every restart recomputes the true
 * residual from x, so a solve paused and resumed makes exactly the
 * computation of an uninterrupted one, and a scheduler can interleave several
 * problems on one stream at restart boundaries while their vectors stay in
 * device memory.  x: device, canonical; on entry the initial guess,
 * on exit the solution (or the last iterate).  Stops when the true residual
 * satisfies ||b - A x||_2 <= options.tol ||b||_2.  st may be NULL.
 * Synchronises ``stream`` before returning.
 * Returns PINTOC_OK, or PINTOC_NOT_CONVERGED after options.max_outer
 * iterations or a Krylov breakdown without convergence (x then holds the
 * last iterate, st the residual reached), or PINTOC_PAUSED (see above);
 * PINTOC_ESTATE for a resume without a paused solve. */
int pintoc_solve(pintoc_problem* p, const double* b, double* x, pintoc_solve_stats* st,
                 void* stream);

/* Solve n independent problems concurrently (batched solve of several control
 * problems, the paper's per-problem solve of section 5 applied to a set of
 * problems at once).  Problem k runs pintoc_solve(p[k], b[k], x[k], &st[k],
 * streams[k]) on its own host thread, so the kernels of different problems
 * overlap on the device.
 *   p, b, x, streams: host arrays of n entries; the handles must be distinct
 *     and bound, the streams distinct and non-NULL (streams of the same device);
 *     b[k], x[k] are device vectors of problem k as for pintoc_solve.
 *   st: host array of n stats records, or NULL.
 * Every kernel and reduction of a solve is deterministic and depends only on
 * its own problem, so each x[k] equals the result of a separate pintoc_solve
 * call bit for bit.  Returns PINTOC_OK when all converged, PINTOC_NOT_CONVERGED
 * when some did not (see st), or the first negative code in problem order
 * (its message names the problem); n = 0 is a no-op.  Invalid arguments are
 * rejected before any work starts.  Synchronises every stream before return. */
int pintoc_solve_batch(pintoc_problem* const* p, const double* const* b, double* const* x,
                       pintoc_solve_stats* st, void* const* streams, int32_t n);

/* ---------------------------------------------------------------- groups
 * Fused batched form: the all-at-once systems of n problems solved by one
 * handle (the per-problem solve of section 5 for a set of problems at once).
 * The members share N, the flow, the domain (the unit square), the wind
 * (Oseen: the same nodal values) and the options; nt, T, nu and beta may
 * differ.  The kept frequencies of all members form one batch: every
 * per-frequency kernel of the block preconditioner (multigrid, Chebyshev,
 * Uzawa, inner GMRES; sections 3.2-4) runs once for all members, each
 * frequency with its own member's constants.  Each member runs its own FGMRES
 * (section 3.4) in lockstep with the others; members that have converged sit
 * out (their frequencies are masked).  Every kernel and reduction acts on one
 * member's data in a fixed order, so each member's result equals that of a
 * lone pintoc_solve bit for bit.
 *
 * pintoc_group_create: d is a host array of n descriptors (1 <= n <= 4096);
 * errors as pintoc_problem_create, plus PINTOC_EINVAL for members that differ
 * in N, flow, domain or wind, a domain other than the unit square, or MINRES.
 * The handle takes pintoc_workspace_bytes / pintoc_bind_workspace /
 * pintoc_problem_destroy like a lone problem; the lone vector entry points
 * (pintoc_assemble_rhs, _kkt_apply, _precond_apply, _solve) refuse it with
 * PINTOC_EINVAL.  Vectors of member k have pintoc_group_vector_length(p, k)
 * entries in the canonical layout of that member. */
int pintoc_group_create(const pintoc_problem_desc* d, int32_t n, const pintoc_options* o,
                        pintoc_problem** out);
int32_t pintoc_group_size(const pintoc_problem* p);               /* n, or 0 for NULL    */
int64_t pintoc_group_vector_length(const pintoc_problem* p, int32_t k); /* 0 if k is out of range */
/* b = right-hand side of member k for its desired state (as pintoc_assemble_rhs). */
int pintoc_group_assemble_rhs(pintoc_problem* p, int32_t k, const double* vd, double* b, void* stream);
/* y = A_k x for member k (as pintoc_kkt_apply). */
int pintoc_group_kkt_apply(pintoc_problem* p, int32_t k, const double* x, double* y, void* stream);
/* z[k] = P_k^{-1} r[k] for every member k with r[k] != NULL, in one fused
 * application (r, z: host arrays of n device pointers; z[k] must not alias
 * r[k]).  Members with r[k] == NULL are skipped (z[k] untouched). */
int pintoc_group_precond_apply(pintoc_problem* p, const double* const* r, double* const* z, void* stream);
/* Solve every member: x[k] (in: initial guess, out: solution) for b[k];
 * st: host array of n stats records or NULL (history and inner counts per
 * member as for pintoc_solve; model_bytes and the phase times are the
 * group's; cycle_budget / resume are not supported and ignored).  Returns
 * PINTOC_OK when every member converged, else PINTOC_NOT_CONVERGED (see st).
 * Synchronises ``stream`` before returning. */
int pintoc_group_solve(pintoc_problem* p, const double* const* b, double* const* x, pintoc_solve_stats* st,
                       void* stream);

/* Release the handle (does not free the bound workspace, which the caller owns). */
void pintoc_problem_destroy(pintoc_problem* p);

/* Message for the last error on this thread ("" if none). */
const char* pintoc_last_error(void);

/* Vector length of the canonical layout, for the caller's allocations. */
int64_t pintoc_vector_length(const pintoc_problem* p);

/* Inner GMRES iteration counts of the most recent preconditioner application
 * in GMRES mode, one per kept frequency j = 0..nt/2 (Algorithm 2 reports these
 * per block).  counts: host array of at least n entries; writes
 * min(n, nt/2 + 1) entries and returns that number, or a negative error code
 * (PINTOC_EINVAL for a NULL handle/array, PINTOC_ESTATE before any GMRES-mode
 * application).  Entries are zero in LINEAR mode. */
int pintoc_last_inner_iterations(const pintoc_problem* p, int32_t* counts, int32_t n);

/* Live timing of the multigrid smoother at the finest grid, for roofline
 * reports: the tiled Gauss-Seidel sweeps of section 3.4 applied to W_j
 * (Stokes) or Q_j (Oseen) on all kept frequencies at once, before (pre-) and
 * after (post-smoothing, with the prolonged coarse correction added while the
 * tile loads) the coarse-grid correction.  While enabled, each such launch is
 * bracketed by HIP events recorded on the stream it runs on; the most recent
 * 4096 launches of each kind are kept.  Enabling allocates the events
 * (host-side HIP objects, no device memory from the workspace).  The global
 * multicolour smoother (PINTOC_SMOOTHER_GLOBAL) is not timed. */
typedef struct {
  double avg_ms;             /* pre-smoothing: mean duration of the timed launches */
  int64_t launches;          /* number of launches averaged (<= 4096)         */
  double algorithmic_bytes;  /* mean compulsory bytes of one launch over the
                                grids it updates (frequencies skipped by the
                                inner GMRES excluded): read b, read x (not on
                                the first V-cycle, which starts from x = 0),
                                write the new iterate                         */
  double post_avg_ms;        /* post-smoothing: the same three figures; the   */
  int64_t post_launches;     /* bytes read the pre-smoothed iterate, b and    */
  double post_algorithmic_bytes; /* the coarse correction (a quarter field)
                                and write x                                   */
} pintoc_kernel_timing;

/* enable != 0 starts a new recording (clears previous samples); 0 stops.
 * Errors: PINTOC_EINVAL (NULL), PINTOC_EHIP (event creation failed). */
int pintoc_profile_enable(pintoc_problem* p, int32_t enable);

/* Waits for the recorded launches to finish and fills *out.
 * Errors: PINTOC_EINVAL (NULL), PINTOC_ESTATE (nothing recorded), PINTOC_EHIP. */
int pintoc_profile_read(pintoc_problem* p, pintoc_kernel_timing* out);

#ifdef __cplusplus
}
#endif
#endif /* PINTOC_H */
