/*
 * sgml.h -- C-ABI of the MI355X single-grid multi-level (SGML) solver.
 *
 * Method: Becerra-Sagredo, Mandujano and Malaga, "A GPU-based Multi-level
 * Algorithm for Boundary Value Problems" (2016).  The library solves
 *
 *     dL(u) = f,    L = div(sigma grad) + a        (Sec. 2 eq. (1), Sec. 3)
 *
 * on the unit square / cube with N = 2^n + 1 nodes per axis (Sec. 2), by
 * the saw-like refining cycle of Algorithm 3 built from the restriction of
 * Algorithm 1 (eq. (3) / (4)) and the relaxation-interpolation of
 * Algorithm 2, repeated on accumulated residuals (Sec. 2, last paragraphs)
 * until the relative residual of Sec. 3.1 reaches the tolerance.
 *
 * Conventions shared by every entry point
 *   - Arrays are dense, row-major, N^d doubles, index (k*N + j)*N + i with i
 *     along x (fastest), j along y, k along z (absent in 2D); node (i,j,k)
 *     sits at (i h, j h, k h), h = 2^-n.  Boundary nodes are included.
 *   - Faces are ordered x-, x+, y-, y+, z-, z+.  A node on any Dirichlet face
 *     is a Dirichlet node (it carries no equation); every other node is an
 *     unknown.  Neumann faces are imposed by node images (Sec. 2: reflection
 *     about the face); their solves are homogeneous, and Neumann data enter
 *     through the source (sgml_neumann_source).
 *   - With no Dirichlet face at all (the pure Neumann problem of Sec. 3.2,
 *     eq. (10)) the source is taken minus its mean and the solution has zero
 *     mean (Sec. 2, last paragraph): means are trapezoid-rule means (weight
 *     1/2 per face a node lies on), the discrete integral under which the
 *     operator with node images is symmetric.
 *   - "device" pointers are HIP device memory of the device that is current
 *     when the plan is created; "host" pointers are ordinary host memory.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is stream-ordered; entry points that return host results
 *     synchronise that stream before returning.
 *   - The caller owns every buffer.  The library allocates no device
 *     memory; a plan borrows a caller-provided device workspace for its
 *     lifetime and a small block of pinned host memory of its own.
 *   - Errors are returned as sgml_status values; nothing is thrown.  A plan
 *     is not thread-safe: one host thread at a time per plan.
 */
#ifndef SGML_H
#define SGML_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SGML_OK = 0,
    SGML_E_ARG = -1,         /* invalid argument (NULL, bad enum, bad size) */
    SGML_E_SHAPE = -2,       /* grid not of the form N = 2^n + 1 supported here */
    SGML_E_WORKSPACE = -3,   /* workspace missing, too small or misaligned */
    SGML_E_HIP = -4,         /* a HIP runtime call failed */
    SGML_E_DIVERGED = -5,    /* residual non-finite or grew above 1e3 x initial */
    SGML_E_STAGNATED = -6,   /* residual fell by less than 2x over stall_window cycles */
    SGML_E_MAXCYCLES = -7,   /* max_cycles reached above the tolerance */
    SGML_E_UNSUPPORTED = -8  /* valid request outside what this build implements */
} sgml_status;

enum { SGML_DIRICHLET = 0, SGML_NEUMANN = 1 };

/* Finite-difference molecule of dL.
 *   SGML_AXIS:   5-point (2D) / 7-point (3D) -- the "simple molecules"
 *                discussed in the conclusions.
 *   SGML_RADIAL: 9-point (2D) / 27-point (3D) radial stencil of eq. (5)
 *                (Fig. 2): every neighbour d contributes
 *                (2d/(3^d-1)) / h^2 * (sigma_d + sigma_c)/2 * (u_d - u_c) / |d|^2. */
enum { SGML_AXIS = 0, SGML_RADIAL = 1 };

/* Arithmetic of the cycle (restriction and relaxation-interpolation).
 *   SGML_FP64:  everything in FP64.
 *   SGML_MIXED: the cycle runs in FP32 on the residual scaled by a power of
 *               two; the residual recurrence, its norm and the collected
 *               solution stay FP64 (outer iterative refinement). */
enum { SGML_FP64 = 0, SGML_MIXED = 1 };

/* Visit order of Algorithm 3.  SGML_SCHEDULE_ONCE: the closing level-0
 * relaxations run once after the loop over teeth; SGML_SCHEDULE_EACH: they
 * run after every tooth. */
enum { SGML_SCHEDULE_ONCE = 0, SGML_SCHEDULE_EACH = 1 };

typedef struct {
    int dim;          /* 2 or 3 */
    int n;            /* N = 2^n + 1; 2 <= n <= 13 (2D), 2 <= n <= 10 (3D) */
    int stencil;      /* SGML_AXIS or SGML_RADIAL */
    int face[6];      /* SGML_DIRICHLET or SGML_NEUMANN per face (2D: first 4) */
    double a;         /* constant term of L; a <= 0 keeps forward Euler stable */
    double theta;     /* pseudo-time step dtau = theta / D(x), D the local
                         diagonal (Sec. 2, Sec. 3.4); <= 0 selects the default
                         0.8 (5-pt), 6/7 (7-pt), 1.0 (radial) */
} sgml_problem;

typedef struct {
    double tol;       /* stop when max|r| / max|r_0| <= tol (Sec. 3.1) */
    int max_cycles;   /* >= 1 */
    int n_r;          /* max relaxation-interpolations per visit (Sec. 3.1
                         runs use 2); <= 0 means full doubling (Fig. 1) */
    int schedule;     /* SGML_SCHEDULE_ONCE or SGML_SCHEDULE_EACH */
    int precision;    /* SGML_FP64 or SGML_MIXED; must not exceed the plan's */
    int record_pres;  /* 1: keep the per-visit pseudo-residuals of the last cycle */
    int profile;      /* 1: time every level-0 launch (fused visit, relaxation,
                         cycle-end pass) with stream events (prof_* in the stats) */
    int coarse_nodes; /* levels of at most this many nodes run together in one
                         single-workgroup launch per run of coarse operations
                         (their arrays staged in LDS when they fit);
                         0: default (1100 in 2D, 5000 in 3D), < 0: every operation
                         launched alone */
    int stall_window; /* SGML_E_STAGNATED when the residual has not halved over
                         this many cycles; 0: default (3), < 0: never */
    int fuse;         /* 2D levels with at least this many nodes per axis (and
                         too large for the coarse kernel) run each visit as one
                         fused row-marching pass; 0: default (65), < 0: never (one
                         launch per interpolation, relaxation and injection, and
                         the generic relaxation, transfer and cycle-end kernels in
                         2D and 3D); values below 64 act as 64 */
    int chunk_rows;   /* rows each wavefront marches through in the 2D row-marching
                         passes; 0: chosen per launch (short visits: 8 rows, 4 on
                         levels of at most 1025 nodes per axis, 2 on levels of at
                         most 257; long visits of large levels: the shortest chunk
                         that fills the device's wavefront slots for the kernel in
                         one round, half of them in FP64 and in the fused closing
                         visit; the cycle end: two wavefronts per SIMD, 137 rows
                         on 4097^2, fewer on levels too small to fill the device),
                         values below 8 act as 8, odd values are rounded up to even
                         in the visits */
    int z_chunk;      /* planes each workgroup marches through in the 3D z-marching
                         passes (relaxation, paired relaxation, interpolation,
                         restriction, constant-coefficient cycle end) on levels of
                         at least 33 nodes per axis; 0: chosen per level (about
                         1024 workgroups, at most 16 / 32 planes), otherwise clamped
                         to the level (the paired relaxation balances its chunks,
                         the interpolation rounds up to an even count) */
    int graphs;       /* >= 0 (default): the cycles after the first, which repeat
                         the same launches, are captured once as a HIP graph
                         (two for the two buffers of a double-buffered residual)
                         and replayed, the graph kept by the plan for later
                         solves with the same options, output and coefficient;
                         < 0: every launch issued one by one.  Profiled solves
                         never use graphs. */
    int fuse_end;     /* 2D FP32 cycles with a constant coefficient: the cycle's
                         closing level-0 visit and the cycle end run as one pass
                         in every cycle without Dirichlet data to impose and
                         nothing recorded per visit; 0: default, on levels large
                         enough for the pass to be bound by memory traffic (4097^2
                         and above at n_r = 2), > 0: on every level where it
                         applies, < 0: never.  The results are the same. */
} sgml_opts;

#define SGML_HIST 512
#define SGML_MAX_VISITS 128
#define SGML_PROF_CLASSES 5
enum {
    SGML_PROF_SWEEP0 = 0,
    SGML_PROF_VISIT0_INJ = 1,
    SGML_PROF_VISIT0 = 2,
    SGML_PROF_CYCLE_END = 3,
    SGML_PROF_VISIT0_END = 4
};
typedef struct {
    int status;                     /* same value as returned */
    int cycles;                     /* cycles run */
    double norm0;                   /* max|f - dL(u_init)| over unknowns, u_init = G on
                                       Dirichlet nodes and 0 elsewhere */
    double relres;                  /* recursive residual max|r_i| / norm0 */
    double history[SGML_HIST];      /* relres after each cycle */
    int visits;                     /* visits per cycle */
    double pres[SGML_MAX_VISITS];   /* per-visit pseudo-residual of the last
                                       relaxation, last cycle (record_pres) */
    long long node_updates;         /* level-node relaxations performed */
    float ms;                       /* device time of the solve, stream events */
    /* profile: launches, summed device time and relaxations of the level-0
     * kernels by class: SGML_PROF_SWEEP0 one relaxation per launch;
     * SGML_PROF_VISIT0_INJ / SGML_PROF_VISIT0 fused visits (interpolation
     * prologue, several relaxations) with / without the injection epilogue;
     * SGML_PROF_CYCLE_END the cycle-end pass (residual recurrence);
     * SGML_PROF_VISIT0_END the cycle's closing level-0 visit and the cycle
     * end in one pass (2D mixed-precision cycles after the first, constant
     * coefficient).  At most 32 launches of a cycle are timed; prof_untimed
     * counts the others. */
    int prof_launches[SGML_PROF_CLASSES];
    float prof_ms[SGML_PROF_CLASSES];
    int prof_sweeps[SGML_PROF_CLASSES];
    int prof_untimed;
} sgml_stats;

typedef struct sgml_plan sgml_plan;

/* Bytes of device workspace a plan for `prob` at `precision` needs (the
 * MIXED size also serves FP64 solves).  Returns 0 for an invalid problem.
 * Workspace must be 256-byte aligned. */
size_t sgml_workspace_bytes(const sgml_problem *prob, int precision);

/* Create a plan: validates prob (SGML_E_ARG / SGML_E_SHAPE), checks that
 * `workspace` (device, ws_bytes long, 256-byte aligned) holds at least
 * sgml_workspace_bytes(prob, precision) (SGML_E_WORKSPACE), and records the
 * current device.  The plan uses sigma = 1 until sgml_plan_set_coeffs.
 * workspace NULL with ws_bytes 0 creates a plan without workspace, which only
 * sgml_solve_noalloc and sgml_coeff_grad accept (the others return
 * SGML_E_WORKSPACE). */
sgml_status sgml_plan_create(const sgml_problem *prob, int precision, void *workspace,
                             size_t ws_bytes, sgml_plan **out);

/* Bind the coefficient field sigma (device, N^d doubles, sigma > 0) or NULL
 * for sigma = 1, and build its per-level restrictions (Algorithm 1 applied
 * to the coefficient, "restricted sources and coefficients", Sec. 2) in the
 * workspace.  The plan borrows sigma: it must stay valid and unchanged
 * while the plan solves, computes residuals or gradients. */
sgml_status sgml_plan_set_coeffs(sgml_plan *plan, const double *sigma, void *stream);

/* Solve dL(u) = f (Sec. 2) to opts->tol.
 *   f: device, N^d; values at Dirichlet nodes are ignored.
 *   G: device, N^d Dirichlet values (read at Dirichlet nodes only), or NULL
 *      for zero.  Imposed through the variation in the first cycle (Sec. 2).
 *   u: device, N^d, output (overwritten; may not alias f or G).
 *   stats: host, optional.
 * Returns SGML_OK on convergence, else a failure status with u holding the
 * last collected solution.  Synchronises the stream once per cycle (stop
 * test). */
sgml_status sgml_solve(sgml_plan *plan, const double *f, const double *G, double *u,
                       const sgml_opts *opts, void *stream, sgml_stats *stats);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): sgml_solve with a
 * static workspace the library holds on each device in place of the plan's.
 *   - The static workspace is SGML_NOALLOC_WORKSPACE_BYTES (64 MiB) per
 *     device, reserved when the library's code is loaded on the device and
 *     held until the process ends; sgml_workspace_bytes(prob, precision)
 *     must not exceed it (2D up to 1025^2 in either precision, 3D up to
 *     65^3, and 129^3 in FP64 plans), else SGML_E_WORKSPACE and nothing is
 *     enqueued.
 *   - plan may have been created with a workspace or without one
 *     (sgml_plan_create with workspace NULL and ws_bytes 0, a plan only this
 *     entry point can solve with).  The plan's own workspace is not touched.
 *   - The call allocates nothing: no device, pinned or managed memory, no
 *     events (opts->profile must be 0, else SGML_E_ARG); the coefficient
 *     pyramid of the plan's sigma is rebuilt in the static workspace on every
 *     call, since the previous call on the device may have been another plan's.
 *   - Every call on a device shares that device's workspace: calls that
 *     overlap in time on one device (other host threads, other streams) race
 *     and give wrong results.  Calls ordered on one stream, or separated by
 *     synchronisation, are safe.
 * Other arguments, results and statuses as sgml_solve. */
#define SGML_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)
sgml_status sgml_solve_noalloc(sgml_plan *plan, const double *f, const double *G, double *u,
                               const sgml_opts *opts, void *stream, sgml_stats *stats);

/* Batches of right-hand sides (the vector Poisson problem of Sec. 3.3 solves
 * one equation per component with the same operator).  A batch plan holds
 * nrhs solvers of one problem: one coefficient pyramid (built once by
 * sgml_plan_set_coeffs) and, per right-hand side, a slice of the workspace
 * (sgml_workspace_bytes_batch = nrhs x sgml_workspace_bytes) and, beyond the
 * first, a stream of its own (default priority) created with the plan.
 * sgml_solve_batch solves the first k <= nrhs right-hand sides at once:
 *   f, u: device, k x N^d doubles (component r at offset r N^d; u may not
 *   overlap f or G); G: device k x N^d Dirichlet values or NULL;
 *   stats: host array of k (optional).
 * The right-hand sides advance in lock step, one cycle each per round, on
 * their own streams, forked from and joined to `stream` by events, so that
 * the latency-bound coarse levels of one overlap the others' work; one host
 * synchronisation per round serves all stop tests.  A right-hand side stops
 * at its own tolerance.  Results equal k calls of sgml_solve.  Returns
 * SGML_OK when all converged, else the first other status in component
 * order.  Other entry points use the first right-hand side's solver only.
 * nrhs <= SGML_MAX_BATCH. */
#define SGML_MAX_BATCH 16
size_t sgml_workspace_bytes_batch(const sgml_problem *prob, int precision, int nrhs);
sgml_status sgml_plan_create_batch(const sgml_problem *prob, int precision, int nrhs, void *workspace,
                                   size_t ws_bytes, sgml_plan **out);
sgml_status sgml_solve_batch(sgml_plan *plan, int nrhs, const double *f, const double *G, double *u,
                             const sgml_opts *opts, void *stream, sgml_stats *stats);

/* Residual of a candidate solution (Sec. 2 recurrence, Sec. 3.1 norm):
 *   r = f - dL(u) at unknowns, 0 at Dirichlet nodes (r: device N^d or NULL);
 *   *rmax = max |r| (host, optional);
 *   *norm0 = max |f - dL(u_init)| (host, optional; u_init = G on Dirichlet
 *   nodes, 0 elsewhere).  u must hold the Dirichlet values on Dirichlet
 *   nodes for r to be the residual of the boundary value problem. */
sgml_status sgml_residual(sgml_plan *plan, const double *f, const double *G, const double *u,
                          double *r, double *rmax, double *norm0, void *stream);

/* Adjoint solve dL^T(lambda) = g on the unknowns with lambda = 0 on
 * Dirichlet nodes (the transposed system of the implicit-function theorem
 * on dL(u) = f).  For all-Dirichlet faces the operator is symmetric and this
 * is sgml_solve with source g and zero Dirichlet values.  With Neumann faces
 * the node images make dL symmetric only under the trapezoid weights W (1/2
 * per Neumann face a node lies on), dL^T = W dL W^-1: the library solves
 * dL mu = W^-1 g with the same cycle and returns lambda = W mu.  With no
 * Dirichlet face at all: SGML_E_UNSUPPORTED.  g, lambda: device N^d (lambda
 * may not alias g). */
sgml_status sgml_adjoint(sgml_plan *plan, const double *g, double *lambda, const sgml_opts *opts,
                         void *stream, sgml_stats *stats);

/* Gradient of a loss with respect to sigma, given the solution u and the
 * adjoint lambda of dLoss/du (implicit-function theorem on dL(u) = f):
 *   grad[m] = -sum_x lambda[x] d(dL u)[x] / dsigma[m],
 * every stencil term C/h^2 w_k (sigma_s + sigma_x)/2 (u_s - u_x) of row x
 * (s the node neighbour k samples, an image across a Neumann face)
 * contributing to sigma_s and sigma_x.  For all-Dirichlet faces
 *   grad[m] = -C/(2h^2) sum_k w_k (u[m+d_k] - u[m]) (lambda[m] - lambda[m+d_k])
 * over neighbours inside the grid.  u, lambda, grad: device N^d. */
sgml_status sgml_coeff_grad(sgml_plan *plan, const double *u, const double *lambda, double *grad,
                            void *stream);

/* Neumann data (Sec. 2: the derivative at the boundary imposed by substituting
 * the data lying outside the domain).  flux[f] (f = x-, x+, y-, y+, z-, z+;
 * host array of 6 device pointers, entries of Dirichlet faces and of faces
 * beyond the dimension ignored, NULL = zero) holds the outward normal
 * derivative on face f at its N^(d-1) nodes, indexed by the face's other
 * coordinates in axis order, the lower axis fastest: x faces (k N + j), y
 * faces (k N + i), z faces (j N + i); in 2D j, resp. i.  A neighbour sample
 * that crosses a Neumann face takes the image's value plus 2 h g (the
 * central difference across the face), one term per face crossed, g read at
 * the image's other coordinates.  These terms do not depend on u: this call
 * writes f_out = f - (their part of dL) at the unknowns (f elsewhere), and
 * sgml_solve(f_out) then solves the problem with the Neumann data.  f, f_out:
 * device N^d (may alias). */
sgml_status sgml_neumann_source(sgml_plan *plan, const double *f, const double *const *flux, double *f_out,
                                void *stream);

/* Visit list of Algorithm 3 for N = 2^n + 1: level[v], count[v] for
 * v < min(*len, cap); *len receives the full length.  Host only. */
sgml_status sgml_schedule(int n, int n_r, int schedule, int *level, int *count, int cap, int *len);

/* Static description of a status code. */
const char *sgml_status_string(sgml_status status);

/* Release the plan's host resources (the workspace and sigma stay the
 * caller's). */
void sgml_plan_destroy(sgml_plan *plan);

#ifdef __cplusplus
}
#endif
#endif /* SGML_H */
