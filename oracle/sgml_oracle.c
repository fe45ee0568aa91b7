/*
 * sgml_oracle.c -- plain, slow FP64 CPU reference of the single-grid
 * multi-level (SGML) method of Becerra-Sagredo, Mandujano and Malaga,
 * "A GPU-based Multi-level Algorithm for Boundary Value Problems" (2016).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file.  The product library shares
 * no code, header, table or helper with it.
 *
 * Everything here acts on the full single grid, as the paper states the
 * method (Sec. 2): one array per field, levels are index subsets.
 *   - restriction: Algorithm 1 with the averages of eq. (3) / eq. (4);
 *   - relaxation-interpolation: Algorithm 2, forward Euler of eq. (2) at the
 *     level nodes, multilinear hat interpolation of the variation elsewhere;
 *   - single cycle: Algorithm 3 (saw-like refining cycle);
 *   - recurrence on accumulated residuals and the stop test: Sec. 2 (last
 *     two paragraphs) and Sec. 3.1;
 *   - operator: L = div(sigma grad) + a (Sec. 3) with the radial stencil of
 *     eq. (5) or the axis ("simple molecule") stencil.
 * Readings of passages that are silent or ambiguous are stated at the
 * function that takes them.  No blocking, fusion or reordering is done
 * beyond caching the restriction pyramid of a cycle, whose values are the
 * ones Algorithm 1 recomputes before each visit (its input does not change
 * inside a cycle).
 *
 * Layout: arrays hold N^d doubles, N = 2^n + 1, index (k*N + j)*N + i with
 * i along x (fastest), j along y, k along z (absent in 2D).  Faces are
 * ordered x-, x+, y-, y+, z-, z+.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_DIRICHLET 0
#define ORC_NEUMANN 1
#define ORC_AXIS 0
#define ORC_RADIAL 1
#define ORC_RADIAL_PRINTED 2

enum {
    ORC_OK = 0,
    ORC_E_ARG = -1,
    ORC_E_DIVERGED = -5,
    ORC_E_STAGNATED = -6,
    ORC_E_MAXCYCLES = -7
};

typedef struct {
    int dim;              /* 2 or 3 */
    int n;                /* N = 2^n + 1 nodes per axis, h = 1 / 2^n */
    int stencil;          /* ORC_AXIS, ORC_RADIAL or ORC_RADIAL_PRINTED */
    int face[6];          /* ORC_DIRICHLET / ORC_NEUMANN, x-, x+, y-, y+, z-, z+ */
    double a;             /* constant of L = div(sigma grad) + a */
    double theta;         /* pseudo-time step as a fraction of 1/diagonal */
    const double *sigma;  /* N^d coefficient, NULL means sigma = 1 */
} orc_problem;

typedef struct {
    double tol;       /* stop when the recursive relative residual <= tol */
    int max_cycles;
    int n_r;          /* cap on relaxation-interpolations per visit, <= 0: none */
    int reading;      /* 0: the closing level-0 relaxations of Algorithm 3 run once after the loop; 1: inside it */
    int stall_window; /* STAGNATED when the residual has not halved over this many
                         cycles; 0: 3, < 0: never */
} orc_opts;

#define ORC_HIST 512
typedef struct {
    int status;
    int cycles;
    double norm0;               /* max-norm of the initial residual f - L(u_init) */
    double relres;              /* recursive residual / norm0 */
    double relres_true;         /* max|f - L(u)| / norm0 */
    double history[ORC_HIST];   /* recursive relres after each cycle */
    long long relax_updates;    /* level-node relaxations (the method's own work) */
    long long restrict_updates; /* level-node restriction averages */
    long long interp_updates;   /* off-level interpolations */
    long long fullgrid_updates; /* node visits of the literal full-grid routines */
} orc_stats;

/* ------------------------------------------------------------------ grid */

typedef struct {
    int dim, n, N;
    long long M;
    double h;
    int face[6];
    double a, theta;
    int K;            /* number of neighbours of the stencil */
    int off[26][3];   /* neighbour offsets (x, y, z) */
    double w[26];     /* neighbour weights */
    double C;         /* stencil prefactor */
} grid_t;

/* The axis stencil is the classic 5-point (2D) / 7-point (3D) Laplacian.
 * The radial stencil follows eq. (5): every one of the 3^d - 1 neighbours
 * contributes a radial difference quotient, and the flux is averaged over
 * the sphere of radius h/2 (Fig. 2), which gives the prefactor 2d/(3^d - 1)
 * (3/13 in 3D, 1/2 in 2D).  Reading: each term divides the difference by
 * the squared distance (h l)^2 -- a first difference over h*l is a radial
 * derivative; the flux integral adds the second factor 1/(h l).  With this
 * reading the stencil reproduces the Laplacian of quadratics exactly and
 * its forward-Euler limit is the paper's dtau < h^2/2 (Sec. 2).
 * ORC_RADIAL_PRINTED keeps eq. (5) as printed, one factor 1/(h l) per term
 * (weights 1/l, same prefactor); it exists to measure the discrepancy. */
static void grid_init(grid_t *g, const orc_problem *p)
{
    g->dim = p->dim;
    g->n = p->n;
    g->N = (1 << p->n) + 1;
    g->M = (long long)g->N * g->N * (p->dim == 3 ? g->N : 1);
    g->h = 1.0 / (double)(1 << p->n);
    for (int f = 0; f < 6; ++f) g->face[f] = p->face[f];
    g->a = p->a;
    g->theta = p->theta;
    g->K = 0;
    int zr = (p->dim == 3) ? 1 : 0;
    for (int dz = -zr; dz <= zr; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int nz = (dx != 0) + (dy != 0) + (dz != 0);
                if (nz == 0) continue;
                if (p->stencil == ORC_AXIS && nz != 1) continue;
                g->off[g->K][0] = dx;
                g->off[g->K][1] = dy;
                g->off[g->K][2] = dz;
                g->w[g->K] = (p->stencil == ORC_AXIS) ? 1.0
                             : (p->stencil == ORC_RADIAL) ? 1.0 / (double)nz : 1.0 / sqrt((double)nz);
                g->K++;
            }
    g->C = (p->stencil == ORC_AXIS) ? 1.0 : (2.0 * p->dim) / (double)g->K;
}

static long long node_index(const grid_t *g, int i, int j, int k)
{
    return ((long long)k * g->N + j) * g->N + i;
}

static void node_coords(const grid_t *g, long long id, int c[3])
{
    c[0] = (int)(id % g->N);
    c[1] = (int)((id / g->N) % g->N);
    c[2] = (g->dim == 3) ? (int)(id / ((long long)g->N * g->N)) : 0;
}

/* Image of a coordinate outside the grid: reflection about the face node
 * (Sec. 2, Neumann conditions by images). */
static int mirror(int i, int N)
{
    if (i < 0) return -i;
    if (i > N - 1) return 2 * (N - 1) - i;
    return i;
}

static double sample(const grid_t *g, const double *f, const int c[3], int lam, const int d[3])
{
    int i = mirror(c[0] + lam * d[0], g->N);
    int j = mirror(c[1] + lam * d[1], g->N);
    int k = (g->dim == 3) ? mirror(c[2] + lam * d[2], g->N) : 0;
    return f[node_index(g, i, j, k)];
}

/* A node is a Dirichlet node when it lies on any Dirichlet face; it is then
 * not an unknown, whatever its other faces are. */
static int is_dirichlet(const grid_t *g, const int c[3])
{
    for (int ax = 0; ax < g->dim; ++ax) {
        if (c[ax] == 0 && g->face[2 * ax] == ORC_DIRICHLET) return 1;
        if (c[ax] == g->N - 1 && g->face[2 * ax + 1] == ORC_DIRICHLET) return 1;
    }
    return 0;
}

/* Trapezoid weight of a node: 1/2 for every Neumann face it lies on.  With
 * node images on Neumann faces, the coupling of a face node to its inner
 * neighbour is counted twice in the face node's row and once in the
 * neighbour's, so W dL is symmetric (on the unknowns) for W = diag(weights). */
static double trap_weight(const grid_t *g, const int c[3])
{
    double w = 1.0;
    for (int ax = 0; ax < g->dim; ++ax) {
        if (c[ax] == 0 && g->face[2 * ax] == ORC_NEUMANN) w *= 0.5;
        if (c[ax] == g->N - 1 && g->face[2 * ax + 1] == ORC_NEUMANN) w *= 0.5;
    }
    return w;
}

static int has_dirichlet_face(const grid_t *g)
{
    for (int f = 0; f < 2 * g->dim; ++f)
        if (g->face[f] == ORC_DIRICHLET) return 1;
    return 0;
}

/* v minus its mean under the trapezoid rule (weights trap_weight): the
 * discrete integral over the domain divided by its volume. */
static void remove_mean(const grid_t *g, double *v)
{
    double sw = 0.0, swv = 0.0;
    for (long long id = 0; id < g->M; ++id) {
        int c[3];
        node_coords(g, id, c);
        double w = trap_weight(g, c);
        sw += w;
        swv += w * v[id];
    }
    double mean = swv / sw;
    for (long long id = 0; id < g->M; ++id) v[id] -= mean;
}

static int on_level(const grid_t *g, const int c[3], int lam)
{
    for (int ax = 0; ax < g->dim; ++ax)
        if (c[ax] % lam != 0) return 0;
    return 1;
}

static long long level_count(const grid_t *g, int nu)
{
    long long m = ((long long)g->N - 1) / (1LL << nu) + 1;
    return g->dim == 3 ? m * m * m : m * m;
}

/* hat function of unit half-width */
static double hat(double t)
{
    double v = 1.0 - fabs(t);
    return v > 0.0 ? v : 0.0;
}

/* ----------------------------------------------------------- restriction */

/* Eq. (3) / eq. (4): weighted average of the 3^d neighbours at distance
 * lam*h, weights hat(p/2) per axis and the factor 2^-d.  Samples outside the
 * grid are images (Sec. 2, Neumann conditions); Dirichlet-node values are
 * never read by an unknown's average, so images are used on every face. */
static double restrict_at(const grid_t *g, const double *f, const int c[3], int lam)
{
    double acc = 0.0;
    int zr = (g->dim == 3) ? 1 : 0;
    for (int r = -zr; r <= zr; ++r)
        for (int q = -1; q <= 1; ++q)
            for (int p = -1; p <= 1; ++p) {
                int d[3] = {p, q, r};
                double wgt = hat(p / 2.0) * hat(q / 2.0) * hat(r / 2.0);
                acc += wgt * sample(g, f, c, lam, d);
            }
    return acc / (double)(1 << g->dim);
}

/* One pass of Algorithm 1's loop body: out = R_lam(in) at every node. */
static void restrict_step(const grid_t *g, const double *in, double *out, int lam)
{
#pragma omp parallel for schedule(static)
    for (long long id = 0; id < g->M; ++id) {
        int c[3];
        node_coords(g, id, c);
        out[id] = restrict_at(g, in, c, lam);
    }
}

/* Algorithm 1, restriction(nu).  Reading of its loop bound: nu
 * applications, m = 0 .. nu-1, so that restriction(0) is the identity and
 * the level-0 pseudo-residual is the true residual on the full mesh
 * (Sec. 3.1).  Each application R_{2^m} reads level-m nodes at the
 * level-(m+1) nodes. */
static void restriction(const grid_t *g, const double *f, double *g_out, int nu, double *tmp,
                        orc_stats *st)
{
    memcpy(g_out, f, sizeof(double) * (size_t)g->M);
    for (int m = 0; m < nu; ++m) {
        restrict_step(g, g_out, tmp, 1 << m);
        memcpy(g_out, tmp, sizeof(double) * (size_t)g->M);
        if (st) {
            st->restrict_updates += level_count(g, m + 1);
            st->fullgrid_updates += g->M;
        }
    }
}

/* ---------------------------------------------------------------- operator */

/* The stride-lam finite-difference operator dL_lam of L = div(sigma grad) + a
 * at node c (Sec. 3, eq. (5)): sum over neighbours of
 *   C/(lam h)^2 * w_k * (sigma_k + sigma_c)/2 * (u_k - u_c)  +  a u_c.
 * Also returns the magnitude of its diagonal, D = C/(lam h)^2 sum w_k
 * (sigma_k + sigma_c)/2 - a, which sets the local pseudo-time step. */
static double apply_op(const grid_t *g, const double *sig, const double *u, const int c[3], int lam,
                       double *diag)
{
    long long id = node_index(g, c[0], c[1], c[2]);
    double sc = sig ? sig[id] : 1.0;
    double uc = u[id];
    double acc = 0.0, dsum = 0.0;
    for (int k = 0; k < g->K; ++k) {
        double sk = sig ? sample(g, sig, c, lam, g->off[k]) : 1.0;
        double coef = g->w[k] * 0.5 * (sk + sc);
        acc += coef * (sample(g, u, c, lam, g->off[k]) - uc);
        dsum += coef;
    }
    double scale = g->C / ((lam * g->h) * (lam * g->h));
    if (diag) *diag = scale * dsum - g->a;
    return scale * acc + g->a * uc;
}

/* ---------------------------------------------------- relaxation-interp. */

/* Multilinear interpolation of a level variation to node y: the sum over
 * level nodes x of prod_i hat((y_i - x_i)/lam) * delta(x), i.e. tensor hat
 * functions of support 2 lam h (Sec. 2).  Only the 2^d corners of the
 * level cell containing y have non-zero weight. */
static double interp_at(const grid_t *g, const double *delta, const int y[3], int lam)
{
    int lo[3] = {0, 0, 0};
    for (int ax = 0; ax < g->dim; ++ax) lo[ax] = (y[ax] / lam) * lam;
    double acc = 0.0;
    int corners = 1 << g->dim;
    for (int b = 0; b < corners; ++b) {
        int x[3] = {0, 0, 0};
        double wgt = 1.0;
        int inside = 1;
        for (int ax = 0; ax < g->dim; ++ax) {
            x[ax] = lo[ax] + ((b >> ax) & 1) * lam;
            if (x[ax] > g->N - 1) inside = 0;
            wgt *= hat((double)(y[ax] - x[ax]) / lam);
        }
        if (!inside || wgt == 0.0) continue;
        acc += wgt * delta[node_index(g, x[0], x[1], x[2])];
    }
    return acc;
}

/* Algorithm 2, relaxation-interpolation(nu), acting on the whole grid.
 *   u1 = u;  level nodes: u = D_lam(u1);  other nodes: u = u1 + I_lam(delta).
 * D_lam is one forward-Euler step of eq. (2) with the stride-lam operator,
 * the restricted source gnu and restricted coefficient signu, and the local
 * step theta / D(x) (Sec. 3.4 adjusts the step to the local coefficient;
 * reading: the local diagonal, which contains the neighbours' averages).
 * Dirichlet level nodes take the variation delta = G - u1 (Sec. 2: the
 * Dirichlet condition is imposed in the variation); G == NULL means zero.
 * Reading of the interpolated variation "of the previous iteration": each
 * variation is interpolated once, in the call that made it; since the
 * relaxation reads level nodes only, this equals the lagged form with a
 * final flush.  Returns the pseudo-residual max |dL_lam u1 - gnu| over
 * unknown level nodes (Sec. 3.1). */
static double relax_interp(const grid_t *g, int nu, const double *u1, double *u, const double *gnu,
                           const double *signu, const double *G, double *delta, orc_stats *st)
{
    int lam = 1 << nu;
    double pres = 0.0;
#pragma omp parallel for schedule(static) reduction(max : pres)
    for (long long id = 0; id < g->M; ++id) {
        int c[3];
        node_coords(g, id, c);
        delta[id] = 0.0;
        if (!on_level(g, c, lam)) continue;
        if (is_dirichlet(g, c)) {
            delta[id] = (G ? G[id] : 0.0) - u1[id];
        } else {
            double D;
            double Lu = apply_op(g, signu, u1, c, lam, &D);
            double r = Lu - gnu[id];
            delta[id] = (g->theta / D) * r;
            if (fabs(r) > pres) pres = fabs(r);
        }
    }
#pragma omp parallel for schedule(static)
    for (long long id = 0; id < g->M; ++id) {
        int c[3];
        node_coords(g, id, c);
        if (on_level(g, c, lam))
            u[id] = u1[id] + delta[id];
        else
            u[id] = u1[id] + interp_at(g, delta, c, lam);
    }
    if (st) {
        long long lv = level_count(g, nu);
        st->relax_updates += lv;
        st->interp_updates += g->M - lv;
        st->fullgrid_updates += g->M;
    }
    return pres;
}

/* -------------------------------------------------------------- schedule */

/* Algorithm 3 as a list of visits (level, number of relaxation-interpolations).
 * Tooth nu1 = n-1 .. 0 visits nu1, nu1-1 (skipped when negative) and nu1,
 * each min(n_r, 2^(n-nu1)) times.  Reading 0: the closing level-0
 * relaxations (min(n_r, 2^n) times) run once after the loop; reading 1: at
 * the end of every tooth.  n_r <= 0 means full doubling (Fig. 1). */
int orc_schedule(int n, int n_r, int reading, int *level, int *count, int cap)
{
    int len = 0;
#define PUSH(L, C)                        \
    do {                                  \
        if (len < cap) {                  \
            level[len] = (L);             \
            count[len] = (C);             \
        }                                 \
        len++;                            \
    } while (0)
    for (int nu1 = n - 1; nu1 >= 0; --nu1) {
        long long full = 1LL << (n - nu1);
        int c = (int)((n_r > 0 && n_r < full) ? n_r : full);
        PUSH(nu1, c);
        if (nu1 >= 1) PUSH(nu1 - 1, c);
        PUSH(nu1, c);
        if (reading == 1) {
            long long f0 = 1LL << n;
            PUSH(0, (int)((n_r > 0 && n_r < f0) ? n_r : f0));
        }
    }
    if (reading != 1) {
        long long f0 = 1LL << n;
        PUSH(0, (int)((n_r > 0 && n_r < f0) ? n_r : f0));
    }
#undef PUSH
    return len;
}

/* ----------------------------------------------------------------- cycle */

typedef struct {
    grid_t g;
    double **sig;     /* restricted coefficient per level (NULL entries when sigma = 1) */
    double **pyr;     /* restricted source per level for the current cycle */
    double *tmp, *u1, *delta;
} ctx_t;

static void ctx_free(ctx_t *x)
{
    if (x->sig) {
        for (int l = 1; l < x->g.n; ++l) free(x->sig[l]);
        free(x->sig);
    }
    if (x->pyr) {
        for (int l = 1; l < x->g.n; ++l) free(x->pyr[l]);
        free(x->pyr);
    }
    free(x->tmp);
    free(x->u1);
    free(x->delta);
    memset(x, 0, sizeof(*x));
}

static int valid_problem(const orc_problem *p)
{
    if (!p) return 0;
    if (p->dim != 2 && p->dim != 3) return 0;
    if (p->n < 1 || p->n > 14) return 0;
    if (p->stencil != ORC_AXIS && p->stencil != ORC_RADIAL && p->stencil != ORC_RADIAL_PRINTED) return 0;
    for (int f = 0; f < 2 * p->dim; ++f)
        if (p->face[f] != ORC_DIRICHLET && p->face[f] != ORC_NEUMANN) return 0;
    if (!(p->theta > 0.0)) return 0;
    return 1;
}

static int ctx_init(ctx_t *x, const orc_problem *p, orc_stats *st)
{
    memset(x, 0, sizeof(*x));
    grid_init(&x->g, p);
    size_t bytes = sizeof(double) * (size_t)x->g.M;
    int n = x->g.n;
    x->tmp = malloc(bytes);
    x->u1 = malloc(bytes);
    x->delta = malloc(bytes);
    x->sig = calloc((size_t)n, sizeof(double *));
    x->pyr = calloc((size_t)n, sizeof(double *));
    if (!x->tmp || !x->u1 || !x->delta || !x->sig || !x->pyr) return 0;
    /* restricted coefficients: Algorithm 1 applied to sigma (Sec. 2,
     * "restricted sources and coefficients"), once per solve */
    x->sig[0] = (double *)p->sigma;
    for (int l = 1; l < n; ++l) {
        x->pyr[l] = malloc(bytes);
        if (!x->pyr[l]) return 0;
        if (p->sigma) {
            x->sig[l] = malloc(bytes);
            if (!x->sig[l]) return 0;
            restriction(&x->g, p->sigma, x->sig[l], l, x->tmp, st);
        }
    }
    return 1;
}

/* Algorithm 3: one saw-like refining cycle from e = 0 with source src.
 * Each visit calls restriction(nu) on src (Algorithm 1); src does not change
 * inside a cycle, so a level's result is kept after its first call.
 * pres_out (optional, one entry per visit) receives the pseudo-residual of
 * the last relaxation of each visit; trace (optional, one N^d block per
 * visit) receives e after each visit. */
static void cycle_run(ctx_t *x, const double *src, const double *G, double *e, const orc_opts *o,
                      double *pres_out, double *trace, orc_stats *st)
{
    grid_t *g = &x->g;
    int n = g->n;
    int have[32] = {0};
    x->pyr[0] = (double *)src;
    have[0] = 1;
    int cap = 4 * n + 8;
    int *lev = malloc(sizeof(int) * cap), *cnt = malloc(sizeof(int) * cap);
    int len = orc_schedule(n, o->n_r, o->reading, lev, cnt, cap);
    memset(e, 0, sizeof(double) * (size_t)g->M);
    for (int v = 0; v < len; ++v) {
        int nu = lev[v];
        if (!have[nu]) {
            restriction(g, src, x->pyr[nu], nu, x->tmp, st);
            have[nu] = 1;
        }
        double pres = 0.0;
        for (int r = 0; r < cnt[v]; ++r) {
            memcpy(x->u1, e, sizeof(double) * (size_t)g->M);
            pres = relax_interp(g, nu, x->u1, e, x->pyr[nu], x->sig[nu], G, x->delta, st);
        }
        if (pres_out) pres_out[v] = pres;
        if (trace) memcpy(trace + (size_t)v * (size_t)g->M, e, sizeof(double) * (size_t)g->M);
    }
    free(lev);
    free(cnt);
    x->pyr[0] = NULL;
}

/* ------------------------------------------------------------ public API */

/* dL_1 applied on the full grid at unknown nodes; 0 at Dirichlet nodes. */
int orc_apply(const orc_problem *p, const double *u, double *out)
{
    if (!valid_problem(p) || !u || !out) return ORC_E_ARG;
    grid_t g;
    grid_init(&g, p);
#pragma omp parallel for schedule(static)
    for (long long id = 0; id < g.M; ++id) {
        int c[3];
        node_coords(&g, id, c);
        out[id] = is_dirichlet(&g, c) ? 0.0 : apply_op(&g, p->sigma, u, c, 1, NULL);
    }
    return ORC_OK;
}

/* Stride-2^nu operator at level-nu nodes with coefficient signu (NULL = 1);
 * other nodes get 0.  diag (optional) receives the diagonal magnitude D. */
int orc_apply_level(const orc_problem *p, int nu, const double *signu, const double *u, double *out,
                    double *diag)
{
    if (!valid_problem(p) || !u || !out || nu < 0 || nu >= p->n) return ORC_E_ARG;
    grid_t g;
    grid_init(&g, p);
    int lam = 1 << nu;
#pragma omp parallel for schedule(static)
    for (long long id = 0; id < g.M; ++id) {
        int c[3];
        node_coords(&g, id, c);
        double D = 0.0;
        out[id] = on_level(&g, c, lam) ? apply_op(&g, signu, u, c, lam, &D) : 0.0;
        if (diag) diag[id] = D;
    }
    return ORC_OK;
}

/* Algorithm 1: g_out = restriction(nu)(f) on the full grid. */
int orc_restriction(const orc_problem *p, const double *f, double *g_out, int nu)
{
    if (!valid_problem(p) || !f || !g_out || nu < 0 || nu >= p->n) return ORC_E_ARG;
    grid_t g;
    grid_init(&g, p);
    double *tmp = malloc(sizeof(double) * (size_t)g.M);
    if (!tmp) return ORC_E_ARG;
    restriction(&g, f, g_out, nu, tmp, NULL);
    free(tmp);
    return ORC_OK;
}

/* I_lam: out = multilinear interpolation of the level-nu values of delta. */
int orc_interp(const orc_problem *p, int nu, const double *delta, double *out)
{
    if (!valid_problem(p) || !delta || !out || nu < 0 || nu >= p->n) return ORC_E_ARG;
    grid_t g;
    grid_init(&g, p);
    int lam = 1 << nu;
#pragma omp parallel for schedule(static)
    for (long long id = 0; id < g.M; ++id) {
        int c[3];
        node_coords(&g, id, c);
        out[id] = interp_at(&g, delta, c, lam);
    }
    return ORC_OK;
}

/* One call of Algorithm 2 at level nu on state u (in place), with source
 * gnu and coefficient signu at that level.  Returns the pseudo-residual in
 * *pres (optional). */
int orc_relax_interp(const orc_problem *p, int nu, double *u, const double *gnu, const double *signu,
                     const double *G, double *pres)
{
    if (!valid_problem(p) || !u || !gnu || nu < 0 || nu >= p->n) return ORC_E_ARG;
    grid_t g;
    grid_init(&g, p);
    double *u1 = malloc(sizeof(double) * (size_t)g.M), *delta = malloc(sizeof(double) * (size_t)g.M);
    if (!u1 || !delta) {
        free(u1);
        free(delta);
        return ORC_E_ARG;
    }
    memcpy(u1, u, sizeof(double) * (size_t)g.M);
    double r = relax_interp(&g, nu, u1, u, gnu, signu, G, delta, NULL);
    if (pres) *pres = r;
    free(u1);
    free(delta);
    return ORC_OK;
}

/* One cycle (Algorithm 3) from zero with source src and Dirichlet values G
 * (NULL: homogeneous); e receives the cycle's solution.  pres_out: optional
 * per-visit pseudo-residuals; trace: optional per-visit copies of e. */
int orc_cycle(const orc_problem *p, const orc_opts *o, const double *src, const double *G, double *e,
              double *pres_out, double *trace, orc_stats *st)
{
    if (!valid_problem(p) || !o || !src || !e) return ORC_E_ARG;
    ctx_t x;
    if (!ctx_init(&x, p, st)) {
        ctx_free(&x);
        return ORC_E_ARG;
    }
    cycle_run(&x, src, G, e, o, pres_out, trace, st);
    ctx_free(&x);
    return ORC_OK;
}

/* Recurrence on accumulated residuals (Sec. 2): cycle i solves
 * dL(e_i) = r_i approximately, r_{i+1} = r_i - dL(e_i), u = sum e_i.
 * Cycle 0 carries the given Dirichlet values G; later cycles have
 * homogeneous conditions.  The residual is zero at Dirichlet nodes, which
 * carry no equation.  Stop test (Sec. 3.1): max-norm of the recursive
 * residual over the max-norm of the sources.  Reading: the sources are the
 * initial residual f - dL(u_init), u_init = G on Dirichlet nodes and 0
 * elsewhere, which is f itself for homogeneous conditions and stays defined
 * when f = 0 (a problem driven by its boundary values).
 * Failure statuses: DIVERGED (non-finite or growth above 1e3),
 * STAGNATED (less than a factor 2 over stall_window cycles), MAXCYCLES. */
int orc_solve(const orc_problem *p, const orc_opts *o, const double *f, const double *G, double *u,
              orc_stats *st)
{
    if (!valid_problem(p) || !o || !f || !u || !st || o->max_cycles < 1 || !(o->tol >= 0.0))
        return ORC_E_ARG;
    memset(st, 0, sizeof(*st));
    ctx_t x;
    if (!ctx_init(&x, p, st)) {
        ctx_free(&x);
        return ORC_E_ARG;
    }
    grid_t *g = &x.g;
    size_t bytes = sizeof(double) * (size_t)g->M;
    double *s = malloc(bytes), *e = malloc(bytes), *Le = malloc(bytes);
    if (!s || !e || !Le) {
        free(s);
        free(e);
        free(Le);
        ctx_free(&x);
        return ORC_E_ARG;
    }
    /* Pure Neumann problems (no Dirichlet face; Sec. 2, last paragraph, and
     * eq. (10)): the source must integrate to zero, so it is taken minus its
     * mean; the trapezoid rule is the discrete integral, its weights being
     * the ones that make W dL symmetric, so that a zero-mean source keeps the
     * recurrence away from the constant mode (the null space for a = 0).
     * Each cycle's correction is taken minus its mean before it is collected
     * (the solution keeps zero mean, which fixes the shift for a = 0 and is
     * the exact solution's mean otherwise), and the residual is re-projected
     * against rounding. */
    const int pure = !has_dirichlet_face(g);
    double *fp = malloc(bytes);
    if (!fp) {
        free(s);
        free(e);
        free(Le);
        ctx_free(&x);
        return ORC_E_ARG;
    }
    memcpy(fp, f, bytes);
    if (pure) remove_mean(g, fp);
    /* u_init and the normaliser */
    for (long long id = 0; id < g->M; ++id) {
        int c[3];
        node_coords(g, id, c);
        u[id] = (is_dirichlet(g, c) && G) ? G[id] : 0.0;
    }
    orc_apply(p, u, Le);
    double norm0 = 0.0;
    for (long long id = 0; id < g->M; ++id) {
        int c[3];
        node_coords(g, id, c);
        if (is_dirichlet(g, c)) {
            s[id] = 0.0;
        } else {
            s[id] = fp[id];
            double r = fabs(fp[id] - Le[id]);
            if (r > norm0) norm0 = r;
        }
    }
    st->norm0 = norm0;
    int status = ORC_E_MAXCYCLES;
    if (norm0 == 0.0) {
        status = ORC_OK; /* u_init already solves the problem */
    } else {
        memset(u, 0, bytes);
        for (int i = 0; i < o->max_cycles; ++i) {
            cycle_run(&x, s, i == 0 ? G : NULL, e, o, NULL, NULL, st);
            if (pure) remove_mean(g, e);
            orc_apply(p, e, Le);
            for (long long id = 0; id < g->M; ++id) {
                int c[3];
                node_coords(g, id, c);
                u[id] += e[id];
                s[id] = is_dirichlet(g, c) ? 0.0 : s[id] - Le[id];
            }
            if (pure) remove_mean(g, s);
            double rmax = 0.0;
            for (long long id = 0; id < g->M; ++id)
                if (!(fabs(s[id]) <= rmax)) rmax = fabs(s[id]); /* propagates NaN */
            double rel = rmax / norm0;
            st->cycles = i + 1;
            st->relres = rel;
            if (i < ORC_HIST) st->history[i] = rel;
            if (!isfinite(rel) || rel > 1e3) {
                status = ORC_E_DIVERGED;
                break;
            }
            if (rel <= o->tol) {
                status = ORC_OK;
                break;
            }
            const int win = o->stall_window == 0 ? 3 : o->stall_window;
            if (win > 0 && i >= win && i < ORC_HIST && rel > 0.5 * st->history[i - win]) {
                status = ORC_E_STAGNATED;
                break;
            }
        }
    }
    /* true residual of the collected solution */
    orc_apply(p, u, Le);
    double tmax = 0.0;
    for (long long id = 0; id < g->M; ++id) {
        int c[3];
        node_coords(g, id, c);
        if (!is_dirichlet(g, c)) {
            double r = fabs(fp[id] - Le[id]);
            if (!(r <= tmax)) tmax = r;
        }
    }
    st->relres_true = norm0 > 0.0 ? tmax / norm0 : tmax;
    st->status = status;
    free(fp);
    free(s);
    free(e);
    free(Le);
    ctx_free(&x);
    return status;
}

/* Adjoint solve: dL^T lam = g on the unknowns, lam = 0 on Dirichlet nodes.
 * Since W dL is symmetric, dL^T = W dL W^-1: lam = W mu where dL mu = W^-1 g
 * is solved by the recurrence of Sec. 2 (orc_solve) with homogeneous
 * conditions.  With Dirichlet faces only, W = 1 and this is the solve of g.
 * At least one face must be Dirichlet (the pure Neumann problem, solved on
 * zero-mean sources, is not covered). */
int orc_adjoint(const orc_problem *p, const orc_opts *o, const double *g, double *lam, orc_stats *st)
{
    if (!valid_problem(p) || !o || !g || !lam || !st) return ORC_E_ARG;
    grid_t gr;
    grid_init(&gr, p);
    if (!has_dirichlet_face(&gr)) return ORC_E_ARG; /* pure Neumann: not covered */
    double *gw = malloc(sizeof(double) * (size_t)gr.M);
    if (!gw) return ORC_E_ARG;
    for (long long id = 0; id < gr.M; ++id) {
        int c[3];
        node_coords(&gr, id, c);
        gw[id] = is_dirichlet(&gr, c) ? 0.0 : g[id] / trap_weight(&gr, c);
    }
    int rc = orc_solve(p, o, gw, NULL, lam, st);
    for (long long id = 0; id < gr.M; ++id) {
        int c[3];
        node_coords(&gr, id, c);
        lam[id] = is_dirichlet(&gr, c) ? 0.0 : lam[id] * trap_weight(&gr, c);
    }
    free(gw);
    return rc;
}

/* Gradient of a scalar loss with respect to the coefficient sigma, given the
 * solution u and the adjoint lam of dLoss/du (lam = 0 at Dirichlet nodes).
 * From dL(u; sigma) = f (implicit-function theorem):
 *   dLoss/dsigma_m = - sum_x lam_x d(dL u)_x / dsigma_m.
 * Each term C/h^2 w_k (sigma_s + sigma_x)/2 (u_s - u_x) of row x, with s the
 * node its neighbour k samples (an image across a Neumann face), depends on
 * sigma_s and sigma_x with derivative C/(2h^2) w_k (u_s - u_x) each; the sum
 * is taken literally, term by term, over the unknowns x. */
int orc_coeff_grad(const orc_problem *p, const double *u, const double *lam, double *grad)
{
    if (!valid_problem(p) || !u || !lam || !grad) return ORC_E_ARG;
    grid_t g;
    grid_init(&g, p);
    double scale = g.C / (2.0 * g.h * g.h);
    memset(grad, 0, sizeof(double) * (size_t)g.M);
    for (long long id = 0; id < g.M; ++id) {
        int c[3];
        node_coords(&g, id, c);
        if (is_dirichlet(&g, c)) continue;
        for (int k = 0; k < g.K; ++k) {
            int si = mirror(c[0] + g.off[k][0], g.N);
            int sj = mirror(c[1] + g.off[k][1], g.N);
            int sk = (g.dim == 3) ? mirror(c[2] + g.off[k][2], g.N) : 0;
            long long sid = node_index(&g, si, sj, sk);
            double d = -lam[id] * scale * g.w[k] * (u[sid] - u[id]);
            grad[sid] += d;
            grad[id] += d;
        }
    }
    return ORC_OK;
}

/* Neumann data (Sec. 2: the derivative is imposed at the boundary by
 * substituting the data lying outside the domain).  flux[f] (NULL: zero)
 * holds the outward normal derivative on Neumann face f (x-, x+, y-, y+,
 * z-, z+) at its N^(d-1) nodes, indexed by the face's other coordinates in
 * axis order, the lower axis fastest (x- / x+: (k N + j), y- / y+: (k N + i),
 * z- / z+: (j N + i); 2D: j or i).  A neighbour sample that crosses a Neumann
 * face takes the image node's value plus 2 h g at the face point (the
 * central difference across the face), one such term for every face it
 * crosses, g read at the image's other coordinates.  These terms do not
 * depend on u: they are the affine part b of dL_1 at the unknowns, moved to
 * the source, f_out = f - b, so that the solve with homogeneous images
 * (Algorithms 1-3 unchanged) solves the problem with the Neumann data.
 * Values at Dirichlet nodes are copied. */
int orc_neumann_source(const orc_problem *p, const double *const flux[6], const double *f, double *f_out)
{
    if (!valid_problem(p) || !flux || !f || !f_out) return ORC_E_ARG;
    grid_t g;
    grid_init(&g, p);
    double scale = g.C / (g.h * g.h);
    for (long long id = 0; id < g.M; ++id) {
        int c[3];
        node_coords(&g, id, c);
        f_out[id] = f[id];
        if (is_dirichlet(&g, c)) continue;
        double sc = p->sigma ? p->sigma[id] : 1.0;
        double b = 0.0;
        for (int k = 0; k < g.K; ++k) {
            int q[3] = {c[0] + g.off[k][0], c[1] + g.off[k][1], c[2] + g.off[k][2]};
            int s3[3] = {mirror(q[0], g.N), mirror(q[1], g.N), g.dim == 3 ? mirror(q[2], g.N) : 0};
            double shift = 0.0;
            for (int ax = 0; ax < g.dim; ++ax) {
                int face = q[ax] < 0 ? 2 * ax : (q[ax] > g.N - 1 ? 2 * ax + 1 : -1);
                if (face < 0 || g.face[face] != ORC_NEUMANN || !flux[face]) continue;
                int t[2], nt = 0;
                for (int bx = 0; bx < g.dim; ++bx)
                    if (bx != ax) t[nt++] = s3[bx];
                long long fi = nt == 2 ? (long long)t[1] * g.N + t[0] : t[0];
                shift += 2.0 * g.h * flux[face][fi];
            }
            if (shift == 0.0) continue;
            long long sid = node_index(&g, s3[0], s3[1], s3[2]);
            double ss = p->sigma ? p->sigma[sid] : 1.0;
            b += g.w[k] * 0.5 * (ss + sc) * shift;
        }
        f_out[id] = f[id] - scale * b;
    }
    return ORC_OK;
}

/* Node kinds: 1 for Dirichlet nodes, 0 for unknowns. */
int orc_dirichlet_mask(const orc_problem *p, uint8_t *mask)
{
    if (!valid_problem(p) || !mask) return ORC_E_ARG;
    grid_t g;
    grid_init(&g, p);
    for (long long id = 0; id < g.M; ++id) {
        int c[3];
        node_coords(&g, id, c);
        mask[id] = (uint8_t)is_dirichlet(&g, c);
    }
    return ORC_OK;
}

int orc_hist_cap(void) { return ORC_HIST; }

/* Threads the parallel loops use (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
#else
int orc_threads(void) { return 1; }
#endif
