// sgml_internal.h -- shared declarations of the SGML HIP library (not part
// of the public C-ABI, which is include/sgml.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sgml {

// Devices a process may drive (per-device state of the library is kept in
// arrays of this size).
constexpr int kMaxDevices = 64;

// Compute units of the current device (queried once per device; 0 when the
// query fails).
int device_cus();

// Geometry and operator constants of one level of the nested grid
// (Sec. 2: level nu holds the nodes whose indices are multiples of
// lam = 2^nu; stored compactly as m^d values, m = 2^(n-nu) + 1).
struct Level {
    int m;            // nodes per axis on this level
    int lam;          // stride of the level on the full grid
    int N;            // nodes per axis of the full grid
    unsigned dir;     // bit f set when face f (x-, x+, y-, y+, z-, z+) is Dirichlet
    double scale;     // C / (lam h)^2 of the stencil
    double a;         // constant term of L
    double theta;     // dtau = theta / D
};

// A max-reduction target: kRedSlots partial maxima, kRedStride u64 apart
// (one 128-byte line each), so that the per-block atomics of a large grid
// spread over many L2 lines instead of serialising on one address.  The
// host takes the max of the slots.
constexpr int kRedSlots = 64;
constexpr int kRedStride = 16;
constexpr int kRedWords = kRedSlots * kRedStride;

// Which kernel variant: dimension, stencil, heterogeneous coefficient.
struct Variant {
    int dim;          // 2 or 3
    int radial;       // 0 axis stencil, 1 radial stencil
    int sigma;        // 0: sigma = 1, 1: coefficient array
};

// One operation of a coarse-level run executed by k_coarse.
enum { kOpFill = 0, kOpSweep = 1, kOpProlong = 2, kOpInject = 3, kOpRestrict = 4 };
struct CoarseOp {
    int kind;         // kOp*
    int m;            // nodes per axis of the level written
    int level;        // sweeps: index into the level table
    int first;        // prolongation: the finer level's stale values are zero
    int target;       // sweeps: reduction target of the pseudo-residual, -1 for none
    int pad;
    const void *in0;  // sweep: e in; prolong: coarse e; inject / restrict: finer level
    const void *in1;  // sweep: source g; prolong: stale finer e
    const void *in2;  // sweep: coefficient (or null)
    void *out;
};
// threads of the coarse-level workgroup: 16 waves in 2D; 8 in 3D, where the
// 27-point stencil needs more than the 128 registers a 16-wave group allows
constexpr int coarse_threads(int dim) { return dim == 3 ? 512 : 1024; }

// The same run with its level arrays staged in LDS (k_coarse_lds): operands
// are element offsets into the workgroup's LDS; the coefficient and the
// Dirichlet values stay in global memory.  The largest level a run may touch
// has coarse_lds_nodes() nodes (a fixed number per thread).
constexpr int coarse_lds_nodes(int dim) { return dim == 3 ? 5120 : 5120; }
// k_coarse_lds decodes a node index t into (i, j, k) with one float multiply
// by 1/m, exact while t < 2^13 (t + 1/2 stays 1/(2m) away from a multiple of m)
static_assert(coarse_lds_nodes(2) < (1 << 13) && coarse_lds_nodes(3) < (1 << 13),
              "the coarse kernel's float index decode needs levels below 2^13 nodes");
struct LdsOp {
    int kind;         // kOp*
    int m;            // nodes per axis of the level written
    int first;        // prolongation: the finer level's stale values are zero
    int target;       // sweeps: reduction target of the pseudo-residual, -1 for none
    int in0, in1;     // element offsets of the operands (as CoarseOp::in0 / in1)
    int out;          // element offset of the result
    int nodes;        // m^d
    float inv_m;      // 1 / m in float
    int solo;         // run by wavefront 0 alone (a small level, no reduction target)
    int sync;         // a workgroup barrier follows (every operation but a solo one before another)
    int pad;
    const void *sig;  // sweeps: level coefficient (global memory) or null
    Level L;          // sweeps: constants of the level
    // sweeps: the relaxation's constants in the cycle's precision, computed
    // once on the host (index kK*): level scale, a, theta, theta / D with the
    // sigma = 1 diagonal D, 1 - theta, theta scale / D, a - 4 scale
    float kf[8];
    double kd[8];
};
enum { kKScale = 0, kKA, kKTheta, kKStep, kKOmt, kKBeta, kKAw };
// An operation as the LDS run keeps it in LDS: the fields its control flow
// and arithmetic use, the constants in the cycle's precision.
template <typename T>
struct LdsOpHdr {
    int kind, m, nodes, target, solo, sync, in0, in1, out, first, lam, N;
    unsigned dir;
    float inv_m;
    const void *sig;
    T k[8];
};
// A copy between global memory and the LDS image before (loads) or after
// (stores) the run.
struct LdsXfer {
    void *ptr;
    int off, count;   // LDS element offset, elements
};

// A fused visit of a 2D level: optional interpolation of the next coarser
// level's pending variation (prologue), `sweeps` relaxations, optional
// injection of the result into the next coarser level (epilogue).
constexpr int kMaxFusedSweeps = 6;
struct VisitArgs {
    const void *estale;   // level values before the visit (stale finer copy when interpolating)
    const void *ecoarse;  // interpolation: values of the next coarser level
    const void *g;        // source of the level
    const void *sig;      // coefficient of the level (or null)
    const double *G;      // Dirichlet values (full grid) or null
    void *eout;           // values after the visit
    void *einj;           // injection target (next coarser level) or null
    unsigned long long *targets;
    Level L;
    int first;            // interpolation: the stale values are zero
    int sweeps;           // 1 .. kMaxFusedSweeps
    int prolong, inject;  // prologue / epilogue present
    int pres[kMaxFusedSweeps];  // reduction target per relaxation, -1 for none
    int chunk;            // rows per wavefront
};
bool fused_visit_supported(int sweeps);

// The cycle-end pass on a 2D level 0 (see k_boundary for the general form).
struct CycleEndArgs {
    const void *e;        // level-0 values of the cycle, in the cycle's precision
    double escale;        // e = escale * E
    const double *G;      // Dirichlet values (first cycle) or null
    const double *sigma;  // coefficient (FP64, full grid) or null
    double *u, *s;        // collected solution and recursive residual
    double *s_out;        // the new residual, when not written in place (RES: s is read at halo nodes)
    void *shat;           // next cycle's source in the cycle's precision (mixed) or null
    double shat_scale;
    unsigned long long *norm;  // reduction target of max |s|
    void *g1;             // 2D: next cycle's level-1 source (restriction of the new source) or null
    Level L;
    int chunk;            // rows per wavefront (2D)
    int zchunk;           // planes per workgroup (3D z-marching), 0: chosen per level
};

// Precision-generic launchers (T = double or float); all enqueue on `st`.
template <typename T>
void launch_fill(T *p, size_t count, T value, hipStream_t st);

template <typename T>
void launch_sweep(const Variant &v, const Level &L, const T *ein, T *eout, const T *g, const T *sig,
                  const double *G, unsigned long long *pres, hipStream_t st);

template <typename T>
void launch_coarse(const Variant &v, const CoarseOp *ops, int nops, const Level *levels, const double *G,
                   unsigned long long *targets, hipStream_t st);

// `lds_bytes` covers the level arrays and, from byte hdr_off on, the nops
// operation headers (LdsOpHdr<T>).  Returns false when the launch cannot get
// that much LDS.
template <typename T>
bool launch_coarse_lds(const Variant &v, const LdsOp *ops, int nops, int hdr_off, const LdsXfer *xfer, int nload,
                       int nstore, size_t lds_bytes, const double *G, unsigned long long *targets, hipStream_t st);

template <typename T>
void launch_visit2d(const Variant &v, const VisitArgs &a, hipStream_t st);

// The closing visit of a 2D level 0 (interpolation, sweeps relaxations, no
// injection, not the level's first visit of the cycle) fused with the cycle
// end (FP32 cycles after the first, constant coefficient, the level-1
// restriction written: c.g1 and c.s_out set).
template <typename T>
void launch_visit_end2d(const Variant &v, const VisitArgs &a, const CycleEndArgs &c, hipStream_t st);
bool visit_end_supported(int sweeps, int m, bool any_size);  // m: nodes per axis of level 0

// One restriction step (Algorithm 1) of a 2D level of mc >= 65 coarse nodes
// per axis, row-marching.
template <typename T>
void launch_restrict2d(int mc, const T *fine, T *coarse, hipStream_t st);
// Two restriction steps in one pass: fine -> coarse (mc >= 65 nodes per axis)
// -> coarse2 ((mc + 1) / 2 nodes per axis).
template <typename T>
void launch_restrict2d2(int mc, const T *fine, T *coarse, T *coarse2, hipStream_t st);

template <typename T>
void launch_cycle_end2d(const Variant &v, const CycleEndArgs &a, hipStream_t st);

// One relaxation / the cycle-end pass of a 3D level (m >= 33) marching in z
// through LDS planes.
bool sweep3d_supported(int m);
template <typename T>
void launch_cycle_end3d(const Variant &v, const CycleEndArgs &a, hipStream_t st);
// `zreq` (here and below): planes each workgroup marches, 0 = chosen per level.
template <typename T>
void launch_sweep3d(const Variant &v, const Level &L, const T *ein, T *eout, const T *g, const T *sig,
                    const double *G, unsigned long long *pres, int zreq, hipStream_t st);
// Two chained relaxations of a 3D level with sigma = 1 (m >= 33) in one
// z-marching pass: ein -> (relaxation) -> (relaxation) -> eout.
template <typename T>
void launch_sweep3d2(const Variant &v, const Level &L, const T *ein, T *eout, const T *g, const double *G,
                     unsigned long long *pres, int zreq, hipStream_t st);

template <typename T>
void launch_prolong(int dim, int mc, const T *ec, const T *ef_in, T *ef_out, bool first,
                    hipStream_t st);
// The same interpolation into a 3D level of m = 2 mc - 1 >= 33 nodes per
// axis, marching in z with the pending variation staged in LDS.
template <typename T>
void launch_prolong3d(int mc, const T *ec, const T *ef_in, T *ef_out, bool first, int zreq, hipStream_t st);

template <typename T>
void launch_inject(int dim, int mc, const T *ef, T *ec, hipStream_t st);

template <typename Tin, typename Tout>
void launch_restrict(int dim, int mc, const Tin *fine, Tout *coarse, hipStream_t st);
// The same step from a 3D level of 2 mc - 1 >= 33 nodes per axis, marching in z.
template <typename T>
void launch_restrict3d(int mc, const T *fine, T *coarse, int zreq, hipStream_t st);

template <typename Tin, typename Tout>
void launch_convert(const Tin *in, Tout *out, size_t count, hipStream_t st);

// FP64 work on the full grid (level 0).
template <typename T>
void launch_boundary(const Variant &v, const Level &L, const T *e, double escale, const double *G,
                     const double *sigma, double *u, double *s, T *shat, double shat_scale,
                     unsigned long long *norm, hipStream_t st);

// wscale: the source is W^-1 f, W the trapezoid weights (1/2 per Neumann
// face a node lies on), as the transposed solve needs.  s32 (or null): the
// source also in FP32, unscaled (the mixed cycle's source when it needs no
// scaling).
void launch_init(const Variant &v, const Level &L, const double *f, const double *G,
                 const double *sigma, double *s, double *u, float *s32, unsigned long long *norm0,
                 bool wscale, hipStream_t st);
// u = W u at every node.
void launch_trap_scale(const Level &L, int dim, double *u, hipStream_t st);

// Pure Neumann problems: *mean = scale * (trapezoid mean of v), summed in a
// fixed order through `partial` (wsum_partials(dim, m) doubles); then
// s -= *mean_s, u -= *mean_e (mean_e may be null), shat = s * shat_scale (shat
// may be null) and norm = max |s|.
size_t wsum_partials(int dim, int m);
template <typename T>
void launch_wmean(int dim, const Level &L, const T *v, double scale, double *partial, double *mean,
                  hipStream_t st);
template <typename T>
void launch_project(int dim, const Level &L, double *s, double *u, const double *mean_s, const double *mean_e,
                    T *shat, double shat_scale, unsigned long long *norm, hipStream_t st);

// Neumann data per face (outward normal derivative, N^(d-1) values each, or
// null for zero), moved to the source: out = f - (flux part of dL_1).
struct FaceData {
    const double *g[6];
};
void launch_neumann_source(const Variant &v, const Level &L, const double *f, const FaceData &flux,
                           const double *sigma, double h, double *out, hipStream_t st);

template <typename T>
void launch_source_cast(const Level &L, int dim, const double *s, T *shat, double scale,
                        hipStream_t st);

void launch_set_dirichlet(const Level &L, int dim, const double *G, double *u, hipStream_t st);

void launch_residual(const Variant &v, const Level &L, const double *f, const double *G,
                     const double *sigma, const double *u, double *r, unsigned long long *rmax,
                     unsigned long long *norm0, hipStream_t st);

void launch_coeff_grad(const Variant &v, const Level &L, const double *u, const double *lam,
                       double *grad, hipStream_t st);

}  // namespace sgml
