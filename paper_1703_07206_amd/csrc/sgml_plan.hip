// sgml_plan.hip -- host side of the SGML library: the C-ABI of
// include/sgml.h, the workspace layout, the visit schedule (Algorithm 3) and
// the residual recurrence with its stop test (Sec. 2, Sec. 3.1).
#include "sgml.h"
#include "sgml_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

using namespace sgml;

namespace {

constexpr int kMaxLevels = 16;
constexpr size_t kAlign = 256;
// reduction targets: [0] residual norm, [1] norm0, [2] rmax, [kPres + v] pseudo-residual of visit v
constexpr int kPres = 4;
constexpr int kTargets = kPres + SGML_MAX_VISITS;
constexpr size_t kScalars = (size_t)kTargets * kRedWords;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

constexpr int kMaxCoarseOps = 4096;
constexpr int kMaxXfers = 2048;
// Default coarse runs: 2D levels up to 33^2 (the 65^2 level's fused visits are
// faster than its operations in the single workgroup: 4097^2 solve -2%, 129^2
// solve -10%), 3D levels up to 17^3.
constexpr int kDefaultCoarseNodes2 = 1100, kDefaultCoarseNodes3 = 5000;
constexpr int kDefaultFuseMin = 65;  // smallest 2D level (nodes per axis) visited in one fused pass

struct Layout {
    size_t scal, ops, lops, xfer, levels, s, s2, e0, shat, sig0t, part, means;
    size_t e[kMaxLevels][2], g[kMaxLevels], sig64[kMaxLevels], sigt[kMaxLevels];
    size_t total;
};

bool valid_problem(const sgml_problem *p)
{
    if (!p) return false;
    if (p->dim != 2 && p->dim != 3) return false;
    if (p->stencil != SGML_AXIS && p->stencil != SGML_RADIAL) return false;
    for (int f = 0; f < 2 * p->dim; ++f)
        if (p->face[f] != SGML_DIRICHLET && p->face[f] != SGML_NEUMANN) return false;
    if (!std::isfinite(p->a) || !std::isfinite(p->theta)) return false;
    return true;
}

bool valid_shape(const sgml_problem *p)
{
    return p->n >= 2 && p->n <= (p->dim == 2 ? 13 : 10);
}

size_t level_nodes(int dim, int n, int nu)
{
    size_t m = ((size_t)1 << (n - nu)) + 1;
    return dim == 3 ? m * m * m : m * m;
}

Layout make_layout(const sgml_problem *p, int precision)
{
    Layout L;
    std::memset(&L, 0, sizeof(L));
    const bool mixed = precision == SGML_MIXED;
    const size_t M = level_nodes(p->dim, p->n, 0);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.scal = take(sizeof(unsigned long long) * kScalars);
    L.ops = take(sizeof(CoarseOp) * kMaxCoarseOps);
    L.lops = take(sizeof(LdsOp) * kMaxCoarseOps);
    L.xfer = take(sizeof(LdsXfer) * kMaxXfers);
    L.levels = take(sizeof(Level) * kMaxLevels);
    // trapezoid-mean partial sums and the two means of a pure Neumann solve
    L.part = take(sizeof(double) * wsum_partials(p->dim, (1 << p->n) + 1));
    L.means = take(sizeof(double) * 2);
    L.s = take(8 * M);
    L.e0 = take(2 * 8 * M);  // two level-0 buffers, FP64-sized (FP32 uses half)
    L.shat = mixed ? take(4 * M) : 0;
    L.s2 = mixed ? take(8 * M) : 0;  // second residual buffer (2D mixed cycle end)
    L.sig0t = mixed ? take(4 * M) : 0;
    for (int nu = 1; nu < p->n; ++nu) {
        const size_t c = level_nodes(p->dim, p->n, nu);
        L.e[nu][0] = take(8 * c);
        L.e[nu][1] = take(8 * c);
        L.g[nu] = take(8 * c);
        L.sig64[nu] = take(8 * c);
        L.sigt[nu] = mixed ? take(4 * c) : 0;
    }
    L.total = off;
    return L;
}

// Algorithm 3 as a visit list.  Tooth nu1 = n-1 .. 0 visits nu1, nu1 - 1
// (not below 0) and nu1 again, each min(n_r, 2^(n - nu1)) times; the
// algorithm's closing level-0 relaxations (min(n_r, 2^n) times) end the
// cycle once (SGML_SCHEDULE_ONCE) or every tooth (SGML_SCHEDULE_EACH).
void build_schedule(int n, int n_r, int sched, std::vector<int> &lev, std::vector<int> &cnt)
{
    lev.clear();
    cnt.clear();
    auto cap = [&](long long full) { return (int)((n_r > 0 && n_r < full) ? n_r : full); };
    for (int nu1 = n - 1; nu1 >= 0; --nu1) {
        const int c = cap(1LL << (n - nu1));
        const int tooth[3] = {nu1, nu1 - 1, nu1};
        for (int t = 0; t < 3; ++t) {
            if (tooth[t] < 0) continue;
            lev.push_back(tooth[t]);
            cnt.push_back(c);
        }
        if (sched == SGML_SCHEDULE_EACH) {
            lev.push_back(0);
            cnt.push_back(cap(1LL << n));
        }
    }
    if (sched != SGML_SCHEDULE_EACH) {
        lev.push_back(0);
        cnt.push_back(cap(1LL << n));
    }
}

double default_theta(int dim, int stencil)
{
    if (stencil == SGML_RADIAL) return 1.0;
    return dim == 2 ? 0.8 : 6.0 / 7.0;
}

// A run of consecutive coarse operations, launched as one workgroup.
struct RunDesc {
    int op0, nops;             // range of the device CoarseOp list (k_coarse)
    int lds;                   // staged in LDS (k_coarse_lds)
    int lop0, x0, nload, nstore;
    size_t lds_bytes;
    int hdr_off;               // LDS byte offset of the staged operation headers
};

}  // namespace

struct sgml_plan {
    sgml_problem prob;
    int precision;
    int dim, n, N;
    size_t M;
    double h, C, theta;
    unsigned dir;
    Variant var;
    char *ws;
    size_t ws_bytes;
    Layout lay;
    const double *sigma;
    int device;
    unsigned long long *host;  // pinned copy of the reduction targets (kScalars words)
    hipEvent_t ev0, ev1;
    std::vector<hipEvent_t> pev;  // profiling events, pairs around timed launches
    size_t pev_used = 0;
    int prof_untimed = 0;         // launches of the current solve the pool could not time
    CoarseOp *ops_host;           // pinned staging of the coarse operation list
    LdsOp *lops_host;             // ... and of its LDS form
    LdsXfer *xfer_host;
    Level *levels_host;           // pinned staging of the level table
    size_t lds_max;               // LDS bytes one workgroup may allocate
    std::vector<RunDesc> runs;        // the coarse runs of the compiled cycle, in order
    // batches of right-hand sides: the plans of right-hand sides 1 .. nrhs-1
    // (each with its own slice of the workspace and its own stream, forked
    // from and joined to the caller's stream by events); their coefficient
    // pyramid is the first plan's (sig_ws)
    char *sig_ws = nullptr;
    // cycles replayed as graphs: the executable graph of a cycle (two, for the
    // two parities of a double-buffered residual), valid for the key it was
    // captured with; captured on a private stream
    struct CycleGraph {
        bool valid = false;
        std::vector<long long> key;
        hipGraphExec_t exec = nullptr;
    } graph[2];
    hipStream_t cap_st = nullptr;
    bool graphs_broken = false;  // a capture failed once: eager from then on
    std::vector<sgml_plan *> sub;
    std::vector<hipStream_t> sub_st;
    std::vector<hipEvent_t> sub_ev;  // fork, join per extra right-hand side

    template <typename T>
    T *at(size_t off) const
    {
        return reinterpret_cast<T *>(ws + off);
    }
    template <typename T>
    T *sig_at(size_t off) const
    {
        return reinterpret_cast<T *>((sig_ws ? sig_ws : ws) + off);
    }
    int m(int nu) const { return (1 << (n - nu)) + 1; }
    Level level(int nu) const
    {
        Level L;
        L.m = m(nu);
        L.lam = 1 << nu;
        L.N = N;
        L.dir = dir;
        const double lh = L.lam * h;
        L.scale = C / (lh * lh);
        L.a = prob.a;
        L.theta = theta;
        return L;
    }
};

#define SGML_HIP(call)                                  \
    do {                                                \
        if ((call) != hipSuccess) return SGML_E_HIP;    \
    } while (0)

namespace {

unsigned long long *target(sgml_plan *P, int t)
{
    return P->at<unsigned long long>(P->lay.scal) + (size_t)t * kRedWords;
}

// Copy reduction targets [first, first + count) to the pinned host block:
// enqueued only (fetch_async), or enqueued and waited for (fetch).
sgml_status fetch_async(sgml_plan *P, int first, int count, hipStream_t st)
{
    SGML_HIP(hipMemcpyAsync(P->host + (size_t)first * kRedWords, target(P, first),
                            sizeof(unsigned long long) * kRedWords * count, hipMemcpyDeviceToHost, st));
    return SGML_OK;
}

sgml_status fetch(sgml_plan *P, int first, int count, hipStream_t st)
{
    sgml_status rc = fetch_async(P, first, count, st);
    if (rc != SGML_OK) return rc;
    SGML_HIP(hipStreamSynchronize(st));
    return SGML_OK;
}

void clear_targets(sgml_plan *P, int first, int count, hipStream_t st)
{
    launch_fill<unsigned long long>(target(P, first), (size_t)kRedWords * count, 0ull, st);
}

double as_double(unsigned long long b);

// max over the slots of a fetched target
double host_max(const sgml_plan *P, int t)
{
    unsigned long long m = 0;
    for (int s = 0; s < kRedSlots; ++s) {
        const unsigned long long v = P->host[(size_t)t * kRedWords + (size_t)s * kRedStride];
        m = v > m ? v : m;
    }
    return as_double(m);
}

// Profiling: a pair of events around a launch; drained once per cycle.  The
// pool has a fixed size, created in full before the first profiled solve
// enqueues anything and never grown: a cycle times at most kProfPairs
// launches, the rest run untimed (counted in the stats).
constexpr int kProfPairs = 32;

sgml_status prof_pool(sgml_plan *P)
{
    while (P->pev.size() < 2 * (size_t)kProfPairs) {
        hipEvent_t e;
        // timing only: no system-scope fence (no cache writeback) at each record
        SGML_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        P->pev.push_back(e);
    }
    return SGML_OK;
}

// Index of the next free pair's first event in P->pev, or -1 when the pool
// is used up for this cycle.
long prof_pair(sgml_plan *P)
{
    if (P->pev_used + 2 > P->pev.size()) {
        ++P->prof_untimed;
        return -1;
    }
    const long pr = (long)P->pev_used;
    P->pev_used += 2;
    return pr;
}

double as_double(unsigned long long b)
{
    double d;
    std::memcpy(&d, &b, sizeof(d));
    return d;
}

// A launch timed with a pair of events (profiling): P->pev[ev], P->pev[ev + 1].
struct Timed {
    int cls, sweeps;
    long ev;
};

// A cycle compiled to a list of operations (the same list every cycle).
constexpr int kOpVisit = 5;   // fused visit of a 2D level (host-side operation)
constexpr int kOpSweep2 = 6;  // two relaxations of a 3D level in one pass (host-side operation)

struct HostOp {
    CoarseOp op;
    bool coarse;     // runs inside the one-workgroup coarse kernel
    VisitArgs visit;  // kOpVisit
};

// Compile one cycle of Algorithm 3 from e = 0 on the level-0 source src0, in
// T: the restriction pyramid of the source (Algorithm 1), then every visit
// with the level transitions it needs.  Returns the level-0 buffer that holds
// the cycle's e at the end.
template <typename T>
const T *compile_cycle(sgml_plan *P, const T *src0, const std::vector<int> &lev, const std::vector<int> &cnt,
                       bool record, int coarse_level, int fuse_min, bool restrict1_outside, std::vector<HostOp> &ops,
                       long long &updates_per_cycle)
{
    const int n = P->n;
    const bool mixed = sizeof(T) == 4;
    T *E[kMaxLevels][2];
    const T *g[kMaxLevels];
    const T *sig[kMaxLevels];
    E[0][0] = P->at<T>(P->lay.e0);
    E[0][1] = E[0][0] + P->M;
    g[0] = src0;
    sig[0] = P->var.sigma ? (mixed ? (const T *)P->sig_at<T>(P->lay.sig0t) : (const T *)P->sigma) : nullptr;
    ops.clear();
    updates_per_cycle = 0;
    auto push = [&](int kind, int level, int first, int target, const void *in0, const void *in1,
                    const void *in2, void *out, bool coarse) {
        HostOp h;
        std::memset(&h, 0, sizeof(h));
        h.op.kind = kind;
        h.op.m = P->m(level);
        h.op.level = level;
        h.op.first = first;
        h.op.target = target;
        h.op.in0 = in0;
        h.op.in1 = in1;
        h.op.in2 = in2;
        h.op.out = out;
        h.coarse = coarse;
        ops.push_back(h);
    };
    // visits of large 2D levels run as fused passes
    auto fusable = [&](int nu) {
        return fuse_min > 0 && P->dim == 2 && nu < coarse_level && P->m(nu) >= fuse_min;
    };
    auto pairable3d = [&](int nu) {
        return fuse_min > 0 && P->dim == 3 && nu < coarse_level && sweep3d_supported(P->m(nu)) && !P->var.sigma;
    };
    for (int nu = 1; nu < n; ++nu) {
        E[nu][0] = P->at<T>(P->lay.e[nu][0]);
        E[nu][1] = P->at<T>(P->lay.e[nu][1]);
        T *gn = P->at<T>(P->lay.g[nu]);
        g[nu] = gn;
        sig[nu] = P->var.sigma ? (mixed ? (const T *)P->sig_at<T>(P->lay.sigt[nu])
                                        : (const T *)P->sig_at<T>(P->lay.sig64[nu]))
                               : nullptr;
        // restriction(nu) of the cycle source (Algorithm 1), kept for the cycle;
        // the first step may come with the source (restrict1_outside)
        if (nu > 1 || !restrict1_outside)
            push(kOpRestrict, nu, 0, -1, g[nu - 1], nullptr, nullptr, gn, nu - 1 >= coarse_level);
    }
    int cur[kMaxLevels] = {0};
    bool seen[kMaxLevels] = {false};
    int prev = -1;
    for (size_t v = 0; v < lev.size(); ++v) {
        const int nu = lev[v];
        if (prev < 0) push(kOpFill, nu, 0, -1, nullptr, nullptr, nullptr, E[nu][cur[nu]], nu >= coarse_level);
        // walk one level at a time: refining interpolates the pending
        // variation into the finer level, coarsening copies the finer values
        while (prev > nu) {
            const int f = prev - 1;
            push(kOpProlong, f, !seen[f], -1, E[prev][cur[prev]], E[f][cur[f]], nullptr, E[f][cur[f] ^ 1],
                 f >= coarse_level);
            cur[f] ^= 1;
            seen[f] = true;
            prev = f;
        }
        while (prev >= 0 && prev < nu) {
            const int c = prev + 1;
            HostOp *last = ops.empty() ? nullptr : &ops.back();
            if (last && last->op.kind == kOpVisit && last->op.level == prev && !last->visit.inject) {
                // injection as the epilogue of the fused visit; it writes the
                // other buffer of level c, whose current one the visit reads
                last->visit.inject = 1;
                last->visit.einj = E[c][cur[c] ^ 1];
                cur[c] ^= 1;
            } else {
                push(kOpInject, c, 0, -1, E[prev][cur[prev]], nullptr, nullptr, E[c][cur[c]],
                     prev >= coarse_level);
            }
            seen[c] = true;
            prev = c;
        }
        seen[nu] = true;
        updates_per_cycle += (long long)cnt[v] * (long long)level_nodes(P->dim, n, nu);
        const int tgt_last = record ? kPres + (int)v : -1;
        if (!fusable(nu)) {
            for (int r = 0; r < cnt[v];) {
                // pairs of relaxations of a large 3D level in one pass (sigma = 1);
                // the pass writes the other buffer, as one relaxation does
                const bool pair = pairable3d(nu) && r + 1 < cnt[v];
                push(pair ? kOpSweep2 : kOpSweep, nu, 0, r + (pair ? 1 : 0) == cnt[v] - 1 ? tgt_last : -1,
                     E[nu][cur[nu]], g[nu], sig[nu], E[nu][cur[nu] ^ 1], nu >= coarse_level);
                cur[nu] ^= 1;
                r += pair ? 2 : 1;
            }
            prev = nu;
            continue;
        }
        int left = cnt[v];
        // continue the previous fused visit of this level when nothing came between
        HostOp *last = ops.empty() ? nullptr : &ops.back();
        if (last && last->op.kind == kOpVisit && last->op.level == nu && !last->visit.inject &&
            fused_visit_supported(last->visit.sweeps + left)) {
            last->visit.pres[last->visit.sweeps + left - 1] = tgt_last;
            last->visit.sweeps += left;
            prev = nu;
            continue;
        }
        // a preceding interpolation into this level becomes the prologue
        bool pro = false;
        const void *ecoarse = nullptr, *estale = E[nu][cur[nu]];
        int first = 0;
        void *out0 = nullptr;
        if (last && last->op.kind == kOpProlong && last->op.level == nu) {
            pro = true;
            ecoarse = last->op.in0;
            estale = last->op.in1;
            first = last->op.first;
            out0 = last->op.out;  // cur[nu] already points at it
            ops.pop_back();
        }
        while (left > 0) {
            int s = kMaxFusedSweeps;
            while (s > left || !fused_visit_supported(s)) --s;
            HostOp h;
            std::memset(&h, 0, sizeof(h));
            h.op.kind = kOpVisit;
            h.op.level = nu;
            h.op.m = P->m(nu);
            VisitArgs &a = h.visit;
            a.estale = estale;
            a.ecoarse = ecoarse;
            a.g = g[nu];
            a.sig = sig[nu];
            a.first = first;
            a.sweeps = s;
            a.prolong = pro;
            a.inject = 0;
            for (int k = 0; k < kMaxFusedSweeps; ++k) a.pres[k] = -1;
            if (pro) {
                a.eout = out0;
            } else {
                a.eout = E[nu][cur[nu] ^ 1];
                cur[nu] ^= 1;
            }
            left -= s;
            if (left == 0) a.pres[s - 1] = tgt_last;
            ops.push_back(h);
            estale = a.eout;
            pro = false;
            first = 0;
        }
        prev = nu;
    }
    return E[0][cur[0]];
}

// Buffers an operation reads and writes (reads listed first), with their
// lengths.  Level coefficients are not listed: they stay in global memory.
struct Ref {
    const void *p;
    size_t count;
    bool write;
};

int op_refs(const sgml_plan *P, const HostOp &h, Ref r[6])
{
    const CoarseOp &o = h.op;
    int k = 0;
    auto ref = [&](const void *p, int nu, bool w) {
        if (p) r[k++] = {p, level_nodes(P->dim, P->n, nu), w};
    };
    switch (o.kind) {
    case kOpFill:
        ref(o.out, o.level, true);
        break;
    case kOpSweep:
    case kOpSweep2:
        ref(o.in0, o.level, false);
        ref(o.in1, o.level, false);
        ref(o.out, o.level, true);
        break;
    case kOpProlong:
        ref(o.in0, o.level + 1, false);
        if (!o.first) ref(o.in1, o.level, false);
        ref(o.out, o.level, true);
        break;
    case kOpInject:
    case kOpRestrict:
        ref(o.in0, o.level - 1, false);
        ref(o.out, o.level, true);
        break;
    case kOpVisit: {
        const VisitArgs &a = h.visit;
        ref(a.estale, o.level, false);
        if (a.prolong) ref(a.ecoarse, o.level + 1, false);
        ref(a.g, o.level, false);
        ref(a.eout, o.level, true);
        if (a.inject) ref(a.einj, o.level + 1, true);
        break;
    }
    default:
        break;
    }
    return k;
}

// The constants of a constant-coefficient relaxation on level L, in the
// order of the kK* indices, in float and in double: each precision's values
// come from that precision's arithmetic on the level's scale, a and theta
// (the diagonal D = W scale - a, W = 2 dim + 1/2 x edge neighbours + 1/3 x
// corner neighbours of the stencil).
template <typename R>
void relax_constants_as(int dim, int radial, const Level &L, R *k)
{
    const int n2 = radial ? (dim == 3 ? 12 : 4) : 0, n3 = (radial && dim == 3) ? 8 : 0;
    const R scale = (R)L.scale, a = (R)L.a, theta = (R)L.theta;
    const R W = R(2 * dim) + R(0.5) * R(n2) + R(1.0 / 3.0) * R(n3);
    const R D = scale * W - a;
    k[kKScale] = scale;
    k[kKA] = a;
    k[kKTheta] = theta;
    k[kKStep] = theta / D;
    k[kKOmt] = R(1) - theta;
    k[kKBeta] = theta * scale / D;
    k[kKAw] = a - R(4) * scale;
}
void relax_constants(int dim, int radial, const Level &L, float *kf, double *kd)
{
    relax_constants_as<float>(dim, radial, L, kf);
    relax_constants_as<double>(dim, radial, L, kd);
}

// Stage one run [i, j) of coarse operations in LDS: every buffer it touches
// gets an LDS slot; a buffer is loaded when the run reads it before writing
// it, and stored when the next reference after the run (the cycle repeats,
// so the search wraps around) is a read.  live_out, the cycle's result, is
// read at the end of every cycle.  Returns false when the run does
// not fit (its levels or its LDS image too large, or the staging full).
template <typename T>
bool stage_lds_run(sgml_plan *P, const std::vector<HostOp> &ops, const void *live_out, size_t i, size_t j,
                   int &nl, int &nx, RunDesc &R)
{
    struct Slot {
        const void *p;
        size_t count;
        int off;
        bool load, written;
    };
    std::vector<Slot> slots;
    auto find = [&](const void *p) {
        for (size_t q = 0; q < slots.size(); ++q)
            if (slots[q].p == p) return (int)q;
        return -1;
    };
    size_t elems = 0;
    for (size_t k = i; k < j; ++k) {
        if (level_nodes(P->dim, P->n, ops[k].op.level) > (size_t)coarse_lds_nodes(P->dim)) return false;
        Ref r[6];
        const int nr = op_refs(P, ops[k], r);
        for (int q = 0; q < nr; ++q) {
            int s = find(r[q].p);
            if (s < 0) {
                slots.push_back({r[q].p, r[q].count, (int)elems, !r[q].write, false});
                elems += (r[q].count + 3) / 4 * 4;
                s = (int)slots.size() - 1;
            }
            if (r[q].write) slots[s].written = true;
        }
    }
    const size_t hdr_off = (elems * sizeof(T) + 15) / 16 * 16;
    const size_t bytes = hdr_off + (j - i) * sizeof(LdsOpHdr<T>);
    const size_t budget = P->lds_max > 1024 ? P->lds_max - 1024 : 0;  // static LDS of the kernel
    if (bytes > budget || nl + (j - i) > (size_t)kMaxCoarseOps || nx + 2 * slots.size() > (size_t)kMaxXfers)
        return false;
    const size_t nops = ops.size();
    auto stored = [&](const void *p) {
        for (size_t d = 0; d < nops; ++d) {
            if ((j + d) % nops == 0 && p == live_out) return true;
            Ref r[6];
            const int nr = op_refs(P, ops[(j + d) % nops], r);
            for (int q = 0; q < nr; ++q)
                if (r[q].p == p) return !r[q].write;
        }
        return false;
    };
    auto off = [&](const void *p) {
        const int s = find(p);
        return s < 0 ? 0 : slots[s].off;
    };
    R.lds = 1;
    R.lop0 = nl;
    R.x0 = nx;
    R.lds_bytes = bytes;
    R.hdr_off = (int)hdr_off;
    for (size_t k = i; k < j; ++k) {
        const CoarseOp &o = ops[k].op;
        LdsOp &lo = P->lops_host[nl++];
        std::memset(&lo, 0, sizeof(lo));
        lo.kind = o.kind;
        lo.m = o.m;
        lo.first = o.first;
        lo.target = o.target;
        lo.in0 = off(o.in0);
        lo.in1 = off(o.in1);
        lo.out = off(o.out);
        lo.nodes = (int)level_nodes(P->dim, P->n, o.level);
        lo.inv_m = 1.0f / (float)o.m;
        // small levels: one wavefront, one node per lane
        lo.solo = lo.nodes <= 64 && o.target < 0;
        lo.sync = 1;
        lo.sig = o.in2;
        lo.L = P->level(o.level);
        relax_constants(P->dim, P->var.radial, lo.L, lo.kf, lo.kd);
    }
    for (int q = R.lop0; q + 1 < nl; ++q)  // a solo operation followed by another needs no barrier
        if (P->lops_host[q].solo && P->lops_host[q + 1].solo) P->lops_host[q].sync = 0;
    R.nload = R.nstore = 0;
    for (const Slot &sl : slots)
        if (sl.load) {
            P->xfer_host[nx++] = {const_cast<void *>(sl.p), sl.off, (int)sl.count};
            ++R.nload;
        }
    for (const Slot &sl : slots)
        if (sl.written && stored(sl.p)) {
            P->xfer_host[nx++] = {const_cast<void *>(sl.p), sl.off, (int)sl.count};
            ++R.nstore;
        }
    return true;
}

// Upload the coarse operations (in execution order), their LDS form and the
// level table; the device copy serves every cycle of the solve.  Coarse runs
// beyond the buffer's capacity fall back to separate launches.
template <typename T>
sgml_status upload_ops(sgml_plan *P, std::vector<HostOp> &ops, const void *live_out, hipStream_t st)
{
    int nc = 0;
    for (auto &h : ops) {
        if (!h.coarse) continue;
        if (nc >= kMaxCoarseOps) {
            h.coarse = false;
            continue;
        }
        P->ops_host[nc++] = h.op;
    }
    P->runs.clear();
    int op0 = 0, nl = 0, nx = 0;
    for (size_t i = 0; i < ops.size();) {
        if (!ops[i].coarse) {
            ++i;
            continue;
        }
        size_t j = i;
        while (j < ops.size() && ops[j].coarse) ++j;
        RunDesc R;
        std::memset(&R, 0, sizeof(R));
        R.op0 = op0;
        R.nops = (int)(j - i);
        if (!stage_lds_run<T>(P, ops, live_out, i, j, nl, nx, R)) R.lds = 0;
        P->runs.push_back(R);
        op0 += R.nops;
        i = j;
    }
    for (int nu = 0; nu < P->n; ++nu) P->levels_host[nu] = P->level(nu);
    if (nc) SGML_HIP(hipMemcpyAsync(P->at<CoarseOp>(P->lay.ops), P->ops_host, sizeof(CoarseOp) * nc,
                                    hipMemcpyHostToDevice, st));
    if (nl) SGML_HIP(hipMemcpyAsync(P->at<LdsOp>(P->lay.lops), P->lops_host, sizeof(LdsOp) * nl,
                                    hipMemcpyHostToDevice, st));
    if (nx) SGML_HIP(hipMemcpyAsync(P->at<LdsXfer>(P->lay.xfer), P->xfer_host, sizeof(LdsXfer) * nx,
                                    hipMemcpyHostToDevice, st));
    SGML_HIP(hipMemcpyAsync(P->at<Level>(P->lay.levels), P->levels_host, sizeof(Level) * P->n,
                            hipMemcpyHostToDevice, st));
    return SGML_OK;
}

// Enqueue one cycle: runs of coarse operations as one k_coarse launch each,
// the rest as grid launches; level-0 relaxations timed when profiling.
template <typename T>
// ops [0, end) of the cycle; the level-0 source src0 of the compiled list
// is read from src0_now (the mixed 2D cycle alternates it between two
// buffers, the cycle end writing the next cycle's into the other one).
sgml_status run_ops(sgml_plan *P, const std::vector<HostOp> &ops, size_t end, const void *src0, const void *src0_now,
                    const double *G, bool profile, bool use_sweep3d, int chunk, int zreq, std::vector<Timed> &timed,
                    hipStream_t st)
{
    const CoarseOp *dev_ops = P->at<CoarseOp>(P->lay.ops);
    const Level *dev_levels = P->at<Level>(P->lay.levels);
    const LdsOp *dev_lops = P->at<LdsOp>(P->lay.lops);
    const LdsXfer *dev_xfer = P->at<LdsXfer>(P->lay.xfer);
    unsigned long long *targets = target(P, 0);
    size_t run = 0;
    for (size_t i = 0; i < end;) {
        if (ops[i].coarse) {
            size_t j = i;
            while (j < ops.size() && ops[j].coarse) ++j;
            if (run >= P->runs.size()) return SGML_E_ARG;
            const RunDesc &R = P->runs[run++];
            const bool staged = R.lds && launch_coarse_lds<T>(P->var, dev_lops + R.lop0, R.nops, R.hdr_off,
                                                              dev_xfer + R.x0, R.nload, R.nstore, R.lds_bytes, G,
                                                              targets, st);
            if (!staged) launch_coarse<T>(P->var, dev_ops + R.op0, R.nops, dev_levels, G, targets, st);
            i = j;
            continue;
        }
        const CoarseOp &o = ops[i].op;
        if (o.kind == kOpVisit) {
            VisitArgs a = ops[i].visit;
            if (a.g == src0) a.g = src0_now;
            a.chunk = chunk;
            a.G = G;
            a.targets = targets;
            a.L = P->level(o.level);
            const int cls = a.inject ? SGML_PROF_VISIT0_INJ : SGML_PROF_VISIT0;
            const long ev = (profile && o.level == 0) ? prof_pair(P) : -1;
            if (ev >= 0) SGML_HIP(hipEventRecord(P->pev[ev], st));
            launch_visit2d<T>(P->var, a, st);
            if (ev >= 0) {
                SGML_HIP(hipEventRecord(P->pev[ev + 1], st));
                timed.push_back({cls, a.sweeps, ev});
            }
            ++i;
            continue;
        }
        switch (o.kind) {
        case kOpFill:
            launch_fill<T>((T *)o.out, level_nodes(P->dim, P->n, o.level), T(0), st);
            break;
        case kOpSweep2: {
            const long ev = (profile && o.level == 0) ? prof_pair(P) : -1;
            if (ev >= 0) SGML_HIP(hipEventRecord(P->pev[ev], st));
            launch_sweep3d2<T>(P->var, P->level(o.level), (const T *)o.in0, (T *)o.out, (const T *)o.in1, G,
                               o.target >= 0 ? target(P, o.target) : nullptr, zreq, st);
            if (ev >= 0) {
                SGML_HIP(hipEventRecord(P->pev[ev + 1], st));
                timed.push_back({SGML_PROF_SWEEP0, 2, ev});
            }
            break;
        }
        case kOpRestrict:
            if (P->dim == 3 && use_sweep3d && sweep3d_supported(2 * o.m - 1)) {
                launch_restrict3d<T>(o.m, (const T *)o.in0, (T *)o.out, zreq, st);
            } else if (P->dim == 2 && use_sweep3d && o.m >= 65 && i + 1 < end && !ops[i + 1].coarse &&
                       ops[i + 1].op.kind == kOpRestrict && ops[i + 1].op.in0 == o.out) {
                // this step and the next in one pass
                launch_restrict2d2<T>(o.m, (const T *)o.in0, (T *)o.out, (T *)ops[i + 1].op.out, st);
                ++i;
            } else {
                launch_restrict<T, T>(P->dim, o.m, (const T *)o.in0, (T *)o.out, st);
            }
            break;
        case kOpProlong:
            if (P->dim == 3 && use_sweep3d && sweep3d_supported(o.m))
                launch_prolong3d<T>((o.m + 1) / 2, (const T *)o.in0, (const T *)o.in1, (T *)o.out, o.first != 0,
                                    zreq, st);
            else
                launch_prolong<T>(P->dim, (o.m + 1) / 2, (const T *)o.in0, (const T *)o.in1, (T *)o.out,
                                  o.first != 0, st);
            break;
        case kOpInject:
            launch_inject<T>(P->dim, o.m, (const T *)o.in0, (T *)o.out, st);
            break;
        default: {
            const long ev = (profile && o.level == 0) ? prof_pair(P) : -1;
            if (ev >= 0) SGML_HIP(hipEventRecord(P->pev[ev], st));
            unsigned long long *tg = o.target >= 0 ? target(P, o.target) : nullptr;
            if (P->dim == 3 && use_sweep3d && sweep3d_supported(o.m))
                launch_sweep3d<T>(P->var, P->level(o.level), (const T *)o.in0, (T *)o.out, (const T *)o.in1,
                                  (const T *)o.in2, G, tg, zreq, st);
            else
                launch_sweep<T>(P->var, P->level(o.level), (const T *)o.in0, (T *)o.out, (const T *)o.in1,
                                (const T *)o.in2, G, tg, st);
            if (ev >= 0) {
                SGML_HIP(hipEventRecord(P->pev[ev + 1], st));
                timed.push_back({SGML_PROF_SWEEP0, 1, ev});
            }
            break;
        }
        }
        ++i;
    }
    return SGML_OK;
}

int coarse_level_of(const sgml_plan *P, int coarse_nodes)
{
    if (coarse_nodes < 0) return kMaxLevels;  // disabled
    const size_t limit = coarse_nodes != 0    ? (size_t)coarse_nodes
                         : P->dim == 2 ? kDefaultCoarseNodes2
                                       : kDefaultCoarseNodes3;
    int nu = P->n;
    while (nu > 0 && level_nodes(P->dim, P->n, nu - 1) <= limit) --nu;
    return nu;
}

// One solve of the recurrence (Sec. 2) on one plan, split into phases so that
// several solves (right-hand sides on their own plans and streams) can run in
// lock step: begin() up to the normaliser (synchronises its stream once) and
// the compiled cycle; enqueue_cycle() one cycle and the copy of its residual
// norm to the host, without waiting; finish_cycle() the stop test, after the
// caller has synchronised the stream; end() the per-visit pseudo-residuals,
// the W scaling of a transposed solve and the timing (synchronises).
// wscale: the source is W^-1 f and the result is W times the solution (the
// transposed solve, dL^T = W dL W^-1 under the node images of Neumann faces).
template <typename T>
struct Solve {
    static constexpr bool mixed = sizeof(T) == 4;
    sgml_plan *P;
    const double *f, *G;
    double *u;
    const sgml_opts *o;
    hipStream_t st;
    bool wscale;
    sgml_stats local;
    sgml_stats &S;
    Level L0;
    std::vector<int> lev, cnt;
    std::vector<HostOp> ops;
    std::vector<Timed> timed;
    long long updates_per_cycle = 0;
    bool pure = false, z_march = false, row_march = false, done = false, use_graphs = false;
    int i = 0, k0 = 0, chunk = 0, zreq = 0;
    double norm0 = 0.0;
    double *s = nullptr, *s_next = nullptr, *part = nullptr, *means = nullptr;
    T *shat = nullptr, *g1 = nullptr;
    T *shat2 = nullptr;  // the other level-0 source buffer (2D mixed, level-1 restriction fused)
    const T *src0 = nullptr, *e = nullptr;
    sgml_status status = SGML_E_MAXCYCLES;

    Solve(sgml_plan *P_, const double *f_, const double *G_, double *u_, const sgml_opts *o_, hipStream_t st_,
          sgml_stats *stats, bool wscale_)
        : P(P_), f(f_), G(G_), u(u_), o(o_), st(st_), wscale(wscale_), S(stats ? *stats : local)
    {
    }

    sgml_status begin()
    {
        L0 = P->level(0);
        s = P->at<double>(P->lay.s);
        shat = mixed ? P->at<T>(P->lay.shat) : nullptr;
        src0 = mixed ? shat : (const T *)s;
        build_schedule(P->n, o->n_r, o->schedule, lev, cnt);
        if ((int)lev.size() > SGML_MAX_VISITS) return SGML_E_ARG;
        std::memset(&S, 0, sizeof(S));
        S.visits = (int)lev.size();
        if (o->profile) {
            sgml_status rc = prof_pool(P);
            if (rc != SGML_OK) return rc;
        }
        P->prof_untimed = 0;
        SGML_HIP(hipEventRecord(P->ev0, st));
        clear_targets(P, 1, 1, st);
        // pure Neumann: the source is projected below, its FP32 copy taken after
        pure = P->dir == 0;
        float *s32 = mixed && !pure ? reinterpret_cast<float *>(shat) : nullptr;
        launch_init(P->var, L0, f, G, P->sigma, s, u, s32, target(P, 1), wscale, st);
        // pure Neumann (Sec. 2, last paragraph; eq. (10)): the source minus its
        // trapezoid mean; norm0 is that of the projected source
        part = P->at<double>(P->lay.part);
        means = P->at<double>(P->lay.means);
        if (pure) {
            launch_wmean<double>(P->dim, L0, s, 1.0, part, means, st);
            clear_targets(P, 1, 1, st);
            launch_project<double>(P->dim, L0, s, u, means, nullptr, (double *)nullptr, 0.0, target(P, 1), st);
        }
        SGML_HIP(hipGetLastError());
        sgml_status rc = fetch(P, 1, 1, st);
        if (rc != SGML_OK) return rc;
        norm0 = host_max(P, 1);
        S.norm0 = norm0;
        if (!(norm0 > 0.0)) {
            // u_init = G on Dirichlet nodes, 0 elsewhere, already solves the problem
            launch_set_dirichlet(L0, P->dim, G, u, st);
            status = std::isfinite(norm0) ? SGML_OK : SGML_E_ARG;
            done = true;
            return SGML_OK;
        }
        // the fused cycle ends also write the next cycle's source, which a pure
        // Neumann solve re-projects: it takes the generic cycle end
        z_march = P->dim == 3 && o->fuse >= 0 && sweep3d_supported(P->N) && !pure;
        row_march = P->dim == 2 && o->fuse >= 0 && P->N >= 64 && !pure;
        // the 2D row-marching cycle end of the mixed cycle also restricts the
        // new source to level 1; it then writes the residual to the other buffer
        g1 = mixed && row_march && P->n >= 2 ? P->at<T>(P->lay.g[1]) : nullptr;
        s_next = g1 ? P->at<double>(P->lay.s2) : s;
        // with the level-1 restriction fused, the next source goes to the other
        // source buffer (the closing visit may read the current one while the
        // cycle end writes it): the FP32 half left free by the level-0 buffers
        // (FP64-sized) after the two FP32 ones
        if (g1) shat2 = reinterpret_cast<T *>(P->at<char>(P->lay.e0) + 2 * P->M * sizeof(T));
        e = compile_cycle<T>(P, src0, lev, cnt, o->record_pres != 0, coarse_level_of(P, o->coarse_nodes),
                             o->fuse < 0 ? 0 : (o->fuse == 0 ? kDefaultFuseMin : std::max(o->fuse, 64)),
                             g1 != nullptr, ops, updates_per_cycle);
        // the two buffers alternate only where every reader of the level-0
        // source is a row-marching visit, which takes it per cycle
        for (const HostOp &h : ops)
            if ((h.coarse || h.op.kind != kOpVisit) && (h.op.in0 == src0 || h.op.in1 == src0 || h.op.in2 == src0))
                shat2 = nullptr;
        rc = upload_ops<T>(P, ops, e, st);
        if (rc != SGML_OK) return rc;
        chunk = o->chunk_rows > 0 ? std::max(8, o->chunk_rows) : 0;  // 0: per launch
        zreq = o->z_chunk > 0 ? o->z_chunk : 0;                     // 0: per level
        // MIXED: the cycle runs on 2^-k0 s, an exact scaling that keeps the FP32
        // values of the cycle (down to the tolerance times the source) inside
        // the normal range; within [2^-40, 2^40] no scaling is needed
        const int kn = mixed ? std::ilogb(norm0) : 0;
        k0 = (kn < -40 || kn > 40) ? kn : 0;
        // the FP32 source, unless the initialisation wrote it (unscaled)
        if (mixed && (k0 != 0 || pure)) launch_source_cast<T>(L0, P->dim, s, shat, std::ldexp(1.0, -k0), st);
        if (g1) launch_restrict<T, T>(P->dim, P->m(1), src0, g1, st);  // cycle 0's level-1 source
        i = 0;
        done = o->max_cycles < 1;
        // cycles after the first (which carries the Dirichlet values) repeat the
        // same launches: replayed as graphs unless profiling (events) or asked not to
        use_graphs = o->graphs >= 0 && !o->profile && !P->graphs_broken;
        return SGML_OK;
    }

    // Everything a cycle enqueues, on stream q.
    sgml_status enqueue_body(hipStream_t q)
    {
        const double *Gc = i == 0 ? G : nullptr;
        const double escale = std::ldexp(1.0, k0), sscale = std::ldexp(1.0, -k0);
        clear_targets(P, 0, 1, q);
        if (o->record_pres) clear_targets(P, kPres, (int)lev.size(), q);
        timed.clear();
        P->pev_used = 0;
        // the cycle's closing level-0 visit and the cycle end in one pass: FP32
        // cycles without Dirichlet data to impose, a constant coefficient, the
        // level-1 restriction fused, nothing recorded per visit
        const HostOp *last = ops.empty() ? nullptr : &ops.back();
        bool fuse_end = false;
        if constexpr (mixed) {
            fuse_end = row_march && g1 && shat2 && !Gc && !P->var.sigma && !o->record_pres && last && !last->coarse &&
                       last->op.kind == kOpVisit && last->op.level == 0 && last->visit.prolong &&
                       !last->visit.first && !last->visit.inject && o->fuse_end >= 0 &&
                       visit_end_supported(last->visit.sweeps, P->m(0), o->fuse_end > 0);
        }
        // this cycle's level-0 source and the buffer of the next one (they swap
        // with the residual buffers)
        T *src_now = shat, *src_next = shat;
        if (shat2) {
            const bool first_slot = s == P->at<double>(P->lay.s);
            src_now = first_slot ? shat : shat2;
            src_next = first_slot ? shat2 : shat;
        }
        sgml_status rc = run_ops<T>(P, ops, ops.size() - (fuse_end ? 1 : 0), src0, mixed ? src_now : src0, Gc,
                                    o->profile != 0, o->fuse >= 0, chunk, zreq, timed, q);
        if (rc != SGML_OK) return rc;
        const long ev = o->profile ? prof_pair(P) : -1;
        if (ev >= 0) SGML_HIP(hipEventRecord(P->pev[ev], q));
        // pure Neumann: the cycle's correction is collected minus its mean
        if (pure) launch_wmean<T>(P->dim, L0, e, escale, part, means + 1, q);
        if (row_march || z_march) {
            CycleEndArgs ca;
            ca.e = e;
            ca.escale = escale;
            ca.G = Gc;
            ca.sigma = P->sigma;
            ca.u = u;
            ca.s = s;
            ca.s_out = s_next;
            ca.shat = src_next;
            ca.shat_scale = sscale;
            ca.norm = target(P, 0);
            ca.g1 = g1;
            ca.L = L0;
            ca.chunk = chunk;
            ca.zchunk = zreq;
            if (fuse_end) {
                if constexpr (mixed) {
                    VisitArgs a = last->visit;
                    if (a.g == src0) a.g = src_now;
                    a.chunk = chunk;
                    a.G = nullptr;
                    a.targets = target(P, 0);
                    a.L = L0;
                    launch_visit_end2d<T>(P->var, a, ca, q);
                }
            } else if (z_march) {
                launch_cycle_end3d<T>(P->var, ca, q);
            } else {
                launch_cycle_end2d<T>(P->var, ca, q);
            }
        } else {
            launch_boundary<T>(P->var, L0, e, escale, Gc, P->sigma, u, s, shat, sscale, target(P, 0), q);
        }
        if (ev >= 0) {
            SGML_HIP(hipEventRecord(P->pev[ev + 1], q));
            timed.push_back({fuse_end ? SGML_PROF_VISIT0_END : SGML_PROF_CYCLE_END,
                             fuse_end ? last->visit.sweeps : 0, ev});
        }
        if (pure) {
            // s - dL(e - mean e) = s - dL e + a mean e differs from s - dL e by a
            // constant, which the projection of the residual removes
            launch_wmean<double>(P->dim, L0, s, 1.0, part, means, q);
            clear_targets(P, 0, 1, q);
            launch_project<T>(P->dim, L0, s, u, means, means + 1, shat, sscale, target(P, 0), q);
        }
        SGML_HIP(hipGetLastError());
        return fetch_async(P, 0, 1, q);
    }

    // What a captured cycle depends on beyond the plan: the options that shape
    // the compiled cycle, the buffers it touches and the scaling.
    std::vector<long long> graph_key() const
    {
        return {(long long)sizeof(T),       o->n_r,      o->schedule,         o->record_pres,
                o->coarse_nodes,            o->fuse,     o->fuse_end,         chunk,               zreq,
                (long long)(uintptr_t)u,    (long long)(uintptr_t)P->sigma, P->var.sigma,
                (long long)(uintptr_t)P->ws, (long long)(uintptr_t)s, k0, pure};
    }

    // The cycle as a graph (captured on the plan's private stream the first
    // time this key and residual buffer come up), or null to run it eagerly.
    hipGraphExec_t cycle_graph()
    {
        const int slot = s == P->at<double>(P->lay.s) ? 0 : 1;
        sgml_plan::CycleGraph &cg = P->graph[slot];
        const std::vector<long long> key = graph_key();
        if (cg.valid && cg.key == key) return cg.exec;
        if (cg.exec) (void)hipGraphExecDestroy(cg.exec);
        cg.exec = nullptr;
        cg.valid = false;
        if (!P->cap_st && hipStreamCreateWithFlags(&P->cap_st, hipStreamNonBlocking) != hipSuccess) {
            P->cap_st = nullptr;
            P->graphs_broken = true;
            return nullptr;
        }
        hipGraph_t g = nullptr;
        bool ok = hipStreamBeginCapture(P->cap_st, hipStreamCaptureModeRelaxed) == hipSuccess;
        if (ok) {
            ok = enqueue_body(P->cap_st) == SGML_OK;
            ok = (hipStreamEndCapture(P->cap_st, &g) == hipSuccess) && ok && g;
        }
        if (ok) ok = hipGraphInstantiate(&cg.exec, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
        if (!ok) {
            (void)hipGetLastError();
            cg.exec = nullptr;
            P->graphs_broken = true;
            return nullptr;
        }
        cg.valid = true;
        cg.key = key;
        return cg.exec;
    }

    sgml_status enqueue_cycle()
    {
        S.node_updates += updates_per_cycle;
        if (use_graphs && i >= 1) {
            if (hipGraphExec_t ge = cycle_graph()) {
                SGML_HIP(hipGraphLaunch(ge, st));
                return SGML_OK;
            }
            use_graphs = false;
        }
        return enqueue_body(st);
    }

    sgml_status finish_cycle()
    {
        for (auto &t : timed) {
            float ms = 0.f;
            SGML_HIP(hipEventElapsedTime(&ms, P->pev[t.ev], P->pev[t.ev + 1]));
            S.prof_ms[t.cls] += ms;
            S.prof_launches[t.cls]++;
            S.prof_sweeps[t.cls] += t.sweeps;
        }
        const double norm = host_max(P, 0);
        const double rel = norm / norm0;
        S.cycles = i + 1;
        S.relres = rel;
        if (i < SGML_HIST) S.history[i] = rel;
        std::swap(s, s_next);  // the residual the next cycle end reads
        const int win = o->stall_window == 0 ? 3 : o->stall_window;
        if (!std::isfinite(rel) || rel > 1e3) {
            status = SGML_E_DIVERGED;
            done = true;
        } else if (rel <= o->tol) {
            status = SGML_OK;
            done = true;
        } else if (win > 0 && i >= win && i < SGML_HIST && rel > 0.5 * S.history[i - win]) {
            status = SGML_E_STAGNATED;
            done = true;
        }
        ++i;
        if (i >= o->max_cycles) done = true;
        return SGML_OK;
    }

    sgml_status end()
    {
        if (o->record_pres && !ops.empty()) {
            sgml_status rc = fetch(P, kPres, (int)lev.size(), st);
            if (rc != SGML_OK) return rc;
            for (size_t v = 0; v < lev.size(); ++v) S.pres[v] = host_max(P, kPres + (int)v);
        }
        if (wscale) launch_trap_scale(L0, P->dim, u, st);
        SGML_HIP(hipEventRecord(P->ev1, st));
        SGML_HIP(hipEventSynchronize(P->ev1));
        SGML_HIP(hipEventElapsedTime(&S.ms, P->ev0, P->ev1));
        S.prof_untimed = P->prof_untimed;
        S.status = status;
        return status;
    }
};

template <typename T>
sgml_status run_solve(sgml_plan *P, const double *f, const double *G, double *u, const sgml_opts *o,
                      hipStream_t st, sgml_stats *stats, bool wscale = false)
{
    Solve<T> R(P, f, G, u, o, st, stats, wscale);
    sgml_status rc = R.begin();
    if (rc != SGML_OK) return rc;
    while (!R.done) {
        rc = R.enqueue_cycle();
        if (rc != SGML_OK) return rc;
        SGML_HIP(hipStreamSynchronize(st));
        rc = R.finish_cycle();
        if (rc != SGML_OK) return rc;
    }
    return R.end();
}

bool all_dirichlet(const sgml_plan *P)
{
    for (int f = 0; f < 2 * P->dim; ++f)
        if (P->prob.face[f] != SGML_DIRICHLET) return false;
    return true;
}

// Restricted coefficients per level in the plan's workspace: Algorithm 1
// applied to sigma ("restricted sources and coefficients", Sec. 2), and their
// FP32 copies in mixed plans.
sgml_status build_coeff_pyramid(sgml_plan *P, hipStream_t st)
{
    const double *sigma = P->sigma;
    if (!sigma) return SGML_OK;
    const double *prev = sigma;
    for (int nu = 1; nu < P->n; ++nu) {
        double *cur = P->at<double>(P->lay.sig64[nu]);
        launch_restrict<double, double>(P->dim, P->m(nu), prev, cur, st);
        prev = cur;
    }
    if (P->precision == SGML_MIXED) {
        launch_convert<double, float>(sigma, P->at<float>(P->lay.sig0t), P->M, st);
        for (int nu = 1; nu < P->n; ++nu)
            launch_convert<double, float>(P->at<double>(P->lay.sig64[nu]), P->at<float>(P->lay.sigt[nu]),
                                          level_nodes(P->dim, P->n, nu), st);
    }
    SGML_HIP(hipGetLastError());
    return SGML_OK;
}

// Workspace for sgml_solve_noalloc: one array per device, kept by the
// device's copy of the code object until the process ends.  Host code never
// names it (in host code the name is a host-side stand-in, not a device
// address); it uses the device address looked up once per device.
constexpr size_t kScratchBytes = SGML_NOALLOC_WORKSPACE_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex scratch_lock;
void *scratch_ptr[kMaxDevices];  // device address of `scratch` per device, null until looked up

// Look up the current device's `scratch` (once per device).  Returns null
// when the lookup fails.
void *scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> guard(scratch_lock);
    if (!scratch_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        scratch_ptr[device] = ptr;
    }
    return scratch_ptr[device];
}

}  // namespace

extern "C" {

size_t sgml_workspace_bytes(const sgml_problem *prob, int precision)
{
    if (!valid_problem(prob) || !valid_shape(prob)) return 0;
    if (precision != SGML_FP64 && precision != SGML_MIXED) return 0;
    return make_layout(prob, precision).total;
}

sgml_status sgml_plan_create(const sgml_problem *prob, int precision, void *workspace, size_t ws_bytes,
                             sgml_plan **out)
{
    if (!out) return SGML_E_ARG;
    *out = nullptr;
    if (!valid_problem(prob)) return SGML_E_ARG;
    if (precision != SGML_FP64 && precision != SGML_MIXED) return SGML_E_ARG;
    if (!valid_shape(prob)) return SGML_E_SHAPE;
    const Layout lay = make_layout(prob, precision);
    // no workspace at all: a plan for sgml_solve_noalloc only
    const bool no_ws = !workspace && ws_bytes == 0;
    if (!no_ws && (!workspace || ws_bytes < lay.total || ((uintptr_t)workspace % kAlign) != 0))
        return SGML_E_WORKSPACE;
    sgml_plan *P = new (std::nothrow) sgml_plan();
    if (!P) return SGML_E_ARG;
    P->prob = *prob;
    P->precision = precision;
    P->dim = prob->dim;
    P->n = prob->n;
    P->N = (1 << prob->n) + 1;
    P->M = level_nodes(prob->dim, prob->n, 0);
    P->h = 1.0 / (double)(1 << prob->n);
    const int K = prob->stencil == SGML_RADIAL ? (prob->dim == 3 ? 26 : 8) : 2 * prob->dim;
    P->C = prob->stencil == SGML_RADIAL ? (2.0 * prob->dim) / K : 1.0;
    P->theta = prob->theta > 0.0 ? prob->theta : default_theta(prob->dim, prob->stencil);
    P->dir = 0;
    for (int f = 0; f < 2 * prob->dim; ++f)
        if (prob->face[f] == SGML_DIRICHLET) P->dir |= 1u << f;
    P->var.dim = prob->dim;
    P->var.radial = prob->stencil == SGML_RADIAL;
    P->var.sigma = 0;
    P->ws = static_cast<char *>(workspace);
    P->ws_bytes = ws_bytes;
    P->lay = lay;
    P->sigma = nullptr;
    // set-up of the device's static workspace (sgml_solve_noalloc) happens here,
    // once per device, so that the no-allocation entry point never triggers it
    if (hipGetDevice(&P->device) != hipSuccess || !scratch_of(P->device) ||
        hipHostMalloc((void **)&P->host, sizeof(unsigned long long) * kScalars, hipHostMallocDefault) !=
            hipSuccess) {
        delete P;
        return SGML_E_HIP;
    }
    P->ops_host = nullptr;
    P->lops_host = nullptr;
    P->xfer_host = nullptr;
    P->levels_host = nullptr;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device) != hipSuccess) lds = 0;
    P->lds_max = lds > 0 ? (size_t)lds : 0;
    if (hipEventCreate(&P->ev0) != hipSuccess || hipEventCreate(&P->ev1) != hipSuccess ||
        hipHostMalloc((void **)&P->ops_host, sizeof(CoarseOp) * kMaxCoarseOps, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void **)&P->lops_host, sizeof(LdsOp) * kMaxCoarseOps, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void **)&P->xfer_host, sizeof(LdsXfer) * kMaxXfers, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&P->levels_host, sizeof(Level) * kMaxLevels, hipHostMallocDefault) !=
            hipSuccess) {
        if (P->ops_host) (void)hipHostFree(P->ops_host);
        if (P->lops_host) (void)hipHostFree(P->lops_host);
        if (P->xfer_host) (void)hipHostFree(P->xfer_host);
        (void)hipHostFree(P->host);
        delete P;
        return SGML_E_HIP;
    }
    *out = P;
    return SGML_OK;
}

sgml_status sgml_plan_set_coeffs(sgml_plan *P, const double *sigma, void *stream)
{
    if (!P) return SGML_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    SGML_HIP(hipSetDevice(P->device));
    P->sigma = sigma;
    P->var.sigma = sigma ? 1 : 0;
    for (sgml_plan *Q : P->sub) {  // a batch shares the pyramid built here
        Q->sigma = sigma;
        Q->var.sigma = P->var.sigma;
    }
    if (!sigma || !P->ws) return SGML_OK;  // a plan without workspace builds it per solve
    return build_coeff_pyramid(P, st);
}

sgml_status sgml_solve(sgml_plan *P, const double *f, const double *G, double *u, const sgml_opts *o,
                       void *stream, sgml_stats *stats)
{
    if (!P || !f || !u || !o) return SGML_E_ARG;
    if (o->max_cycles < 1 || !(o->tol >= 0.0)) return SGML_E_ARG;
    if (o->precision != SGML_FP64 && o->precision != SGML_MIXED) return SGML_E_ARG;
    if (o->precision == SGML_MIXED && P->precision != SGML_MIXED) return SGML_E_WORKSPACE;
    if (o->schedule != SGML_SCHEDULE_ONCE && o->schedule != SGML_SCHEDULE_EACH) return SGML_E_ARG;
    if (u == f || (G && u == G)) return SGML_E_ARG;
    if (!P->ws) return SGML_E_WORKSPACE;
    SGML_HIP(hipSetDevice(P->device));
    hipStream_t st = (hipStream_t)stream;
    sgml_status rc = o->precision == SGML_MIXED ? run_solve<float>(P, f, G, u, o, st, stats)
                                                : run_solve<double>(P, f, G, u, o, st, stats);
    if (stats) stats->status = rc;
    return rc;
}

sgml_status sgml_solve_noalloc(sgml_plan *P, const double *f, const double *G, double *u, const sgml_opts *o,
                               void *stream, sgml_stats *stats)
{
    if (!P || !f || !u || !o) return SGML_E_ARG;
    if (o->max_cycles < 1 || !(o->tol >= 0.0)) return SGML_E_ARG;
    if (o->precision != SGML_FP64 && o->precision != SGML_MIXED) return SGML_E_ARG;
    if (o->precision == SGML_MIXED && P->precision != SGML_MIXED) return SGML_E_WORKSPACE;
    if (o->schedule != SGML_SCHEDULE_ONCE && o->schedule != SGML_SCHEDULE_EACH) return SGML_E_ARG;
    if (o->profile) return SGML_E_ARG;  // profiling creates events
    if (u == f || (G && u == G)) return SGML_E_ARG;
    if (P->lay.total > kScratchBytes) return SGML_E_WORKSPACE;  // beyond the static workspace
    SGML_HIP(hipSetDevice(P->device));
    void *ptr = scratch_ptr[P->device];  // looked up when the plan was created
    if (!ptr) return SGML_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    // the static workspace stands in for the plan's own for this call; other
    // calls on the device may have left anything there, so the coefficient
    // pyramid is rebuilt (every other region is initialised by the solve)
    char *own = P->ws;
    P->ws = static_cast<char *>(ptr);
    sgml_opts oo = *o;
    oo.graphs = -1;  // capturing and instantiating a graph allocates
    sgml_status rc = build_coeff_pyramid(P, st);
    if (rc == SGML_OK)
        rc = oo.precision == SGML_MIXED ? run_solve<float>(P, f, G, u, &oo, st, stats)
                                        : run_solve<double>(P, f, G, u, &oo, st, stats);
    P->ws = own;
    if (stats) stats->status = rc;
    return rc;
}

size_t sgml_workspace_bytes_batch(const sgml_problem *prob, int precision, int nrhs)
{
    if (nrhs < 1 || nrhs > SGML_MAX_BATCH) return 0;
    return sgml_workspace_bytes(prob, precision) * (size_t)nrhs;
}

sgml_status sgml_plan_create_batch(const sgml_problem *prob, int precision, int nrhs, void *workspace,
                                   size_t ws_bytes, sgml_plan **out)
{
    if (!out) return SGML_E_ARG;
    *out = nullptr;
    if (nrhs < 1 || nrhs > SGML_MAX_BATCH) return SGML_E_ARG;
    const size_t one = sgml_workspace_bytes(prob, precision);
    if (one == 0) return valid_problem(prob) && (precision == SGML_FP64 || precision == SGML_MIXED) ? SGML_E_SHAPE
                                                                                                    : SGML_E_ARG;
    if (!workspace || ws_bytes < one * (size_t)nrhs) return SGML_E_WORKSPACE;
    sgml_plan *P = nullptr;
    sgml_status rc = sgml_plan_create(prob, precision, workspace, one, &P);
    if (rc != SGML_OK) return rc;
    for (int r = 1; r < nrhs; ++r) {
        sgml_plan *Q = nullptr;
        rc = sgml_plan_create(prob, precision, static_cast<char *>(workspace) + one * (size_t)r, one, &Q);
        hipStream_t q = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (rc == SGML_OK) {
            Q->sig_ws = P->ws;
            P->sub.push_back(Q);
            // default priority; ordered against the caller's stream by events only
            if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess) rc = SGML_E_HIP;
            else P->sub_st.push_back(q);
        }
        if (rc == SGML_OK) {
            if (hipEventCreateWithFlags(&e0, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&e1, hipEventDisableTiming) != hipSuccess)
                rc = SGML_E_HIP;
            if (e0) P->sub_ev.push_back(e0);
            if (e1) P->sub_ev.push_back(e1);
        }
        if (rc != SGML_OK) {
            sgml_plan_destroy(P);
            return rc;
        }
    }
    *out = P;
    return SGML_OK;
}

sgml_status sgml_solve_batch(sgml_plan *P, int nrhs, const double *f, const double *G, double *u,
                             const sgml_opts *o, void *stream, sgml_stats *stats)
{
    if (!P || !f || !u || !o) return SGML_E_ARG;
    if (nrhs < 1 || nrhs > 1 + (int)P->sub.size()) return SGML_E_ARG;
    if (o->max_cycles < 1 || !(o->tol >= 0.0)) return SGML_E_ARG;
    if (o->precision != SGML_FP64 && o->precision != SGML_MIXED) return SGML_E_ARG;
    if (o->precision == SGML_MIXED && P->precision != SGML_MIXED) return SGML_E_WORKSPACE;
    if (o->schedule != SGML_SCHEDULE_ONCE && o->schedule != SGML_SCHEDULE_EACH) return SGML_E_ARG;
    const size_t M = P->M;
    auto overlap = [&](const double *a, const double *b) {
        const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b, len = sizeof(double) * M * (size_t)nrhs;
        return pa < pb + len && pb < pa + len;
    };
    if (overlap(u, f) || (G && overlap(u, G))) return SGML_E_ARG;
    if (!P->ws) return SGML_E_WORKSPACE;
    SGML_HIP(hipSetDevice(P->device));
    hipStream_t st = (hipStream_t)stream;
    for (int r = 1; r < nrhs; ++r) {  // fork: every stream starts after the caller's work so far
        SGML_HIP(hipEventRecord(P->sub_ev[2 * (r - 1)], st));
        SGML_HIP(hipStreamWaitEvent(P->sub_st[r - 1], P->sub_ev[2 * (r - 1)], 0));
    }
    auto run = [&](auto tag) -> sgml_status {
        using T = decltype(tag);
        std::vector<std::unique_ptr<Solve<T>>> runs;
        for (int r = 0; r < nrhs; ++r)
            runs.emplace_back(new Solve<T>(r == 0 ? P : P->sub[r - 1], f + M * r, G ? G + M * r : nullptr,
                                           u + M * r, o, r == 0 ? st : P->sub_st[r - 1],
                                           stats ? stats + r : nullptr, false));
        for (auto &R : runs) {
            sgml_status rc = R->begin();
            if (rc != SGML_OK) return rc;
        }
        // lock step: every unfinished right-hand side enqueues a cycle on its
        // stream, then all are waited for and tested
        for (;;) {
            bool any = false;
            for (auto &R : runs)
                if (!R->done) {
                    sgml_status rc = R->enqueue_cycle();
                    if (rc != SGML_OK) return rc;
                    any = true;
                }
            if (!any) break;
            for (auto &R : runs)
                if (!R->done) {
                    SGML_HIP(hipStreamSynchronize(R->st));
                    sgml_status rc = R->finish_cycle();
                    if (rc != SGML_OK) return rc;
                }
        }
        sgml_status worst = SGML_OK;
        for (auto &R : runs) {
            const sgml_status rc = R->end();
            if (rc == SGML_E_HIP) return rc;
            if (worst == SGML_OK) worst = rc;
        }
        return worst;
    };
    const sgml_status rc = o->precision == SGML_MIXED ? run(float()) : run(double());
    for (int r = 1; r < nrhs; ++r) {  // join: the caller's stream continues after every right-hand side
        SGML_HIP(hipEventRecord(P->sub_ev[2 * (r - 1) + 1], P->sub_st[r - 1]));
        SGML_HIP(hipStreamWaitEvent(st, P->sub_ev[2 * (r - 1) + 1], 0));
    }
    return rc;
}

sgml_status sgml_residual(sgml_plan *P, const double *f, const double *G, const double *u, double *r,
                          double *rmax, double *norm0, void *stream)
{
    if (!P || !f || !u) return SGML_E_ARG;
    if (!P->ws) return SGML_E_WORKSPACE;
    SGML_HIP(hipSetDevice(P->device));
    hipStream_t st = (hipStream_t)stream;
    clear_targets(P, 1, 2, st);
    launch_residual(P->var, P->level(0), f, G, P->sigma, u, r, target(P, 2), target(P, 1), st);
    SGML_HIP(hipGetLastError());
    sgml_status rc = fetch(P, 1, 2, st);
    if (rc != SGML_OK) return rc;
    if (norm0) *norm0 = host_max(P, 1);
    if (rmax) *rmax = host_max(P, 2);
    return SGML_OK;
}

sgml_status sgml_adjoint(sgml_plan *P, const double *g, double *lambda, const sgml_opts *o, void *stream,
                         sgml_stats *stats)
{
    if (!P) return SGML_E_ARG;
    if (all_dirichlet(P)) {
        // symmetric operator: the transposed solve is the solve itself, with
        // the adjoint vanishing on Dirichlet nodes
        return sgml_solve(P, g, nullptr, lambda, o, stream, stats);
    }
    if (P->dir == 0) return SGML_E_UNSUPPORTED;  // pure Neumann: not covered
    // W dL is symmetric for the trapezoid weights W (node images of Neumann
    // faces): lambda = W mu with dL mu = W^-1 g
    if (!P || !g || !lambda || !o) return SGML_E_ARG;
    if (o->max_cycles < 1 || !(o->tol >= 0.0)) return SGML_E_ARG;
    if (o->precision != SGML_FP64 && o->precision != SGML_MIXED) return SGML_E_ARG;
    if (o->precision == SGML_MIXED && P->precision != SGML_MIXED) return SGML_E_WORKSPACE;
    if (o->schedule != SGML_SCHEDULE_ONCE && o->schedule != SGML_SCHEDULE_EACH) return SGML_E_ARG;
    if (lambda == g) return SGML_E_ARG;
    if (!P->ws) return SGML_E_WORKSPACE;
    SGML_HIP(hipSetDevice(P->device));
    hipStream_t st = (hipStream_t)stream;
    sgml_status rc = o->precision == SGML_MIXED ? run_solve<float>(P, g, nullptr, lambda, o, st, stats, true)
                                                : run_solve<double>(P, g, nullptr, lambda, o, st, stats, true);
    if (stats) stats->status = rc;
    return rc;
}

sgml_status sgml_neumann_source(sgml_plan *P, const double *f, const double *const *flux, double *f_out,
                                void *stream)
{
    if (!P || !f || !flux || !f_out) return SGML_E_ARG;
    SGML_HIP(hipSetDevice(P->device));
    FaceData fd;
    for (int q = 0; q < 6; ++q)
        fd.g[q] = (q < 2 * P->dim && !(P->dir & (1u << q))) ? flux[q] : nullptr;
    launch_neumann_source(P->var, P->level(0), f, fd, P->sigma, P->h, f_out, (hipStream_t)stream);
    SGML_HIP(hipGetLastError());
    return SGML_OK;
}

sgml_status sgml_coeff_grad(sgml_plan *P, const double *u, const double *lambda, double *grad, void *stream)
{
    if (!P || !u || !lambda || !grad) return SGML_E_ARG;
    SGML_HIP(hipSetDevice(P->device));
    launch_coeff_grad(P->var, P->level(0), u, lambda, grad, (hipStream_t)stream);
    SGML_HIP(hipGetLastError());
    return SGML_OK;
}

sgml_status sgml_schedule(int n, int n_r, int schedule, int *level, int *count, int cap, int *len)
{
    if (n < 1 || n > 30 || !len || cap < 0 || (cap > 0 && (!level || !count))) return SGML_E_ARG;
    if (schedule != SGML_SCHEDULE_ONCE && schedule != SGML_SCHEDULE_EACH) return SGML_E_ARG;
    std::vector<int> lev, cnt;
    build_schedule(n, n_r, schedule, lev, cnt);
    for (int v = 0; v < (int)lev.size() && v < cap; ++v) {
        level[v] = lev[v];
        count[v] = cnt[v];
    }
    *len = (int)lev.size();
    return SGML_OK;
}

const char *sgml_status_string(sgml_status s)
{
    switch (s) {
    case SGML_OK: return "ok";
    case SGML_E_ARG: return "invalid argument";
    case SGML_E_SHAPE: return "unsupported grid shape";
    case SGML_E_WORKSPACE: return "workspace missing, too small or misaligned";
    case SGML_E_HIP: return "HIP runtime error";
    case SGML_E_DIVERGED: return "diverged";
    case SGML_E_STAGNATED: return "stagnated";
    case SGML_E_MAXCYCLES: return "maximum number of cycles reached";
    case SGML_E_UNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

void sgml_plan_destroy(sgml_plan *P)
{
    if (!P) return;
    for (auto &cg : P->graph)
        if (cg.exec) (void)hipGraphExecDestroy(cg.exec);
    if (P->cap_st) (void)hipStreamDestroy(P->cap_st);
    for (sgml_plan *Q : P->sub) sgml_plan_destroy(Q);
    for (hipStream_t q : P->sub_st) (void)hipStreamDestroy(q);
    for (hipEvent_t e : P->sub_ev) (void)hipEventDestroy(e);
    (void)hipEventDestroy(P->ev0);
    (void)hipEventDestroy(P->ev1);
    for (hipEvent_t e : P->pev) (void)hipEventDestroy(e);
    (void)hipHostFree(P->ops_host);
    (void)hipHostFree(P->lops_host);
    (void)hipHostFree(P->xfer_host);
    (void)hipHostFree(P->levels_host);
    (void)hipHostFree(P->host);
    delete P;
}

}  // extern "C"
