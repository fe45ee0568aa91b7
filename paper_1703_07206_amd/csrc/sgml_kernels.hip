// sgml_kernels.hip -- HIP kernels of the SGML solver for gfx950.
//
// Every routine of the method is bandwidth bound (a few flops per byte), so
// the kernels are plain coalesced streaming kernels: one lane per node along
// x (the contiguous axis), 64-lane wavefronts covering 64 consecutive nodes
// of a row.  Stencil neighbours are re-read through L1/L2, which holds the
// rows above and below.
//
// Levels (Sec. 2): level nu holds the nodes whose indices are multiples of
// lam = 2^nu.  The full grid keeps level 0; every coarser level is stored
// compactly (m^d values, m = 2^(n-nu) + 1), so that a relaxation at level nu
// reads and writes only its own nodes.  Algorithm 2 interpolates each
// variation of level nu to all other nodes; here that interpolation is
// deferred: a level keeps its values, and when the schedule moves to the next
// finer level the pending variation (coarse value minus the finer level's
// stale copy at the coarse nodes) is interpolated once (k_prolong).  Since a
// relaxation at level nu reads only level-nu nodes and the hat interpolation
// is linear and nested (interpolating level nu to level nu-1 and then on
// reproduces the direct interpolation), this gives the values the full-grid
// formulation gives, up to rounding order.
#include "sgml_device.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <utility>

namespace sgml {

namespace {

constexpr int BX = 64;  // one wavefront along x
constexpr int BY = 4;

__device__ __forceinline__ void block_max(unsigned long long v, unsigned long long *out)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    __shared__ unsigned long long wmax[16];
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthr = blockDim.x * blockDim.y * blockDim.z;
    if ((tid & 63) == 0) wmax[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < (nthr + 63) / 64; ++w) v = wmax[w] > v ? wmax[w] : v;
        const unsigned b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        if (v) atomicMax(out + (b % kRedSlots) * kRedStride, v);
    }
    __syncthreads();  // wmax may be reused by a second reduction in the same kernel
}

// Stride-lam finite-difference operator of L = div(sigma grad) + a at a node
// of a compact level array (eq. (5) and the axis molecule):
//   Lu = scale * sum_k w_k (sigma_k + sigma_c)/2 (u_k - u_c) + a u_c,
//   D  = scale * sum_k w_k (sigma_k + sigma_c)/2 - a,
// w = 1 for face neighbours, 1/2 for edge and 1/3 for corner neighbours
// (radial), scale = C/(lam h)^2 with C = 1 (axis) or 2d/(3^d - 1) (radial).
// Differences are taken before summing, per neighbour class.
template <typename T, int DIM, int RAD, int SIG, typename I = size_t>
__device__ __forceinline__ void stencil(const T *__restrict__ u, const T *__restrict__ sig, int i,
                                        int j, int k, int m, T scale, T a, T &Lu, T &D)
{
    const I c = lin_as<I>(i, j, k, m);
    const T uc = u[c];
    const T sc = SIG ? sig[c] : T(1);
    T acc[3] = {T(0), T(0), T(0)};
    T ds[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz) {
        const int kk = DIM == 3 ? mir(k + dz, m) : 0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const int jj = mir(j + dy, m);
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int cls = (dx != 0) + (dy != 0) + (dz != 0);
                if (cls == 0 || (!RAD && cls != 1)) continue;
                const I q = lin_as<I>(mir(i + dx, m), jj, kk, m);
                const T du = u[q] - uc;
                if (SIG) {
                    const T t = sig[q] + sc;
                    acc[cls - 1] += t * du;
                    ds[cls - 1] += t;
                } else {
                    acc[cls - 1] += du;
                }
            }
        }
    }
    const T third = T(1.0 / 3.0);
    if (SIG) {
        const T sw = acc[0] + T(0.5) * acc[1] + third * acc[2];
        const T dw = ds[0] + T(0.5) * ds[1] + third * ds[2];
        Lu = scale * T(0.5) * sw + a * uc;
        D = scale * T(0.5) * dw - a;
    } else {
        constexpr int n2 = RAD ? (DIM == 3 ? 12 : 4) : 0;
        constexpr int n3 = (RAD && DIM == 3) ? 8 : 0;
        const T W = T(2 * DIM) + T(0.5) * T(n2) + third * T(n3);
        const T sw = acc[0] + T(0.5) * acc[1] + third * acc[2];
        Lu = scale * sw + a * uc;
        D = scale * W - a;
    }
}

// Full-grid operator in FP64 on a field whose Dirichlet-node values are
// replaced by G (or 0): used by the residual recurrence.  `val` maps a node
// to its value.
template <int DIM, int RAD, int SIG, typename F>
__device__ __forceinline__ double stencil_full(F val, const double *__restrict__ sig, int i, int j,
                                               int k, int m, unsigned dir, double scale, double a)
{
    const double uc = val(i, j, k);
    const double sc = SIG ? sig[lin(i, j, k, m)] : 1.0;
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz) {
        const int kk = DIM == 3 ? mir(k + dz, m) : 0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const int jj = mir(j + dy, m);
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int cls = (dx != 0) + (dy != 0) + (dz != 0);
                if (cls == 0 || (!RAD && cls != 1)) continue;
                const int ii = mir(i + dx, m);
                const double du = val(ii, jj, kk) - uc;
                if (SIG)
                    acc[cls - 1] += (sig[lin(ii, jj, kk, m)] + sc) * du;
                else
                    acc[cls - 1] += du;
            }
        }
    }
    const double sw = acc[0] + 0.5 * acc[1] + (1.0 / 3.0) * acc[2];
    (void)dir;
    return (SIG ? 0.5 * scale * sw : scale * sw) + a * uc;
}

template <int DIM>
__device__ __forceinline__ bool node_of(int m, int &i, int &j, int &k)
{
    i = blockIdx.x * blockDim.x + threadIdx.x;
    j = blockIdx.y * blockDim.y + threadIdx.y;
    k = DIM == 3 ? (int)blockIdx.z : 0;
    return i < m && j < m;
}

dim3 grid_of(int dim, int m)
{
    return dim3((m + BX - 1) / BX, (m + BY - 1) / BY, dim == 3 ? m : 1);
}

// ------------------------------------------------------------------ kernels

template <typename T>
__global__ void k_fill(T *p, size_t count, T value)
{
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; t < count; t += stride) p[t] = value;
}

// One relaxation (forward-Euler step of eq. (2), Algorithm 2) of one node of
// a level, Jacobi style: the new value from ein.  Unknowns:
// e + theta/D (dL e - g).  Dirichlet nodes take the prescribed value G (the
// variation G - e of Sec. 2) or 0.  rb: the bits of |dL e - g| (0 at
// Dirichlet nodes).
template <typename T, int DIM, int RAD, int SIG, typename I = size_t>
__device__ __forceinline__ T sweep_value(const T *__restrict__ ein, const T *__restrict__ g,
                                         const T *__restrict__ sig, const double *__restrict__ G,
                                         const Level &L, int i, int j, int k, unsigned long long &rb)
{
    const I c = lin_as<I>(i, j, k, L.m);
    if (is_dir<DIM>(i, j, k, L.m, L.dir)) {
        rb = 0;
        return G ? (T)G[lin(i * L.lam, j * L.lam, k * L.lam, L.N)] : T(0);
    }
    T Lu, D;
    stencil<T, DIM, RAD, SIG, I>(ein, sig, i, j, k, L.m, (T)L.scale, (T)L.a, Lu, D);
    const T r = Lu - g[c];
    rb = dbits((double)r);
    return ein[c] + ((T)L.theta / D) * r;
}

// sweep_value for a level held in LDS: 32-bit indices, the level constants
// already in T, theta/D precomputed when sigma = 1 (D is then the same at
// every node), and the residual bits only when they are recorded.
template <typename T>
struct SweepConst {
    T scale, a, theta, step;  // step = theta / D (sigma = 1)
};

template <typename T, int DIM, int RAD, int SIG>
__device__ __forceinline__ T lds_sweep_value(const T *__restrict__ ein, const T *__restrict__ g,
                                             const T *__restrict__ sig, const double *__restrict__ G,
                                             const Level &L, const SweepConst<T> &K, int i, int j, int k,
                                             bool want_rb, unsigned long long &rb)
{
    const int c = lin_as<int>(i, j, k, L.m);
    if (is_dir<DIM>(i, j, k, L.m, L.dir)) return G ? (T)G[lin(i * L.lam, j * L.lam, k * L.lam, L.N)] : T(0);
    T Lu, D;
    stencil<T, DIM, RAD, SIG, int>(ein, sig, i, j, k, L.m, K.scale, K.a, Lu, D);
    const T r = Lu - g[c];
    if (want_rb) {
        const unsigned long long b = dbits((double)r);
        rb = b > rb ? b : rb;
    }
    return ein[c] + (SIG ? K.theta / D : K.step) * r;
}

// The diagonal D of the operator when sigma = 1 (see stencil).
template <typename T, int DIM, int RAD>
__device__ __forceinline__ T const_diag(T scale, T a)
{
    constexpr int n2 = RAD ? (DIM == 3 ? 12 : 4) : 0;
    constexpr int n3 = (RAD && DIM == 3) ? 8 : 0;
    const T W = T(2 * DIM) + T(0.5) * T(n2) + T(1.0 / 3.0) * T(n3);
    return scale * W - a;
}

template <typename T, int DIM, int RAD, int SIG>
__device__ __forceinline__ unsigned long long sweep_node(const T *__restrict__ ein, T *__restrict__ eout,
                                                         const T *__restrict__ g, const T *__restrict__ sig,
                                                         const double *__restrict__ G, const Level &L,
                                                         int i, int j, int k)
{
    unsigned long long rb;
    eout[lin(i, j, k, L.m)] = sweep_value<T, DIM, RAD, SIG>(ein, g, sig, G, L, i, j, k, rb);
    return rb;
}

// Interpolation of the pending variation of level nu (compact, mc nodes per
// axis) to node (i,j,k) of level nu-1 (mf = 2 mc - 1): the pending variation
// at a coarse node X is ec(X) - ef_in(2X) (zero stale values on the level's
// first visit of a cycle); coarse nodes take ec directly, the others add the
// multilinear (tensor hat) interpolation -- the mean of the 2, 4 or 8
// enclosing coarse nodes.
template <typename T, int DIM, typename I = size_t>
__device__ __forceinline__ T prolong_value(const T *__restrict__ ec, const T *__restrict__ efin, int mc,
                                           int first, int i, int j, int k)
{
    const int mf = 2 * mc - 1;
    const int ci = i >> 1, cj = j >> 1, ck = k >> 1;
    const int oi = i & 1, oj = j & 1, ok = DIM == 3 ? (k & 1) : 0;
    if (!(oi | oj | ok)) return ec[lin_as<I>(ci, cj, ck, mc)];
    T acc = T(0);
#pragma unroll
    for (int c = 0; c <= (DIM == 3 ? 1 : 0); ++c) {
        if (c && !ok) continue;
#pragma unroll
        for (int b = 0; b <= 1; ++b) {
            if (b && !oj) continue;
#pragma unroll
            for (int a = 0; a <= 1; ++a) {
                if (a && !oi) continue;
                const int X = ci + a, Y = cj + b, Z = ck + c;
                T p = ec[lin_as<I>(X, Y, Z, mc)];
                if (!first) p -= efin[lin_as<I>(2 * X, 2 * Y, 2 * Z, mf)];
                acc += p;
            }
        }
    }
    const T w = T(1) / T(1 << (oi + oj + ok));
    return (first ? T(0) : efin[lin_as<I>(i, j, k, mf)]) + w * acc;
}

template <typename T, int DIM>
__device__ __forceinline__ void prolong_node(const T *__restrict__ ec, const T *__restrict__ efin,
                                             T *__restrict__ efout, int mc, int first, int i, int j, int k)
{
    efout[lin(i, j, k, 2 * mc - 1)] = prolong_value<T, DIM>(ec, efin, mc, first, i, j, k);
}

// Values of level nu-1 at the level-nu nodes (the schedule climbs a level).
template <typename T>
__device__ __forceinline__ void inject_node(const T *__restrict__ ef, T *__restrict__ ec, int mc, int i, int j,
                                            int k)
{
    ec[lin(i, j, k, mc)] = ef[lin(2 * i, 2 * j, 2 * k, 2 * mc - 1)];
}

// One restriction step, eq. (3) / eq. (4): the coarse node X averages the
// fine level's 3^d neighbours of 2X with weights hat(p/2) per axis over 2^d;
// samples outside the grid are images.  Summed in the same order (z, y, x
// outer to inner) with exactly representable weights.
template <typename Tin, typename Tout, int DIM, typename I = size_t>
__device__ __forceinline__ Tout restrict_value(const Tin *__restrict__ fine, int mc, int i, int j, int k)
{
    using Acc = typename std::conditional<sizeof(Tin) == 8 || sizeof(Tout) == 8, double, float>::type;
    const int mf = 2 * mc - 1;
    Acc acc = Acc(0);
#pragma unroll
    for (int r = (DIM == 3 ? -1 : 0); r <= (DIM == 3 ? 1 : 0); ++r) {
        const int kk = DIM == 3 ? mir(2 * k + r, mf) : 0;
        const Acc wr = r == 0 ? Acc(1) : Acc(0.5);
#pragma unroll
        for (int q = -1; q <= 1; ++q) {
            const int jj = mir(2 * j + q, mf);
            const Acc wq = q == 0 ? Acc(1) : Acc(0.5);
#pragma unroll
            for (int p = -1; p <= 1; ++p) {
                const Acc wp = p == 0 ? Acc(1) : Acc(0.5);
                acc += (wp * wq * wr) * (Acc)fine[lin_as<I>(mir(2 * i + p, mf), jj, kk, mf)];
            }
        }
    }
    return (Tout)(acc / Acc(1 << DIM));
}

template <typename Tin, typename Tout, int DIM>
__device__ __forceinline__ void restrict_node(const Tin *__restrict__ fine, Tout *__restrict__ coarse, int mc,
                                              int i, int j, int k)
{
    coarse[lin(i, j, k, mc)] = restrict_value<Tin, Tout, DIM>(fine, mc, i, j, k);
}

template <typename T, int DIM, int RAD, int SIG>
__global__ __launch_bounds__(256) void k_sweep(const T *__restrict__ ein, T *__restrict__ eout,
                                               const T *__restrict__ g, const T *__restrict__ sig,
                                               const double *__restrict__ G, Level L,
                                               unsigned long long *__restrict__ pres)
{
    int i, j, k;
    unsigned long long rb = 0;
    if (node_of<DIM>(L.m, i, j, k)) rb = sweep_node<T, DIM, RAD, SIG>(ein, eout, g, sig, G, L, i, j, k);
    if (pres) block_max(rb, pres);
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_prolong(const T *__restrict__ ec, const T *__restrict__ efin,
                                                 T *__restrict__ efout, int mc, int first)
{
    int i, j, k;
    if (node_of<DIM>(2 * mc - 1, i, j, k)) prolong_node<T, DIM>(ec, efin, efout, mc, first, i, j, k);
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_inject(const T *__restrict__ ef, T *__restrict__ ec, int mc)
{
    int i, j, k;
    if (node_of<DIM>(mc, i, j, k)) inject_node<T>(ef, ec, mc, i, j, k);
}

template <typename Tin, typename Tout, int DIM>
__global__ __launch_bounds__(256) void k_restrict(const Tin *__restrict__ fine, Tout *__restrict__ coarse,
                                                  int mc)
{
    int i, j, k;
    if (node_of<DIM>(mc, i, j, k)) restrict_node<Tin, Tout, DIM>(fine, coarse, mc, i, j, k);
}

// The coarse levels of a cycle in one launch of one workgroup: a run of
// consecutive operations (restriction, zero fill, relaxation, interpolation,
// injection) on levels small enough to live in L2, executed in order with a
// workgroup barrier between operations.  Waves stride over rows, lanes over
// the nodes of a row.
template <typename T, int DIM, int RAD, int SIG>
__global__ __launch_bounds__(coarse_threads(DIM)) void k_coarse(const CoarseOp *__restrict__ ops, int nops,
                                                           const Level *__restrict__ levels,
                                                           const double *__restrict__ G,
                                                           unsigned long long *__restrict__ targets)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int waves = coarse_threads(DIM) / 64;
    for (int o = 0; o < nops; ++o) {
        const CoarseOp op = ops[o];
        const int m = op.m;
        const int rows = DIM == 3 ? m * m : m;
        unsigned long long rb = 0;
        for (int r = wave; r < rows; r += waves) {
            const int j = DIM == 3 ? r % m : r, k = DIM == 3 ? r / m : 0;
            for (int i = lane; i < m; i += 64) {
                switch (op.kind) {
                case kOpFill:
                    ((T *)op.out)[lin(i, j, k, m)] = T(0);
                    break;
                case kOpSweep: {
                    const unsigned long long b = sweep_node<T, DIM, RAD, SIG>(
                        (const T *)op.in0, (T *)op.out, (const T *)op.in1, (const T *)op.in2, G,
                        levels[op.level], i, j, k);
                    rb = b > rb ? b : rb;
                    break;
                }
                case kOpProlong:
                    prolong_node<T, DIM>((const T *)op.in0, (const T *)op.in1, (T *)op.out, (m + 1) / 2,
                                         op.first, i, j, k);
                    break;
                case kOpInject:
                    inject_node<T>((const T *)op.in0, (T *)op.out, m, i, j, k);
                    break;
                default:  // kOpRestrict
                    restrict_node<T, T, DIM>((const T *)op.in0, (T *)op.out, m, i, j, k);
                    break;
                }
            }
        }
        if (op.kind == kOpSweep && op.target >= 0) block_max(rb, targets + (size_t)op.target * kRedWords);
        __syncthreads();
    }
}

// The coarse run of k_coarse with its level arrays in LDS: the arrays the run
// reads before writing are copied in, every operation works LDS to LDS (one
// barrier each), and the arrays read after the run are copied back.  The
// operations' headers are staged in LDS too (one per thread, all at once),
// with the relaxation constants precomputed on the host; the next header is
// read while the current operation runs.  Thread
// t owns nodes t, t + threads, ... of the level an operation writes; it
// computes all of them before storing any, so the loads of a thread issue
// together.  Each operation reads one buffer of a level and writes the other
// (or another level), as in k_coarse.
//
// Operations on small levels (at most one node per lane of a wavefront,
// flagged solo by the host) run on wavefront 0 alone, back to back, ordered
// by waiting on its own LDS accesses; the other wavefronts skip them and
// meet wavefront 0 at the barrier that closes the section (op.sync).  A
// barrier costs every wavefront's issue slots, and on these levels one
// wavefront has all the parallelism there is.
template <typename T, int DIM, int RAD, int SIG>
__global__ __launch_bounds__(coarse_threads(DIM)) void k_coarse_lds(const LdsOp *__restrict__ ops, int nops,
                                                               int hdr_off, const LdsXfer *__restrict__ xfer,
                                                               int nload, int nstore,
                                                               const double *__restrict__ G,
                                                               unsigned long long *__restrict__ targets)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    using Hdr = LdsOpHdr<T>;
    T *sm = reinterpret_cast<T *>(lds_raw);
    Hdr *hdr = reinterpret_cast<Hdr *>(lds_raw + hdr_off);
    constexpr int NT = coarse_threads(DIM);
    constexpr int KMAX = coarse_lds_nodes(DIM) / NT;
    const int tid = threadIdx.x;
    for (int q = tid; q < nops; q += NT) {
        const LdsOp &g = ops[q];
        Hdr h;
        h.kind = g.kind;
        h.m = g.m;
        h.nodes = g.nodes;
        h.target = g.target;
        h.solo = g.solo;
        h.sync = g.sync;
        h.in0 = g.in0;
        h.in1 = g.in1;
        h.out = g.out;
        h.first = g.first;
        h.lam = g.L.lam;
        h.N = g.L.N;
        h.dir = g.L.dir;
        h.inv_m = g.inv_m;
        h.sig = g.sig;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if constexpr (sizeof(T) == 4) h.k[c] = g.kf[c];
            else h.k[c] = g.kd[c];
        }
        hdr[q] = h;
    }
    for (int x = 0; x < nload; ++x) {
        const T *src = static_cast<const T *>(xfer[x].ptr);
        const int off = xfer[x].off, count = xfer[x].count;
#pragma unroll 4
        for (int t = tid; t < count; t += NT) sm[off + t] = src[t];
    }
    __syncthreads();
    const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63);  // first node of this wave
    const int lane = tid & 63;
    Hdr op = hdr[0];
    for (int o = 0; o < nops; ++o) {
        const Hdr nxt = hdr[o + 1 < nops ? o + 1 : o];  // in flight during this operation
        // uniform over the workgroup: the fields the control flow uses go to scalars
        const int kind = __builtin_amdgcn_readfirstlane(op.kind);
        const int m = __builtin_amdgcn_readfirstlane(op.m);
        const int nodes = __builtin_amdgcn_readfirstlane(op.nodes);
        const int target = __builtin_amdgcn_readfirstlane(op.target);
        const int solo = __builtin_amdgcn_readfirstlane(op.solo);
        const int sync = __builtin_amdgcn_readfirstlane(op.sync);
        // nodes of this thread: base, base + stride, ...; first: of the wave
        const int base = solo ? lane : tid, stride = solo ? 64 : NT, first_node = solo ? 0 : wbase;
        unsigned long long rb = 0;
        if (solo ? wbase == 0 : wbase < nodes) {  // the other waves only meet the barrier
            const float inv = op.inv_m;
            const int in0 = __builtin_amdgcn_readfirstlane(op.in0);
            const int in1 = __builtin_amdgcn_readfirstlane(op.in1);
            const int first = __builtin_amdgcn_readfirstlane(op.first);
            // node t = (k m + j) m + i; (t + 1/2) / m is at least 1/(2m) away
            // from an integer, far beyond the float error for t < 2^13
            auto decode = [&](int t, int &i, int &j, int &k) {
                const int q = (int)(((float)t + 0.5f) * inv);
                i = t - q * m;
                if (DIM == 3) {
                    k = (int)(((float)q + 0.5f) * inv);
                    j = q - k * m;
                } else {
                    j = q;
                    k = 0;
                }
            };
            T val[KMAX];
            // f(t, i, j, k) -> value of node t, for the nodes of this thread
            auto each = [&](auto f) {
#pragma unroll
                for (int q = 0; q < KMAX; ++q) {
                    const int t = base + q * stride;
                    if (first_node + q * stride < nodes && t < nodes) {
                        int i, j, k;
                        decode(t, i, j, k);
                        val[q] = f(t, i, j, k);
                    }
                }
            };
            switch (kind) {
            case kOpSweep: {
                const T *ein = sm + in0, *g = sm + in1;
                const T *sig = static_cast<const T *>(op.sig);
                Level L;  // the geometry lds_sweep_value reads; the constants are in K
                L.scale = L.a = L.theta = 0.0;
                L.m = m;
                L.lam = __builtin_amdgcn_readfirstlane(op.lam);
                L.N = __builtin_amdgcn_readfirstlane(op.N);
                L.dir = __builtin_amdgcn_readfirstlane(op.dir);
                const auto kc = [&](int q) -> T { return op.k[q]; };
                SweepConst<T> K;
                K.scale = kc(kKScale);
                K.a = kc(kKA);
                K.theta = kc(kKTheta);
                K.step = kc(kKStep);
                const bool want_rb = target >= 0;
                if (DIM == 2 && !RAD && !SIG) {
                    // 5-point, sigma = 1: e' = (1 - theta) e + beta (sum of neighbours) - gamma g,
                    // beta = theta scale / D, gamma = theta / D; images at the faces
                    const T omt = kc(kKOmt), beta = kc(kKBeta), gamma = K.step, aw = kc(kKAw);
                    const unsigned dir = L.dir;
                    each([&](int t, int i, int j, int) {
                        const int il = i > 0 ? t - 1 : t + 1, ir = i < m - 1 ? t + 1 : t - 1;
                        const int ju = j > 0 ? t - m : t + m, jd = j < m - 1 ? t + m : t - m;
                        const T c = ein[t], gt = g[t];
                        const T sum = (ein[il] + ein[ir]) + (ein[ju] + ein[jd]);
                        const bool d = (((dir & 1u) != 0) & (i == 0)) | (((dir & 2u) != 0) & (i == m - 1)) |
                                       (((dir & 4u) != 0) & (j == 0)) | (((dir & 8u) != 0) & (j == m - 1));
                        if (want_rb && !d) {
                            const unsigned long long b = dbits((double)(K.scale * sum + aw * c - gt));
                            rb = b > rb ? b : rb;
                        }
                        if (d) return G ? (T)G[lin(i * L.lam, j * L.lam, 0, L.N)] : T(0);
                        return omt * c + (beta * sum - gamma * gt);
                    });
                } else {
                    each([&](int, int i, int j, int k) {
                        return lds_sweep_value<T, DIM, RAD, SIG>(ein, g, sig, G, L, K, i, j, k, want_rb, rb);
                    });
                }
                break;
            }
            case kOpProlong: {
                const T *ec = sm + in0, *efin = sm + in1;
                const int mc = (m + 1) / 2;
                each([&](int, int i, int j, int k) { return prolong_value<T, DIM, int>(ec, efin, mc, first, i, j, k); });
                break;
            }
            case kOpInject: {
                const T *ef = sm + in0;
                const int mf = 2 * m - 1;
                each([&](int, int i, int j, int k) { return ef[lin_as<int>(2 * i, 2 * j, 2 * k, mf)]; });
                break;
            }
            case kOpRestrict: {
                const T *fine = sm + in0;
                each([&](int, int i, int j, int k) { return restrict_value<T, T, DIM, int>(fine, m, i, j, k); });
                break;
            }
            default:  // kOpFill
                each([&](int, int, int, int) { return T(0); });
                break;
            }
            T *out = sm + __builtin_amdgcn_readfirstlane(op.out);
#pragma unroll
            for (int q = 0; q < KMAX; ++q) {
                const int t = base + q * stride;
                if (first_node + q * stride < nodes && t < nodes) out[t] = val[q];
            }
        }
        if (kind == kOpSweep && target >= 0) block_max(rb, targets + (size_t)target * kRedWords);  // not solo
        if (sync)
            __syncthreads();
        else  // solo, within a section: wavefront 0's writes complete before its next reads
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        op = nxt;
    }
    for (int x = nload; x < nload + nstore; ++x) {
        T *dst = static_cast<T *>(xfer[x].ptr);
        const int off = xfer[x].off, count = xfer[x].count;
#pragma unroll 4
        for (int t = tid; t < count; t += NT) dst[t] = sm[off + t];
    }
}

template <typename Tin, typename Tout>
__global__ void k_convert(const Tin *__restrict__ in, Tout *__restrict__ out, size_t count)
{
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; t < count; t += stride) out[t] = (Tout)in[t];
}

// End of a cycle (recurrence of Sec. 2), FP64 on the full grid:
//   e = escale * E (E at Dirichlet nodes replaced by G in the first cycle, 0
//   after), u += e, and at unknowns s -= dL_1 e; s = 0 at Dirichlet nodes.
//   norm: max |s| over unknowns.  shat (optional): next cycle's source,
//   shat = (T)(s * shat_scale).
template <typename T, int DIM, int RAD, int SIG>
__global__ __launch_bounds__(256) void k_boundary(const T *__restrict__ E, double escale,
                                                  const double *__restrict__ G,
                                                  const double *__restrict__ sigma, double *__restrict__ u,
                                                  double *__restrict__ s, T *__restrict__ shat,
                                                  double shat_scale, Level L,
                                                  unsigned long long *__restrict__ norm)
{
    int i, j, k;
    unsigned long long rb = 0;
    const int m = L.m;
    if (node_of<DIM>(m, i, j, k)) {
        const size_t c = lin(i, j, k, m);
        auto val = [&](int a, int b, int d) -> double {
            if (is_dir<DIM>(a, b, d, m, L.dir)) return G ? G[lin(a, b, d, m)] : 0.0;
            return escale * (double)E[lin(a, b, d, m)];
        };
        if (is_dir<DIM>(i, j, k, m, L.dir)) {
            if (G) u[c] += G[c];
            s[c] = 0.0;
            if (shat) shat[c] = T(0);
        } else {
            const double Le = stencil_full<DIM, RAD, SIG>(val, sigma, i, j, k, m, L.dir, L.scale, L.a);
            const double sn = s[c] - Le;
            u[c] += escale * (double)E[c];
            s[c] = sn;
            if (shat) shat[c] = (T)(sn * shat_scale);
            rb = dbits(sn);
        }
    }
    block_max(rb, norm);
}

// Trapezoid weight of node (i, j, k): 1/2 for every Neumann face (a face not
// in dir) it lies on.  W dL is symmetric under the node images of Neumann
// faces, so dL^T = W dL W^-1.
template <int DIM>
__device__ __forceinline__ double trap_weight(int i, int j, int k, int m, unsigned dir)
{
    double w = 1.0;
    if (i == 0 && !(dir & 1u)) w *= 0.5;
    if (i == m - 1 && !(dir & 2u)) w *= 0.5;
    if (j == 0 && !(dir & 4u)) w *= 0.5;
    if (j == m - 1 && !(dir & 8u)) w *= 0.5;
    if (DIM == 3) {
        if (k == 0 && !(dir & 16u)) w *= 0.5;
        if (k == m - 1 && !(dir & 32u)) w *= 0.5;
    }
    return w;
}

// Start of a solve: u = 0, s = f at unknowns (0 at Dirichlet nodes), s32
// (if not null) = s in FP32, and norm0 = max |f - dL_1 u_init| with u_init =
// G on Dirichlet nodes, 0 else.  WS: the source is W^-1 f (first step of the
// transposed solve).
template <int DIM, int RAD, int SIG, bool WS>
__global__ __launch_bounds__(256) void k_init(const double *__restrict__ f, const double *__restrict__ G,
                                              const double *__restrict__ sigma, double *__restrict__ s,
                                              double *__restrict__ u, float *__restrict__ s32, Level L,
                                              unsigned long long *__restrict__ norm0)
{
    int i, j, k;
    unsigned long long rb = 0;
    const int m = L.m;
    if (node_of<DIM>(m, i, j, k)) {
        const size_t c = lin(i, j, k, m);
        u[c] = 0.0;
        if (is_dir<DIM>(i, j, k, m, L.dir)) {
            s[c] = 0.0;
            if (s32) s32[c] = 0.0f;
        } else {
            auto val = [&](int a, int b, int d) -> double {
                return (G && is_dir<DIM>(a, b, d, m, L.dir)) ? G[lin(a, b, d, m)] : 0.0;
            };
            const double Lb = stencil_full<DIM, RAD, SIG>(val, sigma, i, j, k, m, L.dir, L.scale, L.a);
            const double fc = WS ? f[c] / trap_weight<DIM>(i, j, k, m, L.dir) : f[c];
            s[c] = fc;
            if (s32) s32[c] = (float)fc;
            rb = dbits(fc - Lb);
        }
    }
    block_max(rb, norm0);
}

// u = W u (last step of the transposed solve).
template <int DIM>
__global__ __launch_bounds__(256) void k_trap_scale(double *__restrict__ u, Level L)
{
    int i, j, k;
    if (!node_of<DIM>(L.m, i, j, k)) return;
    u[lin(i, j, k, L.m)] *= trap_weight<DIM>(i, j, k, L.m, L.dir);
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_source_cast(const double *__restrict__ s, T *__restrict__ shat,
                                                     double scale, int m)
{
    int i, j, k;
    if (!node_of<DIM>(m, i, j, k)) return;
    const size_t c = lin(i, j, k, m);
    shat[c] = (T)(s[c] * scale);
}

template <int DIM>
__global__ __launch_bounds__(256) void k_set_dirichlet(const double *__restrict__ G, double *__restrict__ u,
                                                       Level L)
{
    int i, j, k;
    if (!node_of<DIM>(L.m, i, j, k)) return;
    if (is_dir<DIM>(i, j, k, L.m, L.dir)) {
        const size_t c = lin(i, j, k, L.m);
        u[c] = G ? G[c] : 0.0;
    }
}

// r = f - dL_1 u at unknowns (0 at Dirichlet nodes); rmax = max |r|;
// norm0 as in k_init.
template <int DIM, int RAD, int SIG>
__global__ __launch_bounds__(256) void k_residual(const double *__restrict__ f, const double *__restrict__ G,
                                                  const double *__restrict__ sigma,
                                                  const double *__restrict__ u, double *__restrict__ r,
                                                  Level L, unsigned long long *__restrict__ rmax,
                                                  unsigned long long *__restrict__ norm0)
{
    int i, j, k;
    unsigned long long rb = 0, nb = 0;
    const int m = L.m;
    if (node_of<DIM>(m, i, j, k)) {
        const size_t c = lin(i, j, k, m);
        if (is_dir<DIM>(i, j, k, m, L.dir)) {
            if (r) r[c] = 0.0;
        } else {
            auto val = [&](int a, int b, int d) -> double { return u[lin(a, b, d, m)]; };
            auto val0 = [&](int a, int b, int d) -> double {
                return (G && is_dir<DIM>(a, b, d, m, L.dir)) ? G[lin(a, b, d, m)] : 0.0;
            };
            const double rr = f[c] - stencil_full<DIM, RAD, SIG>(val, sigma, i, j, k, m, L.dir, L.scale, L.a);
            const double r0 = f[c] - stencil_full<DIM, RAD, SIG>(val0, sigma, i, j, k, m, L.dir, L.scale, L.a);
            if (r) r[c] = rr;
            rb = dbits(rr);
            nb = dbits(r0);
        }
    }
    block_max(rb, rmax);
    block_max(nb, norm0);
}

// dLoss/dsigma_m = -sum_x lam_x d(dL u)_x / dsigma_m (lam = 0 on Dirichlet
// nodes).  Row x holds scale w_k (sigma_s + sigma_x)/2 (u_s - u_x) for each
// neighbour k, s the node it samples (an image across a Neumann face), so
// sigma_m enters
//   (a) its own row:  scale/2 sum_k w_k (u_s(m,k) - u_m), times lam_m;
//   (b) every row x whose neighbour k samples m:  scale/2 w_k (u_m - u_x),
//       times lam_x.  x + d_k is then m itself or one of m's images (per
//       axis -1 for m = 1, m for m = m - 2: the positions that reflect onto m).
// Nodes of Dirichlet faces have lam = 0, so their rows drop out by themselves.
template <int DIM, int RAD>
__global__ __launch_bounds__(256) void k_coeff_grad(const double *__restrict__ u,
                                                    const double *__restrict__ lam,
                                                    double *__restrict__ grad, Level L)
{
    int i, j, k;
    const int m = L.m;
    if (!node_of<DIM>(m, i, j, k)) return;
    const size_t c = lin(i, j, k, m);
    const double uc = u[c], lc = lam[c];
    // positions reflecting onto this node, per axis (the node itself first)
    int px[3], py[3], pz[3], nx = 0, ny = 0, nz = 0;
    auto images = [&](int v, int *p, int &np) {
        p[np++] = v;
        if (v == 1) p[np++] = -1;
        if (v == m - 2) p[np++] = m;
    };
    images(i, px, nx);
    images(j, py, ny);
    if (DIM == 3) images(k, pz, nz);
    else pz[nz++] = 0;
    double own[3] = {0.0, 0.0, 0.0}, oth[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz) {
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int cls = (dx != 0) + (dy != 0) + (dz != 0);
                if (cls == 0 || (!RAD && cls != 1)) continue;
                // (a) the node's own row
                const size_t q = lin(mir(i + dx, m), mir(j + dy, m), DIM == 3 ? mir(k + dz, m) : 0, m);
                own[cls - 1] += u[q] - uc;
                // (b) rows x = p - d over the images p of the node
                for (int a = 0; a < nz; ++a)
                    for (int b = 0; b < ny; ++b)
                        for (int e = 0; e < nx; ++e) {
                            const int xi = px[e] - dx, xj = py[b] - dy, xk = pz[a] - dz;
                            if (xi < 0 || xi >= m || xj < 0 || xj >= m) continue;
                            if (DIM == 3 && (xk < 0 || xk >= m)) continue;
                            const size_t x = lin(xi, xj, DIM == 3 ? xk : 0, m);
                            oth[cls - 1] += lam[x] * (uc - u[x]);
                        }
            }
        }
    }
    const double third = 1.0 / 3.0;
    const double sa = own[0] + 0.5 * own[1] + third * own[2];
    const double sb = oth[0] + 0.5 * oth[1] + third * oth[2];
    grad[c] = -0.5 * L.scale * (lc * sa + sb);
}

// ------------------------------------------------- pure Neumann problems

// Trapezoid-weighted sums, in a fixed order (so that a solve stays bitwise
// reproducible): each block sums kSumChunk consecutive nodes (thread t the
// nodes t, t + 256, ...; then a tree over the block) into partial[block];
// k_wmean_finish adds the partials the same way and divides by the total
// weight.
constexpr int kSumThreads = 256, kSumPerThread = 16, kSumChunk = kSumThreads * kSumPerThread;

__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double part[kSumThreads];
    part[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int w = kSumThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    return part[0];
}

template <typename T, int DIM>
__global__ __launch_bounds__(kSumThreads) void k_wsum(const T *__restrict__ v, Level L,
                                                      double *__restrict__ partial)
{
    const int m = L.m;
    const long long total = DIM == 3 ? (long long)m * m * m : (long long)m * m;
    const long long base = (long long)blockIdx.x * kSumChunk;
    double acc = 0.0;
    for (int q = 0; q < kSumPerThread; ++q) {
        const long long id = base + q * kSumThreads + threadIdx.x;
        if (id >= total) break;
        const int i = (int)(id % m), j = (int)((id / m) % m), k = DIM == 3 ? (int)(id / ((long long)m * m)) : 0;
        acc += trap_weight<DIM>(i, j, k, m, L.dir) * (double)v[id];
    }
    const double b = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = b;
}

__global__ __launch_bounds__(kSumThreads) void k_wmean_finish(const double *__restrict__ partial, int nparts,
                                                              double scale, double weight,
                                                              double *__restrict__ mean)
{
    double acc = 0.0;
    for (int q = threadIdx.x; q < nparts; q += kSumThreads) acc += partial[q];
    const double b = block_sum(acc);
    if (threadIdx.x == 0) *mean = scale * b / weight;
}

// s -= mean_s; u -= mean_e (when given); shat = s * shat_scale (when given);
// norm = max |s|.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_project(double *__restrict__ s, double *__restrict__ u,
                                                 const double *__restrict__ mean_s,
                                                 const double *__restrict__ mean_e, T *__restrict__ shat,
                                                 double shat_scale, Level L, unsigned long long *__restrict__ norm)
{
    int i, j, k;
    unsigned long long rb = 0;
    const int m = L.m;
    if (node_of<DIM>(m, i, j, k)) {
        const size_t c = lin(i, j, k, m);
        const double sn = s[c] - *mean_s;
        s[c] = sn;
        if (mean_e) u[c] -= *mean_e;
        if (shat) shat[c] = (T)(sn * shat_scale);
        rb = dbits(sn);
    }
    block_max(rb, norm);
}

// Neumann data moved to the source: f_out = f - b at unknowns (f elsewhere),
// b the part of dL_1 the flux contributes through the values substituted
// outside the domain: a neighbour sample crossing Neumann face f takes the
// image's value plus 2 h g_f, g_f read on the face at the image's other
// coordinates (x faces indexed (k N + j), y faces (k N + i), z faces
// (j N + i); 2D: j or i).
template <int DIM, int RAD, int SIG>
__global__ __launch_bounds__(256) void k_neumann_source(const double *__restrict__ f, FaceData flux,
                                                        const double *__restrict__ sigma, double h,
                                                        double *__restrict__ out, Level L)
{
    int i, j, k;
    const int m = L.m;
    if (!node_of<DIM>(m, i, j, k)) return;
    const size_t c = lin(i, j, k, m);
    if (is_dir<DIM>(i, j, k, m, L.dir)) {
        out[c] = f[c];
        return;
    }
    const double sc = SIG ? sigma[c] : 1.0;
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz) {
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int cls = (dx != 0) + (dy != 0) + (dz != 0);
                if (cls == 0 || (!RAD && cls != 1)) continue;
                const int qi = i + dx, qj = j + dy, qk = k + dz;
                const int si = mir(qi, m), sj = mir(qj, m), sk = DIM == 3 ? mir(qk, m) : 0;
                double shift = 0.0;
                // faces crossed: x (index by image's (k, j)), y ((k, i)), z ((j, i))
                if (qi < 0 && flux.g[0]) shift += flux.g[0][(size_t)sk * m + sj];
                if (qi > m - 1 && flux.g[1]) shift += flux.g[1][(size_t)sk * m + sj];
                if (qj < 0 && flux.g[2]) shift += flux.g[2][(size_t)sk * m + si];
                if (qj > m - 1 && flux.g[3]) shift += flux.g[3][(size_t)sk * m + si];
                if (DIM == 3) {
                    if (qk < 0 && flux.g[4]) shift += flux.g[4][(size_t)sj * m + si];
                    if (qk > m - 1 && flux.g[5]) shift += flux.g[5][(size_t)sj * m + si];
                }
                if (shift == 0.0) continue;
                const double ss = SIG ? sigma[lin(si, sj, sk, m)] : 1.0;
                acc[cls - 1] += 0.5 * (ss + sc) * 2.0 * h * shift;
            }
        }
    }
    out[c] = f[c] - L.scale * (acc[0] + 0.5 * acc[1] + (1.0 / 3.0) * acc[2]);
}

// ----------------------------------------------------------- dispatch glue

template <template <int, int, int> class K, typename... A>
void dispatch3(const Variant &v, A &&...args)
{
#define SGML_CASE(D, R, S)                                  \
    if (v.dim == D && v.radial == R && v.sigma == S) {      \
        K<D, R, S>::run(std::forward<A>(args)...);          \
        return;                                             \
    }
    SGML_CASE(2, 0, 0) SGML_CASE(2, 0, 1) SGML_CASE(2, 1, 0) SGML_CASE(2, 1, 1)
    SGML_CASE(3, 0, 0) SGML_CASE(3, 0, 1) SGML_CASE(3, 1, 0) SGML_CASE(3, 1, 1)
#undef SGML_CASE
}

template <typename R, template <int, int, int> class K, typename... A>
R dispatch3r(const Variant &v, A &&...args)
{
#define SGML_CASE(D, RA, S) \
    if (v.dim == D && v.radial == RA && v.sigma == S) return K<D, RA, S>::run(std::forward<A>(args)...);
    SGML_CASE(2, 0, 0) SGML_CASE(2, 0, 1) SGML_CASE(2, 1, 0) SGML_CASE(2, 1, 1)
    SGML_CASE(3, 0, 0) SGML_CASE(3, 0, 1) SGML_CASE(3, 1, 0) SGML_CASE(3, 1, 1)
#undef SGML_CASE
    return R();
}

dim3 block_of() { return dim3(BX, BY, 1); }

}  // namespace

// ---------------------------------------------------------------- launchers

template <typename T>
void launch_fill(T *p, size_t count, T value, hipStream_t st)
{
    if (count == 0) return;
    unsigned blocks = (unsigned)std::min<size_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks), dim3(256), 0, st, p, count, value);
}

namespace {
template <typename T>
struct SweepRun {
    template <int D, int R, int S>
    struct K {
        static void run(const Level &L, const T *ein, T *eout, const T *g, const T *sig, const double *G,
                        unsigned long long *pres, hipStream_t st)
        {
            hipLaunchKernelGGL((k_sweep<T, D, R, S>), grid_of(D, L.m), block_of(), 0, st, ein, eout, g, sig,
                               G, L, pres);
        }
    };
};
}  // namespace

template <typename T>
void launch_sweep(const Variant &v, const Level &L, const T *ein, T *eout, const T *g, const T *sig,
                  const double *G, unsigned long long *pres, hipStream_t st)
{
    dispatch3<SweepRun<T>::template K>(v, L, ein, eout, g, sig, G, pres, st);
}

namespace {
template <typename T>
struct CoarseRun {
    template <int D, int R, int S>
    struct K {
        static void run(const CoarseOp *ops, int nops, const Level *levels, const double *G,
                        unsigned long long *targets, hipStream_t st)
        {
            hipLaunchKernelGGL((k_coarse<T, D, R, S>), dim3(1), dim3(coarse_threads(D)), 0, st, ops, nops,
                               levels, G, targets);
        }
    };
};
}  // namespace

template <typename T>
void launch_coarse(const Variant &v, const CoarseOp *ops, int nops, const Level *levels, const double *G,
                   unsigned long long *targets, hipStream_t st)
{
    dispatch3<CoarseRun<T>::template K>(v, ops, nops, levels, G, targets, st);
}

int device_cus()
{
    static std::mutex lock;
    static int cus[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 0;
    std::lock_guard<std::mutex> guard(lock);
    if (cus[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            return 0;
        }
        cus[dev] = n;
    }
    return cus[dev];
}

namespace {
template <typename T>
struct CoarseLdsRun {
    template <int D, int R, int S>
    struct K {
        static bool run(const LdsOp *ops, int nops, int hdr_off, const LdsXfer *xfer, int nload, int nstore,
                        size_t bytes, const double *G, unsigned long long *targets, hipStream_t st)
        {
            // dynamic LDS this instantiation may use, per device; raised under a
            // lock and never lowered, so a launch never exceeds what is granted
            static std::mutex lock;
            static size_t granted[kMaxDevices] = {};
            int dev = 0;
            if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return false;
            {
                std::lock_guard<std::mutex> guard(lock);
                if (bytes > granted[dev]) {
                    if (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_coarse_lds<T, D, R, S>),
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) {
                        (void)hipGetLastError();
                        return false;
                    }
                    granted[dev] = bytes;
                }
            }
            hipLaunchKernelGGL((k_coarse_lds<T, D, R, S>), dim3(1), dim3(coarse_threads(D)), bytes, st, ops,
                               nops, hdr_off, xfer, nload, nstore, G, targets);
            return true;
        }
    };
};
}  // namespace

template <typename T>
bool launch_coarse_lds(const Variant &v, const LdsOp *ops, int nops, int hdr_off, const LdsXfer *xfer, int nload,
                       int nstore, size_t lds_bytes, const double *G, unsigned long long *targets, hipStream_t st)
{
    return dispatch3r<bool, CoarseLdsRun<T>::template K>(v, ops, nops, hdr_off, xfer, nload, nstore, lds_bytes, G,
                                                         targets, st);
}

template <typename T>
void launch_prolong(int dim, int mc, const T *ec, const T *ef_in, T *ef_out, bool first, hipStream_t st)
{
    const int mf = 2 * mc - 1;
    if (dim == 2)
        hipLaunchKernelGGL((k_prolong<T, 2>), grid_of(2, mf), block_of(), 0, st, ec, ef_in, ef_out, mc,
                           (int)first);
    else
        hipLaunchKernelGGL((k_prolong<T, 3>), grid_of(3, mf), block_of(), 0, st, ec, ef_in, ef_out, mc,
                           (int)first);
}

template <typename T>
void launch_inject(int dim, int mc, const T *ef, T *ec, hipStream_t st)
{
    if (dim == 2)
        hipLaunchKernelGGL((k_inject<T, 2>), grid_of(2, mc), block_of(), 0, st, ef, ec, mc);
    else
        hipLaunchKernelGGL((k_inject<T, 3>), grid_of(3, mc), block_of(), 0, st, ef, ec, mc);
}

template <typename Tin, typename Tout>
void launch_restrict(int dim, int mc, const Tin *fine, Tout *coarse, hipStream_t st)
{
    if constexpr (std::is_same<Tin, Tout>::value) {
        if (dim == 2 && mc >= 65) {
            launch_restrict2d<Tin>(mc, fine, coarse, st);
            return;
        }
    }
    if (dim == 2)
        hipLaunchKernelGGL((k_restrict<Tin, Tout, 2>), grid_of(2, mc), block_of(), 0, st, fine, coarse, mc);
    else
        hipLaunchKernelGGL((k_restrict<Tin, Tout, 3>), grid_of(3, mc), block_of(), 0, st, fine, coarse, mc);
}

template <typename Tin, typename Tout>
void launch_convert(const Tin *in, Tout *out, size_t count, hipStream_t st)
{
    if (count == 0) return;
    unsigned blocks = (unsigned)std::min<size_t>((count + 255) / 256, 8192);
    hipLaunchKernelGGL((k_convert<Tin, Tout>), dim3(blocks), dim3(256), 0, st, in, out, count);
}

namespace {
template <typename T>
struct BoundaryRun {
    template <int D, int R, int S>
    struct K {
        static void run(const Level &L, const T *e, double escale, const double *G, const double *sigma,
                        double *u, double *s, T *shat, double shat_scale, unsigned long long *norm,
                        hipStream_t st)
        {
            hipLaunchKernelGGL((k_boundary<T, D, R, S>), grid_of(D, L.m), block_of(), 0, st, e, escale, G,
                               sigma, u, s, shat, shat_scale, L, norm);
        }
    };
};
template <int D, int R, int S>
struct InitRun {
    static void run(const Level &L, const double *f, const double *G, const double *sigma, double *s,
                    double *u, float *s32, unsigned long long *norm0, bool wscale, hipStream_t st)
    {
        if (wscale)
            hipLaunchKernelGGL((k_init<D, R, S, true>), grid_of(D, L.m), block_of(), 0, st, f, G, sigma, s, u,
                               s32, L, norm0);
        else
            hipLaunchKernelGGL((k_init<D, R, S, false>), grid_of(D, L.m), block_of(), 0, st, f, G, sigma, s,
                               u, s32, L, norm0);
    }
};
template <int D, int R, int S>
struct ResidualRun {
    static void run(const Level &L, const double *f, const double *G, const double *sigma,
                    const double *u, double *r, unsigned long long *rmax, unsigned long long *norm0,
                    hipStream_t st)
    {
        hipLaunchKernelGGL((k_residual<D, R, S>), grid_of(D, L.m), block_of(), 0, st, f, G, sigma, u, r,
                           L, rmax, norm0);
    }
};
}  // namespace

template <typename T>
void launch_boundary(const Variant &v, const Level &L, const T *e, double escale, const double *G,
                     const double *sigma, double *u, double *s, T *shat, double shat_scale,
                     unsigned long long *norm, hipStream_t st)
{
    dispatch3<BoundaryRun<T>::template K>(v, L, e, escale, G, sigma, u, s, shat, shat_scale, norm, st);
}

void launch_init(const Variant &v, const Level &L, const double *f, const double *G, const double *sigma,
                 double *s, double *u, float *s32, unsigned long long *norm0, bool wscale, hipStream_t st)
{
    dispatch3<InitRun>(v, L, f, G, sigma, s, u, s32, norm0, wscale, st);
}

void launch_trap_scale(const Level &L, int dim, double *u, hipStream_t st)
{
    if (dim == 2)
        hipLaunchKernelGGL((k_trap_scale<2>), grid_of(2, L.m), block_of(), 0, st, u, L);
    else
        hipLaunchKernelGGL((k_trap_scale<3>), grid_of(3, L.m), block_of(), 0, st, u, L);
}

template <typename T>
void launch_source_cast(const Level &L, int dim, const double *s, T *shat, double scale, hipStream_t st)
{
    if (dim == 2)
        hipLaunchKernelGGL((k_source_cast<T, 2>), grid_of(2, L.m), block_of(), 0, st, s, shat, scale, L.m);
    else
        hipLaunchKernelGGL((k_source_cast<T, 3>), grid_of(3, L.m), block_of(), 0, st, s, shat, scale, L.m);
}

void launch_set_dirichlet(const Level &L, int dim, const double *G, double *u, hipStream_t st)
{
    if (dim == 2)
        hipLaunchKernelGGL((k_set_dirichlet<2>), grid_of(2, L.m), block_of(), 0, st, G, u, L);
    else
        hipLaunchKernelGGL((k_set_dirichlet<3>), grid_of(3, L.m), block_of(), 0, st, G, u, L);
}

void launch_residual(const Variant &v, const Level &L, const double *f, const double *G,
                     const double *sigma, const double *u, double *r, unsigned long long *rmax,
                     unsigned long long *norm0, hipStream_t st)
{
    dispatch3<ResidualRun>(v, L, f, G, sigma, u, r, rmax, norm0, st);
}

void launch_coeff_grad(const Variant &v, const Level &L, const double *u, const double *lam, double *grad,
                       hipStream_t st)
{
    if (v.dim == 2 && !v.radial)
        hipLaunchKernelGGL((k_coeff_grad<2, 0>), grid_of(2, L.m), block_of(), 0, st, u, lam, grad, L);
    else if (v.dim == 2)
        hipLaunchKernelGGL((k_coeff_grad<2, 1>), grid_of(2, L.m), block_of(), 0, st, u, lam, grad, L);
    else if (!v.radial)
        hipLaunchKernelGGL((k_coeff_grad<3, 0>), grid_of(3, L.m), block_of(), 0, st, u, lam, grad, L);
    else
        hipLaunchKernelGGL((k_coeff_grad<3, 1>), grid_of(3, L.m), block_of(), 0, st, u, lam, grad, L);
}

size_t wsum_partials(int dim, int m)
{
    const size_t total = dim == 3 ? (size_t)m * m * m : (size_t)m * m;
    return (total + kSumChunk - 1) / kSumChunk;
}

template <typename T>
void launch_wmean(int dim, const Level &L, const T *v, double scale, double *partial, double *mean,
                  hipStream_t st)
{
    const int nparts = (int)wsum_partials(dim, L.m);
    const double weight = std::pow((double)(L.m - 1), dim);  // total trapezoid weight, all faces Neumann
    if (dim == 2)
        hipLaunchKernelGGL((k_wsum<T, 2>), dim3(nparts), dim3(kSumThreads), 0, st, v, L, partial);
    else
        hipLaunchKernelGGL((k_wsum<T, 3>), dim3(nparts), dim3(kSumThreads), 0, st, v, L, partial);
    hipLaunchKernelGGL(k_wmean_finish, dim3(1), dim3(kSumThreads), 0, st, partial, nparts, scale, weight, mean);
}

template <typename T>
void launch_project(int dim, const Level &L, double *s, double *u, const double *mean_s, const double *mean_e,
                    T *shat, double shat_scale, unsigned long long *norm, hipStream_t st)
{
    if (dim == 2)
        hipLaunchKernelGGL((k_project<T, 2>), grid_of(2, L.m), block_of(), 0, st, s, u, mean_s, mean_e, shat,
                           shat_scale, L, norm);
    else
        hipLaunchKernelGGL((k_project<T, 3>), grid_of(3, L.m), block_of(), 0, st, s, u, mean_s, mean_e, shat,
                           shat_scale, L, norm);
}

namespace {
template <int D, int R, int S>
struct NeumannSourceRun {
    static void run(const Level &L, const double *f, const FaceData &flux, const double *sigma, double h,
                    double *out, hipStream_t st)
    {
        hipLaunchKernelGGL((k_neumann_source<D, R, S>), grid_of(D, L.m), block_of(), 0, st, f, flux, sigma, h,
                           out, L);
    }
};
}  // namespace

void launch_neumann_source(const Variant &v, const Level &L, const double *f, const FaceData &flux,
                           const double *sigma, double h, double *out, hipStream_t st)
{
    dispatch3<NeumannSourceRun>(v, L, f, flux, sigma, h, out, st);
}

template void launch_wmean<double>(int, const Level &, const double *, double, double *, double *, hipStream_t);
template void launch_wmean<float>(int, const Level &, const float *, double, double *, double *, hipStream_t);
template void launch_project<double>(int, const Level &, double *, double *, const double *, const double *,
                                     double *, double, unsigned long long *, hipStream_t);
template void launch_project<float>(int, const Level &, double *, double *, const double *, const double *,
                                    float *, double, unsigned long long *, hipStream_t);

// explicit instantiations
template void launch_fill<double>(double *, size_t, double, hipStream_t);
template void launch_fill<float>(float *, size_t, float, hipStream_t);
template void launch_fill<unsigned long long>(unsigned long long *, size_t, unsigned long long, hipStream_t);
template void launch_sweep<double>(const Variant &, const Level &, const double *, double *, const double *,
                                   const double *, const double *, unsigned long long *, hipStream_t);
template void launch_sweep<float>(const Variant &, const Level &, const float *, float *, const float *,
                                  const float *, const double *, unsigned long long *, hipStream_t);
template void launch_coarse<double>(const Variant &, const CoarseOp *, int, const Level *, const double *,
                                    unsigned long long *, hipStream_t);
template void launch_coarse<float>(const Variant &, const CoarseOp *, int, const Level *, const double *,
                                   unsigned long long *, hipStream_t);
template bool launch_coarse_lds<double>(const Variant &, const LdsOp *, int, int, const LdsXfer *, int, int, size_t,
                                        const double *, unsigned long long *, hipStream_t);
template bool launch_coarse_lds<float>(const Variant &, const LdsOp *, int, int, const LdsXfer *, int, int, size_t,
                                       const double *, unsigned long long *, hipStream_t);
template void launch_prolong<double>(int, int, const double *, const double *, double *, bool, hipStream_t);
template void launch_prolong<float>(int, int, const float *, const float *, float *, bool, hipStream_t);
template void launch_inject<double>(int, int, const double *, double *, hipStream_t);
template void launch_inject<float>(int, int, const float *, float *, hipStream_t);
template void launch_restrict<double, double>(int, int, const double *, double *, hipStream_t);
template void launch_restrict<float, float>(int, int, const float *, float *, hipStream_t);
template void launch_restrict<double, float>(int, int, const double *, float *, hipStream_t);
template void launch_convert<double, float>(const double *, float *, size_t, hipStream_t);
template void launch_boundary<double>(const Variant &, const Level &, const double *, double, const double *,
                                      const double *, double *, double *, double *, double,
                                      unsigned long long *, hipStream_t);
template void launch_boundary<float>(const Variant &, const Level &, const float *, double, const double *,
                                     const double *, double *, double *, float *, double,
                                     unsigned long long *, hipStream_t);
template void launch_source_cast<float>(const Level &, int, const double *, float *, double, hipStream_t);
template void launch_source_cast<double>(const Level &, int, const double *, double *, double, hipStream_t);

}  // namespace sgml
