// sgml_visit2d.hip -- one visit of a 2D level in one pass over memory.
//
// A visit of Algorithm 3 at level nu is: interpolate the pending variation of
// level nu+1 (when the schedule refines), run c relaxations (Algorithm 2,
// Jacobi), and copy the result to level nu+1's nodes (when the schedule
// climbs).  Run one launch per step and each relaxation streams the level
// through HBM again.  Here every wavefront owns a strip of 64 columns and
// marches down the rows of a chunk; each relaxation is a pipeline stage that
// keeps a three-row window of its input in registers, so relaxation s+1
// consumes relaxation s's rows as they are produced.  Horizontal neighbours
// come from the adjacent lanes (cross-lane moves), vertical ones from the
// window.  The strip and the chunk carry a halo as wide as the number of
// relaxations (plus one column for the interpolation), recomputed by the
// neighbouring wavefronts; only the interior is written.  Values outside the
// grid are images (node reflection), so Neumann faces need no special case,
// and a Dirichlet node takes its prescribed value at every relaxation.
// Wavefronts are independent: no LDS, no barriers.
#include "sgml_device.h"

namespace sgml {

namespace {

constexpr int kVisitBlock = 256;  // four independent wavefronts
constexpr int kChunkRows = 64;

template <typename T>
__device__ __forceinline__ T from_left(T v)  // value held by lane - 1
{
    return __shfl_up(v, 1, 64);
}

template <typename T>
__device__ __forceinline__ T from_right(T v)  // value held by lane + 1
{
    return __shfl_down(v, 1, 64);
}

// One relaxation of the node in the middle row of the window w (rows r-1,
// r, r+1 of this lane's column); sg: the coefficient in the same rows.
// All lanes must call it (cross-lane moves).
template <typename T, int RAD, int SIG>
__device__ __forceinline__ T relax(const T (&w)[3], const T (&sg)[3], T g, bool dir, T gval, T scale, T a,
                                   T theta, T &resid)
{
    const T c = w[1];
    const T ul = from_left(c), ur = from_right(c);
    T nl = T(0), nr = T(0), sl = T(0), sr = T(0);  // corner values (radial)
    if (RAD) {
        nl = from_left(w[0]);
        nr = from_right(w[0]);
        sl = from_left(w[2]);
        sr = from_right(w[2]);
    }
    T acc1, acc2 = T(0), D;
    if (SIG) {
        const T sc = sg[1];
        const T tl = from_left(sc) + sc, tr = from_right(sc) + sc;
        const T tn = sg[0] + sc, ts = sg[2] + sc;
        acc1 = tl * (ul - c) + tr * (ur - c) + tn * (w[0] - c) + ts * (w[2] - c);
        T ds1 = tl + tr + tn + ts, ds2 = T(0);
        if (RAD) {
            const T tnl = from_left(sg[0]) + sc, tnr = from_right(sg[0]) + sc;
            const T tsl = from_left(sg[2]) + sc, tsr = from_right(sg[2]) + sc;
            acc2 = tnl * (nl - c) + tnr * (nr - c) + tsl * (sl - c) + tsr * (sr - c);
            ds2 = tnl + tnr + tsl + tsr;
        }
        D = scale * T(0.5) * (ds1 + T(0.5) * ds2) - a;
        acc1 = T(0.5) * (acc1 + T(0.5) * acc2);
        acc2 = T(0);
    } else {
        acc1 = (ul - c) + (ur - c) + (w[0] - c) + (w[2] - c);
        if (RAD) acc2 = (nl - c) + (nr - c) + (sl - c) + (sr - c);
        D = scale * (RAD ? T(6) : T(4)) - a;
    }
    const T Lu = scale * (acc1 + T(0.5) * acc2) + a * c;
    const T r = Lu - g;
    resid = dir ? T(0) : r;
    return dir ? gval : c + (theta / D) * r;
}

// The level's value at (rm, xm) with the pending variation of the next
// coarser level interpolated (mc = (m + 1) / 2 nodes per axis there).  rm is
// the same in every lane.  All lanes must call it (cross-lane moves).
template <typename T>
__device__ __forceinline__ T prolonged(const T *__restrict__ estale, const T *__restrict__ ec, int first, int xm,
                                       int rm, int m)
{
    const int mc = (m + 1) >> 1;
    const bool xe = !(xm & 1);
    // pending variation of coarse row Y, interpolated along x to this column
    auto pend = [&](int Y) -> T {
        T p = T(0);
        if (xe) {
            p = ec[lin(xm >> 1, Y, 0, mc)];
            if (!first) p -= estale[lin(xm, 2 * Y, 0, m)];
        }
        const T pl = from_left(p), pr = from_right(p);
        return xe ? p : T(0.5) * (pl + pr);
    };
    const T st = first ? T(0) : estale[lin(xm, rm, 0, m)];
    const int Y = rm >> 1;
    if (!(rm & 1)) {
        const T p = pend(Y);
        return xe ? ec[lin(xm >> 1, Y, 0, mc)] : st + p;
    }
    const T p0 = pend(Y), p1 = pend(Y + 1);
    return st + T(0.5) * (p0 + p1);
}

template <typename T, int RAD, int SIG, int S, int PRO, int INJ>
__global__ __launch_bounds__(kVisitBlock) void k_visit2d(VisitArgs A)
{
    constexpr int HX = S + PRO;     // halo columns on each side of a strip
    constexpr int W = 64 - 2 * HX;  // columns a wavefront writes
    const Level L = A.L;
    const int m = L.m;
    const int lane = threadIdx.x & 63;
    const int strips = (m + W - 1) / W;
    const int wid = blockIdx.x * (kVisitBlock / 64) + (threadIdx.x >> 6);
    const int sx = wid % strips, sy = wid / strips;
    const int y0 = sy * kChunkRows;
    if (y0 >= m) return;  // the whole wavefront: past the last chunk
    const int y1 = min(m, y0 + kChunkRows);
    const int x = sx * W - HX + lane;
    const int xm = mir(x, m);
    const bool xout = lane >= HX && lane < HX + W && x < m;

    const T *__restrict__ estale = (const T *)A.estale;
    const T *__restrict__ ec = (const T *)A.ecoarse;
    const T *__restrict__ g = (const T *)A.g;
    const T *__restrict__ sig = (const T *)A.sig;
    T *__restrict__ eout = (T *)A.eout;
    T *__restrict__ einj = (T *)A.einj;
    const T scale = (T)L.scale, a = (T)L.a, theta = (T)L.theta;

    T w[S][3];
    T gh[S + 1];  // gh[k]: source at input row - k
    T sh[S + 2];  // sh[k]: coefficient at input row - k
    unsigned long long pr[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        w[s][0] = w[s][1] = w[s][2] = T(0);
        pr[s] = 0;
    }
#pragma unroll
    for (int k = 0; k < S + 1; ++k) gh[k] = T(0);
#pragma unroll
    for (int k = 0; k < S + 2; ++k) sh[k] = T(1);

    const int rows = (y1 - y0) + 2 * S;
    for (int t = 0; t < rows; ++t) {
        const int rho = y0 - S + t;  // input row, outside the grid: its image
        const int rm = mir(rho, m);
        const size_t q = lin(xm, rm, 0, m);
        T val = PRO ? prolonged<T>(estale, ec, A.first, xm, rm, m) : estale[q];
#pragma unroll
        for (int k = S; k > 0; --k) gh[k] = gh[k - 1];
        gh[0] = g[q];
        if (SIG) {
#pragma unroll
            for (int k = S + 1; k > 0; --k) sh[k] = sh[k - 1];
            sh[0] = sig[q];
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            w[s][0] = w[s][1];
            w[s][1] = w[s][2];
            w[s][2] = val;
            const int r = rho - s - 1;  // row relaxation s+1 produces now
            const int rmr = mir(r, m);
            const bool dir = is_dir<2>(xm, rmr, 0, m, L.dir);
            const T gval = (dir && A.G) ? (T)A.G[lin(xm * L.lam, rmr * L.lam, 0, L.N)] : T(0);
            const T sg[3] = {sh[s + 2], sh[s + 1], sh[s]};
            T resid;
            val = relax<T, RAD, SIG>(w[s], sg, gh[s + 1], dir, gval, scale, a, theta, resid);
            if (A.pres[s] >= 0 && r >= y0 && r < y1 && xout) {
                const unsigned long long b = dbits((double)resid);
                pr[s] = b > pr[s] ? b : pr[s];
            }
        }
        const int ro = rho - S;
        if (ro >= y0 && ro < y1 && xout) {
            eout[lin(x, ro, 0, m)] = val;
            if (INJ && !(ro & 1) && !(x & 1)) einj[lin(x >> 1, ro >> 1, 0, (m + 1) >> 1)] = val;
        }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        if (A.pres[s] < 0) continue;
        unsigned long long v = pr[s];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(v, off, 64);
            v = o > v ? o : v;
        }
        if (lane == 0 && v)
            atomicMax(A.targets + (size_t)A.pres[s] * kRedWords + (size_t)(wid % kRedSlots) * kRedStride, v);
    }
}

template <typename T, int RAD, int SIG, int S, int PRO, int INJ>
void launch_one(const VisitArgs &a, hipStream_t st)
{
    constexpr int W = 64 - 2 * (S + PRO);
    const int m = a.L.m;
    const long long waves = (long long)((m + W - 1) / W) * ((m + kChunkRows - 1) / kChunkRows);
    const unsigned blocks = (unsigned)((waves + kVisitBlock / 64 - 1) / (kVisitBlock / 64));
    hipLaunchKernelGGL((k_visit2d<T, RAD, SIG, S, PRO, INJ>), dim3(blocks), dim3(kVisitBlock), 0, st, a);
}

template <typename T, int RAD, int SIG, int S>
void launch_s(const VisitArgs &a, hipStream_t st)
{
    if (a.prolong && a.inject)
        launch_one<T, RAD, SIG, S, 1, 1>(a, st);
    else if (a.prolong)
        launch_one<T, RAD, SIG, S, 1, 0>(a, st);
    else if (a.inject)
        launch_one<T, RAD, SIG, S, 0, 1>(a, st);
    else
        launch_one<T, RAD, SIG, S, 0, 0>(a, st);
}

template <typename T, int RAD, int SIG>
void launch_rs(const VisitArgs &a, hipStream_t st)
{
    switch (a.sweeps) {
    case 1: launch_s<T, RAD, SIG, 1>(a, st); break;
    case 2: launch_s<T, RAD, SIG, 2>(a, st); break;
    case 4: launch_s<T, RAD, SIG, 4>(a, st); break;
    default: launch_s<T, RAD, SIG, 6>(a, st); break;
    }
}

}  // namespace

bool fused_visit_supported(int sweeps) { return sweeps == 1 || sweeps == 2 || sweeps == 4 || sweeps == 6; }

template <typename T>
void launch_visit2d(const Variant &v, const VisitArgs &a, hipStream_t st)
{
    if (v.radial && v.sigma)
        launch_rs<T, 1, 1>(a, st);
    else if (v.radial)
        launch_rs<T, 1, 0>(a, st);
    else if (v.sigma)
        launch_rs<T, 0, 1>(a, st);
    else
        launch_rs<T, 0, 0>(a, st);
}

template void launch_visit2d<double>(const Variant &, const VisitArgs &, hipStream_t);
template void launch_visit2d<float>(const Variant &, const VisitArgs &, hipStream_t);

}  // namespace sgml
