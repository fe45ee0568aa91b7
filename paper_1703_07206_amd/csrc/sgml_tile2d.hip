// sgml_tile2d.hip -- one visit of a 2D level (levels 1 and coarser) in LDS.
//
// A visit of Algorithm 3 at level nu: interpolate the pending variation of
// level nu+1 (when the schedule refines), run c relaxations (Algorithm 2,
// Jacobi), copy the result to level nu+1's nodes (when the schedule climbs).
// The row-marching visit (sgml_visit2d_impl.h) streams a level through
// registers, which suits the 4097^2 level 0; on the smaller levels its
// wavefronts are few and each one's row chain is long, so the visit is
// latency bound.  Here a workgroup takes a 64 x 32 tile of the level plus a
// halo as wide as the work needs (one node per relaxation, one more for the
// interpolation), loads it into LDS once, performs the whole visit there with
// one barrier per step, and writes the tile's interior back: one round trip
// to memory per visit whatever the level's size.
//
// Values outside the grid are images (node reflection), loaded as such, so
// every step is computed in tile coordinates without special cases at
// Neumann faces; a Dirichlet node takes its prescribed value (G in the first
// cycle, else 0) at every relaxation, held in the source slot of the tile
// (a Dirichlet node has no use for its source).
#include "sgml_device.h"

namespace sgml {

namespace {

constexpr int kTileX = 64, kTileY = 32, kTileThreads = 512;

template <typename T>
struct TileK {
    T scale, a, theta, omt, beta, gamma, aw;
};

template <typename T>
__device__ __forceinline__ T tile_step(T theta, T D);
template <>
__device__ __forceinline__ float tile_step(float theta, float D)
{
    return theta * __builtin_amdgcn_rcpf(D);
}
template <>
__device__ __forceinline__ double tile_step(double theta, double D)
{
    return theta / D;
}

// One relaxation of tile node t (pitch FX) from src; resid: dL e - g.
template <typename T, int RAD, int SIG, int FX>
__device__ __forceinline__ T tile_relax(const T *src, const T *sg, int t, T g, const TileK<T> &K, T &resid)
{
    const T c = src[t];
    const T l = src[t - 1], r = src[t + 1], u = src[t - FX], d = src[t + FX];
    if (SIG) {
        const T sc = sg[t];
        const T tl = sg[t - 1] + sc, tr = sg[t + 1] + sc, tu = sg[t - FX] + sc, td = sg[t + FX] + sc;
        T acc = tl * (l - c) + tr * (r - c) + tu * (u - c) + td * (d - c);
        T ds = tl + tr + tu + td;
        if (RAD) {
            const T tul = sg[t - FX - 1] + sc, tur = sg[t - FX + 1] + sc;
            const T tdl = sg[t + FX - 1] + sc, tdr = sg[t + FX + 1] + sc;
            acc += T(0.5) * (tul * (src[t - FX - 1] - c) + tur * (src[t - FX + 1] - c) +
                             tdl * (src[t + FX - 1] - c) + tdr * (src[t + FX + 1] - c));
            ds += T(0.5) * (tul + tur + tdl + tdr);
        }
        resid = K.scale * T(0.5) * acc + K.a * c - g;
        return c + tile_step(K.theta, K.scale * T(0.5) * ds - K.a) * resid;
    }
    T sum = (l + r) + (u + d);
    if (RAD) sum += T(0.5) * ((src[t - FX - 1] + src[t - FX + 1]) + (src[t + FX - 1] + src[t + FX + 1]));
    resid = K.scale * sum + K.aw * c - g;
    return K.omt * c + (K.beta * sum - K.gamma * g);
}

__device__ __forceinline__ void tile_max(unsigned long long v, unsigned long long *red, unsigned long long *out,
                                         int slot)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kTileThreads / 64; ++w) v = red[w] > v ? red[w] : v;
        if (v) atomicMax(out + (size_t)(slot % kRedSlots) * kRedStride, v);
    }
}

template <typename T, int RAD, int SIG, int S, int PRO>
__global__ __launch_bounds__(kTileThreads) void k_visit_tile(VisitArgs A)
{
    constexpr int H = S + PRO;                      // halo on every side
    constexpr int FX = kTileX + 2 * H, FY = kTileY + 2 * H, NF = FX * FY;
    constexpr int HC = (H + 1) / 2;                 // coarse halo (interpolation)
    constexpr int CX = FX / 2 + 2, CY = FY / 2 + 2;  // coarse tile
    __shared__ T buf[2][NF];
    __shared__ T gS[NF];
    __shared__ T sgS[SIG ? NF : 1];
    __shared__ T ecS[PRO ? CX * CY : 1];
    __shared__ unsigned long long red[kTileThreads / 64];

    const Level L = A.L;
    const int m = L.m;
    const int tiles_x = (m + kTileX - 1) / kTileX;
    const int bx = blockIdx.x % tiles_x, by = blockIdx.x / tiles_x;
    const int x0 = bx * kTileX, y0 = by * kTileY;  // interior origin, even
    const int tid = threadIdx.x;
    const unsigned um = (unsigned)m;
    const T *__restrict__ estale = (const T *)A.estale;
    const T *__restrict__ gsrc = (const T *)A.g;
    const T *__restrict__ sig = (const T *)A.sig;
    const double *__restrict__ G = A.G;
    const bool zero_stale = PRO && A.first;

    TileK<T> K;
    K.scale = (T)L.scale;
    K.a = (T)L.a;
    K.theta = (T)L.theta;
    {
        const double W = RAD ? 6.0 : 4.0, D = W * L.scale - L.a;
        K.omt = (T)(1.0 - L.theta);
        K.beta = (T)(L.theta * L.scale / D);
        K.gamma = (T)(L.theta / D);
        K.aw = (T)(L.a - W * L.scale);
    }

    // Dirichlet nodes of the tile: the tile columns / rows of the grid's
    // Dirichlet faces (their images are unknowns); -1 when absent
    const int xd0 = (L.dir & 1u) ? H - x0 : -1, xd1 = (L.dir & 2u) ? m - 1 - x0 + H : -1;
    const int yd0 = (L.dir & 4u) ? H - y0 : -1, yd1 = (L.dir & 8u) ? m - 1 - y0 + H : -1;
    auto tile_dir = [&](int lx, int ly) { return (lx == xd0) | (lx == xd1) | (ly == yd0) | (ly == yd1); };

    // ---- load the tile (images outside the grid)
    // every thread issues all its loads before storing any (the loads of a
    // thread are independent; this keeps them in flight together)
    {
        constexpr int LI = (NF + kTileThreads - 1) / kTileThreads;
        constexpr int CI = PRO ? (CX * CY + kTileThreads - 1) / kTileThreads : 1;
        T ve[LI], vg[LI], vs[SIG ? LI : 1], vc[CI];
#pragma unroll
        for (int i = 0; i < LI; ++i) {
            const int t = tid + i * kTileThreads;
            if (t < NF) {
                const int ly = t / FX, lx = t - ly * FX;
                const int xm = mir(x0 - H + lx, m), ym = mir(y0 - H + ly, m);
                const unsigned q = (unsigned)ym * um + (unsigned)xm;
                ve[i] = zero_stale ? T(0) : estale[q];
                if (is_dir<2>(xm, ym, 0, m, L.dir))
                    vg[i] = G ? (T)G[(size_t)ym * (size_t)L.lam * (size_t)L.N + (size_t)xm * (size_t)L.lam] : T(0);
                else
                    vg[i] = gsrc[q];
                if (SIG) vs[i] = sig[q];
            }
        }
        if (PRO) {
            const T *__restrict__ ec = (const T *)A.ecoarse;
            const int mc = (m + 1) / 2;
            const int Xb = x0 / 2 - HC, Yb = y0 / 2 - HC;
#pragma unroll
            for (int i = 0; i < CI; ++i) {
                const int t = tid + i * kTileThreads;
                if (t < CX * CY) {
                    const int cy = t / CX, cx = t - cy * CX;
                    const int Xm = mir(Xb + cx, mc), Ym = mir(Yb + cy, mc);
                    vc[i] = ec[(unsigned)Ym * (unsigned)mc + (unsigned)Xm];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < LI; ++i) {
            const int t = tid + i * kTileThreads;
            if (t < NF) {
                buf[0][t] = ve[i];
                gS[t] = vg[i];
                if (SIG) sgS[t] = vs[i];
            }
        }
        if (PRO) {
#pragma unroll
            for (int i = 0; i < CI; ++i) {
                const int t = tid + i * kTileThreads;
                if (t < CX * CY) ecS[t] = vc[i];
            }
        }
    }
    __syncthreads();

    // ---- interpolation of the pending variation (prologue), on [1, F-1),
    // into buf[1]
    if (PRO) {
        constexpr int RW = FX - 2, RH = FY - 2, RI = (RW * RH + kTileThreads - 1) / kTileThreads;
        T v[RI];
#pragma unroll
        for (int i = 0; i < RI; ++i) {
            const int t = tid + i * kTileThreads;
            if (t < RW * RH) {
                const int ry = t / RW, lx = 1 + (t - ry * RW), ly = 1 + ry;
                const int gx = lx - H, gy = ly - H;  // offsets from the even origin
                const int oi = gx & 1, oj = gy & 1;
                const int cx = (gx >> 1) + HC, cy = (gy >> 1) + HC;
                // coarse node (cx + a, cy + b) sits at fine tile node (lx - oi + 2a, ly - oj + 2b);
                // the terms with a > oi or b > oj are absent (read in range, then dropped)
                T p[2][2];
#pragma unroll
                for (int b = 0; b <= 1; ++b)
#pragma unroll
                    for (int a = 0; a <= 1; ++a) {
                        const int aa = a & oi, bb = b & oj;
                        T q = ecS[(cy + bb) * CX + cx + aa];
                        if (!zero_stale) q -= buf[0][(ly - oj + 2 * bb) * FX + lx - oi + 2 * aa];
                        p[b][a] = q;
                    }
                // summed in the order of the separate interpolation kernel
                const T acc = ((p[0][0] + (oi ? p[0][1] : T(0))) + (oj ? p[1][0] : T(0))) + ((oi & oj) ? p[1][1] : T(0));
                const T w = (oi & oj) ? T(0.25) : T(0.5);
                const T stale = zero_stale ? T(0) : buf[0][ly * FX + lx];
                v[i] = (oi | oj) ? stale + w * acc : ecS[cy * CX + cx];
            }
        }
#pragma unroll
        for (int i = 0; i < RI; ++i) {
            const int t = tid + i * kTileThreads;
            if (t < RW * RH) {
                const int ry = t / RW;
                buf[1][(1 + ry) * FX + 1 + (t - ry * RW)] = v[i];
            }
        }
        __syncthreads();
    }

    // ---- relaxations: sweep k updates [PRO + k, F - PRO - k); the buffers
    // alternate, starting from buf[PRO]
#pragma unroll
    for (int k = 1; k <= S; ++k) {
        const int lo = PRO + k;
        const int RW = FX - 2 * lo, RH = FY - 2 * lo;
        constexpr int RI = (FX * FY + kTileThreads - 1) / kTileThreads;  // bound for every k
        const T *src = buf[(PRO + k - 1) & 1];
        T *dst = buf[(PRO + k) & 1];
        const bool rec = A.pres[k - 1] >= 0;
        unsigned long long rb = 0;
        T v[RI];
#pragma unroll
        for (int i = 0; i < RI; ++i) {
            const int t = tid + i * kTileThreads;
            if (t < RW * RH) {
                const int ry = t / RW, lx = lo + (t - ry * RW), ly = lo + ry;
                const int f = ly * FX + lx;
                const T gf = gS[f];
                T resid;
                const T nv = tile_relax<T, RAD, SIG, FX>(src, sgS, f, gf, K, resid);
                const bool d = tile_dir(lx, ly);
                v[i] = d ? gf : nv;
                if (rec && !d && lx >= H && lx < H + kTileX && ly >= H && ly < H + kTileY && x0 - H + lx < m &&
                    y0 - H + ly < m) {
                    const unsigned long long b = dbits((double)resid);
                    rb = b > rb ? b : rb;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < RI; ++i) {
            const int t = tid + i * kTileThreads;
            if (t < RW * RH) {
                const int ry = t / RW;
                dst[(lo + ry) * FX + lo + (t - ry * RW)] = v[i];
            }
        }
        __syncthreads();
        if (rec) tile_max(rb, red, A.targets + (size_t)A.pres[k - 1] * kRedWords, blockIdx.x);
    }
    constexpr int cur = (PRO + S) & 1;

    // ---- write the interior; injection into the next coarser level
    T *__restrict__ eout = (T *)A.eout;
    T *__restrict__ einj = (T *)A.einj;
    const bool inject = A.inject != 0;
    const int mc = (m + 1) / 2;
    for (int t = tid; t < kTileX * kTileY; t += kTileThreads) {
        const int iy = t / kTileX, ix = t - iy * kTileX;
        const int x = x0 + ix, y = y0 + iy;
        if (x >= m || y >= m) continue;
        const T v = buf[cur][(iy + H) * FX + ix + H];
        eout[(unsigned)y * um + (unsigned)x] = v;
        if (inject && !((x | y) & 1)) einj[(unsigned)(y >> 1) * (unsigned)mc + (unsigned)(x >> 1)] = v;
    }
}

template <typename T, int RAD, int SIG, int S>
void launch_tile_s(const VisitArgs &a, hipStream_t st)
{
    const int m = a.L.m;
    const unsigned blocks = (unsigned)(((m + kTileX - 1) / kTileX) * ((m + kTileY - 1) / kTileY));
    if (a.prolong)
        hipLaunchKernelGGL((k_visit_tile<T, RAD, SIG, S, 1>), dim3(blocks), dim3(kTileThreads), 0, st, a);
    else
        hipLaunchKernelGGL((k_visit_tile<T, RAD, SIG, S, 0>), dim3(blocks), dim3(kTileThreads), 0, st, a);
}

template <typename T, int RAD, int SIG>
void launch_tile_rs(const VisitArgs &a, hipStream_t st)
{
    switch (a.sweeps) {
    case 1: launch_tile_s<T, RAD, SIG, 1>(a, st); break;
    case 2: launch_tile_s<T, RAD, SIG, 2>(a, st); break;
    case 4: launch_tile_s<T, RAD, SIG, 4>(a, st); break;
    default: launch_tile_s<T, RAD, SIG, 6>(a, st); break;
    }
}

}  // namespace

// Levels of 129 .. 1025 nodes per axis.  Below, the tile and its images
// would not stay within one reflection of the grid; above, the level is
// large enough to be bandwidth bound, where the row-marching visit, whose
// halo costs less traffic, is the faster one.
bool tile_visit_supported(int m) { return m >= 129 && m <= 1025; }

template <typename T>
void launch_visit_tile(const Variant &v, const VisitArgs &a, hipStream_t st)
{
    if (v.radial && v.sigma)
        launch_tile_rs<T, 1, 1>(a, st);
    else if (v.radial)
        launch_tile_rs<T, 1, 0>(a, st);
    else if (v.sigma)
        launch_tile_rs<T, 0, 1>(a, st);
    else
        launch_tile_rs<T, 0, 0>(a, st);
}

template void launch_visit_tile<double>(const Variant &, const VisitArgs &, hipStream_t);
template void launch_visit_tile<float>(const Variant &, const VisitArgs &, hipStream_t);

}  // namespace sgml
