// sgml_sweep3d.hip -- the 3D level kernels, marching in z: one relaxation,
// two chained relaxations (sigma = 1), the cycle-end pass, interpolation and
// restriction.
//
// A block owns a tile of (x, y) columns and a chunk of z planes (sized by the
// level so that small levels still get many blocks).  Each plane of the
// level's values (and of the coefficient) is staged once, with its halo, in a
// ring of LDS planes; a node's 26 (radial) or 6 (axis) neighbours are then
// read from LDS instead of from L1/L2, and every value crosses the memory
// hierarchy about once.  Halo cells outside the grid hold the image node, so
// Neumann faces need no special case.  With a constant coefficient the 26
// neighbours are summed by class from per-plane partial sums (face and corner
// neighbours within a plane), 8 LDS reads per node instead of 26.  The paired
// relaxation, the interpolation and the constant-coefficient cycle end load
// their planes straight into LDS (global_load_lds_dword) ahead of use.  Every
// level from 65 on has 64k + 1 columns: the last one runs in 4 x 128 tiles.
#include "sgml_device.h"

#include <type_traits>

namespace sgml {

namespace {

constexpr int TX = 64, TY = 8, ZC = 16;  // tile and z chunk
constexpr int kThreads = TX * TY;
constexpr int PX = TX + 2, PY = TY + 2;  // staged plane with halo
constexpr int NP = PX * PY;               // staged plane cells (660)
static_assert(NP <= 2 * kThreads, "two staged cells per thread");
constexpr int RING = 4;  // planes in LDS: z-1, z, z+1 being read, z+2 being written

// theta / D: the hardware reciprocal in FP32 (the mixed mode's approximate
// inner solver), a division in FP64.
__device__ __forceinline__ float step_of3(float theta, float D) { return theta * __builtin_amdgcn_rcpf(D); }
__device__ __forceinline__ double step_of3(double theta, double D) { return theta / D; }

// The two cells of a staged plane that thread t fills (t and t + kThreads)
// and their in-plane image offsets, the same for every plane.
struct StageCells {
    unsigned q[2];
    int ly[2], lx[2];
    bool two;
};
__device__ __forceinline__ StageCells stage_cells(int x0, int y0, int m)
{
    StageCells c;
    for (int k = 0; k < 2; ++k) {
        const int idx = (int)threadIdx.x + k * kThreads;
        const int i = idx < NP ? idx : 0;
        c.ly[k] = i / PX;
        c.lx[k] = i - c.ly[k] * PX;
        c.q[k] = (unsigned)mir(y0 - 1 + c.ly[k], m) * (unsigned)m + (unsigned)mir(x0 - 1 + c.lx[k], m);
    }
    c.two = (int)threadIdx.x + kThreads < NP;
    return c;
}

// Each plane is staged once with a one-node halo (images outside the grid)
// in a ring of four LDS planes; the loads of plane z+2 are issued into
// registers before plane z is computed and stored to LDS after, so their
// latency overlaps the computation, and one barrier per plane suffices (the
// plane being written is never one being read).
// Tile index of a block in XCD-grouped order: dispatch deals blocks to the 8
// XCDs in turn, so blocks b, b + 8, b + 16 ... share an XCD and its L2; they
// take consecutive tiles, whose shared halo rows then meet in one L2 (used by
// the paired relaxation).  A bijection of 0 .. nb - 1.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    constexpr int kX = 8;
    const int per = nb / kX, rem = nb % kX, xcd = b % kX, k = b / kX;
    return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k;
}

// Tile shapes of the single relaxation: 64 x 8 columns, and 4 x 128 for the
// last column of a level whose other columns fill whole 64-wide tiles
// (m = 64 k + 1, every level from 65 on): that column then costs 1/16 of a
// tile column of wavefronts instead of a whole one.
constexpr int kColW = 4, kColRows = kThreads / kColW;
constexpr int NPMAX = (kColW + 2) * (kColRows + 2);  // staged cells of the larger shape (780)
static_assert(NP <= NPMAX && NPMAX <= 2 * kThreads, "two staged cells per thread");

// StageCells for a tile TW columns wide (kThreads / TW rows); cells past one
// reflection (small levels) are clamped into the grid and never used.
template <int TW>
__device__ __forceinline__ StageCells stage_cells_t(int x0, int y0, int m)
{
    constexpr int PXT = TW + 2, NPT = PXT * (kThreads / TW + 2);
    auto img = [&](int c) { return min(max(mir(c, m), 0), m - 1); };
    StageCells c;
    for (int k = 0; k < 2; ++k) {
        const int idx = (int)threadIdx.x + k * kThreads;
        const int i = idx < NPT ? idx : 0;
        c.ly[k] = i / PXT;
        c.lx[k] = i - c.ly[k] * PXT;
        c.q[k] = (unsigned)img(y0 - 1 + c.ly[k]) * (unsigned)m + (unsigned)img(x0 - 1 + c.lx[k]);
    }
    c.two = (int)threadIdx.x + kThreads < NPT;
    return c;
}

template <typename T, int RAD, int SIG, int TW>
__device__ __forceinline__ void sweep3d_tile(T (*su)[NPMAX], T (*ss)[NPMAX], const T *__restrict__ ein,
                                             T *__restrict__ eout, const T *__restrict__ g,
                                             const T *__restrict__ sig, const double *__restrict__ G,
                                             const Level &L, unsigned long long *__restrict__ pres, int x0,
                                             int y0, int z0, int z1)
{
    constexpr int PXT = TW + 2;  // pitch of a staged plane
    const int m = L.m;
    const int tx = threadIdx.x % TW, ty = threadIdx.x / TW;
    const int x = x0 + tx, y = y0 + ty;
    const bool own = x < m && y < m;
    const size_t plane = (size_t)m * m;
    const unsigned cxy = (unsigned)(own ? y : 0) * (unsigned)m + (unsigned)(own ? x : 0);
    const StageCells cells = stage_cells_t<TW>(x0, y0, m);
    const int ctr = (ty + 1) * PXT + tx + 1;  // this thread's node in a staged plane

    T pe[2] = {T(0), T(0)}, ps[2] = {T(1), T(1)};
    auto fetch = [&](int zz) {
        const T *__restrict__ ez = ein + (size_t)mir(zz, m) * plane;
        pe[0] = ez[cells.q[0]];
        if (cells.two) pe[1] = ez[cells.q[1]];
        if (SIG) {
            const T *__restrict__ sz = sig + (size_t)mir(zz, m) * plane;
            ps[0] = sz[cells.q[0]];
            if (cells.two) ps[1] = sz[cells.q[1]];
        }
    };
    auto put = [&](int slot) {
        su[slot][threadIdx.x] = pe[0];
        if (cells.two) su[slot][threadIdx.x + kThreads] = pe[1];
        if (SIG) {
            ss[slot][threadIdx.x] = ps[0];
            if (cells.two) ss[slot][threadIdx.x + kThreads] = ps[1];
        }
    };
    const T scale = (T)L.scale, a = (T)L.a, theta = (T)L.theta;
    // constant coefficient: D is the same everywhere
    const T Wc = RAD ? T(6) + T(0.5) * T(12) + T(1.0 / 3.0) * T(8) : T(6);
    const T tD = theta / (scale * Wc - a);
    unsigned long long rb = 0;
    // constant coefficient: per plane and column, the centre value, the sum
    // of the 4 in-plane face neighbours and of the 4 in-plane corners; the
    // 26 neighbours of the middle plane's node are classes of these sums
    T cc[3] = {T(0), T(0), T(0)}, cx[3] = {T(0), T(0), T(0)}, ck[3] = {T(0), T(0), T(0)};
    auto plane_sums = [&](int slot, int at) {
        const T *P = su[slot];
        cc[at] = P[ctr];
        cx[at] = (P[ctr - 1] + P[ctr + 1]) + (P[ctr - PXT] + P[ctr + PXT]);
        if (RAD) ck[at] = (P[ctr - PXT - 1] + P[ctr - PXT + 1]) + (P[ctr + PXT - 1] + P[ctr + PXT + 1]);
    };
    fetch(z0 - 1);
    put(0);
    fetch(z0);
    put(1);
    fetch(z0 + 1);
    T gnext = own ? g[(size_t)z0 * plane + cxy] : T(0);
    __syncthreads();
    if (!SIG) {
        plane_sums(0, 1);  // at = 1: plane z-1 of the first node, shifted in below
        plane_sums(1, 2);
    }
    for (int z = z0; z < z1; ++z) {
        const int k = z - z0;
        const int sm = k % RING, sc = (k + 1) % RING, sp = (k + 2) % RING;  // planes z-1, z, z+1
        put(sp);  // plane z+1
        const T gc = gnext;
        if (z + 1 < z1) {  // the next plane's loads, in flight while this one is computed
            fetch(z + 2);
            if (own) gnext = g[(size_t)(z + 1) * plane + cxy];
        }
        __syncthreads();
        if (!SIG) {
            cc[0] = cc[1], cc[1] = cc[2];
            cx[0] = cx[1], cx[1] = cx[2];
            ck[0] = ck[1], ck[1] = ck[2];
            plane_sums(sp, 2);  // cc/cx/ck[0..2]: planes z-1, z, z+1
        }
        if (own) {
            const size_t c = (size_t)z * plane + cxy;
            if (is_dir<3>(x, y, z, m, L.dir)) {
                eout[c] = G ? (T)G[lin(x * L.lam, y * L.lam, z * L.lam, L.N)] : T(0);
            } else if (!SIG) {
                const T uc = cc[1];
                T faces = cx[1] + (cc[0] + cc[2]);
                T sum = faces;
                if (RAD) {
                    const T edges = ck[1] + (cx[0] + cx[2]);
                    const T corners = ck[0] + ck[2];
                    sum = faces + T(0.5) * edges + T(1.0 / 3.0) * corners;
                }
                const T r = scale * (sum - Wc * uc) + a * uc - gc;
                eout[c] = uc + tD * r;
                if (pres) {
                    const unsigned long long b = dbits((double)r);
                    rb = b > rb ? b : rb;
                }
            } else {
                const T *Pu[3] = {su[sm], su[sc], su[sp]};
                const T *Ps[3] = {ss[sm], ss[sc], ss[sp]};
                const T uc = Pu[1][ctr];
                const T sgc = Ps[1][ctr];
                T acc[3] = {T(0), T(0), T(0)}, ds[3] = {T(0), T(0), T(0)};
#pragma unroll
                for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int cls = (dx != 0) + (dy != 0) + (dz != 0);
                            if (cls == 0 || (!RAD && cls != 1)) continue;
                            const int o = ctr + dy * PXT + dx;
                            const T du = Pu[dz + 1][o] - uc;
                            const T t = Ps[dz + 1][o] + sgc;
                            acc[cls - 1] += t * du;
                            ds[cls - 1] += t;
                        }
                    }
                }
                const T third = T(1.0 / 3.0);
                const T sw = acc[0] + T(0.5) * acc[1] + third * acc[2];
                const T Lu = scale * T(0.5) * sw + a * uc;
                const T D = scale * T(0.5) * (ds[0] + T(0.5) * ds[1] + third * ds[2]) - a;
                const T r = Lu - gc;
                eout[c] = uc + step_of3(theta, D) * r;
                if (pres) {
                    const unsigned long long b = dbits((double)r);
                    rb = b > rb ? b : rb;
                }
            }
        }
    }
    if (pres) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(rb, off, 64);
            rb = o > rb ? o : rb;
        }
        if ((threadIdx.x & 63) == 0 && rb) {
            const unsigned b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z) + threadIdx.x / 64;
            atomicMax(pres + (b % kRedSlots) * kRedStride, rb);
        }
    }
}

template <typename T, int RAD, int SIG>
__global__ __launch_bounds__(kThreads) void k_sweep3d(const T *__restrict__ ein, T *__restrict__ eout,
                                                      const T *__restrict__ g, const T *__restrict__ sig,
                                                      const double *__restrict__ G, Level L,
                                                      unsigned long long *__restrict__ pres, int zc, int ntx,
                                                      int nty, int ncy)
{
    __shared__ T su[RING][NPMAX];
    __shared__ T ss[SIG ? RING : 1][NPMAX];
    // per z chunk: ntx x nty tiles of 64 x 8, then ncy column tiles of 4 x 128
    const int per = ntx * nty + ncy;
    const int bz = blockIdx.x / per, r = blockIdx.x - bz * per;
    const int z0 = bz * zc, z1 = min(L.m, z0 + zc);
    if (r < ntx * nty)
        sweep3d_tile<T, RAD, SIG, TX>(su, ss, ein, eout, g, sig, G, L, pres, (r % ntx) * TX, (r / ntx) * TY, z0, z1);
    else
        sweep3d_tile<T, RAD, SIG, kColW>(su, ss, ein, eout, g, sig, G, L, pres, ntx * TX, (r - ntx * nty) * kColRows,
                                         z0, z1);
}

// End of a cycle on a 3D level 0 (recurrence of Sec. 2, FP64), marching in
// z like k_sweep3d: e = escale * E with Dirichlet values replaced by G (first
// cycle) or 0 is staged per plane in LDS, then u += e, s -= dL_1 e at
// unknowns (s = 0 at Dirichlet nodes), shat = s * shat_scale, max |s|.  The
// next plane's e, coefficient, s and u are loaded into registers while the
// current plane is computed.
template <typename T, int RAD, int SIG>
__global__ __launch_bounds__(kThreads) void k_cycle_end3d(CycleEndArgs A)
{
    __shared__ double se[RING][NP];
    __shared__ double ss[SIG ? RING : 1][SIG ? NP : 1];
    const Level L = A.L;
    const int m = L.m;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * ZC;
    const int z1 = min(m, z0 + ZC);
    const int x = x0 + tx, y = y0 + ty;
    const bool own = x < m && y < m;
    const size_t plane = (size_t)m * m;
    const unsigned cxy = (unsigned)(own ? y : 0) * (unsigned)m + (unsigned)(own ? x : 0);
    const StageCells cells = stage_cells(x0, y0, m);
    const int ctr = (ty + 1) * PX + tx + 1;
    const T *__restrict__ E = (const T *)A.e;
    const double *__restrict__ G = A.G;
    const double *__restrict__ sig = A.sigma;
    T *__restrict__ shat = (T *)A.shat;
    // whether each staged cell lies on a Dirichlet x or y face (z: per plane)
    bool dxy[2];
    for (int k = 0; k < 2; ++k) {
        const int xm = mir(x0 - 1 + cells.lx[k], m), ym = mir(y0 - 1 + cells.ly[k], m);
        dxy[k] = is_dir<2>(xm, ym, 0, m, L.dir);
    }

    double pe[2] = {0.0, 0.0}, ps[2] = {1.0, 1.0};
    double s_next = 0.0, u_next = 0.0;
    auto fetch = [&](int zz) {
        const int zm = mir(zz, m);
        const size_t zoff = (size_t)zm * plane;
        const bool dz = ((L.dir & 16u) && zm == 0) || ((L.dir & 32u) && zm == m - 1);
        for (int k = 0; k < 2; ++k) {
            if (k == 1 && !cells.two) break;
            const size_t q = zoff + cells.q[k];
            double v = A.escale * (double)E[q];
            if (dz || dxy[k]) v = G ? G[q] : 0.0;
            pe[k] = v;
            if (SIG) ps[k] = sig[q];
        }
    };
    auto put = [&](int slot) {
        se[slot][threadIdx.x] = pe[0];
        if (cells.two) se[slot][threadIdx.x + kThreads] = pe[1];
        if (SIG) {
            ss[slot][threadIdx.x] = ps[0];
            if (cells.two) ss[slot][threadIdx.x + kThreads] = ps[1];
        }
    };
    unsigned long long nb = 0;
    fetch(z0 - 1);
    put(0);
    fetch(z0);
    put(1);
    fetch(z0 + 1);
    if (own) {
        s_next = A.s[(size_t)z0 * plane + cxy];
        u_next = A.u[(size_t)z0 * plane + cxy];
    }
    for (int z = z0; z < z1; ++z) {
        const int k = z - z0;
        const int sm = k % RING, sc = (k + 1) % RING, sp = (k + 2) % RING;
        put(sp);
        const double s_c = s_next, u_c = u_next;
        if (z + 1 < z1) {
            fetch(z + 2);
            if (own) {
                s_next = A.s[(size_t)(z + 1) * plane + cxy];
                u_next = A.u[(size_t)(z + 1) * plane + cxy];
            }
        }
        __syncthreads();
        if (own) {
            const size_t c = (size_t)z * plane + cxy;
            const double *Pe[3] = {se[sm], se[sc], se[sp]};
            const double *Ps[3] = {ss[SIG ? sm : 0], ss[SIG ? sc : 0], ss[SIG ? sp : 0]};
            const double ec = Pe[1][ctr];
            A.u[c] = u_c + ec;
            if (is_dir<3>(x, y, z, m, L.dir)) {
                A.s[c] = 0.0;
                if (shat) shat[c] = T(0);
            } else {
                const double sgc = SIG ? Ps[1][ctr] : 1.0;
                double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int cls = (dx != 0) + (dy != 0) + (dz != 0);
                            if (cls == 0 || (!RAD && cls != 1)) continue;
                            const int o = ctr + dy * PX + dx;
                            const double du = Pe[dz + 1][o] - ec;
                            if (SIG)
                                acc[cls - 1] += (Ps[dz + 1][o] + sgc) * du;
                            else
                                acc[cls - 1] += du;
                        }
                    }
                }
                const double sw = acc[0] + 0.5 * acc[1] + (1.0 / 3.0) * acc[2];
                const double Le = (SIG ? 0.5 * L.scale * sw : L.scale * sw) + L.a * ec;
                const double sn = s_c - Le;
                A.s[c] = sn;
                if (shat) shat[c] = (T)(sn * A.shat_scale);
                const unsigned long long b = dbits(sn);
                nb = b > nb ? b : nb;
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(nb, off, 64);
        nb = o > nb ? o : nb;
    }
    if ((threadIdx.x & 63) == 0 && nb) {
        const unsigned b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z) + threadIdx.x / 64;
        atomicMax(A.norm + (b % kRedSlots) * kRedStride, nb);
    }
}

// Two relaxations of a 3D level (sigma = 1) in one pass, marching in z:
// relaxation 1 runs on the tile plus a one-node halo of every plane as soon
// as the input planes below and above it are in LDS, relaxation 2 on the tile
// itself one plane behind, from relaxation 1's plane; the level is read and
// written once for both.  Each plane's part in the neighbour sums (as the
// plane below or above a node, and as its own plane) is formed once per cell;
// a node carries its partial sum from plane to plane in one register.
//
// The input planes (values on the tile plus a two-node halo, source on the
// relaxation-1 region) travel from global memory straight into a ring of
// LDS slots (direct-to-LDS loads, no registers), two planes ahead of the
// plane being relaxed, so that a block keeps several planes of loads in
// flight.  Every wavefront issues the same number of those loads per plane
// (the slots are padded to two loads per thread), which makes the number of
// loads still outstanding when a plane is needed a constant: the wait before
// the barrier names it.
//
// Tiles are balanced: the tile width is m / ceil(m / 64) rounded up (57 at
// m = 513 rather than eight tiles of 64 and one of a single column), and so
// are the z chunks.  Consecutive tiles in (x, y, z) order go to one XCD
// (dispatch deals blocks to the XCDs in turn), so that the halo rows two
// neighbouring tiles share are read through the same L2.
constexpr int TY2 = 8, ZC2 = 32, kThreads2 = TX * TY2;  // tile rows, z chunk (at most) and block
constexpr int IXM = TX + 4, IY = TY2 + 4;               // input plane, halo 2 (at most 68 x 12)
constexpr int SXM = TX + 2, SY = TY2 + 2;               // relaxation-1 plane, halo 1 (at most 66 x 10)
constexpr int kSlotCells = 2 * kThreads2;               // 1024 cells per staged array of a slot
static_assert(IXM * IY <= kSlotCells && SXM * SY <= kSlotCells, "two staged cells per thread");

// s_waitcnt: at most VM vector-memory and LGKM LDS operations of this
// wavefront still outstanding (expcnt not waited for).
template <int VM, int LGKM>
__device__ __forceinline__ void wait_counts()
{
    static_assert(VM >= 0 && VM < 64 && LGKM >= 0 && LGKM < 16, "counter range");
    __builtin_amdgcn_s_waitcnt((VM & 15) | ((VM >> 4) << 14) | (7 << 4) | (LGKM << 8));
}

// Workgroup barrier for LDS traffic: the wavefront's own LDS writes are done
// and at most VM of its direct-to-LDS loads are outstanding; the compiler may
// not move memory accesses across it.
template <int VM>
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    wait_counts<VM, 0>();
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Direct-to-LDS load in the scalar-base form: lane i reads base + off (off
// per lane, 32 bits) and writes LDS byte address lds + 4 i.
__device__ __forceinline__ void lds_load_word_s(const void *base, unsigned off, unsigned lds)
{
    asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dword %0, %1" ::"v"(off), "s"(base), "s"(lds)
                 : "memory", "m0");
}

// Running max of |r| as the bit pattern the stop test uses (order-independent,
// NaN above +inf): in FP32 the max of the float bits, widened at the end
// (the widening is monotone), in FP64 the bits themselves.
__device__ __forceinline__ unsigned res_bits(float r) { return __float_as_uint(r) & 0x7fffffffu; }
__device__ __forceinline__ unsigned long long res_bits(double r) { return dbits(r); }
__device__ __forceinline__ unsigned long long res_widen(unsigned b) { return dbits((double)__uint_as_float(b)); }
__device__ __forceinline__ unsigned long long res_widen(unsigned long long b) { return b; }

// The ring holds NSLOT planes (values on the tile plus halo 2, source on the
// relaxation-1 region): plane i + 2 is staged while plane i is relaxed, into
// the slot of plane i - 1.  With three slots, the march is unrolled by three
// so that the slots are fixed per copy.
constexpr int NSLOT = 3, kAhead = NSLOT - 1;

// One tile of the paired relaxation: TWL lanes across (tw <= TWL of them own
// columns x0 .. x0 + tw - 1), kThreads2 / TWL rows from y0, planes z0 .. z1 - 1.
template <typename T, int RAD, int TWL>
__device__ __forceinline__ void pair3d_tile(T (*ring)[2][kSlotCells], T *s1, const T *__restrict__ ein,
                                            T *__restrict__ eout, const T *__restrict__ g,
                                            const double *__restrict__ G, const Level &L,
                                            unsigned long long *__restrict__ pres, int x0, int y0, int z0, int z1,
                                            int tw)
{
    constexpr int WPC = sizeof(T) / 4;     // 32-bit words per cell
    constexpr int LPA = 2 * WPC;           // direct loads per wavefront per staged array and plane
    constexpr int LPP = 2 * LPA;           // ... per plane (values and source)
    constexpr int THL = kThreads2 / TWL;   // rows of the tile
    constexpr int TWMAX = TWL == TX ? TX : 1;  // widest tw of the shape (the column tiles own one column)
    static_assert((TWMAX + 4) * (THL + 4) <= kSlotCells && (TWMAX + 2) * (THL + 2) <= SXM * SY, "tile fits the LDS");
    typedef decltype(res_bits(T(0))) RB;

    const int m = L.m;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
    const int lane = tid & 63;
    const unsigned ring_lds = __builtin_amdgcn_readfirstlane(
        (unsigned)(size_t)(__attribute__((address_space(3))) T *)&ring[0][0][0]);  // LDS byte address
    const int IX = tw + 4, SX = tw + 2;
    const int NI = IX * (THL + 4), NS = SX * (THL + 2);
    const int tx = tid % TWL, ty = tid / TWL;
    const int x = x0 + tx, y = y0 + ty;
    const bool own = tx < tw && x < m && y < m;
    const size_t plane_bytes = (size_t)m * m * sizeof(T);
    const unsigned own_off = own ? ((unsigned)y * (unsigned)m + (unsigned)x) * (unsigned)sizeof(T) : 0u;
    const unsigned lam = (unsigned)L.lam, Nf = (unsigned)L.N;

    // image of a coordinate; the cells an owned node depends on lie within
    // one reflection, those past it (small levels, padding) are clamped into
    // the grid and never used
    auto img = [&](int c) { return min(max(mir(c, m), 0), m - 1); };
    // per-lane byte offsets (within a plane) of this thread's direct loads:
    // load j of the wavefront fills words (wave * LPA + j) * 64 + lane of the array
    unsigned qe[LPA], qg[LPA];
#pragma unroll
    for (int j = 0; j < LPA; ++j) {
        const int w = (wave * LPA + j) * 64 + lane;
        const int cell = w / WPC, half = w % WPC;
        int ly = cell / IX, lx = cell - ly * IX;
        if (cell >= NI) ly = lx = 2;  // padding: any cell of the grid
        qe[j] = ((unsigned)img(y0 - 2 + ly) * (unsigned)m + (unsigned)img(x0 - 2 + lx)) * sizeof(T) + 4 * half;
        ly = cell / SX, lx = cell - ly * SX;
        if (cell >= NS) ly = lx = 1;
        qg[j] = ((unsigned)img(y0 - 1 + ly) * (unsigned)m + (unsigned)img(x0 - 1 + lx)) * sizeof(T) + 4 * half;
    }
    // stage input plane zz into slot s
    auto issue = [&](int zz, int s) {
        const size_t zo = (size_t)mir(zz, m) * plane_bytes;
        const char *pe = (const char *)ein + zo, *pg = (const char *)g + zo;
        const unsigned se = ring_lds + (unsigned)(s * 2 * kSlotCells * sizeof(T)) + wave * LPA * 256;
        const unsigned sg = se + kSlotCells * sizeof(T);
#pragma unroll
        for (int j = 0; j < LPA; ++j) lds_load_word_s(pe, qe[j], se + j * 256);
#pragma unroll
        for (int j = 0; j < LPA; ++j) lds_load_word_s(pg, qg[j], sg + j * 256);
    };

    // relaxation-1 cells of this thread (tid, tid + kThreads2): position in
    // the input and relaxation-1 planes, x/y Dirichlet faces and the offset
    // of their Dirichlet value in G
    const bool one_s = tid < NS, two_s = tid + kThreads2 < NS;
    int sidx[2], sin_c[2], swr;  // swr: where the first cell's result goes (an unused cell when tid >= NS)
    unsigned gxy[2];
    bool sdxy[2];
    for (int k = 0; k < 2; ++k) {
        const int idx = k == 0 ? min(tid, NS - 1) : (two_s ? tid + kThreads2 : 0);
        const int ly = idx / SX, lx = idx - ly * SX;
        sidx[k] = idx;
        sin_c[k] = (ly + 1) * IX + lx + 1;
        const int xm = img(x0 - 1 + lx), ym = img(y0 - 1 + ly);
        gxy[k] = (unsigned)ym * lam * Nf + (unsigned)xm * lam;
        sdxy[k] = is_dir<2>(xm, ym, 0, m, L.dir);
    }
    swr = one_s ? sidx[0] : SXM * SY - 1;  // tid >= NS only when NS < kThreads2 <= SXM * SY - 1
    const int c2 = (ty + 1) * SX + min(tx, SX - 3) + 1;  // own node in a relaxation-1 plane

    const T scale = (T)L.scale, a = (T)L.a, theta = (T)L.theta;
    const T Wc = RAD ? T(6) + T(0.5) * T(12) + T(1.0 / 3.0) * T(8) : T(6);
    const T tD = theta / (scale * Wc - a);
    // one relaxation of a node with centre value uc and neighbour sum nsum
    auto relax = [&](T uc, T nsum, T gv, T &r) {
        r = scale * (nsum - Wc * uc) + a * uc - gv;
        return uc + tD * r;
    };
    // a plane's part in the neighbour sums, at cell c: its centre value cc, its
    // weight B as the plane below or above a node (centre, faces / 2, corners
    // / 3) and C as the node's own plane (faces, corners / 2)
    auto sums = [&](const T *P, int c, int pitch, T &cc, T &B, T &C) {
        cc = P[c];
        const T cx = (P[c - 1] + P[c + 1]) + (P[c - pitch] + P[c + pitch]);
        if (RAD) {
            const T ck = (P[c - pitch - 1] + P[c - pitch + 1]) + (P[c + pitch - 1] + P[c + pitch + 1]);
            B = cc + T(0.5) * cx + T(1.0 / 3.0) * ck;
            C = cx + T(0.5) * ck;
        } else {
            B = cc;
            C = cx;
        }
    };

    // per node, carried from plane to plane: the neighbour sum of the node's
    // own plane and the one below (part), the last plane's B and centre value;
    // the sum of a node is complete when the plane above arrives
    T a_part[2] = {}, a_B[2] = {}, a_uc[2] = {};  // relaxation-1 cells (input planes)
    T b_part = T(0), b_B = T(0), b_uc = T(0);      // own node (relaxation-1 planes)
    T g_next = T(0), g_cur = T(0);                 // source at the own node, planes zs and z
    RB rb = 0;

    const int np = (z1 + 1) - (z0 - 2) + 1;  // input planes of the chunk (>= 5)
    issue(z0 - 2, 0);
    issue(z0 - 1, 1);
    // iteration it: input plane zi = z0 - 2 + it arrives (slot it % 3),
    // relaxation 1 on plane zi - 1, relaxation 2 on plane zi - 2
    auto step = [&](int it, auto PC) {
        constexpr int P = decltype(PC)::value;                        // it % 3
        constexpr int Pm1 = (P + 2) % 3;                               // (it - 1) % 3
        if (it + 1 < np) lds_barrier<LPP>();  // plane it + 1 was issued after plane it
        else lds_barrier<0>();
        const int zi = z0 - 2 + it;
        const T *E = &ring[P][0][0];
        T ncc[2], nB[2], nC[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (k == 1 && !two_s) break;
            sums(E, sin_c[k], IX, ncc[k], nB[k], nC[k]);
        }
        const int zs = zi - 1;
        g_cur = g_next;
        if (it >= 2) {
            const int zsm = mir(zs, m);
            const bool zd = ((L.dir & 16u) && zsm == 0) || ((L.dir & 32u) && zsm == m - 1);
            const T *S = &ring[Pm1][1][0];
            g_next = S[c2];
            // Dirichlet cells take their value by selection, so that the
            // common case (no Dirichlet data: zero) runs without branches
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (k == 1 && !two_s) break;
                T r;
                T v = relax(a_uc[k], a_part[k] + nB[k], S[sidx[k]], r);
                const bool dir = zd || sdxy[k];
                if (G) {
                    if (dir) v = (T)G[(size_t)zsm * lam * Nf * Nf + gxy[k]];
                } else {
                    v = dir ? T(0) : v;
                }
                s1[k == 0 ? swr : sidx[1]] = v;
            }
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (k == 1 && !two_s) break;
            a_part[k] = a_B[k] + nC[k];
            a_B[k] = nB[k];
            a_uc[k] = ncc[k];
        }
        lds_barrier<63>();
        // the slot of plane it - 1 is free: stage plane it + 2 there
        if (it + kAhead < np) issue(zi + kAhead, Pm1);
        if (it >= 2) {
            T bcc, bB, bC;
            sums(s1, c2, SX, bcc, bB, bC);  // relaxation-1 plane zs
            const int z = zs - 1;
            if (it >= 4 && z < z1) {
                T r;
                T v = relax(b_uc, b_part + bB, g_cur, r);
                const bool dir = is_dir<3>(x, y, z, m, L.dir);
                if (G) {
                    if (dir && own) v = (T)G[lin(x * L.lam, y * L.lam, z * L.lam, L.N)];
                } else {
                    v = dir ? T(0) : v;
                }
                if (pres) {
                    const RB b = res_bits(r);
                    rb = (own && !dir && b > rb) ? b : rb;
                }
                if (own) *(T *)((char *)eout + (size_t)z * plane_bytes + own_off) = v;
            }
            b_part = b_B + bC;
            b_B = bB;
            b_uc = bcc;
        }
    };
    for (int it = 0; it < np; it += 3) {
        step(it, std::integral_constant<int, 0>());
        if (it + 1 >= np) break;
        step(it + 1, std::integral_constant<int, 1>());
        if (it + 2 >= np) break;
        step(it + 2, std::integral_constant<int, 2>());
    }
    if (pres) {
        unsigned long long rw = res_widen(rb);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(rw, off, 64);
            rw = o > rw ? o : rw;
        }
        if ((threadIdx.x & 63) == 0 && rw) {
            const unsigned b = blockIdx.x + threadIdx.x / 64;
            atomicMax(pres + (b % kRedSlots) * kRedStride, rw);
        }
    }
}

// The paired relaxation's launch: per z chunk, ntx x nty tiles of tw x 8
// columns, then ncy tiles of 4 x 128 for the last column of a 64k + 1 level
// (as in k_sweep3d).  Consecutive tiles go to one XCD (dispatch deals blocks
// to the XCDs in turn), so that the halo rows two neighbouring tiles share are
// read through the same L2.
template <typename T, int RAD>
__global__ __launch_bounds__(kThreads2) void k_sweep3d2(const T *__restrict__ ein, T *__restrict__ eout,
                                                       const T *__restrict__ g, const double *__restrict__ G,
                                                       Level L, unsigned long long *__restrict__ pres,
                                                       int tw, int zc, int ntx, int nty, int ncy)
{
    __shared__ T ring[NSLOT][2][kSlotCells];  // [slot][values, source][cell]
    __shared__ T s1[SXM * SY];                // relaxation-1 plane
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int per = ntx * nty + ncy;
    const int bz = t / per, r = t - bz * per;
    const int z0 = bz * zc, z1 = min(L.m, z0 + zc);
    if (r < ntx * nty)
        pair3d_tile<T, RAD, TX>(ring, s1, ein, eout, g, G, L, pres, (r % ntx) * tw, (r / ntx) * TY2, z0, z1, tw);
    else
        pair3d_tile<T, RAD, kColW>(ring, s1, ein, eout, g, G, L, pres, ntx * tw, (r - ntx * nty) * kColRows, z0,
                                   z1, 1);
}

// s_waitcnt for a vector-memory count known only at run time (wave-uniform,
// 0 .. 15): a branch to the matching constant wait.
__device__ __forceinline__ void wait_vm(int n)
{
    switch (n) {
    case 0: wait_counts<0, 15>(); break;
    case 1: wait_counts<1, 15>(); break;
    case 2: wait_counts<2, 15>(); break;
    case 3: wait_counts<3, 15>(); break;
    case 4: wait_counts<4, 15>(); break;
    case 5: wait_counts<5, 15>(); break;
    case 6: wait_counts<6, 15>(); break;
    case 7: wait_counts<7, 15>(); break;
    case 8: wait_counts<8, 15>(); break;
    case 9: wait_counts<9, 15>(); break;
    case 10: wait_counts<10, 15>(); break;
    case 11: wait_counts<11, 15>(); break;
    case 12: wait_counts<12, 15>(); break;
    case 13: wait_counts<13, 15>(); break;
    case 14: wait_counts<14, 15>(); break;
    default: wait_counts<15, 15>(); break;
    }
}

// Interpolation of the pending variation of level nu+1 into level nu (3D,
// m >= 33), marching in z.  The pending variation at coarse node X is
// p(X) = ec(X) - efin(2X) (efin = 0 on the level's first visit of a cycle);
// every fine node takes efin + the trilinear interpolant of p, which at a
// coarse node is ec itself.  A block owns 64 x 8 fine columns (4 x 128 for
// the last column of a 64k + 1 level) and a chunk of fine planes, and marches
// in steps of one coarse plane (two fine planes), with p of the 33 x 5
// (3 x 65) coarse columns it needs for two coarse planes in an LDS ring.
// Every input travels straight into LDS (direct-to-LDS loads, as in
// k_sweep3d2), two steps before it is needed: the stale values of the fine
// planes (a wavefront loads the cells of its own threads) and ec, efin(2X)
// of the coarse cells (wavefronts 0 .. 2, one cell per thread).  A step waits
// once, for the loads issued two steps back: the loads issued one step back
// may stay in flight, and their count is known.
constexpr int kProStages = 4;  // fine planes of stale values in the ring (two steps)

// largest staged coarse region of the two tile shapes: 3 x 65 (4 x 128 fine
// columns), against 33 x 5 for 64 x 8
constexpr int kProNC = 3 * 65, kProCW = (kProNC + 63) / 64;

template <typename T, bool FIRST, int TW>
__device__ __forceinline__ void prolong3d_tile(T (*sp)[kProNC], T (*sc)[FIRST ? 1 : 2][kProCW * 64],
                                               T (*sst)[kThreads], const T *__restrict__ ec,
                                               const T *__restrict__ efin, T *__restrict__ efout, int mc, int x0,
                                               int y0, int z0, int z1)
{
    constexpr int TH = kThreads / TW;                  // fine rows of the tile
    constexpr int CXT = TW / 2 + 1, CYT = TH / 2 + 1;  // coarse columns of the tile
    constexpr int NC = CXT * CYT;                      // staged coarse cells
    constexpr int CW = (NC + 63) / 64;                 // wavefronts that stage them
    constexpr int WPC = sizeof(T) / 4;                 // 32-bit words per cell
    constexpr int NPA = FIRST ? 1 : 2;                 // staged coarse arrays: ec (and efin(2X))
    static_assert(NC <= kProNC && CW <= kProCW, "staging fits");
    const int m = 2 * mc - 1;
    const int tid = threadIdx.x;
    const int tx = tid % TW, ty = tid / TW;
    const int x = x0 + tx, y = y0 + ty;
    const bool own = x < m && y < m;
    const size_t plane = (size_t)m * m, cplane = (size_t)mc * mc;
    const unsigned cxy = (unsigned)(own ? y : 0) * (unsigned)m + (unsigned)(own ? x : 0);
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid & 63;
    const bool cwave = wave < CW;

    // direct loads of the coarse cells: load j of a staging wavefront fills
    // words (wave * WPC + j) * 64 + lane, i.e. cells of its own threads
    // (beyond the staged cells: a clamped cell, never used)
    unsigned qc[WPC], qf[WPC];
#pragma unroll
    for (int j = 0; j < WPC; ++j) {
        const int w = (wave * WPC + j) * 64 + lane;
        const int cell = min(w / WPC, NC - 1), half = w % WPC;
        const int cy = cell / CXT, cx = cell - cy * CXT;
        const int X = min(x0 / 2 + cx, mc - 1), Y = min(y0 / 2 + cy, mc - 1);
        qc[j] = ((unsigned)Y * (unsigned)mc + (unsigned)X) * sizeof(T) + 4 * half;
        qf[j] = ((unsigned)(2 * Y) * (unsigned)m + (unsigned)(2 * X)) * sizeof(T) + 4 * half;
    }
    // direct loads of the stale values of this wavefront's cells
    unsigned qst[WPC];
#pragma unroll
    for (int j = 0; j < WPC; ++j) {
        const int w = (wave * WPC + j) * 64 + lane;
        const int cell = w / WPC, half = w % WPC;
        const int cx = x0 + cell % TW, cy = y0 + cell / TW;
        const unsigned off = (cx < m && cy < m) ? (unsigned)cy * (unsigned)m + (unsigned)cx : 0u;
        qst[j] = off * sizeof(T) + 4 * half;
    }
    const unsigned sc_lds = __builtin_amdgcn_readfirstlane(
        (unsigned)(size_t)(__attribute__((address_space(3))) T *)&sc[0][0][0]);
    const unsigned sst_lds = __builtin_amdgcn_readfirstlane(
        (unsigned)(size_t)(__attribute__((address_space(3))) T *)&sst[0][0]);
    // stage coarse plane Z (clamped into the grid) into staging slot Z & 1;
    // returns the loads this wavefront issued
    auto issue_coarse = [&](int Z) {
        if (!cwave) return 0;
        Z = min(Z, mc - 1);
        const unsigned lds = sc_lds + (unsigned)((Z & 1) * NPA * kProCW * 64 * sizeof(T)) + wave * WPC * 256;
        const char *bc = (const char *)ec + (size_t)Z * cplane * sizeof(T);
#pragma unroll
        for (int j = 0; j < WPC; ++j) lds_load_word_s(bc, qc[j], lds + j * 256);
        if (!FIRST) {
            const char *bf = (const char *)efin + (size_t)(2 * Z) * plane * sizeof(T);
#pragma unroll
            for (int j = 0; j < WPC; ++j) lds_load_word_s(bf, qf[j], lds + kProCW * 64 * sizeof(T) + j * 256);
        }
        return NPA * WPC;
    };
    // stage the stale values of fine plane z (if it is in the chunk)
    auto issue_stale = [&](int z) {
        if (FIRST || z >= z1) return 0;
        const char *base = (const char *)efin + (size_t)z * plane * sizeof(T);
        const unsigned lds = sst_lds + (unsigned)((z - z0) % kProStages * kThreads * sizeof(T)) + wave * WPC * 256;
#pragma unroll
        for (int j = 0; j < WPC; ++j) lds_load_word_s(base, qst[j], lds + j * 256);
        return WPC;
    };
    // p of the staged coarse plane Z into ring slot Z & 1 (staging threads)
    auto build_p = [&](int Z) {
        if (tid < NC) {
            const T c = sc[Z & 1][0][tid];
            sp[Z & 1][tid] = FIRST ? c : c - sc[Z & 1][FIRST ? 0 : 1][tid];
        }
    };
    const int oi = x & 1, oj = y & 1;
    const int c00 = (ty >> 1) * CXT + (tx >> 1);  // coarse cell (X, Y) of this column in the tile
    const T wxy = (oi && oj) ? T(0.25) : ((oi || oj) ? T(0.5) : T(1));
    // the interpolant of p within one coarse plane at this column (x, y)
    auto in_plane = [&](int slot) {
        const T *P = sp[slot];
        T acc = P[c00];
        if (oi) acc += P[c00 + 1];
        if (oj) acc += P[c00 + CXT];
        if (oi && oj) acc += P[c00 + CXT + 1];
        return acc;
    };

    // prologue: coarse planes Zs, Zs + 1 (built now) and the first two fine
    // planes; then coarse plane Zs + 2 and fine planes z0 + 2, z0 + 3 (in flight)
    const int Zs = z0 / 2;
    issue_coarse(Zs);
    asm volatile("" ::: "memory");
    wait_counts<0, 15>();
    asm volatile("" ::: "memory");
    build_p(Zs);
    issue_coarse(Zs + 1);
    issue_stale(z0);
    issue_stale(z0 + 1);
    asm volatile("" ::: "memory");
    wait_counts<0, 15>();
    asm volatile("" ::: "memory");
    build_p(Zs + 1);
    int inflight = issue_coarse(Zs + 2);  // loads issued one step back
    inflight += issue_stale(z0 + 2);
    inflight += issue_stale(z0 + 3);
    for (int z = z0; z < z1; z += 2) {
        const int Z = z >> 1;
        if (z > z0) {
            // the loads of two steps back (coarse plane Z + 1, fine planes z, z + 1) are complete
            asm volatile("" ::: "memory");
            wait_vm(inflight);
            asm volatile("" ::: "memory");
            __syncthreads();  // every thread is done with p of coarse plane Z - 1
            build_p(Z + 1);
            __syncthreads();
            // loads for two steps on: coarse plane Z + 3 (staging slot of Z + 1,
            // just read), fine planes z + 4, z + 5 (slots of z, z + 1, read below)
        } else {
            lds_barrier<63>();
        }
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            if (z + d >= z1) break;
            const T stale = FIRST ? T(0) : sst[(z + d - z0) % kProStages][tid];
            if (own) {
                T acc = in_plane(Z & 1);
                if (d) acc += in_plane((Z + 1) & 1);
                const T w = d ? T(0.5) * wxy : wxy;
                efout[(size_t)(z + d) * plane + cxy] = stale + w * acc;
            }
        }
        asm volatile("" ::: "memory");
        wait_counts<63, 0>();  // this thread's stale reads are done before their slots are refilled
        inflight = z + 4 < z1 ? issue_coarse(Z + 3) : 0;  // needed two steps on, if there is such a step
        inflight += issue_stale(z + 4);
        inflight += issue_stale(z + 5);
    }
    wait_counts<0, 15>();  // no load may still write the workgroup's LDS when it ends
}

// The interpolation's launch: per z chunk, ntx x nty tiles of 64 x 8 fine
// columns, then ncy tiles of 4 x 128 for the last column of a 64k + 1 level.
template <typename T, bool FIRST>
__global__ __launch_bounds__(kThreads) void k_prolong3d(const T *__restrict__ ec, const T *__restrict__ efin,
                                                        T *__restrict__ efout, int mc, int zc, int ntx, int nty,
                                                        int ncy)
{
    __shared__ T sp[2][kProNC];                            // p of two coarse planes
    __shared__ T sc[2][FIRST ? 1 : 2][kProCW * 64];        // staged ec, efin(2X) of two coarse planes
    __shared__ T sst[FIRST ? 1 : kProStages][kThreads];    // stale values, one fine plane per slot
    const int m = 2 * mc - 1;
    const int per = ntx * nty + ncy;
    const int bz = blockIdx.x / per, r = blockIdx.x - bz * per;
    const int z0 = bz * zc, z1 = min(m, z0 + zc);  // zc even: z0 even
    if (r < ntx * nty)
        prolong3d_tile<T, FIRST, TX>(sp, sc, sst, ec, efin, efout, mc, (r % ntx) * TX, (r / ntx) * TY, z0, z1);
    else
        prolong3d_tile<T, FIRST, kColW>(sp, sc, sst, ec, efin, efout, mc, ntx * TX, (r - ntx * nty) * kColRows, z0,
                                        z1);
}

// The cycle-end pass with a constant coefficient, its inputs loaded straight
// into LDS two planes ahead (direct-to-LDS loads, as in k_sweep3d2): the
// values of the cycle (precision T) on the tile plus a one-node halo, and u,
// s at the tile's nodes.  Each thread converts its two staged cells to FP64
// (escale, Dirichlet values) into the ring of FP64 planes the stencil reads.
// A wavefront loads exactly the cells its own threads convert or own, so its
// own wait suffices before it reads them, and one barrier per plane
// publishes the converted plane.  Per plane and wavefront: 2 WPC loads of
// values, 2 of u and 2 of s, whatever the tile.
template <typename T, int RAD, int TW, bool HASG>
__device__ __forceinline__ void cycle_end3d_tile(double (*se)[NPMAX], T (*sraw)[kSlotCells],
                                                 double (*sus)[2][kThreads], const CycleEndArgs &A, int x0,
                                                 int y0, int z0, int z1, unsigned long long &nb)
{
    constexpr int WPC = sizeof(T) / 4;             // 32-bit words per value
    constexpr int GS = 2 * WPC + 4;                // loads per wavefront and plane
    constexpr int PXT = TW + 2, NPT = PXT * (kThreads / TW + 2);
    const Level &L = A.L;
    const int m = L.m;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
    const int tx = tid % TW, ty = tid / TW;
    const int x = x0 + tx, y = y0 + ty;
    const bool own = x < m && y < m;
    const size_t plane = (size_t)m * m;
    const unsigned cxy = (unsigned)(own ? y : 0) * (unsigned)m + (unsigned)(own ? x : 0);
    const int ctr = (ty + 1) * PXT + tx + 1;
    auto img = [&](int c) { return min(max(mir(c, m), 0), m - 1); };
    const T *__restrict__ E = (const T *)A.e;
    const double *__restrict__ G = A.G;  // used only when HASG (the first cycle)
    T *__restrict__ shat = (T *)A.shat;

    // this thread's staged cells (tid, tid + kThreads): offsets and x/y Dirichlet faces
    unsigned qc[2];
    bool dxy[2], has[2];
    for (int k = 0; k < 2; ++k) {
        const int c = tid + k * kThreads;
        has[k] = c < NPT;
        const int ly = (has[k] ? c : 0) / PXT, lx = (has[k] ? c : 0) % PXT;
        const int xm = img(x0 - 1 + lx), ym = img(y0 - 1 + ly);
        qc[k] = (unsigned)ym * (unsigned)m + (unsigned)xm;
        dxy[k] = is_dir<2>(xm, ym, 0, m, L.dir);
    }
    // direct loads: values, load j = kk * WPC + jj fills words jj * 64 + lane of
    // cells kk * kThreads + wave * 64 .. + 63 (this wavefront's threads' cells);
    // u and s, load j fills words j * 64 + lane of cells wave * 64 .. + 63
    unsigned qe[2 * WPC], qo[2];
#pragma unroll
    for (int j = 0; j < 2 * WPC; ++j) {
        const int kk = j / WPC, jj = j % WPC;
        const int w = jj * 64 + lane, c = kk * kThreads + wave * 64 + w / WPC, half = w % WPC;
        const int cc = c < NPT ? c : 0;
        const int ly = cc / PXT, lx = cc % PXT;
        qe[j] = ((unsigned)img(y0 - 1 + ly) * (unsigned)m + (unsigned)img(x0 - 1 + lx)) * sizeof(T) + 4 * half;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int w = j * 64 + lane, c = wave * 64 + w / 2, half = w % 2;
        const int cx = x0 + c % TW, cy = y0 + c / TW;
        const unsigned off = (cx < m && cy < m) ? (unsigned)cy * (unsigned)m + (unsigned)cx : 0u;
        qo[j] = off * 8 + 4 * half;
    }
    const unsigned raw_lds = __builtin_amdgcn_readfirstlane(
        (unsigned)(size_t)(__attribute__((address_space(3))) T *)&sraw[0][0]);
    const unsigned us_lds = __builtin_amdgcn_readfirstlane(
        (unsigned)(size_t)(__attribute__((address_space(3))) double *)&sus[0][0][0]);
    // values of plane zz into raw slot (zz - z0) & 1
    auto issue_e = [&](int zz) {
        const char *base = (const char *)E + (size_t)mir(zz, m) * plane * sizeof(T);
        const unsigned lds = raw_lds + (unsigned)(((zz - z0) & 1) * kSlotCells * sizeof(T));
#pragma unroll
        for (int j = 0; j < 2 * WPC; ++j) {
            const int kk = j / WPC, jj = j % WPC;
            lds_load_word_s(base, qe[j], lds + (unsigned)((kk * kThreads + wave * 64) * sizeof(T)) + jj * 256);
        }
    };
    // u and s of plane zz into slot (zz - z0) & 1
    auto issue_us = [&](int zz) {
        const size_t zo = (size_t)zz * plane * sizeof(double);
        const unsigned lds = us_lds + (unsigned)(((zz - z0) & 1) * 2 * kThreads * sizeof(double)) + wave * 512;
#pragma unroll
        for (int j = 0; j < 2; ++j) lds_load_word_s((const char *)A.u + zo, qo[j], lds + j * 256);
#pragma unroll
        for (int j = 0; j < 2; ++j)
            lds_load_word_s((const char *)A.s + zo, qo[j], lds + kThreads * sizeof(double) + j * 256);
    };
    // this thread's cells of plane zz, converted into FP64 ring slot (zz - z0 + 1) & 3
    auto convert = [&](int zz) {
        const int zm = mir(zz, m);
        const bool dz = ((L.dir & 16u) && zm == 0) || ((L.dir & 32u) && zm == m - 1);
        const T *R = sraw[(zz - z0) & 1];
        double *P = se[(zz - z0 + 1) & 3];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (!has[k]) continue;
            double v = A.escale * (double)R[tid + k * kThreads];
            if (dz || dxy[k]) v = HASG ? G[(size_t)zm * plane + qc[k]] : 0.0;
            P[tid + k * kThreads] = v;
        }
    };

    issue_e(z0 - 1);
    issue_e(z0);
    asm volatile("" ::: "memory");
    wait_counts<0, 15>();
    asm volatile("" ::: "memory");
    convert(z0 - 1);
    convert(z0);
    asm volatile("" ::: "memory");
    wait_counts<63, 0>();  // the raw slots are read before they are refilled
    issue_e(z0 + 1);
    issue_us(z0);
    if (z0 + 1 < z1) {
        issue_e(z0 + 2);
        issue_us(z0 + 1);
    }
    for (int z = z0; z < z1; ++z) {
        // plane z's group (values of z + 1, u and s of z) is complete; the next one may be in flight
        asm volatile("" ::: "memory");
        if (z + 1 < z1) wait_counts<GS, 15>();
        else wait_counts<0, 15>();
        asm volatile("" ::: "memory");
        convert(z + 1);
        lds_barrier<63>();
        const double u_c = sus[(z - z0) & 1][0][tid], s_c = sus[(z - z0) & 1][1][tid];
        if (own) {
            const size_t c = (size_t)z * plane + cxy;
            const double *Pe[3] = {se[(z - z0) & 3], se[(z - z0 + 1) & 3], se[(z - z0 + 2) & 3]};
            const double ec = Pe[1][ctr];
            A.u[c] = u_c + ec;
            if (is_dir<3>(x, y, z, m, L.dir)) {
                A.s[c] = 0.0;
                if (shat) shat[c] = T(0);
            } else {
                double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int cls = (dx != 0) + (dy != 0) + (dz != 0);
                            if (cls == 0 || (!RAD && cls != 1)) continue;
                            acc[cls - 1] += Pe[dz + 1][ctr + dy * PXT + dx] - ec;
                        }
                    }
                }
                const double sw = acc[0] + 0.5 * acc[1] + (1.0 / 3.0) * acc[2];
                const double Le = L.scale * sw + L.a * ec;
                const double sn = s_c - Le;
                A.s[c] = sn;
                if (shat) shat[c] = (T)(sn * A.shat_scale);
                const unsigned long long b = dbits(sn);
                nb = b > nb ? b : nb;
            }
        }
        asm volatile("" ::: "memory");
        wait_counts<63, 0>();  // this thread's reads of the slots refilled below are done
        if (z + 2 < z1) {
            issue_e(z + 3);
            issue_us(z + 2);
        }
    }
    wait_counts<0, 15>();  // no load may still write the workgroup's LDS when it ends
}

template <typename T, int RAD, bool HASG>
__global__ __launch_bounds__(kThreads) void k_cycle_end3d_lds(CycleEndArgs A, int zc, int ntx, int nty, int ncy)
{
    __shared__ double se[4][NPMAX];              // FP64 value planes z - 1, z, z + 1 and the next
    __shared__ T sraw[2][kSlotCells];            // raw value planes in flight
    __shared__ double sus[2][2][kThreads];       // u, s of two planes
    const int per = ntx * nty + ncy;
    const int bz = blockIdx.x / per, r = blockIdx.x - bz * per;
    const int z0 = bz * zc, z1 = min(A.L.m, z0 + zc);
    unsigned long long nb = 0;
    if (r < ntx * nty)
        cycle_end3d_tile<T, RAD, TX, HASG>(se, sraw, sus, A, (r % ntx) * TX, (r / ntx) * TY, z0, z1, nb);
    else
        cycle_end3d_tile<T, RAD, kColW, HASG>(se, sraw, sus, A, ntx * TX, (r - ntx * nty) * kColRows, z0, z1, nb);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(nb, off, 64);
        nb = o > nb ? o : nb;
    }
    if ((threadIdx.x & 63) == 0 && nb) {
        const unsigned b = blockIdx.x + threadIdx.x / 64;
        atomicMax(A.norm + (b % kRedSlots) * kRedStride, nb);
    }
}

// One restriction step (Algorithm 1, eq. (4)) from a 3D level of mf >= 33
// nodes per axis, marching in z.  Coarse node X averages the fine 3^3 block
// around 2X with weights hat(p/2) per axis over 8; images outside the grid.
// A block owns 64 x 8 coarse columns; each fine plane (a 129 x 17 region) is
// staged once, loaded straight into a three-slot LDS ring two planes ahead of
// use (direct-to-LDS loads, the same number per wavefront and plane); each
// thread forms its column's in-plane weighted sum h(zf) and combines
// h(2Z-1), h(2Z), h(2Z+1) with (1/2, 1, 1/2).
constexpr int RCX = 64, RCY = 8;                                   // coarse tile
constexpr int RFX = 2 * RCX + 1, RFY = 2 * RCY + 1, RNP = RFX * RFY;  // staged fine plane
constexpr int kRSlots = 3;                                         // ring: the plane summed, two in flight

template <typename T>
__global__ __launch_bounds__(kThreads) void k_restrict3d(const T *__restrict__ fine, T *__restrict__ coarse, int mc,
                                                         int zc)
{
    constexpr int WPC = sizeof(T) / 4;                       // 32-bit words per value
    constexpr int NW = kThreads / 64;                        // wavefronts
    constexpr int LPW = (RNP * WPC + 64 * NW - 1) / (64 * NW);  // direct loads per wavefront and plane
    constexpr int SLOT = LPW * NW * 64 / WPC;                // staged cells per slot (padded)
    __shared__ T sf[kRSlots][SLOT];
    const int mf = 2 * mc - 1;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
    const int tx = tid % RCX, ty = tid / RCX;
    const int X0 = blockIdx.x * RCX, Y0 = blockIdx.y * RCY, Z0 = blockIdx.z * zc;
    const int Z1 = min(mc, Z0 + zc);
    const int X = X0 + tx, Y = Y0 + ty;
    const bool own = X < mc && Y < mc;
    const size_t fplane = (size_t)mf * mf;
    // in-plane byte offsets of this wavefront's direct loads: load j fills
    // words (j * NW + wave) * 64 + lane of a slot (fine columns 2 X0 - 1 ..
    // 2 X0 + 2 RCX - 1); the nodes of coarse columns in range need at most
    // one reflection, the rest (past the grid, for small levels, and the
    // padding) are clamped into it and never used
    auto img = [&](int c) { return min(max(mir(c, mf), 0), mf - 1); };
    unsigned q[LPW];
#pragma unroll
    for (int j = 0; j < LPW; ++j) {
        const int w = (j * NW + wave) * 64 + lane;
        const int cell = w / WPC, half = w % WPC;
        const int i = cell < RNP ? cell : 0;
        const int ly = i / RFX, lx = i - ly * RFX;
        q[j] = ((unsigned)img(2 * Y0 - 1 + ly) * (unsigned)mf + (unsigned)img(2 * X0 - 1 + lx)) * sizeof(T) + 4 * half;
    }
    const unsigned sf_lds = __builtin_amdgcn_readfirstlane(
        (unsigned)(size_t)(__attribute__((address_space(3))) T *)&sf[0][0]);
    // fine planes 2 Z0 - 1 .. 2 Z1 - 1; plane zf goes to slot (zf - zf0) % kRSlots
    const int zf0 = 2 * Z0 - 1, zf1 = 2 * Z1 - 1;
    auto issue = [&](int zf) {
        const char *base = (const char *)fine + (size_t)img(zf) * fplane * sizeof(T);
        const unsigned lds = sf_lds + (unsigned)((zf - zf0) % kRSlots * SLOT * sizeof(T)) + wave * 256;
#pragma unroll
        for (int j = 0; j < LPW; ++j) lds_load_word_s(base, q[j], lds + j * NW * 256);
    };
    const int c = (2 * ty + 1) * RFX + 2 * tx + 1;  // fine node 2X, 2Y in the staged plane
    auto hsum = [&](int slot) {
        const T *P = sf[slot];
        const T r0 = T(0.5) * P[c - RFX - 1] + P[c - RFX] + T(0.5) * P[c - RFX + 1];
        const T r1 = T(0.5) * P[c - 1] + P[c] + T(0.5) * P[c + 1];
        const T r2 = T(0.5) * P[c + RFX - 1] + P[c + RFX] + T(0.5) * P[c + RFX + 1];
        return T(0.5) * r0 + r1 + T(0.5) * r2;
    };
    issue(zf0);
    issue(zf0 + 1);  // zf1 >= zf0 + 2
    T hm = T(0), hc = T(0);  // h(2Z - 1), h(2Z)
    for (int zf = zf0; zf <= zf1; ++zf) {
        const int k = zf - zf0;
        // plane zf is complete (plane zf + 1 may be in flight); every thread
        // is done with the slot of plane zf - 1, refilled below
        if (zf + 1 <= zf1) lds_barrier<LPW>();
        else lds_barrier<0>();
        if (zf + 2 <= zf1) issue(zf + 2);
        const T h = hsum(k % kRSlots);
        if (k == 0) {
            hm = h;
        } else if (k & 1) {
            hc = h;
        } else {
            // zf = 2Z + 1: coarse plane Z complete
            const int Z = (zf - 1) / 2;
            if (own) coarse[((size_t)Z * mc + Y) * mc + X] = (T(0.5) * hm + hc + T(0.5) * h) * T(0.125);
            hm = h;
        }
    }
}

}  // namespace

bool sweep3d_supported(int m) { return m >= 33; }

// z chunk of a z-marching launch: at most zmax planes, fewer on small levels
// so that the grid still has about kMinBlocks workgroups.  A chunk costs a
// few halo planes, which a small level can afford; a long chain of dependent
// plane steps on a handful of workgroups it cannot.  Rounded up to `multiple`.
// A positive `req` (the caller's choice) replaces the per-level choice; it is
// clamped to the level.
static int z_chunk(int m, int blocks_xy, int zmax, int multiple, int req)
{
    constexpr long long kMinBlocks = 1024;
    int zc = (int)((long long)m * blocks_xy / kMinBlocks);
    zc = zc < 1 ? 1 : (zc > zmax ? zmax : zc);
    if (req > 0) zc = req < m ? req : m;
    return (zc + multiple - 1) / multiple * multiple;
}

template <typename T>
void launch_cycle_end3d(const Variant &v, const CycleEndArgs &a, hipStream_t st)
{
    const int m = a.L.m;
    if (!v.sigma) {
        // the constant-coefficient pass with its inputs loaded straight into LDS
        const bool split = m >= 65 && (m - 1) % TX == 0;
        const int ntx = split ? (m - 1) / TX : (m + TX - 1) / TX, nty = (m + TY - 1) / TY;
        const int ncy = split ? (m + kColRows - 1) / kColRows : 0;
        const int zc = z_chunk(m, ntx * nty + ncy, ZC, 1, a.zchunk);
        const dim3 grid((ntx * nty + ncy) * ((m + zc - 1) / zc)), block(kThreads);
        // Dirichlet data (the first cycle) in an instantiation of its own, so
        // that the common one has no load the compiler waits for
        if (v.radial && a.G)
            hipLaunchKernelGGL((k_cycle_end3d_lds<T, 1, true>), grid, block, 0, st, a, zc, ntx, nty, ncy);
        else if (v.radial)
            hipLaunchKernelGGL((k_cycle_end3d_lds<T, 1, false>), grid, block, 0, st, a, zc, ntx, nty, ncy);
        else if (a.G)
            hipLaunchKernelGGL((k_cycle_end3d_lds<T, 0, true>), grid, block, 0, st, a, zc, ntx, nty, ncy);
        else
            hipLaunchKernelGGL((k_cycle_end3d_lds<T, 0, false>), grid, block, 0, st, a, zc, ntx, nty, ncy);
        return;
    }
    const dim3 grid((m + TX - 1) / TX, (m + TY - 1) / TY, (m + ZC - 1) / ZC), block(kThreads);
    if (v.radial)
        hipLaunchKernelGGL((k_cycle_end3d<T, 1, 1>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((k_cycle_end3d<T, 0, 1>), grid, block, 0, st, a);
}

template void launch_cycle_end3d<double>(const Variant &, const CycleEndArgs &, hipStream_t);
template void launch_cycle_end3d<float>(const Variant &, const CycleEndArgs &, hipStream_t);

template <typename T>
void launch_sweep3d(const Variant &v, const Level &L, const T *ein, T *eout, const T *g, const T *sig,
                    const double *G, unsigned long long *pres, int zreq, hipStream_t st)
{
    const int m = L.m;
    // m = 64 k + 1: k tiles of 64 columns and the last column in 4 x 128 tiles
    const bool split = m >= 65 && (m - 1) % TX == 0;
    const int ntx = split ? (m - 1) / TX : (m + TX - 1) / TX, nty = (m + TY - 1) / TY;
    const int ncy = split ? (m + kColRows - 1) / kColRows : 0;
    const int zc = z_chunk(m, ntx * nty + ncy, ZC, 1, zreq);
    const dim3 grid((ntx * nty + ncy) * ((m + zc - 1) / zc)), block(kThreads);
    if (v.radial && v.sigma)
        hipLaunchKernelGGL((k_sweep3d<T, 1, 1>), grid, block, 0, st, ein, eout, g, sig, G, L, pres, zc, ntx, nty, ncy);
    else if (v.radial)
        hipLaunchKernelGGL((k_sweep3d<T, 1, 0>), grid, block, 0, st, ein, eout, g, sig, G, L, pres, zc, ntx, nty, ncy);
    else if (v.sigma)
        hipLaunchKernelGGL((k_sweep3d<T, 0, 1>), grid, block, 0, st, ein, eout, g, sig, G, L, pres, zc, ntx, nty, ncy);
    else
        hipLaunchKernelGGL((k_sweep3d<T, 0, 0>), grid, block, 0, st, ein, eout, g, sig, G, L, pres, zc, ntx, nty, ncy);
}

template <typename T>
void launch_sweep3d2(const Variant &v, const Level &L, const T *ein, T *eout, const T *g, const double *G,
                     unsigned long long *pres, int zreq, hipStream_t st)
{
    const int m = L.m;
    // m = 64 k + 1: k tiles of 64 columns and the last column in 4 x 128
    // tiles; otherwise balanced tile widths (at most 64)
    const bool split = m >= 65 && (m - 1) % TX == 0;
    const int tw = split ? TX : (m + (m + TX - 1) / TX - 1) / ((m + TX - 1) / TX);
    const int ntx = split ? (m - 1) / TX : (m + tw - 1) / tw, nty = (m + TY2 - 1) / TY2;
    const int ncy = split ? (m + kColRows - 1) / kColRows : 0;
    const int zt = z_chunk(m, ntx * nty + ncy, ZC2, 1, zreq);          // target z chunk
    const int nzc = (m + zt - 1) / zt, zc = (m + nzc - 1) / nzc;       // balanced
    const int nz = (m + zc - 1) / zc;
    const dim3 grid((ntx * nty + ncy) * nz), block(kThreads2);
    if (v.radial)
        hipLaunchKernelGGL((k_sweep3d2<T, 1>), grid, block, 0, st, ein, eout, g, G, L, pres, tw, zc, ntx, nty, ncy);
    else
        hipLaunchKernelGGL((k_sweep3d2<T, 0>), grid, block, 0, st, ein, eout, g, G, L, pres, tw, zc, ntx, nty, ncy);
}

template void launch_sweep3d2<double>(const Variant &, const Level &, const double *, double *, const double *,
                                      const double *, unsigned long long *, int, hipStream_t);
template void launch_sweep3d2<float>(const Variant &, const Level &, const float *, float *, const float *,
                                     const double *, unsigned long long *, int, hipStream_t);

template <typename T>
void launch_prolong3d(int mc, const T *ec, const T *ef_in, T *ef_out, bool first, int zreq, hipStream_t st)
{
    const int m = 2 * mc - 1;
    // m = 64 k + 1: k tiles of 64 columns and the last column in 4 x 128 tiles
    const bool split = m >= 65 && (m - 1) % TX == 0;
    const int ntx = split ? (m - 1) / TX : (m + TX - 1) / TX, nty = (m + TY - 1) / TY;
    const int ncy = split ? (m + kColRows - 1) / kColRows : 0;
    const int zc = z_chunk(m, ntx * nty + ncy, ZC, 2, zreq);
    const dim3 grid((ntx * nty + ncy) * ((m + zc - 1) / zc)), block(kThreads);
    if (first)
        hipLaunchKernelGGL((k_prolong3d<T, true>), grid, block, 0, st, ec, ef_in, ef_out, mc, zc, ntx, nty, ncy);
    else
        hipLaunchKernelGGL((k_prolong3d<T, false>), grid, block, 0, st, ec, ef_in, ef_out, mc, zc, ntx, nty, ncy);
}

template void launch_prolong3d<double>(int, const double *, const double *, double *, bool, int, hipStream_t);
template void launch_prolong3d<float>(int, const float *, const float *, float *, bool, int, hipStream_t);

template <typename T>
void launch_restrict3d(int mc, const T *fine, T *coarse, int zreq, hipStream_t st)
{
    const int bx = (mc + RCX - 1) / RCX, by = (mc + RCY - 1) / RCY, zc = z_chunk(mc, bx * by, ZC, 1, zreq);
    const dim3 grid(bx, by, (mc + zc - 1) / zc), block(kThreads);
    hipLaunchKernelGGL((k_restrict3d<T>), grid, block, 0, st, fine, coarse, mc, zc);
}

template void launch_restrict3d<double>(int, const double *, double *, int, hipStream_t);
template void launch_restrict3d<float>(int, const float *, float *, int, hipStream_t);

template void launch_sweep3d<double>(const Variant &, const Level &, const double *, double *, const double *,
                                     const double *, const double *, unsigned long long *, int, hipStream_t);
template void launch_sweep3d<float>(const Variant &, const Level &, const float *, float *, const float *,
                                    const float *, const double *, unsigned long long *, int, hipStream_t);

}  // namespace sgml
