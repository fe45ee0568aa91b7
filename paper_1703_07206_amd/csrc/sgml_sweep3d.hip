// sgml_sweep3d.hip -- one relaxation of a 3D level, marching in z.
//
// A block owns a 64 x 8 tile of (x, y) columns and a chunk of z planes.
// Each plane of the level's values (and of the coefficient) is staged once,
// with a one-node halo, in a ring of three LDS planes; a node's 26 (radial)
// or 6 (axis) neighbours are then read from LDS instead of from L1/L2, and
// every value crosses the memory hierarchy about once.  Halo cells outside
// the grid hold the image node, so Neumann faces need no special case.  With
// a constant coefficient the 26 neighbours are summed by class from per-plane
// partial sums (face and corner neighbours within a plane), 8 LDS reads per
// node instead of 26.
#include "sgml_device.h"

namespace sgml {

namespace {

constexpr int TX = 64, TY = 8, ZC = 16;  // tile and z chunk
constexpr int kThreads = TX * TY;
constexpr int PX = TX + 2, PY = TY + 2;  // staged plane with halo

// theta / D: the hardware reciprocal in FP32 (the mixed mode's approximate
// inner solver), a division in FP64.
__device__ __forceinline__ float step_of3(float theta, float D) { return theta * __builtin_amdgcn_rcpf(D); }
__device__ __forceinline__ double step_of3(double theta, double D) { return theta / D; }

template <typename T, int RAD, int SIG>
__global__ __launch_bounds__(kThreads) void k_sweep3d(const T *__restrict__ ein, T *__restrict__ eout,
                                                      const T *__restrict__ g, const T *__restrict__ sig,
                                                      const double *__restrict__ G, Level L,
                                                      unsigned long long *__restrict__ pres)
{
    __shared__ T su[3][PY][PX];
    __shared__ T ss[SIG ? 3 : 1][SIG ? PY : 1][SIG ? PX : 1];
    const int m = L.m;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * ZC;
    const int z1 = min(m, z0 + ZC);
    const int x = x0 + tx, y = y0 + ty;
    const bool own = x < m && y < m;
    const size_t plane = (size_t)m * m;

    auto stage = [&](int slot, int zz) {
        const size_t zoff = (size_t)mir(zz, m) * plane;
        for (int idx = threadIdx.x; idx < PX * PY; idx += kThreads) {
            const int ly = idx / PX, lx = idx % PX;
            const size_t q = zoff + (size_t)mir(y0 - 1 + ly, m) * m + mir(x0 - 1 + lx, m);
            su[slot][ly][lx] = ein[q];
            if (SIG) ss[slot][ly][lx] = sig[q];
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
        cc[at] = su[slot][ty + 1][tx + 1];
        cx[at] = (su[slot][ty + 1][tx] + su[slot][ty + 1][tx + 2]) + (su[slot][ty][tx + 1] + su[slot][ty + 2][tx + 1]);
        if (RAD)
            ck[at] = (su[slot][ty][tx] + su[slot][ty][tx + 2]) + (su[slot][ty + 2][tx] + su[slot][ty + 2][tx + 2]);
    };
    stage(0, z0 - 1);
    stage(1, z0);
    if (!SIG) {
        __syncthreads();
        plane_sums(0, 1);  // at = 1: plane z-1 of the first node, shifted in below
        plane_sums(1, 2);
    }
    for (int z = z0; z < z1; ++z) {
        const int k = z - z0;
        const int sm = k % 3, sc = (k + 1) % 3, sp = (k + 2) % 3;  // planes z-1, z, z+1
        stage(sp, z + 1);
        __syncthreads();
        if (!SIG) {
            cc[0] = cc[1], cc[1] = cc[2];
            cx[0] = cx[1], cx[1] = cx[2];
            ck[0] = ck[1], ck[1] = ck[2];
            plane_sums(sp, 2);  // cc/cx/ck[0..2]: planes z-1, z, z+1
        }
        if (own) {
            const size_t c = (size_t)z * plane + (size_t)y * m + x;
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
                const T r = scale * (sum - Wc * uc) + a * uc - g[c];
                eout[c] = uc + tD * r;
                if (pres) {
                    const unsigned long long b = dbits((double)r);
                    rb = b > rb ? b : rb;
                }
            } else {
                const int slots[3] = {sm, sc, sp};
                const T uc = su[sc][ty + 1][tx + 1];
                const T sgc = ss[sc][ty + 1][tx + 1];
                T acc[3] = {T(0), T(0), T(0)}, ds[3] = {T(0), T(0), T(0)};
#pragma unroll
                for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int cls = (dx != 0) + (dy != 0) + (dz != 0);
                            if (cls == 0 || (!RAD && cls != 1)) continue;
                            const int s = slots[dz + 1];
                            const T du = su[s][ty + 1 + dy][tx + 1 + dx] - uc;
                            const T t = ss[s][ty + 1 + dy][tx + 1 + dx] + sgc;
                            acc[cls - 1] += t * du;
                            ds[cls - 1] += t;
                        }
                    }
                }
                const T third = T(1.0 / 3.0);
                const T sw = acc[0] + T(0.5) * acc[1] + third * acc[2];
                const T Lu = scale * T(0.5) * sw + a * uc;
                const T D = scale * T(0.5) * (ds[0] + T(0.5) * ds[1] + third * ds[2]) - a;
                const T r = Lu - g[c];
                eout[c] = uc + step_of3(theta, D) * r;
                if (pres) {
                    const unsigned long long b = dbits((double)r);
                    rb = b > rb ? b : rb;
                }
            }
        }
        __syncthreads();  // the next iteration overwrites plane z-1's slot
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

// End of a cycle on a 3D level 0 (recurrence of Sec. 2, FP64), marching in
// z like k_sweep3d: e = escale * E with Dirichlet values replaced by G (first
// cycle) or 0 is staged per plane in LDS, then u += e, s -= dL_1 e at
// unknowns (s = 0 at Dirichlet nodes), shat = s * shat_scale, max |s|.
template <typename T, int RAD, int SIG>
__global__ __launch_bounds__(kThreads) void k_cycle_end3d(CycleEndArgs A)
{
    __shared__ double se[3][PY][PX];
    __shared__ double ss[SIG ? 3 : 1][SIG ? PY : 1][SIG ? PX : 1];
    const Level L = A.L;
    const int m = L.m;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * ZC;
    const int z1 = min(m, z0 + ZC);
    const int x = x0 + tx, y = y0 + ty;
    const bool own = x < m && y < m;
    const size_t plane = (size_t)m * m;
    const T *__restrict__ E = (const T *)A.e;
    const double *__restrict__ G = A.G;
    const double *__restrict__ sig = A.sigma;
    T *__restrict__ shat = (T *)A.shat;

    auto stage = [&](int slot, int zz) {
        const int zm = mir(zz, m);
        const size_t zoff = (size_t)zm * plane;
        for (int idx = threadIdx.x; idx < PX * PY; idx += kThreads) {
            const int ly = idx / PX, lx = idx % PX;
            const int ym = mir(y0 - 1 + ly, m), xm = mir(x0 - 1 + lx, m);
            const size_t q = zoff + (size_t)ym * m + xm;
            double v = A.escale * (double)E[q];
            if (is_dir<3>(xm, ym, zm, m, L.dir)) v = G ? G[q] : 0.0;
            se[slot][ly][lx] = v;
            if (SIG) ss[slot][ly][lx] = sig[q];
        }
    };
    unsigned long long nb = 0;
    stage(0, z0 - 1);
    stage(1, z0);
    for (int z = z0; z < z1; ++z) {
        const int k = z - z0;
        const int sm = k % 3, sc = (k + 1) % 3, sp = (k + 2) % 3;
        stage(sp, z + 1);
        __syncthreads();
        if (own) {
            const size_t c = (size_t)z * plane + (size_t)y * m + x;
            const double ec = se[sc][ty + 1][tx + 1];
            A.u[c] += ec;
            if (is_dir<3>(x, y, z, m, L.dir)) {
                A.s[c] = 0.0;
                if (shat) shat[c] = T(0);
            } else {
                const int slots[3] = {sm, sc, sp};
                const double sgc = SIG ? ss[sc][ty + 1][tx + 1] : 1.0;
                double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int cls = (dx != 0) + (dy != 0) + (dz != 0);
                            if (cls == 0 || (!RAD && cls != 1)) continue;
                            const int sl = slots[dz + 1];
                            const double du = se[sl][ty + 1 + dy][tx + 1 + dx] - ec;
                            if (SIG)
                                acc[cls - 1] += (ss[sl][ty + 1 + dy][tx + 1 + dx] + sgc) * du;
                            else
                                acc[cls - 1] += du;
                        }
                    }
                }
                const double sw = acc[0] + 0.5 * acc[1] + (1.0 / 3.0) * acc[2];
                const double Le = (SIG ? 0.5 * L.scale * sw : L.scale * sw) + L.a * ec;
                const double sn = A.s[c] - Le;
                A.s[c] = sn;
                if (shat) shat[c] = (T)(sn * A.shat_scale);
                const unsigned long long b = dbits(sn);
                nb = b > nb ? b : nb;
            }
        }
        __syncthreads();
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

}  // namespace

bool sweep3d_supported(int m) { return m >= 33; }

template <typename T>
void launch_cycle_end3d(const Variant &v, const CycleEndArgs &a, hipStream_t st)
{
    const int m = a.L.m;
    const dim3 grid((m + TX - 1) / TX, (m + TY - 1) / TY, (m + ZC - 1) / ZC), block(kThreads);
    if (v.radial && v.sigma)
        hipLaunchKernelGGL((k_cycle_end3d<T, 1, 1>), grid, block, 0, st, a);
    else if (v.radial)
        hipLaunchKernelGGL((k_cycle_end3d<T, 1, 0>), grid, block, 0, st, a);
    else if (v.sigma)
        hipLaunchKernelGGL((k_cycle_end3d<T, 0, 1>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((k_cycle_end3d<T, 0, 0>), grid, block, 0, st, a);
}

template void launch_cycle_end3d<double>(const Variant &, const CycleEndArgs &, hipStream_t);
template void launch_cycle_end3d<float>(const Variant &, const CycleEndArgs &, hipStream_t);

template <typename T>
void launch_sweep3d(const Variant &v, const Level &L, const T *ein, T *eout, const T *g, const T *sig,
                    const double *G, unsigned long long *pres, hipStream_t st)
{
    const int m = L.m;
    const dim3 grid((m + TX - 1) / TX, (m + TY - 1) / TY, (m + ZC - 1) / ZC), block(kThreads);
    if (v.radial && v.sigma)
        hipLaunchKernelGGL((k_sweep3d<T, 1, 1>), grid, block, 0, st, ein, eout, g, sig, G, L, pres);
    else if (v.radial)
        hipLaunchKernelGGL((k_sweep3d<T, 1, 0>), grid, block, 0, st, ein, eout, g, sig, G, L, pres);
    else if (v.sigma)
        hipLaunchKernelGGL((k_sweep3d<T, 0, 1>), grid, block, 0, st, ein, eout, g, sig, G, L, pres);
    else
        hipLaunchKernelGGL((k_sweep3d<T, 0, 0>), grid, block, 0, st, ein, eout, g, sig, G, L, pres);
}

template void launch_sweep3d<double>(const Variant &, const Level &, const double *, double *, const double *,
                                     const double *, const double *, unsigned long long *, hipStream_t);
template void launch_sweep3d<float>(const Variant &, const Level &, const float *, float *, const float *,
                                    const float *, const double *, unsigned long long *, hipStream_t);

}  // namespace sgml
