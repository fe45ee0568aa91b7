// sgml_visit2d_impl.h -- one visit of a 2D level in one pass over memory
// (included by sgml_visit2d_f32.hip and sgml_visit2d_f64.hip, which
// instantiate it for one precision each).
//
// A visit of Algorithm 3 at level nu is: interpolate the pending variation of
// level nu+1 (when the schedule refines), run c relaxations (Algorithm 2,
// Jacobi), and copy the result to level nu+1's nodes (when the schedule
// climbs).  Run one launch per step and each relaxation streams the level
// through HBM again.  Here every wavefront owns a strip of 128 columns, two
// per lane, and marches down the rows of a chunk; each relaxation is a
// pipeline stage that keeps a three-row window of its input in registers, so
// relaxation s+1 consumes relaxation s's rows as they are produced.
// Horizontal neighbours come from the lane's other column or the adjacent
// lane (cross-lane moves), vertical ones from the window.  The strip and the chunk carry a halo as wide as the number of
// relaxations (plus one column for the interpolation), recomputed by the
// neighbouring wavefronts; only the interior is written.  Values outside the
// grid are images (node reflection), so Neumann faces need no special case,
// and a Dirichlet node takes its prescribed value at every relaxation.
// Wavefronts are independent: no LDS, no barriers.
#pragma once

#include "sgml_device.h"

#include <type_traits>
#include <utility>

namespace sgml {

namespace {

constexpr int kVisitBlock = 256;  // four independent wavefronts

// f(std::integral_constant<int, 0>()) .. f(std::integral_constant<int, N - 1>()):
// a loop whose index is a compile-time constant in the body.
template <typename F, int... I>
__device__ __forceinline__ void unroll_seq(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>()), ...);
}
template <int N, typename F>
__device__ __forceinline__ void unroll(F &&f)
{
    unroll_seq(f, std::make_integer_sequence<int, N>());
}

// Element idx of a level array through a 32-bit byte offset (2D levels are
// below 4 GiB): a scalar base plus one per-lane register, no 64-bit address
// arithmetic per lane.
template <typename T>
__device__ __forceinline__ T ld(const T *base, unsigned idx)
{
    return *(const T *)((const char *)base + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st(T *base, unsigned idx, T v)
{
    *(T *)((char *)base + idx * (unsigned)sizeof(T)) = v;
}

// Whole-wavefront shifts by one lane (DPP wave_shr:1 / wave_shl:1): lane i
// receives lane i-1's (from_left) or lane i+1's (from_right) value; the end
// lanes, which have no source, receive 0 (they are halo lanes).  A few
// cycles, no LDS crossbar.
__device__ __forceinline__ int dpp_from_left(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_from_right(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }

__device__ __forceinline__ float from_left(float v) { return __int_as_float(dpp_from_left(__float_as_int(v))); }
__device__ __forceinline__ float from_right(float v) { return __int_as_float(dpp_from_right(__float_as_int(v))); }
__device__ __forceinline__ double from_left(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_from_left((int)(b & 0xffffffff)), hi = dpp_from_left((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double from_right(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_from_right((int)(b & 0xffffffff)), hi = dpp_from_right((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// A copy the compiler cannot fold into the source register (its value in a
// new register).
__device__ __forceinline__ float fresh(float v)
{
    float r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}
__device__ __forceinline__ double fresh(double v)
{
    double r;
    asm("v_mov_b64 %0, %1" : "=v"(r) : "v"(v));
    return r;
}
// The same copy into a register other than the source's (an early-clobber
// output): a value computed in place in a loaded register (v_fmac on it)
// moves out of it, which frees that register for the next batch's load.
__device__ __forceinline__ float fresh_apart(float v)
{
    float r;
    asm("v_mov_b32 %0, %1" : "=&v"(r) : "v"(v));
    return r;
}
__device__ __forceinline__ double fresh_apart(double v)
{
    double r;
    asm("v_mov_b64 %0, %1" : "=&v"(r) : "v"(v));
    return r;
}

// theta / D with D the local diagonal: FP32 uses the hardware reciprocal
// (the relaxation is the approximate inner solver of the mixed mode), FP64
// divides.
__device__ __forceinline__ float step_of(float theta, float D) { return theta * __builtin_amdgcn_rcpf(D); }
__device__ __forceinline__ double step_of(double theta, double D) { return theta / D; }

// Constants of one relaxation with a constant coefficient: the update
// e + theta/D (dL e - g) with dL e = scale (sum of neighbours - W e) + a e and
// D = W scale - a is the damped-Jacobi form
//   e' = (1 - theta) e + beta * (sum of neighbours) - gamma * g,
// beta = theta scale / D, gamma = theta / D (W = 4 axis, 6 radial: corners
// weigh 1/2).  The residual dL e - g is formed only when it is recorded.
template <typename T>
struct RelaxK {
    T scale, a, theta, omt, beta, gamma, aw;  // aw = a - W scale
};

// Lane l of a strip holds the column pair (x, x + 1), x even.  The left neighbour of x and the right
// neighbour of x + 1 come from the adjacent lanes (one cross-lane move each
// per row and relaxation, for two nodes); the row and pipeline bookkeeping,
// which is per row and per wavefront, serves twice the nodes; a strip is 128
// columns wide with an even halo, so 128 - 2 * HX of them are written.

template <typename T>
struct RowIn2 {
    T sta, stb, ga, gb, sga, sgb, c0, c1, s0, s1;
};

// Loads of input row rho (mirrored into the grid; a mirrored row keeps the
// parity of rho).  The row's parity is a template argument (chunks start at
// even rows, so it follows from the row's place in the march): every row of
// one parity issues the same loads in the same order, with no branch, and
// the compiler waits for each load by count at its use while the next batch
// of rows stays in flight.  Odd rows also load the second coarse row and
// the stale values at the coarse nodes above and below.  FIRST: the stale
// values are zero and are not read.
template <typename T, int PRO, int SIG, bool FIRST, bool ODD>
__device__ __forceinline__ void load_row2(RowIn2<T> &R, const VisitArgs &A, int xma, int xmb, int rho, int m)
{
    const unsigned rm = (unsigned)mir(rho, m), um = (unsigned)m;
    const unsigned row = rm * um;
    const T *__restrict__ estale = (const T *)A.estale;
    const T *__restrict__ g = (const T *)A.g;
    if (PRO && FIRST) {
        R.sta = R.stb = T(0);
    } else {
        R.sta = ld(estale, row + (unsigned)xma);
        R.stb = ld(estale, row + (unsigned)xmb);
    }
    R.ga = ld(g, row + (unsigned)xma);
    R.gb = ld(g, row + (unsigned)xmb);
    if (SIG) {
        const T *__restrict__ sig = (const T *)A.sig;
        R.sga = ld(sig, row + (unsigned)xma);
        R.sgb = ld(sig, row + (unsigned)xmb);
    }
    if (PRO) {
        // coarse node X = xma / 2 (xma is even), rows Y = rm / 2 and, odd
        // rows, Y + 1 (<= mc - 1), with fine rows 2Y and 2Y + 2 (<= m - 1)
        const T *__restrict__ ec = (const T *)A.ecoarse;
        const unsigned mc = (um + 1) >> 1, Y = rm >> 1, X = (unsigned)xma >> 1;
        R.c0 = ld(ec, Y * mc + X);
        if (ODD) {
            R.c1 = ld(ec, (Y + 1) * mc + X);
            if (FIRST) {
                R.s0 = R.s1 = T(0);
            } else {
                R.s0 = ld(estale, 2 * Y * um + (unsigned)xma);
                R.s1 = ld(estale, (2 * Y + 2) * um + (unsigned)xma);
            }
        }
    }
}

// The level's values at (rm, x) and (rm, x + 1) with the pending variation
// of the next coarser level interpolated: coarse nodes take the coarse
// value, the others add the tensor-hat mean of the pending variation (coarse
// value minus stale finer value) of the enclosing coarse nodes.  x is a coarse
// column, x + 1 lies between coarse columns x / 2 and x / 2 + 1, the latter
// held by the next lane.  All lanes must call it.
template <typename T, bool ODD>
__device__ __forceinline__ void prolonged2(const RowIn2<T> &R, T &va, T &vb)
{
    if (!ODD) {
        const T p = R.c0 - R.sta;
        const T pr = from_right(p);
        va = R.c0;
        vb = R.stb + T(0.5) * (p + pr);
    } else {
        const T p0 = R.c0 - R.s0, p1 = R.c1 - R.s1;
        const T p0r = from_right(p0), p1r = from_right(p1);
        va = R.sta + T(0.5) * (p0 + p1);
        vb = R.stb + T(0.5) * (T(0.5) * (p0 + p0r) + T(0.5) * (p1 + p1r));
    }
}

// One relaxation of the column pair in the middle row of the windows wa, wb
// (rows r-1, r, r+1); sa, sb: the coefficient there.  All lanes must call it.
template <typename T, int RAD, int SIG, int REC>
__device__ __forceinline__ void relax2(const T (&wa)[3], const T (&wb)[3], const T (&sa)[3], const T (&sb)[3], T ga,
                                       T gb, bool da, bool db, T gva, T gvb, const RelaxK<T> &K, T &na, T &nb,
                                       T &resa, T &resb)
{
    const T ca = wa[1], cb = wb[1];
    const T la = from_left(cb), rb = from_right(ca);  // left of x, right of x + 1
    T ula = T(0), dla = T(0), urb = T(0), drb = T(0);  // corners across the lane boundary (radial)
    if (RAD) {
        ula = from_left(wb[0]);
        dla = from_left(wb[2]);
        urb = from_right(wa[0]);
        drb = from_right(wa[2]);
    }
    if (SIG) {
        const T sca = sa[1], scb = sb[1];
        // column x: left (la), right (cb), up, down
        const T tla = from_left(scb) + sca, tra = scb + sca, tna = sa[0] + sca, tsa = sa[2] + sca;
        T acca = tla * (la - ca) + tra * (cb - ca) + tna * (wa[0] - ca) + tsa * (wa[2] - ca);
        T dsa = tla + tra + tna + tsa;
        // column x + 1: left (ca), right (rb), up, down
        const T tlb = sca + scb, trb = from_right(sca) + scb, tnb = sb[0] + scb, tsb = sb[2] + scb;
        T accb = tlb * (ca - cb) + trb * (rb - cb) + tnb * (wb[0] - cb) + tsb * (wb[2] - cb);
        T dsb = tlb + trb + tnb + tsb;
        if (RAD) {
            const T tnla = from_left(sb[0]) + sca, tnra = sb[0] + sca;
            const T tsla = from_left(sb[2]) + sca, tsra = sb[2] + sca;
            acca += T(0.5) * (tnla * (ula - ca) + tnra * (wb[0] - ca) + tsla * (dla - ca) + tsra * (wb[2] - ca));
            dsa += T(0.5) * (tnla + tnra + tsla + tsra);
            const T tnlb = sa[0] + scb, tnrb = from_right(sa[0]) + scb;
            const T tslb = sa[2] + scb, tsrb = from_right(sa[2]) + scb;
            accb += T(0.5) * (tnlb * (wa[0] - cb) + tnrb * (urb - cb) + tslb * (wa[2] - cb) + tsrb * (drb - cb));
            dsb += T(0.5) * (tnlb + tnrb + tslb + tsrb);
        }
        const T ra = K.scale * T(0.5) * acca + K.a * ca - ga;
        const T rbr = K.scale * T(0.5) * accb + K.a * cb - gb;
        if (REC) {
            resa = da ? T(0) : ra;
            resb = db ? T(0) : rbr;
        }
        na = da ? gva : ca + step_of(K.theta, K.scale * T(0.5) * dsa - K.a) * ra;
        nb = db ? gvb : cb + step_of(K.theta, K.scale * T(0.5) * dsb - K.a) * rbr;
        return;
    }
    T suma = (la + cb) + (wa[0] + wa[2]);
    T sumb = (ca + rb) + (wb[0] + wb[2]);
    if (RAD) {
        suma += T(0.5) * ((ula + wb[0]) + (dla + wb[2]));
        sumb += T(0.5) * ((wa[0] + urb) + (wa[2] + drb));
    }
    if (REC) {
        resa = da ? T(0) : K.scale * suma + K.aw * ca - ga;
        resb = db ? T(0) : K.scale * sumb + K.aw * cb - gb;
    }
    // without recording, ga and gb arrive as gamma * g
    const T gga = REC ? K.gamma * ga : ga, ggb = REC ? K.gamma * gb : gb;
    na = da ? gva : K.omt * ca + (K.beta * suma - gga);
    nb = db ? gvb : K.omt * cb + (K.beta * sumb - ggb);
}

// The relaxation of relax2 with a constant coefficient, no recording and no
// Dirichlet row in the window: the damped-Jacobi form with the source
// already scaled (gga = gamma * g) and per-lane constants, which a Dirichlet
// column sets to omt = 1, beta = 0 and a zero source, so that it keeps its
// value (zero after the first cycle) without a select per relaxation.
template <typename T, int RAD>
__device__ __forceinline__ void relax2_fast(const T (&wa)[3], const T (&wb)[3], T gga, T ggb, T oma, T omb, T bea,
                                            T beb, T &na, T &nb)
{
    const T ca = wa[1], cb = wb[1];
    const T la = from_left(cb), rb = from_right(ca);
    T suma = (la + cb) + (wa[0] + wa[2]);
    T sumb = (ca + rb) + (wb[0] + wb[2]);
    if (RAD) {
        const T ula = from_left(wb[0]), dla = from_left(wb[2]);
        const T urb = from_right(wa[0]), drb = from_right(wa[2]);
        suma += T(0.5) * ((ula + wb[0]) + (dla + wb[2]));
        sumb += T(0.5) * ((wa[0] + urb) + (wa[2] + drb));
    }
    na = oma * ca + (bea * suma - gga);
    nb = omb * cb + (beb * sumb - ggb);
}

template <typename T, int RAD, int SIG, int S, int PRO, int REC>
__global__ __launch_bounds__(kVisitBlock) void k_visit2d(VisitArgs A)
{
    constexpr int HX = (S + PRO + 1) / 2 * 2;  // halo columns on each side, even
    constexpr int W = 128 - 2 * HX;            // columns a wavefront writes
    const Level L = A.L;
    const int m = L.m;
    const int lane = threadIdx.x & 63;
    const int strips = (m + W - 1) / W;
    const int wid = blockIdx.x * (kVisitBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sx = wid % strips, sy = wid / strips;
    const int y0 = sy * A.chunk;
    if (y0 >= m) return;  // the whole wavefront: past the last chunk
    const int y1 = min(m, y0 + A.chunk);
    const int xa = sx * W - HX + 2 * lane;  // even
    const int xma = mir(xa, m), xmb = mir(xa + 1, m);
    const bool lane_out = lane >= HX / 2 && lane < (HX + W) / 2;
    const bool outa = lane_out && xa < m, outb = lane_out && xa + 1 < m;

    T *__restrict__ eout = (T *)A.eout;
    T *__restrict__ einj = (T *)A.einj;
    RelaxK<T> K;
    K.scale = (T)L.scale;
    K.a = (T)L.a;
    K.theta = (T)L.theta;
    {
        const double Wd = RAD ? 6.0 : 4.0, D = Wd * L.scale - L.a;
        K.omt = (T)(1.0 - L.theta);
        K.beta = (T)(L.theta * L.scale / D);
        K.gamma = (T)(L.theta / D);
        K.aw = (T)(L.a - Wd * L.scale);
    }
    const bool inject = A.inject != 0;
    const bool xda = ((L.dir & 1u) && xma == 0) || ((L.dir & 2u) && xma == m - 1);
    const bool xdb = ((L.dir & 1u) && xmb == 0) || ((L.dir & 2u) && xmb == m - 1);
    const double *__restrict__ G = A.G;
    const int gpitch = L.lam * L.N;
    // constants of the fast relaxation (Dirichlet columns keep their value)
    const T oma = xda ? T(1) : K.omt, omb = xdb ? T(1) : K.omt;
    const T bea = xda ? T(0) : K.beta, beb = xdb ? T(0) : K.beta;
    const T gama = xda ? T(0) : K.gamma, gamb = xdb ? T(0) : K.gamma;

    T wa[S][3], wb[S][3];
    T gha[S + 1], ghb[S + 1];  // source at input row - k
    T sha[S + 2], shb[S + 2];  // coefficient at input row - k
    unsigned long long pr[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        wa[s][0] = wa[s][1] = wa[s][2] = wb[s][0] = wb[s][1] = wb[s][2] = T(0);
        pr[s] = 0;
    }
#pragma unroll
    for (int k = 0; k < S + 1; ++k) gha[k] = ghb[k] = T(0);
#pragma unroll
    for (int k = 0; k < S + 2; ++k) sha[k] = shb[k] = T(1);

    const int rows = (y1 - y0) + 2 * S;
    unsigned ymask = 0;  // bit k: input row - k lies on a Dirichlet y face
    auto step_row = [&](const RowIn2<T> &R, int t, auto hasg, auto odd, auto fast) __attribute__((always_inline)) {
        constexpr bool HASG = decltype(hasg)::value;
        constexpr bool FAST = decltype(fast)::value;
        const int rho = y0 - S + t;
        const int rm = mir(rho, m);
        T va, vb;
        if (PRO) {
            prolonged2<T, decltype(odd)::value>(R, va, vb);
        } else {
            va = R.sta;
            vb = R.stb;
        }
        // window values, moved out of the loaded registers (computed in place
        // there or copies), which the next batch's loads then reuse
        va = fresh_apart(va);
        vb = fresh_apart(vb);
#pragma unroll
        for (int k = S; k > 0; --k) {
            gha[k] = gha[k - 1];
            ghb[k] = ghb[k - 1];
        }
        // the source enters its delay line as gamma * g where the relaxation
        // uses that product alone, else as a copy: either way the loaded
        // register is free once its row is consumed, so the next batch's load
        // reuses it (no copy of a load in flight at the end of a turn)
        if (FAST) {
            gha[0] = gama * R.ga;
            ghb[0] = gamb * R.gb;
        } else if (!SIG && !REC) {
            gha[0] = K.gamma * R.ga;
            ghb[0] = K.gamma * R.gb;
        } else {
            gha[0] = fresh(R.ga);
            ghb[0] = fresh(R.gb);
        }
        if (!FAST) ymask = (ymask << 1) | (unsigned)(((L.dir & 4u) && rm == 0) || ((L.dir & 8u) && rm == m - 1));
        if (SIG) {
#pragma unroll
            for (int k = S + 1; k > 0; --k) {
                sha[k] = sha[k - 1];
                shb[k] = shb[k - 1];
            }
            sha[0] = fresh(R.sga);
            shb[0] = fresh(R.sgb);
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            wa[s][0] = wa[s][1];
            wa[s][1] = wa[s][2];
            wa[s][2] = va;
            wb[s][0] = wb[s][1];
            wb[s][1] = wb[s][2];
            wb[s][2] = vb;
            if (FAST) {
                relax2_fast<T, RAD>(wa[s], wb[s], gha[s + 1], ghb[s + 1], oma, omb, bea, beb, va, vb);
                continue;
            }
            const int r = rho - s - 1;  // row relaxation s+1 produces now
            const bool yd = (ymask >> (s + 1)) & 1u;
            const bool da = xda || yd, db = xdb || yd;
            T gva = T(0), gvb = T(0);
            if (HASG) {
                const unsigned grow = (unsigned)mir(r, m) * (unsigned)gpitch;
                if (da) gva = (T)ld(G, grow + (unsigned)(xma * L.lam));
                if (db) gvb = (T)ld(G, grow + (unsigned)(xmb * L.lam));
            }
            const T sga[3] = {sha[s + 2], sha[s + 1], sha[s]};
            const T sgb[3] = {shb[s + 2], shb[s + 1], shb[s]};
            T resa = T(0), resb = T(0);
            relax2<T, RAD, SIG, REC>(wa[s], wb[s], sga, sgb, gha[s + 1], ghb[s + 1], da, db, gva, gvb, K, va, vb,
                                     resa, resb);
            if (REC && A.pres[s] >= 0 && r >= y0 && r < y1) {
                unsigned long long b = 0;
                if (outa) b = dbits((double)resa);
                if (outb) {
                    const unsigned long long bb = dbits((double)resb);
                    b = bb > b ? bb : b;
                }
                pr[s] = b > pr[s] ? b : pr[s];
            }
        }
        const int ro = rho - S;
        if (ro >= y0 && ro < y1) {
            const unsigned q = (unsigned)ro * (unsigned)m + (unsigned)xa;
            if (outa) {
                st(eout, q, va);
                if (inject && !(ro & 1))
                    st(einj, (unsigned)(ro >> 1) * (unsigned)((m + 1) >> 1) + (unsigned)(xa >> 1), va);
            }
            if (outb) st(eout, q + 1u, vb);
        }
    };
    constexpr int B = 3;
    RowIn2<T> qa[B], qb[B];
    // Row t of the march has the parity of S + t (chunks start at even
    // rows); a turn is 2B = 6 rows, so position K of a turn has the parity
    // of S + K.  Rows past the last one load the last row of the same parity
    // again (the batch ahead of the tail), so that every batch issues the
    // same loads.
    auto load_batch = [&](RowIn2<T>(&q)[B], int t0, auto first, auto k0) __attribute__((always_inline)) {
        constexpr bool FIRST = decltype(first)::value;
        constexpr int K0 = decltype(k0)::value;
        unroll<B>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            int t = t0 + k;
            if (t > rows - 1) t -= 2 * ((t - rows + 2) >> 1);
            load_row2<T, PRO, SIG, FIRST, ((S + K0 + k) & 1) != 0>(q[k], A, xma, xmb, y0 - S + t, m);
        });
    };
    using K0a = std::integral_constant<int, 0>;
    using K0b = std::integral_constant<int, B>;
    auto step_batch = [&](const RowIn2<T>(&q)[B], int t0, auto hasg, auto fast, auto k0, bool guard) __attribute__((always_inline)) {
        constexpr int K0 = decltype(k0)::value;
        unroll<B>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            if (!guard || t0 + k < rows)
                step_row(q[k], t0 + k, hasg, std::integral_constant<bool, ((S + K0 + k) & 1) != 0>(), fast);
        });
    };
    // two batches of B rows per turn, B a multiple of the window period
    // (three rows), so that the windows rotate by renaming; the rows past
    // the last full turn take the guarded tail
    auto march = [&](auto hasg, auto first, auto fast) __attribute__((always_inline)) {
        load_batch(qa, 0, first, K0a());
        int t0 = 0;
        // turns with rows after them (their refill of qa loads real rows)
        for (; t0 + 2 * B < rows; t0 += 2 * B) {
            load_batch(qb, t0 + B, first, K0b());
            step_batch(qa, t0, hasg, fast, K0a(), false);
            load_batch(qa, t0 + 2 * B, first, K0a());
            step_batch(qb, t0 + B, hasg, fast, K0b(), false);
        }
        // the last turn: rows t0 .. rows - 1; in the short visits (8-row
        // chunks, two turns) a full turn, without guards
        if (S <= 2 && rows - t0 == 2 * B) {
            load_batch(qb, t0 + B, first, K0b());
            step_batch(qa, t0, hasg, fast, K0a(), false);
            step_batch(qb, t0 + B, hasg, fast, K0b(), false);
        } else {
            if (t0 + B < rows) load_batch(qb, t0 + B, first, K0b());
            step_batch(qa, t0, hasg, fast, K0a(), true);
            step_batch(qb, t0 + B, hasg, fast, K0b(), true);
        }
    };
    using yes = std::true_type;
    using no = std::false_type;
    const bool first_visit = PRO && A.first;
    // the fast relaxation: later cycles (Dirichlet values zero), constant
    // coefficient, no recording, and no Dirichlet row among the rows the
    // chunk reads (y0 - S .. y1 + S - 1)
    const bool ydir_rows = ((L.dir & 4u) && y0 <= S) || ((L.dir & 8u) && y1 + S >= m);
    if (G) {
        if (first_visit) march(yes(), yes(), no());
        else march(yes(), no(), no());
    } else if (SIG || REC || ydir_rows) {
        if (first_visit) march(no(), yes(), no());
        else march(no(), no(), no());
    } else {
        if constexpr (!SIG && !REC) {
            if (first_visit) march(no(), yes(), yes());
            else march(no(), no(), yes());
        }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        if (!REC || A.pres[s] < 0) continue;
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

// End of a cycle on a 2D level 0 (the recurrence of Sec. 2, FP64): u += e,
// s -= dL_1 e at unknowns (s = 0 at Dirichlet nodes), next cycle's source
// shat = s * shat_scale, and max |s|.  e is escale * E with E's Dirichlet
// values replaced by G (first cycle) or 0.  Same strip/row marching as the
// visit: e is read once per node, its vertical neighbours come from a
// three-row window and the horizontal ones from the adjacent lanes.
//
// RES: the pass also writes the next cycle's level-1 source, the first step
// of the restriction pyramid (Algorithm 1, eq. (3)) of the new source (shat,
// or s itself in FP64).  Level-1 node (I, J) averages the source at fine
// rows 2J-1 .. 2J+1 and columns 2I-1 .. 2I+1 (images outside the grid).
// For that a wavefront computes the source one column beyond its strip on
// each side (halo of two) and one row above its chunk (chunks start at even
// rows), keeps the last three rows per lane, and on each odd row r
// completes level-1 row (r-1)/2: vertical weights (1/2, 1, 1/2) in the
// lane, horizontal ones across lanes, over 4.  It writes the level-1 nodes
// whose centre it owns.  The halo nodes belong to other wavefronts, which
// write their new residual meanwhile: with RES the new residual goes to
// s_out, a second buffer, and s is only read.
template <typename T, int RAD, int SIG, int RES>
__global__ __launch_bounds__(kVisitBlock) void k_cycle_end2d(CycleEndArgs A)
{
    constexpr int HX = RES ? 2 : 1;
    constexpr int W = 64 - 2 * HX;
    const Level L = A.L;
    const int m = L.m;
    const int lane = threadIdx.x & 63;
    const int strips = (m + W - 1) / W;
    // wavefront index, known to be uniform: row and strip arithmetic stays scalar
    const int wid = blockIdx.x * (kVisitBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sx = wid % strips, sy = wid / strips;
    const int y0 = sy * A.chunk;
    if (y0 >= m) return;
    const int y1 = min(m, y0 + A.chunk);
    const int x = sx * W - HX + lane;
    const int xm = mir(x, m);
    const bool xout = lane >= HX && lane < HX + W && x < m;
    const bool xdir = ((L.dir & 1u) && xm == 0) || ((L.dir & 2u) && xm == m - 1);
    const T *__restrict__ E = (const T *)A.e;
    const double *__restrict__ G = A.G;
    const double *__restrict__ sig = A.sigma;
    double *__restrict__ u = A.u;
    const double *__restrict__ sres = A.s;
    double *__restrict__ sout = RES ? A.s_out : A.s;
    T *__restrict__ shat = (T *)A.shat;
    T *__restrict__ g1 = (T *)A.g1;
    const int m1 = (m + 1) / 2;
    const double scale = L.scale, a = L.a, escale = A.escale;
    // first output row: one above the chunk when restricting (for the
    // level-1 row centred on the chunk's first row)
    const int r_first = RES ? max(y0 - 1, 0) : y0;
    const int rows = (y1 - y0) + 2 + RES;
    double w[3] = {0.0, 0.0, 0.0}, sw[3] = {1.0, 1.0, 1.0};
    T hs[3] = {T(0), T(0), T(0)};  // source at output rows r-2, r-1, r (RES)
    unsigned long long nb = 0;
    // raw loads of input row rho (e, coefficient) and of output row rho - 1
    // (s, u).  Every lane and row issues the same loads, from the mirrored
    // column and a row clamped into the grid, so that the compiler waits for
    // each by count at its use and the next batch stays in flight; values
    // outside the lanes and rows that use them are ignored.  u is read from
    // the nearest column and row it is written at, s (read also beside the
    // strip and above the chunk when restricting) from the nearest row it is
    // used at: the ignored values are cache hits, not fetched from memory.
    struct Raw {
        T e;
        double sg, s, u;
    };
    const unsigned xum = (unsigned)min(max(x, sx * W), min(sx * W + W, m) - 1);
    const unsigned xsm = RES ? (unsigned)xm : xum;
    auto load = [&](Raw &R, int t) {
        const int rho = y0 - 1 - RES + t;
        const unsigned rm = (unsigned)mir(rho, m), um = (unsigned)m;
        R.e = ld(E, rm * um + (unsigned)xm);
        if (SIG) R.sg = ld(sig, rm * um + (unsigned)xm);
        const unsigned rs = (unsigned)min(max(rho - 1, r_first), y1 - 1);
        const unsigned ru = (unsigned)min(max(rho - 1, y0), y1 - 1);
        R.s = ld(sres, rs * um + xsm);
        R.u = ld((const double *)u, ru * um + xum);
    };
    auto step_row = [&](const Raw &R, int t, auto hasg) {
        constexpr bool HASG = decltype(hasg)::value;
        const int rho = y0 - 1 - RES + t, rm = mir(rho, m);
        const bool ydir_in = ((L.dir & 4u) && rm == 0) || ((L.dir & 8u) && rm == m - 1);
        double ev = escale * (double)R.e;
        if (xdir || ydir_in) ev = HASG ? ld(G, (unsigned)rm * (unsigned)m + (unsigned)xm) : 0.0;  // Dirichlet values
        w[0] = w[1];
        w[1] = w[2];
        w[2] = ev;
        if (SIG) {
            sw[0] = sw[1];
            sw[1] = sw[2];
            sw[2] = R.sg;
        }
        const int r = rho - 1;
        // dL_1 e at row r (all lanes: cross-lane moves)
        const double c = w[1];
        const double ul = from_left(c), ur = from_right(c);
        double Le;
        if (SIG) {
            const double sc = sw[1];
            const double tl = from_left(sc) + sc, tr = from_right(sc) + sc, tn = sw[0] + sc, ts = sw[2] + sc;
            double acc = tl * (ul - c) + tr * (ur - c) + tn * (w[0] - c) + ts * (w[2] - c);
            if (RAD) {
                const double nl = from_left(w[0]), nr = from_right(w[0]), sl = from_left(w[2]),
                             sr = from_right(w[2]);
                const double tnl = from_left(sw[0]) + sc, tnr = from_right(sw[0]) + sc;
                const double tsl = from_left(sw[2]) + sc, tsr = from_right(sw[2]) + sc;
                acc += 0.5 * (tnl * (nl - c) + tnr * (nr - c) + tsl * (sl - c) + tsr * (sr - c));
            }
            Le = 0.5 * scale * acc + a * c;
        } else {
            double acc = (ul - c) + (ur - c) + (w[0] - c) + (w[2] - c);
            if (RAD) {
                const double nl = from_left(w[0]), nr = from_right(w[0]), sl = from_left(w[2]),
                             sr = from_right(w[2]);
                acc += 0.5 * ((nl - c) + (nr - c) + (sl - c) + (sr - c));
            }
            Le = scale * acc + a * c;
        }
        if (t < 2 || r < r_first || r >= y1) return;  // uniform: rows outside the chunk
        const bool ydir = ((L.dir & 4u) && r == 0) || ((L.dir & 8u) && r == m - 1);
        const bool dirn = xdir || ydir;
        const double snew = dirn ? 0.0 : R.s - Le;
        const T sh = shat ? (T)(snew * A.shat_scale) : (T)snew;  // next cycle's source
        if (xout && r >= y0) {
            const unsigned q = (unsigned)r * (unsigned)m + (unsigned)x;
            st(u, q, R.u + c);
            st(sout, q, snew);
            if (shat) st(shat, q, sh);
            if (!dirn) {
                const unsigned long long b = dbits(snew);
                nb = b > nb ? b : nb;
            }
        }
        if (RES) {
            hs[0] = hs[1];
            hs[1] = hs[2];
            hs[2] = sh;
            // level-1 row J: fine rows 2J-1, 2J, 2J+1 (images at the faces)
            int J = -1;
            T up = hs[0], mid = hs[1], dn = hs[2];
            if ((r & 1) && r - 1 >= y0) {
                J = (r - 1) / 2;
                if (r == 1) up = dn;  // row -1 is the image of row 1
            } else if (!(r & 1) && r == m - 1) {
                J = r / 2;  // last row: row m is the image of row m - 2
                up = hs[1];
                mid = hs[2];
                dn = hs[1];
            }
            if (J >= 0) {
                const T v = T(0.5) * up + mid + T(0.5) * dn;
                const T vl = from_left(v), vr = from_right(v);
                const T res = (T(0.5) * vl + v + T(0.5) * vr) * T(0.25);
                if (xout && !(x & 1)) st(g1, (unsigned)J * (unsigned)m1 + (unsigned)(x >> 1), res);
            }
        }
    };
    constexpr int B = 3;
    Raw qa[B], qb[B];
    // rows past the last one load the last row again (see the visit)
    auto load_batch = [&](Raw(&q)[B], int t0) {
#pragma unroll
        for (int k = 0; k < B; ++k) load(q[k], min(t0 + k, rows - 1));
    };
    auto march = [&](auto hasg) {
        load_batch(qa, 0);
        int t0 = 0;
        for (; t0 + 2 * B <= rows; t0 += 2 * B) {
            load_batch(qb, t0 + B);
#pragma unroll
            for (int k = 0; k < B; ++k) step_row(qa[k], t0 + k, hasg);
            load_batch(qa, t0 + 2 * B);
#pragma unroll
            for (int k = 0; k < B; ++k) step_row(qb[k], t0 + B + k, hasg);
        }
        if (t0 < rows) {
            load_batch(qb, t0 + B);
#pragma unroll
            for (int k = 0; k < B; ++k)
                if (t0 + k < rows) step_row(qa[k], t0 + k, hasg);
#pragma unroll
            for (int k = 0; k < B; ++k)
                if (t0 + B + k < rows) step_row(qb[k], t0 + B + k, hasg);
        }
    };
    if (G)
        march(std::true_type());
    else
        march(std::false_type());
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(nb, off, 64);
        nb = o > nb ? o : nb;
    }
    if (lane == 0 && nb) atomicMax(A.norm + (size_t)(wid % kRedSlots) * kRedStride, nb);
}

// The closing visit of level 0 fused with the end of the cycle (FP32 cycles,
// constant coefficient, every cycle after the first): the visit's row
// pipeline (interpolation, S relaxations) feeds, instead of a store of e, one
// more stage that forms dL e in FP64 on a three-row window of the final e,
// updates u and the residual (written to s_out, s is only read), writes the
// next cycle's source and, RES, its restriction to level 1 -- what
// k_cycle_end2d does, on the same values in the same order, without the
// round trip of e through memory.  The strip's halo is two columns wider than
// the visit's (the operator's and the restriction's neighbour), and the chunk
// reads three more rows (the final e from row y0 - 2 to y1, the next source
// from row y0 - 1).
template <typename T, int RAD, int S>
__global__ __launch_bounds__(kVisitBlock) void k_visit_end2d(VisitArgs A, CycleEndArgs C)
{
    constexpr int PRO = 1;
    constexpr int HXV = (S + PRO + 1) / 2 * 2;  // the visit's halo
    constexpr int HX = HXV + 2;                 // columns a wavefront does not own, each side
    constexpr int W = 128 - 2 * HX;
    const Level L = A.L;
    const int m = L.m;
    const int lane = threadIdx.x & 63;
    const int strips = (m + W - 1) / W;
    const int wid = blockIdx.x * (kVisitBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sx = wid % strips, sy = wid / strips;
    const int y0 = sy * A.chunk;
    if (y0 >= m) return;
    const int y1 = min(m, y0 + A.chunk);
    const bool ydir_rows = ((L.dir & 4u) && y0 <= S + 2) || ((L.dir & 8u) && y1 + S + 1 >= m);
    const int xa = sx * W - HX + 2 * lane;  // even
    const int xma = mir(xa, m), xmb = mir(xa + 1, m);
    const bool lane_out = lane >= HX / 2 && lane < (HX + W) / 2;
    const bool outa = lane_out && xa < m, outb = lane_out && xa + 1 < m;

    RelaxK<T> K;
    K.scale = (T)L.scale;
    K.a = (T)L.a;
    K.theta = (T)L.theta;
    {
        const double Wd = RAD ? 6.0 : 4.0, D = Wd * L.scale - L.a;
        K.omt = (T)(1.0 - L.theta);
        K.beta = (T)(L.theta * L.scale / D);
        K.gamma = (T)(L.theta / D);
        K.aw = (T)(L.a - Wd * L.scale);
    }
    const bool xda = ((L.dir & 1u) && xma == 0) || ((L.dir & 2u) && xma == m - 1);
    const bool xdb = ((L.dir & 1u) && xmb == 0) || ((L.dir & 2u) && xmb == m - 1);
    const T oma = xda ? T(1) : K.omt, omb = xdb ? T(1) : K.omt;
    const T bea = xda ? T(0) : K.beta, beb = xdb ? T(0) : K.beta;
    const T gama = xda ? T(0) : K.gamma, gamb = xdb ? T(0) : K.gamma;
    const double scale = L.scale, a = L.a, escale = C.escale;
    const double *__restrict__ sres = C.s;
    double *__restrict__ sout = C.s_out;
    double *__restrict__ u = C.u;
    T *__restrict__ shat = (T *)C.shat;
    T *__restrict__ g1 = (T *)C.g1;
    const int m1 = (m + 1) / 2;
    const int r_first = max(y0 - 1, 0);
    // u is read only where it is written, s also one row above the chunk and
    // one column left of the strip (the restriction's neighbours): the other
    // lanes and rows read the nearest such column pair and row (cache hits,
    // values unused), so that the loads stay branch-free without fetching
    // the halo from memory
    const int xu = sx * W + 2 * min(max(lane - HX / 2, 0), W / 2 - 1);
    const unsigned xua = (unsigned)min(xu, m - 1), xub = (unsigned)min(xu + 1, m - 1);
    const bool s_lane = lane >= HX / 2 - 1 && lane < (HX + W) / 2;
    const unsigned xsa = s_lane ? (unsigned)xma : xua, xsb = s_lane ? (unsigned)xmb : xub;

    T wa[S][3], wb[S][3];
    T gha[S + 1], ghb[S + 1];
#pragma unroll
    for (int s = 0; s < S; ++s) wa[s][0] = wa[s][1] = wa[s][2] = wb[s][0] = wb[s][1] = wb[s][2] = T(0);
#pragma unroll
    for (int k = 0; k < S + 1; ++k) gha[k] = ghb[k] = T(0);
    double Ea[3] = {0.0, 0.0, 0.0}, Eb[3] = {0.0, 0.0, 0.0};  // final e at rows ro - 2, ro - 1, ro
    T Ha[3] = {T(0), T(0), T(0)}, Hb[3] = {T(0), T(0), T(0)};  // next source at rows rc - 2 .. rc
    unsigned long long nb = 0;

    const int r0 = y0 - S - 2;
    const int rows = (y1 - y0) + 2 * S + 3;
    unsigned ymask = 0;
    struct Row {
        RowIn2<T> v;
        double ua, ub, sa, sb;  // u and s at row rho - S - 1
    };
    auto step_row = [&](const Row &R, int t, auto odd, auto fast) __attribute__((always_inline)) {
        constexpr bool FAST = decltype(fast)::value;
        const int rho = r0 + t;
        const int rm = mir(rho, m);
        T va, vb;
        prolonged2<T, decltype(odd)::value>(R.v, va, vb);
        va = fresh_apart(va);
        vb = fresh_apart(vb);
#pragma unroll
        for (int k = S; k > 0; --k) {
            gha[k] = gha[k - 1];
            ghb[k] = ghb[k - 1];
        }
        if (FAST) {
            gha[0] = gama * R.v.ga;
            ghb[0] = gamb * R.v.gb;
        } else {
            gha[0] = K.gamma * R.v.ga;
            ghb[0] = K.gamma * R.v.gb;
            ymask = (ymask << 1) | (unsigned)(((L.dir & 4u) && rm == 0) || ((L.dir & 8u) && rm == m - 1));
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            wa[s][0] = wa[s][1];
            wa[s][1] = wa[s][2];
            wa[s][2] = va;
            wb[s][0] = wb[s][1];
            wb[s][1] = wb[s][2];
            wb[s][2] = vb;
            if (FAST) {
                relax2_fast<T, RAD>(wa[s], wb[s], gha[s + 1], ghb[s + 1], oma, omb, bea, beb, va, vb);
            } else {
                const bool yd = (ymask >> (s + 1)) & 1u;
                const T one[3] = {T(1), T(1), T(1)};
                T resa, resb;
                relax2<T, RAD, 0, 0>(wa[s], wb[s], one, one, gha[s + 1], ghb[s + 1], xda || yd, xdb || yd, T(0),
                                     T(0), K, va, vb, resa, resb);
            }
        }
        // final e at row ro = rho - S, in FP64 (Dirichlet nodes hold zero after the first cycle)
        Ea[0] = Ea[1];
        Ea[1] = Ea[2];
        Ea[2] = escale * (double)va;
        Eb[0] = Eb[1];
        Eb[1] = Eb[2];
        Eb[2] = escale * (double)vb;
        const int rc = rho - S - 1;
        // dL e at row rc, both columns (all lanes: cross-lane moves)
        const double ca = Ea[1], cb = Eb[1];
        const double la = from_left(cb), rb = from_right(ca);
        double acca = (la - ca) + (cb - ca) + (Ea[0] - ca) + (Ea[2] - ca);
        double accb = (ca - cb) + (rb - cb) + (Eb[0] - cb) + (Eb[2] - cb);
        if (RAD) {
            const double nla = from_left(Eb[0]), sla = from_left(Eb[2]);
            const double nrb = from_right(Ea[0]), srb = from_right(Ea[2]);
            acca += 0.5 * ((nla - ca) + (Eb[0] - ca) + (sla - ca) + (Eb[2] - ca));
            accb += 0.5 * ((Ea[0] - cb) + (nrb - cb) + (Ea[2] - cb) + (srb - cb));
        }
        const double Lea = scale * acca + a * ca, Leb = scale * accb + a * cb;
        const bool ydir = ((L.dir & 4u) && rc == 0) || ((L.dir & 8u) && rc == m - 1);
        const bool dira = xda || ydir, dirb = xdb || ydir;
        const double sna = dira ? 0.0 : R.sa - Lea, snb = dirb ? 0.0 : R.sb - Leb;
        const T sha = (T)(sna * C.shat_scale), shb = (T)(snb * C.shat_scale);
        // the next source's window shifts on every row (so that it rotates by
        // renaming); rows before r_first are never read from it
        Ha[0] = Ha[1];
        Ha[1] = Ha[2];
        Ha[2] = sha;
        Hb[0] = Hb[1];
        Hb[1] = Hb[2];
        Hb[2] = shb;
        if (t < 2 * S + 2 || rc < r_first || rc >= y1) return;  // uniform: rows outside the chunk
        if (rc >= y0) {
            const unsigned q = (unsigned)rc * (unsigned)m + (unsigned)xa;
            if (outa) {
                st(u, q, R.ua + ca);
                st(sout, q, sna);
                st(shat, q, sha);
                if (!dira) {
                    const unsigned long long bb = dbits(sna);
                    nb = bb > nb ? bb : nb;
                }
            }
            if (outb) {
                st(u, q + 1u, R.ub + cb);
                st(sout, q + 1u, snb);
                st(shat, q + 1u, shb);
                if (!dirb) {
                    const unsigned long long bb = dbits(snb);
                    nb = bb > nb ? bb : nb;
                }
            }
        }
        // level-1 row J of the next source: fine rows 2J - 1 .. 2J + 1 (images at the faces)
        int J = -1;
        T upa = Ha[0], mida = Ha[1], dna = Ha[2], upb = Hb[0], midb = Hb[1], dnb = Hb[2];
        if ((rc & 1) && rc - 1 >= y0) {
            J = (rc - 1) / 2;
            if (rc == 1) {
                upa = dna;
                upb = dnb;
            }
        } else if (!(rc & 1) && rc == m - 1) {
            J = rc / 2;
            upa = Ha[1];
            mida = Ha[2];
            dna = Ha[1];
            upb = Hb[1];
            midb = Hb[2];
            dnb = Hb[1];
        }
        if (J >= 0) {
            const T vva = T(0.5) * upa + mida + T(0.5) * dna;
            const T vvb = T(0.5) * upb + midb + T(0.5) * dnb;
            const T vl = from_left(vvb);
            const T res = (T(0.5) * vl + vva + T(0.5) * vvb) * T(0.25);
            if (outa) st(g1, (unsigned)J * (unsigned)m1 + (unsigned)(xa >> 1), res);
        }
    };
    constexpr int B = 3;
    Row qa[B], qb[B];
    auto load_batch = [&](Row(&q)[B], int t0, auto k0) __attribute__((always_inline)) {
        constexpr int K0 = decltype(k0)::value;
        unroll<B>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            int t = t0 + k;
            if (t > rows - 1) t -= 2 * ((t - rows + 2) >> 1);
            const int rho = r0 + t;
            load_row2<T, PRO, 0, false, ((S + K0 + k) & 1) != 0>(q[k].v, A, xma, xmb, rho, m);
            const unsigned ru = (unsigned)min(max(rho - S - 1, y0), y1 - 1) * (unsigned)m;
            const unsigned rs = (unsigned)min(max(rho - S - 1, r_first), y1 - 1) * (unsigned)m;
            q[k].ua = ld((const double *)u, ru + xua);
            q[k].ub = ld((const double *)u, ru + xub);
            q[k].sa = ld(sres, rs + xsa);
            q[k].sb = ld(sres, rs + xsb);
        });
    };
    using K0a = std::integral_constant<int, 0>;
    using K0b = std::integral_constant<int, B>;
    auto step_batch = [&](const Row(&q)[B], int t0, auto k0, auto fast, bool guard) __attribute__((always_inline)) {
        constexpr int K0 = decltype(k0)::value;
        unroll<B>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            if (!guard || t0 + k < rows)
                step_row(q[k], t0 + k, std::integral_constant<bool, ((S + K0 + k) & 1) != 0>(), fast);
        });
    };
    auto march = [&](auto fast) __attribute__((always_inline)) {
        load_batch(qa, 0, K0a());
        int t0 = 0;
        for (; t0 + 2 * B < rows; t0 += 2 * B) {
            load_batch(qb, t0 + B, K0b());
            step_batch(qa, t0, K0a(), fast, false);
            load_batch(qa, t0 + 2 * B, K0a());
            step_batch(qb, t0 + B, K0b(), fast, false);
        }
        if (t0 + B < rows) load_batch(qb, t0 + B, K0b());
        step_batch(qa, t0, K0a(), fast, true);
        step_batch(qb, t0 + B, K0b(), fast, true);
    };
    // chunks that read a Dirichlet row take the per-node select of the relaxation
    if (ydir_rows)
        march(std::false_type());
    else
        march(std::true_type());
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(nb, off, 64);
        nb = o > nb ? o : nb;
    }
    if (lane == 0 && nb) atomicMax(C.norm + (size_t)(wid % kRedSlots) * kRedStride, nb);
}

// One restriction step (Algorithm 1, eq. (3)) of a 2D level, row-marching:
// coarse node (I, J) = 1/4 of the sum over fine rows 2J - 1 .. 2J + 1 and
// columns 2I - 1 .. 2I + 1 of the tensor weights (1/2, 1, 1/2)^2 times the
// fine values, images outside the grid, accumulated row by row in the order
// of the per-node kernel (so the results are the same).  Lane l of a
// wavefront holds coarse column X = x0 - 1 + l and loads fine columns 2X and
// 2X + 1; 2X - 1 is the previous lane's 2X + 1 (lane 0 is that halo, 63
// columns written).  The wavefront marches down a chunk of coarse rows,
// loading each fine row once (the odd row below a coarse row is the odd row
// above the next), two coarse rows per turn with the next turn's rows in
// flight.
template <typename T>
__global__ __launch_bounds__(kVisitBlock) void k_restrict2d(const T *__restrict__ fine, T *__restrict__ coarse, int mc,
                                                         int chunk)
{
    const int mf = 2 * mc - 1;
    const int lane = threadIdx.x & 63;
    const int strips = (mc + 62) / 63;
    const int wid = blockIdx.x * (kVisitBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sx = wid % strips, sy = wid / strips;
    const int J0 = sy * chunk;
    if (J0 >= mc) return;
    const int J1 = min(mc, J0 + chunk);
    const int X = sx * 63 - 1 + lane;
    const bool out = lane >= 1 && X < mc;
    const unsigned ca = (unsigned)mir(min(2 * X, 2 * mf - 2), mf), cb = (unsigned)mir(min(2 * X + 1, 2 * mf - 2), mf);
    struct Rows {
        T a0, b0, a1, b1;  // fine rows 2J and 2J + 1, columns 2X and 2X + 1
    };
    auto load = [&](Rows &R, int J) __attribute__((always_inline)) {
        const unsigned r0 = (unsigned)mir(2 * J, mf) * (unsigned)mf, r1 = (unsigned)mir(2 * J + 1, mf) * (unsigned)mf;
        R.a0 = ld(fine, r0 + ca);
        R.b0 = ld(fine, r0 + cb);
        R.a1 = ld(fine, r1 + ca);
        R.b1 = ld(fine, r1 + cb);
    };
    // fine row 2J - 1 at columns 2X - 1, 2X, 2X + 1
    T ul, ua, ub;
    {
        const unsigned r = (unsigned)mir(2 * J0 - 1, mf) * (unsigned)mf;
        ua = fresh(ld(fine, r + ca));
        ub = fresh(ld(fine, r + cb));
        ul = from_left(ub);
    }
    auto step = [&](const Rows &R, int J) __attribute__((always_inline)) {
        const T ml = from_left(R.b0), dl = from_left(R.b1);
        T acc = T(0);
        acc += T(0.25) * ul;
        acc += T(0.5) * ua;
        acc += T(0.25) * ub;
        acc += T(0.5) * ml;
        acc += T(1) * R.a0;
        acc += T(0.5) * R.b0;
        acc += T(0.25) * dl;
        acc += T(0.5) * R.a1;
        acc += T(0.25) * R.b1;
        if (out && J < J1) st(coarse, (unsigned)J * (unsigned)mc + (unsigned)X, acc / T(4));
        ul = dl;
        ua = fresh(R.a1);
        ub = fresh(R.b1);
    };
    Rows qa, qb;
    load(qa, J0);
    int J = J0;
    for (; J + 2 < J1; J += 2) {
        load(qb, J + 1);
        step(qa, J);
        load(qa, J + 2);
        step(qb, J + 1);
    }
    if (J + 1 < J1) load(qb, J + 1);
    step(qa, J);
    if (J + 1 < J1) step(qb, J + 1);
}

// Two restriction steps in one pass: the level of mc nodes per axis
// (written, as k_restrict2d writes it) and the next coarser one.  Lane l
// holds column X = x0 - 2 + l of the first, as in k_restrict2d; lane 0 lacks
// its left fine column and lane 1 is the left neighbour of the strip's first
// even column, so lanes 2..63 are written (62 columns).  The wavefront
// marches its chunk of rows from one row above, keeps the last three rows,
// and each time they are rows 2K - 1, 2K, 2K + 1 (images at the faces) writes
// row K of the second level at the even columns, summed row by row as the
// per-node kernel sums, so that both levels are the same as from two
// k_restrict2d launches.
template <typename T>
__global__ __launch_bounds__(kVisitBlock) void k_restrict2d2(const T *__restrict__ fine, T *__restrict__ coarse,
                                                          T *__restrict__ coarse2, int mc, int chunk)
{
    const int mf = 2 * mc - 1, mc2 = (mc + 1) / 2;
    const int lane = threadIdx.x & 63;
    const int strips = (mc + 61) / 62;
    const int wid = blockIdx.x * (kVisitBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sx = wid % strips, sy = wid / strips;
    const int J0 = sy * chunk;  // even
    if (J0 >= mc) return;
    const int J1 = min(mc, J0 + chunk);
    const int Js = max(J0 - 1, 0);  // first row computed
    const int X = sx * 62 - 2 + lane;
    const bool out = lane >= 2 && X < mc;
    const bool out2 = out && !(X & 1);
    const unsigned ca = (unsigned)mir(min(2 * X, 2 * mf - 2), mf), cb = (unsigned)mir(min(2 * X + 1, 2 * mf - 2), mf);
    struct Rows {
        T a0, b0, a1, b1;  // fine rows 2J and 2J + 1, columns 2X and 2X + 1
    };
    auto load = [&](Rows &R, int J) __attribute__((always_inline)) {
        const unsigned r0 = (unsigned)mir(2 * J, mf) * (unsigned)mf, r1 = (unsigned)mir(2 * J + 1, mf) * (unsigned)mf;
        R.a0 = ld(fine, r0 + ca);
        R.b0 = ld(fine, r0 + cb);
        R.a1 = ld(fine, r1 + ca);
        R.b1 = ld(fine, r1 + cb);
    };
    // fine row 2J - 1 at columns 2X - 1, 2X, 2X + 1
    T ul, ua, ub;
    {
        const unsigned r = (unsigned)mir(2 * Js - 1, mf) * (unsigned)mf;
        ua = fresh(ld(fine, r + ca));
        ub = fresh(ld(fine, r + cb));
        ul = from_left(ub);
    }
    T h0 = T(0), h1 = T(0), h2 = T(0);  // first-level rows J - 2, J - 1, J
    auto restrict2 = [&](T up, T mid, T dn, int K) __attribute__((always_inline)) {
        T acc = T(0);
        acc += T(0.25) * from_left(up);
        acc += T(0.5) * up;
        acc += T(0.25) * from_right(up);
        acc += T(0.5) * from_left(mid);
        acc += T(1) * mid;
        acc += T(0.5) * from_right(mid);
        acc += T(0.25) * from_left(dn);
        acc += T(0.5) * dn;
        acc += T(0.25) * from_right(dn);
        if (out2) st(coarse2, (unsigned)K * (unsigned)mc2 + (unsigned)(X >> 1), acc / T(4));
    };
    auto step = [&](const Rows &R, int J) __attribute__((always_inline)) {
        const T ml = from_left(R.b0), dl = from_left(R.b1);
        T acc = T(0);
        acc += T(0.25) * ul;
        acc += T(0.5) * ua;
        acc += T(0.25) * ub;
        acc += T(0.5) * ml;
        acc += T(1) * R.a0;
        acc += T(0.5) * R.b0;
        acc += T(0.25) * dl;
        acc += T(0.5) * R.a1;
        acc += T(0.25) * R.b1;
        const T v = acc / T(4);
        if (out && J >= J0) st(coarse, (unsigned)J * (unsigned)mc + (unsigned)X, v);
        ul = dl;
        ua = fresh(R.a1);
        ub = fresh(R.b1);
        h0 = h1;
        h1 = h2;
        h2 = v;
        // second-level row K: rows 2K - 1 (row 1 for K = 0), 2K, 2K + 1 (row
        // 2K - 1 for the last row)
        if ((J & 1) && J - 1 >= J0)
            restrict2(J == 1 ? h2 : h0, h1, h2, (J - 1) / 2);
        else if (!(J & 1) && J == mc - 1)
            restrict2(h1, h2, h1, J / 2);
    };
    Rows qa, qb;
    load(qa, Js);
    int J = Js;
    for (; J + 2 < J1; J += 2) {
        load(qb, J + 1);
        step(qa, J);
        load(qa, J + 2);
        step(qb, J + 1);
    }
    if (J + 1 < J1) load(qb, J + 1);
    step(qa, J);
    if (J + 1 < J1) step(qb, J + 1);
}

// Rows of strips (strips x rows per strip) from which a level is large
// enough for its visits to be bound by memory traffic rather than by the
// length of one wavefront's row pipeline (4097^2 and above at six
// relaxations).
constexpr long long kLargeLevelRows = 1 << 17;

// Rows per wavefront: short chunks give more wavefronts (the row chain of a
// wavefront is sequential) at the cost of 2S recomputed halo rows per chunk.
// Short visits take short chunks: 8 rows (1% faster solves than 6, 12, 16,
// 24 or 32), 4 on levels of at most 1025 nodes per axis and 2 on levels of at
// most 257, which have few wavefronts to spread their latency over (each 1%
// faster on the 4097^2 solves, 3% on the 129^2 ones).  Long visits on a large
// level take the shortest chunk for which the launch fills the wavefront
// slots the chip has for the kernel in one round (slots), no workgroup
// waiting for a second: all of them in FP32 (38 rows on the 4097^2 level),
// half of them in FP64 and in the fused closing visit, whose registers allow
// two wavefronts per SIMD (152 rows, one wavefront per SIMD).  Measured on
// the 4097^2 solves: the FP64 and mixed solves 1% faster with half the slots,
// the FP32 visit 1% slower (unfused mixed solve).  Every SIMD must get the
// same whole number of wavefronts: 3/8 or 5/8 of the slots (some SIMDs with
// one more than others, or none) made the mixed solve 8% / 15% slower, a
// third or a quarter 13% / 24%.
int chunk_rows(int requested, int m, int strips, int sweeps, long long slots)
{
    if (requested > 0) return requested;
    if (sweeps < 4 || (long long)strips * m < kLargeLevelRows) return m <= 257 ? 2 : m <= 1025 ? 4 : 8;
    const long long per = slots / strips;  // chunks per strip that fill the slots once
    if (per < 1) return std::min(m, 96);
    return std::max(8, (int)((m + per - 1) / per));
}

// Wavefronts of one visit kernel the chip holds at once (occupancy from the
// kernel's registers, times the compute units); 0 when unknown.
template <typename T, int RAD, int SIG, int S, int PRO, int REC>
long long resident_waves()
{
    static const int per_cu = [] {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_visit2d<T, RAD, SIG, S, PRO, REC>, kVisitBlock, 0) !=
            hipSuccess) {
            (void)hipGetLastError();
            b = 0;
        }
        return b;
    }();
    return (long long)per_cu * device_cus() * (kVisitBlock / 64);
}

template <typename T, int RAD, int SIG, int S, int PRO, int REC>
void launch_one(const VisitArgs &a0, hipStream_t st)
{
    VisitArgs a = a0;
    const int m = a.L.m;
    constexpr int W = 128 - 2 * ((S + PRO + 1) / 2 * 2);
    const int strips = (m + W - 1) / W;
    if (a0.chunk <= 0 && S >= 4)
        a.chunk = chunk_rows(0, m, strips, S, resident_waves<T, RAD, SIG, S, PRO, REC>() / (sizeof(T) == 8 ? 2 : 1));
    else a.chunk = chunk_rows(a0.chunk, m, strips, S, 0);
    a.chunk += a.chunk & 1;  // chunks start at even rows: row parity follows from the place in the march
    const long long waves = (long long)strips * ((m + a.chunk - 1) / a.chunk);
    const unsigned blocks = (unsigned)((waves + kVisitBlock / 64 - 1) / (kVisitBlock / 64));
    hipLaunchKernelGGL((k_visit2d<T, RAD, SIG, S, PRO, REC>), dim3(blocks), dim3(kVisitBlock), 0, st, a);
}

template <typename T, int RAD, int SIG, int S>
void launch_s(const VisitArgs &a, hipStream_t st)
{
    bool rec = false;
    for (int k = 0; k < a.sweeps; ++k) rec = rec || a.pres[k] >= 0;
    if (a.prolong && rec)
        launch_one<T, RAD, SIG, S, 1, 1>(a, st);
    else if (a.prolong)
        launch_one<T, RAD, SIG, S, 1, 0>(a, st);
    else if (rec)
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


// The fused closing visit and cycle end: chunks sized like the long FP64
// visits (half of this kernel's wavefront slots: one wavefront per SIMD).
template <typename T, int RAD, int S>
long long visit_end_resident_waves()
{
    static const int per_cu = [] {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_visit_end2d<T, RAD, S>, kVisitBlock, 0) != hipSuccess) {
            (void)hipGetLastError();
            b = 0;
        }
        return b;
    }();
    return (long long)per_cu * device_cus() * (kVisitBlock / 64);
}

template <typename T, int RAD, int S>
void launch_visit_end_s(const VisitArgs &a0, const CycleEndArgs &c, hipStream_t st)
{
    VisitArgs a = a0;
    const int m = a.L.m;
    constexpr int W = 128 - 2 * ((S + 2) / 2 * 2 + 2);
    const int strips = (m + W - 1) / W;
    if (a0.chunk <= 0 && S >= 4)
        a.chunk = chunk_rows(0, m, strips, S, visit_end_resident_waves<T, RAD, S>() / 2);
    else a.chunk = chunk_rows(a0.chunk, m, strips, S, 0);
    a.chunk += a.chunk & 1;
    const long long waves = (long long)strips * ((m + a.chunk - 1) / a.chunk);
    const unsigned blocks = (unsigned)((waves + kVisitBlock / 64 - 1) / (kVisitBlock / 64));
    hipLaunchKernelGGL((k_visit_end2d<T, RAD, S>), dim3(blocks), dim3(kVisitBlock), 0, st, a, c);
}

template <typename T, int RAD>
void launch_visit_end_r(const VisitArgs &a, const CycleEndArgs &c, hipStream_t st)
{
    switch (a.sweeps) {
    case 1: launch_visit_end_s<T, RAD, 1>(a, c, st); break;
    case 2: launch_visit_end_s<T, RAD, 2>(a, c, st); break;
    case 4: launch_visit_end_s<T, RAD, 4>(a, c, st); break;
    default: launch_visit_end_s<T, RAD, 6>(a, c, st); break;
    }
}

// One row-marching restriction step of a 2D level of mc >= 65 coarse nodes
// per axis: chunks of coarse rows sized for about 8192 wavefronts (short
// chains: the pass is latency bound below a few million nodes).
template <typename T>
void launch_restrict2d(int mc, const T *fine, T *coarse, hipStream_t st)
{
    const long long strips = (mc + 62) / 63;
    int chunk = (int)((mc * strips + 8191) / 8192);
    chunk = std::max(4, chunk + (chunk & 1));
    const long long waves = strips * ((mc + chunk - 1) / chunk);
    const dim3 grid((unsigned)((waves + kVisitBlock / 64 - 1) / (kVisitBlock / 64))), block(kVisitBlock);
    hipLaunchKernelGGL((k_restrict2d<T>), grid, block, 0, st, fine, coarse, mc, chunk);
}

template <typename T>
void launch_restrict2d2(int mc, const T *fine, T *coarse, T *coarse2, hipStream_t st)
{
    const long long strips = (mc + 61) / 62;
    int chunk = (int)((mc * strips + 8191) / 8192);
    chunk = std::max(4, chunk + (chunk & 1));  // even: second-level rows start at even rows
    const long long waves = strips * ((mc + chunk - 1) / chunk);
    const dim3 grid((unsigned)((waves + kVisitBlock / 64 - 1) / (kVisitBlock / 64))), block(kVisitBlock);
    hipLaunchKernelGGL((k_restrict2d2<T>), grid, block, 0, st, fine, coarse, coarse2, mc, chunk);
}

template <typename T>
void launch_cycle_end2d(const Variant &v, const CycleEndArgs &a0, hipStream_t st)
{
    CycleEndArgs a = a0;
    const int m = a.L.m;
    const bool res = a.g1 != nullptr && a.s_out != nullptr && a.s_out != a.s;
    const int W = res ? 60 : 62;
    const long long strips = (m + W - 1) / W;
    // Two wavefronts per SIMD and no SIMD with a third (at most twice as many
    // wavefronts as SIMDs): on 4097^2 137 rows in FP64 (2010 wavefronts), the
    // FP64 solve 0.5% faster than with 136 rows (2077: a third wavefront on
    // some SIMDs), 1% faster than with 92 or 96 (about three per SIMD), 3%
    // faster than with 192.  A level too small to give the chip's 1024 SIMDs
    // a wavefront each at 96 rows takes shorter chunks (129^2: 8 rows, 51
    // wavefronts).
    if (a0.chunk > 0) {
        a.chunk = a0.chunk;
    } else if (strips * ((m + 95) / 96) < 1024) {
        a.chunk = std::max(8, (int)(((long long)m * strips + 1023) / 1024));
    } else {
        const long long per = std::max(1LL, 8LL * device_cus() / strips);  // chunks per strip
        a.chunk = (int)((m + per - 1) / per);
    }
    if (res) a.chunk = (a.chunk + 1) & ~1;  // chunks start at even rows
    const long long waves = strips * ((m + a.chunk - 1) / a.chunk);
    const dim3 grid((unsigned)((waves + kVisitBlock / 64 - 1) / (kVisitBlock / 64))), block(kVisitBlock);
#define SGML_CE(R, S)                                                                       \
    if (res)                                                                                \
        hipLaunchKernelGGL((k_cycle_end2d<T, R, S, 1>), grid, block, 0, st, a);             \
    else                                                                                    \
        hipLaunchKernelGGL((k_cycle_end2d<T, R, S, 0>), grid, block, 0, st, a);
    if (v.radial && v.sigma) {
        SGML_CE(1, 1)
    } else if (v.radial) {
        SGML_CE(1, 0)
    } else if (v.sigma) {
        SGML_CE(0, 1)
    } else {
        SGML_CE(0, 0)
    }
#undef SGML_CE
}


// The visits of one stencil (RAD), with or without a coefficient field;
// each (precision, stencil) pair is instantiated in a file of its own, so
// that the four compile in parallel.
template <typename T, int RAD>
void launch_visit2d_r(const VisitArgs &a, bool sigma, hipStream_t st)
{
    if (sigma)
        launch_rs<T, RAD, 1>(a, st);
    else
        launch_rs<T, RAD, 0>(a, st);
}
template <typename T, int RAD>
void launch_visit_end2d_r(const VisitArgs &a, const CycleEndArgs &c, hipStream_t st)
{
    launch_visit_end_r<T, RAD>(a, c, st);
}
extern template void launch_visit_end2d_r<float, 0>(const VisitArgs &, const CycleEndArgs &, hipStream_t);
extern template void launch_visit_end2d_r<float, 1>(const VisitArgs &, const CycleEndArgs &, hipStream_t);

template <typename T>
void launch_visit_end2d(const Variant &v, const VisitArgs &a, const CycleEndArgs &c, hipStream_t st)
{
    if (v.radial)
        launch_visit_end2d_r<T, 1>(a, c, st);
    else
        launch_visit_end2d_r<T, 0>(a, c, st);
}

extern template void launch_visit2d_r<float, 0>(const VisitArgs &, bool, hipStream_t);
extern template void launch_visit2d_r<float, 1>(const VisitArgs &, bool, hipStream_t);
extern template void launch_visit2d_r<double, 0>(const VisitArgs &, bool, hipStream_t);
extern template void launch_visit2d_r<double, 1>(const VisitArgs &, bool, hipStream_t);

template <typename T>
void launch_visit2d(const Variant &v, const VisitArgs &a, hipStream_t st)
{
    if (v.radial)
        launch_visit2d_r<T, 1>(a, v.sigma, st);
    else
        launch_visit2d_r<T, 0>(a, v.sigma, st);
}


}  // namespace sgml
