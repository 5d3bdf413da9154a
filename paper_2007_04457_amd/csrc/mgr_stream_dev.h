// Device code of the streaming level step (see mgr_stream.hip for the
// method): shared by the per-level kernels and the batched work-queue
// kernel.  Internal; included by .hip files only.
#pragma once
#include <algorithm>
#include <type_traits>

#include "mgr_internal.h"

namespace mgr {
namespace {

constexpr int kThreads = 256;

// Workgroup barrier that waits only for this wave's LDS traffic.  HIP's
// __syncthreads() also drains outstanding global loads, which would stall the
// register prefetch of the next plane at every barrier; nothing here needs
// global memory ordered across the barrier (each output is written by one
// thread and never read back inside the kernel).
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Consecutive workgroup ids are dealt round-robin to the 8 XCDs; renumber so
// each XCD works on a contiguous range of tiles and neighbouring tiles share
// its L2 for the halo re-reads.
__device__ __forceinline__ int remap_xcd(int bid, int nb)
{
    const int nx = 8;
    const int lo = nb / nx, rem = nb % nx;
    const int x = bid % nx, local = bid / nx;
    return (x < rem) ? x * (lo + 1) + local : rem * (lo + 1) + (x - rem) * lo + local;
}

// Geometry of the streaming level kernel, per problem dimensionality.
//  3-D: a workgroup owns kT1 = 8 coarse rows x kT2 = 30 coarse columns; its
//       staged region is 19 fine rows x 64 columns (63 used), one wave per
//       row (rows r = wave, wave + 4, ...), lane = column.
//  2-D (m0, 1, m2) and 1-D (1, 1, m2): one staged row of 256 columns (255
//       used), four waves side by side; kT2 = 126 coarse columns.
template <bool kAct1>
struct LevelGeom {
    static constexpr int kT1 = kAct1 ? 8 : 1;
    static constexpr int kT2 = kAct1 ? 30 : 126;
    static constexpr int NR = kAct1 ? 2 * kT1 + 3 : 1;  // staged rows
    static constexpr int CW = kAct1 ? 1 : 4;            // waves per staged row
    static constexpr int NCW = 64 * CW;                 // staged columns
    static constexpr int RW = 4 / CW;                   // rows handled at once
    static constexpr int NRW = (NR + RW - 1) / RW;      // rows per wave
    static constexpr int H = NCW / 2;                   // even (odd) columns per row
    static constexpr int GW = kAct1 ? 32 : 256;         // dim-2 outputs per pass row
    static constexpr int OB = NR * H + 16;              // odd-column block (bank offset 16)
    static_assert(2 * kT2 + 3 <= NCW, "region fits the staged width");
    static_assert(kT2 + 2 <= H && kT2 <= GW, "stencil windows fit");
};

constexpr int kMaxChunk = 128;       // coarse planes per workgroup (LDS tables)
constexpr unsigned kOut = 0x80000000u;  // buffer offset past every range: loads 0, stores dropped

// Marks a value the same in every lane (kept in scalar registers).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uni(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Raw buffer access (gfx9 descriptor): the hardware range check turns an
// offset at or past `bytes` into a load of zero or a dropped store.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, unsigned bytes)
{
    // base and size are wave-uniform; say so, or the compiler loops over lanes
    const unsigned long long b = (unsigned long long)base;
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    void* ub = (void*)(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(ub, (short)0, __builtin_amdgcn_readfirstlane((int)bytes), 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, unsigned off)
{
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}

// LDS of one streaming level tile.  sU: the staged plane (even planes); sC:
// coefficients (zero at coarse and outside nodes), even columns [r][H] then
// odd columns, so that the dim-2 stencil reads consecutive words; sG: dim-2
// results [r][GW]; sW0, sK0: dim-0 interpolation weights and stencil rows of
// the chunk.
template <typename T, bool kAct0, bool kAct1, bool kDec>
struct LevelSmem {
    using G = LevelGeom<kAct1>;
    T sU[kDec ? G::NR * G::NCW : 1];
    T sC[G::OB + G::NR * G::H];
    T sG[G::NR * G::GW];
    T sW0[kDec && kAct0 ? 2 * (2 * kMaxChunk + 3) : 1];
    T sK0[kAct0 ? 5 * (kMaxChunk + 3) : 1];  // planes P0-1 .. P1+1
};

// One workgroup's share of a level step: tile (t1, t2) of coarse columns and
// chunk ch of coarse planes, bid = (ch * nt1 + t1) * nt2 + t2.  Used by the
// per-level launch below and by the batched work-queue kernel.
template <typename T, bool kAct0, bool kAct1, bool kDec, bool kZ>
__device__ __forceinline__ void stream_level_tile(const StreamArgs<T>& a, int bid,
                                                  LevelSmem<T, kAct0, kAct1, kDec>& sm)
{
    using G = LevelGeom<kAct1>;
    constexpr int NR = G::NR, NCW = G::NCW, NRW = G::NRW, RW = G::RW, H = G::H, GW = G::GW;
    constexpr int kT1 = G::kT1, kT2 = G::kT2, OB = G::OB;
    constexpr int NGP = (NR + (kThreads / GW) - 1) / (kThreads / GW);  // dim-2 passes
    constexpr unsigned S = sizeof(T);
    T* const sU = sm.sU;
    T* const sC = sm.sC;
    T* const sG = sm.sG;
    T* const sW0 = sm.sW0;
    T* const sK0 = sm.sK0;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = uni(tid >> 6);
    const int nt1 = a.nt1, nt2 = a.nt2;
    const int t2 = bid % nt2;
    const int t1 = (bid / nt2) % nt1;
    const int ch = bid / (nt2 * nt1);

    const int m0 = (int)a.av.n[0], m1 = (int)a.av.n[1], m2 = (int)a.av.n[2];
    const int c0 = (int)a.fv.n[0], c1 = (int)a.fv.n[1], c2 = (int)a.fv.n[2];
    const int I1 = t1 * kT1, I2 = t2 * kT2;
    const int P0 = ch * a.chunk, P1 = min(P0 + a.chunk, c0);
    const int R0 = kAct1 ? 2 * I1 - 2 : 0;  // region origin (may be negative)
    const int C0 = 2 * I2 - 2;
    const int RB = max(R0, 0);              // first in-grid region row
    const int F0 = kAct0 ? max(2 * P0 - 2, 0) : 0;
    const int F1 = kAct0 ? min(2 * P1, m0 - 1) : 0;
    const int oF0 = kAct0 ? 2 * P0 : 0, oF1 = kAct0 ? min(2 * P1, m0) : 1;

    if (kDec && kAct0)
        for (int e = tid; e < 2 * (F1 - F0 + 1); e += kThreads) sW0[e] = a.tb.w[0][2 * F0 + e];
    if (kAct0)
        // rows P0-1 .. P1+1, zero outside [P0, P1): no plane of another chunk
        // receives contributions from this one
        for (int e = tid; e < 5 * (P1 - P0 + 3); e += kThreads) {
            const int i = P0 - 1 + e / 5;
            sK0[e] = (i >= P0 && i < P1) ? a.tb.K[0][5 * i + e % 5] : T(0);
        }

    // ---- this lane's staged column
    const int c = (wave % G::CW) * 64 + lane;
    const int gc = C0 + c;
    const bool cin = c < 2 * kT2 + 3 && gc >= 0 && gc < m2;
    const bool cown = cin && gc >= 2 * I2 && gc < min(2 * (I2 + kT2), m2);
    const bool ceven = !(c & 1);
    // interpolation weights: zero outside the grid, so outside nodes get a
    // zero coefficient (their loads return zero); (1, 0) at even columns, so
    // coarse nodes get exactly u - u = 0
    T wcl = T(0), wch = T(0);
    int ucl = 0, ucr = 0;
    if (kDec && cin) {
        ucl = c & ~1;
        ucr = ucl + 2 * (c & 1);
        wcl = (c & 1) ? a.tb.w[2][2 * gc] : T(1);
        wch = (c & 1) ? a.tb.w[2][2 * gc + 1] : T(0);
    }
    // ---- this wave's staged rows r = rg + RW * k (wave-uniform)
    const int rg = wave / G::CW;
    T* const sUw = sU + rg * NCW + c;
    const T* const sUl = sU + rg * NCW + ucl;
    const T* const sUr = sU + rg * NCW + ucr;
    T* const sCw = sC + rg * H + (c & 1) * OB + (c >> 1);
    const int as1 = (int)a.av.s[1], as2 = (int)a.av.s[2];
    const int cs1 = (int)a.cv.s[1], cs2 = (int)a.cv.s[2];
    const int ws1 = (int)a.wv.s[1], ws2 = (int)a.wv.s[2];
    const int oR0 = kAct1 ? 2 * I1 : 0, oR1 = kAct1 ? min(2 * (I1 + kT1), m1) : 1;
    unsigned vA[NRW], vC[NRW], vW[NRW];  // byte offsets from the region's first in-grid row
    T wrl[NRW], wrh[NRW];
#pragma unroll
    for (int k = 0; k < NRW; k++) {
        const int r = rg + RW * k;
        const int gr = R0 + r;
        const bool rin = r < NR && gr >= 0 && gr < m1;
        const bool own = rin && cown && gr >= oR0 && gr < oR1;
        vA[k] = (rin && cin) ? (unsigned)((gr - RB) * as1 + gc * as2) * S : kOut;
        vC[k] = own ? (unsigned)((gr - RB) * cs1 + gc * cs2) * S : kOut;
        vW[k] = (own && !(gr & 1) && ceven) ? (unsigned)(((gr - RB) >> 1) * ws1 + (gc >> 1) * ws2) * S : kOut;
        wrl[k] = T(0);
        wrh[k] = T(0);
        if (kDec && rin) {
            wrl[k] = (kAct1 && (r & 1)) ? uni(a.tb.w[1][2 * gr]) : T(1);
            wrh[k] = (kAct1 && (r & 1)) ? uni(a.tb.w[1][2 * gr + 1]) : T(0);
        }
    }
    // bytes reachable from the region's first in-grid row, per array
    const unsigned spanA = (unsigned)((min(R0 + NR, m1) - RB) * as1 + m2 * as2) * S;
    const unsigned spanC = (unsigned)((min(R0 + NR, m1) - RB) * cs1 + m2 * cs2) * S;
    const unsigned spanW = (unsigned)(((min(R0 + NR, m1) - RB) / 2 + 1) * ws1 + ((m2 + 1) / 2) * ws2) * S;

    // ---- dim-2 / dim-1 stencil weights of this thread's output column
    const int g2 = tid % GW, g1 = tid / GW;  // output: coarse row I1+g1, column I2+g2
    T k2[5], k1[5];
#pragma unroll
    for (int t = 0; t < 5; t++) {
        k2[t] = (g2 < kT2 && I2 + g2 < c2) ? a.tb.K[2][5 * (I2 + g2) + t] : T(0);
        k1[t] = (kAct1 && g1 < kT1 && I1 + g1 < c1) ? a.tb.K[1][5 * (I1 + g1) + t] : T(0);
    }
    const bool gvalid = g1 < kT1 && g2 < kT2 && I1 + g1 < c1 && I2 + g2 < c2;
    const unsigned vF = gvalid ? (unsigned)((I1 + g1) * (int)a.fv.s[1] + (I2 + g2) * (int)a.fv.s[2]) * S : kOut;
    const unsigned spanF = (unsigned)((c1 - 1) * (int)a.fv.s[1] + c2 * (int)a.fv.s[2]) * S;

    // plane strides are below 2^31 (checked by the launcher): 32 x 32 -> 64 products
    const unsigned as0 = (unsigned)a.av.s[0], cs0 = (unsigned)a.cv.s[0], ws0 = (unsigned)a.wv.s[0],
                   fs0 = (unsigned)a.fv.s[0];
    auto mul64 = [](int i, unsigned st) { return (int64_t)((uint64_t)(unsigned)i * st); };
    // all loads are unconditional: a load under a branch makes the compiler
    // wait for every outstanding load where the paths join
    auto load_plane = [&](int f, T (&v)[NRW], T (&vz)[NRW]) {
        const int64_t po = mul64(f, as0) + (int64_t)RB * as1;
        const __amdgpu_buffer_rsrc_t rA = make_rsrc(a.A + po, spanA);
        const __amdgpu_buffer_rsrc_t rZ = make_rsrc(kZ ? a.Z + po : a.A, spanA);
#pragma unroll
        for (int k = 0; k < NRW; k++) {
            v[k] = buf_load<T>(rA, vA[k]);
            if (kZ) vz[k] = buf_load<T>(rZ, vA[k]);
        }
    };

    // The loop body is specialised on the parity RP of this wave's rows
    // (rows rg, rg + RW, ... all share it), so per-row branches are static.
    auto run = [&](auto rpc) {
    constexpr bool RP = decltype(rpc)::value;
    // row k of this wave exists (the last one may fall past the region)
    auto row_exists = [&](int k) {
        constexpr int rgmax = RP ? ((RW - 1) % 2 ? RW - 1 : RW - 2) : ((RW - 1) % 2 ? RW - 2 : RW - 1);
        return (rgmax + RW * k < NR) || (rg + RW * k < NR);
    };
    // Coefficients of plane f into sC (and C, W); returns through P the 2-D
    // interpolant of an even plane.  Ends with a barrier after the sC writes.
    auto coef_plane = [&](int f, bool even, const T (&cur)[NRW], T (&P)[NRW], const T (&Pa)[NRW],
                          const T (&Pb)[NRW]) {
        if (!kDec) {
#pragma unroll
            for (int k = 0; k < NRW; k++) {
                if (!row_exists(k)) continue;
                // coarse positions hold other classes: read them as zero
                sCw[RW * k * H] = (even && !RP && ceven) ? T(0) : cur[k];
            }
            lds_barrier();
            return;
        }
        const bool fown = f >= oF0 && f < oF1;
        const __amdgpu_buffer_rsrc_t rC = make_rsrc(a.C + mul64(f, cs0) + (int64_t)RB * cs1, fown ? spanC : 0u);
        if (even) {
            const __amdgpu_buffer_rsrc_t rW =
                make_rsrc(a.W + mul64(f >> 1, ws0) + (int64_t)(RB >> 1) * ws1, fown ? spanW : 0u);
#pragma unroll
            for (int k = 0; k < NRW; k++)
                if (row_exists(k)) sUw[RW * k * NCW] = cur[k];
            lds_barrier();
#pragma unroll
            for (int k = 0; k < NRW; k++) {
                if (!row_exists(k)) continue;
                T p;
                if (RP) {
                    const T lo = lerp2(wcl, sUl[(RW * k - 1) * NCW], wch, sUr[(RW * k - 1) * NCW]);
                    const T hi = lerp2(wcl, sUl[(RW * k + 1) * NCW], wch, sUr[(RW * k + 1) * NCW]);
                    p = lerp2(wrl[k], lo, wrh[k], hi);
                } else {
                    p = wrl[k] * lerp2(wcl, sUl[RW * k * NCW], wch, sUr[RW * k * NCW]);
                }
                P[k] = p;
                const T cv = cur[k] - p;  // 0 at coarse and outside nodes
                sCw[RW * k * H] = cv;
                // coarse positions take u: the output of the finest step
                // needs it, deeper steps' values there are overwritten later
                buf_store((!RP && ceven) ? cur[k] : cv, rC, vC[k]);
                if (!RP) buf_store(cur[k], rW, vW[k]);
            }
        } else {
            // odd plane: every node is fine; interpolate along dim 0 between
            // the 2-D interpolants of the even neighbours
            const T wl = sW0[2 * (f - F0)], wh = sW0[2 * (f - F0) + 1];
#pragma unroll
            for (int k = 0; k < NRW; k++) {
                if (!row_exists(k)) continue;
                const T cv = cur[k] - lerp2(wl, Pa[k], wh, Pb[k]);
                sCw[RW * k * H] = cv;
                buf_store(cv, rC, vC[k]);
            }
        }
        lds_barrier();
    };

    // dim-2 then dim-1 stencils of the plane in sC: this thread's value of
    // the plane's contribution (zeros stand in for coarse and outside nodes,
    // so there are no masks or bounds)
    auto reduce_plane = [&]() -> T {
#pragma unroll
        for (int ps = 0; ps < NGP; ps++) {
            const int r = g1 + ps * (kThreads / GW);
            if (NR % (kThreads / GW) != 0 && r >= NR) continue;
            const T* E = sC + r * H + g2;
            const T* O = sC + OB + r * H + g2;
            if (g2 < kT2)
                sG[r * GW + g2] = k2[0] * E[0] + k2[1] * O[0] + k2[2] * E[1] + k2[3] * O[1] + k2[4] * E[2];
        }
        lds_barrier();
        if (kAct1) {
            const T* Gp = sG + 2 * g1 * GW + g2;
            return k1[0] * Gp[0] + k1[1] * Gp[GW] + k1[2] * Gp[2 * GW] + k1[3] * Gp[3 * GW] +
                   k1[4] * Gp[4 * GW];
        }
        return sG[g2];
    };
    // The next plane writes sU and sC only before its first barrier and sG
    // only after it; every reader of sC passed the dim-2 barrier and every
    // reader of sG reaches the next plane's first barrier only after reading.
    auto store_f = [&](int i, T v) { buf_store(v, make_rsrc(a.F + mul64(i, fs0), spanF), vF); };

    T X[NRW], XZ[NRW], Y[NRW], YZ[NRW], cur[NRW], Pp[NRW], Pn[NRW];
#pragma unroll
    for (int k = 0; k < NRW; k++) {
        X[k] = XZ[k] = Y[k] = YZ[k] = Pp[k] = Pn[k] = T(0);
    }
    lds_barrier();  // tables

    if (!kAct0) {
        load_plane(0, X, XZ);
#pragma unroll
        for (int k = 0; k < NRW; k++) cur[k] = kZ ? X[k] + XZ[k] : X[k];
        coef_plane(0, true, cur, Pn, Pp, Pp);
        store_f(0, reduce_plane());
        return;
    }

    // Planes in the order F0, then pairs (F0+2k+2, F0+2k+1): an odd plane
    // follows both even neighbours.  Two planes are in flight: X holds the
    // odd planes, Y the even ones (planes past F1 re-read F1).  Each buffer
    // is reloaded right after its last use, so no loaded register is copied
    // (a copy would wait for the load).
    const int K = (F1 - F0) / 2;
    load_plane(F0, X, XZ);
    load_plane(min(F0 + 2, F1), Y, YZ);
    // running dim-0 sums of coarse planes A = F0/2 + k, B = A + 1, Cc = A + 2
    T accA = T(0), accB = T(0), accC = T(0);
    const T* const k0 = sK0 + 5 * (F0 / 2 - P0 + 1) + 2;  // k0[5 (i - F0/2) + t]
    auto consume = [&](int f, bool even, T (&B)[NRW], T (&BZ)[NRW], int fnext) {
        if (kZ) {
#pragma unroll
            for (int q = 0; q < NRW; q++) cur[q] = B[q] + BZ[q];
            load_plane(fnext, B, BZ);
            coef_plane(f, even, cur, Pn, Pp, Pn);
        } else {
            coef_plane(f, even, B, Pn, Pp, Pn);
            load_plane(fnext, B, BZ);
        }
    };
    consume(F0, true, X, XZ, min(F0 + 1, F1));
    {
        const T g = reduce_plane();
        accA += k0[0] * g;
        accB += k0[5 - 2] * g;
    }
    for (int k = 0; k < K; k++) {
        const T* const kk = k0 + 5 * k;  // coarse plane ia = F0/2 + k completes in this step
#pragma unroll
        for (int q = 0; q < NRW; q++) Pp[q] = Pn[q];
        consume(F0 + 2 * k + 2, true, Y, YZ, min(F0 + 2 * k + 4, F1));
        T g = reduce_plane();
        accA += kk[2] * g;
        accB += kk[5] * g;
        accC += kk[10 - 2] * g;
        consume(F0 + 2 * k + 1, false, X, XZ, min(F0 + 2 * k + 3, F1));
        g = reduce_plane();
        accA += kk[1] * g;
        accB += kk[5 - 1] * g;
        const int ia = F0 / 2 + k;
        if (ia >= P0) store_f(ia, accA);
        accA = accB;
        accB = accC;
        accC = T(0);
    }
    // last coarse plane of the grid: its stencil has no right half
    if (F1 == m0 - 1 && F1 / 2 < P1) store_f(F1 / 2, accA);
    };
    if (kAct1 && (rg & 1))
        run(std::true_type{});
    else
        run(std::false_type{});
}

}  // namespace
}  // namespace mgr
