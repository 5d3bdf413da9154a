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

// Five-term dot product with a fixed association and rounding (an explicit
// FMA chain), so that every kernel that inlines it rounds identically.
template <typename T>
__device__ __forceinline__ T dot5(T a0, T b0, T a1, T b1, T a2, T b2, T a3, T b3, T a4, T b4)
{
    return fma(a4, b4, fma(a3, b3, fma(a2, b2, fma(a1, b1, a0 * b0))));
}

// Workgroups of `kern` that one compute unit holds at once (cached per kernel).
template <typename K>
int resident_per_cu(K kern, int& cache)
{
    if (cache == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, kThreads, 0) != hipSuccess || n <= 0) n = 2;
        cache = n;
    }
    return cache;
}

// Geometry of the streaming level kernel, per problem dimensionality,
// columns per lane CPL (cols_per_lane below: 1 for both element types) and
// tile width.
//  3-D: a workgroup owns kT1 = 8 coarse rows x kT2 = (64 CW CPL - 3) / 2
//       coarse columns; its staged region is 19 fine rows x 2 kT2 + 3
//       columns.  Narrow: CW = 1 wave per staged row, kT2 = 30 (rows
//       r = wave, wave + 4, ...).  Wide: CW = 2 waves side by side
//       per row, kT2 = 62 (rows r = wave / 2, wave / 2 + 2, ...): half as
//       many tile edges per row (cache lines split between two tiles' stores)
//       and a slightly smaller halo, for twice the rows per wave, which only
//       the two-plane register ring leaves room for.  The per-field
//       launches take the geometry wide_tile gives; the batch's 3-D items
//       take either, as its autotuner chose.
//  2-D (m0, 1, m2) and 1-D (1, 1, m2): one staged row, four waves side by
//       side (kT2 = (256 CPL - 3) / 2 = 126 at CPL = 1).
template <bool kAct1, int CPL, bool kWide>
struct LevelGeom {
    static constexpr int CW = kAct1 ? (kWide ? 2 : 1) : 4;  // waves per staged row
    static constexpr int NL = 64 * CW;                  // lanes per staged row
    static constexpr int NCW = CPL * NL;                // staged columns
    static constexpr int kT1 = kAct1 ? 8 : 1;
    static constexpr int kT2 = (NCW - 3) / 2;
    static constexpr int NR = kAct1 ? 2 * kT1 + 3 : 1;  // staged rows
    static constexpr int RW = 4 / CW;                   // rows handled at once
    static constexpr int NRW = (NR + RW - 1) / RW;      // rows per wave
    static constexpr int H = NCW / 2;                   // even (odd) columns per row
    static constexpr int GW = kAct1 ? 32 * CW * CPL : 256;  // dim-2 outputs per pass row
    static constexpr int OB = NR * H + 16;              // odd-column block (bank offset 16)
    static_assert(2 * kT2 + 3 <= NCW, "region fits the staged width");
    static_assert(kT2 + 2 <= H && kT2 <= GW, "stencil windows fit");
};
// One column per lane for both types.  FP32 column pairs (CPL = 2, one
// 8-byte access per lane) are supported by the code but not used: rows of
// 2^k + 1 elements start at odd element offsets on every other row, and an
// 8-byte buffer access at a 4-byte-aligned address is not performed as an
// unaligned access on this device, so half of the rows would need two
// accesses; measured, the pair layout was slower.
template <typename T>
constexpr int cols_per_lane()
{
    return 1;
}
// Wide 3-D tiles for FP64 (measured: level 0 of 513^3 0.75 -> 0.68 ms) and
// for the FP32 load-vector pass (kDec false, which runs the two-plane ring
// anyway); the FP32 decomposition pass keeps narrow tiles, whose fewer rows
// per wave leave room for its deeper register ring (wide tiles with the
// two-plane ring measured slower there).
template <typename T, bool kDec>
constexpr bool wide_tile()
{
    return sizeof(T) == 8 || !kDec;
}

constexpr int kMaxChunk = 128;       // coarse planes per workgroup (LDS tables)
// Plane buffers of the streaming tile (its prefetch depth plus one): four
// for the FP32 decomposition pass without a correction array, two where the
// registers are needed elsewhere (FP64, the correction's second array, or
// the load-vector pass, which runs at higher occupancy).
template <typename T, bool kDec, bool kZ>
constexpr int stream_ring()
{
    return (sizeof(T) == 4 && kDec && !kZ) ? 4 : 2;
}
// Minimum waves per SIMD the streaming kernel is compiled for: the deep ring
// is held at five (at most 96 registers, a few spilled), which measured
// faster than four waves without spills.
template <typename T, bool kDec, bool kZ>
constexpr int stream_min_waves()
{
    return stream_ring<T, kDec, kZ>() == 4 ? 5 : 1;
}

// A lane's CPL consecutive columns of one row: the row at scalar byte offset
// `so` from the descriptor's base.  FP32 pairs move as one 8-byte access
// where the columns are adjacent in memory (kU), else as two 4-byte accesses
// `step` bytes apart.  The hardware range check is per dword, so a pair that
// straddles the end of the range keeps its first element.
template <bool kU, typename T, int N>
__device__ __forceinline__ void buf_load_cols(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned so, unsigned step,
                                              T (&v)[N])
{
    static_assert(N == 1 || (N == 2 && sizeof(T) == 4), "one column, or an FP32 pair");
    if constexpr (N == 1) {
        v[0] = buf_load_so<T>(r, off, so);
    } else if (kU) {
        const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, off, __builtin_amdgcn_readfirstlane((int)so), 0);
        v[0] = __builtin_bit_cast(T, w.x);
        v[1] = __builtin_bit_cast(T, w.y);
    } else {
        v[0] = buf_load_so<T>(r, off, so);
        v[1] = buf_load_so<T>(r, off + step, so);
    }
}
template <bool kU, typename T, int N>
__device__ __forceinline__ void buf_store_cols(const T (&v)[N], __amdgpu_buffer_rsrc_t r, unsigned off, unsigned so,
                                               unsigned step)
{
    static_assert(N == 1 || (N == 2 && sizeof(T) == 4), "one column, or an FP32 pair");
    if constexpr (N == 1) {
        buf_store_so(v[0], r, off, so);
    } else if (kU) {
        u32x2 w;
        w.x = __builtin_bit_cast(unsigned, v[0]);
        w.y = __builtin_bit_cast(unsigned, v[1]);
        __builtin_amdgcn_raw_buffer_store_b64(w, r, off, __builtin_amdgcn_readfirstlane((int)so), 0);
    } else {
        buf_store_so(v[0], r, off, so);
        buf_store_so(v[1], r, off + step, so);
    }
}

// LDS of one streaming level tile.  sU: the staged plane (even planes); sC:
// coefficients (zero at coarse and outside nodes), even columns [r][H] then
// odd columns, so that the dim-2 stencil reads consecutive words; sG: dim-2
// results [r][GW]; sW0, sK0: dim-0 interpolation weights and stencil rows of
// the chunk.
template <typename T, bool kAct0, bool kAct1, bool kDec, bool kWide = wide_tile<T, kDec>()>
struct alignas(16) LevelSmem {
    using G = LevelGeom<kAct1, cols_per_lane<T>(), kWide>;
    T sU[kDec ? G::NR * G::NCW : 1];
    T sC[G::OB + G::NR * G::H];
    T sG[G::NR * G::GW];
    T sW0[kDec && kAct0 ? 2 * (2 * kMaxChunk + 3) : 1];
    T sK0[kAct0 ? 5 * (kMaxChunk + 3) : 1];  // planes P0-1 .. P1+1
};

// One workgroup's share of a level step: tile (t1, t2) of coarse columns and
// chunk ch of coarse planes, bid = (ch * nt1 + t1) * nt2 + t2.  Used by the
// per-level launch and by the batched kernel.  kU: the input (and, when
// decomposing, the coefficient output) has unit column stride, so a lane's
// columns move in one access.
// kWide: the tile geometry (defaults to the per-level launch's; the batch
// chooses it per plan).
template <typename T, bool kAct0, bool kAct1, bool kDec, bool kZ, bool kU, bool kWide = wide_tile<T, kDec>()>
__device__ __forceinline__ void stream_level_tile(const StreamArgs<T>& a, int bid,
                                                  LevelSmem<T, kAct0, kAct1, kDec, kWide>& sm)
{
    constexpr int CPL = cols_per_lane<T>();
    using G = LevelGeom<kAct1, CPL, kWide>;
    constexpr int NR = G::NR, NCW = G::NCW, NRW = G::NRW, RW = G::RW, H = G::H, GW = G::GW;
    constexpr int kT1 = G::kT1, kT2 = G::kT2, OB = G::OB;
    constexpr int NGP = (NR + (kThreads / GW) - 1) / (kThreads / GW);  // dim-2 passes
    constexpr int NOUT = kAct1 ? kT1 / (kThreads / GW) : 1;            // dim-1 outputs per thread
    constexpr bool kRowUni = (GW == 64);  // a dim-2 pass row (and dim-1 output row) per wave
    constexpr unsigned S = sizeof(T);
    static_assert(!kAct1 || NOUT * (kThreads / GW) == kT1, "dim-1 outputs cover the tile");
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
    const int F0 = kAct0 ? max(2 * P0 - 2, 0) : 0;
    const int F1 = kAct0 ? min(2 * P1, m0 - 1) : 0;
    const int oF0 = kAct0 ? 2 * P0 : 0, oF1 = kAct0 ? min(2 * P1, m0) : 1;

    // dim-0 tables of the chunk, staged once the first planes' loads are
    // issued (one memory latency then covers both)
    auto stage_tables = [&] {
        if (kDec && kAct0)
            for (int e = tid; e < 2 * (F1 - F0 + 1); e += kThreads) sW0[e] = a.tb.w[0][2 * F0 + e];
        if (kAct0)
            // rows P0-1 .. P1+1, zero outside [P0, P1): no plane of another
            // chunk receives contributions from this one
            for (int e = tid; e < 5 * (P1 - P0 + 3); e += kThreads) {
                const int i = P0 - 1 + e / 5;
                sK0[e] = (i >= P0 && i < P1) ? a.tb.K[0][5 * i + e % 5] : T(0);
            }
    };

    // ---- this lane's staged columns cb .. cb + CPL - 1
    const int cb = ((wave % G::CW) * 64 + lane) * CPL;
    const int gc = C0 + cb;  // global column of cb
    constexpr int RC = 2 * kT2 + 3;  // region columns
    // column j of the lane: in the region and the grid / owned by the tile
    auto col_in = [&](int j) { return cb + j < RC && gc + j >= 0 && gc + j < m2; };
    auto col_own = [&](int j) { return col_in(j) && gc + j >= 2 * I2 && gc + j < min(2 * (I2 + kT2), m2); };
    // Interpolation weights per column: zero outside the grid, so outside
    // nodes get a zero coefficient (their loads return zero); (1, 0) at even
    // columns, so coarse nodes get exactly u - u = 0.  ul, ur: staged columns
    // of the two coarse neighbours (the column itself at even columns).
    T wcl[CPL], wch[CPL];
    int ul[CPL], ur[CPL];
#pragma unroll
    for (int j = 0; j < CPL; j++) {
        const int cj = cb + j;
        const bool odd = cj & 1;
        wcl[j] = wch[j] = T(0);
        ul[j] = ur[j] = cb;
        if (kDec && col_in(j)) {
            ul[j] = cj & ~1;
            ur[j] = odd ? cj + 1 : cj & ~1;
            wcl[j] = odd ? a.tb.w[2][2 * (gc + j)] : T(1);
            wch[j] = odd ? a.tb.w[2][2 * (gc + j) + 1] : T(0);
        }
    }
    // byte offsets of the lane's first column, per array (kOut: no column
    // of the lane in range); the pair's second column is `step` bytes on
    bool any_in = false, any_own = false;
#pragma unroll
    for (int j = 0; j < CPL; j++) {
        any_in = any_in || col_in(j);
        any_own = any_own || col_own(j);
    }
    const int as1 = (int)a.av.s[1], as2 = (int)a.av.s[2];
    const int cs1 = (int)a.cv.s[1], cs2 = (int)a.cv.s[2];
    const int ws1 = (int)a.wv.s[1], ws2 = (int)a.wv.s[2];
    // the coarse value goes to W from the lane's column 0 (even in FP32, where
    // cb is even; in FP64 only at even lanes)
    constexpr int jw = 0;
    const bool w_own = col_own(jw) && !((cb + jw) & 1);
    const unsigned cA = any_in ? (unsigned)(gc * as2) * S : kOut;
    const unsigned cC = any_own ? (unsigned)(gc * cs2) * S : kOut;
    const unsigned cW = w_own ? (unsigned)(((gc + jw) >> 1) * ws2) * S : kOut;
    const unsigned stepA = (unsigned)as2 * S, stepC = (unsigned)cs2 * S;

    // ---- this wave's staged rows r = rg + RW * k (wave-uniform)
    const int rg = wave / G::CW;
    T* const sUw = sU + rg * NCW + cb;
    const T* const sUrow = sU + rg * NCW;
    T* const sCrow = sC + rg * H;
    const int oR0 = kAct1 ? 2 * I1 : 0, oR1 = kAct1 ? min(2 * (I1 + kT1), m1) : 1;
    // One buffer descriptor per array and plane, holding the plane's bytes;
    // each row is reached through the instruction's scalar offset (the row's
    // byte offset in the plane, kept in a scalar register for the whole
    // kernel).  A row outside the grid loads a grid row instead and its
    // values are replaced by zero where they are used (rin), so the loads
    // stay unconditional and need no per-row lane offsets.
    const unsigned spanA = (unsigned)((m1 - 1) * as1 + (m2 - 1) * as2 + 1) * S;
    const unsigned spanC = (unsigned)((m1 - 1) * cs1 + (m2 - 1) * cs2 + 1) * S;
    const unsigned spanW = (unsigned)(((m1 - 1) / 2) * ws1 + ((m2 - 1) / 2) * ws2 + 1) * S;
    int gr[NRW];               // grid row (uniform)
    bool rin[NRW], rown[NRW];  // in the grid / owned (uniform)
    unsigned soA[NRW], soC[NRW], soW[NRW];  // row byte offsets in a plane (uniform)
    T wrl[NRW], wrh[NRW];
#pragma unroll
    for (int k = 0; k < NRW; k++) {
        const int r = rg + RW * k;
        gr[k] = R0 + r;
        rin[k] = r < NR && gr[k] >= 0 && gr[k] < m1;
        rown[k] = rin[k] && gr[k] >= oR0 && gr[k] < oR1;
        // a row past the staged region re-reads this wave's previous row (the
        // same lines: no further memory traffic), a row outside the grid the
        // nearest grid row
        const int grc = min(max(r < NR ? gr[k] : gr[k] - RW, 0), m1 - 1);
        soA[k] = (unsigned)uni((int)((unsigned)(grc * as1) * S));
        soC[k] = (unsigned)uni((int)((unsigned)(grc * cs1) * S));
        soW[k] = (unsigned)uni((int)((unsigned)((grc >> 1) * ws1) * S));
        wrl[k] = T(0);
        wrh[k] = T(0);
        if (kDec && rin[k]) {
            wrl[k] = (kAct1 && (r & 1)) ? uni(a.tb.w[1][2 * gr[k]]) : T(1);
            wrh[k] = (kAct1 && (r & 1)) ? uni(a.tb.w[1][2 * gr[k] + 1]) : T(0);
        }
    }

    // ---- dim-2 / dim-1 stencil weights of this thread's outputs: coarse
    // column I2 + g2, coarse rows I1 + g1 + q (kThreads / GW), q < NOUT
    const int g2 = tid % GW;
    const int g1 = kRowUni ? wave : tid / GW;
    T k2[5], k1[NOUT][5];
#pragma unroll
    for (int t = 0; t < 5; t++) {
        k2[t] = (g2 < kT2 && I2 + g2 < c2) ? a.tb.K[2][5 * (I2 + g2) + t] : T(0);
#pragma unroll
        for (int q = 0; q < NOUT; q++) {
            const int i1 = I1 + g1 + q * (kThreads / GW);
            const T kv = (kAct1 && i1 < c1) ? a.tb.K[1][5 * i1 + t] : T(0);
            k1[q][t] = kRowUni ? uni(kv) : kv;
        }
    }
    // load-vector outputs: with one output row per wave the row goes into
    // the (scalar) descriptor, else into the lane's offset
    const bool cvalid = g2 < kT2 && I2 + g2 < c2;
    const int fs1 = (int)a.fv.s[1], fs2 = (int)a.fv.s[2];
    const unsigned rowF = (unsigned)((c2 - 1) * fs2 + 1) * S;
    const unsigned spanF = (unsigned)((c1 - 1) * fs1 + (c2 - 1) * fs2 + 1) * S;
    unsigned vF[NOUT];
#pragma unroll
    for (int q = 0; q < NOUT; q++) {
        const int i1 = I1 + g1 + q * (kThreads / GW);
        const bool ok = cvalid && (!kAct1 || i1 < c1);
        vF[q] = ok ? (unsigned)((kRowUni ? 0 : i1 * fs1) + (I2 + g2) * fs2) * S : kOut;
    }

    // plane strides are below 2^31 (a plane is under 2 GiB, checked when the
    // arguments are validated): 32 x 32 -> 64 products
    const unsigned as0 = (unsigned)a.av.s[0], cs0 = (unsigned)a.cv.s[0], ws0 = (unsigned)a.wv.s[0],
                   fs0 = (unsigned)a.fv.s[0];
    auto mul64 = [](int i, unsigned st) { return (int64_t)((uint64_t)(unsigned)i * st); };
    // all loads are unconditional: a load under a branch makes the compiler
    // wait for every outstanding load where the paths join
    using Cols = T[CPL];
    auto load_plane = [&](int f, Cols (&v)[NRW], Cols (&vz)[NRW]) {
        const int64_t po = mul64(f, as0);
        const __amdgpu_buffer_rsrc_t rA = make_rsrc(a.A + po, spanA);
        const __amdgpu_buffer_rsrc_t rZ = make_rsrc(kZ ? a.Z + po : a.A, kZ ? spanA : 0u);
#pragma unroll
        for (int k = 0; k < NRW; k++) {
            buf_load_cols<kU>(rA, cA, soA[k], stepA, v[k]);
            if (kZ) buf_load_cols<kU>(rZ, cA, soA[k], stepA, vz[k]);
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
    auto sC_at = [&](int k, int j) -> T& {
        const int cj = cb + j;
        return sCrow[RW * k * H + (cj & 1) * OB + (cj >> 1)];
    };
    // Coefficients of plane f into sC (and C, W); returns through P the 2-D
    // interpolant of an even plane.  Ends with a barrier after the sC writes.
    // The caller has replaced the values of rows outside the grid by zero.
    auto coef_plane = [&](int f, bool even, const Cols (&cur)[NRW], Cols (&P)[NRW], const Cols (&Pa)[NRW],
                          const Cols (&Pb)[NRW]) {
        if (!kDec) {
#pragma unroll
            for (int k = 0; k < NRW; k++) {
                if (!row_exists(k)) continue;
#pragma unroll
                for (int j = 0; j < CPL; j++) {
                    // coarse positions hold other classes: read them as zero
                    const bool ce = !((cb + j) & 1);
                    sC_at(k, j) = (even && !RP && ce) ? T(0) : cur[k][j];
                }
            }
            lds_barrier();
            return;
        }
        const bool fown = f >= oF0 && f < oF1;
        const int64_t pc = mul64(f, cs0);
        const __amdgpu_buffer_rsrc_t rC = make_rsrc(a.C + pc, spanC);
        Cols cv[NRW];
        if (even) {
            const int64_t pw = mul64(f >> 1, ws0);
            const __amdgpu_buffer_rsrc_t rW = make_rsrc(a.W + pw, spanW);
#pragma unroll
            for (int k = 0; k < NRW; k++) {
                if (!row_exists(k)) continue;
                if constexpr (CPL == 2) {
                    typedef T T2 __attribute__((ext_vector_type(2)));
                    T2 w2;
                    w2.x = cur[k][0];
                    w2.y = cur[k][1];
                    *reinterpret_cast<T2*>(sUw + RW * k * NCW) = w2;
                } else {
                    sUw[RW * k * NCW] = cur[k][0];
                }
            }
            lds_barrier();
#pragma unroll
            for (int k = 0; k < NRW; k++) {
                if (!row_exists(k)) continue;
                const T* const ru = sUrow + RW * k * NCW;
#pragma unroll
                for (int j = 0; j < CPL; j++) {
                    const bool ce = !((cb + j) & 1);
                    T p;
                    if (CPL == 2 && j == 0) {
                        // even column: the column weights are (1, 0)
                        p = RP ? lerp2(wrl[k], ru[ul[0] - NCW], wrh[k], ru[ul[0] + NCW]) : wrl[k] * cur[k][0];
                    } else if (RP) {
                        const T lo = lerp2(wcl[j], ru[ul[j] - NCW], wch[j], ru[ur[j] - NCW]);
                        const T hi = lerp2(wcl[j], ru[ul[j] + NCW], wch[j], ru[ur[j] + NCW]);
                        p = lerp2(wrl[k], lo, wrh[k], hi);
                    } else {
                        p = wrl[k] * lerp2(wcl[j], ru[ul[j]], wch[j], ru[ur[j]]);
                    }
                    P[k][j] = p;
                    const T c = cur[k][j] - p;  // 0 at coarse and outside nodes
                    sC_at(k, j) = c;
                    // coarse positions take u: the output of the finest step
                    // needs it, deeper steps' values there are overwritten later
                    cv[k][j] = (!RP && ce) ? cur[k][j] : c;
                }
                if (fown && rown[k]) {
                    buf_store_cols<kU>(cv[k], rC, cC, soC[k], stepC);
                    if (!RP) buf_store_so(cur[k][jw], rW, cW, soW[k]);
                }
            }
        } else {
            // odd plane: every node is fine; interpolate along dim 0 between
            // the 2-D interpolants of the even neighbours
            const T wl = sW0[2 * (f - F0)], wh = sW0[2 * (f - F0) + 1];
#pragma unroll
            for (int k = 0; k < NRW; k++) {
                if (!row_exists(k)) continue;
#pragma unroll
                for (int j = 0; j < CPL; j++) {
                    cv[k][j] = cur[k][j] - lerp2(wl, Pa[k][j], wh, Pb[k][j]);
                    sC_at(k, j) = cv[k][j];
                }
                if (fown && rown[k]) buf_store_cols<kU>(cv[k], rC, cC, soC[k], stepC);
            }
        }
        lds_barrier();
    };

    // dim-2 then dim-1 stencils of the plane in sC: this thread's values of
    // the plane's contribution (zeros stand in for coarse and outside nodes,
    // so there are no masks or bounds)
    auto reduce_plane = [&](T (&g)[NOUT]) {
#pragma unroll
        for (int ps = 0; ps < NGP; ps++) {
            const int r = g1 + ps * (kThreads / GW);
            if (NR % (kThreads / GW) != 0 && r >= NR) continue;
            const T* E = sC + r * H + g2;
            const T* O = sC + OB + r * H + g2;
            if (g2 < kT2)
                sG[r * GW + g2] = dot5(k2[0], E[0], k2[1], O[0], k2[2], E[1], k2[3], O[1], k2[4], E[2]);
        }
        lds_barrier();
#pragma unroll
        for (int q = 0; q < NOUT; q++) {
            if (kAct1) {
                const T* Gp = sG + 2 * (g1 + q * (kThreads / GW)) * GW + g2;
                g[q] = dot5(k1[q][0], Gp[0], k1[q][1], Gp[GW], k1[q][2], Gp[2 * GW], k1[q][3], Gp[3 * GW],
                            k1[q][4], Gp[4 * GW]);
            } else {
                g[q] = sG[g2];
            }
        }
    };
    // The next plane writes sU and sC only before its first barrier and sG
    // only after it; every reader of sC passed the dim-2 barrier and every
    // reader of sG reaches the next plane's first barrier only after reading.
    auto store_f = [&](int i, const T (&v)[NOUT], bool keep) {
#pragma unroll
        for (int q = 0; q < NOUT; q++) {
            if constexpr (kRowUni) {
                const int i1 = I1 + g1 + q * (kThreads / GW);
                buf_store(v[q], make_rsrc(a.F + mul64(i, fs0) + (int64_t)i1 * fs1, keep ? rowF : 0u), vF[q]);
            } else {
                buf_store(v[q], make_rsrc(a.F + mul64(i, fs0), keep ? spanF : 0u), vF[q]);
            }
        }
    };

    // plane buffers: a ring of D, so that D - 1 planes are in flight while
    // one is consumed
    constexpr int D = stream_ring<T, kDec, kZ>();
    Cols B0[NRW], B1[NRW], B2[NRW], B3[NRW];  // B2, B3 unused (and dropped) when D = 2
    Cols Z0[NRW], Z1[NRW];                    // unused (and dropped) without the correction
    Cols cur[NRW], Pp[NRW], Pn[NRW];
#pragma unroll
    for (int k = 0; k < NRW; k++)
#pragma unroll
        for (int j = 0; j < CPL; j++) Pp[k][j] = Pn[k][j] = T(0);
    T g[NOUT];

    if (!kAct0) {
        load_plane(0, B0, Z0);
        lds_barrier();  // (no dim-0 tables)
#pragma unroll
        for (int k = 0; k < NRW; k++)
#pragma unroll
            for (int j = 0; j < CPL; j++) cur[k][j] = rin[k] ? (kZ ? B0[k][j] + Z0[k][j] : B0[k][j]) : T(0);
        coef_plane(0, true, cur, Pn, Pp, Pp);
        reduce_plane(g);
        store_f(0, g, true);
        return;
    }

    // Planes in the order s_0 = F0, then pairs s_{2k+1} = F0+2k+2 (even),
    // s_{2k+2} = F0+2k+1 (odd): an odd plane follows both even neighbours.
    // Plane s_j sits in buffer j mod D and is replaced by s_{j+D} right
    // after its last use, so no loaded register is ever copied (a copy would
    // wait for the load); planes past F1 re-read F1.
    auto seq = [&](int j) { return min(j == 0 ? F0 : ((j & 1) ? F0 + j + 1 : F0 + j - 1), F1); };
    const int K = (F1 - F0) / 2;
    load_plane(seq(0), B0, Z0);
    load_plane(seq(1), B1, Z1);
    if constexpr (D > 2) {
        load_plane(seq(2), B2, Z0);
        load_plane(seq(3), B3, Z0);
    }
    stage_tables();
    lds_barrier();  // tables
    // running dim-0 sums of coarse planes A = F0/2 + k, B = A + 1, Cc = A + 2
    T accA[NOUT], accB[NOUT], accC[NOUT];
#pragma unroll
    for (int q = 0; q < NOUT; q++) accA[q] = accB[q] = accC[q] = T(0);
    const T* const k0 = sK0 + 5 * (F0 / 2 - P0 + 1) + 2;  // k0[5 (i - F0/2) + t]
    // rows outside the grid (they loaded the nearest grid row) read as zero
    auto mask_rows = [&](Cols (&B)[NRW]) {
#pragma unroll
        for (int q = 0; q < NRW; q++)
#pragma unroll
            for (int jj = 0; jj < CPL; jj++) B[q][jj] = rin[q] ? B[q][jj] : T(0);
    };
    auto consume = [&](int j, Cols (&B)[NRW], Cols (&BZ)[NRW]) {
        const int f = seq(j);
        const bool even = (j & 1) || j == 0;
        if (kZ) {
#pragma unroll
            for (int q = 0; q < NRW; q++)
#pragma unroll
                for (int jj = 0; jj < CPL; jj++) cur[q][jj] = rin[q] ? B[q][jj] + BZ[q][jj] : T(0);
            load_plane(seq(j + D), B, BZ);
            coef_plane(f, even, cur, Pn, Pp, Pn);
        } else {
            mask_rows(B);
            coef_plane(f, even, B, Pn, Pp, Pn);
            load_plane(seq(j + D), B, BZ);
        }
    };
    consume(0, B0, Z0);
    reduce_plane(g);
#pragma unroll
    for (int q = 0; q < NOUT; q++) {
        accA[q] = fma(k0[0], g[q], accA[q]);
        accB[q] = fma(k0[5 - 2], g[q], accB[q]);
    }
    // step k: even plane F0+2k+2 from buffer E, odd plane F0+2k+1 from O
    auto step = [&](int k, Cols (&E)[NRW], Cols (&EZ)[NRW], Cols (&O)[NRW], Cols (&OZ)[NRW]) {
        const T* const kk = k0 + 5 * k;  // coarse plane ia = F0/2 + k completes in this step
#pragma unroll
        for (int q = 0; q < NRW; q++)
#pragma unroll
            for (int j = 0; j < CPL; j++) Pp[q][j] = Pn[q][j];
        consume(2 * k + 1, E, EZ);
        reduce_plane(g);
#pragma unroll
        for (int q = 0; q < NOUT; q++) {
            accA[q] = fma(kk[2], g[q], accA[q]);
            accB[q] = fma(kk[5], g[q], accB[q]);
            accC[q] = fma(kk[10 - 2], g[q], accC[q]);
        }
        consume(2 * k + 2, O, OZ);
        reduce_plane(g);
#pragma unroll
        for (int q = 0; q < NOUT; q++) {
            accA[q] = fma(kk[1], g[q], accA[q]);
            accB[q] = fma(kk[5 - 1], g[q], accB[q]);
        }
        const int ia = F0 / 2 + k;
        store_f(ia, accA, ia >= P0);
#pragma unroll
        for (int q = 0; q < NOUT; q++) {
            accA[q] = accB[q];
            accB[q] = accC[q];
            accC[q] = T(0);
        }
    };
    if constexpr (D > 2) {
        int k = 0;
        for (; k + 1 < K; k += 2) {
            step(k, B1, Z1, B2, Z0);
            step(k + 1, B3, Z1, B0, Z0);
        }
        if (k < K) step(k, B1, Z1, B2, Z0);
    } else {
        for (int k = 0; k < K; k++) step(k, B1, Z1, B0, Z0);
    }
    // last coarse plane of the grid: its stencil has no right half
    store_f(F1 / 2, accA, F1 == m0 - 1 && F1 / 2 < P1);
    };
    if (kAct1 && (rg & 1))
        run(std::true_type{});
    else
        run(std::false_type{});
}

}  // namespace
}  // namespace mgr
