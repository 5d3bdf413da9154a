// Recomposition of a level step (Sec. II-A, the inverse of the streaming
// decomposition): coarse nodes take the corrected coarse values W - Z (Z the
// correction of the level step), fine-only nodes c + Pi (W - Z), streamed
// plane by plane along dim 0 with the corrected coarse tile in LDS.
#include <algorithm>
#include <cstdint>

#include "mgr_stream_dev.h"

namespace mgr {
namespace {

// Recomposition of one level step (Sec. II-A, the inverse of the above):
// coarse nodes take the corrected coarse values W - Z (Z the correction of
// this level step), fine-only nodes c + Pi (W - Z).
// A workgroup owns a tile of fine rows x columns (3-D: 16 x 64, one wave per
// set of 4 rows of one parity, lane = column; 2-D and 1-D: one row of 256
// columns) and a chunk of coarse planes.  For each coarse plane a it stages
// the corrected coarse tile in LDS, forms the 2-D prolongation Q(a) at its
// fine nodes (kept in registers) and emits fine plane 2a - 1 (between Q(a-1)
// and Q(a)) and plane 2a.  Coefficients are read with buffer loads whose
// offsets at coarse positions and outside the grid are out of range (they
// read 0), so every output is A + Q with no select; stores outside the
// tile's own nodes are dropped the same way.
template <bool kAct1>
struct ReconGeom {
    static constexpr int kT1 = kAct1 ? 8 : 1;     // coarse rows per tile
    static constexpr int kT2 = kAct1 ? 32 : 128;  // coarse columns per tile
    static constexpr int FR = kAct1 ? 2 * kT1 : 1;
    static constexpr int CW = kAct1 ? 1 : 4;      // waves per fine row
    static constexpr int RW = 4 / CW;             // rows handled at once
    static constexpr int NRW = FR / RW;           // fine rows per wave
    static constexpr int CR = kAct1 ? kT1 + 1 : 1;
    static constexpr int CC = kT2 + 1;
    static constexpr int NCT = (CR * CC + kThreads - 1) / kThreads;  // coarse tile slots per thread
    static_assert(64 * CW == 2 * kT2, "one lane per fine column");
};

template <typename T, bool kAct0, bool kAct1>
__global__ void __launch_bounds__(kThreads) k_stream_recon(StreamArgs<T> a)
{
    using G = ReconGeom<kAct1>;
    constexpr int kT1 = G::kT1, kT2 = G::kT2, NRW = G::NRW, RW = G::RW, CC = G::CC, CR = G::CR, NCT = G::NCT;
    constexpr unsigned S = sizeof(T);
    __shared__ T sW[2][CR * CC];
    __shared__ T sW0[2 * (2 * kMaxChunk + 1)];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = uni(tid >> 6);
    const int bid = remap_xcd((int)blockIdx.x, (int)gridDim.x);
    const int nt1 = a.nt1, nt2 = a.nt2;
    const int t2 = bid % nt2;
    const int t1 = (bid / nt2) % nt1;
    const int ch = bid / (nt2 * nt1);
    // a.av: coefficients (level grid view), a.cv: output view, a.wv: coarse W (= Z's layout)
    const int m0 = (int)a.av.n[0], m1 = (int)a.av.n[1], m2 = (int)a.av.n[2];
    const int c0 = (int)a.wv.n[0], c1 = (int)a.wv.n[1], c2 = (int)a.wv.n[2];
    const int I1 = t1 * kT1, I2 = t2 * kT2;
    const int P0 = ch * a.chunk, P1 = min(P0 + a.chunk, c0);
    const int A1 = min(P1, c0 - 1);  // last coarse plane whose prolongation is needed

    // dim-0 weights of the chunk, staged once the first loads are issued
    // (one memory latency then covers both)
    auto stage_tables = [&] {
        if (kAct0)
            for (int e = tid; e < 2 * (2 * (A1 - P0) + 1); e += kThreads) {
                const int f = 2 * P0 + e / 2;
                sW0[e] = (f & 1) ? a.tb.w[0][2 * f + (e & 1)] : T(0);
            }
    };

    // ---- this lane's fine column and the wave's fine rows
    const int c = (wave % G::CW) * 64 + lane;
    const int gc = 2 * I2 + c;
    const bool cin = gc < m2;
    const bool ceven = !(c & 1);
    const int ucl = c >> 1, ucr = (c >> 1) + (c & 1);  // coarse tile columns
    T wcl = T(1), wch = T(0);
    if (cin && (c & 1)) {
        wcl = a.tb.w[2][2 * gc];
        wch = a.tb.w[2][2 * gc + 1];
    }
    const int rg = wave / G::CW;
    const int as1 = (int)a.av.s[1], as2 = (int)a.av.s[2];
    const int cs1 = (int)a.cv.s[1], cs2 = (int)a.cv.s[2];
    const int R0 = kAct1 ? 2 * I1 : 0;
    // byte offsets from the tile's first fine row; coarse positions of even
    // planes (vAe) and everything outside the grid read zero
    unsigned vAe[NRW], vAo[NRW], vC[NRW];
    T wrl[NRW], wrh[NRW];
#pragma unroll
    for (int k = 0; k < NRW; k++) {
        const int r = rg + RW * k, gr = R0 + r;
        const bool in = cin && gr < m1;
        const unsigned oa = (unsigned)((gr - R0) * as1 + gc * as2) * S;
        vAo[k] = in ? oa : kOut;
        vAe[k] = (in && !((r & 1) == 0 && ceven)) ? oa : kOut;
        vC[k] = in ? (unsigned)((gr - R0) * cs1 + gc * cs2) * S : kOut;
        const bool rodd = kAct1 && (r & 1) && gr < m1;
        wrl[k] = rodd ? uni(a.tb.w[1][2 * gr]) : T(1);
        wrh[k] = rodd ? uni(a.tb.w[1][2 * gr + 1]) : T(0);
    }
    const unsigned spanA = (unsigned)((min(R0 + G::FR, m1) - R0 - 1) * as1 + m2 * as2) * S;
    const unsigned spanC = (unsigned)((min(R0 + G::FR, m1) - R0 - 1) * cs1 + m2 * cs2) * S;
    // coarse tile slots: (I1 + idx / CC, I2 + idx % CC)
    const int ws1 = (int)a.wv.s[1], ws2 = (int)a.wv.s[2];
    unsigned vW[NCT];
#pragma unroll
    for (int q = 0; q < NCT; q++) {
        const int idx = tid + q * kThreads;
        const int cr = idx / CC, cc = idx - (idx / CC) * CC;
        const bool in = idx < CR * CC && I1 + cr < c1 && I2 + cc < c2;
        vW[q] = in ? (unsigned)(cr * ws1 + (I2 + cc) * ws2) * S : kOut;
    }
    const unsigned spanW = (unsigned)((min(I1 + CR, c1) - I1 - 1) * ws1 + c2 * ws2) * S;

    const unsigned as0 = (unsigned)a.av.s[0], cs0 = (unsigned)a.cv.s[0], ws0 = (unsigned)a.wv.s[0];
    auto mul64 = [](int i, unsigned st) { return (int64_t)((uint64_t)(unsigned)i * st); };
    const int64_t wrow = (int64_t)I1 * ws1;
    auto load_tile = [&](int ac, T (&w)[NCT], T (&z)[NCT]) {
        const int64_t o = mul64(ac, ws0) + wrow;
        const __amdgpu_buffer_rsrc_t rw = make_rsrc(a.W + o, spanW);
        const __amdgpu_buffer_rsrc_t rz = make_rsrc(a.Z + o, spanW);
#pragma unroll
        for (int q = 0; q < NCT; q++) {
            w[q] = buf_load<T>(rw, vW[q]);
            z[q] = buf_load<T>(rz, vW[q]);
        }
    };
    // fine plane f, clamped into [0, m0), of the coefficients
    auto load_fine = [&](int f, bool even, T (&v)[NRW]) {
        const __amdgpu_buffer_rsrc_t r =
            make_rsrc(a.A + mul64(max(min(f, m0 - 1), 0), as0) + (int64_t)R0 * as1, spanA);
#pragma unroll
        for (int k = 0; k < NRW; k++) v[k] = buf_load<T>(r, even ? vAe[k] : vAo[k]);
    };
    auto store_fine = [&](int f, bool own, const T (&v)[NRW]) {
        const __amdgpu_buffer_rsrc_t r = make_rsrc(a.C + mul64(f, cs0) + (int64_t)R0 * cs1, own ? spanC : 0u);
#pragma unroll
        for (int k = 0; k < NRW; k++) buf_store(v[k], r, vC[k]);
    };

    T pW[NCT], pZ[NCT], fo[NRW], fe[NRW], Qp[NRW], Q[NRW], o[NRW];
    load_tile(P0, pW, pZ);
    load_fine(2 * P0 - 1, false, fo);  // unused for the first plane (read but not emitted)
    load_fine(2 * P0, true, fe);
    stage_tables();
#pragma unroll
    for (int k = 0; k < NRW; k++) Qp[k] = T(0);
    lds_barrier();  // tables

    for (int ac = P0; ac <= A1; ac++) {
        T* sWb = sW[(ac - P0) & 1];
#pragma unroll
        for (int q = 0; q < NCT; q++)
            if (tid + q * kThreads < CR * CC) sWb[tid + q * kThreads] = pW[q] - pZ[q];
        load_tile(min(ac + 1, A1), pW, pZ);
        lds_barrier();
        // 2-D prolongation of the corrected coarse plane at this thread's nodes
#pragma unroll
        for (int k = 0; k < NRW; k++) {
            const int r = rg + RW * k;
            const int cr = r >> 1;
            const T lo = lerp2(wcl, sWb[cr * CC + ucl], wch, sWb[cr * CC + ucr]);
            if (kAct1 && (r & 1)) {
                const T hi = lerp2(wcl, sWb[(cr + 1) * CC + ucl], wch, sWb[(cr + 1) * CC + ucr]);
                Q[k] = lerp2(wrl[k], lo, wrh[k], hi);
            } else {
                Q[k] = lo;
            }
        }
        if (kAct0 && ac > P0) {
            // fine plane 2ac - 1 between Q(ac - 1) and Q(ac)
            const T wl = sW0[2 * (2 * (ac - P0) - 1)], wh = sW0[2 * (2 * (ac - P0) - 1) + 1];
#pragma unroll
            for (int k = 0; k < NRW; k++) o[k] = fo[k] + lerp2(wl, Qp[k], wh, Q[k]);
            store_fine(2 * ac - 1, true, o);
        }
        load_fine(2 * ac + 1, false, fo);
        // fine plane 2ac (coarse positions read 0 from the coefficients)
#pragma unroll
        for (int k = 0; k < NRW; k++) {
            o[k] = fe[k] + Q[k];
            Qp[k] = Q[k];
        }
        store_fine(2 * ac, ac < P1, o);
        load_fine(2 * ac + 2, true, fe);
        // the tile buffer written next is the other one, last read before
        // the barrier above
    }
}

// Recomposition of a 3-D level step with line-aligned output ownership.
// The output rows (2^k + 1 elements) start at arbitrary offsets within the
// 128-byte cache lines; a tile that stores a fixed column range per row
// leaves partly written lines at both of its edges, which costs the HBM
// far more than the whole-line writes of a linear stream.  Here the column
// range a tile owns in a row is aligned to the lines of that row: the
// boundary between tiles t - 1 and t lies at the first line boundary at or
// below column 64 t, so an interior tile owns exactly 64 columns (two FP32
// lines, four FP64 lines) of every row, shifted per row and plane, and each
// line is written by one workgroup.  Lanes map to those memory positions;
// the prolongation is evaluated at each lane's column (weights and coarse
// values from LDS), so the arithmetic per node is that of k_stream_recon.
template <typename T>
struct AlignedRecon {
    static constexpr int kT1 = 8, kT2 = 32;  // nominal tile: coarse rows, columns
    static constexpr int FR = 2 * kT1;       // fine rows
    static constexpr int TW = 2 * kT2;       // nominal fine columns (64 lanes)
    static constexpr int LE = 128 / (int)sizeof(T);  // elements per cache line
    static constexpr int NRW = FR / 4;       // fine rows per wave
    // columns a tile may own: [64 t - (LE - 1), 64 t + 64); coarse tile and
    // column weights cover them
    static constexpr int CO = LE / 2, CR = kT1 + 1, CC = kT2 + CO + 2;
    static constexpr int WO = LE, WC = TW + LE;  // weight table: columns 64 t - LE ..
    static constexpr int NCT = (CR * CC + kThreads - 1) / kThreads;
};

template <typename T, bool kAct0>
__global__ void __launch_bounds__(kThreads) k_stream_recon_al(StreamArgs<T> a)
{
    using G = AlignedRecon<T>;
    constexpr int kT1 = G::kT1, kT2 = G::kT2, TW = G::TW, LE = G::LE, NRW = G::NRW, CO = G::CO, CR = G::CR,
                  CC = G::CC, WO = G::WO, WC = G::WC, NCT = G::NCT;
    constexpr unsigned S = sizeof(T);
    __shared__ T sW[3][CR * CC];   // corrected coarse tiles of planes a - 1, a (three in rotation)
    __shared__ T sW0[2 * (2 * kMaxChunk + 1)];
    __shared__ T sWc[2 * WC];      // column weights (1, 0 at even and outside columns)

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = uni(tid >> 6);
    const int bid = remap_xcd((int)blockIdx.x, (int)gridDim.x);
    const int nt1 = a.nt1, nt2 = a.nt2;
    const int t2 = bid % nt2;
    const int t1 = (bid / nt2) % nt1;
    const int ch = bid / (nt2 * nt1);
    const int m0 = (int)a.av.n[0], m1 = (int)a.av.n[1], m2 = (int)a.av.n[2];
    const int c0 = (int)a.wv.n[0], c1 = (int)a.wv.n[1], c2 = (int)a.wv.n[2];
    const int I1 = t1 * kT1, I2 = t2 * kT2;
    const int P0 = ch * a.chunk, P1 = min(P0 + a.chunk, c0);
    const int A1 = min(P1, c0 - 1);
    const int R0 = 2 * I1, C0 = 2 * I2;
    const bool first = t2 == 0, last = t2 == nt2 - 1;

    // dim-0 and column weights, staged once the first loads are issued
    auto stage_tables = [&] {
        if (kAct0)
            for (int e = tid; e < 2 * (2 * (A1 - P0) + 1); e += kThreads) {
                const int f = 2 * P0 + e / 2;
                sW0[e] = (f & 1) ? a.tb.w[0][2 * f + (e & 1)] : T(0);
            }
        for (int e = tid; e < WC; e += kThreads) {
            const int gc = C0 - WO + e;
            const bool odd = (gc & 1) && gc > 0 && gc < m2;
            sWc[2 * e] = odd ? a.tb.w[2][2 * gc] : T(1);
            sWc[2 * e + 1] = odd ? a.tb.w[2][2 * gc + 1] : T(0);
        }
    };
    const int rg = wave;
    T wrl[NRW], wrh[NRW];
#pragma unroll
    for (int k = 0; k < NRW; k++) {
        const int r = rg + 4 * k, gr = R0 + r;
        const bool rodd = (r & 1) && gr < m1;
        wrl[k] = rodd ? uni(a.tb.w[1][2 * gr]) : T(1);
        wrh[k] = rodd ? uni(a.tb.w[1][2 * gr + 1]) : T(0);
    }

    // coarse tile slots (I1 + cr, I2 - CO + cc)
    const int ws1 = (int)a.wv.s[1], ws2 = (int)a.wv.s[2];
    unsigned vW[NCT];
#pragma unroll
    for (int q = 0; q < NCT; q++) {
        const int idx = tid + q * kThreads;
        const int cr = idx / CC, cc = idx - (idx / CC) * CC;
        const int ci = I2 - CO + cc;
        const bool in = idx < CR * CC && I1 + cr < c1 && ci >= 0 && ci < c2;
        vW[q] = in ? (unsigned)(cr * ws1 + ci * ws2) * S : kOut;
    }
    const unsigned spanW = (unsigned)((min(I1 + CR, c1) - I1 - 1) * ws1 + c2 * ws2) * S;
    const unsigned ws0 = (unsigned)a.wv.s[0];
    auto mul64 = [](int i, unsigned st) { return (int64_t)((uint64_t)(unsigned)i * st); };
    const int64_t wrow = (int64_t)I1 * ws1;
    auto load_tile = [&](int ac, T (&w)[NCT], T (&z)[NCT]) {
        const int64_t o = mul64(ac, ws0) + wrow;
        const __amdgpu_buffer_rsrc_t rw = make_rsrc(a.W + o, spanW);
        const __amdgpu_buffer_rsrc_t rz = make_rsrc(a.Z + o, spanW);
#pragma unroll
        for (int q = 0; q < NCT; q++) {
            w[q] = buf_load<T>(rw, vW[q]);
            z[q] = buf_load<T>(rz, vW[q]);
        }
    };

    // ---- per (plane, row): the lane's fine column, relative to C0
    // Element offset of C's column C0 in row gr of plane f, modulo a line.
    const unsigned cs0 = (unsigned)a.cv.s[0], cs1 = (unsigned)a.cv.s[1];
    const unsigned cbase = (unsigned)(((uintptr_t)a.C / S) & (LE - 1));
    auto col_of = [&](int f, int gr, bool& ok) {
        const int sh = (int)((cbase + (unsigned)f * cs0 + (unsigned)gr * cs1 + (unsigned)C0) & (unsigned)(LE - 1));
        const int olo = first ? 0 : -sh;
        const int ohi = last ? m2 - C0 : TW - sh;
        const int x = olo + lane;
        ok = x < ohi && gr < m1;
        return x;
    };
    const unsigned as0 = (unsigned)a.av.s[0], as1 = (unsigned)a.av.s[1], as2 = (unsigned)a.av.s[2];
    const unsigned spanA = (unsigned)((m1 - 1) * as1 + (m2 - 1) * as2 + 1) * S;
    const unsigned spanC = (unsigned)((m1 - 1) * cs1 + (m2 - 1) + 1) * S;
    // coefficients of fine plane f (clamped into the grid) at this lane's
    // nodes; coarse positions of even planes and columns the tile does not
    // own read zero
    auto load_fine = [&](int f, T (&v)[NRW]) {
        f = max(min(f, m0 - 1), 0);
        const __amdgpu_buffer_rsrc_t r = make_rsrc(a.A + mul64(f, as0), spanA);
#pragma unroll
        for (int k = 0; k < NRW; k++) {
            const int gr = R0 + rg + 4 * k;
            bool ok;
            const int x = col_of(f, gr, ok);
            const int gc = C0 + x;
            const bool coarse = !(f & 1) && !(gr & 1) && !(gc & 1);
            v[k] = buf_load<T>(r, (ok && !coarse) ? (unsigned)gr * as1 * S + (unsigned)gc * as2 * S : kOut);
        }
    };
    // 2-D prolongation of the corrected coarse tile b at (row r, column gc)
    auto prolong = [&](const T* sWb, int k, int gc) {
        const int r = rg + 4 * k, cr = r >> 1;
        const int e = gc - (C0 - WO);
        const T wcl = sWc[2 * e], wch = sWc[2 * e + 1];
        const int ucl = (gc >> 1) - (I2 - CO), ucr = ucl + (gc & 1);
        const T lo = lerp2(wcl, sWb[cr * CC + ucl], wch, sWb[cr * CC + ucr]);
        if (r & 1) {
            const T hi = lerp2(wcl, sWb[(cr + 1) * CC + ucl], wch, sWb[(cr + 1) * CC + ucr]);
            return lerp2(wrl[k], lo, wrh[k], hi);
        }
        return lo;
    };
    auto store_row = [&](const __amdgpu_buffer_rsrc_t& r, int k, int f, T v) {
        const int gr = R0 + rg + 4 * k;
        bool ok;
        const int x = col_of(f, gr, ok);
        // the user's output, in whole lines, read by nothing after
        buf_store_nt(v, r, ok ? ((unsigned)gr * cs1 + (unsigned)(C0 + x)) * S : kOut);
    };

    T pW[NCT], pZ[NCT], fo[NRW], fe[NRW];
    load_tile(P0, pW, pZ);
    load_fine(2 * P0 - 1, fo);  // unused for the first plane (read but not emitted)
    load_fine(2 * P0, fe);
    stage_tables();
    __syncthreads();  // tables

    for (int ac = P0; ac <= A1; ac++) {
        T* sWb = sW[(ac - P0) % 3];
        const T* sWp = sW[(ac - P0 + 2) % 3];  // plane ac - 1
#pragma unroll
        for (int q = 0; q < NCT; q++)
            if (tid + q * kThreads < CR * CC) sWb[tid + q * kThreads] = pW[q] - pZ[q];
        load_tile(min(ac + 1, A1), pW, pZ);
        lds_barrier();
        if (kAct0 && ac > P0) {
            // fine plane 2ac - 1 between the prolongations of ac - 1 and ac
            const int f = 2 * ac - 1;
            const T wl = sW0[2 * (2 * (ac - P0) - 1)], wh = sW0[2 * (2 * (ac - P0) - 1) + 1];
            const __amdgpu_buffer_rsrc_t r = make_rsrc(a.C + mul64(f, cs0), spanC);
#pragma unroll
            for (int k = 0; k < NRW; k++) {
                bool ok;
                const int gc = C0 + col_of(f, R0 + rg + 4 * k, ok);
                store_row(r, k, f, fo[k] + lerp2(wl, prolong(sWp, k, gc), wh, prolong(sWb, k, gc)));
            }
        }
        load_fine(2 * ac + 1, fo);
        {
            // fine plane 2ac (coarse positions read 0 from the coefficients)
            const int f = 2 * ac;
            const __amdgpu_buffer_rsrc_t r = make_rsrc(a.C + mul64(f, cs0), ac < P1 ? spanC : 0u);
#pragma unroll
            for (int k = 0; k < NRW; k++) {
                bool ok;
                const int gc = C0 + col_of(f, R0 + rg + 4 * k, ok);
                store_row(r, k, f, fe[k] + prolong(sWb, k, gc));
            }
        }
        load_fine(2 * ac + 2, fe);
        // tile buffers rotate through three: the one written next was last
        // read before the barrier of the previous plane
    }
}

template <typename T, bool kAct0, bool kAct1>
hipError_t launch_recon_cfg(StreamArgs<T> a, hipStream_t st)
{
    using G = ReconGeom<kAct1>;
    const int c0 = (int)a.wv.n[0], c1 = (int)a.wv.n[1], c2 = (int)a.wv.n[2];
    a.nt1 = kAct1 ? (c1 + G::kT1 - 1) / G::kT1 : 1;
    a.nt2 = (c2 + G::kT2 - 1) / G::kT2;
    const int tiles = a.nt1 * a.nt2;
    auto kern = k_stream_recon<T, kAct0, kAct1>;
    int chunk = c0;
    if (kAct0) {
        static int occ = 0;
        const int slots = resident_per_cu(kern, occ) * device_cu_count();
        const int nch = std::max(1, slots / tiles);
        chunk = (c0 + nch - 1) / nch;
        chunk = std::min(std::max(chunk, 2), kMaxChunk);
    }
    a.chunk = chunk;
    a.nch = kAct0 ? (c0 + chunk - 1) / chunk : 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)(tiles * a.nch)), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_recon_al(StreamArgs<T> a, hipStream_t st)
{
    using G = AlignedRecon<T>;
    const int c0 = (int)a.wv.n[0], c1 = (int)a.wv.n[1];
    const int m2 = (int)a.av.n[2];
    a.nt1 = (c1 + G::kT1 - 1) / G::kT1;
    a.nt2 = (m2 + G::TW - 1) / G::TW;
    const int tiles = a.nt1 * a.nt2;
    // Chunks of at most 8 coarse planes: on large grids that is several
    // rounds of workgroups, and the tiles of a plane region then stream it
    // nearly in step, which keeps the concurrent writes close together in
    // memory (measured: 8 planes per chunk ran 12% faster than one long
    // round); small grids keep the one-round split, whose chunks are shorter.
    static int occ = 0;
    const int slots = resident_per_cu(k_stream_recon_al<T, true>, occ) * device_cu_count();
    const int nch = std::max(1, slots / tiles);
    const int chunk = std::min(std::max((c0 + nch - 1) / nch, 2), 8);
    a.chunk = chunk;
    a.nch = (c0 + chunk - 1) / chunk;
    hipLaunchKernelGGL((k_stream_recon_al<T, true>), dim3((unsigned)(tiles * a.nch)), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

// The line-aligned form takes 3-D grids whose coefficients and output both
// have unit column stride (the finest level step: on coarser steps the
// coefficients are strided and the per-lane kernel measured faster) and rows
// short enough that the last tile of a row owns at most 64 columns
// (m2 = 64 q + 1, or m2 <= 33), with offsets below 2^31 bytes.
template <typename T>
bool recon_al_ok(const StreamArgs<T>& a)
{
    if (a.av.n[0] < 2 || a.av.n[1] < 2 || a.av.s[2] != 1 || a.cv.s[2] != 1 || ((uintptr_t)a.C % sizeof(T)) != 0)
        return false;
    const int64_t m2 = a.av.n[2];
    if (!((m2 - 1) % 64 == 0 || m2 <= 33)) return false;
    const int64_t span = std::max((a.av.n[1] - 1) * a.av.s[1] + (m2 - 1) * a.av.s[2] + 1,
                                  (a.cv.n[1] - 1) * a.cv.s[1] + m2);
    return span * (int64_t)sizeof(T) < ((int64_t)1 << 31);
}

}  // namespace

template <typename T>
hipError_t launch_stream_recon(StreamArgs<T> a, hipStream_t st)
{
    if (recon_al_ok(a)) return launch_recon_al(a, st);
    const bool act0 = a.av.n[0] > 1, act1 = a.av.n[1] > 1;
    if (act0 && act1) return launch_recon_cfg<T, true, true>(a, st);
    if (act0) return launch_recon_cfg<T, true, false>(a, st);
    if (!act1) return launch_recon_cfg<T, false, false>(a, st);
    return hipErrorInvalidValue;
}


template hipError_t launch_stream_recon<float>(StreamArgs<float>, hipStream_t);
template hipError_t launch_stream_recon<double>(StreamArgs<double>, hipStream_t);

}  // namespace mgr
