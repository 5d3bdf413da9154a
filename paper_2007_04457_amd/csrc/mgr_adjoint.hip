// Streaming adjoint level step (the transpose of one decomposition level
// step, derived from Eq. 1-2; not in the paper).  With y = M_c^{-1} G (the
// correction solves, done before this kernel) the level-grid output is
//   O(p) = g(p) + t(p)                 at fine-only nodes p,
//   O(q) = G(q) - sum_p w(p, q) O(p)   at coarse nodes q,
// where t = (K0^T x K1^T x K2^T) y expands the coarse y with the transposed
// load-vector stencils (5 fine nodes per coarse node and dimension) and the
// sum gathers the fine neighbours with the interpolation weights: the
// transposed interpolation, separable as a 3-point restriction per
// dimension applied to O with zeros at coarse nodes.
//
// A workgroup owns a tile of 31 coarse columns x 7 coarse rows (2-D and 1-D
// problems: 127 coarse columns in one row) and a chunk of coarse planes.  It
// computes O on 63 fine columns x 15 fine rows (255 columns), offset by one
// fine node so that every coarse node it owns has its fine neighbours inside
// the tile, and streams the fine planes 2P0-1 .. 2P1-1 of its chunk in
// order.  Per coarse plane b it stages the coarse tile of y in LDS and forms
// the 2-D expansion X_b at its fine nodes (registers; the last three planes
// are kept); fine plane f then combines the X of the coarse planes within
// two nodes.  The restriction of each fine plane goes through LDS along
// columns and rows and into one running sum per coarse column along planes,
// which is complete after the plane above the coarse plane.
#include "mgr_stream_dev.h"

namespace mgr {
namespace {

template <bool kAct1>
struct AdjGeom {
    static constexpr int OT1 = kAct1 ? 7 : 1;     // coarse rows owned per tile
    static constexpr int OT2 = kAct1 ? 31 : 127;  // coarse columns owned per tile
    static constexpr int RU = kAct1 ? 2 * OT1 + 1 : 1;  // fine rows computed
    static constexpr int LC = 2 * OT2 + 1;        // fine columns computed
    static constexpr int CW = kAct1 ? 1 : 4;      // waves per fine row
    static constexpr int RW = 4 / CW;             // rows handled at once
    static constexpr int NRW = (RU + RW - 1) / RW;
    static constexpr int NR = NRW * RW;           // fine row slots
    static constexpr int NCW = 64 * CW;           // fine column slots
    static constexpr int CR = kAct1 ? OT1 + 2 : 1;  // staged coarse rows
    static constexpr int CC = OT2 + 2;            // staged coarse columns
    static constexpr int GW = kAct1 ? 32 : 128;   // restriction outputs per row pass
    static_assert(LC <= NCW && OT2 <= GW, "tile fits");
};

template <typename T>
struct AdjArgs {
    const T* g;  // input at the fine nodes of the level grid
    View3 gv;
    const T* y;  // solved corrections, packed coarse grid
    const T* G;  // coarse-node input, packed coarse grid (same layout as y)
    View3 yv;
    T* O;        // output, level grid
    View3 ov;
    DimTables<T> tb;
    int chunk, nt1, nt2, nch;
};

template <typename T, bool kAct0, bool kAct1>
__global__ void __launch_bounds__(kThreads) k_stream_adjoint(AdjArgs<T> a)
{
    using G = AdjGeom<kAct1>;
    constexpr int OT1 = G::OT1, OT2 = G::OT2, RU = G::RU, LC = G::LC, RW = G::RW, NRW = G::NRW, NR = G::NR;
    constexpr int NCW = G::NCW, CR = G::CR, CC = G::CC, GW = G::GW;
    constexpr unsigned S = sizeof(T);
    __shared__ T sY[CR * CC];
    __shared__ T sXc[CR * NCW];
    __shared__ T sO[NR * NCW];
    __shared__ T sS2[NR * GW];
    __shared__ T sK0[5 * (kMaxChunk + 2)];      // coarse planes P0-1 .. P1
    __shared__ T sW0[2 * (2 * kMaxChunk + 1)];  // fine planes 2P0-1 .. 2P1-1

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = uni(tid >> 6);
    const int bid = remap_xcd((int)blockIdx.x, (int)gridDim.x);
    const int nt1 = a.nt1, nt2 = a.nt2;
    const int t2 = bid % nt2;
    const int t1 = (bid / nt2) % nt1;
    const int ch = bid / (nt2 * nt1);

    const int m0 = (int)a.ov.n[0], m1 = (int)a.ov.n[1], m2 = (int)a.ov.n[2];
    const int c0 = (int)a.yv.n[0], c1 = (int)a.yv.n[1], c2 = (int)a.yv.n[2];
    const int J1 = t1 * OT1, J2 = t2 * OT2;  // first owned coarse row / column
    const int Y0 = kAct1 ? 2 * J1 - 1 : 0;   // first computed fine row
    const int X0 = 2 * J2 - 1;               // first computed fine column
    const int P0 = ch * a.chunk, P1 = min(P0 + a.chunk, c0);

    // plane tables: K0 rows of coarse planes P0-1 .. P1, w0 pairs of fine
    // planes 2P0-1 .. 2P1-1 (zero outside the grid)
    if (kAct0) {
        for (int e = tid; e < 5 * (P1 - P0 + 2); e += kThreads) {
            const int i = P0 - 1 + e / 5;
            sK0[e] = (i >= 0 && i < c0) ? a.tb.K[0][5 * i + e % 5] : T(0);
        }
        for (int e = tid; e < 2 * (2 * (P1 - P0) + 1); e += kThreads) {
            const int f = 2 * P0 - 1 + e / 2;
            sW0[e] = (f >= 0 && f < m0 && (f & 1)) ? a.tb.w[0][2 * f + (e & 1)] : T(0);
        }
    }

    // ---- this lane's fine column: expansion along dim 2 from the staged
    // coarse columns (uc: tile column of coarse column m = gc >> 1)
    const int c = (wave % G::CW) * 64 + lane;
    const int gc = X0 + c;
    const bool cin = c < LC && gc >= 0 && gc < m2;
    int xa = 0, xb = 0, xc = 0;
    T ka = T(0), kb = T(0), kc = T(0);
    if (cin) {
        const int m = gc >> 1, uc = m - (J2 - 1);
        const T* K2 = a.tb.K[2];
        if (gc & 1) {
            xa = uc;
            xb = uc + 1;
            xc = uc + 1;
            ka = K2[5 * m + 3];
            kb = (m + 1 < c2) ? K2[5 * (m + 1) + 1] : T(0);
        } else {
            xa = max(uc - 1, 0);
            xb = uc;
            xc = min(uc + 1, CC - 1);
            ka = (m >= 1) ? K2[5 * (m - 1) + 4] : T(0);
            kb = K2[5 * m + 2];
            kc = (m + 1 < c2) ? K2[5 * (m + 1)] : T(0);
        }
    }
    // ---- this wave's fine rows r = rg + RW * k (wave-uniform), expansion
    // along dim 1 from the tile's coarse rows
    const int rg = wave / G::CW;
    int ra[NRW], rb[NRW], rc[NRW];
    T qa[NRW], qb[NRW], qc[NRW];
    unsigned vg[NRW], vo[NRW];  // input and output offsets from the tile's first row
    const int as1 = (int)a.gv.s[1], as2 = (int)a.gv.s[2];
    const int os1 = (int)a.ov.s[1], os2 = (int)a.ov.s[2];
    const int RB = max(Y0, 0);
    const bool cown = cin && c < 2 * OT2;
#pragma unroll
    for (int k = 0; k < NRW; k++) {
        const int r = rg + RW * k, gr = Y0 + r;
        const bool rin = r < RU && gr >= 0 && gr < m1;
        const bool rown = rin && (!kAct1 || r < 2 * OT1);
        ra[k] = rb[k] = rc[k] = 0;
        qa[k] = qb[k] = qc[k] = T(0);
        if (kAct1 && rin) {
            const int m = gr >> 1, ur = m - (J1 - 1);
            const T* K1 = a.tb.K[1];
            if (gr & 1) {
                ra[k] = ur;
                rb[k] = ur + 1;
                rc[k] = ur + 1;
                qa[k] = uni(K1[5 * m + 3]);
                qb[k] = (m + 1 < c1) ? uni(K1[5 * (m + 1) + 1]) : T(0);
            } else {
                ra[k] = max(ur - 1, 0);
                rb[k] = ur;
                rc[k] = min(ur + 1, CR - 1);
                qa[k] = (m >= 1) ? uni(K1[5 * (m - 1) + 4]) : T(0);
                qb[k] = uni(K1[5 * m + 2]);
                qc[k] = (m + 1 < c1) ? uni(K1[5 * (m + 1)]) : T(0);
            }
        } else if (!kAct1) {
            qb[k] = T(1);
        }
        vg[k] = (rin && cin) ? (unsigned)((gr - RB) * as1 + gc * as2) * S : kOut;
        vo[k] = (rown && cown) ? (unsigned)((gr - RB) * os1 + gc * os2) * S : kOut;
    }
    // coarse-position masks of even planes: even fine row and column
    const bool codd = gc & 1;

    // ---- restriction outputs: coarse row J1 + h1, column J2 + h2
    const int h2 = tid % GW, h1 = tid / GW;
    const bool hvalid = h1 < OT1 && h2 < OT2 && J1 + h1 < c1 && J2 + h2 < c2;
    T wl2 = T(0), wr2 = T(0), wl1 = T(0), wr1 = T(0);
    {
        const int q2 = 2 * (J2 + h2);
        if (h2 < OT2 && q2 < m2) {
            wl2 = (q2 - 1 >= 0) ? a.tb.w[2][2 * (q2 - 1) + 1] : T(0);
            wr2 = (q2 + 1 < m2) ? a.tb.w[2][2 * (q2 + 1)] : T(0);
        }
        const int q1 = 2 * (J1 + h1);
        if (kAct1 && h1 < OT1 && q1 < m1) {
            wl1 = (q1 - 1 >= 0) ? a.tb.w[1][2 * (q1 - 1) + 1] : T(0);
            wr1 = (q1 + 1 < m1) ? a.tb.w[1][2 * (q1 + 1)] : T(0);
        }
    }
    const int ys1 = (int)a.yv.s[1], ys2 = (int)a.yv.s[2];
    const unsigned vG = hvalid ? (unsigned)((J1 + h1) * ys1 + (J2 + h2) * ys2) * S : kOut;
    const unsigned vOc = hvalid ? (unsigned)(2 * (J1 + h1) * os1 + 2 * (J2 + h2) * os2) * S : kOut;
    const unsigned spanY = (unsigned)((c1 - 1) * ys1 + c2 * ys2) * S;
    const unsigned spanOc = (unsigned)((m1 - 1) * os1 + m2 * os2) * S;

    // coarse tile of y: coarse (J1 - 1 + idx / CC, J2 - 1 + idx % CC)
    constexpr int NYS = (CR * CC + kThreads - 1) / kThreads;
    unsigned vy[NYS];
#pragma unroll
    for (int q = 0; q < NYS; q++) {
        const int idx = tid + q * kThreads;
        const int cr = idx / CC, cc = idx - (idx / CC) * CC;
        const int yr = kAct1 ? J1 - 1 + cr : 0, yc = J2 - 1 + cc;
        const bool in = idx < CR * CC && yr >= 0 && yr < c1 && yc >= 0 && yc < c2;
        vy[q] = in ? (unsigned)(yr * ys1 + yc * ys2) * S : kOut;
    }

    const unsigned gs0 = (unsigned)a.gv.s[0], os0 = (unsigned)a.ov.s[0], ys0 = (unsigned)a.yv.s[0];
    auto mul64 = [](int i, unsigned st) { return (int64_t)((uint64_t)(unsigned)i * st); };
    const unsigned spanG = (unsigned)((min(Y0 + RU, m1) - RB - 1) * as1 + m2 * as2) * S;
    const unsigned spanO = (unsigned)((min(Y0 + RU, m1) - RB - 1) * os1 + m2 * os2) * S;

    T Xm2[NRW], Xm1[NRW], Xb[NRW], gf[NRW];
#pragma unroll
    for (int k = 0; k < NRW; k++) Xm2[k] = Xm1[k] = Xb[k] = T(0);
    T acc = T(0);
    lds_barrier();  // tables

    const int bfirst = kAct0 ? P0 - 1 : 0, blast = kAct0 ? P1 : 0;
    for (int b = bfirst; b <= blast; b++) {
        // stage the coarse tile of y in plane b (zeros outside the grid)
        {
            const bool bin = b >= 0 && b < c0;
            const __amdgpu_buffer_rsrc_t r = make_rsrc(a.y + mul64(bin ? b : 0, ys0), bin ? spanY : 0u);
#pragma unroll
            for (int q = 0; q < NYS; q++)
                if (tid + q * kThreads < CR * CC) sY[tid + q * kThreads] = buf_load<T>(r, vy[q]);
        }
        lds_barrier();
        // expansion along dim 2 of every staged coarse row
#pragma unroll
        for (int j = 0; j < (CR + RW - 1) / RW; j++) {
            const int ur = rg + RW * j;
            if (ur < CR)
                sXc[ur * NCW + c] = ka * sY[ur * CC + xa] + kb * sY[ur * CC + xb] + kc * sY[ur * CC + xc];
        }
        lds_barrier();
        // along dim 1: X_b at this thread's fine nodes
#pragma unroll
        for (int k = 0; k < NRW; k++) {
            Xm2[k] = Xm1[k];
            Xm1[k] = Xb[k];
            Xb[k] = qa[k] * sXc[ra[k] * NCW + c] + qb[k] * sXc[rb[k] * NCW + c] + qc[k] * sXc[rc[k] * NCW + c];
        }
        // fine planes 2b - 2 (even) and 2b - 1 (odd), those of this chunk
#pragma unroll
        for (int par = 0; par < 2; par++) {
            const int f = kAct0 ? 2 * b - 2 + par : 0;
            const bool even = kAct0 ? par == 0 : true;
            if (kAct0 && (f < 2 * P0 - 1 || f > 2 * P1 - 1)) continue;
            const bool fin = f >= 0 && f < m0;
            const bool fown = fin && f < 2 * P1 - 1;
            // transposed stencil along dim 0
            T wA = T(0), wB = T(0), wC = T(0);
            if (kAct0) {
                const T* k0 = sK0 + 5 * (b - (P0 - 1));  // row of coarse plane b
                if (even) {
                    wA = (b - 2 >= P0 - 1) ? k0[-10 + 4] : T(0);
                    wB = k0[-5 + 2];
                    wC = k0[0];
                } else {
                    wB = k0[-5 + 3];
                    wC = k0[1];
                }
            } else {
                wC = T(1);
            }
            const __amdgpu_buffer_rsrc_t rg_ = make_rsrc(a.g + mul64(fin ? f : 0, gs0) + (int64_t)RB * as1,
                                                         fin ? spanG : 0u);
#pragma unroll
            for (int k = 0; k < NRW; k++) gf[k] = buf_load<T>(rg_, vg[k]);
            const __amdgpu_buffer_rsrc_t ro = make_rsrc(a.O + mul64(fin ? f : 0, os0) + (int64_t)RB * os1,
                                                        fown ? spanO : 0u);
#pragma unroll
            for (int k = 0; k < NRW; k++) {
                const int r = rg + RW * k, gr = Y0 + r;
                const T t = wA * Xm2[k] + wB * Xm1[k] + wC * Xb[k];
                const bool coarse = even && !(gr & 1) && !codd;
                const T o = (fin && !coarse) ? gf[k] + t : T(0);
                if (!coarse) buf_store(o, ro, vo[k]);
                if (r < NR) sO[r * NCW + c] = (cin && r < RU) ? o : T(0);
            }
            lds_barrier();
            // restriction along dim 2 at the tile's coarse columns
#pragma unroll
            for (int ps = 0; ps < (RU + (kThreads / GW) - 1) / (kThreads / GW); ps++) {
                const int r = h1 + ps * (kThreads / GW);
                if (r < RU && h2 < OT2) {
                    const T* o = sO + r * NCW + 2 * h2 + 1;
                    sS2[r * GW + h2] = o[0] + wl2 * o[-1] + wr2 * o[1];
                }
            }
            lds_barrier();
            // along dim 1, then the running sum along dim 0
            T s1 = T(0);
            if (h1 < OT1 && h2 < OT2) {
                if (kAct1) {
                    const T* s = sS2 + (2 * h1 + 1) * GW + h2;
                    s1 = s[0] + wl1 * s[-GW] + wr1 * s[GW];
                } else {
                    s1 = sS2[h2];
                }
            }
            if (kAct0) {
                const int e = 2 * (f - (2 * P0 - 1));
                if (even) {
                    acc += s1;
                } else {
                    // f = 2a + 1 completes coarse plane a and starts a + 1
                    acc += sW0[e] * s1;
                    const int ac = (f - 1) >> 1;
                    if (ac >= P0 && ac < P1) {
                        const __amdgpu_buffer_rsrc_t rG = make_rsrc(a.G + mul64(ac, ys0), spanY);
                        const __amdgpu_buffer_rsrc_t rC = make_rsrc(a.O + mul64(2 * ac, os0), spanOc);
                        buf_store(buf_load<T>(rG, vG) - acc, rC, vOc);
                    }
                    acc = sW0[e + 1] * s1;
                }
            } else {
                const __amdgpu_buffer_rsrc_t rG = make_rsrc(a.G, spanY);
                const __amdgpu_buffer_rsrc_t rC = make_rsrc(a.O, spanOc);
                buf_store(buf_load<T>(rG, vG) - s1, rC, vOc);
            }
        }
    }
}

template <typename T, bool kAct0, bool kAct1>
hipError_t launch_adj_cfg(AdjArgs<T> a, hipStream_t st)
{
    using G = AdjGeom<kAct1>;
    const int c0 = (int)a.yv.n[0], c1 = (int)a.yv.n[1], c2 = (int)a.yv.n[2];
    a.nt1 = kAct1 ? (c1 + G::OT1 - 1) / G::OT1 : 1;
    a.nt2 = (c2 + G::OT2 - 1) / G::OT2;
    const int tiles = a.nt1 * a.nt2;
    auto kern = k_stream_adjoint<T, kAct0, kAct1>;
    int chunk = c0;
    if (kAct0) {
        static int occ = 0;
        const int nch = std::max(1, resident_per_cu(kern, occ) * device_cu_count() / tiles);
        chunk = (c0 + nch - 1) / nch;
        chunk = std::min(std::max(chunk, 1), kMaxChunk);
    }
    a.chunk = chunk;
    a.nch = kAct0 ? (c0 + chunk - 1) / chunk : 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)(tiles * a.nch)), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace

// One adjoint level step: g / gv the input at the level grid's fine nodes, y
// the solved corrections and G the coarse-node input (packed coarse grid
// yv), O / ov the level-grid output.  O must not overlap g.
template <typename T>
hipError_t launch_stream_adjoint(const T* g, View3 gv, const T* y, const T* G, View3 yv, T* O, View3 ov,
                                 DimTables<T> tb, hipStream_t st)
{
    AdjArgs<T> a;
    a.g = g;
    a.gv = gv;
    a.y = y;
    a.G = G;
    a.yv = yv;
    a.O = O;
    a.ov = ov;
    a.tb = tb;
    a.chunk = a.nt1 = a.nt2 = a.nch = 0;
    const bool act0 = ov.n[0] > 1, act1 = ov.n[1] > 1;
    if (act0 && act1) return launch_adj_cfg<T, true, true>(a, st);
    if (act0) return launch_adj_cfg<T, true, false>(a, st);
    if (!act1) return launch_adj_cfg<T, false, false>(a, st);
    return hipErrorInvalidValue;
}

template hipError_t launch_stream_adjoint<float>(const float*, View3, const float*, const float*, View3, float*,
                                                 View3, DimTables<float>, hipStream_t);
template hipError_t launch_stream_adjoint<double>(const double*, View3, const double*, const double*, View3,
                                                  double*, View3, DimTables<double>, hipStream_t);

}  // namespace mgr
