// Streaming level kernel: one HBM pass per level step computes the
// coefficients (Sec. II-A.1) and the whole load vector f = R M vec(C)
// (Sec. II-A.2, merged mass-transfer stencil of Sec. III-A.2) along all
// dimensions.
//
// Layout of the work.  The level grid is (m0, m1, m2) with m2 contiguous; its
// coarse grid is (c0, c1, c2), c = (m + 1) / 2.  A workgroup owns a tile of
// kT1 x kT2 coarse columns (dims 1, 2) and a chunk of coarse planes along
// dim 0, and streams the fine planes of that chunk (plus a 2-plane halo).
// Each fine plane is staged in LDS with a 2-node halo; its coefficients are
// formed in LDS; the dim-2 and dim-1 stencils reduce it to a kT1 x kT2
// coarse plane; each thread keeps the running sums of the dim-0 stencil for
// its coarse column in registers, so the load vector is written once and
// nothing intermediate goes to HBM.  The next plane's values are loaded into
// registers while the current plane is processed.  Two-dimensional problems
// run as (m0, 1, m2), one-dimensional ones as (1, 1, m2).
//
// Planes are visited in the order e0, e0+2, e0+1, e0+4, e0+3, ... so that an
// odd plane is handled right after both even neighbours, whose 2-D
// interpolants (kept in LDS) it needs.  Interpolation is the separable
// evaluation of the multilinear form from the coarse nodes only.
//
// kDec = true : input u; writes coefficients (and, optionally, u at coarse
//               positions so that level-0 output rows are written whole), the
//               coarse values W and f.
// kDec = false: input already holds coefficients at fine-only nodes (values
//               at coarse positions are ignored); writes f only.
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

constexpr int kMaxChunk = 64;  // coarse planes per workgroup (LDS tables)

template <typename T, bool kAct0, bool kAct1, int kT1, int kT2, bool kDec, bool kZ>
__global__ void __launch_bounds__(kThreads) k_stream_level(StreamArgs<T> a)
{
    static_assert(kT1 * kT2 == kThreads, "one coarse column per thread");
    constexpr int NR = kAct1 ? 2 * kT1 + 3 : 1;
    constexpr int NC = 2 * kT2 + 3;
    constexpr int NS = (NR * NC + kThreads - 1) / kThreads;   // region slots per thread
    constexpr int NG = (NR * kT2 + kThreads - 1) / kThreads;  // dim-2 outputs per thread
    constexpr int NF = kAct0 ? 2 * kMaxChunk + 3 : 1;         // staged fine planes
    __shared__ T sU[NR * NC];
    __shared__ T sP[kDec ? 2 * NR * NC : 1];
    __shared__ T sG[NR * kT2];
    // Every table the plane loop needs lives in LDS: a global load inside the
    // loop would have to wait for the next plane's prefetch (vector memory
    // counters retire in order).
    __shared__ T sWr[2 * NR];        // row interpolation weights (lower, upper)
    __shared__ T sWc[2 * NC];        // column interpolation weights
    __shared__ T sW0[2 * NF];        // plane interpolation weights
    __shared__ T sK2[5 * kT2];       // dim-2 stencil of the tile's coarse columns
    __shared__ T sK1[5 * kT1];       // dim-1 stencil of the tile's coarse rows
    __shared__ T sK0[5 * kMaxChunk]; // dim-0 stencil of the chunk's coarse planes

    const int tid = threadIdx.x;
    const int bid = remap_xcd((int)blockIdx.x, (int)gridDim.x);
    const int nt1 = a.nt1, nt2 = a.nt2;
    const int t2 = bid % nt2;
    const int t1 = (bid / nt2) % nt1;
    const int ch = bid / (nt2 * nt1);

    const int m0 = (int)a.av.n[0], m1 = (int)a.av.n[1], m2 = (int)a.av.n[2];
    const int c0 = (int)a.fv.n[0], c1 = (int)a.fv.n[1], c2 = (int)a.fv.n[2];
    // in-plane strides fit 32 bits (the driver keeps planes below 2^31 nodes)
    const int as1 = (int)a.av.s[1], as2 = (int)a.av.s[2];
    const int cs1 = (int)a.cv.s[1], cs2 = (int)a.cv.s[2];
    const int ws1 = (int)a.wv.s[1], ws2 = (int)a.wv.s[2];
    const int fs1 = (int)a.fv.s[1], fs2 = (int)a.fv.s[2];

    const int I1 = t1 * kT1, I2 = t2 * kT2;
    const int P0 = ch * a.chunk, P1 = min(P0 + a.chunk, c0);
    // staged fine region (starts and ends on even indices)
    const int R0 = kAct1 ? max(2 * I1 - 2, 0) : 0;
    const int R1 = kAct1 ? min(2 * (min(I1 + kT1, c1) - 1) + 2, m1 - 1) : 0;
    const int C0 = max(2 * I2 - 2, 0);
    const int C1 = min(2 * (min(I2 + kT2, c2) - 1) + 2, m2 - 1);
    const int nr = R1 - R0 + 1, nc = C1 - C0 + 1, nrc = nr * nc;
    const int F0 = kAct0 ? max(2 * P0 - 2, 0) : 0;
    const int F1 = kAct0 ? min(2 * (P1 - 1) + 2, m0 - 1) : 0;
    // fine nodes this workgroup writes: rows [oR0, oR1), cols [oC0, oC1), planes [oF0, oF1)
    const int oR0 = kAct1 ? 2 * I1 : 0, oR1 = kAct1 ? min(2 * (I1 + kT1), m1) : 1;
    const int oC0 = 2 * I2, oC1 = min(2 * (I2 + kT2), m2);
    const int oF0 = kAct0 ? 2 * P0 : 0, oF1 = kAct0 ? min(2 * P1, m0) : 1;
    const float inv_nc = 1.0f / (float)nc;

    // ---- tables -> LDS
    if (kDec) {
        const T* __restrict__ w1 = a.tb.w[1];
        const T* __restrict__ w2 = a.tb.w[2];
        for (int r = tid; r < nr; r += kThreads) {
            const int gr = R0 + r;
            sWr[2 * r] = (gr & 1) ? w1[2 * gr] : T(1);
            sWr[2 * r + 1] = (gr & 1) ? w1[2 * gr + 1] : T(0);
        }
        for (int c = tid; c < nc; c += kThreads) {
            const int gc = C0 + c;
            sWc[2 * c] = (gc & 1) ? w2[2 * gc] : T(1);
            sWc[2 * c + 1] = (gc & 1) ? w2[2 * gc + 1] : T(0);
        }
        if (kAct0)
            for (int e = tid; e < 2 * (F1 - F0 + 1); e += kThreads) sW0[e] = a.tb.w[0][2 * F0 + e];
    }
    for (int e = tid; e < 5 * kT2; e += kThreads) sK2[e] = (I2 + e / 5 < c2) ? a.tb.K[2][5 * I2 + e] : T(0);
    if (kAct1)
        for (int e = tid; e < 5 * kT1; e += kThreads) sK1[e] = (I1 + e / 5 < c1) ? a.tb.K[1][5 * I1 + e] : T(0);
    if (kAct0)
        for (int e = tid; e < 5 * (P1 - P0); e += kThreads) sK0[e] = a.tb.K[0][5 * P0 + e];

    // ---- this thread's coarse column of the output tile
    const int g1 = tid / kT2, g2 = tid % kT2;
    const int i1 = I1 + g1, i2 = I2 + g2;
    const bool gvalid = (i1 < c1) && (i2 < c2);
    const int foff = i1 * fs1 + i2 * fs2;
    T acc0 = T(0), acc1 = T(0), acc2 = T(0);

    const int nplanes = F1 - F0 + 1;
    auto plane_of = [=](int j) { return (j == 0) ? F0 : ((j & 1) ? F0 + j + 1 : F0 + j - 1); };
    // slot q of this thread covers region node tid + q * kThreads; idle slots
    // re-load the region's first node so that every load is unconditional
    auto slot_rc = [=](int q, int& r, int& c) {
        const int idx = tid + q * kThreads;
        r = (int)(((float)idx + 0.5f) * inv_nc);
        c = idx - r * nc;
        return idx < nrc;
    };
    int aoff[NS];
#pragma unroll
    for (int q = 0; q < NS; q++) {
        int r, c;
        const bool ok = slot_rc(q, r, c);
        aoff[q] = ok ? (R0 + r) * as1 + (C0 + c) * as2 : R0 * as1 + C0 * as2;
    }

    // kZ: the input level grid is A + Z (coarse values plus the correction
    // of the previous level step, added here instead of in a separate pass)
    T pre[NS], preZ[NS];
    {
        const int64_t po = (int64_t)plane_of(0) * a.av.s[0];
#pragma unroll
        for (int q = 0; q < NS; q++) {
            pre[q] = a.A[po + aoff[q]];
            preZ[q] = kZ ? a.Z[po + aoff[q]] : T(0);
        }
    }

    for (int j = 0; j < nplanes; j++) {
        const int f = plane_of(j);
        const bool even = (f & 1) == 0;
        // stage the prefetched plane, then start loading the next one
#pragma unroll
        for (int q = 0; q < NS; q++) {
            const int idx = tid + q * kThreads;
            if (idx < nrc) {
                int r, c;
                slot_rc(q, r, c);
                sU[r * NC + c] = kZ ? pre[q] + preZ[q] : pre[q];
            }
        }
        if (j + 1 < nplanes) {
            const int64_t po = (int64_t)plane_of(j + 1) * a.av.s[0];
#pragma unroll
            for (int q = 0; q < NS; q++) {
                pre[q] = a.A[po + aoff[q]];
                if (kZ) preZ[q] = a.Z[po + aoff[q]];
            }
        }
        lds_barrier();

        if (kDec) {
            const bool fown = f >= oF0 && f < oF1;
            T* __restrict__ Cp = a.C + (int64_t)f * a.cv.s[0];
            if (even) {
                // 2-D interpolant P from the plane's coarse nodes, kept for the
                // odd neighbours; C = u - P in place at fine positions (other
                // threads read only coarse positions, which stay u).
                T* P = sP + (((f - F0) >> 1) & 1) * (NR * NC);
                T* __restrict__ Wp = a.W + (int64_t)(f >> 1) * a.wv.s[0];
#pragma unroll 1
                for (int idx = tid; idx < nrc; idx += kThreads) {
                    const int r = (int)(((float)idx + 0.5f) * inv_nc), c = idx - r * nc;
                    const int r0 = r - (r & 1), r1 = r + (r & 1);
                    const int cl = c - (c & 1), cr = c + (c & 1);
                    const T wcl = sWc[2 * c], wch = sWc[2 * c + 1];
                    const T lo = wcl * sU[r0 * NC + cl] + wch * sU[r0 * NC + cr];
                    const T hi = wcl * sU[r1 * NC + cl] + wch * sU[r1 * NC + cr];
                    const T p = sWr[2 * r] * lo + sWr[2 * r + 1] * hi;
                    const T u = sU[r * NC + c];
                    P[r * NC + c] = p;
                    const bool coarse = !((r | c) & 1);
                    const T cv = u - p;
                    if (!coarse) sU[r * NC + c] = cv;
                    const int gr = R0 + r, gc = C0 + c;
                    if (fown && gr >= oR0 && gr < oR1 && gc >= oC0 && gc < oC1) {
                        if (!coarse || a.write_coarse) Cp[gr * cs1 + gc * cs2] = coarse ? u : cv;
                        if (coarse) Wp[(gr >> 1) * ws1 + (gc >> 1) * ws2] = u;
                    }
                }
            } else {
                // odd plane: every node is fine; interpolate along dim 0
                // between the 2-D interpolants of the even neighbours
                const T* Pa = sP + (((f - 1 - F0) >> 1) & 1) * (NR * NC);
                const T* Pb = sP + (((f + 1 - F0) >> 1) & 1) * (NR * NC);
                const T wl = sW0[2 * (f - F0)], wh = sW0[2 * (f - F0) + 1];
#pragma unroll 1
                for (int idx = tid; idx < nrc; idx += kThreads) {
                    const int r = (int)(((float)idx + 0.5f) * inv_nc), c = idx - r * nc;
                    const int qq = r * NC + c;
                    const T cv = sU[qq] - (wl * Pa[qq] + wh * Pb[qq]);
                    sU[qq] = cv;
                    const int gr = R0 + r, gc = C0 + c;
                    if (fown && gr >= oR0 && gr < oR1 && gc >= oC0 && gc < oC1) Cp[gr * cs1 + gc * cs2] = cv;
                }
            }
            lds_barrier();
        }

        // dim-2 stencil on every staged row; coarse positions of even planes read 0
#pragma unroll
        for (int q = 0; q < NG; q++) {
            const int idx = tid + q * kThreads;
            if (idx >= nr * kT2) continue;
            const int r = idx / kT2, g = idx % kT2;
            const int ii = I2 + g;
            T s = T(0);
            if (ii < c2) {
                const bool maskrow = even && !(r & 1);
#pragma unroll
                for (int t = -2; t <= 2; t++) {
                    const int gc = 2 * ii + t;
                    if (gc < 0 || gc >= m2) continue;
                    T v = sU[r * NC + gc - C0];
                    if (maskrow && !(t & 1)) v = T(0);
                    s += sK2[5 * g + t + 2] * v;
                }
            }
            sG[r * kT2 + g] = s;
        }
        lds_barrier();

        // dim-1 stencil for this thread's column, then the dim-0 stencil into
        // the running sums of the coarse planes that fine plane f touches
        if (gvalid) {
            T g;
            if (kAct1) {
                g = T(0);
#pragma unroll
                for (int t = -2; t <= 2; t++) {
                    const int gr = 2 * i1 + t;
                    if (gr < 0 || gr >= m1) continue;
                    g += sK1[5 * g1 + t + 2] * sG[(gr - R0) * kT2 + g2];
                }
            } else {
                g = sG[g2];
            }
            if (kAct0) {
                const int ilo = (f - 1) >> 1;  // first coarse plane with |f - 2i| <= 2
#pragma unroll
                for (int r = 0; r < 3; r++) {
                    const int i = ilo + r;
                    const int t = f - 2 * i;
                    if (t < -2 || t > 2 || i < P0 || i >= P1) continue;
                    const T add = sK0[5 * (i - P0) + t + 2] * g;
                    const int qs = i % 3;
                    acc0 += (qs == 0) ? add : T(0);
                    acc1 += (qs == 1) ? add : T(0);
                    acc2 += (qs == 2) ? add : T(0);
                }
                if (!even) {
                    // both neighbours of coarse plane i = (f-1)/2 are done
                    const int i = (f - 1) >> 1;
                    if (i >= P0 && i < P1) {
                        const int qs = i % 3;
                        const T v = (qs == 0) ? acc0 : (qs == 1) ? acc1 : acc2;
                        a.F[(int64_t)i * a.fv.s[0] + foff] = v;
                        acc0 = (qs == 0) ? T(0) : acc0;
                        acc1 = (qs == 1) ? T(0) : acc1;
                        acc2 = (qs == 2) ? T(0) : acc2;
                    }
                }
            } else {
                a.F[foff] = g;
            }
        }
        // sU is rewritten by the next iteration only after this barrier
        lds_barrier();
    }
    if (kAct0 && gvalid && F1 == m0 - 1) {
        // last coarse plane of the grid: its stencil has no right half
        const int i = F1 / 2;
        if (i >= P0 && i < P1) {
            const int qs = i % 3;
            a.F[(int64_t)i * a.fv.s[0] + foff] = (qs == 0) ? acc0 : (qs == 1) ? acc1 : acc2;
        }
    }
}

// Recomposition of one level step (Sec. II-A, the inverse of the above):
// coarse nodes take the corrected coarse values W - Z (Z the correction of
// this level step), fine-only nodes c + Pi (W - Z).
// Same tiling and streaming as k_stream_level, over coarse planes: for each
// coarse plane a the workgroup stages its kT1+1 x kT2+1 coarse tile in LDS,
// every thread forms the 2-D prolongation Q(a) at its NQ fine nodes (kept in
// registers), and emits fine plane 2a-1 (between Q(a-1) and Q(a)) and 2a.
// The next coarse tile and the coefficients of the next two fine planes are
// loaded into registers one step ahead.
template <typename T, bool kAct0, bool kAct1, int kT1, int kT2>
__global__ void __launch_bounds__(kThreads) k_stream_recon(StreamArgs<T> a)
{
    constexpr int FR = kAct1 ? 2 * kT1 : 1;  // fine rows of a tile
    constexpr int FC = 2 * kT2;              // fine cols of a tile
    constexpr int NQ = FR * FC / kThreads;   // fine nodes per thread
    constexpr int CR = kAct1 ? kT1 + 1 : 1;  // staged coarse rows
    constexpr int CC = kT2 + 1;              // staged coarse cols
    constexpr int NW = (CR * CC + kThreads - 1) / kThreads;
    static_assert(FR * FC % kThreads == 0, "whole fine nodes per thread");
    __shared__ T sW[2][CR * CC];
    __shared__ T sWr[2 * FR], sWc[2 * FC];
    __shared__ T sW0[2 * (2 * kMaxChunk + 1)];

    const int tid = threadIdx.x;
    const int bid = remap_xcd((int)blockIdx.x, (int)gridDim.x);
    const int nt1 = a.nt1, nt2 = a.nt2;
    const int t2 = bid % nt2;
    const int t1 = (bid / nt2) % nt1;
    const int ch = bid / (nt2 * nt1);
    // a.av: coefficients (level grid view), a.cv: output view, a.wv: coarse W
    const int m0 = (int)a.av.n[0], m1 = (int)a.av.n[1], m2 = (int)a.av.n[2];
    const int c0 = (int)a.wv.n[0], c1 = (int)a.wv.n[1], c2 = (int)a.wv.n[2];
    const int as1 = (int)a.av.s[1], as2 = (int)a.av.s[2];
    const int cs1 = (int)a.cv.s[1], cs2 = (int)a.cv.s[2];
    const int ws1 = (int)a.wv.s[1], ws2 = (int)a.wv.s[2];

    const int I1 = t1 * kT1, I2 = t2 * kT2;
    const int P0 = ch * a.chunk, P1 = min(P0 + a.chunk, c0);
    const int A1 = min(P1, c0 - 1);  // last coarse plane whose prolongation is needed
    const int ncr = min(CR, c1 - I1), ncc = min(CC, c2 - I2);

    // interpolation weights of the tile's fine rows, columns and planes
    for (int e = tid; e < FR; e += kThreads) {
        const int gr = kAct1 ? 2 * I1 + e : 0;
        const bool odd = gr & 1, ok = gr < m1;
        sWr[2 * e] = (odd && ok) ? a.tb.w[1][2 * gr] : T(1);
        sWr[2 * e + 1] = (odd && ok) ? a.tb.w[1][2 * gr + 1] : T(0);
    }
    for (int e = tid; e < FC; e += kThreads) {
        const int gc = 2 * I2 + e;
        const bool odd = gc & 1, ok = gc < m2;
        sWc[2 * e] = (odd && ok) ? a.tb.w[2][2 * gc] : T(1);
        sWc[2 * e + 1] = (odd && ok) ? a.tb.w[2][2 * gc + 1] : T(0);
    }
    if (kAct0)
        for (int e = tid; e < 2 * (2 * (A1 - P0) + 1); e += kThreads) {
            const int f = 2 * P0 + e / 2;
            sW0[e] = (f & 1) ? a.tb.w[0][2 * f + (e & 1)] : T(0);
        }

    // this thread's fine nodes (idx = tid + q * kThreads; FC is a power of 2)
    int woff[NW];
#pragma unroll
    for (int q = 0; q < NW; q++) {
        const int idx = tid + q * kThreads;
        const int r = idx / CC, c = idx - (idx / CC) * CC;
        woff[q] = (idx < ncr * CC && c < ncc) ? (I1 + r) * ws1 + (I2 + c) * ws2 : I1 * ws1 + I2 * ws2;
    }
    int coff[NQ], ooff[NQ];
    bool fok[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        const int idx = tid + q * kThreads;
        const int fr = idx / FC, fc = idx % FC;
        const int gr = kAct1 ? 2 * I1 + fr : 0, gc = 2 * I2 + fc;
        fok[q] = gr < m1 && gc < m2;
        coff[q] = fok[q] ? gr * as1 + gc * as2 : 0;
        ooff[q] = fok[q] ? gr * cs1 + gc * cs2 : 0;
    }
    const T* const Abase = a.A;
    const int64_t as0 = a.av.s[0];
    auto planeA = [=](int f) { return Abase + (int64_t)f * as0; };

    // coarse values of this level step: W minus the correction Z (same layout)
    T preW[NW], preZ[NW], preC0[NQ], preC1[NQ];
    {
        const int64_t wo = (int64_t)P0 * a.wv.s[0];
#pragma unroll
        for (int q = 0; q < NW; q++) {
            preW[q] = a.W[wo + woff[q]];
            preZ[q] = a.Z[wo + woff[q]];
        }
        // coefficients of fine planes 2P0 - 1 (if it belongs to us: never,
        // plane 2P0-1 is the previous chunk's) and 2P0
        const T* cb = planeA(2 * P0);
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            preC0[q] = T(0);
            preC1[q] = cb[coff[q]];
        }
    }
    T Qprev[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) Qprev[q] = T(0);

    for (int ac = P0; ac <= A1; ac++) {
        const int buf = (ac - P0) & 1;
        T* sWb = sW[buf];
#pragma unroll
        for (int q = 0; q < NW; q++) {
            const int idx = tid + q * kThreads;
            if (idx < CR * CC) sWb[idx] = preW[q] - preZ[q];
        }
        T cOdd[NQ], cEven[NQ];
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            cOdd[q] = preC0[q];
            cEven[q] = preC1[q];
        }
        if (ac + 1 <= A1) {
            const int64_t wo = (int64_t)(ac + 1) * a.wv.s[0];
#pragma unroll
            for (int q = 0; q < NW; q++) {
                preW[q] = a.W[wo + woff[q]];
                preZ[q] = a.Z[wo + woff[q]];
            }
            const T* co = planeA(2 * ac + 1);
            const T* ce = planeA(min(2 * ac + 2, m0 - 1));
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                preC0[q] = co[coff[q]];
                preC1[q] = ce[coff[q]];
            }
        }
        lds_barrier();
        const bool emit_odd = kAct0 && ac > P0;
        const bool emit_even = ac < P1;
        const T wl0 = emit_odd ? sW0[2 * (2 * (ac - P0) - 1)] : T(0);
        const T wh0 = emit_odd ? sW0[2 * (2 * (ac - P0) - 1) + 1] : T(0);
        T* Oodd = a.C + (int64_t)(2 * ac - 1) * a.cv.s[0];
        T* Oeven = a.C + (int64_t)(2 * ac) * a.cv.s[0];
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            const int idx = tid + q * kThreads;
            const int fr = idx / FC, fc = idx % FC;
            const int rl = fr >> 1, rh = rl + (fr & 1);
            const int cl = fc >> 1, chh = cl + (fc & 1);
            const T wcl = sWc[2 * fc], wch = sWc[2 * fc + 1];
            T Q = T(0);
            if (fok[q]) {
                const T lo = wcl * sWb[rl * CC + cl] + wch * sWb[rl * CC + chh];
                const T hi = (fr & 1) ? wcl * sWb[rh * CC + cl] + wch * sWb[rh * CC + chh] : T(0);
                Q = sWr[2 * fr] * lo + sWr[2 * fr + 1] * hi;
                if (emit_odd) Oodd[ooff[q]] = cOdd[q] + (wl0 * Qprev[q] + wh0 * Q);
                const bool fine = (fr | fc) & 1;
                if (emit_even) Oeven[ooff[q]] = fine ? cEven[q] + Q : Q;
            }
            Qprev[q] = Q;
        }
        // the buffer staged next step is the other one; it was last read two
        // steps ago, before the barrier above
    }
}

template <typename T, bool kAct0, bool kAct1, int kT1, int kT2>
hipError_t launch_cfg(StreamArgs<T> a, bool dec, hipStream_t st)
{
    const int c0 = (int)a.fv.n[0], c1 = (int)a.fv.n[1], c2 = (int)a.fv.n[2];
    a.nt1 = kAct1 ? (c1 + kT1 - 1) / kT1 : 1;
    a.nt2 = (c2 + kT2 - 1) / kT2;
    const int tiles = a.nt1 * a.nt2;
    int chunk = c0;
    if (kAct0) {
        // enough workgroups to fill 256 CUs several times over, but at least
        // 8 coarse planes per chunk to keep the 2-plane halo cheap
        const int want = 2048;
        const int nch = (want + tiles - 1) / tiles;
        chunk = (c0 + nch - 1) / nch;
        if (chunk < 2) chunk = 2;
        if (chunk > kMaxChunk) chunk = kMaxChunk;
    }
    a.chunk = chunk;
    a.nch = kAct0 ? (c0 + chunk - 1) / chunk : 1;
    const unsigned grid = (unsigned)(tiles * a.nch);
    if (dec && a.Z)
        hipLaunchKernelGGL((k_stream_level<T, kAct0, kAct1, kT1, kT2, true, true>), dim3(grid), dim3(kThreads), 0, st, a);
    else if (dec)
        hipLaunchKernelGGL((k_stream_level<T, kAct0, kAct1, kT1, kT2, true, false>), dim3(grid), dim3(kThreads), 0, st, a);
    else
        hipLaunchKernelGGL((k_stream_level<T, kAct0, kAct1, kT1, kT2, false, false>), dim3(grid), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

template <typename T, bool kAct0, bool kAct1, int kT1, int kT2>
hipError_t launch_recon_cfg(StreamArgs<T> a, hipStream_t st)
{
    const int c0 = (int)a.wv.n[0], c1 = (int)a.wv.n[1], c2 = (int)a.wv.n[2];
    a.nt1 = kAct1 ? (c1 + kT1 - 1) / kT1 : 1;
    a.nt2 = (c2 + kT2 - 1) / kT2;
    const int tiles = a.nt1 * a.nt2;
    int chunk = c0;
    if (kAct0) {
        const int nch = (2048 + tiles - 1) / tiles;
        chunk = (c0 + nch - 1) / nch;
        if (chunk < 2) chunk = 2;
        if (chunk > kMaxChunk) chunk = kMaxChunk;
    }
    a.chunk = chunk;
    a.nch = kAct0 ? (c0 + chunk - 1) / chunk : 1;
    hipLaunchKernelGGL((k_stream_recon<T, kAct0, kAct1, kT1, kT2>), dim3((unsigned)(tiles * a.nch)),
                       dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace

// Recomposition interpolation of one level step: a.A/av = coefficients
// (level grid view), a.C/cv = output view, a.W/wv = corrected coarse values.
template <typename T>
hipError_t launch_stream_recon(StreamArgs<T> a, hipStream_t st)
{
    const bool act0 = a.av.n[0] > 1, act1 = a.av.n[1] > 1;
    if (act0 && act1) return launch_recon_cfg<T, true, true, 8, 32>(a, st);
    if (act0) return launch_recon_cfg<T, true, false, 1, 256>(a, st);
    if (!act1) return launch_recon_cfg<T, false, false, 1, 256>(a, st);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_stream_level(StreamArgs<T> a, bool dec, hipStream_t st)
{
    const bool act0 = a.av.n[0] > 1, act1 = a.av.n[1] > 1;
    if (act0 && act1) return launch_cfg<T, true, true, 8, 32>(a, dec, st);
    if (act0) return launch_cfg<T, true, false, 1, 256>(a, dec, st);
    if (!act1) return launch_cfg<T, false, false, 1, 256>(a, dec, st);
    return hipErrorInvalidValue;  // (1, m1, m2) is never formed by the driver
}

template hipError_t launch_stream_level<float>(StreamArgs<float>, bool, hipStream_t);
template hipError_t launch_stream_recon<float>(StreamArgs<float>, hipStream_t);
template hipError_t launch_stream_recon<double>(StreamArgs<double>, hipStream_t);
template hipError_t launch_stream_level<double>(StreamArgs<double>, bool, hipStream_t);

}  // namespace mgr
