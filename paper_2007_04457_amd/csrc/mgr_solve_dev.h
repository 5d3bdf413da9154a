// Device code of the partitioned Thomas solve (see mgr_solve.hip for the
// method): shared by the per-level kernels and the batched work-queue
// kernel.  Internal; included by .hip files only.
#pragma once
#include "mgr_internal.h"

namespace mgr {
namespace {

constexpr int kBlk = 256;
constexpr int kMaxSegWG = 16;  // strided single-launch form: S <= 16

struct FibreMap {
    int64_t n, inner, outer, nfib;
    int S;
};

// Interior [lo, lo + len) of segment s.
__device__ __forceinline__ void seg_range(const FibreMap& m, int s, int& lo, int& len)
{
    lo = s * kSeg + (s > 0 ? 1 : 0);
    const int hi = (s == m.S - 1) ? (int)m.n : (s + 1) * kSeg;
    len = hi - lo;
}

// Segment-local Thomas solve in registers with padded tables (L = forward
// multipliers, U = super-diagonal, IP = inverse pivots; zero past the
// segment so padded slots come out as 0).
// Returns y at the segment's last node (slot len - 1); it is picked up during
// the backward sweep, as the first nonzero-pivot slot from the end, so that
// the compiler never indexes the register array with a runtime value.
template <typename T>
__device__ __forceinline__ T seg_solve(T (&v)[kSlot], const T* L, const T* U, const T* IP)
{
#pragma unroll
    for (int q = 1; q < kSlot; q++) v[q] -= L[q] * v[q - 1];
    T z = T(0), last = T(0);
    bool found = false;
#pragma unroll
    for (int q = kSlot - 1; q >= 0; q--) {
        const T ip = IP[q];
        z = (v[q] - U[q] * z) * ip;
        v[q] = z;
        const bool here = !found && ip != T(0);
        last = here ? z : last;
        found = found || here;
    }
    return last;
}

// Separator elimination and the segments' final values with one fixed
// rounding (explicit FMAs), shared by every solve form so that they all give
// the same values: right-hand side of separator k from f there and the
// neighbouring segments' end values, its forward elimination, its back
// substitution, and z = y + alpha z_left + beta z_right in a segment.
template <typename T>
__device__ __forceinline__ T sep_rhs(T f, T sub, T ylast, T sup, T yfirst)
{
    return fma(-sup, yfirst, fma(-sub, ylast, f));
}
template <typename T>
__device__ __forceinline__ T sep_fwd(T rhs, T l, T g)
{
    return fma(-l, g, rhs);
}
template <typename T>
__device__ __forceinline__ T sep_bwd(T f, T u, T z, T ip)
{
    return fma(-u, z, f) * ip;
}
template <typename T>
__device__ __forceinline__ T seg_final(T y, T alpha, T zl, T beta, T zr)
{
    return fma(beta, zr, fma(alpha, zl, y));
}

// Separator system of one fibre from the separator f values (in sep[], which
// receives z) and the segment-end values; coefficient tables per separator.
template <typename T>
__device__ __forceinline__ void sep_solve(int S, T* sep, int64_t sstride, const T* yfirst,
                                          const T* ylast, int64_t ystride, const T* ssub,
                                          const T* ssup, const T* sl, const T* sip,
                                          const T* su)
{
    T g = T(0);
    for (int k = 1; k < S; k++) {
        const T rhs = sep_rhs(sep[k * sstride], ssub[k], ylast[(k - 1) * ystride], ssup[k], yfirst[k * ystride]);
        g = (k == 1) ? rhs : sep_fwd(rhs, sl[k], g);
        sep[k * sstride] = g;
    }
    T z = T(0);
    for (int k = S - 1; k >= 1; k--) {
        z = (k == S - 1) ? sep[k * sstride] * sip[k] : sep_bwd(sep[k * sstride], su[k], z, sip[k]);
        sep[k * sstride] = z;
    }
}

// ---- strided dimensions, one launch ---------------------------------------
// A tile of FB neighbouring fibres (coalesced) x S segments; lane j of
// segment s handles fibre fib0 + j.  The per-level launch uses FB = 64 (one
// wave per segment); the batched kernel packs FB = 16 fibres x up to 16
// segments into 256 threads.
template <typename T>
struct StridedSmem {
    T tab[5][kMaxSegWG * kSlot];  // L, U, IP, alpha, beta
    T septab[5][kMaxSegWG];       // sub, sup, sl, sip, su at separators
    T end[2][kMaxSegWG * 64];     // y at the two ends of each segment [s][j]
    T sep[kMaxSegWG * 64];        // f, then z, at each separator [s][j]
};

template <typename T, int FB, bool kAllSeg>  // kAllSeg: every s < S
__device__ __forceinline__ void solve_strided_tile(T* __restrict__ F, const FibreMap& m,
                                                   const SolveTables<T>& tb, int64_t fib0, int s,
                                                   int j, int nthr, int tid, StridedSmem<T>& sm)
{
    const int S = m.S;
    const bool inseg = kAllSeg || s < S;
    const int sc = kAllSeg ? s : (inseg ? s : S - 1);
    const int64_t fib = fib0 + j;
    const bool active = inseg && fib < m.nfib;
    const int64_t fc = fib < m.nfib ? fib : m.nfib - 1;  // idle lanes read a valid fibre
    const int64_t base = (fc / m.inner) * m.n * m.inner + fc % m.inner;
    int lo, len;
    seg_range(m, sc, lo, len);
    // the fibre loads are issued first and the tables' after them, so that
    // one memory latency covers both (staging the tables first would wait
    // for their loads before the fibre loads were issued)
    T v[kSlot];
#pragma unroll
    for (int q = 0; q < kSlot; q++) v[q] = F[base + (int64_t)(lo + min(q, len - 1)) * m.inner];
    const T fsep = F[base + (int64_t)(sc * kSeg) * m.inner];  // f at the segment's left separator
    for (int e = tid; e < S * kSlot; e += nthr) {
        sm.tab[0][e] = tb.L[e];
        sm.tab[1][e] = tb.U[e];
        sm.tab[2][e] = tb.IP[e];
        sm.tab[3][e] = tb.A[e];
        sm.tab[4][e] = tb.B[e];
    }
    for (int e = tid; e < S; e += nthr) {
        sm.septab[0][e] = tb.ssub[e];
        sm.septab[1][e] = tb.ssup[e];
        sm.septab[2][e] = tb.sl[e];
        sm.septab[3][e] = tb.sip[e];
        sm.septab[4][e] = tb.su[e];
    }
    if (inseg) sm.sep[s * FB + j] = (s > 0) ? fsep : T(0);
    __syncthreads();  // tables staged
    const T ylast = seg_solve(v, &sm.tab[0][sc * kSlot], &sm.tab[1][sc * kSlot], &sm.tab[2][sc * kSlot]);
    if (inseg) {
        sm.end[0][s * FB + j] = v[0];
        sm.end[1][s * FB + j] = ylast;
    }
    __syncthreads();
    if (s == 0 && S > 1)
        sep_solve(S, &sm.sep[j], FB, &sm.end[0][j], &sm.end[1][j], FB, sm.septab[0], sm.septab[1],
                  sm.septab[2], sm.septab[3], sm.septab[4]);
    __syncthreads();
    if (!active) return;
    const T zl = (s > 0) ? sm.sep[s * FB + j] : T(0);
    const T zr = (s < S - 1) ? sm.sep[(s + 1) * FB + j] : T(0);
    const T* ta = &sm.tab[3][s * kSlot];
    const T* tbt = &sm.tab[4][s * kSlot];
#pragma unroll
    for (int q = 0; q < kSlot; q++)
        if (q < len) F[base + (int64_t)(lo + q) * m.inner] = seg_final(v[q], ta[q], zl, tbt[q], zr);
    if (s > 0) F[base + (int64_t)(s * kSeg) * m.inner] = zl;
}

// ---- contiguous dimension, one launch --------------------------------------
// ---- contiguous dimension: rows staged through LDS ------------------------
constexpr int kSpanMax = kBlk * kSlot;
// Elements a per-level rows workgroup stages: the same bytes for either type
// (FP64 stages half the elements), so both keep three workgroups per CU.
template <typename T>
constexpr int rows_span()
{
    return kSpanMax * 4 / (int)sizeof(T);
}
__device__ __forceinline__ int padded(int e) { return e + (e >> 5); }

template <typename T, int kSpan, bool kLdsTab>
struct RowsSmem {
    T f[kSpan + kSpan / 32 + 1];
    T end[2][kBlk];
    T tab[5][kLdsTab ? kMaxSegWG * kSlot : 1];  // segment tables (S <= kMaxSegWG)
    T septab[5][kLdsTab ? kMaxSegWG : kBlk];    // sub, sup, sl, sip, su at separators
};

// Rows row0 .. row0 + nrows - 1 (nrows * S <= kBlk, nrows * n <= kSpan),
// in phases: the span's loads into registers (all in flight together,
// indices clamped into the span so the loads are unconditional), their LDS
// staging, the segment tables, the solve in LDS, and the span's stores.
template <typename T, int kSpan>
__device__ __forceinline__ void rows_load(const T* __restrict__ F, int64_t row0, int span, int n,
                                          T (&tmp)[(kSpan + kBlk - 1) / kBlk], int tid)
{
    // one descriptor over the span (past its end the loads read zero), one
    // 32-bit offset per load; the whole offset is in the per-lane operand,
    // which is what the hardware range check covers (the instruction's
    // scalar offset is added after the check)
    const __amdgpu_buffer_rsrc_t r = make_rsrc(F + row0 * n, (unsigned)span * (unsigned)sizeof(T));
    const unsigned o = (unsigned)tid * (unsigned)sizeof(T);
#pragma unroll
    for (int q = 0; q < (kSpan + kBlk - 1) / kBlk; q++) tmp[q] = buf_load<T>(r, o + (unsigned)(q * kBlk * sizeof(T)));
}

template <typename T, int kSpan, bool kLdsTab>
__device__ __forceinline__ void rows_stage(const T (&tmp)[(kSpan + kBlk - 1) / kBlk], int span,
                                           RowsSmem<T, kSpan, kLdsTab>& sm)
{
    // padded(q kBlk + t) = q (kBlk + kBlk / 32) + padded(t): one address
    // register, the rest in the instructions' offsets
    T* const f = sm.f + padded((int)threadIdx.x);
#pragma unroll
    for (int q = 0; q < (kSpan + kBlk - 1) / kBlk; q++)
        if (q * kBlk + (int)threadIdx.x < span) f[q * (kBlk + kBlk / 32)] = tmp[q];
}

template <typename T, int kSpan, bool kLdsTab>
__device__ __forceinline__ void rows_tables(const FibreMap& m, const SolveTables<T>& tb,
                                            RowsSmem<T, kSpan, kLdsTab>& sm)
{
    if (kLdsTab)
        for (int e = threadIdx.x; e < m.S * kSlot; e += kBlk) {
            sm.tab[0][e] = tb.L[e];
            sm.tab[1][e] = tb.U[e];
            sm.tab[2][e] = tb.IP[e];
            sm.tab[3][e] = tb.A[e];
            sm.tab[4][e] = tb.B[e];
        }
    // separator tables: the separator sweep is serial, so each of its steps
    // must find them in LDS rather than wait on a global load
    for (int e = threadIdx.x; e < m.S; e += kBlk) {
        sm.septab[0][e] = tb.ssub[e];
        sm.septab[1][e] = tb.ssup[e];
        sm.septab[2][e] = tb.sl[e];
        sm.septab[3][e] = tb.sip[e];
        sm.septab[4][e] = tb.su[e];
    }
}

// The solve of the staged rows, in LDS.  Starts after a barrier that
// follows the staging, ends with the solution in sm.f and a barrier.
// tid: threadIdx.x (a caller in a loop passes it through an opaque copy, so
// that the compiler does not hoist the per-slot LDS addresses out of the
// loop and keep them all in registers).
template <typename T, int kSpan, bool kLdsTab>
__device__ __forceinline__ void rows_solve_lds(const FibreMap& m, const SolveTables<T>& tb, int nrows,
                                               RowsSmem<T, kSpan, kLdsTab>& sm, int tid)
{
    auto bar = [] { __syncthreads(); };
    const int n = (int)m.n;
    const int r = tid / m.S, s = tid % m.S;
    const bool active = r < nrows;
    const int rr = active ? r : 0;
    int lo, len;
    seg_range(m, s, lo, len);
    const int so = s * kSlot;
    const T* tL = kLdsTab ? &sm.tab[0][so] : tb.L + so;
    const T* tU = kLdsTab ? &sm.tab[1][so] : tb.U + so;
    const T* tI = kLdsTab ? &sm.tab[2][so] : tb.IP + so;
    const T* tA = kLdsTab ? &sm.tab[3][so] : tb.A + so;
    const T* tB = kLdsTab ? &sm.tab[4][so] : tb.B + so;
    T v[kSlot];
#pragma unroll
    for (int q = 0; q < kSlot; q++) v[q] = sm.f[padded(rr * n + lo + min(q, len - 1))];
    const T ylast = seg_solve(v, tL, tU, tI);
    sm.end[0][tid] = v[0];
    sm.end[1][tid] = ylast;
    bar();
    if (active && s == 0 && m.S > 1) {
        // row r's separators live in sm.f at r*n + k*kSeg
        const int t0 = tid;
        T gg = T(0);
        for (int k = 1; k < m.S; k++) {
            const int e = padded(r * n + k * kSeg);
            const T rhs = sep_rhs(sm.f[e], sm.septab[0][k], sm.end[1][t0 + k - 1], sm.septab[1][k], sm.end[0][t0 + k]);
            gg = (k == 1) ? rhs : sep_fwd(rhs, sm.septab[2][k], gg);
            sm.f[e] = gg;
        }
        T z = T(0);
        for (int k = m.S - 1; k >= 1; k--) {
            const int e = padded(r * n + k * kSeg);
            z = (k == m.S - 1) ? sm.f[e] * sm.septab[3][k] : sep_bwd(sm.f[e], sm.septab[4][k], z, sm.septab[3][k]);
            sm.f[e] = z;
        }
    }
    bar();
    const T zl = (s > 0) ? sm.f[padded(rr * n + s * kSeg)] : T(0);
    const T zr = (s < m.S - 1) ? sm.f[padded(rr * n + (s + 1) * kSeg)] : T(0);
    bar();  // every lane has read its separators
    if (active) {
#pragma unroll
        for (int q = 0; q < kSlot; q++)
            if (q < len) sm.f[padded(r * n + lo + q)] = seg_final(v[q], tA[q], zl, tB[q], zr);
    }
    bar();
}

template <typename T, int kSpan, bool kLdsTab>
__device__ __forceinline__ void rows_store(T* __restrict__ F, int64_t row0, int span, int n,
                                           const RowsSmem<T, kSpan, kLdsTab>& sm)
{
    T* g = F + row0 * n;
    for (int e = threadIdx.x; e < span; e += kBlk) g[e] = sm.f[padded(e)];
}

template <typename T, int kSpan, bool kLdsTab>
__device__ __forceinline__ void solve_rows_tile(T* __restrict__ F, const FibreMap& m,
                                                const SolveTables<T>& tb, int64_t row0, int nrows,
                                                RowsSmem<T, kSpan, kLdsTab>& sm)
{
    const int n = (int)m.n;
    const int span = nrows * n;
    {
        T tmp[(kSpan + kBlk - 1) / kBlk];
        rows_load<T, kSpan>(F, row0, span, n, tmp, (int)threadIdx.x);
        rows_stage<T, kSpan, kLdsTab>(tmp, span, sm);
    }
    rows_tables(m, tb, sm);
    __syncthreads();
    rows_solve_lds<T, kSpan, kLdsTab>(m, tb, nrows, sm, (int)threadIdx.x);
    rows_store(F, row0, span, n, sm);
}

// The span's stores with their LDS reads issued in batches (a loop of single
// read-then-store steps waits a full LDS round trip per element): one
// descriptor over the span, past whose end the stores are dropped, so the
// unrolled batches need no per-element branch; element indices past the span
// read its last element instead.
template <typename T, int kSpan, bool kLdsTab>
__device__ __forceinline__ void rows_store_batched(T* __restrict__ F, int64_t row0, int span, int n,
                                                   const RowsSmem<T, kSpan, kLdsTab>& sm, int tid)
{
    constexpr int NQ = (kSpan + kBlk - 1) / kBlk;
    constexpr int CH = (sizeof(T) == 4) ? 11 : 9;  // values in flight per lane
    const __amdgpu_buffer_rsrc_t r = make_rsrc(F + row0 * n, (unsigned)span * (unsigned)sizeof(T));
    const unsigned o = (unsigned)tid * (unsigned)sizeof(T);
#pragma unroll
    for (int q0 = 0; q0 < NQ; q0 += CH) {
        T v[CH];
#pragma unroll
        for (int q = 0; q < CH; q++)
            if (q0 + q < NQ) v[q] = sm.f[padded(min((q0 + q) * kBlk + tid, span - 1))];
#pragma unroll
        for (int q = 0; q < CH; q++)
            if (q0 + q < NQ) buf_store(v[q], r, o + (unsigned)((q0 + q) * kBlk * sizeof(T)));
    }
}

// The per-level launch: each workgroup runs blocks blockIdx.x, + gridDim.x,
// ... (every block rpb rows, the last one fewer), with the loads of its next
// block issued right after the current block is staged, so that they are in
// flight during the solve and the stores.  A block past the last reads
// through an empty descriptor (no memory access), so the loads stay
// unconditional.
template <typename T, int kSpan, bool kLdsTab>
__device__ __forceinline__ void solve_rows_loop(T* __restrict__ F, const FibreMap& m, const SolveTables<T>& tb,
                                                int rpb, RowsSmem<T, kSpan, kLdsTab>& sm)
{
    const int n = (int)m.n;
    const int64_t nblk = (m.nfib + rpb - 1) / rpb;
    auto span_of = [&](int64_t b) {
        return b < nblk ? (int)min((int64_t)rpb, m.nfib - b * rpb) * n : 0;
    };
    T tmp[(kSpan + kBlk - 1) / kBlk];
    int64_t b = blockIdx.x;
    rows_load<T, kSpan>(F, b < nblk ? b * rpb : 0, span_of(b), n, tmp, (int)threadIdx.x);
    // after the first block's loads were issued: one memory latency covers both
    rows_tables(m, tb, sm);
    for (; b < nblk; b += gridDim.x) {
        const int span = span_of(b);
        rows_stage<T, kSpan, kLdsTab>(tmp, span, sm);
        // an opaque copy of the thread index: the per-load and per-slot
        // offsets derived from it are then formed inside the loop rather than
        // hoisted out of it and held in registers for its whole length
        int tid = (int)threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int64_t bn = b + gridDim.x;
        rows_load<T, kSpan>(F, bn < nblk ? bn * rpb : 0, span_of(bn), n, tmp, tid);
        __syncthreads();
        rows_solve_lds<T, kSpan, kLdsTab>(m, tb, span / n, sm, tid);
        rows_store_batched<T, kSpan, kLdsTab>(F, b * rpb, span, n, sm, tid);
        __syncthreads();  // every lane has read sm.f before the next block is staged
    }
}

// ---- long fibres: three launches through global memory ---------------------
// Phase 1 and 3 work item: strided dimensions use blockIdx.y as the segment
// and x over fibres; the contiguous dimension runs x over (row, segment).
__device__ __forceinline__ bool locate(const FibreMap& m, int bx, int by, int64_t& base, int64_t& fib, int& s)
{
    const int64_t gx = (int64_t)bx * kBlk + threadIdx.x;
    int64_t in, o;
    if (m.inner > 1) {
        if (gx >= m.nfib) return false;
        s = by;
        in = gx % m.inner;
        o = gx / m.inner;
    } else {
        if (gx >= m.nfib * m.S) return false;
        s = (int)(gx % m.S);
        o = gx / m.S;
        in = 0;
    }
    fib = o * m.inner + in;
    base = o * m.n * m.inner + in;
    return true;
}

__device__ __forceinline__ int64_t yb_index(const FibreMap& m, int64_t fib, int s)
{
    return 2 * ((m.inner > 1) ? (int64_t)s * m.nfib + fib : fib * m.S + s);
}

template <typename T>
__device__ __forceinline__ T load_solve(const T* F, const FibreMap& m, int64_t base, int s,
                                        const SolveTables<T>& tb, T (&v)[kSlot], int& lo, int& len)
{
    seg_range(m, s, lo, len);
#pragma unroll
    for (int q = 0; q < kSlot; q++) v[q] = F[base + (int64_t)(lo + min(q, len - 1)) * m.inner];
    return seg_solve(v, tb.L + s * kSlot, tb.U + s * kSlot, tb.IP + s * kSlot);
}

template <typename T>
__device__ __forceinline__ void seg_ends_tile(const T* __restrict__ F, T* __restrict__ Yb, const FibreMap& m,
                                              const SolveTables<T>& tb, int bx, int by)
{
    int64_t base, fib;
    int s, lo, len;
    if (!locate(m, bx, by, base, fib, s)) return;
    T v[kSlot];
    const T ylast = load_solve(F, m, base, s, tb, v, lo, len);
    const int64_t yi = yb_index(m, fib, s);
    Yb[yi] = v[0];
    Yb[yi + 1] = ylast;
}

template <typename T>
__device__ __forceinline__ void separators_tile(T* __restrict__ F, const T* __restrict__ Yb, const FibreMap& m,
                                                const SolveTables<T>& tb, int bx)
{
    const int64_t fib = (int64_t)bx * kBlk + threadIdx.x;
    if (fib >= m.nfib) return;
    const int64_t o = fib / m.inner, in = fib % m.inner;
    T* p = F + o * m.n * m.inner + in;
    const int64_t ys = (m.inner > 1) ? 2 * m.nfib : 2;
    const T* y0 = Yb + yb_index(m, fib, 0);
    sep_solve(m.S, p, (int64_t)kSeg * m.inner, y0, y0 + 1, ys, tb.ssub, tb.ssup, tb.sl, tb.sip, tb.su);
}

template <typename T>
__device__ __forceinline__ void seg_final_tile(T* __restrict__ F, const FibreMap& m, const SolveTables<T>& tb,
                                               int bx, int by)
{
    int64_t base, fib;
    int s, lo, len;
    if (!locate(m, bx, by, base, fib, s)) return;
    T v[kSlot];
    load_solve(F, m, base, s, tb, v, lo, len);
    const T zl = (s > 0) ? F[base + (int64_t)(s * kSeg) * m.inner] : T(0);
    const T zr = (s < m.S - 1) ? F[base + (int64_t)((s + 1) * kSeg) * m.inner] : T(0);
#pragma unroll
    for (int q = 0; q < kSlot; q++)
        if (q < len)
            F[base + (int64_t)(lo + q) * m.inner] = seg_final(v[q], tb.A[s * kSlot + q], zl, tb.B[s * kSlot + q], zr);
}

}  // namespace
}  // namespace mgr
