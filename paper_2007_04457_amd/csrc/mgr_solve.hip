// Correction solve M_{l-1} z = f along one dimension (Sec. II-A.2; the
// paper's iterative processing kernel, Sec. III-A.3) as a partitioned Thomas
// algorithm.
//
// The coarse mass matrix is the same for every fibre along a dimension, so
// the partition is fixed per (level, dimension) and all of its matrix-only
// quantities are tables built on the host in FP64:
//  - each fibre of length n is cut into S segments of kSeg nodes; the first
//    node of every segment but the first is a separator;
//  - inside a segment, z_i = y_i + alpha_i z_left + beta_i z_right, where y
//    solves the segment's interior rows with zero separators (local Thomas
//    factors) and alpha, beta are its responses to the two separators;
//  - substituting into the separator rows gives a tridiagonal system in the
//    S-1 separator values, whose right-hand side needs only f at the
//    separators and y next to them.
// Segment tables are stored padded to kSlot entries (zeros past the segment's
// length), so every lane runs the same straight-line code: all loads are
// unconditional (indices clamped into the segment) and can be issued
// together, with no per-element branches between them.
//
// Thread mapping: along a strided dimension a workgroup of 64 x S lanes holds
// 64 neighbouring fibres (coalesced), wave s solving segment s; along the
// contiguous dimension a workgroup stages whole rows through LDS and lanes
// take (row, segment) pairs.  Separators are solved in LDS by one lane per
// fibre.  Longer fibres fall back to three launches (segment ends,
// separators, final) through global memory.
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
        const T rhs = sep[k * sstride] - ssub[k] * ylast[(k - 1) * ystride] - ssup[k] * yfirst[k * ystride];
        g = (k == 1) ? rhs : rhs - sl[k] * g;
        sep[k * sstride] = g;
    }
    T z = T(0);
    for (int k = S - 1; k >= 1; k--) {
        z = (k == S - 1) ? sep[k * sstride] * sip[k] : (sep[k * sstride] - su[k] * z) * sip[k];
        sep[k * sstride] = z;
    }
}

// ---- strided dimensions, one launch ---------------------------------------
template <typename T>
__global__ void __launch_bounds__(64 * kMaxSegWG)
k_solve_strided_wg(T* __restrict__ F, FibreMap m, SolveTables<T> tb)
{
    __shared__ T sTab[5][kMaxSegWG * kSlot];  // L, U, IP, alpha, beta
    __shared__ T sSepTab[5][kMaxSegWG];       // sub, sup, sl, sip, su at separators
    __shared__ T sEnd[2][kMaxSegWG][64];      // y at the two ends of each segment
    __shared__ T sSep[kMaxSegWG][64];         // f, then z, at each separator
    const int S = m.S;
    const int nthr = 64 * S;
    const int tid = threadIdx.y * 64 + threadIdx.x;
    for (int e = tid; e < S * kSlot; e += nthr) {
        sTab[0][e] = tb.L[e];
        sTab[1][e] = tb.U[e];
        sTab[2][e] = tb.IP[e];
        sTab[3][e] = tb.A[e];
        sTab[4][e] = tb.B[e];
    }
    for (int e = tid; e < S; e += nthr) {
        sSepTab[0][e] = tb.ssub[e];
        sSepTab[1][e] = tb.ssup[e];
        sSepTab[2][e] = tb.sl[e];
        sSepTab[3][e] = tb.sip[e];
        sSepTab[4][e] = tb.su[e];
    }
    const int lane = threadIdx.x;
    const int s = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int64_t fib = (int64_t)blockIdx.x * 64 + lane;
    const bool active = fib < m.nfib;
    const int64_t fc = active ? fib : m.nfib - 1;  // idle lanes read a valid fibre
    const int64_t base = (fc / m.inner) * m.n * m.inner + fc % m.inner;
    int lo, len;
    seg_range(m, s, lo, len);
    T v[kSlot];
#pragma unroll
    for (int q = 0; q < kSlot; q++) v[q] = F[base + (int64_t)(lo + min(q, len - 1)) * m.inner];
    sSep[s][lane] = (s > 0) ? F[base + (int64_t)(s * kSeg) * m.inner] : T(0);
    __syncthreads();  // tables staged
    const T ylast = seg_solve(v, &sTab[0][s * kSlot], &sTab[1][s * kSlot], &sTab[2][s * kSlot]);
    sEnd[0][s][lane] = v[0];
    sEnd[1][s][lane] = ylast;
    __syncthreads();
    if (s == 0 && S > 1)
        sep_solve(S, &sSep[0][lane], 64, &sEnd[0][0][lane], &sEnd[1][0][lane], 64, sSepTab[0],
                  sSepTab[1], sSepTab[2], sSepTab[3], sSepTab[4]);
    __syncthreads();
    if (!active) return;
    const T zl = (s > 0) ? sSep[s][lane] : T(0);
    const T zr = (s < S - 1) ? sSep[s + 1][lane] : T(0);
    const T* ta = &sTab[3][s * kSlot];
    const T* tbt = &sTab[4][s * kSlot];
#pragma unroll
    for (int q = 0; q < kSlot; q++)
        if (q < len) F[base + (int64_t)(lo + q) * m.inner] = v[q] + ta[q] * zl + tbt[q] * zr;
    if (s > 0) F[base + (int64_t)(s * kSeg) * m.inner] = zl;
}

// ---- contiguous dimension, one launch --------------------------------------
// A block takes whole rows (rows_per_block * S lanes); their data are one
// contiguous span of F, staged through LDS with one pad element per 32 so
// that each lane's segment reads are bank-conflict free.
constexpr int kSpanMax = kBlk * kSlot;
__device__ __forceinline__ int padded(int e) { return e + (e >> 5); }

template <typename T, bool kLdsTab>
__global__ void __launch_bounds__(kBlk)
k_solve_rows_wg(T* __restrict__ F, FibreMap m, SolveTables<T> tb, int rows_per_block)
{
    __shared__ T sF[kSpanMax + kSpanMax / 32 + 1];
    __shared__ T sEnd[2][kBlk];
    __shared__ T sTab[5][kLdsTab ? kMaxSegWG * kSlot : 1];  // segment tables (S <= kMaxSegWG)
    const int64_t row0 = (int64_t)blockIdx.x * rows_per_block;
    const int nrows = (int)min((int64_t)rows_per_block, m.nfib - row0);
    const int n = (int)m.n;
    const int span = nrows * n;
    T* g = F + row0 * n;
    for (int e = threadIdx.x; e < span; e += kBlk) sF[padded(e)] = g[e];
    constexpr bool lds_tab = kLdsTab;
    if (lds_tab)
        for (int e = threadIdx.x; e < m.S * kSlot; e += kBlk) {
            sTab[0][e] = tb.L[e];
            sTab[1][e] = tb.U[e];
            sTab[2][e] = tb.IP[e];
            sTab[3][e] = tb.A[e];
            sTab[4][e] = tb.B[e];
        }
    const int r = threadIdx.x / m.S, s = threadIdx.x % m.S;
    const bool active = r < nrows;
    const int rr = active ? r : 0;
    int lo, len;
    seg_range(m, s, lo, len);
    const int so = s * kSlot;
    const T* tL = lds_tab ? &sTab[0][so] : tb.L + so;
    const T* tU = lds_tab ? &sTab[1][so] : tb.U + so;
    const T* tI = lds_tab ? &sTab[2][so] : tb.IP + so;
    const T* tA = lds_tab ? &sTab[3][so] : tb.A + so;
    const T* tB = lds_tab ? &sTab[4][so] : tb.B + so;
    __syncthreads();
    T v[kSlot];
#pragma unroll
    for (int q = 0; q < kSlot; q++) v[q] = sF[padded(rr * n + lo + min(q, len - 1))];
    const T ylast = seg_solve(v, tL, tU, tI);
    sEnd[0][threadIdx.x] = v[0];
    sEnd[1][threadIdx.x] = ylast;
    __syncthreads();
    if (active && s == 0 && m.S > 1) {
        // row r's separators live in sF at r*n + k*kSeg
        const int t0 = threadIdx.x;
        T gg = T(0);
        for (int k = 1; k < m.S; k++) {
            const int e = padded(r * n + k * kSeg);
            const T rhs = sF[e] - tb.ssub[k] * sEnd[1][t0 + k - 1] - tb.ssup[k] * sEnd[0][t0 + k];
            gg = (k == 1) ? rhs : rhs - tb.sl[k] * gg;
            sF[e] = gg;
        }
        T z = T(0);
        for (int k = m.S - 1; k >= 1; k--) {
            const int e = padded(r * n + k * kSeg);
            z = (k == m.S - 1) ? sF[e] * tb.sip[k] : (sF[e] - tb.su[k] * z) * tb.sip[k];
            sF[e] = z;
        }
    }
    __syncthreads();
    const T zl = (s > 0) ? sF[padded(rr * n + s * kSeg)] : T(0);
    const T zr = (s < m.S - 1) ? sF[padded(rr * n + (s + 1) * kSeg)] : T(0);
    __syncthreads();  // every lane has read its separators
    if (active) {
#pragma unroll
        for (int q = 0; q < kSlot; q++)
            if (q < len) sF[padded(r * n + lo + q)] = v[q] + tA[q] * zl + tB[q] * zr;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < span; e += kBlk) g[e] = sF[padded(e)];
}

// ---- long fibres: three launches through global memory ---------------------
// Phase 1 and 3 work item: strided dimensions use blockIdx.y as the segment
// and x over fibres; the contiguous dimension runs x over (row, segment).
__device__ __forceinline__ bool locate(const FibreMap& m, int64_t& base, int64_t& fib, int& s)
{
    const int64_t gx = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    int64_t in, o;
    if (m.inner > 1) {
        if (gx >= m.nfib) return false;
        s = (int)blockIdx.y;
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
__global__ void __launch_bounds__(kBlk)
k_seg_ends(const T* __restrict__ F, T* __restrict__ Yb, FibreMap m, SolveTables<T> tb)
{
    int64_t base, fib;
    int s, lo, len;
    if (!locate(m, base, fib, s)) return;
    T v[kSlot];
    const T ylast = load_solve(F, m, base, s, tb, v, lo, len);
    const int64_t yi = yb_index(m, fib, s);
    Yb[yi] = v[0];
    Yb[yi + 1] = ylast;
}

template <typename T>
__global__ void __launch_bounds__(kBlk)
k_separators(T* __restrict__ F, const T* __restrict__ Yb, FibreMap m, SolveTables<T> tb)
{
    const int64_t fib = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (fib >= m.nfib) return;
    const int64_t o = fib / m.inner, in = fib % m.inner;
    T* p = F + o * m.n * m.inner + in;
    const int64_t ys = (m.inner > 1) ? 2 * m.nfib : 2;
    const T* y0 = Yb + yb_index(m, fib, 0);
    sep_solve(m.S, p, (int64_t)kSeg * m.inner, y0, y0 + 1, ys, tb.ssub, tb.ssup, tb.sl, tb.sip, tb.su);
}

template <typename T>
__global__ void __launch_bounds__(kBlk)
k_seg_final(T* __restrict__ F, FibreMap m, SolveTables<T> tb)
{
    int64_t base, fib;
    int s, lo, len;
    if (!locate(m, base, fib, s)) return;
    T v[kSlot];
    load_solve(F, m, base, s, tb, v, lo, len);
    const T zl = (s > 0) ? F[base + (int64_t)(s * kSeg) * m.inner] : T(0);
    const T zr = (s < m.S - 1) ? F[base + (int64_t)((s + 1) * kSeg) * m.inner] : T(0);
#pragma unroll
    for (int q = 0; q < kSlot; q++)
        if (q < len) F[base + (int64_t)(lo + q) * m.inner] = v[q] + tb.A[s * kSlot + q] * zl + tb.B[s * kSlot + q] * zr;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kBlk - 1) / kBlk); }

}  // namespace

// Solve along dimension d of the packed array F (shape fv.n), in place.  Yb
// is scratch of at least 2 * S * (number of fibres) elements.
template <typename T>
hipError_t launch_solve_partitioned(T* F, View3 fv, int d, SolveTables<T> tb, T* Yb, hipStream_t st)
{
    FibreMap m;
    m.n = fv.n[d];
    m.inner = 1;
    for (int e = d + 1; e < 3; e++) m.inner *= fv.n[e];
    m.outer = 1;
    for (int e = 0; e < d; e++) m.outer *= fv.n[e];
    m.nfib = m.inner * m.outer;
    m.S = tb.S;
    if (m.inner == 1 && m.S <= kBlk) {
        const int rpb = kBlk / m.S;
        const unsigned nb = (unsigned)((m.nfib + rpb - 1) / rpb);
        if (m.S <= kMaxSegWG)
            hipLaunchKernelGGL((k_solve_rows_wg<T, true>), dim3(nb), dim3(kBlk), 0, st, F, m, tb, rpb);
        else
            hipLaunchKernelGGL((k_solve_rows_wg<T, false>), dim3(nb), dim3(kBlk), 0, st, F, m, tb, rpb);
        return hipGetLastError();
    }
    if (m.inner > 1 && m.S <= kMaxSegWG) {
        hipLaunchKernelGGL(k_solve_strided_wg<T>, dim3((unsigned)((m.nfib + 63) / 64)), dim3(64, m.S), 0, st,
                           F, m, tb);
        return hipGetLastError();
    }
    const dim3 grid = (m.inner > 1) ? dim3(blocks(m.nfib), (unsigned)m.S) : dim3(blocks(m.nfib * m.S));
    hipLaunchKernelGGL(k_seg_ends<T>, grid, dim3(kBlk), 0, st, F, Yb, m, tb);
    hipLaunchKernelGGL(k_separators<T>, dim3(blocks(m.nfib)), dim3(kBlk), 0, st, F, Yb, m, tb);
    hipLaunchKernelGGL(k_seg_final<T>, grid, dim3(kBlk), 0, st, F, m, tb);
    return hipGetLastError();
}

template hipError_t launch_solve_partitioned<float>(float*, View3, int, SolveTables<float>, float*,
                                                    hipStream_t);
template hipError_t launch_solve_partitioned<double>(double*, View3, int, SolveTables<double>, double*,
                                                     hipStream_t);

}  // namespace mgr
