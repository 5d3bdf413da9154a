// Correction solve M_{l-1} z = f along one dimension (Sec. II-A.2; the
// paper's iterative processing kernel, Sec. III-A.3) as a partitioned Thomas
// algorithm.
//
// The coarse mass matrix is the same for every fibre along a dimension, so
// the partition is fixed per (level, dimension) and all of its matrix-only
// quantities are tables built on the host in FP64:
//  - each fibre of length n is cut into S segments of B = kSeg nodes; the
//    first node of every segment but the first is a separator;
//  - inside a segment, z_i = y_i + alpha_i z_left + beta_i z_right, where y
//    solves the segment's interior rows with zero separators (local Thomas
//    factors lseg/ipseg) and alpha, beta are its responses to the two
//    separators;
//  - substituting into the separator rows gives a tridiagonal system in the
//    S-1 separator values (factors sl/sip/su), whose right-hand side needs
//    only f at the separators and y next to them.
// Phase 1: per segment, y at its two ends.  Phase 2: per fibre, the
// separator system.  Phase 3: per segment, y again and z (optionally added
// to the coarse values: the "apply correction" of Eq. (1)).  Fibres with
// n <= kSeg + 1 are one segment and need phase 3 only.
//
// Thread mapping: along a strided dimension, neighbouring lanes take
// neighbouring fibres (coalesced); along the contiguous dimension they take
// neighbouring segments of one row.  Segment values live in registers.
#include "mgr_internal.h"

namespace mgr {
namespace {

constexpr int kBlk = 256;

struct FibreMap {
    int64_t n, inner, outer, nfib;
    int S;
};

// Work item of phases 1 and 3.  Strided dimensions: blockIdx.y is the
// segment (uniform per block, so table reads are scalar) and x runs over
// fibres.  Contiguous dimension: x runs over (row, segment), segment fastest.
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

// Interior [lo, hi) of segment s.
__device__ __forceinline__ void seg_range(const FibreMap& m, int s, int& lo, int& hi)
{
    lo = s * kSeg + (s > 0 ? 1 : 0);
    hi = (s == m.S - 1) ? (int)m.n : (s + 1) * kSeg;
}

// Local Thomas solve of a segment interior held in registers v[0..len).
template <typename T>
__device__ __forceinline__ void local_solve(T (&v)[kSeg + 1], int lo, int len,
                                            const SolveTables<T>& tb)
{
#pragma unroll
    for (int q = 1; q < kSeg + 1; q++)
        if (q < len) v[q] -= tb.lseg[lo + q] * v[q - 1];
    T z = T(0);
#pragma unroll
    for (int q = kSeg; q >= 0; q--) {
        if (q < len) {
            z = (q == len - 1) ? v[q] * tb.ipseg[lo + q] : (v[q] - tb.sup[lo + q] * z) * tb.ipseg[lo + q];
            v[q] = z;
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlk)
k_seg_ends(const T* __restrict__ F, T* __restrict__ Yb, FibreMap m, SolveTables<T> tb)
{
    int64_t base, fib;
    int s, lo, hi;
    if (!locate(m, base, fib, s)) return;
    seg_range(m, s, lo, hi);
    const int len = hi - lo;
    T v[kSeg + 1];
#pragma unroll
    for (int q = 0; q < kSeg + 1; q++) v[q] = (q < len) ? F[base + (int64_t)(lo + q) * m.inner] : T(0);
    local_solve(v, lo, len, tb);
    T first = v[0], last = v[0];
#pragma unroll
    for (int q = 0; q < kSeg + 1; q++)
        if (q == len - 1) last = v[q];
    const int64_t yi = yb_index(m, fib, s);
    Yb[yi] = first;
    Yb[yi + 1] = last;
}

// Separator system of one fibre; writes z at the separator nodes into F
// (the forward sweep parks its intermediate values there too).
template <typename T>
__global__ void __launch_bounds__(kBlk)
k_separators(T* __restrict__ F, const T* __restrict__ Yb, FibreMap m, SolveTables<T> tb)
{
    const int64_t fib = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (fib >= m.nfib) return;
    const int64_t o = fib / m.inner, in = fib % m.inner;
    T* p = F + o * m.n * m.inner + in;
    T g = T(0);
    for (int s = 1; s < m.S; s++) {
        const int k = s * kSeg;
        const T rhs = p[(int64_t)k * m.inner] - tb.sub[k] * Yb[yb_index(m, fib, s - 1) + 1] -
                      tb.sup[k] * Yb[yb_index(m, fib, s)];
        g = (s == 1) ? rhs : rhs - tb.sl[s] * g;
        p[(int64_t)k * m.inner] = g;
    }
    T z = T(0);
    for (int s = m.S - 1; s >= 1; s--) {
        const int k = s * kSeg;
        z = (s == m.S - 1) ? p[(int64_t)k * m.inner] * tb.sip[s]
                           : (p[(int64_t)k * m.inner] - tb.su[s] * z) * tb.sip[s];
        p[(int64_t)k * m.inner] = z;
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlk)
k_seg_final(T* __restrict__ F, T* __restrict__ W, T sign, FibreMap m, SolveTables<T> tb)
{
    int64_t base, fib;
    int s, lo, hi;
    if (!locate(m, base, fib, s)) return;
    seg_range(m, s, lo, hi);
    const int len = hi - lo;
    T v[kSeg + 1];
#pragma unroll
    for (int q = 0; q < kSeg + 1; q++) v[q] = (q < len) ? F[base + (int64_t)(lo + q) * m.inner] : T(0);
    local_solve(v, lo, len, tb);
    const T zl = (s > 0) ? F[base + (int64_t)(s * kSeg) * m.inner] : T(0);
    const T zr = (s < m.S - 1) ? F[base + (int64_t)((s + 1) * kSeg) * m.inner] : T(0);
#pragma unroll
    for (int q = 0; q < kSeg + 1; q++) {
        if (q < len) {
            const int i = lo + q;
            const T z = v[q] + tb.alpha[i] * zl + tb.beta[i] * zr;
            const int64_t off = base + (int64_t)i * m.inner;
            F[off] = z;
            if (W) W[off] += sign * z;
        }
    }
    if (W && s > 0) W[base + (int64_t)(s * kSeg) * m.inner] += sign * zl;
}

// Contiguous dimension: a block takes whole rows (rows_per_block * S
// threads) whose data are one contiguous span of F, staged through LDS with
// one pad element per 32 so that each lane's segment reads are bank-conflict
// free.  Span <= 256 rows' worth of 33 nodes.  (Used by k_solve_rows_wg.)
constexpr int kSpanMax = kBlk * (kSeg + 1);
__device__ __forceinline__ int padded(int e) { return e + (e >> 5); }

// Single-launch form for strided dimensions with S <= kMaxSegWG segments: a
// workgroup of 64 x S threads holds 64 neighbouring fibres; wave s solves
// segment s of each, one lane per fibre, and keeps its segment in registers
// while lane-per-fibre threads of wave 0 solve the separator systems in LDS.
// One read and one write of F.
constexpr int kMaxSegWG = 16;

template <typename T>
__global__ void __launch_bounds__(64 * kMaxSegWG)
k_solve_strided_wg(T* __restrict__ F, T* __restrict__ W, T sign, FibreMap m, SolveTables<T> tb)
{
    __shared__ T sEnd[2][kMaxSegWG][64];  // y at the two ends of each segment
    __shared__ T sSep[kMaxSegWG][64];     // f, then z, at each separator
    const int lane = threadIdx.x, s = threadIdx.y;
    const int64_t fib = (int64_t)blockIdx.x * 64 + lane;
    const bool active = fib < m.nfib;
    const int64_t in = fib % m.inner, o = fib / m.inner;
    const int64_t base = o * m.n * m.inner + in;
    int lo, hi;
    seg_range(m, s, lo, hi);
    const int len = hi - lo;
    T v[kSeg + 1];
#pragma unroll
    for (int q = 0; q < kSeg + 1; q++)
        v[q] = (active && q < len) ? F[base + (int64_t)(lo + q) * m.inner] : T(0);
    if (s > 0) sSep[s][lane] = active ? F[base + (int64_t)(s * kSeg) * m.inner] : T(0);
    local_solve(v, lo, len, tb);
    T last = v[0];
#pragma unroll
    for (int q = 0; q < kSeg + 1; q++)
        if (q == len - 1) last = v[q];
    sEnd[0][s][lane] = v[0];
    sEnd[1][s][lane] = last;
    __syncthreads();
    if (s == 0) {
        T g = T(0);
        for (int k = 1; k < m.S; k++) {
            const int p = k * kSeg;
            const T rhs = sSep[k][lane] - tb.sub[p] * sEnd[1][k - 1][lane] - tb.sup[p] * sEnd[0][k][lane];
            g = (k == 1) ? rhs : rhs - tb.sl[k] * g;
            sSep[k][lane] = g;
        }
        T z = T(0);
        for (int k = m.S - 1; k >= 1; k--) {
            z = (k == m.S - 1) ? sSep[k][lane] * tb.sip[k] : (sSep[k][lane] - tb.su[k] * z) * tb.sip[k];
            sSep[k][lane] = z;
        }
    }
    __syncthreads();
    if (!active) return;
    const T zl = (s > 0) ? sSep[s][lane] : T(0);
    const T zr = (s < m.S - 1) ? sSep[s + 1][lane] : T(0);
#pragma unroll
    for (int q = 0; q < kSeg + 1; q++) {
        if (q < len) {
            const int i = lo + q;
            const T z = v[q] + tb.alpha[i] * zl + tb.beta[i] * zr;
            const int64_t off = base + (int64_t)i * m.inner;
            F[off] = z;
            if (W) W[off] += sign * z;
        }
    }
    if (s > 0) {
        const int64_t off = base + (int64_t)(s * kSeg) * m.inner;
        F[off] = zl;
        if (W) W[off] += sign * zl;
    }
}

// Single-launch form for the contiguous dimension: whole rows staged in LDS
// (see kSpanMax); after the segment solves, one lane per row solves that row's
// separator system in LDS, then every lane finishes its segment.
template <typename T>
__global__ void __launch_bounds__(kBlk)
k_solve_rows_wg(T* __restrict__ F, T* __restrict__ W, T sign, FibreMap m, SolveTables<T> tb,
                int rows_per_block)
{
    __shared__ T sF[kSpanMax + kSpanMax / 32 + 1];
    __shared__ T sEnd[2][kBlk];
    const int64_t row0 = (int64_t)blockIdx.x * rows_per_block;
    const int nrows = (int)min((int64_t)rows_per_block, m.nfib - row0);
    const int n = (int)m.n;
    const int span = nrows * n;
    T* g = F + row0 * n;
    for (int e = threadIdx.x; e < span; e += kBlk) sF[padded(e)] = g[e];
    __syncthreads();
    const int r = threadIdx.x / m.S, s = threadIdx.x % m.S;
    const bool active = r < nrows;
    int lo, hi;
    seg_range(m, s, lo, hi);
    const int len = hi - lo;
    T v[kSeg + 1];
    if (active) {
#pragma unroll
        for (int q = 0; q < kSeg + 1; q++) v[q] = (q < len) ? sF[padded(r * n + lo + q)] : T(0);
        local_solve(v, lo, len, tb);
        T last = v[0];
#pragma unroll
        for (int q = 0; q < kSeg + 1; q++)
            if (q == len - 1) last = v[q];
        sEnd[0][threadIdx.x] = v[0];
        sEnd[1][threadIdx.x] = last;
    }
    __syncthreads();
    if (active && s == 0) {
        const int t0 = threadIdx.x;  // row r's segment 0
        T gg = T(0);
        for (int k = 1; k < m.S; k++) {
            const int p = k * kSeg;
            const int e = padded(r * n + p);
            const T rhs = sF[e] - tb.sub[p] * sEnd[1][t0 + k - 1] - tb.sup[p] * sEnd[0][t0 + k];
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
    const T zl = (active && s > 0) ? sF[padded(r * n + s * kSeg)] : T(0);
    const T zr = (active && s < m.S - 1) ? sF[padded(r * n + (s + 1) * kSeg)] : T(0);
    __syncthreads();  // every lane has read its separators
    if (active) {
#pragma unroll
        for (int q = 0; q < kSeg + 1; q++)
            if (q < len) sF[padded(r * n + lo + q)] = v[q] + tb.alpha[lo + q] * zl + tb.beta[lo + q] * zr;
    }
    __syncthreads();
    T* w = W ? W + row0 * n : nullptr;
    for (int e = threadIdx.x; e < span; e += kBlk) {
        const T z = sF[padded(e)];
        g[e] = z;
        if (w) w[e] += sign * z;
    }
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kBlk - 1) / kBlk); }

}  // namespace

// Solve along dimension d of the packed array F (shape fv.n).  With W non-null
// the solution is also added, times sign, to W (same packed shape).  Yb is
// scratch of at least 2 * S * (number of fibres) elements.
template <typename T>
hipError_t launch_solve_partitioned(T* F, View3 fv, int d, SolveTables<T> tb, T* Yb, T* W, T sign,
                                    hipStream_t st)
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
        hipLaunchKernelGGL(k_solve_rows_wg<T>, dim3(nb), dim3(kBlk), 0, st, F, W, sign, m, tb, rpb);
        return hipGetLastError();
    }
    if (m.inner > 1 && m.S <= kMaxSegWG) {
        hipLaunchKernelGGL(k_solve_strided_wg<T>, dim3((unsigned)((m.nfib + 63) / 64)), dim3(64, m.S), 0, st,
                           F, W, sign, m, tb);
        return hipGetLastError();
    }
    const dim3 grid = (m.inner > 1) ? dim3(blocks(m.nfib), (unsigned)m.S) : dim3(blocks(m.nfib * m.S));
    if (m.S > 1) {
        hipLaunchKernelGGL(k_seg_ends<T>, grid, dim3(kBlk), 0, st, F, Yb, m, tb);
        hipLaunchKernelGGL(k_separators<T>, dim3(blocks(m.nfib)), dim3(kBlk), 0, st, F, Yb, m, tb);
    }
    hipLaunchKernelGGL(k_seg_final<T>, grid, dim3(kBlk), 0, st, F, W, sign, m, tb);
    return hipGetLastError();
}

template hipError_t launch_solve_partitioned<float>(float*, View3, int, SolveTables<float>, float*,
                                                    float*, float, hipStream_t);
template hipError_t launch_solve_partitioned<double>(double*, View3, int, SolveTables<double>,
                                                     double*, double*, double, hipStream_t);

}  // namespace mgr
