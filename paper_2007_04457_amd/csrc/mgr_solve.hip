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
#include <algorithm>
#include <cstring>

#include "mgr_solve_dev.h"

namespace mgr {
namespace {

template <typename T>
__global__ void __launch_bounds__(64 * kMaxSegWG)
k_solve_strided_wg(T* __restrict__ F, FibreMap m, SolveTables<T> tb)
{
    __shared__ StridedSmem<T> sm;
    const int s = __builtin_amdgcn_readfirstlane(threadIdx.y);
    // neighbouring fibre groups split cache lines of every segment row they
    // write: keep them on one XCD (one L2)
    const int bx = remap_xcd((int)blockIdx.x, (int)gridDim.x);
    solve_strided_tile<T, 64, true>(F, m, tb, (int64_t)bx * 64, s, (int)threadIdx.x, 64 * m.S,
                              (int)(threadIdx.y * 64 + threadIdx.x), sm);
}


// A workgroup takes blocks of whole rows (rows_per_block * S lanes), one
// after the other with the next block's loads in flight; a block's data are
// one contiguous span of F, staged through LDS with one pad element per 32
// so that each lane's segment reads are bank-conflict free.
template <typename T, int kSpan, bool kLdsTab>
__global__ void __launch_bounds__(kBlk)
k_solve_rows_wg(T* __restrict__ F, FibreMap m, SolveTables<T> tb, int rows_per_block)
{
    __shared__ RowsSmem<T, kSpan, kLdsTab> sm;
    solve_rows_loop<T, kSpan, kLdsTab>(F, m, tb, rows_per_block, sm);
}

// Rows launch with a span of kSpan elements per block.
template <typename T, int kSpan>
hipError_t launch_rows(T* F, const FibreMap& m, const SolveTables<T>& tb, hipStream_t st)
{
    // rows per block: as many as fit, but at most an even share of two
    // workgroups per CU, so that small levels still spread over the chip
    const int64_t share = (m.nfib + 2 * (int64_t)device_cu_count() - 1) / (2 * (int64_t)device_cu_count());
    const int rpb = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)(kBlk / m.S), (int64_t)(kSpan / m.n), share}));
    const int64_t nb = (m.nfib + rpb - 1) / rpb;
    // one round of resident workgroups, each looping over blocks
    static int occ_t = 0, occ_g = 0;
    const int res = (m.S <= kMaxSegWG) ? rows_resident(k_solve_rows_wg<T, kSpan, true>, occ_t)
                                       : rows_resident(k_solve_rows_wg<T, kSpan, false>, occ_g);
    const unsigned grid = (unsigned)std::min<int64_t>(nb, (int64_t)res * device_cu_count());
    if (m.S <= kMaxSegWG)
        hipLaunchKernelGGL((k_solve_rows_wg<T, kSpan, true>), dim3(grid), dim3(kBlk), 0, st, F, m, tb, rpb);
    else
        hipLaunchKernelGGL((k_solve_rows_wg<T, kSpan, false>), dim3(grid), dim3(kBlk), 0, st, F, m, tb, rpb);
    return hipGetLastError();
}

// Workgroups of the rows kernel one CU holds (cached per kernel).
template <typename K>
int rows_resident(K kern, int& cache)
{
    if (cache == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, kBlk, 0) != hipSuccess || n <= 0) n = 2;
        cache = n;
    }
    return cache;
}

template <typename T>
__global__ void __launch_bounds__(kBlk) k_seg_ends(const T* __restrict__ F, T* __restrict__ Yb, FibreMap m,
                                                   SolveTables<T> tb)
{
    seg_ends_tile(F, Yb, m, tb, (int)blockIdx.x, (int)blockIdx.y);
}

template <typename T>
__global__ void __launch_bounds__(kBlk) k_separators(T* __restrict__ F, const T* __restrict__ Yb, FibreMap m,
                                                     SolveTables<T> tb)
{
    separators_tile(F, Yb, m, tb, (int)blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(kBlk) k_seg_final(T* __restrict__ F, FibreMap m, SolveTables<T> tb)
{
    seg_final_tile(F, m, tb, (int)blockIdx.x, (int)blockIdx.y);
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kBlk - 1) / kBlk); }


// ---- small coarse grids: every dimension in one workgroup -----------------
// Once the coarse grid is a few ten thousand nodes, each of the per-dimension
// launches above is bound by its own latency (load, a short serial sweep,
// store).  This kernel keeps the grid in LDS and runs the dimensions one after
// the other, one fibre per lane, with each fibre solved by seg_solve exactly
// as above (one segment: no separators, and the separator terms the other
// kernels add are zero), so it yields the values of the per-dimension
// launches.
constexpr int kSmallThreads = 1024;

template <typename T>
struct SmallSolveArgs {
    T* F;
    int n[3];
    int nd, dims[3];
    const T* L[3];
    const T* U[3];
    const T* IP[3];
};

template <typename T>
__global__ void __launch_bounds__(kSmallThreads) k_solve_small(SmallSolveArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char small_lds[];
    T* const tab = reinterpret_cast<T*>(small_lds);  // [dim slot][L, U, IP][kSlot]
    T* const g = tab + 9 * kSlot;
    const int tid = threadIdx.x;
    const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
    const int V = n0 * n1 * n2;
    // the grid in batches of NB loads per lane, all in flight together
    // (indices clamped into the grid: the loads are unconditional); one
    // batch covers every grid that fits the LDS, and the tables are staged
    // after its loads are issued, so one memory latency covers all
    constexpr int NB = (sizeof(T) == 4) ? 40 : 20;
    for (int b0 = 0; b0 < V; b0 += NB * kSmallThreads) {
        T tmp[NB];
#pragma unroll
        for (int q = 0; q < NB; q++) tmp[q] = a.F[min(b0 + q * kSmallThreads + tid, V - 1)];
        if (b0 == 0)
            for (int e = tid; e < a.nd * 3 * kSlot; e += kSmallThreads) {
                const int dd = e / (3 * kSlot), w = (e / kSlot) % 3, q = e % kSlot;
                const T* src = (w == 0) ? a.L[dd] : (w == 1) ? a.U[dd] : a.IP[dd];
                tab[e] = src[q];
            }
#pragma unroll
        for (int q = 0; q < NB; q++)
            if (b0 + q * kSmallThreads + tid < V) g[b0 + q * kSmallThreads + tid] = tmp[q];
    }
    __syncthreads();
    const int cs[3] = {n1 * n2, n2, 1};
    for (int dd = 0; dd < a.nd; dd++) {
        const int d = a.dims[dd];
        const int n = a.n[d], sd = cs[d];
        // fibres along d, indexed by the other two coordinates (inner first)
        const int da = (d == 0) ? 1 : 0, db = (d == 2) ? 1 : 2;
        const int nb = a.n[db], nfib = a.n[da] * nb;
        const T* L = tab + (3 * dd + 0) * kSlot;
        const T* U = tab + (3 * dd + 1) * kSlot;
        const T* IP = tab + (3 * dd + 2) * kSlot;
        for (int f = tid; f < nfib; f += kSmallThreads) {
            T* p = g + (f / nb) * cs[da] + (f % nb) * cs[db];
            T v[kSlot];
#pragma unroll
            for (int q = 0; q < kSlot; q++) v[q] = p[min(q, n - 1) * sd];
            seg_solve(v, L, U, IP);
#pragma unroll
            for (int q = 0; q < kSlot; q++)
                if (q < n) p[q * sd] = v[q];
        }
        __syncthreads();
    }
    for (int e = tid; e < V; e += kSmallThreads) a.F[e] = g[e];
}

// Largest plane-solve workgroup: ten waves, so that the compiler may give a
// lane up to 168 registers (the FP64 kernel spilled at the 128 of 16 waves).
constexpr int kPlaneThreads = 640;

// Dimensions 2 and then 1 of a coarse grid whose planes (a fixed index along
// dim 0) fit in LDS: one workgroup per plane stages it, solves every row and
// then every column in LDS with the partitioned arithmetic of the
// per-dimension kernels (seg_solve, the separator system, seg_final: the same
// values), and writes it back, in one launch and one pass over the array
// instead of two.  One thread per (segment, fibre) task, fibres fastest, so
// that lanes read LDS at the fibres' stride (odd for 2^k + 1 sizes: no bank
// conflicts) or contiguously.
template <typename T>
struct PlaneSolveArgs {
    T* F;
    int n1, n2;
    SolveTables<T> tb[2];  // dimension 2, dimension 1
};

template <typename T>
__device__ __forceinline__ void plane_dim(T* P, T* end0, T* end1, const T* tab, const T* septab, int n, int S,
                                          int nf, int sd, int sf, int tid)
{
    // task tid: segment s of fibre f; fibre f starts at P[f sf], node i of it
    // is at P[f sf + i sd]
    const bool active = tid < S * nf;
    const int s = active ? tid / nf : 0, f = active ? tid % nf : 0;
    FibreMap m;
    m.n = n;
    m.S = S;
    int lo, len;
    seg_range(m, s, lo, len);
    T* const p = P + f * sf;
    T v[kSlot];
#pragma unroll
    for (int q = 0; q < kSlot; q++) v[q] = p[(lo + min(q, len - 1)) * sd];
    const T ylast = seg_solve(v, tab + 0 * kMaxSegWG * kSlot + s * kSlot, tab + 1 * kMaxSegWG * kSlot + s * kSlot,
                              tab + 2 * kMaxSegWG * kSlot + s * kSlot);
    if (active) {
        end0[s * nf + f] = v[0];
        end1[s * nf + f] = ylast;
    }
    __syncthreads();
    if (active && s == 0 && S > 1)
        sep_solve(S, p, (int64_t)kSeg * sd, end0 + f, end1 + f, nf, septab + 0 * kMaxSegWG,
                  septab + 1 * kMaxSegWG, septab + 2 * kMaxSegWG, septab + 3 * kMaxSegWG, septab + 4 * kMaxSegWG);
    __syncthreads();
    const T zl = (s > 0) ? p[(s * kSeg) * sd] : T(0);
    const T zr = (s < S - 1) ? p[((s + 1) * kSeg) * sd] : T(0);
    __syncthreads();  // every task has read its separators
    if (active) {
        const T* ta = tab + 3 * kMaxSegWG * kSlot + s * kSlot;
        const T* tb = tab + 4 * kMaxSegWG * kSlot + s * kSlot;
#pragma unroll
        for (int q = 0; q < kSlot; q++)
            if (q < len) p[(lo + q) * sd] = seg_final(v[q], ta[q], zl, tb[q], zr);
    }
    __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(kPlaneThreads) k_solve_plane(PlaneSolveArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char plane_lds[];
    constexpr int TAB = 5 * kMaxSegWG * kSlot, SEP = 5 * kMaxSegWG;
    T* const tab = reinterpret_cast<T*>(plane_lds);  // [dim][L, U, IP, A, B][segment][slot]
    T* const septab = tab + 2 * TAB;                  // [dim][sub, sup, sl, sip, su][separator]
    T* const end = septab + 2 * SEP;                  // [2][kPlaneThreads]
    T* const P = end + 2 * kPlaneThreads;             // the plane, n1 x n2
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int n1 = a.n1, n2 = a.n2, V = n1 * n2;
    T* const F = a.F + (int64_t)blockIdx.x * V;
    // the plane's loads first (one batch covers every plane that fits), the
    // tables' after them: one memory latency covers both
    constexpr int NB = (sizeof(T) == 4) ? 20 : 10;
    for (int b0 = 0; b0 < V; b0 += NB * nthr) {
        T tmp[NB];
#pragma unroll
        for (int q = 0; q < NB; q++) tmp[q] = F[min(b0 + q * nthr + tid, V - 1)];
        if (b0 == 0)
            for (int d = 0; d < 2; d++) {
                const SolveTables<T>& t = a.tb[d];
                for (int e = tid; e < t.S * kSlot; e += nthr) {
                    T* o = tab + d * TAB + e;
                    o[0 * kMaxSegWG * kSlot] = t.L[e];
                    o[1 * kMaxSegWG * kSlot] = t.U[e];
                    o[2 * kMaxSegWG * kSlot] = t.IP[e];
                    o[3 * kMaxSegWG * kSlot] = t.A[e];
                    o[4 * kMaxSegWG * kSlot] = t.B[e];
                }
                for (int e = tid; e < t.S; e += nthr) {
                    T* o = septab + d * SEP + e;
                    o[0 * kMaxSegWG] = t.ssub[e];
                    o[1 * kMaxSegWG] = t.ssup[e];
                    o[2 * kMaxSegWG] = t.sl[e];
                    o[3 * kMaxSegWG] = t.sip[e];
                    o[4 * kMaxSegWG] = t.su[e];
                }
            }
#pragma unroll
        for (int q = 0; q < NB; q++)
            if (b0 + q * nthr + tid < V) P[b0 + q * nthr + tid] = tmp[q];
    }
    __syncthreads();
    // rows (dimension 2): fibre f = row, node i at f n2 + i
    plane_dim(P, end, end + kPlaneThreads, tab, septab, n2, a.tb[0].S, n1, 1, n2, tid);
    // columns (dimension 1): fibre f = column, node i at i n2 + f
    plane_dim(P, end, end + kPlaneThreads, tab + TAB, septab + SEP, n1, a.tb[1].S, n2, n2, 1, tid);
    for (int e = tid; e < V; e += nthr) F[e] = P[e];
}

// Solves of several level steps along one dimension in one grid: block b
// belongs to the step l with start[l] <= b < start[l + 1].  Contiguous
// dimension: each block solves rpb[l] rows staged through LDS (the rows
// kernel's arithmetic); strided: 64 fibres, one wave per segment, waves past
// a step's segment count idle through the barriers.
template <typename T>
struct MultiSolve {
    T* F[kMultiLevels];
    FibreMap m[kMultiLevels];
    SolveTables<T> tb[kMultiLevels];
    int rpb[kMultiLevels];
    int start[kMultiLevels + 1];
    int n;
};
static_assert(sizeof(MultiSolve<double>) <= 4096, "fits the kernel argument segment");

template <typename T>
__device__ __forceinline__ int multi_entry(const MultiSolve<T>& a, int b)
{
    int l = 0;
    for (int i = 1; i < a.n; i++) l += (b >= a.start[i]) ? 1 : 0;
    return l;
}

template <typename T, int kSpan>
__global__ void __launch_bounds__(kBlk) k_solve_rows_multi(MultiSolve<T> a)
{
    __shared__ RowsSmem<T, kSpan, true> sm;
    const int b = (int)blockIdx.x;
    const int l = multi_entry(a, b);
    const FibreMap& m = a.m[l];
    const int64_t row0 = (int64_t)(b - a.start[l]) * a.rpb[l];
    const int nrows = (int)min((int64_t)a.rpb[l], m.nfib - row0);
    solve_rows_tile<T, kSpan, true>(a.F[l], m, a.tb[l], row0, nrows, sm);
}

// kMaxThr: the launch's bound (512 when every step has at most 8 segments,
// which leaves the compiler twice the registers of the 1024-thread form).
template <typename T, int kMaxThr>
__global__ void __launch_bounds__(kMaxThr) k_solve_strided_multi(MultiSolve<T> a)
{
    __shared__ StridedSmem<T> sm;
    const int b = remap_xcd((int)blockIdx.x, (int)gridDim.x);
    const int l = multi_entry(a, b);
    const int s = __builtin_amdgcn_readfirstlane(threadIdx.y);
    solve_strided_tile<T, 64, false>(a.F[l], a.m[l], a.tb[l], (int64_t)(b - a.start[l]) * 64, s, (int)threadIdx.x,
                                     (int)(64 * blockDim.y), (int)(threadIdx.y * 64 + threadIdx.x), sm);
}

}  // namespace

template <typename T>
bool solve_multi_fits(View3 fv, int d, const SolveTables<T>& tb)
{
    int64_t inner = 1;
    for (int e = d + 1; e < 3; e++) inner *= fv.n[e];
    if (tb.S < 1 || tb.S > kMaxSegWG) return false;
    return inner > 1 || fv.n[d] <= rows_span<T>();
}

template <typename T>
hipError_t launch_solve_multi(T* const* F, const View3* fv, int d, const SolveTables<T>* tb, int n, hipStream_t st)
{
    if (n < 1 || n > kMultiLevels) return hipErrorInvalidValue;
    MultiSolve<T> a;
    std::memset(&a, 0, sizeof(a));
    a.n = n;
    bool rows = false;
    int tot = 0, smax = 1;
    for (int i = 0; i < n; i++) {
        if (!solve_multi_fits<T>(fv[i], d, tb[i])) return hipErrorNotSupported;
        FibreMap& m = a.m[i];
        m.n = fv[i].n[d];
        m.inner = 1;
        m.outer = 1;
        for (int e = d + 1; e < 3; e++) m.inner *= fv[i].n[e];
        for (int e = 0; e < d; e++) m.outer *= fv[i].n[e];
        m.nfib = m.inner * m.outer;
        m.S = tb[i].S;
        if (i == 0) rows = m.inner == 1;
        if (rows != (m.inner == 1)) return hipErrorInvalidValue;
        a.F[i] = F[i];
        a.tb[i] = tb[i];
        a.start[i] = tot;
        if (rows) {
            // the per-level rows launch's block size
            const int64_t cus = 2 * (int64_t)device_cu_count();
            const int64_t share = (m.nfib + cus - 1) / cus;
            a.rpb[i] = (int)std::max<int64_t>(
                1, std::min<int64_t>({(int64_t)(kBlk / m.S), (int64_t)(rows_span<T>() / m.n), share}));
            tot += (int)((m.nfib + a.rpb[i] - 1) / a.rpb[i]);
        } else {
            a.rpb[i] = 64;
            tot += (int)((m.nfib + 63) / 64);
            smax = std::max(smax, m.S);
        }
    }
    for (int i = n; i <= kMultiLevels; i++) a.start[i] = tot;
    if (rows)
        hipLaunchKernelGGL((k_solve_rows_multi<T, rows_span<T>()>), dim3((unsigned)tot), dim3(kBlk), 0, st, a);
    else if (smax <= 8)
        hipLaunchKernelGGL((k_solve_strided_multi<T, 512>), dim3((unsigned)tot), dim3(64, (unsigned)smax), 0, st, a);
    else
        hipLaunchKernelGGL((k_solve_strided_multi<T, 64 * kMaxSegWG>), dim3((unsigned)tot), dim3(64, (unsigned)smax), 0,
                           st, a);
    return hipGetLastError();
}

template bool solve_multi_fits<float>(View3, int, const SolveTables<float>&);
template bool solve_multi_fits<double>(View3, int, const SolveTables<double>&);
template hipError_t launch_solve_multi<float>(float* const*, const View3*, int, const SolveTables<float>*, int,
                                              hipStream_t);
template hipError_t launch_solve_multi<double>(double* const*, const View3*, int, const SolveTables<double>*, int,
                                               hipStream_t);

// Solve along dimension d of the packed array F (shape fv.n), in place.  Yb
// is scratch of at least 2 * S * (number of fibres) elements.
template <typename T>
hipError_t launch_solve_partitioned(T* F, View3 fv, int d, SolveTables<T> tb, T* Yb, hipStream_t st)
{
    int64_t inner = 1, outer = 1;
    for (int e = d + 1; e < 3; e++) inner *= fv.n[e];
    for (int e = 0; e < d; e++) outer *= fv.n[e];
    return launch_solve_fibres<T>(F, fv.n[d], inner, outer, tb, Yb, st);
}

template <typename T>
hipError_t launch_solve_fibres(T* F, int64_t n, int64_t inner, int64_t outer, SolveTables<T> tb, T* Yb,
                               hipStream_t st)
{
    FibreMap m;
    m.n = n;
    m.inner = inner;
    m.outer = outer;
    m.nfib = m.inner * m.outer;
    m.S = tb.S;
    if (m.inner == 1 && m.S <= kBlk && m.n <= rows_span<T>()) {
        return launch_rows<T, rows_span<T>()>(F, m, tb, st);
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

// LDS the small-grid kernel may use on the current device (0: none).
template <typename T>
int small_solve_lds()
{
    static int max_lds[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (max_lds[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 65536;
        max_lds[dev] = v;
        if (v > 65536 &&
            hipFuncSetAttribute((const void*)k_solve_small<T>, hipFuncAttributeMaxDynamicSharedMemorySize, v) !=
                hipSuccess) {
            (void)hipGetLastError();  // not sticky: keep it from the next launch check
            max_lds[dev] = 65536;
        }
    }
    return max_lds[dev];
}

template <typename T>
size_t small_solve_bytes(View3 fv)
{
    return (9 * (size_t)kSlot + (size_t)(fv.n[0] * fv.n[1] * fv.n[2])) * sizeof(T);
}

template <typename T>
bool solve_small_fits(View3 fv, const int* dims, int nd, const SolveTables<T>* tb)
{
    if (nd < 1 || nd > 3) return false;
    for (int i = 0; i < nd; i++)
        if (tb[i].S != 1 || fv.n[dims[i]] > kSlot) return false;
    return small_solve_bytes<T>(fv) <= (size_t)small_solve_lds<T>();
}

template <typename T>
hipError_t launch_solve_small(T* F, View3 fv, const int* dims, int nd, const SolveTables<T>* tb, hipStream_t st)
{
    if (!solve_small_fits(fv, dims, nd, tb)) return hipErrorNotSupported;
    SmallSolveArgs<T> a;
    a.F = F;
    for (int d = 0; d < 3; d++) a.n[d] = (int)fv.n[d];
    a.nd = nd;
    for (int i = 0; i < nd; i++) {
        a.dims[i] = dims[i];
        a.L[i] = tb[i].L;
        a.U[i] = tb[i].U;
        a.IP[i] = tb[i].IP;
    }
    hipLaunchKernelGGL(k_solve_small<T>, dim3(1), dim3(kSmallThreads), small_solve_bytes<T>(fv), st, a);
    return hipGetLastError();
}

// LDS the plane-solve kernel may use on the current device (0: none).
template <typename T>
int plane_solve_lds()
{
    static int max_lds[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (max_lds[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 65536;
        max_lds[dev] = v;
        if (v > 65536 &&
            hipFuncSetAttribute((const void*)k_solve_plane<T>, hipFuncAttributeMaxDynamicSharedMemorySize, v) !=
                hipSuccess) {
            (void)hipGetLastError();  // not sticky: keep it from the next launch check
            max_lds[dev] = 65536;
        }
    }
    return max_lds[dev];
}

template <typename T>
size_t plane_solve_bytes(View3 fv)
{
    return (size_t)(10 * kMaxSegWG * kSlot + 10 * kMaxSegWG + 2 * kPlaneThreads + fv.n[1] * fv.n[2]) * sizeof(T);
}

template <typename T>
bool solve_plane_fits(View3 fv, const SolveTables<T>& t2, const SolveTables<T>& t1)
{
    if (fv.n[1] < 2 || fv.n[2] < 2 || t2.S < 1 || t1.S < 1 || t2.S > kMaxSegWG || t1.S > kMaxSegWG) return false;
    if (t2.S * fv.n[1] > kPlaneThreads || t1.S * fv.n[2] > kPlaneThreads) return false;
    if (fv.n[1] > kSlot * kMaxSegWG || fv.n[2] > kSlot * kMaxSegWG) return false;
    return plane_solve_bytes<T>(fv) <= (size_t)plane_solve_lds<T>();
}

template <typename T>
hipError_t launch_solve_plane(T* F, View3 fv, const SolveTables<T>& t2, const SolveTables<T>& t1, hipStream_t st)
{
    if (!solve_plane_fits<T>(fv, t2, t1)) return hipErrorNotSupported;
    PlaneSolveArgs<T> a;
    a.F = F;
    a.n1 = (int)fv.n[1];
    a.n2 = (int)fv.n[2];
    a.tb[0] = t2;
    a.tb[1] = t1;
    const int64_t tasks = std::max<int64_t>(t2.S * fv.n[1], t1.S * fv.n[2]);
    const unsigned thr = (unsigned)std::min<int64_t>(kPlaneThreads, std::max<int64_t>(64, (tasks + 63) / 64 * 64));
    hipLaunchKernelGGL(k_solve_plane<T>, dim3((unsigned)fv.n[0]), dim3(thr), plane_solve_bytes<T>(fv), st, a);
    return hipGetLastError();
}

template bool solve_plane_fits<float>(View3, const SolveTables<float>&, const SolveTables<float>&);
template bool solve_plane_fits<double>(View3, const SolveTables<double>&, const SolveTables<double>&);
template hipError_t launch_solve_plane<float>(float*, View3, const SolveTables<float>&, const SolveTables<float>&,
                                              hipStream_t);
template hipError_t launch_solve_plane<double>(double*, View3, const SolveTables<double>&,
                                               const SolveTables<double>&, hipStream_t);

template bool solve_small_fits<float>(View3, const int*, int, const SolveTables<float>*);
template bool solve_small_fits<double>(View3, const int*, int, const SolveTables<double>*);
template hipError_t launch_solve_small<float>(float*, View3, const int*, int, const SolveTables<float>*, hipStream_t);
template hipError_t launch_solve_small<double>(double*, View3, const int*, int, const SolveTables<double>*,
                                               hipStream_t);
template hipError_t launch_solve_fibres<float>(float*, int64_t, int64_t, int64_t, SolveTables<float>, float*,
                                               hipStream_t);
template hipError_t launch_solve_fibres<double>(double*, int64_t, int64_t, int64_t, SolveTables<double>, double*,
                                               hipStream_t);
template hipError_t launch_solve_partitioned<float>(float*, View3, int, SolveTables<float>, float*,
                                                    hipStream_t);
template hipError_t launch_solve_partitioned<double>(double*, View3, int, SolveTables<double>, double*,
                                                    hipStream_t);

}  // namespace mgr
