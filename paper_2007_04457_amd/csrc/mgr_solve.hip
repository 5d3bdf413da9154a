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

#include "mgr_solve_dev.h"

namespace mgr {
namespace {

template <typename T>
__global__ void __launch_bounds__(64 * kMaxSegWG)
k_solve_strided_wg(T* __restrict__ F, FibreMap m, SolveTables<T> tb)
{
    __shared__ StridedSmem<T> sm;
    const int s = __builtin_amdgcn_readfirstlane(threadIdx.y);
    solve_strided_tile<T, 64, true>(F, m, tb, (int64_t)blockIdx.x * 64, s, (int)threadIdx.x, 64 * m.S,
                              (int)(threadIdx.y * 64 + threadIdx.x), sm);
}


// A block takes whole rows (rows_per_block * S lanes); their data are one
// contiguous span of F, staged through LDS with one pad element per 32 so
// that each lane's segment reads are bank-conflict free.
template <typename T, bool kLdsTab>
__global__ void __launch_bounds__(kBlk)
k_solve_rows_wg(T* __restrict__ F, FibreMap m, SolveTables<T> tb, int rows_per_block)
{
    __shared__ RowsSmem<T, rows_span<T>(), kLdsTab> sm;
    const int64_t row0 = (int64_t)blockIdx.x * rows_per_block;
    const int nrows = (int)min((int64_t)rows_per_block, m.nfib - row0);
    solve_rows_tile<T, rows_span<T>(), kLdsTab>(F, m, tb, row0, nrows, sm);
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
    if (m.inner == 1 && m.S <= kBlk && m.n <= rows_span<T>()) {
        // rows per block: as many as fit, but at most an even share of two
        // workgroups per CU, so that small levels still spread over the chip
        const int64_t share = (m.nfib + 2 * (int64_t)device_cu_count() - 1) / (2 * (int64_t)device_cu_count());
        const int rpb = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)(kBlk / m.S), (int64_t)(rows_span<T>() / m.n), share}));
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
