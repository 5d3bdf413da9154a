// gfx950 kernels of the multigrid refactoring path (arXiv 2007.04457,
// Sec. II-A and III-A).  All kernels are memory bound; none is a dense
// contraction, so nothing here uses MFMA.
//
// Every kernel works on strided 3-D views (mgr::View3) of either the caller's
// array at the stride 2^k of level step k, or packed workspace arrays.
#include "mgr_internal.h"

namespace mgr {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ void decode3(int64_t idx, const int64_t* n, int64_t* j)
{
    j[2] = idx % n[2];
    int64_t t = idx / n[2];
    j[1] = t % n[1];
    j[0] = t / n[1];
}

__device__ __forceinline__ int64_t at(const View3& v, int64_t j0, int64_t j1, int64_t j2)
{
    return j0 * v.s[0] + j1 * v.s[1] + j2 * v.s[2];
}

inline unsigned grid_for(int64_t total)
{
    int64_t b = (total + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > (int64_t)1 << 22) b = (int64_t)1 << 22;  // grid-stride beyond this
    return (unsigned)b;
}

// Interpolation corners of level-grid node j: per dimension the lower and
// upper coarse neighbour and their weights (an even index is its own corner
// with weight 1 and a zero-weight upper duplicate).
template <typename T>
struct Corners {
    int64_t lo[3], hi[3];
    T wl[3], wh[3];
};

template <typename T>
__device__ __forceinline__ void corners(const int64_t* j, const DimTables<T>& tb, Corners<T>& c)
{
#pragma unroll
    for (int d = 0; d < 3; d++) {
        if (j[d] & 1) {
            c.lo[d] = j[d] - 1;
            c.hi[d] = j[d] + 1;
            c.wl[d] = tb.w[d][2 * j[d]];
            c.wh[d] = tb.w[d][2 * j[d] + 1];
        } else {
            c.lo[d] = j[d];
            c.hi[d] = j[d];
            c.wl[d] = T(1);
            c.wh[d] = T(0);
        }
    }
}

// Multilinear interpolation from the coarse corners, evaluated separably
// (along dim 2, then 1, then 0).  `half` maps level-grid corner indices to
// a packed coarse array (index / 2) when set.
template <typename T, bool kHalf>
__device__ __forceinline__ T interp_corners(const T* __restrict__ A, const View3& av,
                                            const Corners<T>& c)
{
    T r0[2];
#pragma unroll
    for (int a = 0; a < 2; a++) {
        int64_t i0 = a ? c.hi[0] : c.lo[0];
        T r1[2];
#pragma unroll
        for (int b = 0; b < 2; b++) {
            int64_t i1 = b ? c.hi[1] : c.lo[1];
            int64_t l2 = c.lo[2], h2 = c.hi[2];
            int64_t q0 = kHalf ? i0 >> 1 : i0, q1 = kHalf ? i1 >> 1 : i1;
            T vlo = A[at(av, q0, q1, kHalf ? l2 >> 1 : l2)];
            T vhi = (h2 != l2) ? A[at(av, q0, q1, kHalf ? h2 >> 1 : h2)] : T(0);
            r1[b] = lerp2(c.wl[2], vlo, c.wh[2], vhi);
            if (c.hi[1] == c.lo[1]) { r1[1] = T(0); break; }
        }
        r0[a] = lerp2(c.wl[1], r1[0], c.wh[1], r1[1]);
        if (c.hi[0] == c.lo[0]) { r0[1] = T(0); break; }
    }
    return lerp2(c.wl[0], r0[0], c.wh[0], r0[1]);
}

// Coefficients (Sec. II-A.1) of one level step: c(p) = u(p) - Pi u(p) at
// fine-only nodes, written to C; coarse values copied packed to W.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_coef_decompose(const T* A, View3 av, T* C, View3 cv,  // A and C may alias (in place)
                 T* __restrict__ W, View3 wv, DimTables<T> tb, int64_t total)
{
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kBlock) {
        int64_t j[3];
        decode3(idx, av.n, j);
        T u = A[at(av, j[0], j[1], j[2])];
        if (((j[0] | j[1] | j[2]) & 1) == 0) {
            W[at(wv, j[0] >> 1, j[1] >> 1, j[2] >> 1)] = u;
            continue;
        }
        Corners<T> c;
        corners(j, tb, c);
        C[at(cv, j[0], j[1], j[2])] = u - interp_corners<T, false>(A, av, c);
    }
}

// Y = X (+ Z, with Z laid out like X when given): gathers and scatters of
// the coarsest grid between the caller's array and the workspace.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_copy_view(const T* __restrict__ X, const T* __restrict__ Z, View3 xv, T* __restrict__ Y, View3 yv,
            int64_t total)
{
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kBlock) {
        int64_t j[3];
        decode3(idx, yv.n, j);
        const int64_t xo = at(xv, j[0], j[1], j[2]);
        Y[at(yv, j[0], j[1], j[2])] = Z ? X[xo] + Z[xo] : X[xo];
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_add_split(const T* __restrict__ X, View3 xv, const T* Z, T* __restrict__ Y, T* N, int64_t total)
{
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kBlock) {
        int64_t j[3];
        decode3(idx, xv.n, j);
        const T v = X[at(xv, j[0], j[1], j[2])] + Z[idx];
        Y[idx] = v;
        N[idx] = -v;
    }
}

__global__ void __launch_bounds__(kBlock)
k_bench_copy(const uint4* __restrict__ s, uint4* __restrict__ d, int64_t n16)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n16;
         i += (int64_t)gridDim.x * kBlock)
        d[i] = s[i];
}

inline int64_t vol(const View3& v) { return v.n[0] * v.n[1] * v.n[2]; }

}  // namespace

template <typename T>
hipError_t launch_coef_decompose(const T* A, View3 av, T* C, View3 cv, T* W, View3 wv,
                                 DimTables<T> tb, hipStream_t st)
{
    int64_t total = vol(av);
    hipLaunchKernelGGL(k_coef_decompose<T>, dim3(grid_for(total)), dim3(kBlock), 0, st, A, av,
                       C, cv, W, wv, tb, total);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_copy_view(const T* X, const T* Z, View3 xv, T* Y, View3 yv, hipStream_t st)
{
    int64_t total = vol(yv);
    hipLaunchKernelGGL(k_copy_view<T>, dim3(grid_for(total)), dim3(kBlock), 0, st, X, Z, xv, Y,
                       yv, total);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_add_split(const T* X, View3 xv, const T* Z, T* Y, T* N, hipStream_t st)
{
    const int64_t total = vol(xv);
    hipLaunchKernelGGL(k_add_split<T>, dim3(grid_for(total)), dim3(kBlock), 0, st, X, xv, Z, Y, N, total);
    return hipGetLastError();
}

hipError_t launch_bench_copy(const void* src, void* dst, size_t nbytes, hipStream_t st)
{
    int64_t n16 = (int64_t)(nbytes / 16);
    hipLaunchKernelGGL(k_bench_copy, dim3(grid_for(n16)), dim3(kBlock), 0, st,
                       (const uint4*)src, (uint4*)dst, n16);
    return hipGetLastError();
}

#define MGR_INSTANTIATE(T)                                                                      \
    template hipError_t launch_coef_decompose<T>(const T*, View3, T*, View3, T*, View3,         \
                                                 DimTables<T>, hipStream_t);                    \
    template hipError_t launch_copy_view<T>(const T*, const T*, View3, T*, View3, hipStream_t);      \
    template hipError_t launch_add_split<T>(const T*, View3, const T*, T*, T*, hipStream_t);

MGR_INSTANTIATE(float)
MGR_INSTANTIATE(double)

}  // namespace mgr
