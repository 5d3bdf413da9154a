// General tensor grids: 1 to 4 dimensions of any size >= 3 per dimension.
//
// The paper's grids have 2^k + 1 nodes per dimension; for other sizes the
// nested level grids keep, along each dimension, the nodes at multiples of
// 2^k and the last node (a level grid of m nodes keeps its even positions and
// its last one as coarse nodes, so a level grid of even length has no fine
// node in its last interval).  The method's formulas are unchanged
// (Sec. II-A, Eq. (1)-(2)): coefficients by multilinear interpolation from
// the coarse corners, the load vector R M C applied one dimension at a time,
// the tridiagonal correction solve per dimension and the correction added to
// the coarse nodes.  Here each stage is its own kernel over packed level
// grids (the per-stage structure of the paper's GPK / LPK / IPK kernels,
// Sec. III-A), without the fused streaming of the 2^k + 1 path:
//   k_gen_coef      level grid -> coefficients (to the output array at their
//                   nodes) and the coarse values (packed, next level grid);
//   k_gen_masstrans one dimension of the load vector, reading either a
//                   packed array or the coefficients in the full array;
//   solves          the partitioned Thomas kernels of mgr_solve.hip;
//   k_gen_axpy      the correction added to (subtracted from) the coarse
//                   values;
//   k_gen_interp    recomposition: coarse values and interpolated
//                   coefficients back onto the level grid;
//   k_gen_scatter   the coarsest values to / from their nodes.
#include <algorithm>

#include "mgr_internal.h"

namespace mgr {
namespace {

constexpr int kGenBlock = 256;

// Level index j of a level grid of m nodes is fine-only: odd and not the
// last node.
__device__ __forceinline__ bool gen_fine(int64_t j, int64_t m) { return (j & 1) && j != m - 1; }
// Coarse-grid index of a coarse level index j.
__device__ __forceinline__ int64_t gen_coarse(int64_t j, int64_t m) { return (j == m - 1) ? (m >> 1) : (j >> 1); }

// Multi-index of a flat C-order index over a box of nd sizes.
__device__ __forceinline__ void gen_index(int nd, int64_t idx, const int64_t* m, int64_t* j)
{
#pragma unroll
    for (int d = kGenMaxDim - 1; d >= 0; d--) {
        if (d >= nd) continue;
        j[d] = idx % m[d];
        idx /= m[d];
    }
}

// Offset in the full array of level index j (level step k): the j-th
// multiple of 2^k, or the last node.
template <typename T>
__device__ __forceinline__ int64_t gen_full(const GenLevel<T>& a, const int64_t* j, int k)
{
    int64_t o = 0;
#pragma unroll
    for (int d = 0; d < kGenMaxDim; d++) {
        if (d >= a.nd) continue;
        const int64_t i = j[d] << k;
        o += (i < a.n[d] - 1 ? i : a.n[d] - 1) * a.st[d];
    }
    return o;
}

template <typename T>
__device__ __forceinline__ int64_t gen_flat(int nd, const int64_t* j, const int64_t* m)
{
    int64_t o = 0;
#pragma unroll
    for (int d = 0; d < kGenMaxDim; d++)
        if (d < nd) o = o * m[d] + j[d];
    return o;
}

// Multilinear interpolant at a node with fine dimensions `fine` from its
// coarse corners, values read by get(q): sum over the corners in the order of
// the corner mask (bit d: upper neighbour along d), each weighted by the
// product of its one-dimensional weights.
template <typename T, class Get>
__device__ __forceinline__ T gen_interp(const GenLevel<T>& a, const int64_t* j, const bool* fine, Get get)
{
    T acc = T(0);
    for (int mask = 0; mask < (1 << a.nd); mask++) {
        bool skip = false;
        T w = T(1);
        int64_t q[kGenMaxDim];
#pragma unroll
        for (int d = 0; d < kGenMaxDim; d++) {
            if (d >= a.nd) continue;
            const bool up = (mask >> d) & 1;
            if (!fine[d]) {
                skip = skip || up;
                q[d] = j[d];
            } else {
                q[d] = up ? j[d] + 1 : j[d] - 1;
                w *= up ? a.wh[d][j[d]] : a.wl[d][j[d]];
            }
        }
        if (!skip) acc = fma(w, get(q), acc);
    }
    return acc;
}

// Decomposition, level step k: input level grid X (level 0: the full array
// src; deeper: packed Wk), coefficients to dst at their nodes, coarse values
// packed to Wn.
template <typename T>
__global__ void __launch_bounds__(kGenBlock)
    k_gen_coef(const T* __restrict__ src, const T* __restrict__ Wk, T* __restrict__ dst, T* __restrict__ Wn,
               GenLevel<T> a, int k)
{
    int64_t V = 1;
    for (int d = 0; d < a.nd; d++) V *= a.m[d];
    const int64_t stride = (int64_t)gridDim.x * kGenBlock;
    for (int64_t idx = (int64_t)blockIdx.x * kGenBlock + threadIdx.x; idx < V; idx += stride) {
        int64_t j[kGenMaxDim] = {0, 0, 0, 0};
        gen_index(a.nd, idx, a.m, j);
        bool fine[kGenMaxDim] = {false, false, false, false};
        bool any = false;
        for (int d = 0; d < a.nd; d++) {
            fine[d] = gen_fine(j[d], a.m[d]);
            any = any || fine[d];
        }
        auto get = [&](const int64_t* q) { return k == 0 ? src[gen_full(a, q, 0)] : Wk[gen_flat<T>(a.nd, q, a.m)]; };
        const T u = get(j);
        if (!any) {
            int64_t c[kGenMaxDim] = {0, 0, 0, 0};
            for (int d = 0; d < a.nd; d++) c[d] = gen_coarse(j[d], a.m[d]);
            Wn[gen_flat<T>(a.nd, c, a.mc)] = u;
            continue;
        }
        dst[gen_full(a, j, k)] = u - gen_interp(a, j, fine, get);
    }
}

// One dimension d of the load vector: out (sizes sh with sh[d] = mc[d]) =
// K along d applied to in (sizes sh with sh[d] = m[d]).  K row i covers the
// five fine nodes f(i) - 2 .. f(i) + 2, f(i) = 2i or the last node.  With
// full != 0 the input is the level grid's coefficients read from the full
// array y (zero at coarse nodes); else the packed array in.
template <typename T>
__global__ void __launch_bounds__(kGenBlock)
    k_gen_masstrans(const T* __restrict__ in, const T* __restrict__ y, T* __restrict__ out, GenLevel<T> a, GenPass p,
                    int k)
{
    const int d = p.d;
    int64_t Vo = 1;
    for (int e = 0; e < a.nd; e++) Vo *= p.out[e];
    const int64_t stride = (int64_t)gridDim.x * kGenBlock;
    const T* K = a.K[d];
    const int64_t m = a.m[d], mc = a.mc[d];
    for (int64_t idx = (int64_t)blockIdx.x * kGenBlock + threadIdx.x; idx < Vo; idx += stride) {
        int64_t j[kGenMaxDim] = {0, 0, 0, 0};
        gen_index(a.nd, idx, p.out, j);
        const int64_t i = j[d];
        const int64_t f = (i == mc - 1) ? m - 1 : 2 * i;
        T acc = T(0);
        for (int t = 0; t < 5; t++) {
            const int64_t c = f - 2 + t;
            if (c < 0 || c >= m) continue;
            j[d] = c;
            T v;
            if (p.full) {
                bool any = false;
                for (int e = 0; e < a.nd; e++) any = any || gen_fine(j[e], a.m[e]);
                v = any ? y[gen_full(a, j, k)] : T(0);
            } else {
                v = in[gen_flat<T>(a.nd, j, p.in)];
            }
            acc = fma(K[5 * i + t], v, acc);
        }
        out[idx] = acc;
    }
}

// W += sign * Z over n packed values.
template <typename T>
__global__ void __launch_bounds__(kGenBlock) k_gen_axpy(T* __restrict__ W, const T* __restrict__ Z, int64_t n, T sign)
{
    const int64_t stride = (int64_t)gridDim.x * kGenBlock;
    for (int64_t i = (int64_t)blockIdx.x * kGenBlock + threadIdx.x; i < n; i += stride) W[i] = fma(sign, Z[i], W[i]);
}

// Recomposition, level step k: coarse values from the packed Wn (already
// corrected), fine nodes c + interpolant, c read from y at the node; output
// to dst at the nodes (k = 0) or packed into Wk.
template <typename T>
__global__ void __launch_bounds__(kGenBlock)
    k_gen_interp(const T* __restrict__ y, const T* __restrict__ Wn, T* __restrict__ dst, T* __restrict__ Wk,
                 GenLevel<T> a, int k)
{
    int64_t V = 1;
    for (int d = 0; d < a.nd; d++) V *= a.m[d];
    const int64_t stride = (int64_t)gridDim.x * kGenBlock;
    for (int64_t idx = (int64_t)blockIdx.x * kGenBlock + threadIdx.x; idx < V; idx += stride) {
        int64_t j[kGenMaxDim] = {0, 0, 0, 0};
        gen_index(a.nd, idx, a.m, j);
        bool fine[kGenMaxDim] = {false, false, false, false};
        bool any = false;
        for (int d = 0; d < a.nd; d++) {
            fine[d] = gen_fine(j[d], a.m[d]);
            any = any || fine[d];
        }
        auto coarse_val = [&](const int64_t* q) {
            int64_t c[kGenMaxDim] = {0, 0, 0, 0};
            for (int d = 0; d < a.nd; d++) c[d] = gen_coarse(q[d], a.m[d]);
            return Wn[gen_flat<T>(a.nd, c, a.mc)];
        };
        const T v = any ? y[gen_full(a, j, k)] + gen_interp(a, j, fine, coarse_val) : coarse_val(j);
        if (k == 0)
            dst[gen_full(a, j, 0)] = v;
        else
            Wk[idx] = v;
    }
}

// Coarsest grid (level step L, sizes a.m) between the full array and packed
// W: to_full: full[node] = W + Z (Z may be null); else W = full[node].
template <typename T>
__global__ void __launch_bounds__(kGenBlock)
    k_gen_scatter(T* __restrict__ full, T* __restrict__ W, const T* __restrict__ Z, GenLevel<T> a, int k, int to_full)
{
    int64_t V = 1;
    for (int d = 0; d < a.nd; d++) V *= a.m[d];
    const int64_t stride = (int64_t)gridDim.x * kGenBlock;
    for (int64_t idx = (int64_t)blockIdx.x * kGenBlock + threadIdx.x; idx < V; idx += stride) {
        int64_t j[kGenMaxDim] = {0, 0, 0, 0};
        gen_index(a.nd, idx, a.m, j);
        const int64_t o = gen_full(a, j, k);
        if (to_full)
            full[o] = Z ? W[idx] + Z[idx] : W[idx];
        else
            W[idx] = full[o];
    }
}

unsigned gen_blocks(int64_t n)
{
    const int64_t cap = (int64_t)device_cu_count() * 16;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kGenBlock - 1) / kGenBlock, cap));
}

int64_t box(int nd, const int64_t* m)
{
    int64_t v = 1;
    for (int d = 0; d < nd; d++) v *= m[d];
    return v;
}

}  // namespace

template <typename T>
hipError_t launch_gen_coef(const T* src, const T* Wk, T* dst, T* Wn, const GenLevel<T>& a, int k, hipStream_t st)
{
    hipLaunchKernelGGL(k_gen_coef<T>, dim3(gen_blocks(box(a.nd, a.m))), dim3(kGenBlock), 0, st, src, Wk, dst, Wn, a,
                       k);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gen_masstrans(const T* in, const T* y, T* out, const GenLevel<T>& a, const GenPass& p, int k,
                                hipStream_t st)
{
    hipLaunchKernelGGL(k_gen_masstrans<T>, dim3(gen_blocks(box(a.nd, p.out))), dim3(kGenBlock), 0, st, in, y, out, a,
                       p, k);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gen_axpy(T* W, const T* Z, int64_t n, T sign, hipStream_t st)
{
    hipLaunchKernelGGL(k_gen_axpy<T>, dim3(gen_blocks(n)), dim3(kGenBlock), 0, st, W, Z, n, sign);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gen_interp(const T* y, const T* Wn, T* dst, T* Wk, const GenLevel<T>& a, int k, hipStream_t st)
{
    hipLaunchKernelGGL(k_gen_interp<T>, dim3(gen_blocks(box(a.nd, a.m))), dim3(kGenBlock), 0, st, y, Wn, dst, Wk, a,
                       k);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gen_scatter(T* full, T* W, const T* Z, const GenLevel<T>& a, int k, bool to_full, hipStream_t st)
{
    hipLaunchKernelGGL(k_gen_scatter<T>, dim3(gen_blocks(box(a.nd, a.m))), dim3(kGenBlock), 0, st, full, W, Z, a, k,
                       to_full ? 1 : 0);
    return hipGetLastError();
}

#define MGR_GEN_INST(T)                                                                                          \
    template hipError_t launch_gen_coef<T>(const T*, const T*, T*, T*, const GenLevel<T>&, int, hipStream_t);  \
    template hipError_t launch_gen_masstrans<T>(const T*, const T*, T*, const GenLevel<T>&, const GenPass&, int, \
                                                hipStream_t);                                                    \
    template hipError_t launch_gen_axpy<T>(T*, const T*, int64_t, T, hipStream_t);                              \
    template hipError_t launch_gen_interp<T>(const T*, const T*, T*, T*, const GenLevel<T>&, int, hipStream_t); \
    template hipError_t launch_gen_scatter<T>(T*, T*, const T*, const GenLevel<T>&, int, bool, hipStream_t);
MGR_GEN_INST(float)
MGR_GEN_INST(double)

}  // namespace mgr
