// Class-packed layout of the refactored data (include/mgr.h,
// mgr_pack_classes): the paper stores and moves the coefficient classes
// separately and a reader may take only the coarsest ones (Sec. I; Sec. II-A,
// overall process).  Class 0 (the coarsest nodal values), then class 1, ...,
// class L, each a contiguous segment with its nodes in C order of their
// grid indices.
//
// Each thread handles one node of the in-place layout: its class c is read
// off the 2-adic valuations of its indices, and its rank inside the class
// segment has a closed form.  Class c >= 1 holds the nodes of level grid c
// (stride 2^(L-c)) that are not on level grid c - 1, i.e. whose level-c
// indices j are not all even; C order of the full grid restricted to them is
// C order of j, so
//     rank = lex(j) - #{all-even j' before j in C order},
// and the all-even count of a box (m0, m1, m2) before j is
//     E(j0) e1 e2 + [j0 even] (E(j1) e2 + [j1 even] E(j2)),
// with E(x) = (x + 1) / 2 even values in [0, x) and e_d = (m_d + 1) / 2.
// Class 0 is the coarsest grid itself: rank = lex(j).  Reads of the in-place
// array are coalesced; writes are sequential within a class segment (every
// other lane on even rows of the finest class).
#include "mgr_internal.h"

namespace mgr {
namespace {

constexpr int kPackBlock = 256;

__device__ __forceinline__ int v2(int64_t i, int cap)
{
    return (i == 0) ? cap : min(cap, (int)__builtin_ctzll((unsigned long long)i));
}

// Packed position of node (i0, i1, i2) of a grid of sizes n (internal 3-D
// form, inactive dims of size 1) decomposed with L level steps.
__device__ __forceinline__ int64_t packed_index(int64_t i0, int64_t i1, int64_t i2, const PackArgs& a)
{
    const int L = a.L;
    const int v = min(v2(i0, L), min(v2(i1, L), v2(i2, L)));
    const int64_t m0 = ((a.n[0] - 1) >> v) + 1, m1 = ((a.n[1] - 1) >> v) + 1, m2 = ((a.n[2] - 1) >> v) + 1;
    const int64_t j0 = i0 >> v, j1 = i1 >> v, j2 = i2 >> v;
    const int64_t lex = (j0 * m1 + j1) * m2 + j2;
    if (v >= L) return lex;  // class 0: the coarsest grid in C order
    const int64_t e1 = (m1 + 1) >> 1, e2 = (m2 + 1) >> 1;
    const int64_t ev = ((j0 + 1) >> 1) * e1 * e2 +
                       ((j0 & 1) ? 0 : (((j1 + 1) >> 1) * e2 + ((j1 & 1) ? 0 : ((j2 + 1) >> 1))));
    (void)m0;
    return a.off[L - v] + lex - ev;
}

template <typename T, bool kPack>
__global__ void __launch_bounds__(kPackBlock) k_pack(const T* __restrict__ src, T* __restrict__ dst, PackArgs a)
{
    const int64_t total = a.n[0] * a.n[1] * a.n[2];
    const int64_t stride = (int64_t)gridDim.x * kPackBlock;
    for (int64_t idx = (int64_t)blockIdx.x * kPackBlock + threadIdx.x; idx < total; idx += stride) {
        const int64_t i2 = idx % a.n[2];
        const int64_t t = idx / a.n[2];
        const int64_t i1 = t % a.n[1], i0 = t / a.n[1];
        const int64_t p = packed_index(i0, i1, i2, a);
        if (kPack)
            dst[p] = src[idx];
        else
            dst[idx] = src[p];
    }
}

}  // namespace

template <typename T>
hipError_t launch_pack(const T* src, T* dst, const PackArgs& a, bool pack, hipStream_t st)
{
    const int64_t total = a.n[0] * a.n[1] * a.n[2];
    int64_t b = (total + kPackBlock - 1) / kPackBlock;
    b = std::max<int64_t>(1, std::min<int64_t>(b, (int64_t)1 << 20));
    if (pack)
        hipLaunchKernelGGL((k_pack<T, true>), dim3((unsigned)b), dim3(kPackBlock), 0, st, src, dst, a);
    else
        hipLaunchKernelGGL((k_pack<T, false>), dim3((unsigned)b), dim3(kPackBlock), 0, st, src, dst, a);
    return hipGetLastError();
}

template hipError_t launch_pack<float>(const float*, float*, const PackArgs&, bool, hipStream_t);
template hipError_t launch_pack<double>(const double*, double*, const PackArgs&, bool, hipStream_t);

}  // namespace mgr
