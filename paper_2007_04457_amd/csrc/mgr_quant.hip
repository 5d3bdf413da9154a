// Quantisation of the refactored classes (include/mgr.h, mgr_quantize):
// the lossy-compression use of the refactoring quantises every coefficient
// class with its own bin width and keeps the integer codes (Sec. V).  The
// paper names the stage, not the quantiser; the one implemented is a uniform
// scalar quantiser per class:
//     code = round-half-even(y / b_c)   (in the data's precision, b_c rounded
//                                        to it first)
//     value = code * b_c
// with a quotient that is NaN or beyond +-(2^31 - 1) clamped (NaN to 0) and
// counted.
//
// Both layouts are handled.  In-place node order: the class of a node comes
// from the 2-adic valuations of its indices, and a work unit is one segment
// of one row, so the row's outer indices (and their valuation) are
// wave-uniform and no per-element division is needed.  Class-packed: the
// class of an element is the segment its position falls in.
#include <algorithm>

#include "mgr_internal.h"

namespace mgr {
namespace {

constexpr int kQuantBlock = 256;

__device__ __forceinline__ int val2(int64_t i, int cap)
{
    return (i == 0) ? cap : min(cap, (int)__builtin_ctzll((unsigned long long)i));
}

__device__ __forceinline__ float div_round(float y, float b) { return rintf(y / b); }
__device__ __forceinline__ double div_round(double y, double b) { return rint(y / b); }

// Code of one value; *clamped set when the rounded quotient is NaN or out of
// the int32 range that is kept symmetric.
template <typename T>
__device__ __forceinline__ int code_of(T y, T b, bool* clamped)
{
    const double r = (double)div_round(y, b);
    if (r != r) {
        *clamped = true;
        return 0;
    }
    if (r > 2147483647.0) {
        *clamped = true;
        return 2147483647;
    }
    if (r < -2147483647.0) {
        *clamped = true;
        return -2147483647;
    }
    return (int)r;
}

// One atomic per wave for the clamped count.
__device__ __forceinline__ void count_clamped(bool c, unsigned long long* counter)
{
    const unsigned long long m = __ballot(c);
    if (counter && m && (threadIdx.x & 63) == __builtin_ctzll(m)) atomicAdd(counter, (unsigned long long)__popcll(m));
}

template <typename T, bool kQuant>
__global__ void __launch_bounds__(kQuantBlock)
    k_quant_inplace(const T* __restrict__ y, int* __restrict__ q, T* __restrict__ out, QuantArgs a,
                    unsigned long long* counter)
{
    // unit = (row, segment of seg columns); rows are (i0, i1) of the internal 3-D form
    const int L = a.L;
    const int64_t n1 = a.n[1], n2 = a.n[2];
    const int64_t rows = a.n[0] * n1;
    const int64_t units = rows * a.nseg;
    const int wave = uni((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int64_t wstride = (int64_t)gridDim.x * (kQuantBlock / 64);
    bool clamped = false;
    for (int64_t u = (int64_t)blockIdx.x * (kQuantBlock / 64) + wave; u < units; u += wstride) {
        const int64_t row = u / a.nseg;  // wave-uniform
        const int64_t s = u - row * a.nseg;
        const int64_t i0 = row / n1, i1 = row - i0 * n1;
        const int vrow = min(val2(i0, L), val2(i1, L));
        const int64_t c0 = s * a.seg, c1 = min(c0 + a.seg, n2);
        const int64_t base = row * n2;
        for (int64_t i2 = c0 + lane; i2 < c1; i2 += 64) {
            const int cls = L - min(vrow, val2(i2, L));
            const T b = (T)a.bins[cls];
            if (kQuant) {
                q[base + i2] = code_of(y[base + i2], b, &clamped);
            } else {
                out[base + i2] = (T)q[base + i2] * b;
            }
        }
    }
    if (kQuant) count_clamped(clamped, counter);
}

template <typename T, bool kQuant>
__global__ void __launch_bounds__(kQuantBlock)
    k_quant_packed(const T* __restrict__ y, int* __restrict__ q, T* __restrict__ out, QuantArgs a,
                   unsigned long long* counter)
{
    const int64_t total = a.off[a.L + 1];
    const int64_t stride = (int64_t)gridDim.x * kQuantBlock;
    bool clamped = false;
    for (int64_t i = (int64_t)blockIdx.x * kQuantBlock + threadIdx.x; i < total; i += stride) {
        int cls = a.L;  // the finest class holds most elements: scan downwards
        while (i < a.off[cls]) cls--;
        const T b = (T)a.bins[cls];
        if (kQuant)
            q[i] = code_of(y[i], b, &clamped);
        else
            out[i] = (T)q[i] * b;
    }
    if (kQuant) count_clamped(clamped, counter);
}

__global__ void k_zero_u64(unsigned long long* p)
{
    if (threadIdx.x == 0) *p = 0ull;
}

}  // namespace

template <typename T>
hipError_t launch_quant(const T* y, int* q, T* out, QuantArgs a, bool quant, unsigned long long* counter,
                        hipStream_t st)
{
    // a grid of a few rounds of the chip's workgroup slots
    int64_t work;
    if (a.packed) {
        work = (a.off[a.L + 1] + kQuantBlock - 1) / kQuantBlock;
    } else {
        // segments of whole waves (64 columns), enough units to fill the chip
        const int64_t rows = a.n[0] * a.n[1];
        const int64_t want = (int64_t)device_cu_count() * 64;
        int64_t nseg = std::max<int64_t>(1, (want + rows - 1) / rows);
        int64_t seg = (a.n[2] + nseg - 1) / nseg;
        seg = std::max<int64_t>(64, (seg + 63) / 64 * 64);
        a.seg = seg;
        a.nseg = (a.n[2] + seg - 1) / seg;
        work = (rows * a.nseg + (kQuantBlock / 64) - 1) / (kQuantBlock / 64);
    }
    const int64_t cap = (int64_t)device_cu_count() * 32;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min(work, cap));
    if (quant && counter) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, counter);
    if (a.packed) {
        if (quant)
            hipLaunchKernelGGL((k_quant_packed<T, true>), dim3(blocks), dim3(kQuantBlock), 0, st, y, q, out, a,
                               counter);
        else
            hipLaunchKernelGGL((k_quant_packed<T, false>), dim3(blocks), dim3(kQuantBlock), 0, st, y, q, out, a,
                               counter);
    } else {
        if (quant)
            hipLaunchKernelGGL((k_quant_inplace<T, true>), dim3(blocks), dim3(kQuantBlock), 0, st, y, q, out, a,
                               counter);
        else
            hipLaunchKernelGGL((k_quant_inplace<T, false>), dim3(blocks), dim3(kQuantBlock), 0, st, y, q, out, a,
                               counter);
    }
    return hipGetLastError();
}

template hipError_t launch_quant<float>(const float*, int*, float*, QuantArgs, bool, unsigned long long*,
                                        hipStream_t);
template hipError_t launch_quant<double>(const double*, int*, double*, QuantArgs, bool, unsigned long long*,
                                         hipStream_t);

}  // namespace mgr
