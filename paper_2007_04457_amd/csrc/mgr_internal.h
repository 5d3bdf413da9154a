// Internal declarations shared by the host driver (mgr_api.cpp) and the
// gfx950 kernels (mgr_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mgr {

// Strided 3-D view: element (j0, j1, j2) lives at j0*s[0] + j1*s[1] + j2*s[2].
// Problems of fewer dimensions are padded with leading size-1 dimensions
// that never coarsen ("inactive").
struct View3 {
    int64_t n[3];
    int64_t s[3];
};

// Per-dimension device tables of one level step, in the working precision.
//   w  : interpolation weight pairs of the level grid; for an odd level
//        index j, w[2j] weights the lower coarse neighbour (1 - a_j) and
//        w[2j+1] the upper one (a_j).
//   K  : the merged mass-transfer stencil R M (Sec. III-A.2): 5 weights per
//        coarse node i, K[5i + t + 2] multiplying fine node 2i + t.
//   lf, ip, up : Thomas factors of the coarse mass matrix M_{l-1}: forward
//        multipliers, inverse pivots and super-diagonal.
template <typename T>
struct DimTables {
    const T* w[3];
    const T* K[3];
    const T* lf[3];
    const T* ip[3];
    const T* up[3];
};

// Kernel classes (for timing and profiling names).
enum KernelClass {
    KC_COEF = 0,
    KC_MASSTRANS,
    KC_SOLVE,
    KC_APPLY,
    KC_INTERP,
    KC_MASSTRANS_T,
    KC_ADJ_COMBINE,
    KC_COPY_VIEW,
    KC_BENCH_COPY,
    KC_COUNT
};

template <typename T>
hipError_t launch_coef_decompose(const T* A, View3 av, T* C, View3 cv, T* W, View3 wv,
                                 DimTables<T> tb, hipStream_t st);
template <typename T>
hipError_t launch_masstrans(const T* X, View3 xv, T* Y, View3 yv, int d, const T* K,
                            int mask_coarse, hipStream_t st);
template <typename T>
hipError_t launch_solve(T* F, View3 fv, int d, const T* lf, const T* ip, const T* up,
                        hipStream_t st);
template <typename T>
hipError_t launch_apply(T* W, const T* F, int64_t n, T sign, hipStream_t st);
template <typename T>
hipError_t launch_interp_recompose(const T* C, View3 cv, T* Out, View3 ov, const T* W,
                                   View3 wv, DimTables<T> tb, hipStream_t st);
template <typename T>
hipError_t launch_masstrans_t(const T* Y, View3 yv, T* X, View3 xv, int d, const T* K,
                              const T* add, View3 addv, int use_add, hipStream_t st);
template <typename T>
hipError_t launch_adj_combine(const T* Tb, View3 tv, T* Out, View3 ov, const T* G,
                              View3 gv, DimTables<T> tb, hipStream_t st);
template <typename T>
hipError_t launch_copy_view(const T* X, View3 xv, T* Y, View3 yv, hipStream_t st);

hipError_t launch_bench_copy(const void* src, void* dst, size_t nbytes, hipStream_t st);

}  // namespace mgr
