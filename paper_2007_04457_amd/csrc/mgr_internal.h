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
template <typename T>
struct DimTables {
    const T* w[3];
    const T* K[3];
};

// Arguments of the streaming level kernel (mgr_stream.hip).
template <typename T>
struct StreamArgs {
    const T* A;  // level grid input (u, or coefficients)
    View3 av;
    T* C;  // coefficient output (decomposition only)
    View3 cv;
    T* W;  // packed coarse values (decomposition only)
    View3 wv;
    T* F;  // packed load vector
    View3 fv;
    DimTables<T> tb;
    int write_coarse;  // also write u at coarse positions of C
    int chunk, nt1, nt2, nch;  // filled in by the launcher
};

// Segment length of the partitioned Thomas solve (mgr_solve.hip).
constexpr int kSeg = 32;

// Tables of the partitioned solve for one (level, dimension), n coarse nodes:
// per node the off-diagonals of M_{l-1} (sub couples i-1, sup couples i+1),
// the segment-local Thomas factors and the separator responses alpha/beta;
// per separator s = 1..S-1 the factors of the separator system.
template <typename T>
struct SolveTables {
    const T* sub;
    const T* sup;
    const T* lseg;
    const T* ipseg;
    const T* alpha;
    const T* beta;
    const T* sl;
    const T* sip;
    const T* su;
    int S;
};

template <typename T>
hipError_t launch_stream_level(StreamArgs<T> a, bool dec, hipStream_t st);
template <typename T>
hipError_t launch_stream_recon(StreamArgs<T> a, hipStream_t st);
template <typename T>
hipError_t launch_solve_partitioned(T* F, View3 fv, int d, SolveTables<T> tb, T* Yb, T* W, T sign,
                                    hipStream_t st);

// Kernel classes (for timing and profiling names).
enum KernelClass {
    KC_COEF = 0,
    KC_SOLVE,
    KC_INTERP,
    KC_MASSTRANS_T,
    KC_ADJ_COMBINE,
    KC_COPY_VIEW,
    KC_BENCH_COPY,
    KC_STREAM_DEC,
    KC_STREAM_LOAD,
    KC_COUNT
};

template <typename T>
hipError_t launch_coef_decompose(const T* A, View3 av, T* C, View3 cv, T* W, View3 wv,
                                 DimTables<T> tb, hipStream_t st);
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
