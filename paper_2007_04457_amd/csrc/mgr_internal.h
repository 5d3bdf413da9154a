// Internal declarations shared by the host driver (mgr_api.cpp) and the
// gfx950 kernels (mgr_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mgr_queue.h"

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

// Two-point interpolation wl*a + wh*b with one fixed rounding order, shared
// by every kernel that forms the multilinear interpolant, so that different
// kernels computing the same coefficient agree bit for bit (the compiler
// would otherwise pick which product to fuse).
template <typename T>
__device__ __forceinline__ T lerp2(T wl, T a, T wh, T b)
{
    return fma(wh, b, wl * a);
}

// Arguments of the streaming level kernel (mgr_stream.hip).
template <typename T>
struct StreamArgs {
    const T* A;  // level grid input (u, or coefficients)
    const T* Z;  // decomposition: correction added to A on load (or null);
                 // recomposition: correction subtracted from W on load
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

// Segment length of the partitioned Thomas solve (mgr_solve.hip); segment
// tables are padded to kSlot entries.
constexpr int kSeg = 32;
constexpr int kSlot = kSeg + 1;

// Tables of the partitioned solve for one (level, dimension) with S segments:
// per segment s and slot q (index s * kSlot + q, zero past the segment) the
// local Thomas forward multipliers L, super-diagonal U, inverse pivots IP and
// separator responses A (left) and B (right); per separator k = 1..S-1 the
// matrix entries coupling it to its neighbours (ssub, ssup) and the Thomas
// factors of the separator system (sl, sip, su).
template <typename T>
struct SolveTables {
    const T* L;
    const T* U;
    const T* IP;
    const T* A;
    const T* B;
    const T* ssub;
    const T* ssup;
    const T* sl;
    const T* sip;
    const T* su;
    int S;
};

// In-place correction solve of F along dimension d.
template <typename T>
hipError_t launch_solve_partitioned(T* F, View3 fv, int d, SolveTables<T> tb, T* Yb, hipStream_t st);
// All active dimensions of a small coarse grid in one workgroup (order:
// dimensions dims[0], dims[1], ... of the nd listed), each fibre by the same
// segment arithmetic as launch_solve_partitioned; returns hipErrorNotSupported
// (launching nothing) unless every listed dimension is one segment long and
// the grid fits in the workgroup's LDS.
template <typename T>
hipError_t launch_solve_small(T* F, View3 fv, const int* dims, int nd, const SolveTables<T>* tb, hipStream_t st);
template <typename T>
bool solve_small_fits(View3 fv, const int* dims, int nd, const SolveTables<T>* tb);
// Dimensions 2 and then 1 of the packed array F (sizes fv, 3-D) in one
// launch, a workgroup per plane along dim 0, when its planes fit in LDS
// (solve_plane_fits); the values are those of launch_solve_partitioned along
// dimension 2 and then 1.
template <typename T>
bool solve_plane_fits(View3 fv, const SolveTables<T>& t2, const SolveTables<T>& t1);
template <typename T>
hipError_t launch_solve_plane(T* F, View3 fv, const SolveTables<T>& t2, const SolveTables<T>& t1, hipStream_t st);

// Single-workgroup kernel for the small coarse levels (mgr_tail.hip): all
// level steps k0 .. k0 + nlev - 1 in one launch, in LDS.  A level step may
// join it when its level grid, load-vector passes, correction and coarse
// values fit kTailDataElems elements and its tables kTailTabElems.
constexpr int kTailThreads = 1024;
constexpr int kMaxTail = 16;
constexpr int64_t kTailMaxNodes = 5000;
constexpr int kTailDataElems = 11264;
constexpr int kTailTabElems = 3200;

template <typename T>
struct TailLevel {
    int m[3], mc[3];  // level grid and coarse sizes (1 for inactive dims)
    DimTables<T> tb;  // interpolation weights and stencils
    const T* lf[3];   // plain Thomas factors of M_{l-1}: multipliers,
    const T* ip[3];   // inverse pivots
    const T* up[3];   // and super-diagonal
    T* Wk;            // packed level grid k in the workspace (k > 0)
};

template <typename T>
struct TailArgs {
    TailLevel<T> lv[kMaxTail];  // index k - k0
    int k0, nlev;
    int64_t st[3];  // element strides of the user arrays
    const T* src;   // user input
    T* dst;         // user output
    const T* Z0;    // decomposition: correction added to the level-k0 input (or null)
};

template <typename T>
hipError_t launch_tail(const TailArgs<T>& a, bool decompose, hipStream_t st);
// One workgroup per entry: dev_args[i] in device memory, applied to field
// field[i] of the per-field pointer tables src / dst (device memory).
template <typename T>
hipError_t launch_tail_batch(const TailArgs<T>* dev_args, const int* field, const T* const* src, T* const* dst,
                             int n, bool decompose, hipStream_t st);

template <typename T>
hipError_t launch_stream_level(StreamArgs<T> a, bool dec, hipStream_t st);

// Independent level steps in one launch.  A recomposition's corrections
// depend on the stored coefficients alone, so those of several level steps
// can share one grid: its blocks are split between up to kMultiLevels steps,
// each with the work split it would get alone and the same arithmetic.
constexpr int kMultiLevels = 6;
// Load vectors (no coefficients) of n level steps, all with the same active
// dimensions.
template <typename T>
hipError_t launch_stream_load_multi(const StreamArgs<T>* a, int n, hipStream_t st);
// Whether the solve along dimension d of a packed array of sizes fv takes a
// single-launch form that launch_solve_multi can share.
template <typename T>
bool solve_multi_fits(View3 fv, int d, const SolveTables<T>& tb);
// Solves along dimension d of n packed arrays F[i] (sizes fv[i], tables
// tb[i]), in place, each fitting solve_multi_fits; the values are those of
// launch_solve_partitioned.
template <typename T>
hipError_t launch_solve_multi(T* const* F, const View3* fv, int d, const SolveTables<T>* tb, int n,
                              hipStream_t st);
// One adjoint level step (mgr_adjoint.hip): g / gv the input at the level
// grid's fine nodes, y the solved corrections and G the coarse-node input
// (packed coarse grid yv), O / ov the level-grid output (not overlapping g).
template <typename T>
hipError_t launch_stream_adjoint(const T* g, View3 gv, const T* y, const T* G, View3 yv, T* O, View3 ov,
                                 DimTables<T> tb, hipStream_t st);
// Coarse rows and columns per decomposition tile (act1: the problem has a
// second active dimension; elem_bytes: 4 or 8; wide: the two-wave-wide 3-D
// geometry); workgroup id = (chunk * nt1 + t1) * nt2 + t2.
void level_tiling(bool act1, int elem_bytes, bool wide, int* kT1, int* kT2);
template <typename T>
hipError_t launch_stream_recon(StreamArgs<T> a, hipStream_t st);

constexpr unsigned kOut = 0x80000000u;  // buffer offset past every range: loads 0, stores dropped

// Marks a value the same in every lane (kept in scalar registers).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uni(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Raw buffer access (gfx9 descriptor): the hardware range check turns an
// offset at or past `bytes` into a load of zero or a dropped store.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, unsigned bytes)
{
    // base and size are wave-uniform; say so, or the compiler loops over lanes
    const unsigned long long b = (unsigned long long)base;
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    void* ub = (void*)(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(ub, (short)0, __builtin_amdgcn_readfirstlane((int)bytes), 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
// The same with a wave-uniform byte offset `so` added to the address (the
// instruction's scalar-offset field): one descriptor can then serve every row
// of a plane, the row's offset in a scalar register.  Masking by range works
// as above through the per-lane offset.
template <typename T>
__device__ __forceinline__ T buf_load_so(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned so);
template <>
__device__ __forceinline__ float buf_load_so<float>(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned so)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, __builtin_amdgcn_readfirstlane((int)so), 0));
}
template <>
__device__ __forceinline__ double buf_load_so<double>(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned so)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, __builtin_amdgcn_readfirstlane((int)so), 0));
}
// (All overloads of buf_store live here together: an overload declared in a
// nested namespace would hide these from code inside it.)
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_store_so(float v, __amdgpu_buffer_rsrc_t r, unsigned off, unsigned so)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off,
                                          __builtin_amdgcn_readfirstlane((int)so), 0);
}
__device__ __forceinline__ void buf_store_so(double v, __amdgpu_buffer_rsrc_t r, unsigned off, unsigned so)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, __builtin_amdgcn_readfirstlane((int)so),
                                          0);
}
// Non-temporal stores (cache policy bit 1, "nt"): for whole-line output that
// nothing in the call reads again.  Keeping such a stream out of the caches
// spares the next kernel the write-back of its dirty lines.  Stores that
// leave partial lines must not use them: the caches then stop merging the
// two halves of a line written by neighbouring workgroups.
__device__ __forceinline__ void buf_store_nt(float v, __amdgpu_buffer_rsrc_t r, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 2);
}
__device__ __forceinline__ void buf_store_nt(double v, __amdgpu_buffer_rsrc_t r, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 2);
}
// Workgroup barrier that waits only for this wave's LDS traffic.  HIP's
// __syncthreads() also drains outstanding global loads, which would stall a
// register prefetch at every barrier.  Used only where nothing needs global
// memory ordered across the barrier (each output is written by one thread
// and never read back inside the kernel).
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Consecutive workgroup ids are dealt round-robin to the 8 XCDs; renumber so
// each XCD works on a contiguous range of tiles: neighbouring tiles then share
// its L2, for halo re-reads and for the cache lines their stores split.
__device__ __forceinline__ int remap_xcd(int bid, int nb)
{
    const int nx = 8;
    const int lo = nb / nx, rem = nb % nx;
    const int x = bid % nx, local = bid / nx;
    return (x < rem) ? x * (lo + 1) + local : rem * (lo + 1) + (x - rem) * lo + local;
}

// ---- batched decomposition (mgr_batch.hip) ----------------------------------
// Work items: one workgroup's share of one stage of one level step of one
// field.  Items are grouped into waves (level step k, stage s) over all
// fields; one launch per wave, stream order between waves.
enum BatchItemType {
    BI_STREAM3 = 0,  // streaming level tile, 3-D problem, narrow tile geometry
    BI_STREAM2,      // 2-D problem (m0, 1, m2)
    BI_STREAM1,      // 1-D problem
    BI_ROWS,         // solve along the contiguous dimension, a block of rows
    BI_STRIDED,      // solve along a strided dimension, 16 fibres (S <= 16)
    BI_SEG_ENDS,     // long fibres, three phases (three waves)
    BI_SEPARATORS,
    BI_SEG_FINAL,
    BI_SCATTER,      // coarsest values W_L + z_{L-1} to their nodes (fields without a tail)
    BI_STREAM3W,     // streaming level tile, 3-D problem, wide tile geometry
    BI_COUNT
};

struct BatchItem {
    int type;
    int args;    // index into the stream or solve argument table
    int bx, by;  // the workgroup's share: stream tile id; solve block (x, y)
    int field;   // field index (for the caller's data pointers)
};

template <typename T>
struct BatchSolve {
    T* F;  // packed correction array of the level step
    int64_t n, inner, outer, nfib;
    SolveTables<T> tb;
    T* Yb;     // segment-end buffer of the three-phase form
    int rows;  // rows per item (contiguous dimension)
};

template <typename T>
struct BatchScatter {
    const T* W;  // packed coarsest grid
    const T* Z;  // correction of the last level step, same layout
    int64_t n[3];
    int64_t ds[3];  // strides of the coarsest nodes in the field's dst
};

template <typename T>
struct BatchKernelArgs {
    const BatchItem* items;
    const StreamArgs<T>* sargs;  // A == nullptr: read the field's src; C is the field's dst
    const BatchSolve<T>* solves;
    const BatchScatter<T>* scatters;
    const T* const* src;  // per field
    T* const* dst;
};

// Threads of a batch workgroup, and elements of a row block staged by a
// batched contiguous-dimension solve item.
constexpr int kThreadsBatch = 256;
constexpr int kBatchRowSpan = 4096;

// Per-call data pointers of a batch, uploaded by kernel arguments (kPtrChunk
// per launch): entries first .. first + n - 1 of the device pointer table.
constexpr int kPtrChunk = 128;
struct PtrChunk {
    void* p[kPtrChunk];
    int first, n;
};
hipError_t launch_set_ptrs(const PtrChunk& c, void** dst, hipStream_t st);

// Runs items [first, first + n) of the table dev_a->items, one workgroup each.
template <typename T>
hipError_t launch_batch_wave(const BatchKernelArgs<T>* dev_a, int first, int n, hipStream_t st);
// Persistent form: all items in one launch of `grid` workgroups through the
// queue of mgr_queue.h (the queue words zeroed first by a small kernel).
template <typename T>
hipError_t launch_batch_queue(const BatchKernelArgs<T>* dev_a, const QueueTables& qt, const QueueState& qs, int words,
                              int grid, unsigned limit, hipStream_t st);
template <typename T>
int batch_queue_slots();
int device_cu_count();

// Kernel classes (for timing and profiling names).
enum KernelClass {
    KC_COEF = 0,
    KC_SOLVE,
    KC_INTERP,
    KC_ADJOINT,
    KC_COPY_VIEW,
    KC_BENCH_COPY,
    KC_STREAM_DEC,
    KC_STREAM_LOAD,
    KC_TAIL,
    KC_BATCH,
    KC_COUNT
};

template <typename T>
hipError_t launch_coef_decompose(const T* A, View3 av, T* C, View3 cv, T* W, View3 wv,
                                 DimTables<T> tb, hipStream_t st);
template <typename T>
hipError_t launch_copy_view(const T* X, const T* Z, View3 xv, T* Y, View3 yv, hipStream_t st);

hipError_t launch_bench_copy(const void* src, void* dst, size_t nbytes, hipStream_t st);
// Y[i] = X(view xv)[i] + Z[i] and N[i] = -Y[i] for every node i of xv, with
// Z, Y, N packed (N may alias Z).
template <typename T>
hipError_t launch_add_split(const T* X, View3 xv, const T* Z, T* Y, T* N, hipStream_t st);

// Class-packed layout (mgr_packed.hip): grid sizes in the internal 3-D form,
// level count L and the start of every class segment off[0..L+1].
constexpr int kMaxClassLevels = 64;
struct PackArgs {
    int64_t n[3];
    int L;
    int64_t off[kMaxClassLevels + 2];
};
// pack: in-place layout src -> class-packed dst; else the inverse.
template <typename T>
hipError_t launch_pack(const T* src, T* dst, const PackArgs& a, bool pack, hipStream_t st);

// Quantisation of the classes (mgr_quant.hip): internal 3-D sizes, level
// count, layout, class segment starts (class-packed layout) and the bin width
// of every class.  seg / nseg are filled in by the launcher.
struct QuantArgs {
    int64_t n[3];
    int L;
    int packed;
    int64_t seg, nseg;
    int64_t off[kMaxClassLevels + 2];
    double bins[kMaxClassLevels + 1];
};
// quant: codes q <- y; else out <- dequantised q.  counter (device, may be
// null) receives the number of clamped codes.
template <typename T>
hipError_t launch_quant(const T* y, int* q, T* out, QuantArgs a, bool quant, unsigned long long* counter,
                        hipStream_t st);


// ---- general tensor grids (mgr_general.hip) ---------------------------------
// 1..4 dimensions of any size >= 3; level grids keep the multiples of 2^k and
// the last node along each dimension.
constexpr int kGenMaxDim = 4;
// One level step: full-array sizes and strides, level-grid and coarse sizes,
// and per dimension the interpolation weight pairs of the level grid's
// fine-only nodes (wl lower, wh upper neighbour, indexed by level index) and
// the load-vector rows K (5 per coarse node, fine nodes f(i) - 2 .. f(i) + 2).
template <typename T>
struct GenLevel {
    int nd;
    int64_t n[kGenMaxDim], st[kGenMaxDim];
    int64_t m[kGenMaxDim], mc[kGenMaxDim];
    const T* wl[kGenMaxDim];
    const T* wh[kGenMaxDim];
    const T* K[kGenMaxDim];
};
// One load-vector pass along dimension d: input and output box sizes; full:
// read the input from the full array (the level grid's coefficients).
struct GenPass {
    int d, full;
    int64_t in[kGenMaxDim], out[kGenMaxDim];
};
template <typename T>
hipError_t launch_gen_coef(const T* src, const T* Wk, T* dst, T* Wn, const GenLevel<T>& a, int k, hipStream_t st);
template <typename T>
hipError_t launch_gen_masstrans(const T* in, const T* y, T* out, const GenLevel<T>& a, const GenPass& p, int k,
                                hipStream_t st);
template <typename T>
hipError_t launch_gen_axpy(T* W, const T* Z, int64_t n, T sign, hipStream_t st);
template <typename T>
hipError_t launch_gen_interp(const T* y, const T* Wn, T* dst, T* Wk, const GenLevel<T>& a, int k, hipStream_t st);
template <typename T>
hipError_t launch_gen_scatter(T* full, T* W, const T* Z, const GenLevel<T>& a, int k, bool to_full, hipStream_t st);
// Partitioned solve of every fibre of length n along the middle index of a
// packed (outer, n, inner) box, in place; Yb as for launch_solve_partitioned.
template <typename T>
hipError_t launch_solve_fibres(T* F, int64_t n, int64_t inner, int64_t outer, SolveTables<T> tb, T* Yb,
                               hipStream_t st);

}  // namespace mgr
