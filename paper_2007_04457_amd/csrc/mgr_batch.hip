// Batched decomposition of many independent fields.
//
// The host lists every workgroup-sized piece of work of every field (the
// streaming level tiles and the correction-solve blocks of each level step)
// as an item, grouped into waves: wave (k, s) holds stage s of level step k
// of every field that has it (stage 0 the streaming pass, then the solves).
// One launch runs a wave, one workgroup per item, whatever its field, shape
// or dimensionality; stream order between the waves carries every
// dependency (stage s of a field needs its stage s - 1, level step k + 1
// needs the last solve of step k), so no workgroup ever waits for another.
// The whole sequence (a few dozen launches for any number of fields) is
// what a HIP graph captures.
#include "mgr_solve_dev.h"
#include "mgr_stream_dev.h"

namespace mgr {
namespace {

template <typename T>
union BatchSmem {
    LevelSmem<T, true, true, true, false> lv3;
    LevelSmem<T, true, true, true, true> lv3w;
    LevelSmem<T, true, false, true> lv2;
    LevelSmem<T, false, false, true> lv1;
    StridedSmem<T> str;
    RowsSmem<T, kBatchRowSpan, true> rows_t;
    RowsSmem<T, kBatchRowSpan, false> rows_g;
};

// The kernel's LDS (dynamic, sized to BatchSmem<T> at launch).  Each item
// type runs in a function of its own (not inlined), so that its registers
// are allocated on its own: the kernel's register budget is then set by the
// largest item, and items above it spill inside themselves only.
extern __shared__ __align__(16) unsigned char batch_lds[];

// Copy of a wave-uniform struct in scalar registers (the item functions
// reach their arguments through generic pointers, whose loads land in vector
// registers).
template <class S>
__device__ __forceinline__ S load_uniform(const S* p)
{
    static_assert(sizeof(S) % 4 == 0, "whole dwords");
    S out;
    int* o = reinterpret_cast<int*>(&out);
    const int* q = reinterpret_cast<const int*>(p);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(S) / 4); i++) o[i] = __builtin_amdgcn_readfirstlane(q[i]);
    return out;
}

// kWide: the tile geometry the plan chose (3-D only; the 2-D and 1-D
// geometry does not depend on it).
template <typename T, bool kAct0, bool kAct1, bool kWide>
__device__ __attribute__((noinline)) void exec_stream(const BatchKernelArgs<T>* A, const BatchItem* itp)
{
    auto& sm = *reinterpret_cast<LevelSmem<T, kAct0, kAct1, true, kWide>*>(batch_lds);
    const BatchItem it = load_uniform(itp);
    StreamArgs<T> a = load_uniform(A->sargs + it.args);
    if (!a.A) a.A = load_uniform(A->src + it.field);
    a.C = load_uniform(A->dst + it.field);
    // unit column strides: FP32 column pairs move in single 8-byte accesses
    const bool unit = a.av.s[2] == 1 && a.cv.s[2] == 1;
    if constexpr (cols_per_lane<T>() == 2) {
        if (unit) {
            if (a.Z)
                stream_level_tile<T, kAct0, kAct1, true, true, true, kWide>(a, it.bx, sm);
            else
                stream_level_tile<T, kAct0, kAct1, true, false, true, kWide>(a, it.bx, sm);
            return;
        }
    }
    if (a.Z)
        stream_level_tile<T, kAct0, kAct1, true, true, false, kWide>(a, it.bx, sm);
    else
        stream_level_tile<T, kAct0, kAct1, true, false, false, kWide>(a, it.bx, sm);
}

template <typename T>
__device__ __forceinline__ FibreMap fibre_map(const BatchSolve<T>& b)
{
    FibreMap m;
    m.n = b.n;
    m.inner = b.inner;
    m.outer = b.outer;
    m.nfib = b.nfib;
    m.S = b.tb.S;
    return m;
}

template <typename T>
__device__ __attribute__((noinline)) void exec_rows(const BatchKernelArgs<T>* A, const BatchItem* itp)
{
    const BatchItem it = load_uniform(itp);
    const BatchSolve<T> b = load_uniform(A->solves + it.args);
    const FibreMap m = fibre_map(b);
    const int64_t row0 = (int64_t)it.bx * b.rows;
    const int nrows = (int)min((int64_t)b.rows, m.nfib - row0);
    if (m.S <= kMaxSegWG)
        solve_rows_tile<T, kBatchRowSpan, true>(
            b.F, m, b.tb, row0, nrows, *reinterpret_cast<RowsSmem<T, kBatchRowSpan, true>*>(batch_lds));
    else
        solve_rows_tile<T, kBatchRowSpan, false>(
            b.F, m, b.tb, row0, nrows, *reinterpret_cast<RowsSmem<T, kBatchRowSpan, false>*>(batch_lds));
}

template <typename T>
__device__ __attribute__((noinline)) void exec_strided(const BatchKernelArgs<T>* A, const BatchItem* itp)
{
    const BatchItem it = load_uniform(itp);
    const BatchSolve<T> b = load_uniform(A->solves + it.args);
    const int tid = threadIdx.x;
    solve_strided_tile<T, 16, false>(b.F, fibre_map(b), b.tb, (int64_t)it.bx * 16, tid / 16, tid % 16, kThreads,
                                     tid, *reinterpret_cast<StridedSmem<T>*>(batch_lds));
}

template <typename T>
__device__ __attribute__((noinline)) void exec_phase(const BatchKernelArgs<T>* A, const BatchItem* itp)
{
    const BatchItem it = load_uniform(itp);
    const BatchSolve<T> b = load_uniform(A->solves + it.args);
    const FibreMap m = fibre_map(b);
    if (it.type == BI_SEG_ENDS)
        seg_ends_tile(b.F, b.Yb, m, b.tb, it.bx, it.by);
    else if (it.type == BI_SEPARATORS)
        separators_tile(b.F, b.Yb, m, b.tb, it.bx);
    else
        seg_final_tile(b.F, m, b.tb, it.bx, it.by);
}

template <typename T>
__device__ __attribute__((noinline)) void exec_scatter(const BatchKernelArgs<T>* A, const BatchItem* itp)
{
    const BatchItem it = load_uniform(itp);
    const BatchScatter<T> sc = load_uniform(A->scatters + it.args);
    T* dst = load_uniform(A->dst + it.field);
    const int64_t idx = (int64_t)it.bx * kThreads + threadIdx.x;
    if (idx >= sc.n[0] * sc.n[1] * sc.n[2]) return;
    const int64_t j2 = idx % sc.n[2], j1 = (idx / sc.n[2]) % sc.n[1], j0 = idx / (sc.n[1] * sc.n[2]);
    dst[j0 * sc.ds[0] + j1 * sc.ds[1] + j2 * sc.ds[2]] = sc.W[idx] + sc.Z[idx];
}

template <typename T>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_batch(const BatchKernelArgs<T>* __restrict__ A, int first)
{
    const BatchItem* itp = A->items + first + blockIdx.x;
    switch (itp->type) {
        case BI_STREAM3: exec_stream<T, true, true, false>(A, itp); break;
        case BI_STREAM3W: exec_stream<T, true, true, true>(A, itp); break;
        case BI_STREAM2: exec_stream<T, true, false, false>(A, itp); break;
        case BI_STREAM1: exec_stream<T, false, false, false>(A, itp); break;
        case BI_ROWS: exec_rows<T>(A, itp); break;
        case BI_STRIDED: exec_strided<T>(A, itp); break;
        case BI_SCATTER: exec_scatter<T>(A, itp); break;
        default: exec_phase<T>(A, itp); break;
    }
}

// Device side of the queue protocol (mgr_queue.h), run by a whole wave:
// every value it returns is wave-uniform (one lane does each atomic and the
// result is broadcast), so the loops and branches around it are uniform.
// The queue words are accessed with agent-scope atomics; polls are relaxed
// loads with a sleep between them.  An item and the items it depends on run
// on one XCD, under one L2: the producer's stores have reached that L2 when
// its counter moves (the caller waits for them), so no L2 write-back is
// needed.  The consumer must still drop its CU's L1, which may hold lines it
// read before the producer wrote them (a cache line can span the parts of
// two items); on this device only an agent-scope invalidation reaches the L1
// of a workgroup whose waves share one CU (a workgroup-scope one is a no-op
// there), and it also drops the XCD's clean L2 lines, never dirty ones.
struct DevQueueOps {
    __device__ static bool leader() { return (threadIdx.x & 63) == 0; }
    __device__ int load_relaxed(int* p) const
    {
        return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    __device__ void fence_acquire() const { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
    __device__ int fetch_add_relaxed(int* p, int v) const
    {
        int r = 0;
        if (leader()) r = __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return __builtin_amdgcn_readfirstlane(r);
    }
    // the caller has waited until every store of the item reached the L2
    __device__ void add_release(int* p, int v) const
    {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        if (leader()) (void)__hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ void store_relaxed(int* p, int v) const
    {
        if (leader()) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ void cas_relaxed(int* p, int expect, int v) const
    {
        if (leader())
            (void)__hip_atomic_compare_exchange_strong(p, &expect, v, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ void pause() const { __builtin_amdgcn_s_sleep(2); }
};

template <typename T>
__device__ __forceinline__ void run_item(const BatchKernelArgs<T>* A, const BatchItem* itp)
{
    switch (itp->type) {
        case BI_STREAM3: exec_stream<T, true, true, false>(A, itp); break;
        case BI_STREAM3W: exec_stream<T, true, true, true>(A, itp); break;
        case BI_STREAM2: exec_stream<T, true, false, false>(A, itp); break;
        case BI_STREAM1: exec_stream<T, false, false, false>(A, itp); break;
        case BI_ROWS: exec_rows<T>(A, itp); break;
        case BI_STRIDED: exec_strided<T>(A, itp); break;
        case BI_SCATTER: exec_scatter<T>(A, itp); break;
        default: exec_phase<T>(A, itp); break;
    }
}

// The persistent form: every workgroup takes items from the queue of the XCD
// it runs on until that queue is empty (or the run is aborted), waiting for
// each item's dependency group first.  The grid size is free (a workgroup
// takes an item only while it runs; workgroups are dealt to every XCD).
// Wave 0 takes and finishes items as a whole wave (the branch on the wave
// index is uniform); the position is broadcast through LDS and read back as
// a uniform value, so the loop's exit and every branch around its barriers
// are uniform: with a per-thread index the compiler may restructure the loop
// so that the lanes of one wave take different paths around a barrier, and
// the wave never reconverges.  After an item every thread waits until its
// own memory operations have completed (its stores are then in the L2), the
// barrier then lets wave 0 mark the item finished; wave 0's cache
// invalidation after the wait precedes the barrier that starts the next item
// for every thread (all waves of a workgroup share one CU and its L1).
template <typename T>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_batch_queue(const BatchKernelArgs<T>* __restrict__ A, QueueTables qt, QueueState qs, unsigned limit)
{
    __shared__ int s_item;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    unsigned xcc;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
    const int q = (int)(xcc & 0xfu) % qt.nq;
    int last_dg = -1;  // wave 0's
    for (;;) {
        if (wave == 0) {
            const int t = queue_take(qt, qs, q, limit, last_dg, DevQueueOps{});
            if (DevQueueOps::leader()) s_item = t;
        }
        __syncthreads();
        const int i = __builtin_amdgcn_readfirstlane(s_item);
        if (i < 0) break;
        run_item(A, A->items + qt.order[i]);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no memory operation moves below the wait
        __builtin_amdgcn_s_waitcnt(0);             // this wave's loads and stores completed
        __syncthreads();
        if (wave == 0) queue_finish(qt, qs, i, DevQueueOps{});
    }
}

__global__ void __launch_bounds__(256) k_zero_words(int* p, int n)
{
    for (int i = (int)(blockIdx.x * 256 + threadIdx.x); i < n; i += (int)(gridDim.x * 256)) p[i] = 0;
}

}  // namespace

int device_cu_count()
{
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cache[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cache[dev] = n;
    }
    return cache[dev];
}

// One wave of items: dev_a (device memory) lists them; this launch runs
// items [first, first + n).
template <typename T>
hipError_t launch_batch_wave(const BatchKernelArgs<T>* dev_a, int first, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch<T>, dim3((unsigned)n), dim3(kThreads), sizeof(BatchSmem<T>), st, dev_a, first);
    return hipGetLastError();
}

// Writes up to kPtrChunk pointers, passed by value, to dst.  A graph that
// captures the launch keeps the values in its kernel node, so each replay
// restores the pointers of the call that was captured, whatever calls ran
// in between.
__global__ void __launch_bounds__(64) k_set_ptrs(PtrChunk c, void** dst)
{
    for (int i = (int)threadIdx.x; i < c.n; i += 64) dst[c.first + i] = c.p[i];
}

hipError_t launch_set_ptrs(const PtrChunk& c, void** dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_ptrs, dim3(1), dim3(64), 0, st, c, dst);
    return hipGetLastError();
}

// The whole queue in one launch of `grid` workgroups, after zeroing the
// queue words (`words` ints from qs.next: next, abort, err, then done[]).
template <typename T>
hipError_t launch_batch_queue(const BatchKernelArgs<T>* dev_a, const QueueTables& qt, const QueueState& qs, int words,
                              int grid, unsigned limit, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)std::min(64, (words + 255) / 256)), dim3(256), 0, st, qs.abort,
                       words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_queue<T>, dim3((unsigned)grid), dim3(kThreads), sizeof(BatchSmem<T>), st, dev_a, qt, qs,
                       limit);
    return hipGetLastError();
}

// Workgroups of the queue kernel that the device holds at once.
template <typename T>
int batch_queue_slots()
{
    static int cache[2] = {0, 0};
    int& c = cache[sizeof(T) == 8 ? 1 : 0];
    if (c == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_queue<T>, kThreads, sizeof(BatchSmem<T>)) !=
                hipSuccess ||
            n <= 0)
            n = 1;
        c = n * device_cu_count();
    }
    return c;
}

template hipError_t launch_batch_queue<float>(const BatchKernelArgs<float>*, const QueueTables&, const QueueState&, int,
                                              int, unsigned, hipStream_t);
template hipError_t launch_batch_queue<double>(const BatchKernelArgs<double>*, const QueueTables&, const QueueState&,
                                               int, int, unsigned, hipStream_t);
template int batch_queue_slots<float>();
template int batch_queue_slots<double>();
template hipError_t launch_batch_wave<float>(const BatchKernelArgs<float>*, int, int, hipStream_t);
template hipError_t launch_batch_wave<double>(const BatchKernelArgs<double>*, int, int, hipStream_t);

}  // namespace mgr
