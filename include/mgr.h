/*
 * mgr.h - C ABI of libmgr, the MI355X (gfx950) implementation of multigrid
 * hierarchical data refactoring (Chen et al., "Accelerating Multigrid-based
 * Hierarchical Scientific Data Refactoring on GPUs", arXiv 2007.04457).
 *
 * Data model (shared by every entry point)
 * -----------------------------------------
 *  - A field is a C-order array of `prod(shape)` elements of type `dtype`
 *    in device memory (HBM), `ndim` in 1..3, `shape[d] = 2^k_d + 1` with
 *    k_d >= 1 (the structured grids of Sec. II-A; shape[ndim-1] is the
 *    contiguous dimension).  One plane of the array (the contiguous row in
 *    1-D and 2-D, shape[1] * shape[2] elements in 3-D) must stay below 2 GiB:
 *    the kernels address within a plane with 32-bit byte offsets.
 *  - General grids: mgr_decompose, mgr_recompose, mgr_prepare,
 *    mgr_max_levels and mgr_class_map also take `ndim` up to 4 and any
 *    sizes >= 3 (the paper's grids are 2^k + 1 and it says nothing of
 *    others).  Along each dimension the level-k grid is then the nodes at
 *    multiples of 2^k plus the last node, ceil((n - 1) / 2^k) + 1 nodes: a
 *    level grid of m nodes keeps its even positions and its last one as
 *    coarse nodes.  The full decomposition stops when the shortest level grid
 *    has 3 nodes (L = min_d ceil(log2(n_d - 1)) - 1), and 0..L+1 level steps
 *    are accepted.  A node's class is L minus the finest level k <= L whose
 *    grid holds it in every dimension.  These shapes run per-stage kernels
 *    (no per-plane addressing limit); the other entry points refuse them with
 *    MGR_ERR_SHAPE.
 *  - `coords` describes node positions (nonuniform structured grids,
 *    Sec. II-A): NULL, or coords[d] == NULL, means uniform spacing along d;
 *    otherwise coords[d] is a HOST array of shape[d] strictly increasing
 *    doubles.  Only ratios of spacings matter.  The library reads them
 *    during the call only.
 *  - `nlevels` is the number of level steps L.  -1 selects the full
 *    decomposition, L = min_d k_d - 1, whose coarsest grid has 3 nodes along
 *    the shortest dimension; 0..min_d k_d are accepted (0 = identity copy).
 *    All dimensions coarsen together.
 *  - Refactored layout ("in-place node order", the same-shaped refactored
 *    grid of Sec. II-A, overall process): element i of the output belongs to
 *    node i.  Nodes whose indices are all multiples of 2^L hold the
 *    coarsest nodal values (class 0); any other node, with v the smallest
 *    2-adic valuation of its indices, holds its level coefficient (class
 *    L - v, L = finest).  mgr_class_map returns this class map.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every GPU
 *    entry point only enqueues work on it and returns; results are ready
 *    when the stream reaches that point.
 *  - `src` and `dst` are caller-owned device pointers of the same size;
 *    dst == src is allowed (in place); other overlaps are not.
 *  - The library owns its tables and workspace (device memory, cached per
 *    problem; released by mgr_finalize).  Calls that share a problem
 *    (dtype, shape, coords, nlevels) share its workspace, so they must be
 *    ordered on one stream.
 *
 * Errors: every int-returning function returns MGR_OK (0) or a positive
 * status; arguments are validated before anything is enqueued, no
 * exception crosses the ABI, and mgr_last_error() gives a detail string.
 */
#ifndef MGR_H
#define MGR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { MGR_F32 = 0, MGR_F64 = 1 } mgr_dtype;

enum {
    MGR_OK = 0,
    MGR_ERR_ARG = 1,      /* null pointer, bad ndim or dtype */
    MGR_ERR_SHAPE = 2,    /* a size below 3; for the entry points limited to 2^k + 1 grids, a
                             size not 2^k + 1 or ndim 4; a plane of 2 GiB or more */
    MGR_ERR_LEVELS = 3,   /* nlevels outside -1, 0..L+1 (L the full count) */
    MGR_ERR_COORDS = 4,   /* coordinates not strictly increasing or not finite */
    MGR_ERR_HIP = 5,      /* a HIP runtime call or kernel launch failed */
    MGR_ERR_ALLOC = 6,    /* device allocation failed or exceeds MGR_WORKSPACE_MAX */
    MGR_ERR_CAPTURE = 7   /* would allocate while `stream` is being captured */
};

/* Full level count for a shape (min_d k_d - 1 for 2^k + 1 sizes; general
 * grids as above), or minus a status. */
int mgr_max_levels(int ndim, const int64_t* shape);

/* Decomposition (refactoring), Sec. II-A, Eq. (1)-(2): for each level step,
 * finest first, the coefficients (I - Pi_{l-1}) Q_l u at the fine-only nodes
 * (multilinear interpolation from the coarse nodes, Sec. II-A.1), the load
 * vector f = R M vec(C) and the correction solve M_{l-1} z = f along every
 * dimension (Sec. II-A.2, Sec. III-A), and z added to the coarse nodes.
 * Reads src, writes the refactored layout to dst. */
int mgr_decompose(const void* src, void* dst, int dtype, int ndim,
                  const int64_t* shape, const double* const* coords,
                  int nlevels, void* stream);

/* Recomposition: the exact inverse of mgr_decompose, coarsest level first
 * (Sec. II-A, overall process). Reads a refactored array from src.
 * The finest level step's correction (load vector of the stored
 * coefficients and the solves) and the small coarsest levels run on two
 * library-owned streams of the current device, forked from `stream` and
 * joined back into it with events, concurrently with the coarser
 * corrections and interpolations on `stream`; the call may be captured into
 * a graph like any other (prepare the problem first with mgr_prepare, which
 * also creates those streams). Recompositions enqueued on different streams
 * share the two streams: their work there runs in enqueue order, and a
 * recomposition must not be enqueued from another thread while a
 * recomposition is being captured. */
int mgr_recompose(const void* src, void* dst, int dtype, int ndim,
                  const int64_t* shape, const double* const* coords,
                  int nlevels, void* stream);

/* Adjoint (transpose) of mgr_decompose under the Euclidean inner product of
 * the arrays: dst = D^T src.  Derived from Eq. (1)-(2); not in the paper.
 * Per level step, coarse to fine: y = M_{l-1}^{-1} g_c (tridiagonal solves),
 * t = (M P) y (transposed load-vector stencil), out_f = g_f + t at the
 * fine-only nodes, out_c = g_c - Pi^T out_f. */
int mgr_decompose_adjoint(const void* src, void* dst, int dtype, int ndim,
                          const int64_t* shape, const double* const* coords,
                          int nlevels, void* stream);

/* Adjoint (transpose) of mgr_recompose, i.e. the inverse transpose D^{-T} of
 * the decomposition, under the same inner product: dst = D^{-T} src.
 * Derived from Eq. (1)-(2); not in the paper.  Per level step, fine to
 * coarse: g_c' = g_c + Pi^T g_f (transposed interpolation), y = M_{l-1}^{-1}
 * g_c' (tridiagonal solves), out_f = g_f - (M P) y at the fine-only nodes;
 * the coarsest g_c' are the class-0 outputs.  dst == src is allowed. */
int mgr_recompose_adjoint(const void* src, void* dst, int dtype, int ndim,
                          const int64_t* shape, const double* const* coords,
                          int nlevels, void* stream);

/* Allocation-free decomposition, for callers that cannot allocate device
 * memory (code under stream capture, allocation-free serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, arithmetic and result
 * as mgr_decompose (bit for bit), but the problem's tables and workspace
 * live in one library-owned device array of MGR_NOALLOC_SCRATCH_BYTES per
 * device (held from the first call on a device until the process ends)
 * instead of the per-problem cache: the call never allocates device memory.
 * A problem whose tables plus decomposition workspace exceed the array is
 * refused with MGR_ERR_ALLOC before anything is enqueued (513^3 float32
 * needs about 152 MiB; 513^3 float64 does not fit).  Every call on a device
 * shares that device's array and the array keeps the last call's contents:
 * calls that overlap on one device (different streams, or threads) race.
 * The tables are copied into the array from host memory when the previous
 * call on the device was another problem. */
#define MGR_NOALLOC_SCRATCH_BYTES (256ull << 20)
int mgr_decompose_noalloc(const void* src, void* dst, int dtype, int ndim,
                          const int64_t* shape, const double* const* coords,
                          int nlevels, void* stream);

/* Builds and uploads the tables and allocates the workspace of a problem
 * (synchronously), and creates the recomposition's streams of the current
 * device, so that later calls on a capturing stream allocate and create
 * nothing.  Optional: the compute entry points prepare on first use, except
 * on a capturing stream (MGR_ERR_CAPTURE). */
int mgr_prepare(int dtype, int ndim, const int64_t* shape,
                const double* const* coords, int nlevels);

/* Writes the class id of every node (uint8, C order) to host memory out. */
int mgr_class_map(int ndim, const int64_t* shape, int nlevels, uint8_t* out);

/* ---- class-packed layout and progressive recomposition -------------------
 * The paper's use of the refactored data is to store and move coefficient
 * classes separately and to reconstruct a lower-fidelity approximation from
 * the coarsest classes alone (Sec. I; Sec. II-A, overall process).
 *
 * Class-packed layout: class 0 (the coarsest nodal values), then class 1,
 * ..., class L, each a contiguous segment holding its nodes in C order of
 * their grid indices (prod(shape) elements in all).  Class c >= 1 holds the
 * nodes of level grid c (indices multiples of 2^(L-c)) that are not on level
 * grid c - 1, so its segment length is |grid c| - |grid c-1|. */

/* Writes the L + 2 segment starts of the class-packed layout to the host
 * array offsets: class c occupies [offsets[c], offsets[c+1]), and
 * offsets[L+1] = prod(shape). */
int mgr_class_offsets(int ndim, const int64_t* shape, int nlevels, int64_t* offsets);

/* dst (class-packed) <- src (in-place node order), a permutation of the
 * elements; out of place (src != dst), device pointers, asynchronous on
 * `stream`. */
int mgr_pack_classes(const void* src, void* dst, int dtype, int ndim, const int64_t* shape, int nlevels,
                     void* stream);

/* dst (in-place node order) <- src (class-packed): the inverse permutation. */
int mgr_unpack_classes(const void* src, void* dst, int dtype, int ndim, const int64_t* shape, int nlevels,
                       void* stream);

/* Progressive recomposition: dst <- the nodal values of Q_level u (the L2
 * projection onto level `level`, Eq. (1)) at the level-`level` nodes, an
 * array of shape (shape[d] - 1) / 2^(L - level) + 1, from the classes
 * 0..level of a refactored array src; classes finer than `level` are never
 * read.  packed = 0: src is the in-place layout (prod(shape) elements);
 * packed = 1: src is the class-packed layout, of which only the first
 * offsets[level + 1] elements are read (a prefix holding just those classes
 * is enough).  level = L gives the full recomposition.  Uses the cached
 * plan of the level-`level` grid (prepare it like any problem before graph
 * capture: mgr_prepare on that shape, coordinates x[::2^(L-level)] and
 * `level` levels). */
int mgr_recompose_level(const void* src, void* dst, int dtype, int ndim, const int64_t* shape,
                        const double* const* coords, int nlevels, int level, int packed, void* stream);

/* ---- quantisation of the classes ----------------------------------------
 * The lossy-compression use of the refactoring quantises each coefficient
 * class with its own bin width and stores the integer codes (Sec. V; the
 * paper names the stage, not the quantiser).  Quantiser: uniform scalar per
 * class c with bin width b_c (one value per class 0..L, host doubles,
 * positive and finite):
 *     code  = round-half-even(y / b_c)  computed in the data's precision
 *             (b_c rounded to it first; IEEE division),
 *     value = code * b_c                 in the data's precision.
 * A rounded quotient that is NaN, or beyond +-(2^31 - 1), is clamped (NaN to
 * 0, else to +-(2^31 - 1)) and counted.  The class of an element is that of
 * its node (packed = 0, in-place node order) or of the segment it lies in
 * (packed = 1, class-packed layout); shape and nlevels are those of the
 * decomposition.  Device pointers, prod(shape) elements and int32 codes,
 * asynchronous on `stream`. */

/* Bin widths for a bound tol > 0 on the largest pointwise error of the
 * recomposition of the dequantised classes (exact arithmetic):
 * b_0 = 2 tol / (L + 1), b_c = 2 tol / ((L + 1)(1 + 3^ndim)) for c >= 1.
 * The class-0 values reach the field only through interpolation (max-norm
 * nonexpansive); a class-c error reaches it through the level-c interpolant
 * minus its L2 projection onto the coarser space (Eq. (1)), at most
 * (1 + 3^ndim) times its size.  Writes nlevels + 1 values to the host array
 * bins. */
int mgr_quant_bins(int ndim, int nlevels, double tol, double* bins);

/* codes <- quantised src.  nclamped: NULL, or a device pointer to one
 * unsigned 64-bit counter that receives the number of clamped codes (set to
 * zero, then accumulated, in stream order). */
int mgr_quantize(const void* src, int32_t* codes, int dtype, int ndim, const int64_t* shape, int nlevels,
                 int packed, const double* bins, unsigned long long* nclamped, void* stream);

/* dst <- dequantised codes. */
int mgr_dequantize(const int32_t* codes, void* dst, int dtype, int ndim, const int64_t* shape, int nlevels,
                   int packed, const double* bins, void* stream);

/* Human-readable name of a status code (static storage). */
const char* mgr_status_string(int status);

/* Detail of the last error on the calling thread (empty if none). */
const char* mgr_last_error(void);

/* Frees every cached table, workspace and timing event and the
 * recomposition's streams.  Not safe while work that uses them is still in
 * flight: synchronise first. */
void mgr_finalize(void);

/* Level steps whose level grid has at most `max_nodes` nodes run together in
 * one single-workgroup launch (the small coarse levels are launch-bound);
 * larger steps use one streaming launch plus one solve launch per
 * dimension.  Default 5000; 0 disables the combined launch.  Returns the
 * previous value.  Process-wide; affects calls enqueued afterwards. */
int64_t mgr_set_tail_max_nodes(int64_t max_nodes);

/* ---- batched decomposition ----------------------------------------------
 * Many independent fields (any mix of shapes, dimensionalities, coordinates
 * and level counts, one dtype) decomposed together: every workgroup-sized
 * piece of work (field, level step, stage, block) is a work item; the items
 * of one stage of one level step of all fields form a wave, run by one
 * launch with a workgroup per item, and a final launch runs every field's
 * small coarse levels.  A batch of any size is a few dozen launches, which
 * a HIP graph captures.  Results are bit-identical to mgr_decompose on each
 * field.  Batching is not in the paper (its large runs refactor independent
 * partitions side by side, Sec. IV-C); the autotuner follows its
 * model-then-measure tuning of launch shapes (Sec. III-C).
 *
 * Ownership: the plan owns its tables (its own copies, untouched by
 * mgr_finalize), per-field workspaces and a device table of data pointers;
 * all are allocated by mgr_batch_plan_create (synchronously), so
 * mgr_batch_decompose allocates nothing and may be captured into a HIP
 * graph.  Each call writes its src/dst pointers into the plan's table with
 * small kernels that carry them as launch arguments, so a captured graph
 * replays with the pointers of the call that was captured, whatever eager
 * calls ran in between; calls and replays on one plan share its workspace
 * and must be ordered on one stream. */
typedef struct mgr_batch_plan mgr_batch_plan;

/* Plans a batch of nfields fields: field f has ndim[f] dimensions, sizes
 * shapes[f][0..ndim[f]-1] (2^k+1), coordinates coords ? coords[f] : NULL (as
 * for mgr_decompose; host memory, read during the call) and level count
 * nlevels ? nlevels[f] : -1 (>= 1).  Writes the plan to *plan. */
int mgr_batch_plan_create(int nfields, const int* ndim, const int64_t* const* shapes,
                          const double* const* const* coords, const int* nlevels, int dtype,
                          mgr_batch_plan** plan);

/* dst[f] <- decomposition of src[f] for every field.  src and dst are HOST
 * arrays of nfields device pointers (read during the call); src[f] != dst[f]
 * (out of place).  Calls on one plan must be ordered on one stream. */
int mgr_batch_decompose(mgr_batch_plan* plan, const void* const* src, void* const* dst, void* stream);

/* Autotuner (the model-then-measure search of Sec. III-C): for each tile
 * geometry of the 3-D streaming items (narrow, wide; mgr_batch_set_tile:
 * only where a field is 3-D) and each launch form (waves, persistent;
 * mgr_batch_set_mode) it times five probe chunk
 * lengths (coarse planes per streaming item: 2, 4, 16, 64, 128) on these
 * fields, fits a transaction model time = a + x * bytes + y * items +
 * z * depth to them with non-negative constants (bytes: the streaming items'
 * traffic with their re-read plane halos; items: streaming items; depth: the
 * planes the longest streaming item of each level step streams, summed over
 * the level steps), ranks every chunk length 2..128 by the fitted model and
 * times the best top_k; the plan keeps the fastest (tile, form, chunk) measured,
 * with the persistent form's poll bound unchanged.  Synchronous; overwrites
 * dst. */
int mgr_batch_autotune(mgr_batch_plan* plan, const void* const* src, void* const* dst, void* stream,
                       int top_k);

/* The launch form the plan uses (0 waves, 1 persistent) and the fitted model
 * constants of the last autotune of each form, on the tile geometry it kept
 * (model: 8 doubles):
 * model[4 * form + i] = a (ms), x (ms per byte), y (ms per streaming item),
 * z (ms per plane of depth) (zeros for a form not tuned). */
int mgr_batch_tuning(const mgr_batch_plan* plan, int* persistent, double* model);

/* Current configuration: chunk length, kernel launches per call (besides
 * the pointer upload), work items. */
int mgr_batch_config(const mgr_batch_plan* plan, int* chunk, int* launches, int64_t* items);

/* Sets the chunk length (1..128) and rebuilds the work items. */
int mgr_batch_set_config(mgr_batch_plan* plan, int chunk);

/* Launch form of later mgr_batch_decompose calls on the plan (results are
 * bit for bit the same either way):
 *   persistent = 0: one launch per wave of items (the default);
 *   persistent = 1: one launch for every item of every field, whose
 *     workgroups take items from a queue in order and wait, before each, for
 *     the items it depends on (the previous stage of the same field): fields
 *     advance independently of each other.  Then one launch for the small
 *     coarse levels, as in the other form.  Each wait is bounded by
 *     poll_limit polls (0: the default, 2^20, a thousand times any legitimate wait on the
 *     96-field workload);
 *     a wait that runs out aborts the whole launch, which then ends, and
 *     mgr_batch_check reports it.  The queue words live in the plan, so the
 *     calls (and graph replays) on one plan must be ordered on one stream. */
int mgr_batch_set_mode(mgr_batch_plan* plan, int persistent, unsigned poll_limit);

/* Tile geometry of the plan's 3-D streaming items (the fine-level step of a
 * 3-D field): wide = 0 narrow tiles (8 x 30 coarse columns), wide = 1 wide
 * tiles (8 x 62 coarse columns, two per lane: fewer halo re-reads, fewer
 * items, more registers).  A new plan starts on the geometry the per-field
 * calls use for its dtype (narrow FP32, wide FP64).  Results are bit for bit
 * the same either way; mgr_batch_set_tile rebuilds the work items (wide must
 * be 0 or 1, else MGR_ERR_ARG); ordering as mgr_batch_set_config. */
int mgr_batch_tile(const mgr_batch_plan* plan, int* wide);
int mgr_batch_set_tile(mgr_batch_plan* plan, int wide);

/* Synchronises the device and reports whether the plan's last persistent run
 * aborted (MGR_ERR_HIP, with the work item in mgr_last_error) or not. */
int mgr_batch_check(mgr_batch_plan* plan);

/* Host check of the persistent form's scheduling protocol: builds the work
 * items, waves, queues (nqueues of them, 1..16: the device uses one per XCD)
 * and dependency groups of a batch of these fields on the host alone (no
 * device is used) and runs the same queue functions the kernel runs on
 * nthreads host threads standing in for workgroups (thread t serves queue
 * t mod nqueues), each item "executed" as a random delay.  The thread that
 * takes queue position stall_item (>= 0; -1 for none; positions number the
 * queues' items one queue after the other) stops without finishing it, as a
 * workgroup that never completes would.  Writes out[0] items run, out[1]
 * items that started before the items they depend on had finished, out[2]
 * the error word (1 + the position whose wait ran out, 0 if none), out[3]
 * positions never taken. */
int mgr_batch_queue_check(int nfields, const int* ndim, const int64_t* const* shapes, const int* nlevels, int dtype,
                          int chunk, int nqueues, int nthreads, unsigned poll_limit, int stall_item, uint64_t seed,
                          int64_t* out);

/* Frees the plan (hipFree waits for work still using it). */
void mgr_batch_plan_destroy(mgr_batch_plan* plan);

/* ---- measurement support ------------------------------------------------
 * The single-pass copy kernel the paper uses to define achievable
 * bandwidth (Sec. IV-C): dst[i] = src[i] for nbytes (a multiple of 16,
 * 16-byte aligned pointers). */
int mgr_bench_copy(const void* src, void* dst, size_t nbytes, void* stream);

/* Kernel timing: when enabled, every launch of kernel class `kernel` at
 * level step `level` (0 = finest) is bracketed by HIP events on the stream
 * it is launched on.  mgr_timing_read synchronises those events and returns
 * the summed duration (ms) and launch count since the last reset.
 * Kernel classes are listed by mgr_kernel_name(0..). */
int mgr_timing_enable(int kernel, int level);
int mgr_timing_disable(void);
int mgr_timing_read(double* total_ms, int64_t* launches);
const char* mgr_kernel_name(int kernel);

#ifdef __cplusplus
}
#endif
#endif
