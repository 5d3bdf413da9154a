// Streaming level kernel: one HBM pass per level step computes the
// coefficients (Sec. II-A.1) and the whole load vector f = R M vec(C)
// (Sec. II-A.2, merged mass-transfer stencil of Sec. III-A.2) along all
// dimensions.
//
// Layout of the work.  The level grid is (m0, m1, m2) with m2 contiguous; its
// coarse grid is (c0, c1, c2), c = (m + 1) / 2.  A workgroup owns a tile of
// kT1 x kT2 coarse columns (dims 1, 2) and a chunk of coarse planes along
// dim 0, and streams the fine planes of that chunk (plus a 2-plane halo).
// Each fine plane is staged in LDS with a 2-node halo; its coefficients are
// formed in LDS; the dim-2 and dim-1 stencils reduce it to a kT1 x kT2
// coarse plane; each thread keeps the running sums of the dim-0 stencil for
// its coarse column in registers, so the load vector is written once and
// nothing intermediate goes to HBM.  The next plane's values are loaded into
// registers while the current plane is processed.  Two-dimensional problems
// run as (m0, 1, m2), one-dimensional ones as (1, 1, m2).
//
// Planes are visited in the order e0, e0+2, e0+1, e0+4, e0+3, ... so that an
// odd plane is handled right after both even neighbours, whose 2-D
// interpolants (kept in LDS) it needs.  Interpolation is the separable
// evaluation of the multilinear form from the coarse nodes only.
//
// kDec = true : input u; writes coefficients (and, optionally, u at coarse
//               positions so that level-0 output rows are written whole), the
//               coarse values W and f.
// kDec = false: input already holds coefficients at fine-only nodes (values
//               at coarse positions are ignored); writes f only.
#include <cstring>

#include "mgr_stream_dev.h"

namespace mgr {
namespace {

template <typename T, bool kAct0, bool kAct1, bool kDec, bool kZ, bool kU>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(stream_min_waves<T, kDec, kZ>(), 8)))
k_stream_level(StreamArgs<T> a)
{
    __shared__ LevelSmem<T, kAct0, kAct1, kDec> sm;
    stream_level_tile<T, kAct0, kAct1, kDec, kZ, kU>(a, remap_xcd((int)blockIdx.x, (int)gridDim.x), sm);
}

// Tiles and plane chunks of one level step (filled into a); returns its
// workgroup count.
template <typename T, bool kAct0, bool kAct1, bool kDec, bool kZ, bool kU>
int level_cfg(StreamArgs<T>& a)
{
    using G = LevelGeom<kAct1, cols_per_lane<T>(), wide_tile<T, kDec>()>;
    const int c0 = (int)a.fv.n[0], c1 = (int)a.fv.n[1], c2 = (int)a.fv.n[2];
    a.nt1 = kAct1 ? (c1 + G::kT1 - 1) / G::kT1 : 1;
    a.nt2 = (c2 + G::kT2 - 1) / G::kT2;
    const int tiles = a.nt1 * a.nt2;
    int chunk = c0;
    if (kAct0) {
        // One round of resident workgroups: a second, partial round would
        // run latency-bound on a mostly idle chip.
        static int occ = 0;
        const int slots = resident_per_cu(k_stream_level<T, kAct0, kAct1, kDec, kZ, kU>, occ) * device_cu_count();
        const int nch = std::max(1, slots / tiles);
        chunk = (c0 + nch - 1) / nch;
        chunk = std::min(std::max(chunk, 2), kMaxChunk);
    }
    a.chunk = chunk;
    a.nch = kAct0 ? (c0 + chunk - 1) / chunk : 1;
    return tiles * a.nch;
}

template <typename T, bool kAct0, bool kAct1, bool kDec, bool kZ, bool kU>
hipError_t launch_level_cfg(StreamArgs<T> a, hipStream_t st)
{
    const int blocks = level_cfg<T, kAct0, kAct1, kDec, kZ, kU>(a);
    hipLaunchKernelGGL((k_stream_level<T, kAct0, kAct1, kDec, kZ, kU>), dim3((unsigned)blocks), dim3(kThreads), 0,
                       st, a);
    return hipGetLastError();
}

// Load-vector passes of several level steps in one grid: block b belongs to
// the step l with start[l] <= b < start[l + 1] and is that step's workgroup
// b - start[l].
template <typename T>
struct MultiStream {
    StreamArgs<T> a[kMultiLevels];
    int start[kMultiLevels + 1];
    int n;
};
static_assert(sizeof(MultiStream<double>) <= 4096, "fits the kernel argument segment");

template <typename T, bool kAct0, bool kAct1>
__global__ void __launch_bounds__(kThreads) k_stream_load_multi(MultiStream<T> m)
{
    __shared__ LevelSmem<T, kAct0, kAct1, false> sm;
    const int b = remap_xcd((int)blockIdx.x, (int)gridDim.x);
    int l = 0;
    for (int i = 1; i < m.n; i++) l += (b >= m.start[i]) ? 1 : 0;
    stream_level_tile<T, kAct0, kAct1, false, false, false>(m.a[l], b - m.start[l], sm);
}

template <typename T, bool kAct0, bool kAct1>
hipError_t launch_load_multi_cfg(const StreamArgs<T>* a, int n, hipStream_t st)
{
    MultiStream<T> m;
    std::memset(&m, 0, sizeof(m));
    m.n = n;
    int tot = 0;
    for (int i = 0; i < n; i++) {
        m.a[i] = a[i];
        m.start[i] = tot;
        tot += level_cfg<T, kAct0, kAct1, false, false, false>(m.a[i]);
    }
    for (int i = n; i <= kMultiLevels; i++) m.start[i] = tot;
    hipLaunchKernelGGL((k_stream_load_multi<T, kAct0, kAct1>), dim3((unsigned)tot), dim3(kThreads), 0, st, m);
    return hipGetLastError();
}

template <typename T, bool kAct0, bool kAct1, bool kU>
hipError_t launch_cfg_u(StreamArgs<T> a, bool dec, hipStream_t st)
{
    if (dec && a.Z) return launch_level_cfg<T, kAct0, kAct1, true, true, kU>(a, st);
    if (dec) return launch_level_cfg<T, kAct0, kAct1, true, false, kU>(a, st);
    return launch_level_cfg<T, kAct0, kAct1, false, false, kU>(a, st);
}

template <typename T, bool kAct0, bool kAct1>
hipError_t launch_cfg(StreamArgs<T> a, bool dec, hipStream_t st)
{
    // unit column stride of the input and (decomposing) of the coefficients:
    // FP32 column pairs then move in single 8-byte accesses
    const bool unit = a.av.s[2] == 1 && (!dec || a.cv.s[2] == 1);
    if constexpr (cols_per_lane<T>() == 2)
        if (unit) return launch_cfg_u<T, kAct0, kAct1, true>(a, dec, st);
    return launch_cfg_u<T, kAct0, kAct1, false>(a, dec, st);
}

}  // namespace

// Coarse rows and columns of a decomposition tile (for the batch's work
// items): narrow or wide geometry.
void level_tiling(bool act1, int elem_bytes, bool wide, int* kT1, int* kT2)
{
    constexpr int Cf = cols_per_lane<float>(), Cd = cols_per_lane<double>();
    if (!act1) {
        *kT1 = (elem_bytes == 4) ? LevelGeom<false, Cf, false>::kT1 : LevelGeom<false, Cd, false>::kT1;
        *kT2 = (elem_bytes == 4) ? LevelGeom<false, Cf, false>::kT2 : LevelGeom<false, Cd, false>::kT2;
    } else if (elem_bytes == 4) {
        *kT1 = wide ? LevelGeom<true, Cf, true>::kT1 : LevelGeom<true, Cf, false>::kT1;
        *kT2 = wide ? LevelGeom<true, Cf, true>::kT2 : LevelGeom<true, Cf, false>::kT2;
    } else {
        *kT1 = wide ? LevelGeom<true, Cd, true>::kT1 : LevelGeom<true, Cd, false>::kT1;
        *kT2 = wide ? LevelGeom<true, Cd, true>::kT2 : LevelGeom<true, Cd, false>::kT2;
    }
}

template <typename T>
hipError_t launch_stream_level(StreamArgs<T> a, bool dec, hipStream_t st)
{
    const bool act0 = a.av.n[0] > 1, act1 = a.av.n[1] > 1;
    if (act0 && act1) return launch_cfg<T, true, true>(a, dec, st);
    if (act0) return launch_cfg<T, true, false>(a, dec, st);
    if (!act1) return launch_cfg<T, false, false>(a, dec, st);
    return hipErrorInvalidValue;  // (1, m1, m2) is never formed by the driver
}

template <typename T>
hipError_t launch_stream_load_multi(const StreamArgs<T>* a, int n, hipStream_t st)
{
    if (n < 1 || n > kMultiLevels) return hipErrorInvalidValue;
    const bool act0 = a[0].av.n[0] > 1, act1 = a[0].av.n[1] > 1;
    for (int i = 1; i < n; i++)
        if ((a[i].av.n[0] > 1) != act0 || (a[i].av.n[1] > 1) != act1) return hipErrorInvalidValue;
    if (act0 && act1) return launch_load_multi_cfg<T, true, true>(a, n, st);
    if (act0) return launch_load_multi_cfg<T, true, false>(a, n, st);
    if (!act1) return launch_load_multi_cfg<T, false, false>(a, n, st);
    return hipErrorInvalidValue;
}

template hipError_t launch_stream_level<float>(StreamArgs<float>, bool, hipStream_t);
template hipError_t launch_stream_level<double>(StreamArgs<double>, bool, hipStream_t);
template hipError_t launch_stream_load_multi<float>(const StreamArgs<float>*, int, hipStream_t);
template hipError_t launch_stream_load_multi<double>(const StreamArgs<double>*, int, hipStream_t);

}  // namespace mgr
