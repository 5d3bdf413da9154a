// Small coarse levels in one workgroup, entirely in LDS.
//
// Once the level grid is small (a few thousand nodes) every stage of a level
// step is latency bound and a separate launch per stage costs more than the
// work.  This kernel runs all remaining level steps (decomposition: the
// finest of them first; recomposition: the coarsest first) in one workgroup
// of kTailThreads lanes with the level grid, the load-vector passes, the
// correction and the coarse values, and the level's tables, held in LDS.
// Global memory is touched only at the boundary: the input level grid, the
// coefficients of each level (written to / read from the caller's array at
// stride 2^k) and the coarsest values.
//
// The stages are those of Sec. II-A in the paper's order: coefficients by
// multilinear interpolation from the coarse nodes (Sec. II-A.1), the load
// vector R M vec(C) one dimension at a time (Sec. II-A.2, merged stencil of
// Sec. III-A.2), the tridiagonal correction solves (plain Thomas, one lane
// per fibre) and the correction applied to the coarse nodes.
#include "mgr_internal.h"

namespace mgr {
namespace {

constexpr int kT = kTailThreads;
constexpr int kTB = 6;  // grid loads in flight per lane

struct TailShape {
    int m[3], mc[3];
    int V, Vc;
};

__device__ __forceinline__ TailShape shape_of(const int* m, const int* mc)
{
    TailShape s;
    for (int d = 0; d < 3; d++) {
        s.m[d] = m[d];
        s.mc[d] = mc[d];
    }
    s.V = m[0] * m[1] * m[2];
    s.Vc = mc[0] * mc[1] * mc[2];
    return s;
}

__device__ __forceinline__ void dec3(int idx, const int* n, int& j0, int& j1, int& j2)
{
    j2 = idx % n[2];
    const int t = idx / n[2];
    j1 = t % n[1];
    j0 = t / n[1];
}

// Per-level tables staged in LDS (offsets into the table area).
template <typename T>
struct LdsTab {
    T* w[3];   // interpolation weight pairs, 2 m
    T* K[3];   // stencil, 5 mc
    T* lf[3];  // Thomas multipliers, mc
    T* ip[3];  // inverse pivots, mc
    T* up[3];  // super-diagonal, mc
};

template <typename T>
__device__ LdsTab<T> stage_tables(const TailLevel<T>& L, T* stab)
{
    // Layout per active dimension: w (2 m), K (5 mc), lf, ip, up (mc each).
    // All tables are copied in one pass over their concatenation, one
    // element per lane and round, so a level costs one memory latency here
    // rather than one per table.
    LdsTab<T> t;
    const T* src[15];  // segment 5 d + j (empty for inactive dimensions)
    int len[15], off = 0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const bool act = L.m[d] > 1;
        const int m = act ? L.m[d] : 0, mc = act ? L.mc[d] : 0;
        t.w[d] = stab + off;
        t.K[d] = t.w[d] + 2 * m;
        t.lf[d] = t.K[d] + 5 * mc;
        t.ip[d] = t.lf[d] + mc;
        t.up[d] = t.ip[d] + mc;
        src[5 * d + 0] = L.tb.w[d];
        len[5 * d + 0] = 2 * m;
        src[5 * d + 1] = L.tb.K[d];
        len[5 * d + 1] = 5 * mc;
        src[5 * d + 2] = L.lf[d];
        len[5 * d + 2] = mc;
        src[5 * d + 3] = L.ip[d];
        len[5 * d + 3] = mc;
        src[5 * d + 4] = L.up[d];
        len[5 * d + 4] = mc;
        off += 2 * m + 8 * mc;
    }
    for (int e0 = 0; e0 < off; e0 += kT) {
        const int e = e0 + threadIdx.x;
        // the element's source, selected over the (unrolled) segment list
        const T* ps = nullptr;
        int base = 0;
#pragma unroll
        for (int sg = 0; sg < 15; sg++) {
            if (e >= base && e < base + len[sg]) ps = src[sg] + (e - base);
            base += len[sg];
        }
        if (e < off) stab[e] = *ps;
    }
    return t;
}

// Multilinear interpolation at level-grid node (j0, j1, j2) from coarse
// values: in U itself (coarse nodes at even indices, stride (m1*m2, m2, 1))
// or, with kHalf, from the packed coarse array W (index / 2).
template <typename T, bool kHalf>
__device__ __forceinline__ T tail_interp(const T* A, const TailShape& s, const LdsTab<T>& t, int j0,
                                         int j1, int j2)
{
    const int n1 = kHalf ? s.mc[1] : s.m[1], n2 = kHalf ? s.mc[2] : s.m[2];
    const int o0 = j0 & 1, o1 = j1 & 1, o2 = j2 & 1;
    const T a0 = o0 ? t.w[0][2 * j0] : T(1), b0 = o0 ? t.w[0][2 * j0 + 1] : T(0);
    const T a1 = o1 ? t.w[1][2 * j1] : T(1), b1 = o1 ? t.w[1][2 * j1 + 1] : T(0);
    const T a2 = o2 ? t.w[2][2 * j2] : T(1), b2 = o2 ? t.w[2][2 * j2 + 1] : T(0);
    const int l0 = j0 - o0, h0 = j0 + o0, l1 = j1 - o1, h1 = j1 + o1, l2 = j2 - o2, h2 = j2 + o2;
    auto at = [&](int x, int y, int z) {
        return kHalf ? A[((x >> 1) * n1 + (y >> 1)) * n2 + (z >> 1)] : A[(x * n1 + y) * n2 + z];
    };
    auto row = [&](int x, int y) { return a2 * at(x, y, l2) + (o2 ? b2 * at(x, y, h2) : T(0)); };
    const T lo = a1 * row(l0, l1) + (o1 ? b1 * row(l0, h1) : T(0));
    const T hi = o0 ? a1 * row(h0, l1) + (o1 ? b1 * row(h0, h1) : T(0)) : T(0);
    return a0 * lo + b0 * hi;
}

// f = R M vec(U) with U's coarse nodes read as zero; passes last dim first.
template <typename T>
__device__ void lds_load_vector(const T* U, T* P1, T* P2, T* F, const TailShape& s,
                                const LdsTab<T>& t)
{
    int sh[3] = {s.m[0], s.m[1], s.m[2]};
    const T* in = U;
    int npass = 0, done = 0;
#pragma unroll
    for (int d = 0; d < 3; d++) npass += (s.m[d] > 1);
#pragma unroll
    for (int d = 2; d >= 0; d--) {
        if (s.m[d] == 1) continue;
        const int ish[3] = {sh[0], sh[1], sh[2]};
        sh[d] = s.mc[d];
        T* out = (done == npass - 1) ? F : (done == 0 ? P1 : P2);
        const int total = sh[0] * sh[1] * sh[2];
        const int is[3] = {ish[1] * ish[2], ish[2], 1};
        for (int idx = threadIdx.x; idx < total; idx += kT) {
            int o[3];
            dec3(idx, sh, o[0], o[1], o[2]);
            const int i = o[d];
            int oth = 0;
#pragma unroll
            for (int e = 0; e < 3; e++)
                if (e != d) oth |= o[e];
            const bool mask = (done == 0) && ((oth & 1) == 0);
            T acc = T(0);
            for (int tt = -2; tt <= 2; tt++) {
                const int jd = 2 * i + tt;
                if (jd < 0 || jd >= ish[d]) continue;
                if (mask && !(tt & 1)) continue;  // coarse node: C is zero there
                int q = 0;
#pragma unroll
                for (int e = 0; e < 3; e++) q += ((e == d) ? jd : o[e]) * is[e];
                acc += t.K[d][5 * i + tt + 2] * in[q];
            }
            out[idx] = acc;
        }
        __syncthreads();
        in = out;
        done++;
    }
}

// Plain Thomas solves on F along every active dimension (last first), then
// W += sign * F.
template <typename T>
__device__ void lds_solve_apply(T* F, T* W, T sign, const TailShape& s, const LdsTab<T>& t)
{
    const int cs[3] = {s.mc[1] * s.mc[2], s.mc[2], 1};
#pragma unroll
    for (int d = 2; d >= 0; d--) {
        if (s.m[d] == 1) continue;
        const int da = (d == 0) ? 1 : 0, db = (d == 2) ? 1 : 2;
        const int n = s.mc[d], nfib = s.mc[da] * s.mc[db];
        const T* lf = t.lf[d];
        const T* ip = t.ip[d];
        const T* up = t.up[d];
        for (int f = threadIdx.x; f < nfib; f += kT) {
            const int ja = f / s.mc[db], jb = f % s.mc[db];
            T* p = F + ja * cs[da] + jb * cs[db];
            const int sd = cs[d];
            T g = p[0];
            for (int i = 1; i < n; i++) {
                g = p[i * sd] - lf[i] * g;
                p[i * sd] = g;
            }
            T z = g * ip[n - 1];
            p[(n - 1) * sd] = z;
            for (int i = n - 2; i >= 0; i--) {
                z = (p[i * sd] - up[i] * z) * ip[i];
                p[i * sd] = z;
            }
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < s.Vc; q += kT) W[q] += sign * F[q];
    __syncthreads();
}

// LDS regions sized for the first (largest) tail level.
template <typename T>
struct Regions {
    T *U, *P1, *P2, *F, *W;
};

template <typename T>
__device__ Regions<T> carve(T* sbuf, const TailLevel<T>& L0)
{
    const TailShape s = shape_of(L0.m, L0.mc);
    int sh[3] = {s.m[0], s.m[1], s.m[2]};
    int sz[2] = {0, 0}, k = 0;
#pragma unroll
    for (int d = 2; d >= 0; d--) {
        if (k >= 2) break;
        if (s.m[d] == 1) continue;
        sh[d] = s.mc[d];
        sz[k++] = sh[0] * sh[1] * sh[2];
    }
    Regions<T> r;
    r.U = sbuf;
    r.P1 = r.U + s.V;
    r.P2 = r.P1 + sz[0];
    r.F = r.P2 + sz[1];
    r.W = r.F + s.Vc;
    return r;
}

template <typename T, bool kDec>
__device__ __forceinline__ void tail_body(const TailArgs<T>& a, const T* src, T* dst, T* sbuf, T* stab)
{
    const Regions<T> R = carve(sbuf, a.lv[0]);
    const int64_t* st = a.st;

    if (kDec) {
        // input level grid k0: the caller's array (k0 == 0) or workspace
        {
            const TailLevel<T>& L = a.lv[0];
            const TailShape s = shape_of(L.m, L.mc);
            // in batches of kTB loads per lane, all in flight together
            for (int b0 = 0; b0 < s.V; b0 += kTB * kT) {
                T tmp[kTB];
#pragma unroll
                for (int q = 0; q < kTB; q++) {
                    const int idx = min(b0 + q * kT + (int)threadIdx.x, s.V - 1);
                    int j0, j1, j2;
                    dec3(idx, s.m, j0, j1, j2);
                    tmp[q] = (a.k0 == 0) ? src[j0 * st[0] + j1 * st[1] + j2 * st[2]]
                                         : L.Wk[idx] + (a.Z0 ? a.Z0[idx] : T(0));
                }
#pragma unroll
                for (int q = 0; q < kTB; q++)
                    if (b0 + q * kT + (int)threadIdx.x < s.V) R.U[b0 + q * kT + threadIdx.x] = tmp[q];
            }
        }
        for (int l = 0; l < a.nlev; l++) {
            const TailLevel<T>& L = a.lv[l];
            const int k = a.k0 + l;
            const TailShape s = shape_of(L.m, L.mc);
            const LdsTab<T> t = stage_tables(L, stab);
            __syncthreads();
            // coefficients in place (only coarse nodes are read by others)
            const int64_t v0 = st[0] << k, v1 = st[1] << k, v2 = st[2] << k;
            for (int idx = threadIdx.x; idx < s.V; idx += kT) {
                int j0, j1, j2;
                dec3(idx, s.m, j0, j1, j2);
                if (((j0 | j1 | j2) & 1) == 0) {
                    R.W[((j0 >> 1) * s.mc[1] + (j1 >> 1)) * s.mc[2] + (j2 >> 1)] = R.U[idx];
                } else {
                    const T c = R.U[idx] - tail_interp<T, false>(R.U, s, t, j0, j1, j2);
                    R.U[idx] = c;
                    dst[j0 * v0 + j1 * v1 + j2 * v2] = c;
                }
            }
            __syncthreads();
            lds_load_vector(R.U, R.P1, R.P2, R.F, s, t);
            lds_solve_apply(R.F, R.W, T(1), s, t);
            if (l + 1 < a.nlev) {
                for (int q = threadIdx.x; q < s.Vc; q += kT) R.U[q] = R.W[q];
                __syncthreads();
            } else {
                // coarsest values to their nodes
                const int64_t c0 = st[0] << (k + 1), c1 = st[1] << (k + 1), c2 = st[2] << (k + 1);
                for (int idx = threadIdx.x; idx < s.Vc; idx += kT) {
                    int j0, j1, j2;
                    dec3(idx, s.mc, j0, j1, j2);
                    dst[j0 * c0 + j1 * c1 + j2 * c2] = R.W[idx];
                }
            }
        }
    } else {
        {
            const TailLevel<T>& Lc = a.lv[a.nlev - 1];
            const TailShape s = shape_of(Lc.m, Lc.mc);
            const int L = a.k0 + a.nlev;
            const int64_t c0 = st[0] << L, c1 = st[1] << L, c2 = st[2] << L;
            for (int idx = threadIdx.x; idx < s.Vc; idx += kT) {
                int j0, j1, j2;
                dec3(idx, s.mc, j0, j1, j2);
                R.W[idx] = src[j0 * c0 + j1 * c1 + j2 * c2];
            }
        }
        for (int l = a.nlev - 1; l >= 0; l--) {
            const TailLevel<T>& L = a.lv[l];
            const int k = a.k0 + l;
            const TailShape s = shape_of(L.m, L.mc);
            const LdsTab<T> t = stage_tables(L, stab);
            const int64_t v0 = st[0] << k, v1 = st[1] << k, v2 = st[2] << k;
            for (int b0 = 0; b0 < s.V; b0 += kTB * kT) {
                T tmp[kTB];
#pragma unroll
                for (int q = 0; q < kTB; q++) {
                    const int idx = min(b0 + q * kT + (int)threadIdx.x, s.V - 1);
                    int j0, j1, j2;
                    dec3(idx, s.m, j0, j1, j2);
                    tmp[q] = (((j0 | j1 | j2) & 1) == 0) ? T(0) : src[j0 * v0 + j1 * v1 + j2 * v2];
                }
#pragma unroll
                for (int q = 0; q < kTB; q++)
                    if (b0 + q * kT + (int)threadIdx.x < s.V) R.U[b0 + q * kT + threadIdx.x] = tmp[q];
            }
            __syncthreads();
            lds_load_vector(R.U, R.P1, R.P2, R.F, s, t);
            lds_solve_apply(R.F, R.W, T(-1), s, t);
            for (int idx = threadIdx.x; idx < s.V; idx += kT) {
                int j0, j1, j2;
                dec3(idx, s.m, j0, j1, j2);
                if (((j0 | j1 | j2) & 1) == 0)
                    R.U[idx] = R.W[((j0 >> 1) * s.mc[1] + (j1 >> 1)) * s.mc[2] + (j2 >> 1)];
                else
                    R.U[idx] += tail_interp<T, true>(R.W, s, t, j0, j1, j2);
            }
            __syncthreads();
            if (l > 0) {
                for (int q = threadIdx.x; q < s.V; q += kT) R.W[q] = R.U[q];
                __syncthreads();
            }
        }
        // the level-k0 grid goes to the workspace, or to the output if k0 == 0
        const TailLevel<T>& L = a.lv[0];
        const TailShape s = shape_of(L.m, L.mc);
        for (int idx = threadIdx.x; idx < s.V; idx += kT) {
            int j0, j1, j2;
            dec3(idx, s.m, j0, j1, j2);
            if (a.k0 == 0)
                dst[j0 * st[0] + j1 * st[1] + j2 * st[2]] = R.U[idx];
            else
                L.Wk[idx] = R.U[idx];
        }
    }
}

template <typename T, bool kDec>
__global__ void __launch_bounds__(kT) k_tail(TailArgs<T> a)
{
    __shared__ T sbuf[kTailDataElems];
    __shared__ T stab[kTailTabElems];
    tail_body<T, kDec>(a, a.src, a.dst, sbuf, stab);
}

// One workgroup per entry of a batch; arguments in device memory.
template <typename T, bool kDec>
__global__ void __launch_bounds__(kT) k_tail_batch(const TailArgs<T>* __restrict__ args, const int* __restrict__ field,
                                                   const T* const* __restrict__ src, T* const* __restrict__ dst)
{
    __shared__ T sbuf[kTailDataElems];
    __shared__ T stab[kTailTabElems];
    const int f = field[blockIdx.x];
    tail_body<T, kDec>(args[blockIdx.x], src[f], dst[f], sbuf, stab);
}

}  // namespace

template <typename T>
hipError_t launch_tail_batch(const TailArgs<T>* dev_args, const int* field, const T* const* src, T* const* dst,
                             int n, bool decompose, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (decompose)
        hipLaunchKernelGGL((k_tail_batch<T, true>), dim3((unsigned)n), dim3(kT), 0, st, dev_args, field, src, dst);
    else
        hipLaunchKernelGGL((k_tail_batch<T, false>), dim3((unsigned)n), dim3(kT), 0, st, dev_args, field, src, dst);
    return hipGetLastError();
}

template hipError_t launch_tail_batch<float>(const TailArgs<float>*, const int*, const float* const*, float* const*,
                                             int, bool, hipStream_t);
template hipError_t launch_tail_batch<double>(const TailArgs<double>*, const int*, const double* const*,
                                              double* const*, int, bool, hipStream_t);

template <typename T>
hipError_t launch_tail(const TailArgs<T>& a, bool decompose, hipStream_t st)
{
    if (decompose)
        hipLaunchKernelGGL((k_tail<T, true>), dim3(1), dim3(kT), 0, st, a);
    else
        hipLaunchKernelGGL((k_tail<T, false>), dim3(1), dim3(kT), 0, st, a);
    return hipGetLastError();
}

template hipError_t launch_tail<float>(const TailArgs<float>&, bool, hipStream_t);
template hipError_t launch_tail<double>(const TailArgs<double>&, bool, hipStream_t);

}  // namespace mgr
