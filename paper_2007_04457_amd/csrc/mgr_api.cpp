// Host side of libmgr: argument validation, FP64 geometry tables, workspace,
// the level loops of decomposition / recomposition / adjoint, and kernel
// timing.  Implements include/mgr.h.
//
// Level step k (k = 0 finest) acts on the "level grid": the nodes whose
// indices are all multiples of 2^k, of size m_d = (n_d - 1) / 2^k + 1.  Its
// coarse nodes (all level indices even) form the next level grid of size
// (m_d + 1) / 2, which the driver keeps packed in workspace buffers W_{k+1}.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "mgr.h"
#include "mgr_internal.h"

namespace mgr {
namespace {

thread_local std::string g_err;

int fail(int status, const std::string& msg)
{
    g_err = msg;
    return status;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(MGR_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr int kMaxDim = 3;

// Per level step: level-grid and coarse sizes and the element offsets of
// its tables inside the plan's device table buffer (inactive dims unused).
struct LevelLayout {
    int64_t m[3], mc[3];
    size_t w[3], K[3], lf[3], ip[3];  // lf, ip: plain Thomas factors of M_{l-1}
    size_t PT[3];  // P^T as a 5-point row per coarse node (transposed interpolation)
    size_t sup[3];  // plain super-diagonal of M_{l-1}
    size_t L[3], U[3], IP[3], A[3], B[3], ssub[3], ssup[3], sl[3], sip[3], su[3];
    int S[3];
};

struct Plan {
    int device = 0, dtype = 0, ndim = 0, nlevels = 0;
    int64_t n[3] = {1, 1, 1};
    int64_t st[3] = {0, 0, 1};
    bool active[3] = {false, false, false};
    int udim[3] = {-1, -1, -1};  // user dimension of each internal dimension
    std::vector<LevelLayout> lv;
    void* tables = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0, tables_bytes = 0, esize = 4;
    std::vector<size_t> Woff;  // W_k element offsets, k = 1..L (index k)
    size_t F = 0, F2 = 0, Tb = 0, Yb = 0;  // F, F2: corrections of even, odd level steps
    size_t Yb2 = 0;  // long-fibre solve scratch for the coarser level steps of a recomposition
    // Recomposition computes every level's correction before it is applied,
    // so it keeps one buffer per level step: Zrec[0] = F, Zrec[1] = F2, then
    // regions of their own.
    std::vector<size_t> Zrec;
};

std::mutex g_mu;
std::map<std::string, std::unique_ptr<Plan>> g_plans;

// ---- timing ---------------------------------------------------------------
struct Timing {
    bool on = false;
    int kc = -1, level = -1;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
};
Timing g_tm;
std::mutex g_tm_mu;

bool capturing(hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
    return cs != hipStreamCaptureStatusNone;
}

template <class Fn>
hipError_t timed(int kc, int level, hipStream_t st, Fn&& launch)
{
    bool want = false;
    {
        std::lock_guard<std::mutex> lk(g_tm_mu);
        want = g_tm.on && g_tm.kc == kc && (g_tm.level < 0 || g_tm.level == level);
    }
    if (!want || capturing(st)) return launch();
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&b);
    if (e != hipSuccess) { (void)hipEventDestroy(a); return e; }
    (void)hipEventRecord(a, st);
    e = launch();
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_tm_mu);
    g_tm.ev.emplace_back(a, b);
    return e;
}

// ---- validation -----------------------------------------------------------
int log2_exact(int64_t v)
{
    if (v <= 0) return -1;
    int k = 0;
    while (k < 62 && ((int64_t)1 << k) < v) k++;
    return (((int64_t)1 << k) == v) ? k : -1;
}

int validate(int dtype, int ndim, const int64_t* shape, const double* const* coords,
             int* nlevels)
{
    if (dtype != MGR_F32 && dtype != MGR_F64) return fail(MGR_ERR_ARG, "dtype must be MGR_F32 or MGR_F64");
    if (ndim < 1 || ndim > kMaxDim) return fail(MGR_ERR_ARG, "ndim must be 1..3");
    if (!shape) return fail(MGR_ERR_ARG, "shape is NULL");
    int kmin = 63;
    for (int d = 0; d < ndim; d++) {
        int k = (shape[d] >= 3) ? log2_exact(shape[d] - 1) : -1;
        if (k < 1)
            return fail(MGR_ERR_SHAPE, "shape[" + std::to_string(d) + "] = " +
                                           std::to_string(shape[d]) + " is not 2^k+1 with k >= 1");
        kmin = std::min(kmin, k);
    }
    // The kernels address within one plane of the array (the contiguous row
    // in 1-D and 2-D, a dim-1 x dim-2 plane in 3-D) with 32-bit byte offsets,
    // and mark lanes off the grid with an offset of 2^31.
    {
        const int64_t esz = (dtype == MGR_F64) ? 8 : 4;
        const int64_t plane = (ndim == 3) ? shape[1] * shape[2] : shape[ndim - 1];
        if (plane > ((int64_t)1 << 31) / esz - 1)
            return fail(MGR_ERR_SHAPE, "a plane of " + std::to_string(plane) + " elements exceeds the kernels' "
                                       "2 GiB per-plane addressing");
    }
    if (*nlevels == -1) *nlevels = kmin - 1;
    if (*nlevels < 0 || *nlevels > kmin)
        return fail(MGR_ERR_LEVELS, "nlevels = " + std::to_string(*nlevels) + " outside 0.." +
                                        std::to_string(kmin) + " (or -1)");
    if (coords) {
        for (int d = 0; d < ndim; d++) {
            const double* x = coords[d];
            if (!x) continue;
            for (int64_t i = 0; i < shape[d]; i++) {
                if (!std::isfinite(x[i]) || (i > 0 && !(x[i] > x[i - 1])))
                    return fail(MGR_ERR_COORDS, "coords[" + std::to_string(d) +
                                                    "] not finite and strictly increasing at " +
                                                    std::to_string(i));
            }
        }
    }
    return MGR_OK;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---- FP64 geometry tables (Sec. III-A.2 readings) --------------------------
// Node positions along a dimension, scaled so the mean finest spacing is 1
// (only ratios of spacings enter the method).
std::vector<double> axis_positions(int64_t n, const double* x)
{
    std::vector<double> X((size_t)n);
    if (!x) {
        for (int64_t i = 0; i < n; i++) X[(size_t)i] = (double)i;
    } else {
        double sc = (double)(n - 1) / (x[n - 1] - x[0]);
        for (int64_t i = 0; i < n; i++) X[(size_t)i] = (x[i] - x[0]) * sc;
    }
    return X;
}

struct DimTab {
    std::vector<double> w, K, PT;
};

// Tables of one dimension at level step k from the level-grid positions y.
DimTab build_dim(const std::vector<double>& y)
{
    const int64_t m = (int64_t)y.size(), mc = (m + 1) / 2;
    DimTab t;
    t.w.assign((size_t)(2 * m), 0.0);
    for (int64_t j = 1; j < m; j += 2) {
        double a = (y[j] - y[j - 1]) / (y[j + 1] - y[j - 1]);
        t.w[(size_t)(2 * j)] = 1.0 - a;
        t.w[(size_t)(2 * j + 1)] = a;
    }
    auto h = [&](int64_t j) { return (j >= 0 && j < m - 1) ? y[j + 1] - y[j] : 0.0; };
    // Mass matrix entry M(r, c) (piecewise-linear FE mass matrix times 6).
    auto M = [&](int64_t r, int64_t c) {
        if (c == r) return 2.0 * (h(r - 1) + h(r));
        if (c == r - 1) return h(r - 1);
        if (c == r + 1) return h(r);
        return 0.0;
    };
    // R = P^T: coarse node i collects fine 2i (weight 1), 2i-1 (its upper
    // interpolation weight) and 2i+1 (its lower interpolation weight).
    auto PT = [&](int64_t i, int64_t j) {
        if (j == 2 * i) return 1.0;
        if (j == 2 * i - 1) return t.w[(size_t)(2 * j + 1)];
        if (j == 2 * i + 1) return t.w[(size_t)(2 * j)];
        return 0.0;
    };
    t.K.assign((size_t)(5 * mc), 0.0);
    for (int64_t i = 0; i < mc; i++) {
        for (int tt = -2; tt <= 2; tt++) {
            int64_t c = 2 * i + tt;
            if (c < 0 || c >= m) continue;
            double s = 0.0;
            for (int64_t j = 2 * i - 1; j <= 2 * i + 1; j++)
                if (j >= 0 && j < m) s += PT(i, j) * M(j, c);
            t.K[(size_t)(5 * i + tt + 2)] = s;
        }
    }
    // P^T alone in the same 5-point form: coarse node i collects fine 2i - 1,
    // 2i and 2i + 1 (the recomposition adjoint's transposed interpolation)
    t.PT.assign((size_t)(5 * mc), 0.0);
    for (int64_t i = 0; i < mc; i++)
        for (int64_t j = 2 * i - 1; j <= 2 * i + 1; j++)
            if (j >= 0 && j < m) t.PT[(size_t)(5 * i + (j - 2 * i) + 2)] = PT(i, j);
    return t;
}

struct SolveTab {
    std::vector<double> sub, sup;                  // plain off-diagonals, length n
    std::vector<double> L, U, IP, A, B;            // padded, S * kSlot
    std::vector<double> ssub, ssup, sl, sip, su;   // per separator, length S
    int S = 1;
};

// Partitioned-Thomas tables of the coarse mass matrix on positions yc
// (segment length kSeg; see mgr_solve.hip for the scheme).
SolveTab build_solve(const std::vector<double>& yc)
{
    const int64_t n = (int64_t)yc.size();
    SolveTab t;
    auto hc = [&](int64_t i) { return (i >= 0 && i < n - 1) ? yc[(size_t)(i + 1)] - yc[(size_t)i] : 0.0; };
    std::vector<double> diag((size_t)n);
    t.sub.assign((size_t)n, 0.0);
    t.sup.assign((size_t)n, 0.0);
    for (int64_t i = 0; i < n; i++) {
        t.sub[(size_t)i] = hc(i - 1);
        t.sup[(size_t)i] = hc(i);
        diag[(size_t)i] = 2.0 * (hc(i - 1) + hc(i));
    }
    // one segment up to kSlot nodes, else segments of kSeg (the last one
    // shorter when kSeg does not divide n - 1; for 2^k + 1 sizes it does)
    t.S = (n <= kSlot) ? 1 : (int)((n - 1 + kSeg - 1) / kSeg);
    const int S = t.S;
    const size_t P = (size_t)S * kSlot;
    t.L.assign(P, 0.0);
    t.U.assign(P, 0.0);
    t.IP.assign(P, 0.0);
    t.A.assign(P, 0.0);
    t.B.assign(P, 0.0);
    std::vector<double> alpha((size_t)n, 0.0), beta((size_t)n, 0.0);
    for (int s = 0; s < S; s++) {
        const int64_t lo = (int64_t)s * kSeg + (s > 0 ? 1 : 0);
        const int64_t hi = (s == S - 1) ? n : (int64_t)(s + 1) * kSeg;
        std::vector<double> lf((size_t)(hi - lo), 0.0), ip((size_t)(hi - lo), 0.0);
        double den = 0.0;
        for (int64_t i = lo; i < hi; i++) {
            const size_t q = (size_t)(i - lo);
            if (i == lo) {
                den = diag[(size_t)i];
            } else {
                lf[q] = t.sub[(size_t)i] / den;
                den = diag[(size_t)i] - lf[q] * t.sup[(size_t)(i - 1)];
            }
            ip[q] = 1.0 / den;
        }
        auto local_solve = [&](std::vector<double>& v) {
            for (int64_t i = lo + 1; i < hi; i++) v[(size_t)i] -= lf[(size_t)(i - lo)] * v[(size_t)(i - 1)];
            for (int64_t i = hi - 1; i >= lo; i--) {
                double z = (i == hi - 1) ? 0.0 : v[(size_t)(i + 1)];
                v[(size_t)i] = (v[(size_t)i] - t.sup[(size_t)i] * z) * ip[(size_t)(i - lo)];
            }
        };
        if (s > 0) {
            std::vector<double> v((size_t)n, 0.0);
            v[(size_t)lo] = -t.sub[(size_t)lo];
            local_solve(v);
            for (int64_t i = lo; i < hi; i++) alpha[(size_t)i] = v[(size_t)i];
        }
        if (s < S - 1) {
            std::vector<double> v((size_t)n, 0.0);
            v[(size_t)(hi - 1)] = -t.sup[(size_t)(hi - 1)];
            local_solve(v);
            for (int64_t i = lo; i < hi; i++) beta[(size_t)i] = v[(size_t)i];
        }
        for (int64_t i = lo; i < hi; i++) {
            const size_t q = (size_t)s * kSlot + (size_t)(i - lo);
            t.L[q] = lf[(size_t)(i - lo)];
            // the segment's last row has no coupling inside the segment
            t.U[q] = (i == hi - 1) ? 0.0 : t.sup[(size_t)i];
            t.IP[q] = ip[(size_t)(i - lo)];
            t.A[q] = alpha[(size_t)i];
            t.B[q] = beta[(size_t)i];
        }
    }
    t.ssub.assign((size_t)S, 0.0);
    t.ssup.assign((size_t)S, 0.0);
    t.sl.assign((size_t)S, 0.0);
    t.sip.assign((size_t)S, 0.0);
    t.su.assign((size_t)S, 0.0);
    double den = 0.0;
    for (int s = 1; s < S; s++) {
        const int64_t p = (int64_t)s * kSeg;
        t.ssub[(size_t)s] = t.sub[(size_t)p];
        t.ssup[(size_t)s] = t.sup[(size_t)p];
        const double Lc = t.sub[(size_t)p] * alpha[(size_t)(p - 1)];
        const double D = diag[(size_t)p] + t.sub[(size_t)p] * beta[(size_t)(p - 1)] +
                         t.sup[(size_t)p] * alpha[(size_t)(p + 1)];
        const double Uc = t.sup[(size_t)p] * beta[(size_t)(p + 1)];
        if (s == 1) {
            den = D;
        } else {
            t.sl[(size_t)s] = Lc / den;
            den = D - t.sl[(size_t)s] * t.su[(size_t)(s - 1)];
        }
        t.su[(size_t)s] = Uc;
        t.sip[(size_t)s] = 1.0 / den;
    }
    return t;
}

std::string plan_key(int device, int dtype, int ndim, const int64_t* shape,
                     const double* const* coords, int nlevels)
{
    std::string k;
    auto put = [&](const void* p, size_t n) { k.append((const char*)p, n); };
    put(&device, sizeof device);
    put(&dtype, sizeof dtype);
    put(&ndim, sizeof ndim);
    put(&nlevels, sizeof nlevels);
    put(shape, sizeof(int64_t) * (size_t)ndim);
    for (int d = 0; d < ndim; d++) {
        const double* x = coords ? coords[d] : nullptr;
        char flag = x ? 1 : 0;
        put(&flag, 1);
        if (x) put(x, sizeof(double) * (size_t)shape[d]);
    }
    return k;
}

size_t workspace_cap()
{
    const char* e = std::getenv("MGR_WORKSPACE_MAX");
    if (!e || !*e) return (size_t)-1;
    return (size_t)std::strtoull(e, nullptr, 10);
}

template <typename T>
void push_table(std::vector<T>& buf, const std::vector<double>& v, size_t* off)
{
    *off = buf.size();
    for (double x : v) buf.push_back((T)x);
    while (buf.size() % 64) buf.push_back(T(0));
}

// Host half of a plan: the level layouts, the tables in the working
// precision (into `host`) and the workspace layout, without touching the
// device.  `dec_only` leaves out the buffers that only recomposition and the
// adjoint use.
template <typename T>
void plan_layout(Plan& p, const double* const* coords, bool dec_only, std::vector<T>& host)
{
    const int L = p.nlevels;
    std::vector<std::vector<double>> X(3);
    for (int d = 0; d < 3; d++)
        if (p.active[d]) X[d] = axis_positions(p.n[d], coords ? coords[p.udim[d]] : nullptr);
    host.clear();
    p.lv.resize((size_t)L);
    for (int k = 0; k < L; k++) {
        LevelLayout& ly = p.lv[(size_t)k];
        for (int d = 0; d < 3; d++) {
            ly.m[d] = p.active[d] ? ((p.n[d] - 1) >> k) + 1 : 1;
            ly.mc[d] = p.active[d] ? (ly.m[d] + 1) / 2 : 1;
            ly.w[d] = ly.K[d] = ly.lf[d] = ly.ip[d] = ly.PT[d] = 0;
            ly.sup[d] = ly.L[d] = ly.U[d] = ly.IP[d] = ly.A[d] = ly.B[d] = 0;
            ly.ssub[d] = ly.ssup[d] = ly.sl[d] = ly.sip[d] = ly.su[d] = 0;
            ly.S[d] = 1;
            if (!p.active[d]) continue;
            std::vector<double> y((size_t)ly.m[d]);
            for (int64_t j = 0; j < ly.m[d]; j++) y[(size_t)j] = X[d][(size_t)(j << k)];
            DimTab t = build_dim(y);
            push_table(host, t.w, &ly.w[d]);
            push_table(host, t.K, &ly.K[d]);
            if (!dec_only) push_table(host, t.PT, &ly.PT[d]);
            std::vector<double> yc((size_t)ly.mc[d]);
            for (int64_t i = 0; i < ly.mc[d]; i++) yc[(size_t)i] = y[(size_t)(2 * i)];
            SolveTab sv = build_solve(yc);
            {
                // plain Thomas factors of the whole coarse fibre (small levels)
                const size_t nc = yc.size();
                std::vector<double> lf(nc, 0.0), ip(nc, 0.0);
                double den = 0.0;
                for (size_t i = 0; i < nc; i++) {
                    const double diag = 2.0 * (sv.sub[i] + sv.sup[i]);
                    if (i == 0) {
                        den = diag;
                    } else {
                        lf[i] = sv.sub[i] / den;
                        den = diag - lf[i] * sv.sup[i - 1];
                    }
                    ip[i] = 1.0 / den;
                }
                push_table(host, lf, &ly.lf[d]);
                push_table(host, ip, &ly.ip[d]);
            }
            ly.S[d] = sv.S;
            push_table(host, sv.sup, &ly.sup[d]);
            push_table(host, sv.L, &ly.L[d]);
            push_table(host, sv.U, &ly.U[d]);
            push_table(host, sv.IP, &ly.IP[d]);
            push_table(host, sv.A, &ly.A[d]);
            push_table(host, sv.B, &ly.B[d]);
            push_table(host, sv.ssub, &ly.ssub[d]);
            push_table(host, sv.ssup, &ly.ssup[d]);
            push_table(host, sv.sl, &ly.sl[d]);
            push_table(host, sv.sip, &ly.sip[d]);
            push_table(host, sv.su, &ly.su[d]);
        }
    }
    // workspace: W_1..W_L, corrections F, F2 (and per level for
    // recomposition), adjoint buffer Tb, long-fibre solve scratch Yb
    const size_t al = 256 / sizeof(T);
    size_t off = 0;
    p.Woff.assign((size_t)L + 1, 0);
    for (int k = 1; k <= L; k++) {
        int64_t v = 1;
        for (int d = 0; d < 3; d++) v *= p.active[d] ? ((p.n[d] - 1) >> k) + 1 : 1;
        p.Woff[(size_t)k] = off;
        off = align_up(off + (size_t)v, al);
    }
    int64_t sh[3] = {p.n[0], p.n[1], p.n[2]};
    int64_t V0 = sh[0] * sh[1] * sh[2];
    std::vector<int64_t> pass_sizes;
    for (int d = 2; d >= 0; d--) {
        if (!p.active[d]) continue;
        sh[d] = (sh[d] + 1) / 2;
        pass_sizes.push_back(sh[0] * sh[1] * sh[2]);
    }
    size_t Fn = L > 0 ? (size_t)pass_sizes.back() : 0;
    p.F = off;  off = align_up(off + Fn, al);
    int64_t v1 = 1;  // coarse grid of level step 1 (= level grid 2)
    for (int d = 0; d < 3; d++) v1 *= p.active[d] ? ((p.n[d] - 1) >> 2) + 1 : 1;
    p.F2 = off;
    off = align_up(off + (L > 1 ? (size_t)v1 : 0), al);
    p.Zrec.assign((size_t)L, 0);
    for (int k = 0; k < L; k++) {
        if (k < 2 || dec_only) {
            p.Zrec[(size_t)k] = (k == 0) ? p.F : p.F2;
            continue;
        }
        int64_t v = 1;  // coarse grid of level step k = level grid k + 1
        for (int d = 0; d < 3; d++) v *= p.active[d] ? ((p.n[d] - 1) >> (k + 1)) + 1 : 1;
        p.Zrec[(size_t)k] = off;
        off = align_up(off + (size_t)v, al);
    }
    p.Tb = off; off = align_up(off + (L > 0 && !dec_only ? (size_t)V0 : 0), al);
    p.Yb = off; off = align_up(off + 2 * Fn / kSeg + 64, al);
    p.Yb2 = off; off = align_up(off + (L > 1 && !dec_only ? 2 * (size_t)v1 / kSeg + 64 : 0), al);
    p.esize = sizeof(T);
    p.ws_bytes = off * sizeof(T);
    p.tables_bytes = host.size() * sizeof(T);
}

template <typename T>
int build_plan(Plan& p, const double* const* coords, bool with_ws)
{
    std::vector<T> host;
    plan_layout<T>(p, coords, false, host);
    if ((with_ws ? p.ws_bytes : 0) + p.tables_bytes > workspace_cap())
        return fail(MGR_ERR_ALLOC, "workspace of " + std::to_string(p.ws_bytes) +
                                       " bytes exceeds MGR_WORKSPACE_MAX");
    if (p.tables_bytes) {
        hipError_t e = hipMalloc(&p.tables, p.tables_bytes);
        if (e != hipSuccess) return fail(MGR_ERR_ALLOC, std::string("hipMalloc tables: ") + hipGetErrorString(e));
        e = hipMemcpy(p.tables, host.data(), p.tables_bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "upload tables");
    }
    if (with_ws && p.ws_bytes) {
        hipError_t e = hipMalloc(&p.ws, p.ws_bytes);
        if (e != hipSuccess) {
            p.ws = nullptr;
            return fail(MGR_ERR_ALLOC, std::string("hipMalloc workspace: ") + hipGetErrorString(e));
        }
    }
    return MGR_OK;
}

void free_plan(Plan& p)
{
    if (p.tables) (void)hipFree(p.tables);
    if (p.ws) (void)hipFree(p.ws);
    p.tables = p.ws = nullptr;
}

int new_plan(int dev, int dtype, int ndim, const int64_t* shape, const double* const* coords, int nlevels,
             bool with_ws, std::unique_ptr<Plan>& out);

// Problem dimensions of a plan (validated arguments): 3-D as (n0, n1, n2);
// 2-D as (n0, 1, n1) so the streaming kernel walks rows; 1-D as (1, 1, n0).
void plan_dims(Plan& p, int dev, int dtype, int ndim, const int64_t* shape, int nlevels)
{
    p.device = dev;
    p.dtype = dtype;
    p.ndim = ndim;
    p.nlevels = nlevels;
    static const int kMap[4][3] = {{-1, -1, -1}, {-1, -1, 0}, {0, -1, 1}, {0, 1, 2}};
    for (int d = 0; d < 3; d++) {
        p.udim[d] = kMap[ndim][d];
        if (p.udim[d] >= 0) {
            p.n[d] = shape[p.udim[d]];
            p.active[d] = true;
        }
    }
    p.st[2] = 1;
    p.st[1] = p.n[2];
    p.st[0] = p.n[1] * p.n[2];
}

int get_plan(int dtype, int ndim, const int64_t* shape, const double* const* coords,
             int nlevels, hipStream_t st, bool check_capture, Plan** out)
{
    int rc = validate(dtype, ndim, shape, coords, &nlevels);
    if (rc) return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::string key = plan_key(dev, dtype, ndim, shape, coords, nlevels);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        *out = it->second.get();
        return MGR_OK;
    }
    if (check_capture && capturing(st))
        return fail(MGR_ERR_CAPTURE, "problem not prepared and the stream is capturing; call mgr_prepare first");
    std::unique_ptr<Plan> p;
    rc = new_plan(dev, dtype, ndim, shape, coords, nlevels, true, p);
    if (rc) return rc;
    *out = p.get();
    g_plans.emplace(key, std::move(p));
    return MGR_OK;
}

// A plan of a validated problem: tables uploaded and, with `with_ws`, its
// workspace allocated.
int new_plan(int dev, int dtype, int ndim, const int64_t* shape, const double* const* coords, int nlevels,
             bool with_ws, std::unique_ptr<Plan>& out)
{
    auto p = std::make_unique<Plan>();
    plan_dims(*p, dev, dtype, ndim, shape, nlevels);
    int rc = (dtype == MGR_F32) ? build_plan<float>(*p, coords, with_ws) : build_plan<double>(*p, coords, with_ws);
    if (rc) {
        free_plan(*p);
        return rc;
    }
    out = std::move(p);
    return MGR_OK;
}

// ---- views ----------------------------------------------------------------
View3 level_view(const Plan& p, int k)
{
    View3 v;
    for (int d = 0; d < 3; d++) {
        v.n[d] = p.active[d] ? ((p.n[d] - 1) >> k) + 1 : 1;
        v.s[d] = p.st[d] << k;
    }
    return v;
}

View3 packed(const int64_t* n)
{
    View3 v;
    for (int d = 0; d < 3; d++) v.n[d] = n[d];
    v.s[2] = 1;
    v.s[1] = n[2];
    v.s[0] = n[1] * n[2];
    return v;
}

template <typename T>
DimTables<T> tables_of(const Plan& p, int k)
{
    DimTables<T> tb;
    const T* base = (const T*)p.tables;
    const LevelLayout& ly = p.lv[(size_t)k];
    for (int d = 0; d < 3; d++) {
        bool a = p.active[d];
        tb.w[d] = a ? base + ly.w[d] : nullptr;
        tb.K[d] = a ? base + ly.K[d] : nullptr;
    }
    return tb;
}

// Interpolation weights with P^T in place of the load-vector stencil.
template <typename T>
DimTables<T> pt_tables_of(const Plan& p, int k)
{
    DimTables<T> tb = tables_of<T>(p, k);
    const T* base = (const T*)p.tables;
    for (int d = 0; d < 3; d++) tb.K[d] = p.active[d] ? base + p.lv[(size_t)k].PT[d] : nullptr;
    return tb;
}

#define MGR_TRY(expr, what)                                \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return hip_fail(e_, what);   \
    } while (0)

template <typename T>
SolveTables<T> solve_tables_of(const Plan& p, int k, int d)
{
    const T* base = (const T*)p.tables;
    const LevelLayout& ly = p.lv[(size_t)k];
    SolveTables<T> t;
    t.L = base + ly.L[d];
    t.U = base + ly.U[d];
    t.IP = base + ly.IP[d];
    t.A = base + ly.A[d];
    t.B = base + ly.B[d];
    t.ssub = base + ly.ssub[d];
    t.ssup = base + ly.ssup[d];
    t.sl = base + ly.sl[d];
    t.sip = base + ly.sip[d];
    t.su = base + ly.su[d];
    t.S = ly.S[d];
    return t;
}

// Correction buffer of level step k (even and odd steps alternate so that a
// step can read the previous step's correction while writing its own).
template <typename T>
T* corr(const Plan& p, int k, void* ws = nullptr)
{
    return (T*)(ws ? ws : p.ws) + ((k & 1) ? p.F2 : p.F);
}

// Streaming level kernel of level step k: coefficients + load vector (dec,
// input A + Z) or the load vector from stored coefficients (!dec); the load
// vector goes to corr(k).
template <typename T>
int stream_level(const Plan& p, int k, bool dec, const T* A, const T* Z, View3 av, T* C, View3 cv,
                 T* W, bool write_coarse, hipStream_t st, T* Fout = nullptr)
{
    const LevelLayout& ly = p.lv[(size_t)k];
    StreamArgs<T> a;
    a.A = A;
    a.Z = Z;
    a.av = av;
    a.C = C;
    a.cv = cv;
    a.W = W;
    a.wv = packed(ly.mc);
    a.F = Fout ? Fout : corr<T>(p, k);
    a.fv = packed(ly.mc);
    a.tb = tables_of<T>(p, k);
    a.write_coarse = write_coarse ? 1 : 0;
    a.chunk = a.nt1 = a.nt2 = a.nch = 0;
    MGR_TRY(timed(dec ? KC_STREAM_DEC : KC_STREAM_LOAD, k, st,
                  [&] { return launch_stream_level<T>(a, dec, st); }),
            "level kernel launch");
    return MGR_OK;
}

// Correction solves of level step k on F along every dimension, in place.
// whole_cu: a small grid may be solved by one workgroup that needs a whole
// CU (all dimensions in one launch); a caller whose launches share the
// device with long-running kernels on another stream passes false, since
// such a workgroup waits until one CU has drained completely (the
// per-dimension launches give the same values).
template <typename T>
int solve_all(const Plan& p, int k, bool reverse, T* F, hipStream_t st, T* Yb = nullptr, bool whole_cu = true)
{
    T* ws = (T*)p.ws;
    View3 fv = packed(p.lv[(size_t)k].mc);
    if (whole_cu) {
        // small coarse grids: every dimension in one launch when it fits
        int dims[3], nd = 0;
        SolveTables<T> tbs[3];
        for (int s = 0; s < 3; s++) {
            const int d = reverse ? s : 2 - s;
            if (!p.active[d]) continue;
            dims[nd] = d;
            tbs[nd++] = solve_tables_of<T>(p, k, d);
        }
        if (solve_small_fits<T>(fv, dims, nd, tbs)) {
            MGR_TRY(timed(KC_SOLVE, k, st, [&] { return launch_solve_small<T>(F, fv, dims, nd, tbs, st); }),
                    "small solve launch");
            return MGR_OK;
        }
        // planes that fit in LDS: dimensions 2 and 1 in one launch, then 0
        if (!reverse && p.active[1] && p.active[2]) {
            const SolveTables<T> t2 = solve_tables_of<T>(p, k, 2), t1 = solve_tables_of<T>(p, k, 1);
            if (solve_plane_fits<T>(fv, t2, t1)) {
                MGR_TRY(timed(KC_SOLVE, k, st, [&] { return launch_solve_plane<T>(F, fv, t2, t1, st); }),
                        "plane solve launch");
                if (p.active[0]) {
                    SolveTables<T> t0 = solve_tables_of<T>(p, k, 0);
                    MGR_TRY(timed(KC_SOLVE, k, st,
                                  [&] { return launch_solve_partitioned<T>(F, fv, 0, t0, Yb ? Yb : ws + p.Yb, st); }),
                            "solve launch");
                }
                return MGR_OK;
            }
        }
    }
    for (int s = 0; s < 3; s++) {
        int d = reverse ? s : 2 - s;
        if (!p.active[d]) continue;
        SolveTables<T> tb = solve_tables_of<T>(p, k, d);
        MGR_TRY(timed(KC_SOLVE, k, st,
                      [&] { return launch_solve_partitioned<T>(F, fv, d, tb, Yb ? Yb : ws + p.Yb, st); }),
                "solve launch");
    }
    return MGR_OK;
}

View3 full_view(const Plan& p) { return packed(p.n); }
View3 packed_view3(const int64_t* n) { return packed(n); }

template <typename T>
int identity_copy(const Plan& p, const void* src, void* dst, hipStream_t st)
{
    if (src == dst) return MGR_OK;
    size_t bytes = (size_t)(p.n[0] * p.n[1] * p.n[2]) * sizeof(T);
    MGR_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st), "copy");
    return MGR_OK;
}

// First level step handled by the single-workgroup tail kernel: the finest
// step whose level grid is small, but no more than kMaxTail steps.
std::atomic<int64_t> g_tail_nodes{kTailMaxNodes};

// LDS elements the tail kernel needs for level step k: level grid, the
// load-vector passes, correction and coarse values; and for its tables.
int64_t tail_data_elems(const Plan& p, int k)
{
    const LevelLayout& ly = p.lv[(size_t)k];
    int64_t sh[3] = {ly.m[0], ly.m[1], ly.m[2]};
    const int64_t V = sh[0] * sh[1] * sh[2], Vc = ly.mc[0] * ly.mc[1] * ly.mc[2];
    int64_t tot = V + 2 * Vc, pass = 0;
    for (int d = 2; d >= 0; d--) {
        if (!p.active[d]) continue;
        sh[d] = ly.mc[d];
        if (++pass < 3 && sh[0] * sh[1] * sh[2] != Vc) tot += sh[0] * sh[1] * sh[2];
    }
    return tot;
}

int64_t tail_tab_elems(const Plan& p, int k)
{
    const LevelLayout& ly = p.lv[(size_t)k];
    int64_t tot = 0;
    for (int d = 0; d < 3; d++)
        if (p.active[d]) tot += 2 * ly.m[d] + 8 * ly.mc[d];
    return tot;
}

// First level step handled by the tail kernel: the finest step such that it
// and every coarser step are small, at most kMaxTail steps.
int tail_start(const Plan& p)
{
    const int L = p.nlevels;
    const int64_t limit = g_tail_nodes.load();
    int k = L;
    while (k > 0 && L - (k - 1) <= kMaxTail) {
        const LevelLayout& ly = p.lv[(size_t)(k - 1)];
        if (ly.m[0] * ly.m[1] * ly.m[2] > limit) break;
        if (tail_data_elems(p, k - 1) > kTailDataElems || tail_tab_elems(p, k - 1) > kTailTabElems) break;
        k--;
    }
    return k;
}

template <typename T>
TailArgs<T> tail_args(const Plan& p, int k0, const T* src, T* dst, void* wsp = nullptr)
{
    TailArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    T* ws = (T*)(wsp ? wsp : p.ws);
    const T* base = (const T*)p.tables;
    a.k0 = k0;
    a.nlev = p.nlevels - k0;
    for (int d = 0; d < 3; d++) a.st[d] = p.st[d];
    a.src = src;
    a.dst = dst;
    for (int l = 0; l < a.nlev; l++) {
        const int k = k0 + l;
        const LevelLayout& ly = p.lv[(size_t)k];
        TailLevel<T>& t = a.lv[l];
        for (int d = 0; d < 3; d++) {
            t.m[d] = (int)ly.m[d];
            t.mc[d] = (int)ly.mc[d];
            t.lf[d] = p.active[d] ? base + ly.lf[d] : nullptr;
            t.ip[d] = p.active[d] ? base + ly.ip[d] : nullptr;
            t.up[d] = p.active[d] ? base + ly.sup[d] : nullptr;
        }
        t.tb = tables_of<T>(p, k);
        t.Wk = (k == 0) ? nullptr : ws + p.Woff[(size_t)k];
    }
    return a;
}

template <typename T>
int run_decompose(const Plan& p, const void* src_, void* dst_, hipStream_t st)
{
    const int L = p.nlevels;
    if (L == 0) return identity_copy<T>(p, src_, dst_, st);
    const T* src = (const T*)src_;
    T* dst = (T*)dst_;
    T* ws = (T*)p.ws;
    const int kt = tail_start(p);
    for (int k = 0; k < kt; k++) {
        const LevelLayout& ly = p.lv[(size_t)k];
        // level grid k: the input, or the previous step's coarse values plus its correction
        const T* A = (k == 0) ? src : ws + p.Woff[(size_t)k];
        const T* Z = (k == 0) ? nullptr : corr<T>(p, k - 1);
        View3 av = (k == 0) ? full_view(p) : packed(ly.m);
        View3 cv = level_view(p, k);
        T* W = ws + p.Woff[(size_t)k + 1];
        int rc;
        if (k == 0 && (const void*)src == (const void*)dst) {
            // In place: the streaming kernel's halos would read coefficients
            // written by neighbouring tiles, so form the coefficients first
            // (each node reads only coarse nodes) and then the load vector.
            DimTables<T> tb = tables_of<T>(p, k);
            View3 wv = packed(ly.mc);
            MGR_TRY(timed(KC_COEF, k, st, [&] { return launch_coef_decompose<T>(A, av, dst, cv, W, wv, tb, st); }),
                    "coefficient launch");
            rc = stream_level<T>(p, k, false, dst, nullptr, cv, nullptr, cv, nullptr, false, st);
        } else {
            rc = stream_level<T>(p, k, true, A, Z, av, dst, cv, W, k == 0, st);
        }
        if (rc) return rc;
        rc = solve_all<T>(p, k, false, corr<T>(p, k), st);
        if (rc) return rc;
    }
    if (kt < L) {
        TailArgs<T> a = tail_args<T>(p, kt, src, dst);
        a.Z0 = (kt == 0) ? nullptr : corr<T>(p, kt - 1);
        MGR_TRY(timed(KC_TAIL, kt, st, [&] { return launch_tail<T>(a, true, st); }), "tail launch");
        return MGR_OK;
    }
    View3 cl = level_view(p, L);
    MGR_TRY(timed(KC_COPY_VIEW, L, st,
                  [&] { return launch_copy_view<T>(ws + p.Woff[(size_t)L], corr<T>(p, L - 1), packed(cl.n), dst, cl, st); }),
            "coarsest scatter");
    return MGR_OK;
}

// Two more streams per device for the recomposition (default priority,
// non-blocking): s0 for the finest level step's correction, sr for the tail;
// events for the fork, the tail and the finest correction (done[0]).  The
// enqueueing is serialised.
constexpr int kMaxLevels = 64;  // above any level count of an int64 extent
struct AuxStream {
    hipStream_t s0 = nullptr, sr = nullptr;
    hipEvent_t start = nullptr, rdone = nullptr;
    hipEvent_t done[kMaxLevels] = {};
};
std::mutex g_aux_mu;
AuxStream g_aux[64];

void destroy_aux(AuxStream& a)
{
    for (hipEvent_t& ev : a.done)
        if (ev) (void)hipEventDestroy(ev);
    if (a.start) (void)hipEventDestroy(a.start);
    if (a.rdone) (void)hipEventDestroy(a.rdone);
    if (a.s0) (void)hipStreamDestroy(a.s0);
    if (a.sr) (void)hipStreamDestroy(a.sr);
    a = AuxStream{};
}

hipError_t aux_stream(AuxStream** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    AuxStream& a = g_aux[dev];
    if (!a.sr) {
        // built aside and kept only when complete
        AuxStream n;
        e = hipStreamCreateWithFlags(&n.sr, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&n.s0, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&n.start, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&n.rdone, hipEventDisableTiming);
        for (int k = 0; k < kMaxLevels && e == hipSuccess; k++)
            e = hipEventCreateWithFlags(&n.done[k], hipEventDisableTiming);
        if (e != hipSuccess) {
            destroy_aux(n);
            return e;
        }
        a = n;
    }
    *out = &a;
    return hipSuccess;
}

// Whether the current device's auxiliary streams exist (caller holds g_aux_mu).
bool aux_ready()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
    return g_aux[dev].sr != nullptr;
}

// Recomposition, coarsest level step first: u_k = c_k + Pi (W_{k+1} - z_k).
// The correction z_k of every level step depends on the stored coefficients
// alone (its load vector is formed from them), so they are all independent
// of the coarse-to-fine chain: the finest level step's correction (s0) and
// the tail (sr) run on streams forked from the caller's, while the caller's
// stream runs the coarser corrections (sharing launches where they can) and
// the interpolations.  The latency-bound small levels thus overlap the
// bandwidth-bound finest correction; the coarser corrections use no whole-CU
// workgroup (such a workgroup waits until one CU has drained completely of
// the finest correction's long-lived workgroups).
template <typename T>
int run_recompose(const Plan& p, const void* src_, void* dst_, hipStream_t st)
{
    const int L = p.nlevels;
    if (L == 0) return identity_copy<T>(p, src_, dst_, st);
    const T* src = (const T*)src_;
    T* dst = (T*)dst_;
    T* ws = (T*)p.ws;
    const int kt = tail_start(p);
    std::unique_lock<std::mutex> lk(g_aux_mu);
    AuxStream* aux = nullptr;
    // Streams: the caller's (the coarser corrections and interpolations,
    // then the finest interpolation), sr (the tail) and s0 (the finest
    // correction), both forked from the caller's.  The coarser chain is the
    // longest, so it stays on the caller's stream: no fork delays its start,
    // and it waits on other streams only twice (the tail before its first
    // interpolation, the finest correction before the last); a wait on
    // another stream's event costs the waiting stream several microseconds
    // even when the event has long completed.
    hipStream_t sc = st;  // the stream of the tail
    if (kt > 0) {
        if (!aux_ready() && capturing(st))
            return fail(MGR_ERR_CAPTURE, "auxiliary streams not created and the stream is capturing; call mgr_prepare first");
        MGR_TRY(aux_stream(&aux), "auxiliary stream");
        MGR_TRY(hipEventRecord(aux->start, st), "fork event");
        MGR_TRY(hipStreamWaitEvent(aux->sr, aux->start, 0), "fork wait");
        MGR_TRY(hipStreamWaitEvent(aux->s0, aux->start, 0), "fork wait");
        sc = aux->sr;
    }
    if (kt < L) {
        TailArgs<T> a = tail_args<T>(p, kt, src, dst);
        a.Z0 = nullptr;
        MGR_TRY(timed(KC_TAIL, kt, sc, [&] { return launch_tail<T>(a, false, sc); }), "tail launch");
    } else {
        View3 cl = level_view(p, L);
        MGR_TRY(timed(KC_COPY_VIEW, L, sc,
                      [&] { return launch_copy_view<T>(src, nullptr, cl, ws + p.Woff[(size_t)L], packed(cl.n), sc); }),
                "coarsest gather");
    }
    if (kt > 0) {
        MGR_TRY(hipEventRecord(aux->rdone, sc), "tail event");
        // one level step's correction on its own launches (the finest on s0)
        auto single = [&](int k) -> int {
            hipStream_t sk = (k == 0) ? aux->s0 : st;
            View3 cv = level_view(p, k);
            T* z = ws + p.Zrec[(size_t)k];
            int rc = stream_level<T>(p, k, false, src, nullptr, cv, nullptr, cv, nullptr, false, sk, z);
            if (rc) return rc;
            rc = solve_all<T>(p, k, false, z, sk, (k == 0) ? ws + p.Yb : ws + p.Yb2, k == 0);
            if (rc) return rc;
            if (k == 0) MGR_TRY(hipEventRecord(aux->done[0], sk), "level event");
            return MGR_OK;
        };
        // the finest step's correction first, so that its launches reach the
        // device together with the coarser chain's
        int rc = single(0);
        if (rc) return rc;
        // the coarser steps' corrections (coarsest first) share launches
        // where their solves allow it: one load-vector launch and one launch
        // per dimension for up to kMultiLevels steps, instead of a chain of
        // small launches per step
        std::vector<int> group;
        auto flush = [&]() -> int {
            const int n = (int)group.size();
            if (n == 0) return MGR_OK;
            if (n == 1) {
                const int rc1 = single(group[0]);
                group.clear();
                return rc1;
            }
            StreamArgs<T> la[kMultiLevels];
            T* Fz[kMultiLevels];
            View3 fv[kMultiLevels];
            for (int i = 0; i < n; i++) {
                const int k = group[(size_t)i];
                const LevelLayout& ly = p.lv[(size_t)k];
                StreamArgs<T>& a = la[i];
                std::memset(&a, 0, sizeof(a));
                a.A = src;
                a.av = level_view(p, k);
                a.cv = a.av;
                a.wv = packed(ly.mc);
                a.F = Fz[i] = ws + p.Zrec[(size_t)k];
                a.fv = fv[i] = packed(ly.mc);
                a.tb = tables_of<T>(p, k);
            }
            MGR_TRY(timed(KC_STREAM_LOAD, group[0], st, [&] { return launch_stream_load_multi<T>(la, n, st); }),
                    "shared load-vector launch");
            for (int sd = 0; sd < 3; sd++) {
                const int d = 2 - sd;
                if (!p.active[d]) continue;
                SolveTables<T> tb[kMultiLevels];
                for (int i = 0; i < n; i++) tb[i] = solve_tables_of<T>(p, group[(size_t)i], d);
                MGR_TRY(timed(KC_SOLVE, group[0], st, [&] { return launch_solve_multi<T>(Fz, fv, d, tb, n, st); }),
                        "shared solve launch");
            }
            group.clear();
            return MGR_OK;
        };
        for (int k = kt - 1; k >= 1; k--) {
            bool fits = true;
            for (int d = 0; d < 3; d++)
                if (p.active[d])
                    fits = fits && solve_multi_fits<T>(packed(p.lv[(size_t)k].mc), d, solve_tables_of<T>(p, k, d));
            if (fits) {
                group.push_back(k);
                if ((int)group.size() == kMultiLevels && (rc = flush())) return rc;
            } else {
                if ((rc = flush()) || (rc = single(k))) return rc;
            }
        }
        if ((rc = flush())) return rc;
        // the coarsest values (tail) before the first interpolation
        MGR_TRY(hipStreamWaitEvent(st, aux->rdone, 0), "tail wait");
    }
    for (int k = kt - 1; k >= 0; k--) {
        const LevelLayout& ly = p.lv[(size_t)k];
        View3 cv = level_view(p, k);
        hipStream_t sk = st;
        if (k == 0) MGR_TRY(hipStreamWaitEvent(st, aux->done[0], 0), "join wait");  // the finest correction
        StreamArgs<T> a;
        a.A = src;
        a.Z = ws + p.Zrec[(size_t)k];
        a.av = cv;
        a.C = (k == 0) ? dst : ws + p.Woff[(size_t)k];
        a.cv = (k == 0) ? full_view(p) : packed(ly.m);
        a.W = ws + p.Woff[(size_t)k + 1];
        a.wv = packed(ly.mc);
        a.F = nullptr;
        a.fv = packed(ly.mc);
        a.tb = tables_of<T>(p, k);
        a.write_coarse = 0;
        a.chunk = a.nt1 = a.nt2 = a.nch = 0;
        MGR_TRY(timed(KC_INTERP, k, sk, [&] { return launch_stream_recon<T>(a, sk); }),
                "interpolation launch");
    }
    return MGR_OK;
}

template <typename T>
int run_adjoint(const Plan& p, const void* src_, void* dst_, hipStream_t st)
{
    const int L = p.nlevels;
    if (L == 0) return identity_copy<T>(p, src_, dst_, st);
    const T* src = (const T*)src_;
    T* dst = (T*)dst_;
    T* ws = (T*)p.ws;
    View3 cl = level_view(p, L);
    MGR_TRY(timed(KC_COPY_VIEW, L, st,
                  [&] { return launch_copy_view<T>(src, nullptr, cl, ws + p.Woff[(size_t)L], packed(cl.n), st); }),
            "coarsest gather");
    for (int k = L - 1; k >= 0; k--) {
        const LevelLayout& ly = p.lv[(size_t)k];
        T* G = ws + p.Woff[(size_t)k + 1];
        View3 gv = packed(ly.mc);
        int64_t nc = ly.mc[0] * ly.mc[1] * ly.mc[2];
        MGR_TRY(hipMemcpyAsync(ws + p.F, G, (size_t)nc * sizeof(T), hipMemcpyDeviceToDevice, st),
                "adjoint copy");
        int rc = solve_all<T>(p, k, true, ws + p.F, st);
        if (rc) return rc;
        // the level-grid output: fine nodes g + (M P) y, coarse nodes G minus
        // the transposed interpolation of the fine outputs; in place, the
        // finest step goes through the workspace (its tiles re-read halo
        // inputs that a neighbouring tile has overwritten)
        const bool via_tb = (k == 0) && (const void*)src == (const void*)dst;
        T* out = (k == 0) ? (via_tb ? ws + p.Tb : dst) : ws + p.Woff[(size_t)k];
        View3 ov = (k == 0) ? full_view(p) : packed(ly.m);
        MGR_TRY(timed(KC_ADJOINT, k, st,
                      [&] {
                          return launch_stream_adjoint<T>(src, level_view(p, k), ws + p.F, G, gv, out, ov,
                                                          tables_of<T>(p, k), st);
                      }),
                "adjoint level launch");
        if (via_tb) {
            const size_t bytes = (size_t)(p.n[0] * p.n[1] * p.n[2]) * sizeof(T);
            MGR_TRY(hipMemcpyAsync(dst, ws + p.Tb, bytes, hipMemcpyDeviceToDevice, st), "adjoint copy-out");
        }
    }
    return MGR_OK;
}

// Transpose of the recomposition (D^{-T}), fine to coarse.  Per level step,
// with g the level grid (the input at k = 0, else W_k):
//   Ft = P^T g_f (load-vector pass with P^T as its stencil; coarse positions
//        read as zero),
//   G = g_c + Ft -> W_{k+1} (the next step's grid), and -G into the solve
//        buffer,
//   y = M_c^{-1} (-G) (solves, dimensions first to last),
//   out_f = g_f + (M P) y at the level grid's fine-only nodes, written to their
//        final places in dst (the adjoint kernel; the values it also writes at
//        coarse positions are overwritten by the coarser steps),
// and finally the coarsest grid W_L to its nodes.  In place, each step reads
// the input's coarse values (into W_{k+1}) before the expansion overwrites
// them; the finest step's expansion, whose tiles also read halo inputs of
// their neighbours, writes to the workspace and is copied back.
template <typename T>
int run_recompose_adjoint(const Plan& p, const void* src_, void* dst_, hipStream_t st)
{
    const int L = p.nlevels;
    if (L == 0) return identity_copy<T>(p, src_, dst_, st);
    const T* src = (const T*)src_;
    T* dst = (T*)dst_;
    T* ws = (T*)p.ws;
    for (int k = 0; k < L; k++) {
        const LevelLayout& ly = p.lv[(size_t)k];
        const T* g = (k == 0) ? src : ws + p.Woff[(size_t)k];
        const View3 gv = (k == 0) ? full_view(p) : packed(ly.m);
        T* F = corr<T>(p, k);
        const View3 cv = packed(ly.mc);
        {
            StreamArgs<T> a;
            a.A = g;
            a.Z = nullptr;
            a.av = gv;
            a.C = nullptr;
            a.cv = gv;
            a.W = nullptr;
            a.wv = cv;
            a.F = F;
            a.fv = cv;
            a.tb = pt_tables_of<T>(p, k);
            a.write_coarse = 0;
            a.chunk = a.nt1 = a.nt2 = a.nch = 0;
            MGR_TRY(timed(KC_STREAM_LOAD, k, st, [&] { return launch_stream_level<T>(a, false, st); }),
                    "transposed interpolation launch");
        }
        View3 gc = gv;  // the coarse nodes of the level grid
        for (int d = 0; d < 3; d++) {
            gc.n[d] = ly.mc[d];
            gc.s[d] = p.active[d] ? 2 * gv.s[d] : gv.s[d];
        }
        T* W = ws + p.Woff[(size_t)k + 1];
        MGR_TRY(launch_add_split<T>(g, gc, F, W, F, st), "combine launch");
        int rc = solve_all<T>(p, k, true, F, st);
        if (rc) return rc;
        // in place, the finest step's tiles would re-read halo inputs that a
        // neighbouring tile has already overwritten: it goes through the
        // workspace and is copied back (its coarse positions are overwritten
        // by the coarser steps anyway)
        const bool via_tb = (k == 0) && (const void*)src == (const void*)dst;
        T* out = via_tb ? ws + p.Tb : dst;
        const View3 ov = via_tb ? full_view(p) : level_view(p, k);
        MGR_TRY(timed(KC_ADJOINT, k, st,
                      [&] { return launch_stream_adjoint<T>(g, gv, F, W, cv, out, ov, tables_of<T>(p, k), st); }),
                "recomposition adjoint level launch");
        if (via_tb) {
            const size_t bytes = (size_t)(p.n[0] * p.n[1] * p.n[2]) * sizeof(T);
            MGR_TRY(hipMemcpyAsync(dst, ws + p.Tb, bytes, hipMemcpyDeviceToDevice, st), "adjoint copy-out");
        }
    }
    View3 cl = level_view(p, L);
    MGR_TRY(timed(KC_COPY_VIEW, L, st,
                  [&] { return launch_copy_view<T>(ws + p.Woff[(size_t)L], nullptr, packed(cl.n), dst, cl, st); }),
            "coarsest scatter");
    return MGR_OK;
}

// ---- general grids: 1..4 dimensions of any size >= 3 -------------------------
// Level grids keep, along each dimension, the multiples of 2^k and the last
// node: the level-k grid of a dimension of n nodes has ceil((n - 1) / 2^k) + 1
// nodes, and a level grid of m nodes has m / 2 + 1 coarse nodes (its even
// positions and its last one).  For 2^k + 1 sizes this is the usual nested
// grid, which the fused path handles; the general path (mgr_general.hip)
// runs any other shape, and every shape of four dimensions.
int64_t gen_lsize(int64_t n, int k) { return ((n - 2) >> k) + 2; }

// Level steps after which a dimension of n >= 3 nodes is down to two nodes.
int gen_steps_to_two(int64_t n)
{
    int k = 0;
    while (((int64_t)1 << k) < n - 1) k++;
    return k;
}

bool dyadic_shape(int ndim, const int64_t* shape)
{
    if (ndim < 1 || ndim > kMaxDim) return false;
    for (int d = 0; d < ndim; d++)
        if (shape[d] < 3 || log2_exact(shape[d] - 1) < 1) return false;
    return true;
}

// Validation for every shape the library accepts: ndim 1..4, every size >= 3;
// the full decomposition stops when the shortest level grid has 3 nodes, and
// 0 .. full + 1 level steps are accepted.  (For 2^k + 1 sizes this is the
// same as validate.)
int validate_general(int dtype, int ndim, const int64_t* shape, const double* const* coords, int* nlevels)
{
    if (dtype != MGR_F32 && dtype != MGR_F64) return fail(MGR_ERR_ARG, "dtype must be MGR_F32 or MGR_F64");
    if (ndim < 1 || ndim > kGenMaxDim) return fail(MGR_ERR_ARG, "ndim must be 1..4");
    if (!shape) return fail(MGR_ERR_ARG, "shape is NULL");
    if (dyadic_shape(ndim, shape)) return validate(dtype, ndim, shape, coords, nlevels);
    int kmin = 64;
    for (int d = 0; d < ndim; d++) {
        if (shape[d] < 3)
            return fail(MGR_ERR_SHAPE, "shape[" + std::to_string(d) + "] = " + std::to_string(shape[d]) + " is below 3");
        kmin = std::min(kmin, gen_steps_to_two(shape[d]));
    }
    if (*nlevels == -1) *nlevels = kmin - 1;
    if (*nlevels < 0 || *nlevels > kmin)
        return fail(MGR_ERR_LEVELS, "nlevels = " + std::to_string(*nlevels) + " outside 0.." + std::to_string(kmin) +
                                        " (or -1)");
    if (coords) {
        for (int d = 0; d < ndim; d++) {
            const double* x = coords[d];
            if (!x) continue;
            for (int64_t i = 0; i < shape[d]; i++)
                if (!std::isfinite(x[i]) || (i > 0 && !(x[i] > x[i - 1])))
                    return fail(MGR_ERR_COORDS, "coords[" + std::to_string(d) +
                                                    "] not finite and strictly increasing at " + std::to_string(i));
        }
    }
    return MGR_OK;
}

// Interpolation weights and load-vector rows of a level grid of any length m
// (positions y).  Coarse node i sits at fine position f(i) = 2i, or m - 1 for
// the last one; K = P^T M row i covers fine nodes f(i) - 2 .. f(i) + 2.
struct GenDimTab {
    std::vector<double> wl, wh, K;
};
GenDimTab build_dim_general(const std::vector<double>& y)
{
    const int64_t m = (int64_t)y.size(), mc = m / 2 + 1;
    auto fine = [m](int64_t j) { return (j & 1) && j != m - 1; };
    GenDimTab t;
    t.wl.assign((size_t)m, 0.0);
    t.wh.assign((size_t)m, 0.0);
    for (int64_t j = 1; j < m; j++) {
        if (!fine(j)) continue;
        const double a = (y[(size_t)j] - y[(size_t)(j - 1)]) / (y[(size_t)(j + 1)] - y[(size_t)(j - 1)]);
        t.wl[(size_t)j] = 1.0 - a;
        t.wh[(size_t)j] = a;
    }
    auto h = [&](int64_t j) { return (j >= 0 && j < m - 1) ? y[(size_t)(j + 1)] - y[(size_t)j] : 0.0; };
    auto M = [&](int64_t r, int64_t c) {
        if (c == r) return 2.0 * (h(r - 1) + h(r));
        if (c == r - 1) return h(r - 1);
        if (c == r + 1) return h(r);
        return 0.0;
    };
    t.K.assign((size_t)(5 * mc), 0.0);
    for (int64_t i = 0; i < mc; i++) {
        const int64_t f = (i == mc - 1) ? m - 1 : 2 * i;
        // P(l, i): 1 at the coarse node itself, the interpolation weight of a
        // fine neighbour towards it
        auto P = [&](int64_t l) {
            if (l == f) return 1.0;
            if (l < 0 || l >= m || !fine(l)) return 0.0;
            return (l == f - 1) ? t.wh[(size_t)l] : t.wl[(size_t)l];
        };
        for (int tt = 0; tt < 5; tt++) {
            const int64_t c = f - 2 + tt;
            if (c < 0 || c >= m) continue;
            double s = 0.0;
            for (int64_t l = f - 1; l <= f + 1; l++)
                if (l >= 0 && l < m) s += P(l) * M(l, c);
            t.K[(size_t)(5 * i + tt)] = s;
        }
    }
    return t;
}

struct GenLevelHost {
    int64_t m[kGenMaxDim], mc[kGenMaxDim];
    size_t wl[kGenMaxDim], wh[kGenMaxDim], K[kGenMaxDim];
    size_t solve[kGenMaxDim][10];  // L, U, IP, A, B, ssub, ssup, sl, sip, su
    int S[kGenMaxDim];
};

struct GenPlan {
    int device = 0, dtype = 0, nd = 0, nlevels = 0;
    int64_t n[kGenMaxDim] = {1, 1, 1, 1}, st[kGenMaxDim] = {0, 0, 0, 0};
    std::vector<GenLevelHost> lv;  // level steps 0 .. L - 1
    void* tables = nullptr;
    void* ws = nullptr;
    size_t tables_bytes = 0, ws_bytes = 0;
    std::vector<size_t> Woff;  // packed level grids W_k, k = 1..L (index k)
    size_t A = 0, B = 0, Yb = 0;
};
std::map<std::string, std::unique_ptr<GenPlan>> g_gen_plans;

void free_gen_plan(GenPlan& p)
{
    if (p.tables) (void)hipFree(p.tables);
    if (p.ws) (void)hipFree(p.ws);
    p.tables = p.ws = nullptr;
}

template <typename T>
int build_gen_plan(GenPlan& p, const double* const* coords)
{
    const int nd = p.nd, L = p.nlevels;
    std::vector<std::vector<double>> X((size_t)nd);
    for (int d = 0; d < nd; d++) X[(size_t)d] = axis_positions(p.n[d], coords ? coords[d] : nullptr);
    std::vector<T> host;
    p.lv.resize((size_t)L);
    size_t big = 0, yb = 64;
    for (int k = 0; k < L; k++) {
        GenLevelHost& ly = p.lv[(size_t)k];
        int64_t box[kGenMaxDim];
        for (int d = 0; d < nd; d++) {
            const int64_t m = gen_lsize(p.n[d], k);
            ly.m[d] = m;
            ly.mc[d] = m / 2 + 1;
            std::vector<double> y((size_t)m), yc((size_t)ly.mc[d]);
            for (int64_t j = 0; j < m; j++) y[(size_t)j] = X[(size_t)d][(size_t)std::min(j << k, p.n[d] - 1)];
            for (int64_t i = 0; i < ly.mc[d]; i++) yc[(size_t)i] = y[(size_t)(i == ly.mc[d] - 1 ? m - 1 : 2 * i)];
            GenDimTab t = build_dim_general(y);
            push_table(host, t.wl, &ly.wl[d]);
            push_table(host, t.wh, &ly.wh[d]);
            push_table(host, t.K, &ly.K[d]);
            SolveTab sv = build_solve(yc);
            ly.S[d] = sv.S;
            const std::vector<double>* parts[10] = {&sv.L, &sv.U, &sv.IP, &sv.A, &sv.B,
                                                    &sv.ssub, &sv.ssup, &sv.sl, &sv.sip, &sv.su};
            for (int q = 0; q < 10; q++) push_table(host, *parts[q], &ly.solve[d][q]);
            box[d] = m;
        }
        // load-vector passes, last dimension first: intermediate sizes
        for (int d = nd - 1; d >= 0; d--) {
            box[d] = ly.mc[d];
            int64_t v = 1;
            for (int e = 0; e < nd; e++) v *= box[e];
            big = std::max(big, (size_t)v);
        }
        // three-phase solve scratch: two values per segment and fibre
        int64_t vc = 1;
        for (int e = 0; e < nd; e++) vc *= ly.mc[e];
        for (int d = 0; d < nd; d++) yb = std::max(yb, (size_t)(2 * (int64_t)ly.S[d] * (vc / ly.mc[d])) + 64);
    }
    const size_t al = 256 / sizeof(T);
    size_t off = 0;
    p.Woff.assign((size_t)L + 1, 0);
    for (int k = 1; k <= L; k++) {
        int64_t v = 1;
        for (int d = 0; d < nd; d++) v *= gen_lsize(p.n[d], k);
        p.Woff[(size_t)k] = off;
        off = align_up(off + (size_t)v, al);
    }
    p.A = off; off = align_up(off + big, al);
    p.B = off; off = align_up(off + big, al);
    p.Yb = off; off = align_up(off + yb, al);
    p.ws_bytes = off * sizeof(T);
    p.tables_bytes = host.size() * sizeof(T);
    if (p.ws_bytes + p.tables_bytes > workspace_cap())
        return fail(MGR_ERR_ALLOC, "workspace of " + std::to_string(p.ws_bytes) + " bytes exceeds MGR_WORKSPACE_MAX");
    if (p.tables_bytes) {
        hipError_t e = hipMalloc(&p.tables, p.tables_bytes);
        if (e != hipSuccess) {
            p.tables = nullptr;
            return fail(MGR_ERR_ALLOC, std::string("hipMalloc tables: ") + hipGetErrorString(e));
        }
        e = hipMemcpy(p.tables, host.data(), p.tables_bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "upload tables");
    }
    if (p.ws_bytes) {
        hipError_t e = hipMalloc(&p.ws, p.ws_bytes);
        if (e != hipSuccess) {
            p.ws = nullptr;
            return fail(MGR_ERR_ALLOC, std::string("hipMalloc workspace: ") + hipGetErrorString(e));
        }
    }
    return MGR_OK;
}

int get_gen_plan(int dtype, int ndim, const int64_t* shape, const double* const* coords, int nlevels,
                 hipStream_t st, bool check_capture, GenPlan** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    const std::string key = plan_key(dev, dtype, ndim, shape, coords, nlevels);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_gen_plans.find(key);
    if (it != g_gen_plans.end()) {
        *out = it->second.get();
        return MGR_OK;
    }
    if (check_capture && capturing(st))
        return fail(MGR_ERR_CAPTURE, "problem not prepared and the stream is capturing; call mgr_prepare first");
    auto p = std::make_unique<GenPlan>();
    p->device = dev;
    p->dtype = dtype;
    p->nd = ndim;
    p->nlevels = nlevels;
    int64_t s = 1;
    for (int d = ndim - 1; d >= 0; d--) {
        p->n[d] = shape[d];
        p->st[d] = s;
        s *= shape[d];
    }
    int rc = (dtype == MGR_F32) ? build_gen_plan<float>(*p, coords) : build_gen_plan<double>(*p, coords);
    if (rc) {
        free_gen_plan(*p);
        return rc;
    }
    *out = p.get();
    g_gen_plans.emplace(key, std::move(p));
    return MGR_OK;
}

// Device view of level step k (k = L: sizes only, for the coarsest grid).
template <typename T>
GenLevel<T> gen_level(const GenPlan& p, int k)
{
    GenLevel<T> a;
    std::memset(&a, 0, sizeof(a));
    a.nd = p.nd;
    const T* tb = (const T*)p.tables;
    for (int d = 0; d < p.nd; d++) {
        a.n[d] = p.n[d];
        a.st[d] = p.st[d];
        a.m[d] = gen_lsize(p.n[d], k);
        a.mc[d] = a.m[d] / 2 + 1;
        if (k < p.nlevels) {
            const GenLevelHost& ly = p.lv[(size_t)k];
            a.wl[d] = tb + ly.wl[d];
            a.wh[d] = tb + ly.wh[d];
            a.K[d] = tb + ly.K[d];
        }
    }
    return a;
}

// z of level step k into the plan's A or B buffer: the load vector of the
// level grid's coefficients (read from y at their nodes), then the solves;
// returns the buffer.
template <typename T>
int gen_correction(const GenPlan& p, int k, const T* y, hipStream_t st, T** zout)
{
    T* ws = (T*)p.ws;
    const GenLevel<T> a = gen_level<T>(p, k);
    const GenLevelHost& ly = p.lv[(size_t)k];
    const int nd = p.nd;
    GenPass ps;
    std::memset(&ps, 0, sizeof(ps));
    for (int d = 0; d < nd; d++) ps.in[d] = ps.out[d] = ly.m[d];
    T* bufs[2] = {ws + p.A, ws + p.B};
    const T* in = nullptr;
    T* out = nullptr;
    for (int s = 0; s < nd; s++) {
        const int d = nd - 1 - s;
        ps.d = d;
        ps.full = (s == 0);
        for (int e = 0; e < nd; e++) ps.in[e] = ps.out[e];
        ps.out[d] = ly.mc[d];
        out = bufs[s & 1];
        MGR_TRY(timed(KC_STREAM_LOAD, k, st, [&] { return launch_gen_masstrans<T>(in, y, out, a, ps, k, st); }),
                "load-vector launch");
        in = out;
    }
    const T* tb = (const T*)p.tables;
    for (int s = 0; s < nd; s++) {
        const int d = nd - 1 - s;
        int64_t inner = 1, outer = 1;
        for (int e = d + 1; e < nd; e++) inner *= ly.mc[e];
        for (int e = 0; e < d; e++) outer *= ly.mc[e];
        SolveTables<T> t;
        const T** f[10] = {&t.L, &t.U, &t.IP, &t.A, &t.B, &t.ssub, &t.ssup, &t.sl, &t.sip, &t.su};
        for (int q = 0; q < 10; q++) *f[q] = tb + ly.solve[d][q];
        t.S = ly.S[d];
        MGR_TRY(timed(KC_SOLVE, k, st,
                      [&] { return launch_solve_fibres<T>(out, ly.mc[d], inner, outer, t, ws + p.Yb, st); }),
                "solve launch");
    }
    *zout = out;
    return MGR_OK;
}

template <typename T>
int run_gen_decompose(const GenPlan& p, const void* src_, void* dst_, hipStream_t st)
{
    const int L = p.nlevels;
    const T* src = (const T*)src_;
    T* dst = (T*)dst_;
    T* ws = (T*)p.ws;
    int64_t N = 1;
    for (int d = 0; d < p.nd; d++) N *= p.n[d];
    if (L == 0) {
        if (src != dst) MGR_TRY(hipMemcpyAsync(dst, src, (size_t)N * sizeof(T), hipMemcpyDeviceToDevice, st), "copy");
        return MGR_OK;
    }
    T* z = nullptr;
    for (int k = 0; k < L; k++) {
        const GenLevel<T> a = gen_level<T>(p, k);
        T* Wk = (k == 0) ? nullptr : ws + p.Woff[(size_t)k];
        T* Wn = ws + p.Woff[(size_t)k + 1];
        MGR_TRY(timed(KC_COEF, k, st, [&] { return launch_gen_coef<T>(src, Wk, dst, Wn, a, k, st); }),
                "coefficient launch");
        int rc = gen_correction<T>(p, k, dst, st, &z);
        if (rc) return rc;
        int64_t vc = 1;
        for (int d = 0; d < p.nd; d++) vc *= a.mc[d];
        MGR_TRY(launch_gen_axpy<T>(Wn, z, vc, T(1), st), "correction launch");
    }
    const GenLevel<T> aL = gen_level<T>(p, L);
    MGR_TRY(timed(KC_COPY_VIEW, L, st,
                  [&] { return launch_gen_scatter<T>(dst, ws + p.Woff[(size_t)L], nullptr, aL, L, true, st); }),
            "coarsest scatter");
    return MGR_OK;
}

template <typename T>
int run_gen_recompose(const GenPlan& p, const void* src_, void* dst_, hipStream_t st)
{
    const int L = p.nlevels;
    const T* src = (const T*)src_;
    T* dst = (T*)dst_;
    T* ws = (T*)p.ws;
    int64_t N = 1;
    for (int d = 0; d < p.nd; d++) N *= p.n[d];
    if (L == 0) {
        if (src != dst) MGR_TRY(hipMemcpyAsync(dst, src, (size_t)N * sizeof(T), hipMemcpyDeviceToDevice, st), "copy");
        return MGR_OK;
    }
    const GenLevel<T> aL = gen_level<T>(p, L);
    MGR_TRY(timed(KC_COPY_VIEW, L, st,
                  [&] { return launch_gen_scatter<T>(const_cast<T*>(src), ws + p.Woff[(size_t)L], nullptr, aL, L,
                                                     false, st); }),
            "coarsest gather");
    for (int k = L - 1; k >= 0; k--) {
        const GenLevel<T> a = gen_level<T>(p, k);
        T* z = nullptr;
        int rc = gen_correction<T>(p, k, src, st, &z);
        if (rc) return rc;
        T* Wn = ws + p.Woff[(size_t)k + 1];
        int64_t vc = 1;
        for (int d = 0; d < p.nd; d++) vc *= a.mc[d];
        MGR_TRY(launch_gen_axpy<T>(Wn, z, vc, T(-1), st), "correction launch");
        T* Wk = (k == 0) ? nullptr : ws + p.Woff[(size_t)k];
        MGR_TRY(timed(KC_INTERP, k, st, [&] { return launch_gen_interp<T>(src, Wn, dst, Wk, a, k, st); }),
                "interpolation launch");
    }
    return MGR_OK;
}

enum Direction { DIR_DEC, DIR_REC, DIR_ADJ, DIR_RADJ };

int run(Direction dir, const void* src, void* dst, int dtype, int ndim, const int64_t* shape,
        const double* const* coords, int nlevels, void* stream)
{
    g_err.clear();
    if (!src || !dst) return fail(MGR_ERR_ARG, "src or dst is NULL");
    hipStream_t st = (hipStream_t)stream;
    if (shape && !dyadic_shape(ndim, shape)) {
        int rc = validate_general(dtype, ndim, shape, coords, &nlevels);
        if (rc) return rc;
        if (dir != DIR_DEC && dir != DIR_REC)
            return fail(MGR_ERR_SHAPE, "the adjoints take 1- to 3-D grids of 2^k + 1 nodes per dimension");
        GenPlan* gp = nullptr;
        rc = get_gen_plan(dtype, ndim, shape, coords, nlevels, st, true, &gp);
        if (rc) return rc;
        if (dtype == MGR_F32)
            return dir == DIR_DEC ? run_gen_decompose<float>(*gp, src, dst, st) : run_gen_recompose<float>(*gp, src, dst, st);
        return dir == DIR_DEC ? run_gen_decompose<double>(*gp, src, dst, st) : run_gen_recompose<double>(*gp, src, dst, st);
    }
    Plan* p = nullptr;
    int rc = get_plan(dtype, ndim, shape, coords, nlevels, st, true, &p);
    if (rc) return rc;
    if (dtype == MGR_F32) {
        switch (dir) {
            case DIR_DEC: return run_decompose<float>(*p, src, dst, st);
            case DIR_REC: return run_recompose<float>(*p, src, dst, st);
            case DIR_RADJ: return run_recompose_adjoint<float>(*p, src, dst, st);
            default: return run_adjoint<float>(*p, src, dst, st);
        }
    }
    switch (dir) {
        case DIR_DEC: return run_decompose<double>(*p, src, dst, st);
        case DIR_REC: return run_recompose<double>(*p, src, dst, st);
        case DIR_RADJ: return run_recompose_adjoint<double>(*p, src, dst, st);
        default: return run_adjoint<double>(*p, src, dst, st);
    }
}

const char* const kKernelNames[KC_COUNT] = {
    "coef_decompose", "solve", "interp_recompose",
    "adjoint", "copy_view", "bench_copy", "stream_dec", "stream_load", "tail", "batch"};

// ---- batched decomposition (waves of work items, mgr_batch.hip) --------------
constexpr int kStagesPerLevel = 10;  // stream + up to three solves of up to three phases
constexpr int kMaxBatchChunk = 128;  // coarse planes per streaming item (the kernel's LDS tables)

struct BatchPlan {
    int dtype = 0, nfields = 0, device = 0;
    // per-field plans built for the batch alone (tables only; the batch's
    // workspace replaces theirs), so the cache and mgr_finalize never touch them
    std::vector<std::unique_ptr<Plan>> plans;
    std::vector<int> kt;           // first tail level step per field
    std::vector<size_t> wsoff;     // byte offset of each field's workspace
    void* ws = nullptr;            // the fields' workspaces (same layout as their plans')
    void* dev = nullptr;           // device tables (one allocation)
    size_t off_items = 0, off_sargs = 0, off_solves = 0, off_scat = 0, off_tail = 0, off_tailf = 0, off_ptrs = 0,
           off_args = 0, dev_bytes = 0;
    std::vector<std::pair<int, int>> waves;  // (first item, items) per launch
    int n_items = 0, n_tail = 0;
    int chunk = 8, tuned = 0;
    int wide = 0;                  // 3-D streaming items on the wide tile geometry
    int64_t bytes = 0;             // input bytes of the batch
    // persistent form (mgr_queue.h): queues (one per XCD), the item at each
    // queue position and each queue's first position, the group of each
    // position, dependency group and size of each group (host copies for the
    // host check), device offsets of those tables and of the queue words
    // (abort, err, next[kMaxQueues], done[groups])
    int persistent = 0;
    unsigned poll_limit = 1u << 20;
    double model[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};  // fitted a, x, y, z (batch_terms) per launch form
    int nq = 1, ran_persistent = 0;  // ran_persistent: a persistent run since the tables were uploaded
    std::vector<int> qorder, qstart, qgrp, qdep, qneed;
    size_t off_qorder = 0, off_qgrp = 0, off_qdep = 0, off_qneed = 0, off_qwords = 0;
};

// Queues of the persistent form.  Each field goes to one of nq queues (one
// per XCD), longest estimated work first to the least loaded queue; a
// field's estimate is its streaming bytes plus, per stage, the bytes an XCD
// moves in a stage's fixed latency (about 4 MB).  A queue lists its fields'
// items wave by wave (keeping their order within a wave); the items of one
// field within one wave form a group, which depends on the previous group
// of the same field.  order: item at each position; start: each queue's
// first position (nq + 1 entries); grp: group of each position.
void batch_queues(const BatchPlan& b, const std::vector<BatchItem>& items,
                  const std::vector<std::pair<int, int>>& waves, int nq, std::vector<int>& order,
                  std::vector<int>& start, std::vector<int>& grp, std::vector<int>& dep, std::vector<int>& need)
{
    const int nf = b.nfields;
    const double esz = (b.dtype == MGR_F64) ? 8.0 : 4.0;
    std::vector<double> cost((size_t)nf, 0.0);
    for (int f = 0; f < nf; f++) {
        const Plan& p = *b.plans[(size_t)f];
        for (int k = 0; k < b.kt[(size_t)f]; k++) {
            const LevelLayout& ly = p.lv[(size_t)k];
            cost[(size_t)f] += 2.0 * (double)(ly.m[0] * ly.m[1] * ly.m[2]) * esz;
        }
    }
    for (const auto& w : waves) {
        int cur = -1;
        for (int i = w.first; i < w.first + w.second; i++) {
            const int f = items[(size_t)i].field;
            if (f != cur) cost[(size_t)f] += 4.0e6;
            cur = f;
        }
    }
    std::vector<int> byc((size_t)nf);
    for (int f = 0; f < nf; f++) byc[(size_t)f] = f;
    std::stable_sort(byc.begin(), byc.end(), [&](int a, int c) { return cost[(size_t)a] > cost[(size_t)c]; });
    std::vector<double> load((size_t)nq, 0.0);
    std::vector<int> fq((size_t)nf, 0);
    for (int f : byc) {
        const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        fq[(size_t)f] = q;
        load[(size_t)q] += cost[(size_t)f];
    }
    order.clear();
    grp.clear();
    dep.clear();
    need.clear();
    start.assign((size_t)nq + 1, 0);
    std::vector<int> last((size_t)nf, -1);
    for (int q = 0; q < nq; q++) {
        start[(size_t)q] = (int)order.size();
        for (const auto& w : waves) {
            int cur = -1, g = -1;
            for (int i = w.first; i < w.first + w.second; i++) {
                const int f = items[(size_t)i].field;
                if (fq[(size_t)f] != q) continue;
                if (f != cur) {
                    g = (int)need.size();
                    need.push_back(0);
                    dep.push_back(last[(size_t)f]);
                    last[(size_t)f] = g;
                    cur = f;
                }
                order.push_back(i);
                grp.push_back(g);
                need[(size_t)g]++;
            }
        }
    }
    start[(size_t)nq] = (int)order.size();
}

// XCDs of the current device (queues of the persistent form).
int device_queue_count()
{
    int dev = 0, n = 1;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess)
        n = 1;
    return std::min(std::max(n, 1), kMaxQueues);
}

QueueTables queue_tables(const BatchPlan& b, const int* grp, const int* dep, const int* need, const int* order)
{
    QueueTables qt;
    qt.grp = grp;
    qt.dep = dep;
    qt.need = need;
    qt.order = order;
    qt.nq = b.nq;
    for (int q = 0; q <= kMaxQueues; q++) qt.start[q] = b.qstart[(size_t)std::min(q, b.nq)];
    return qt;
}

QueueState queue_state(int* words)
{
    QueueState qs;
    qs.abort = words;
    qs.err = words + 1;
    qs.next = words + 2;
    qs.done = words + kQueueWordsFixed;
    return qs;
}

template <typename T>
struct BatchTables {
    std::vector<BatchItem> items;
    std::vector<std::pair<int, int>> waves;
    std::vector<StreamArgs<T>> sargs;
    std::vector<BatchSolve<T>> solves;
    std::vector<BatchScatter<T>> scatters;
    std::vector<TailArgs<T>> tail;
    std::vector<int> tailf;
};

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Work items of every field, grouped into waves (level step k, stage s) in
// that order; within a wave, field by field.
template <typename T>
int batch_tables(BatchPlan& b, int chunk, BatchTables<T>& out)
{
    const int nf = b.nfields;
    int maxL = 1;
    for (int f = 0; f < nf; f++) maxL = std::max(maxL, b.plans[(size_t)f]->nlevels);
    std::vector<std::vector<std::vector<std::vector<BatchItem>>>> st((size_t)nf);
    for (int f = 0; f < nf; f++) {
        const Plan& p = *b.plans[(size_t)f];
        void* wsf = (char*)b.ws + b.wsoff[(size_t)f];
        T* ws = (T*)wsf;
        st[(size_t)f].resize((size_t)b.kt[(size_t)f]);
        for (int k = 0; k < b.kt[(size_t)f]; k++) {
            const LevelLayout& ly = p.lv[(size_t)k];
            auto& stages = st[(size_t)f][(size_t)k];
            // streaming stage
            StreamArgs<T> a;
            std::memset(&a, 0, sizeof(a));
            a.A = (k == 0) ? nullptr : ws + p.Woff[(size_t)k];
            a.Z = (k == 0) ? nullptr : corr<T>(p, k - 1, wsf);
            a.av = (k == 0) ? full_view(p) : packed(ly.m);
            a.C = nullptr;
            a.cv = level_view(p, k);
            a.W = ws + p.Woff[(size_t)k + 1];
            a.wv = packed(ly.mc);
            a.F = corr<T>(p, k, wsf);
            a.fv = packed(ly.mc);
            a.tb = tables_of<T>(p, k);
            a.write_coarse = (k == 0) ? 1 : 0;
            const bool act0 = a.av.n[0] > 1, act1 = a.av.n[1] > 1;
            int kT1, kT2;
            level_tiling(act1, (int)sizeof(T), b.wide != 0, &kT1, &kT2);
            a.nt1 = act1 ? (int)cdiv(a.fv.n[1], kT1) : 1;
            a.nt2 = (int)cdiv(a.fv.n[2], kT2);
            const int c0 = (int)a.fv.n[0];
            a.chunk = act0 ? std::min(std::max(chunk, 2), c0) : c0;
            a.nch = act0 ? (int)cdiv(c0, a.chunk) : 1;
            const int sidx = (int)out.sargs.size();
            out.sargs.push_back(a);
            std::vector<BatchItem> s0;
            const int type = (act0 && act1) ? (b.wide ? BI_STREAM3W : BI_STREAM3) : act0 ? BI_STREAM2 : BI_STREAM1;
            for (int t = 0; t < a.nt1 * a.nt2 * a.nch; t++) s0.push_back(BatchItem{type, sidx, t, 0, f});
            stages.push_back(std::move(s0));
            // correction solves, dimensions last to first
            for (int d = 2; d >= 0; d--) {
                if (!p.active[d]) continue;
                BatchSolve<T> bs;
                std::memset(&bs, 0, sizeof(bs));
                bs.F = corr<T>(p, k, wsf);
                bs.n = ly.mc[d];
                bs.inner = 1;
                for (int e = d + 1; e < 3; e++) bs.inner *= ly.mc[e];
                bs.outer = 1;
                for (int e = 0; e < d; e++) bs.outer *= ly.mc[e];
                bs.nfib = bs.inner * bs.outer;
                bs.tb = solve_tables_of<T>(p, k, d);
                bs.Yb = ws + p.Yb;
                const int S = bs.tb.S;
                const int vidx = (int)out.solves.size();
                if (bs.inner == 1 && S <= kThreadsBatch && bs.n <= kBatchRowSpan) {
                    bs.rows = (int)std::max<int64_t>(1, std::min<int64_t>(kThreadsBatch / S, kBatchRowSpan / bs.n));
                    std::vector<BatchItem> sg;
                    for (int64_t x = 0; x < cdiv(bs.nfib, bs.rows); x++) sg.push_back(BatchItem{BI_ROWS, vidx, (int)x, 0, f});
                    stages.push_back(std::move(sg));
                } else if (bs.inner > 1 && S <= 16) {
                    std::vector<BatchItem> sg;
                    for (int64_t x = 0; x < cdiv(bs.nfib, 16); x++) sg.push_back(BatchItem{BI_STRIDED, vidx, (int)x, 0, f});
                    stages.push_back(std::move(sg));
                } else {
                    std::vector<BatchItem> s1, s2, s3;
                    if (bs.inner > 1) {
                        for (int y = 0; y < S; y++)
                            for (int64_t x = 0; x < cdiv(bs.nfib, kThreadsBatch); x++) {
                                s1.push_back(BatchItem{BI_SEG_ENDS, vidx, (int)x, y, f});
                                s3.push_back(BatchItem{BI_SEG_FINAL, vidx, (int)x, y, f});
                            }
                    } else {
                        for (int64_t x = 0; x < cdiv(bs.nfib * S, kThreadsBatch); x++) {
                            s1.push_back(BatchItem{BI_SEG_ENDS, vidx, (int)x, 0, f});
                            s3.push_back(BatchItem{BI_SEG_FINAL, vidx, (int)x, 0, f});
                        }
                    }
                    for (int64_t x = 0; x < cdiv(bs.nfib, kThreadsBatch); x++)
                        s2.push_back(BatchItem{BI_SEPARATORS, vidx, (int)x, 0, f});
                    stages.push_back(std::move(s1));
                    stages.push_back(std::move(s2));
                    stages.push_back(std::move(s3));
                }
                out.solves.push_back(bs);
            }
            if ((int)stages.size() > kStagesPerLevel) return fail(MGR_ERR_ARG, "too many stages per level step");
        }
    }
    // waves: level step, stage, field
    for (int k = 0; k < maxL; k++)
        for (int s = 0; s < kStagesPerLevel; s++) {
            const int first = (int)out.items.size();
            for (int f = 0; f < nf; f++) {
                if (k >= b.kt[(size_t)f]) continue;
                auto& stages = st[(size_t)f][(size_t)k];
                if (s >= (int)stages.size()) continue;
                out.items.insert(out.items.end(), stages[(size_t)s].begin(), stages[(size_t)s].end());
            }
            const int n = (int)out.items.size() - first;
            if (n > 0) out.waves.emplace_back(first, n);
        }
    // fields whose every level step streamed: coarsest values to their nodes
    {
        const int first = (int)out.items.size();
        for (int f = 0; f < nf; f++) {
            const Plan& p = *b.plans[(size_t)f];
            const int L = p.nlevels;
            if (b.kt[(size_t)f] < L) continue;
            void* wsf = (char*)b.ws + b.wsoff[(size_t)f];
            const View3 cl = level_view(p, L);
            BatchScatter<T> sc;
            sc.W = (const T*)wsf + p.Woff[(size_t)L];
            sc.Z = corr<T>(p, L - 1, wsf);
            for (int d = 0; d < 3; d++) {
                sc.n[d] = cl.n[d];
                sc.ds[d] = cl.s[d];
            }
            const int idx = (int)out.scatters.size();
            out.scatters.push_back(sc);
            for (int64_t x = 0; x < cdiv(cl.n[0] * cl.n[1] * cl.n[2], kThreadsBatch); x++)
                out.items.push_back(BatchItem{BI_SCATTER, idx, (int)x, 0, f});
        }
        const int n = (int)out.items.size() - first;
        if (n > 0) out.waves.emplace_back(first, n);
    }
    if (out.items.size() > (size_t)INT32_MAX) return fail(MGR_ERR_ARG, "too many work items");
    // small level steps: one tail workgroup per field that has them
    for (int f = 0; f < nf; f++) {
        const Plan& p = *b.plans[(size_t)f];
        const int kt = b.kt[(size_t)f];
        if (kt >= p.nlevels) continue;
        void* wsf = (char*)b.ws + b.wsoff[(size_t)f];
        TailArgs<T> a = tail_args<T>(p, kt, nullptr, nullptr, wsf);
        a.Z0 = (kt == 0) ? nullptr : corr<T>(p, kt - 1, wsf);
        out.tail.push_back(a);
        out.tailf.push_back(f);
    }
    return MGR_OK;
}

template <typename T>
int batch_upload(BatchPlan& b, int chunk)
{
    BatchTables<T> t;
    int rc = batch_tables<T>(b, chunk, t);
    if (rc) return rc;
    const size_t al = 256;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, al);
        return o;
    };
    b.off_items = take(sizeof(BatchItem) * t.items.size());
    b.off_sargs = take(sizeof(StreamArgs<T>) * t.sargs.size());
    b.off_solves = take(sizeof(BatchSolve<T>) * t.solves.size());
    b.off_scat = take(sizeof(BatchScatter<T>) * t.scatters.size());
    b.off_tail = take(sizeof(TailArgs<T>) * t.tail.size());
    b.off_tailf = take(sizeof(int) * t.tailf.size());
    b.off_ptrs = take(2 * sizeof(void*) * (size_t)b.nfields);
    b.off_args = take(sizeof(BatchKernelArgs<T>));
    b.nq = device_queue_count();
    batch_queues(b, t.items, t.waves, b.nq, b.qorder, b.qstart, b.qgrp, b.qdep, b.qneed);
    b.off_qorder = take(sizeof(int) * b.qorder.size());
    b.off_qgrp = take(sizeof(int) * b.qgrp.size());
    b.off_qdep = take(sizeof(int) * b.qdep.size());
    b.off_qneed = take(sizeof(int) * b.qneed.size());
    b.off_qwords = take(sizeof(int) * (kQueueWordsFixed + b.qneed.size()));
    if (b.dev) (void)hipFree(b.dev);
    b.dev = nullptr;
    hipError_t e = hipMalloc(&b.dev, off);
    if (e != hipSuccess) {
        b.dev = nullptr;
        return fail(MGR_ERR_ALLOC, std::string("hipMalloc batch tables: ") + hipGetErrorString(e));
    }
    b.dev_bytes = off;
    char* d = (char*)b.dev;
    BatchKernelArgs<T> ka;
    ka.items = (const BatchItem*)(d + b.off_items);
    ka.sargs = (const StreamArgs<T>*)(d + b.off_sargs);
    ka.solves = (const BatchSolve<T>*)(d + b.off_solves);
    ka.scatters = (const BatchScatter<T>*)(d + b.off_scat);
    ka.src = (const T* const*)(d + b.off_ptrs);
    ka.dst = (T* const*)(d + b.off_ptrs + sizeof(void*) * (size_t)b.nfields);
    struct Part {
        size_t off;
        const void* src;
        size_t bytes;
    } parts[] = {{b.off_items, t.items.data(), sizeof(BatchItem) * t.items.size()},
                 {b.off_sargs, t.sargs.data(), sizeof(StreamArgs<T>) * t.sargs.size()},
                 {b.off_solves, t.solves.data(), sizeof(BatchSolve<T>) * t.solves.size()},
                 {b.off_scat, t.scatters.data(), sizeof(BatchScatter<T>) * t.scatters.size()},
                 {b.off_tail, t.tail.data(), sizeof(TailArgs<T>) * t.tail.size()},
                 {b.off_tailf, t.tailf.data(), sizeof(int) * t.tailf.size()},
                 {b.off_args, &ka, sizeof(ka)},
                 {b.off_qorder, b.qorder.data(), sizeof(int) * b.qorder.size()},
                 {b.off_qgrp, b.qgrp.data(), sizeof(int) * b.qgrp.size()},
                 {b.off_qdep, b.qdep.data(), sizeof(int) * b.qdep.size()},
                 {b.off_qneed, b.qneed.data(), sizeof(int) * b.qneed.size()}};
    for (const Part& pt : parts) {
        if (!pt.bytes) continue;
        e = hipMemcpy(d + pt.off, pt.src, pt.bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "upload batch tables");
    }
    // the queue words start cleared (a fresh allocation may hold anything),
    // so that mgr_batch_check reads no stale state before the first
    // persistent run on these tables
    const std::vector<int> zeros(kQueueWordsFixed + b.qneed.size(), 0);
    e = hipMemcpy(d + b.off_qwords, zeros.data(), sizeof(int) * zeros.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "clear queue words");
    b.waves = t.waves;
    b.n_items = (int)t.items.size();
    b.n_tail = (int)t.tail.size();
    b.chunk = chunk;
    b.ran_persistent = 0;
    return MGR_OK;
}

void free_batch(BatchPlan* b)
{
    if (!b) return;
    if (b->dev) (void)hipFree(b->dev);
    if (b->ws) (void)hipFree(b->ws);
    for (auto& p : b->plans)
        if (p) free_plan(*p);
    delete b;
}

template <typename T>
int batch_run(BatchPlan& b, const void* const* src, void* const* dst, hipStream_t st)
{
    const int nf = b.nfields;
    char* d = (char*)b.dev;
    // the call's pointers (src then dst) travel as kernel arguments
    for (int i0 = 0; i0 < 2 * nf; i0 += kPtrChunk) {
        PtrChunk c;
        c.first = i0;
        c.n = std::min(kPtrChunk, 2 * nf - i0);
        for (int i = 0; i < c.n; i++) {
            const int j = i0 + i;
            c.p[i] = (j < nf) ? const_cast<void*>(src[j]) : dst[j - nf];
        }
        MGR_TRY(launch_set_ptrs(c, (void**)(d + b.off_ptrs), st), "batch pointer upload");
    }
    const BatchKernelArgs<T>* dev_args = (const BatchKernelArgs<T>*)(d + b.off_args);
    if (b.persistent) {
        QueueTables qt = queue_tables(b, (const int*)(d + b.off_qgrp), (const int*)(d + b.off_qdep),
                                      (const int*)(d + b.off_qneed), (const int*)(d + b.off_qorder));
        QueueState qs = queue_state((int*)(d + b.off_qwords));
        // one round of resident workgroups whatever the item count: the
        // device deals workgroups to its XCDs in turn, so every queue has
        // workgroups (those of an empty queue end at once)
        const int grid = std::max(b.nq, batch_queue_slots<T>());
        b.ran_persistent = 1;
        MGR_TRY(timed(KC_BATCH, -1, st,
                      [&] {
                          return launch_batch_queue<T>(dev_args, qt, qs, kQueueWordsFixed + (int)b.qneed.size(), grid,
                                                       b.poll_limit,
                                                       st);
                      }),
                "batch queue launch");
    } else {
        for (size_t w = 0; w < b.waves.size(); w++) {
            const int first = b.waves[w].first, n = b.waves[w].second;
            MGR_TRY(timed(KC_BATCH, (int)w, st, [&] { return launch_batch_wave<T>(dev_args, first, n, st); }),
                    "batch wave launch");
        }
    }
    MGR_TRY(timed(KC_TAIL, -1, st,
                  [&] {
                      return launch_tail_batch<T>((const TailArgs<T>*)(d + b.off_tail), (const int*)(d + b.off_tailf),
                                                  (const T* const*)(d + b.off_ptrs),
                                                  (T* const*)(d + b.off_ptrs + sizeof(void*) * (size_t)nf), b.n_tail,
                                                  true, st);
                  }),
            "batch tail launch");
    return MGR_OK;
}

int batch_create(int nfields, const int* ndim, const int64_t* const* shapes, const double* const* const* coords,
                 const int* nlevels, int dtype, BatchPlan** out)
{
    if (!out) return fail(MGR_ERR_ARG, "plan is NULL");
    *out = nullptr;
    if (nfields <= 0 || !ndim || !shapes) return fail(MGR_ERR_ARG, "nfields, ndim or shapes invalid");
    auto b = std::unique_ptr<BatchPlan, void (*)(BatchPlan*)>(new BatchPlan, free_batch);
    b->dtype = dtype;
    b->nfields = nfields;
    b->wide = (dtype == MGR_F64) ? 1 : 0;  // the per-field launches' geometry
    size_t ws_total = 0;
    const size_t esz = (dtype == MGR_F64) ? 8 : 4;
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    for (int f = 0; f < nfields; f++) {
        std::unique_ptr<Plan> pp;
        int nl = nlevels ? nlevels[f] : -1;
        const double* const* cf = coords ? coords[f] : nullptr;
        int rc = validate(dtype, ndim ? ndim[f] : 0, shapes[f], cf, &nl);
        if (rc == MGR_OK) rc = new_plan(b->device, dtype, ndim[f], shapes[f], cf, nl, false, pp);
        if (rc) return fail(rc, "field " + std::to_string(f) + ": " + g_err);
        Plan* p = pp.get();
        b->plans.push_back(std::move(pp));
        if (p->nlevels == 0) return fail(MGR_ERR_LEVELS, "field " + std::to_string(f) + ": batches need nlevels >= 1");
        const int kt = tail_start(*p);  // as the per-field path, so results agree bit for bit
        b->kt.push_back(kt);
        b->wsoff.push_back(ws_total);
        ws_total = align_up(ws_total + p->ws_bytes, 256);
        b->bytes += (int64_t)(p->n[0] * p->n[1] * p->n[2]) * (int64_t)esz;
    }
    if (ws_total > workspace_cap()) return fail(MGR_ERR_ALLOC, "batch workspace exceeds MGR_WORKSPACE_MAX");
    e = hipMalloc(&b->ws, std::max<size_t>(ws_total, 256));
    if (e != hipSuccess) {
        b->ws = nullptr;
        return fail(MGR_ERR_ALLOC, std::string("hipMalloc batch workspace: ") + hipGetErrorString(e));
    }
    int rc = (dtype == MGR_F64) ? batch_upload<double>(*b, 8) : batch_upload<float>(*b, 8);
    if (rc) return rc;
    *out = b.release();
    return MGR_OK;
}

// The transaction model of a batch configuration (the paper's
// performance-model pruning of launch shapes, Sec. III-C, applied to the
// streaming items' tile extent along dimension 0, the chunk of coarse
// planes): predicted time = a + x * bytes + y * items + z * depth, with
//   bytes: the streaming items' traffic including the 3-plane halo each item
//          re-reads (falls as the chunk grows),
//   items: the streaming items, each with its start-up and drain (falls),
//   depth: the fine planes the longest streaming item of each level step
//          streams one after the other, summed over the level steps (grows:
//          a level step ends with its longest item, however idle the rest
//          of the device is).
// The constants are not guessed: batch_autotune fits them, per launch form,
// to timed runs of the actual fields.
struct BatchTerms {
    double bytes = 0.0, items = 0.0, depth = 0.0;
};
BatchTerms batch_terms(const BatchPlan& b, int chunk)
{
    BatchTerms t;
    const double esz = (b.dtype == MGR_F64) ? 8.0 : 4.0;
    std::vector<double> longest;
    for (int f = 0; f < b.nfields; f++) {
        const Plan& p = *b.plans[(size_t)f];
        if ((int)longest.size() < b.kt[(size_t)f]) longest.resize((size_t)b.kt[(size_t)f], 0.0);
        for (int k = 0; k < b.kt[(size_t)f]; k++) {
            const LevelLayout& ly = p.lv[(size_t)k];
            const double V = (double)(ly.m[0] * ly.m[1] * ly.m[2]);
            const double c0 = (double)ly.mc[0];
            const bool act0 = ly.m[0] > 1, act1 = ly.m[1] > 1;
            int kT1, kT2;
            level_tiling(act1, (int)esz, b.wide != 0, &kT1, &kT2);
            const double tiles = (act1 ? std::ceil((double)ly.mc[1] / kT1) : 1.0) * std::ceil((double)ly.mc[2] / kT2);
            const double ch = act0 ? std::min<double>(std::max(chunk, 2), c0) : c0;
            const double nch = act0 ? std::ceil(c0 / ch) : 1.0;
            const double halo = act0 ? (2.0 * ch + 3.0) / (2.0 * ch) : 1.0;
            t.bytes += 2.0 * V * esz * halo;
            t.items += tiles * nch;
            longest[(size_t)k] = std::max(longest[(size_t)k], act0 ? 2.0 * ch + 3.0 : 1.0);
        }
    }
    for (double d : longest) t.depth += d;
    return t;
}

// Non-negative least-squares fit of time = a + x bytes + y items + z depth
// to the measured points: every subset of the four terms is fitted without
// constraints (normal equations, Gaussian elimination) and the best fit
// whose coefficients are all non-negative is kept (a negative constant has
// no physical reading; with as many probes as terms an unconstrained fit
// would interpolate the noise).
constexpr int kModelTerms = 4;
void fit_model(const std::vector<BatchTerms>& t, const std::vector<double>& ms, double m[kModelTerms])
{
    const double scale[kModelTerms] = {1.0, 1e-9, 1e-3, 1e-2};  // conditioning
    auto term = [&](size_t i, int c) {
        const double v[kModelTerms] = {1.0, t[i].bytes, t[i].items, t[i].depth};
        return v[c] * scale[c];
    };
    double best_res = 1e300, best[kModelTerms] = {0, 0, 0, 0};
    for (int mask = 1; mask < (1 << kModelTerms); mask++) {
        int idx[kModelTerms], n = 0;
        for (int c = 0; c < kModelTerms; c++)
            if (mask & (1 << c)) idx[n++] = c;
        if ((size_t)n > t.size()) continue;
        double S[kModelTerms][kModelTerms + 1] = {{0}};
        for (size_t i = 0; i < t.size(); i++)
            for (int a = 0; a < n; a++) {
                for (int c = 0; c < n; c++) S[a][c] += term(i, idx[a]) * term(i, idx[c]);
                S[a][n] += term(i, idx[a]) * ms[i];
            }
        bool ok = true;
        for (int c = 0; c < n && ok; c++) {  // elimination with partial pivoting
            int piv = c;
            for (int r = c + 1; r < n; r++)
                if (std::fabs(S[r][c]) > std::fabs(S[piv][c])) piv = r;
            if (std::fabs(S[piv][c]) < 1e-12) {
                ok = false;
                break;
            }
            for (int j = 0; j <= n; j++) std::swap(S[c][j], S[piv][j]);
            for (int r = 0; r < n; r++) {
                if (r == c) continue;
                const double f = S[r][c] / S[c][c];
                for (int j = c; j <= n; j++) S[r][j] -= f * S[c][j];
            }
        }
        if (!ok) continue;
        double sol[kModelTerms] = {0, 0, 0, 0};
        for (int a = 0; a < n; a++) {
            sol[idx[a]] = S[a][n] / S[a][a];
            if (sol[idx[a]] < 0.0) ok = false;
        }
        if (!ok) continue;
        double res = 0.0;
        for (size_t i = 0; i < t.size(); i++) {
            double p = 0.0;
            for (int c = 0; c < kModelTerms; c++) p += sol[c] * term(i, c);
            res += (p - ms[i]) * (p - ms[i]);
        }
        if (res < best_res) {
            best_res = res;
            std::copy(sol, sol + kModelTerms, best);
        }
    }
    for (int c = 0; c < kModelTerms; c++) m[c] = best[c] * scale[c];
}

double model_ms(const double m[kModelTerms], const BatchTerms& t)
{
    return m[0] + m[1] * t.bytes + m[2] * t.items + m[3] * t.depth;
}

// ---- class-packed layout and progressive recomposition --------------------
// Segment starts of the class-packed layout: class 0 is the level-0 grid,
// class c the level-c grid minus the level-(c-1) grid (paper levels, L
// finest); level grid c has stride 2^(L - c).
void class_offsets_of(int ndim, const int64_t* shape, int L, int64_t* off)
{
    auto grid = [&](int c) {
        int64_t v = 1;
        for (int d = 0; d < ndim; d++) v *= ((shape[d] - 1) >> (L - c)) + 1;
        return v;
    };
    off[0] = 0;
    off[1] = grid(0);
    for (int c = 1; c <= L; c++) off[c + 1] = off[c] + grid(c) - grid(c - 1);
}

PackArgs pack_args(int ndim, const int64_t* shape, int L)
{
    Plan p;
    plan_dims(p, 0, MGR_F32, ndim, shape, L);
    PackArgs a;
    std::memset(&a, 0, sizeof(a));
    for (int d = 0; d < 3; d++) a.n[d] = p.n[d];
    a.L = L;
    class_offsets_of(ndim, shape, L, a.off);
    return a;
}

int run_pack(bool pack, const void* src, void* dst, int dtype, int ndim, const int64_t* shape, int nlevels,
             void* stream)
{
    if (!src || !dst) return fail(MGR_ERR_ARG, "src or dst is NULL");
    if (src == dst) return fail(MGR_ERR_ARG, "the class-packed layout is formed out of place");
    int rc = validate(dtype, ndim, shape, nullptr, &nlevels);
    if (rc) return rc;
    if (nlevels > kMaxClassLevels) return fail(MGR_ERR_LEVELS, "too many levels for the class-packed layout");
    const PackArgs a = pack_args(ndim, shape, nlevels);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = (dtype == MGR_F32) ? launch_pack<float>((const float*)src, (float*)dst, a, pack, st)
                                      : launch_pack<double>((const double*)src, (double*)dst, a, pack, st);
    return e == hipSuccess ? MGR_OK : hip_fail(e, "pack launch");
}

// Quantisation of the classes (in-place or class-packed layout): validated
// like a refactored array of the problem, bins = one positive finite width
// per class.
int run_quant(bool quant, const void* y, int32_t* q, void* out, int dtype, int ndim, const int64_t* shape,
              int nlevels, int packed, const double* bins, unsigned long long* nclamped, void* stream)
{
    if (!q || (quant ? !y : !out)) return fail(MGR_ERR_ARG, "data or code pointer is NULL");
    if (!bins) return fail(MGR_ERR_ARG, "bins is NULL");
    if (packed != 0 && packed != 1) return fail(MGR_ERR_ARG, "packed must be 0 or 1");
    int rc = validate(dtype, ndim, shape, nullptr, &nlevels);
    if (rc) return rc;
    if (nlevels > kMaxClassLevels) return fail(MGR_ERR_LEVELS, "too many levels for the class tables");
    QuantArgs a;
    std::memset(&a, 0, sizeof(a));
    const PackArgs pa = pack_args(ndim, shape, nlevels);
    for (int d = 0; d < 3; d++) a.n[d] = pa.n[d];
    a.L = nlevels;
    a.packed = packed;
    std::memcpy(a.off, pa.off, sizeof(a.off));
    for (int c = 0; c <= nlevels; c++) {
        if (!(bins[c] > 0.0) || !std::isfinite(bins[c]))
            return fail(MGR_ERR_ARG, "bin width of class " + std::to_string(c) + " is not positive and finite");
        a.bins[c] = bins[c];
    }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = (dtype == MGR_F32)
                       ? launch_quant<float>((const float*)y, (int*)q, (float*)out, a, quant, nclamped, st)
                       : launch_quant<double>((const double*)y, (int*)q, (double*)out, a, quant, nclamped, st);
    return e == hipSuccess ? MGR_OK : hip_fail(e, "quantisation launch");
}

// Bin widths for a bound tol on the largest pointwise error of the
// recomposed field.  The class-0 values enter the recomposition only through
// interpolation, whose weights are nonnegative and sum to one, so an error e
// there moves the result by at most max|e|.  A class-l error (l >= 1) enters
// as its level-l interpolant minus the correction's projection of it onto the
// coarser space (Eq. (1)), then is interpolated again: at most
// (1 + |Q|) max|e|, with |Q| the max-norm of the nodal L2 projection onto
// piecewise-multilinear functions, a tensor product of one-dimensional
// projections each bounded by 3 on any mesh, so |Q| <= 3^ndim.  Errors of
// half a bin per class, tol split evenly over the L + 1 classes.
int quant_bins(int ndim, int nlevels, double tol, double* bins)
{
    if (!bins) return fail(MGR_ERR_ARG, "bins is NULL");
    if (ndim < 1 || ndim > kMaxDim) return fail(MGR_ERR_ARG, "ndim must be 1..3");
    if (nlevels < 0 || nlevels > kMaxClassLevels) return fail(MGR_ERR_LEVELS, "nlevels out of range");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(MGR_ERR_ARG, "tol must be positive and finite");
    double g = 1.0;  // 3^ndim
    for (int d = 0; d < ndim; d++) g *= 3.0;
    for (int c = 0; c <= nlevels; c++) bins[c] = 2.0 * tol / ((double)(nlevels + 1) * (c == 0 ? 1.0 : 1.0 + g));
    return MGR_OK;
}

// Recomposition from the classes 0..level: the level grid `level` (stride
// s = 2^(L - level)) with its classes is the refactored array of the same
// method on that grid (shape (n - 1) / s + 1, coordinates x[::s], `level`
// level steps: the decomposition's coarser steps only ever see it), so it is
// gathered into the sub-problem's spare buffer (from the strided in-place
// array, or by unpacking the class-packed prefix, which is the sub-problem's
// own class-packed layout) and recomposed by the sub-problem's plan.
template <typename T>
int run_recompose_level(const void* src_, void* dst_, int ndim, const int64_t* shape, const double* const* coords,
                        int L, int level, bool packed, hipStream_t st)
{
    const T* src = (const T*)src_;
    T* dst = (T*)dst_;
    const int sh = L - level;
    int64_t sub[3] = {1, 1, 1};
    for (int d = 0; d < ndim; d++) sub[d] = ((shape[d] - 1) >> sh) + 1;
    Plan full;
    plan_dims(full, 0, sizeof(T) == 8 ? MGR_F64 : MGR_F32, ndim, shape, L);
    View3 sv;  // the level grid inside the in-place array
    for (int d = 0; d < 3; d++) {
        sv.n[d] = full.active[d] ? ((full.n[d] - 1) >> sh) + 1 : 1;
        sv.s[d] = full.st[d] << sh;
    }
    if (level == 0) {
        // the coarsest values: the strided grid, or the first segment
        if (packed) {
            const size_t bytes = (size_t)(sv.n[0] * sv.n[1] * sv.n[2]) * sizeof(T);
            MGR_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st), "copy");
        } else {
            MGR_TRY(launch_copy_view<T>(src, nullptr, sv, dst, packed_view3(sv.n), st), "gather");
        }
        return MGR_OK;
    }
    std::vector<std::vector<double>> cs;
    std::vector<const double*> cp;
    if (coords) {
        cs.resize((size_t)ndim);
        for (int d = 0; d < ndim; d++) {
            if (!coords[d]) {
                cp.push_back(nullptr);
                continue;
            }
            for (int64_t i = 0; i < sub[d]; i++) cs[(size_t)d].push_back(coords[d][i << sh]);
            cp.push_back(cs[(size_t)d].data());
        }
    }
    Plan* ps = nullptr;
    int rc = get_plan(sizeof(T) == 8 ? MGR_F64 : MGR_F32, ndim, sub, coords ? cp.data() : nullptr, level, st, true,
                      &ps);
    if (rc) return rc;
    T* tmp = (T*)ps->ws + ps->Tb;  // the adjoint's buffer: unused by recomposition
    if (packed) {
        const PackArgs a = pack_args(ndim, sub, level);
        MGR_TRY(launch_pack<T>(src, tmp, a, false, st), "unpack launch");
    } else {
        MGR_TRY(launch_copy_view<T>(src, nullptr, sv, tmp, packed_view3(sv.n), st), "gather");
    }
    return run_recompose<T>(*ps, tmp, dst, st);
}

// ---- allocation-free decomposition ------------------------------------------
// For callers that cannot allocate device memory: the tables and the
// decomposition's workspace of the problem live in one file-scope device
// array instead of the per-problem cache.  Each device holds its own copy of
// the array, at its own address, found once per device with
// hipGetSymbolAddress; host code only ever uses that address (the array's
// name in host code is a host-side stand-in).  Every call on a device shares
// its array: calls that overlap on one device race.
constexpr size_t kScratchBytes = (size_t)MGR_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchDev {
    void* ptr = nullptr;      // device address of `scratch` on this device
    std::string tables_key;   // problem whose tables the array holds now
};
std::mutex g_scratch_mu;
ScratchDev g_scratch[64];
// host halves of the allocation-free plans (layouts and host tables, no
// device memory), per problem
struct NoAllocPlan {
    Plan p;
    std::vector<unsigned char> host_tables;
};
std::map<std::string, std::unique_ptr<NoAllocPlan>> g_noalloc_plans;

template <typename T>
void noalloc_layout(NoAllocPlan& q, const double* const* coords)
{
    std::vector<T> host;
    plan_layout<T>(q.p, coords, true, host);
    q.host_tables.resize(host.size() * sizeof(T));
    if (!host.empty()) std::memcpy(q.host_tables.data(), host.data(), q.host_tables.size());
}

int run_decompose_noalloc(const void* src, void* dst, int dtype, int ndim, const int64_t* shape,
                          const double* const* coords, int nlevels, void* stream)
{
    g_err.clear();
    if (!src || !dst) return fail(MGR_ERR_ARG, "src or dst is NULL");
    int rc = validate(dtype, ndim, shape, coords, &nlevels);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(MGR_ERR_ARG, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ScratchDev& sd = g_scratch[dev];
    if (!sd.ptr) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(MGR_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        sd.ptr = ptr;
    }
    const std::string key = plan_key(dev, dtype, ndim, shape, coords, nlevels);
    auto it = g_noalloc_plans.find(key);
    if (it == g_noalloc_plans.end()) {
        auto q = std::make_unique<NoAllocPlan>();
        plan_dims(q->p, dev, dtype, ndim, shape, nlevels);
        if (dtype == MGR_F32)
            noalloc_layout<float>(*q, coords);
        else
            noalloc_layout<double>(*q, coords);
        it = g_noalloc_plans.emplace(key, std::move(q)).first;
    }
    Plan& p = it->second->p;
    const size_t tab = align_up(p.tables_bytes, 256);
    if (tab + p.ws_bytes > kScratchBytes)
        return fail(MGR_ERR_ALLOC, "problem needs " + std::to_string(tab + p.ws_bytes) +
                                       " bytes of tables and workspace; the allocation-free scratch holds " +
                                       std::to_string(kScratchBytes));
    p.tables = sd.ptr;
    p.ws = (unsigned char*)sd.ptr + tab;
    if (sd.tables_key != key) {
        // in stream order before the kernels that read them; the host copy
        // stays alive in the plan
        if (p.tables_bytes) {
            e = hipMemcpyAsync(p.tables, it->second->host_tables.data(), p.tables_bytes, hipMemcpyHostToDevice, st);
            if (e != hipSuccess) {
                sd.tables_key.clear();
                return hip_fail(e, "upload tables to the scratch array");
            }
        }
        sd.tables_key = key;
    }
    return dtype == MGR_F32 ? run_decompose<float>(p, src, dst, st) : run_decompose<double>(p, src, dst, st);
}

// The work items, waves and queue groups of a batch, built on the host
// alone (no device memory: plans keep only their layouts and the pointers in
// the item arguments are never used), for the host check of the queue.
template <typename T>
int batch_host_items_t(int nfields, const int* ndim, const int64_t* const* shapes, const int* nlevels, int chunk,
                       int nq, BatchPlan& b)
{
    char* const base = reinterpret_cast<char*>((uintptr_t)1 << 40);  // stands in for device allocations
    size_t ws_total = 0;
    for (int f = 0; f < nfields; f++) {
        int nl = nlevels ? nlevels[f] : -1;
        int rc = validate(b.dtype, ndim[f], shapes[f], nullptr, &nl);
        if (rc) return fail(rc, "field " + std::to_string(f) + ": " + g_err);
        if (nl == 0) return fail(MGR_ERR_LEVELS, "field " + std::to_string(f) + ": batches need nlevels >= 1");
        auto p = std::make_unique<Plan>();
        plan_dims(*p, 0, b.dtype, ndim[f], shapes[f], nl);
        std::vector<T> host;
        plan_layout<T>(*p, nullptr, false, host);
        p->tables = base;
        b.kt.push_back(tail_start(*p));
        b.wsoff.push_back(ws_total);
        ws_total = align_up(ws_total + p->ws_bytes, 256);
        b.plans.push_back(std::move(p));
    }
    b.ws = base;
    BatchTables<T> t;
    int rc = batch_tables<T>(b, chunk, t);
    b.ws = nullptr;
    for (auto& p : b.plans) p->tables = nullptr;
    if (rc) return rc;
    b.nq = nq;
    batch_queues(b, t.items, t.waves, nq, b.qorder, b.qstart, b.qgrp, b.qdep, b.qneed);
    b.waves = t.waves;
    b.n_items = (int)t.items.size();
    return MGR_OK;
}

int batch_host_items(int nfields, const int* ndim, const int64_t* const* shapes, const int* nlevels, int dtype,
                     int chunk, int nq, BatchPlan& b)
{
    if (nfields <= 0 || !ndim || !shapes) return fail(MGR_ERR_ARG, "nfields, ndim or shapes invalid");
    if (nq < 1 || nq > kMaxQueues) return fail(MGR_ERR_ARG, "nqueues must be 1.." + std::to_string(kMaxQueues));
    if (dtype != MGR_F32 && dtype != MGR_F64) return fail(MGR_ERR_ARG, "dtype must be MGR_F32 or MGR_F64");
    if (chunk < 1 || chunk > kMaxBatchChunk) return fail(MGR_ERR_ARG, "chunk must be 1.." + std::to_string(kMaxBatchChunk));
    b.dtype = dtype;
    b.nfields = nfields;
    b.wide = (dtype == MGR_F64) ? 1 : 0;  // as a new plan starts
    return dtype == MGR_F64 ? batch_host_items_t<double>(nfields, ndim, shapes, nlevels, chunk, nq, b)
                            : batch_host_items_t<float>(nfields, ndim, shapes, nlevels, chunk, nq, b);
}

// Host side of the queue protocol (mgr_queue.h) for mgr_batch_queue_check.
struct HostQueueOps {
    int load_relaxed(int* p) const { return __atomic_load_n(p, __ATOMIC_RELAXED); }
    void fence_acquire() const { __atomic_thread_fence(__ATOMIC_ACQUIRE); }
    int fetch_add_relaxed(int* p, int v) const { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
    void add_release(int* p, int v) const { (void)__atomic_fetch_add(p, v, __ATOMIC_RELEASE); }
    void store_relaxed(int* p, int v) const { __atomic_store_n(p, v, __ATOMIC_RELAXED); }
    void cas_relaxed(int* p, int expect, int v) const
    {
        (void)__atomic_compare_exchange_n(p, &expect, v, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED);
    }
    void pause() const { std::this_thread::yield(); }
};

// Runs the queue protocol of a plan's item list on nthreads host threads
// standing in for workgroups (thread t serves queue t mod nq, as the
// workgroups of a launch are dealt to every XCD); each "runs" an item by
// checking that its dependency group has finished (a separate sequentially
// consistent count kept outside the protocol), spinning for a random while,
// and counting it.  The thread that takes position stall (>= 0) stops there
// without finishing it, as a workgroup that never completes would.  out:
// items run, items that started before their dependency group finished, the
// error word (1 + the position whose wait timed out, or 0), positions left
// untaken.
int queue_check(const BatchPlan& b, int nthreads, unsigned limit, int stall_item, uint64_t seed, int64_t* out)
{
    if (nthreads < 1 || nthreads > 1024) return fail(MGR_ERR_ARG, "nthreads must be 1..1024");
    const int ng = (int)b.qneed.size();
    std::vector<int> words((size_t)(kQueueWordsFixed + ng), 0), fin((size_t)ng, 0);
    const QueueTables qt = queue_tables(b, b.qgrp.data(), b.qdep.data(), b.qneed.data(), b.qorder.data());
    const QueueState qs = queue_state(words.data());
    std::atomic<int64_t> ran{0}, bad{0};
    auto worker = [&](int tid) {
        uint64_t x = seed * 0x9E3779B97F4A7C15ull + (uint64_t)tid + 1;
        const int q = tid % b.nq;
        int last_dg = -1;
        for (;;) {
            const int i = queue_take(qt, qs, q, limit, last_dg, HostQueueOps{});
            if (i < 0) return;
            const int g = b.qgrp[(size_t)i], dg = b.qdep[(size_t)g];
            if (dg >= 0 && __atomic_load_n(&fin[(size_t)dg], __ATOMIC_SEQ_CST) != b.qneed[(size_t)dg]) bad++;
            if (i == stall_item) return;
            x ^= x << 13;
            x ^= x >> 7;
            x ^= x << 17;
            for (volatile unsigned spin = 0; spin < (unsigned)(x % 2000); spin = spin + 1) {
            }
            (void)__atomic_fetch_add(&fin[(size_t)g], 1, __ATOMIC_SEQ_CST);
            ran++;
            queue_finish(qt, qs, i, HostQueueOps{});
        }
    };
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; t++) th.emplace_back(worker, t);
    for (auto& t : th) t.join();
    int64_t untaken = 0;
    for (int q = 0; q < b.nq; q++)
        untaken += std::max<int64_t>(0, (int64_t)(b.qstart[(size_t)q + 1] - b.qstart[(size_t)q]) - qs.next[q]);
    out[0] = ran.load();
    out[1] = bad.load();
    out[2] = *qs.err;
    out[3] = untaken;
    return MGR_OK;
}

}  // namespace


}  // namespace mgr

using namespace mgr;

extern "C" {

int mgr_max_levels(int ndim, const int64_t* shape)
{
    int nl = -1;
    int rc = validate_general(MGR_F32, ndim, shape, nullptr, &nl);
    return rc ? -rc : nl;
}

int mgr_decompose(const void* src, void* dst, int dtype, int ndim, const int64_t* shape,
                  const double* const* coords, int nlevels, void* stream)
{
    try {
        return run(DIR_DEC, src, dst, dtype, ndim, shape, coords, nlevels, stream);
    } catch (const std::bad_alloc&) {
        return fail(MGR_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_decompose_noalloc(const void* src, void* dst, int dtype, int ndim, const int64_t* shape,
                          const double* const* coords, int nlevels, void* stream)
{
    try {
        return run_decompose_noalloc(src, dst, dtype, ndim, shape, coords, nlevels, stream);
    } catch (const std::bad_alloc&) {
        return fail(MGR_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_recompose(const void* src, void* dst, int dtype, int ndim, const int64_t* shape,
                  const double* const* coords, int nlevels, void* stream)
{
    try {
        return run(DIR_REC, src, dst, dtype, ndim, shape, coords, nlevels, stream);
    } catch (const std::bad_alloc&) {
        return fail(MGR_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_decompose_adjoint(const void* src, void* dst, int dtype, int ndim, const int64_t* shape,
                          const double* const* coords, int nlevels, void* stream)
{
    try {
        return run(DIR_ADJ, src, dst, dtype, ndim, shape, coords, nlevels, stream);
    } catch (const std::bad_alloc&) {
        return fail(MGR_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_recompose_adjoint(const void* src, void* dst, int dtype, int ndim, const int64_t* shape,
                          const double* const* coords, int nlevels, void* stream)
{
    try {
        return run(DIR_RADJ, src, dst, dtype, ndim, shape, coords, nlevels, stream);
    } catch (const std::bad_alloc&) {
        return fail(MGR_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_prepare(int dtype, int ndim, const int64_t* shape, const double* const* coords,
                int nlevels)
{
    try {
        g_err.clear();
        if (shape && !dyadic_shape(ndim, shape)) {
            int rc = validate_general(dtype, ndim, shape, coords, &nlevels);
            if (rc) return rc;
            GenPlan* gp = nullptr;
            return get_gen_plan(dtype, ndim, shape, coords, nlevels, nullptr, false, &gp);
        }
        Plan* p = nullptr;
        int rc = get_plan(dtype, ndim, shape, coords, nlevels, nullptr, false, &p);
        if (rc) return rc;
        // the recomposition's auxiliary streams, so that no stream is created
        // while a stream is being captured
        std::lock_guard<std::mutex> lk(g_aux_mu);
        AuxStream* aux = nullptr;
        hipError_t e = aux_stream(&aux);
        if (e != hipSuccess) return hip_fail(e, "auxiliary stream");
        return MGR_OK;
    } catch (const std::bad_alloc&) {
        return fail(MGR_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_class_offsets(int ndim, const int64_t* shape, int nlevels, int64_t* offsets)
{
    g_err.clear();
    if (!offsets) return fail(MGR_ERR_ARG, "offsets is NULL");
    int rc = validate(MGR_F32, ndim, shape, nullptr, &nlevels);
    if (rc) return rc;
    class_offsets_of(ndim, shape, nlevels, offsets);
    return MGR_OK;
}

int mgr_quant_bins(int ndim, int nlevels, double tol, double* bins)
{
    g_err.clear();
    return quant_bins(ndim, nlevels, tol, bins);
}

int mgr_quantize(const void* src, int32_t* codes, int dtype, int ndim, const int64_t* shape, int nlevels,
                 int packed, const double* bins, unsigned long long* nclamped, void* stream)
{
    try {
        g_err.clear();
        return run_quant(true, src, codes, nullptr, dtype, ndim, shape, nlevels, packed, bins, nclamped, stream);
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_dequantize(const int32_t* codes, void* dst, int dtype, int ndim, const int64_t* shape, int nlevels,
                   int packed, const double* bins, void* stream)
{
    try {
        g_err.clear();
        return run_quant(false, nullptr, const_cast<int32_t*>(codes), dst, dtype, ndim, shape, nlevels, packed, bins,
                         nullptr, stream);
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_pack_classes(const void* src, void* dst, int dtype, int ndim, const int64_t* shape, int nlevels,
                     void* stream)
{
    try {
        g_err.clear();
        return run_pack(true, src, dst, dtype, ndim, shape, nlevels, stream);
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_unpack_classes(const void* src, void* dst, int dtype, int ndim, const int64_t* shape, int nlevels,
                       void* stream)
{
    try {
        g_err.clear();
        return run_pack(false, src, dst, dtype, ndim, shape, nlevels, stream);
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_recompose_level(const void* src, void* dst, int dtype, int ndim, const int64_t* shape,
                        const double* const* coords, int nlevels, int level, int packed, void* stream)
{
    try {
        g_err.clear();
        if (!src || !dst) return fail(MGR_ERR_ARG, "src or dst is NULL");
        if (src == dst) return fail(MGR_ERR_ARG, "progressive recomposition is out of place");
        int rc = validate(dtype, ndim, shape, coords, &nlevels);
        if (rc) return rc;
        if (level < 0 || level > nlevels)
            return fail(MGR_ERR_LEVELS, "level = " + std::to_string(level) + " outside 0.." + std::to_string(nlevels));
        if (packed != 0 && packed != 1) return fail(MGR_ERR_ARG, "packed must be 0 or 1");
        hipStream_t st = (hipStream_t)stream;
        return (dtype == MGR_F32)
                   ? run_recompose_level<float>(src, dst, ndim, shape, coords, nlevels, level, packed != 0, st)
                   : run_recompose_level<double>(src, dst, ndim, shape, coords, nlevels, level, packed != 0, st);
    } catch (const std::bad_alloc&) {
        return fail(MGR_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_class_map(int ndim, const int64_t* shape, int nlevels, uint8_t* out)
{
    g_err.clear();
    if (!out) return fail(MGR_ERR_ARG, "out is NULL");
    int rc = validate_general(MGR_F32, ndim, shape, nullptr, &nlevels);
    if (rc) return rc;
    if (!dyadic_shape(ndim, shape)) {
        // a node is on level grid k along d when its index is a multiple of
        // 2^k or the last one; its class is L - (the finest k <= L whose grid
        // holds it in every dimension), 0 on the coarsest grid
        const int L = nlevels;
        std::vector<std::vector<uint8_t>> lev((size_t)ndim);
        for (int d = 0; d < ndim; d++) {
            lev[(size_t)d].resize((size_t)shape[d]);
            for (int64_t i = 0; i < shape[d]; i++) {
                int k = 0;
                while (k < L && (((i >> (k + 1)) << (k + 1)) == i || i == shape[d] - 1)) k++;
                lev[(size_t)d][(size_t)i] = (uint8_t)k;
            }
        }
        int64_t N = 1;
        for (int d = 0; d < ndim; d++) N *= shape[d];
        for (int64_t idx = 0; idx < N; idx++) {
            int64_t r = idx;
            int k = L;
            for (int d = ndim - 1; d >= 0; d--) {
                k = std::min(k, (int)lev[(size_t)d][(size_t)(r % shape[d])]);
                r /= shape[d];
            }
            out[idx] = (uint8_t)(L - k);
        }
        return MGR_OK;
    }
    int64_t n[3] = {1, 1, 1};
    for (int d = 0; d < ndim; d++) n[3 - ndim + d] = shape[d];
    const int L = nlevels;
    auto v2 = [L](int64_t i) {
        if (i == 0) return L;
        int v = 0;
        while (((i >> v) & 1) == 0 && v < L) v++;
        return v;
    };
    size_t idx = 0;
    for (int64_t a = 0; a < n[0]; a++)
        for (int64_t b = 0; b < n[1]; b++) {
            int vab = std::min(v2(a), v2(b));
            for (int64_t c = 0; c < n[2]; c++) {
                int v = std::min(vab, v2(c));
                out[idx++] = (uint8_t)(v >= L ? 0 : L - v);
            }
        }
    return MGR_OK;
}

const char* mgr_status_string(int status)
{
    switch (status) {
        case MGR_OK: return "ok";
        case MGR_ERR_ARG: return "invalid argument";
        case MGR_ERR_SHAPE: return "invalid shape (sizes must be 2^k+1, k>=1)";
        case MGR_ERR_LEVELS: return "invalid level count";
        case MGR_ERR_COORDS: return "invalid coordinates";
        case MGR_ERR_HIP: return "HIP runtime error";
        case MGR_ERR_ALLOC: return "allocation failed";
        case MGR_ERR_CAPTURE: return "allocation needed during stream capture";
        default: return "unknown status";
    }
}

const char* mgr_last_error(void) { return g_err.c_str(); }

void mgr_finalize(void)
{
    // one lock at a time: a recomposition holds the stream lock while its
    // timed launches take the timing lock
    {
        std::lock_guard<std::mutex> lk(g_aux_mu);
        for (AuxStream& a : g_aux) destroy_aux(a);
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (auto& kv : g_plans) free_plan(*kv.second);
        g_plans.clear();
        for (auto& kv : g_gen_plans) free_gen_plan(*kv.second);
        g_gen_plans.clear();
    }
    {
        // the allocation-free plans are host memory only; the scratch array
        // itself stays with the device
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        g_noalloc_plans.clear();
        for (ScratchDev& sd : g_scratch) sd.tables_key.clear();
    }
    std::lock_guard<std::mutex> lk(g_tm_mu);
    for (auto& e : g_tm.ev) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    g_tm.ev.clear();
    g_tm.on = false;
}

int64_t mgr_set_tail_max_nodes(int64_t max_nodes)
{
    if (max_nodes < 0) max_nodes = 0;
    return g_tail_nodes.exchange(max_nodes);
}

int mgr_bench_copy(const void* src, void* dst, size_t nbytes, void* stream)
{
    g_err.clear();
    if (!src || !dst) return fail(MGR_ERR_ARG, "src or dst is NULL");
    if (nbytes % 16 || ((uintptr_t)src % 16) || ((uintptr_t)dst % 16))
        return fail(MGR_ERR_ARG, "nbytes and pointers must be multiples of 16");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = timed(KC_BENCH_COPY, 0, st, [&] { return launch_bench_copy(src, dst, nbytes, st); });
    return e == hipSuccess ? MGR_OK : hip_fail(e, "copy launch");
}

int mgr_timing_enable(int kernel, int level)
{
    if (kernel < 0 || kernel >= KC_COUNT) return fail(MGR_ERR_ARG, "unknown kernel class");
    std::lock_guard<std::mutex> lk(g_tm_mu);
    g_tm.on = true;
    g_tm.kc = kernel;
    g_tm.level = level;
    return MGR_OK;
}

int mgr_timing_disable(void)
{
    std::lock_guard<std::mutex> lk(g_tm_mu);
    g_tm.on = false;
    return MGR_OK;
}

int mgr_timing_read(double* total_ms, int64_t* launches)
{
    if (!total_ms || !launches) return fail(MGR_ERR_ARG, "NULL output");
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    {
        std::lock_guard<std::mutex> lk(g_tm_mu);
        ev.swap(g_tm.ev);
    }
    double sum = 0.0;
    int rc = MGR_OK;
    for (auto& e : ev) {
        float ms = 0.f;
        hipError_t r = hipEventSynchronize(e.second);
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, e.first, e.second);
        if (r != hipSuccess && rc == MGR_OK) rc = hip_fail(r, "timing events");
        sum += ms;
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    *total_ms = sum;
    *launches = (int64_t)ev.size();
    return rc;
}

const char* mgr_kernel_name(int kernel)
{
    if (kernel < 0 || kernel >= KC_COUNT) return nullptr;
    return kKernelNames[kernel];
}

int mgr_batch_plan_create(int nfields, const int* ndim, const int64_t* const* shapes,
                          const double* const* const* coords, const int* nlevels, int dtype, mgr_batch_plan** plan)
{
    try {
        g_err.clear();
        if (dtype != MGR_F32 && dtype != MGR_F64) return fail(MGR_ERR_ARG, "dtype must be MGR_F32 or MGR_F64");
        BatchPlan* b = nullptr;
        int rc = batch_create(nfields, ndim, shapes, coords, nlevels, dtype, &b);
        if (plan) *plan = reinterpret_cast<mgr_batch_plan*>(b);
        return rc;
    } catch (const std::bad_alloc&) {
        return fail(MGR_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_batch_decompose(mgr_batch_plan* plan, const void* const* src, void* const* dst, void* stream)
{
    try {
        g_err.clear();
        BatchPlan* b = reinterpret_cast<BatchPlan*>(plan);
        if (!b || !src || !dst) return fail(MGR_ERR_ARG, "plan, src or dst is NULL");
        for (int f = 0; f < b->nfields; f++) {
            if (!src[f] || !dst[f]) return fail(MGR_ERR_ARG, "NULL data pointer for field " + std::to_string(f));
            if (src[f] == dst[f]) return fail(MGR_ERR_ARG, "batched decomposition is out of place (field " +
                                                               std::to_string(f) + ")");
        }
        hipStream_t st = (hipStream_t)stream;
        return b->dtype == MGR_F64 ? batch_run<double>(*b, src, dst, st) : batch_run<float>(*b, src, dst, st);
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_batch_autotune(mgr_batch_plan* plan, const void* const* src, void* const* dst, void* stream, int top_k)
{
    try {
        g_err.clear();
        BatchPlan* b = reinterpret_cast<BatchPlan*>(plan);
        if (!b || !src || !dst) return fail(MGR_ERR_ARG, "plan, src or dst is NULL");
        hipStream_t st = (hipStream_t)stream;
        if (capturing(st)) return fail(MGR_ERR_CAPTURE, "autotuning times launches; not during capture");
        if (top_k < 1) top_k = 3;
        const int cand[] = {2, 4, 8, 16, 32, 64, 128};
        const int probes[] = {2, 4, 16, 64, 128};
        hipEvent_t e0, e1;
        MGR_TRY(hipEventCreate(&e0), "event");
        MGR_TRY(hipEventCreate(&e1), "event");
        int rc = MGR_OK;
        // median of 3 timed calls after a warm-up, at chunk c
        auto time_chunk = [&](int c, double* out_ms) -> int {
            int r = b->dtype == MGR_F64 ? batch_upload<double>(*b, c) : batch_upload<float>(*b, c);
            if (r) return r;
            std::vector<float> ms;
            for (int i = 0; i < 4 && r == MGR_OK; i++) {
                (void)hipEventRecord(e0, st);
                r = mgr_batch_decompose(plan, src, dst, stream);
                (void)hipEventRecord(e1, st);
                float t = 0.f;
                if (r == MGR_OK && hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&t, e0, e1) == hipSuccess)
                    ms.push_back(t);
            }
            if (r) return r;
            if (ms.size() < 2) return fail(MGR_ERR_HIP, "autotune timing failed");
            std::sort(ms.begin() + 1, ms.end());  // the first run is a warm-up
            *out_ms = ms[1 + (ms.size() - 1) / 2];
            return MGR_OK;
        };
        double best = 1e300;
        int best_chunk = b->chunk, best_mode = b->persistent, best_wide = b->wide;
        double models[2][2][kModelTerms] = {};  // per tile geometry and launch form
        const unsigned limit = b->poll_limit;
        // both tile geometries where a field is 3-D (the others do not
        // depend on it), and both launch forms (waves, persistent), each with
        // its own model
        bool any3d = false;
        for (const auto& pl : b->plans) any3d = any3d || (pl->active[0] && pl->active[1]);
        const int w0 = any3d ? 0 : b->wide, w1 = any3d ? 1 : b->wide;
        for (int wide = w0; wide <= w1 && rc == MGR_OK; wide++) {
            b->wide = wide;
            for (int mode = 0; mode <= 1 && rc == MGR_OK; mode++) {
                b->persistent = mode;
                b->poll_limit = limit;
                // fit the model to the probe configurations, rank every
                // candidate by it, then time the best top_k
                std::vector<BatchTerms> terms;
                std::vector<double> meas;
                std::map<int, double> timed_ms;
                for (int c : probes) {
                    double ms = 0.0;
                    rc = time_chunk(c, &ms);
                    if (rc) break;
                    terms.push_back(batch_terms(*b, c));
                    meas.push_back(ms);
                    timed_ms[c] = ms;
                }
                if (rc) break;
                fit_model(terms, meas, models[wide][mode]);
                std::vector<std::pair<double, int>> ranked;
                for (int c : cand) ranked.emplace_back(model_ms(models[wide][mode], batch_terms(*b, c)), c);
                std::sort(ranked.begin(), ranked.end());
                for (int i = 0; i < std::min<int>(top_k, (int)ranked.size()) && rc == MGR_OK; i++) {
                    const int c = ranked[(size_t)i].second;
                    if (timed_ms.count(c)) continue;
                    double ms = 0.0;
                    rc = time_chunk(c, &ms);
                    if (rc == MGR_OK) timed_ms[c] = ms;
                }
                for (const auto& kv : timed_ms)
                    if (kv.second < best) {
                        best = kv.second;
                        best_chunk = kv.first;
                        best_mode = mode;
                        best_wide = wide;
                    }
            }
        }
        b->wide = best_wide;
        for (int m = 0; m < 2; m++)
            for (int i = 0; i < kModelTerms; i++) b->model[m][i] = models[best_wide][m][i];
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        b->persistent = best_mode;
        if (rc) return rc;
        rc = b->dtype == MGR_F64 ? batch_upload<double>(*b, best_chunk) : batch_upload<float>(*b, best_chunk);
        if (rc == MGR_OK) b->tuned = 1;
        return rc;
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_batch_tuning(const mgr_batch_plan* plan, int* persistent, double* model)
{
    const BatchPlan* b = reinterpret_cast<const BatchPlan*>(plan);
    if (!b) return fail(MGR_ERR_ARG, "plan is NULL");
    if (persistent) *persistent = b->persistent;
    if (model)
        for (int m = 0; m < 2; m++)
            for (int i = 0; i < kModelTerms; i++) model[kModelTerms * m + i] = b->model[m][i];
    return MGR_OK;
}

int mgr_batch_config(const mgr_batch_plan* plan, int* chunk, int* launches, int64_t* items)
{
    const BatchPlan* b = reinterpret_cast<const BatchPlan*>(plan);
    if (!b) return fail(MGR_ERR_ARG, "plan is NULL");
    if (chunk) *chunk = b->chunk;
    // kernel launches per call besides the pointer upload: the waves and the
    // tail, or the queue reset, the queue and the tail
    if (launches) *launches = b->persistent ? 3 : (int)b->waves.size() + 1;
    if (items) *items = b->n_items;
    return MGR_OK;
}

int mgr_batch_set_config(mgr_batch_plan* plan, int chunk)
{
    try {
        g_err.clear();
        BatchPlan* b = reinterpret_cast<BatchPlan*>(plan);
        if (!b) return fail(MGR_ERR_ARG, "plan is NULL");
        if (chunk < 1 || chunk > kMaxBatchChunk) return fail(MGR_ERR_ARG, "chunk must be 1.." + std::to_string(kMaxBatchChunk));
        return b->dtype == MGR_F64 ? batch_upload<double>(*b, chunk) : batch_upload<float>(*b, chunk);
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_batch_tile(const mgr_batch_plan* plan, int* wide)
{
    const BatchPlan* b = reinterpret_cast<const BatchPlan*>(plan);
    if (!b || !wide) return fail(MGR_ERR_ARG, "plan or output is NULL");
    *wide = b->wide;
    return MGR_OK;
}

int mgr_batch_set_tile(mgr_batch_plan* plan, int wide)
{
    try {
        g_err.clear();
        BatchPlan* b = reinterpret_cast<BatchPlan*>(plan);
        if (!b) return fail(MGR_ERR_ARG, "plan is NULL");
        if (wide != 0 && wide != 1) return fail(MGR_ERR_ARG, "wide must be 0 or 1");
        b->wide = wide;
        return b->dtype == MGR_F64 ? batch_upload<double>(*b, b->chunk) : batch_upload<float>(*b, b->chunk);
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_batch_set_mode(mgr_batch_plan* plan, int persistent, unsigned poll_limit)
{
    g_err.clear();
    BatchPlan* b = reinterpret_cast<BatchPlan*>(plan);
    if (!b) return fail(MGR_ERR_ARG, "plan is NULL");
    if (persistent != 0 && persistent != 1) return fail(MGR_ERR_ARG, "persistent must be 0 or 1");
    b->persistent = persistent;
    b->poll_limit = poll_limit ? poll_limit : (1u << 20);
    return MGR_OK;
}

int mgr_batch_check(mgr_batch_plan* plan)
{
    try {
        g_err.clear();
        BatchPlan* b = reinterpret_cast<BatchPlan*>(plan);
        if (!b) return fail(MGR_ERR_ARG, "plan is NULL");
        MGR_TRY(hipDeviceSynchronize(), "synchronise");
        std::vector<int> w(kQueueWordsFixed + b->qneed.size(), 0);
        MGR_TRY(hipMemcpy(w.data(), (char*)b->dev + b->off_qwords, sizeof(int) * w.size(), hipMemcpyDeviceToHost),
                "read queue words");
        const QueueState qs = queue_state(w.data());
        if (*qs.abort || *qs.err) {
            std::string d;
            const int pos = *qs.err - 1;
            int item = -1;
            if (pos >= 0 && pos < (int)b->qorder.size()) {
                item = b->qorder[(size_t)pos];
                int q = 0;
                while (q + 1 < b->nq && b->qstart[(size_t)q + 1] <= pos) q++;
                const int g = b->qgrp[(size_t)pos], dg = b->qdep[(size_t)g];
                d = " (queue " + std::to_string(q) + ", group " + std::to_string(g) + ", waiting on group " +
                    std::to_string(dg);
                if (dg >= 0)
                    d += " with " + std::to_string(qs.done[dg]) + " of " + std::to_string(b->qneed[(size_t)dg]) +
                         " items finished";
                d += "; " + std::to_string(std::min(qs.next[q], b->qstart[(size_t)q + 1] - b->qstart[(size_t)q])) +
                     " of the queue's " + std::to_string(b->qstart[(size_t)q + 1] - b->qstart[(size_t)q]) +
                     " items taken)";
            }
            return fail(MGR_ERR_HIP, "persistent batch: a dependency wait timed out at work item " +
                                         std::to_string(item) + d + "; the outputs of that run are incomplete");
        }
        if (b->ran_persistent)
            for (int q = 0; q < b->nq; q++)
                if (qs.next[q] < b->qstart[(size_t)q + 1] - b->qstart[(size_t)q])
                    return fail(MGR_ERR_HIP, "persistent batch: queue " + std::to_string(q) + " has items no workgroup took (" +
                                                 std::to_string(qs.next[q]) + " of " +
                                                 std::to_string(b->qstart[(size_t)q + 1] - b->qstart[(size_t)q]) +
                                                 "); the outputs of that run are incomplete");
        return MGR_OK;
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

int mgr_batch_queue_check(int nfields, const int* ndim, const int64_t* const* shapes, const int* nlevels, int dtype,
                          int chunk, int nqueues, int nthreads, unsigned poll_limit, int stall_item, uint64_t seed,
                          int64_t* out)
{
    try {
        g_err.clear();
        if (!out) return fail(MGR_ERR_ARG, "out is NULL");
        BatchPlan b;
        int rc = batch_host_items(nfields, ndim, shapes, nlevels, dtype, chunk, nqueues, b);
        if (rc) return rc;
        return queue_check(b, nthreads, poll_limit ? poll_limit : (1u << 20), stall_item, seed, out);
    } catch (const std::bad_alloc&) {
        return fail(MGR_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return fail(MGR_ERR_HIP, "unexpected exception");
    }
}

void mgr_batch_plan_destroy(mgr_batch_plan* plan)
{
    BatchPlan* b = reinterpret_cast<BatchPlan*>(plan);
    if (!b) return;
    free_batch(b);  // hipFree waits for work still using the memory
}

}  // extern "C"
