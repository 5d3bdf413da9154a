/*
 * mgr_oracle.c - plain FP64 CPU oracle for multigrid hierarchical data
 * refactoring (Chen et al., arXiv 2007.04457, Sec. II-A).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg; never by the GPU product path.  It shares no
 * code, header, table or helper with the GPU path.
 *
 * The oracle is deliberately slow and literal.  It works in place on the full
 * array.  Level step k (k = 0 is the finest) acts on the "level grid": the
 * nodes whose every index is a multiple of 2^k; its coarse nodes are those
 * whose every index is a multiple of 2^(k+1) and all others are its fine-only
 * nodes N_l \ N_{l-1} (Sec. II-A, Table I).  One decomposition step is, in
 * the paper's order (Eq. (1)):
 *   1. coefficients  C_l = (I - Pi_{l-1}) Q_l u at the fine-only nodes, by
 *      multilinear interpolation from the coarse nodes (Sec. II-A.1);
 *   2. load vector   f_{l-1} = R_l M_l vec(C_l), C_l zero at coarse nodes,
 *      applied one dimension at a time (Sec. II-A.2 and Sec. III-A.2);
 *   3. correction    M_{l-1} z_{l-1} = f_{l-1}, one tridiagonal (Thomas)
 *      solve per fibre and dimension (Sec. II-A.2, Sec. III-A.3);
 *   4. apply         coarse nodes += z_{l-1}  (Eq. (1), last term).
 * Recomposition runs the same stages in reverse, coarse to fine.
 *
 * Readings of the paper taken here (the printed formulas are garbled):
 *  - The 1D mass matrix (Sec. III-A.2) is the piecewise-linear finite-element
 *    mass matrix scaled by 6: diagonal 2(h_{j-1}+h_j), off-diagonals h_j
 *    between nodes j and j+1, one-sided at the two boundary nodes.
 *  - The transfer matrix R (Sec. III-A.2) is the transpose of the piecewise
 *    linear interpolation P from the coarse to the fine level.
 *  - Multi-dimensional coefficients use direct multilinear interpolation from
 *    the coarse nodes (Sec. II-A.1), never sequential 1D updates.
 *  - Dimensions are processed last-to-first for the load vector and the
 *    solve (rows first, Sec. II-A "Overall process").
 *  - Sizes (the paper's grids are all 2^k + 1 nodes per dimension and it is
 *    silent on others): a level grid of m nodes along a dimension keeps as
 *    coarse nodes its even positions and its last node, so both boundary
 *    nodes stay on every level and a level of even length has no fine node
 *    in its last interval.  The level-k grid along a dimension of n nodes is
 *    then {i : 2^k divides i} plus the node n - 1, of size
 *    ceil((n - 1) / 2^k) + 1; for n = 2^K + 1 this is the usual stride-2^k
 *    grid.  All dimensions coarsen together; the full decomposition stops
 *    when the shortest level grid has 3 nodes.
 */
#include "mgr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXD 4

/* Threads for the loops over independent fibres and nodes (OpenMP when the
 * library is built with it).  Every element is computed by the same
 * arithmetic in the same order whatever the thread count, so results are
 * bitwise independent of it.  Default 1. */
static int g_threads = 1;

int oracle_set_threads(int n)
{
    int prev = g_threads;
    g_threads = (n < 1) ? 1 : n;
    return prev;
}

typedef struct {
    int nd;
    int64_t n[MAXD];     /* full grid sizes */
    int64_t st[MAXD];    /* full-array element strides (C order) */
    const double* const* x;
} grid_t;

/* Node position along dimension d of full-grid index i. */
static double node_x(const grid_t* g, int d, int64_t i)
{
    if (g->x && g->x[d]) return g->x[d][i];
    return (double)i;
}

/* Level steps after which a dimension of n >= 3 nodes is down to 2 nodes:
 * the smallest K with 2^K >= n - 1. */
static int steps_to_two(int64_t n)
{
    int k = 0;
    while (((int64_t)1 << k) < n - 1) k++;
    return k;
}

int oracle_max_levels(int ndim, const int64_t* shape)
{
    if (ndim < 1 || ndim > MAXD || !shape) return -1;
    int kmin = 64;
    for (int d = 0; d < ndim; d++) {
        if (shape[d] < 3) return -2;
        int k = steps_to_two(shape[d]);
        if (k < kmin) kmin = k;
    }
    return kmin - 1;
}

static int setup(grid_t* g, int ndim, const int64_t* shape,
                 const double* const* coords, int* nlevels)
{
    if (ndim < 1 || ndim > MAXD || !shape) return 1;
    int full = oracle_max_levels(ndim, shape);
    if (full < 0) return 2;
    if (*nlevels == -1) *nlevels = full;
    if (*nlevels < 0 || *nlevels > full + 1) return 3;
    g->nd = ndim;
    g->x = coords;
    for (int d = 0; d < ndim; d++) g->n[d] = shape[d];
    int64_t s = 1;
    for (int d = ndim - 1; d >= 0; d--) { g->st[d] = s; s *= shape[d]; }
    if (coords) {
        for (int d = 0; d < ndim; d++) {
            if (!coords[d]) continue;
            for (int64_t i = 1; i < shape[d]; i++)
                if (!(coords[d][i] > coords[d][i - 1])) return 4;
        }
    }
    return 0;
}

/* Level-grid size along d at step k: ceil((n - 1) / 2^k) + 1. */
static int64_t lsize(const grid_t* g, int d, int k)
{
    return ((g->n[d] - 2) >> k) + 2;
}

/* Full-grid index along d of level index j at step k: the j-th multiple of
 * 2^k, or the last node. */
static int64_t lpos(const grid_t* g, int d, int k, int64_t j)
{
    const int64_t i = j << k;
    return (i < g->n[d] - 1) ? i : g->n[d] - 1;
}

/* Whether level index j of a level grid of m nodes is fine-only (odd and
 * not the last node); every other index is coarse. */
static int is_fine(int64_t j, int64_t m)
{
    return (j & 1) && j != m - 1;
}

/* Coarse-grid index of a coarse level index j (m nodes): j / 2, or the last
 * coarse index for the last node. */
static int64_t coarse_index(int64_t j, int64_t m)
{
    return (j == m - 1) ? m / 2 : j / 2;
}

/* Coordinates of the level grid at step k along d (length lsize). */
static double* level_coords(const grid_t* g, int d, int k)
{
    int64_t m = lsize(g, d, k);
    double* y = (double*)malloc(sizeof(double) * (size_t)m);
    if (!y) return NULL;
    for (int64_t j = 0; j < m; j++) y[j] = node_x(g, d, lpos(g, d, k, j));
    return y;
}

/* Linear interpolation weight of the upper coarse neighbour for an odd
 * level index j: a_j = (y_j - y_{j-1}) / (y_{j+1} - y_{j-1}). */
static double interp_a(const double* y, int64_t j)
{
    return (y[j] - y[j - 1]) / (y[j + 1] - y[j - 1]);
}

/* Full-array offset of level-grid multi-index j at step k. */
static int64_t offset_of(const grid_t* g, const int64_t* j, int k)
{
    int64_t o = 0;
    for (int d = 0; d < g->nd; d++) o += lpos(g, d, k, j[d]) * g->st[d];
    return o;
}

/* Multi-index j of the C-order flat index idx in a box of sizes m. */
static void index_of(int nd, int64_t idx, const int64_t* m, int64_t* j)
{
    for (int d = nd - 1; d >= 0; d--) {
        j[d] = idx % m[d];
        idx /= m[d];
    }
}

/* Odometer increment over a box of sizes m; returns 0 when wrapped. */
static int next_index(int nd, int64_t* j, const int64_t* m)
{
    for (int d = nd - 1; d >= 0; d--) {
        if (++j[d] < m[d]) return 1;
        j[d] = 0;
    }
    return 0;
}

/* ---- 1D operators (Sec. III-A.2, readings above) ----------------------- */

/* out = M v on nodes y[0..m-1]. */
static void mass_mult(const double* v, double* out, int64_t m, const double* y)
{
    for (int64_t j = 0; j < m; j++) {
        double hl = (j > 0) ? y[j] - y[j - 1] : 0.0;
        double hr = (j < m - 1) ? y[j + 1] - y[j] : 0.0;
        double s = 2.0 * (hl + hr) * v[j];
        if (j > 0) s += hl * v[j - 1];
        if (j < m - 1) s += hr * v[j + 1];
        out[j] = s;
    }
}

/* out = P^T w: restriction from m fine nodes to the m / 2 + 1 coarse
 * nodes.  Coarse node i (level index f: 2i, or the last node) collects
 * itself and its fine-only neighbours with their interpolation weights. */
static void restrict_t(const double* w, double* out, int64_t m, const double* y)
{
    int64_t mc = m / 2 + 1;
    for (int64_t i = 0; i < mc; i++) {
        int64_t f = (i == mc - 1) ? m - 1 : 2 * i;
        double s = w[f];
        if (f - 1 >= 0 && is_fine(f - 1, m)) s += interp_a(y, f - 1) * w[f - 1];
        if (f + 1 < m && is_fine(f + 1, m)) s += (1.0 - interp_a(y, f + 1)) * w[f + 1];
        out[i] = s;
    }
}

/* out = P z: piecewise-linear prolongation from m / 2 + 1 coarse nodes to
 * m fine nodes. */
static void prolong(const double* z, double* out, int64_t m, const double* y)
{
    for (int64_t j = 0; j < m; j++) {
        if (!is_fine(j, m)) {
            out[j] = z[coarse_index(j, m)];
        } else {
            double a = interp_a(y, j);
            out[j] = (1.0 - a) * z[(j - 1) / 2] + a * z[(j + 1) / 2];
        }
    }
}

/* Solve M z = f in place (M = mass matrix on nodes yc[0..mc-1]) with the
 * textbook Thomas algorithm; no pivoting is needed because M is symmetric
 * positive definite and strictly diagonally dominant. */
static int thomas(double* f, int64_t mc, const double* yc)
{
    double* cp = (double*)malloc(sizeof(double) * (size_t)mc);
    if (!cp) return 6;
    for (int64_t i = 0; i < mc; i++) {
        double hl = (i > 0) ? yc[i] - yc[i - 1] : 0.0;
        double hr = (i < mc - 1) ? yc[i + 1] - yc[i] : 0.0;
        double diag = 2.0 * (hl + hr);
        double sub = hl;   /* coefficient of z_{i-1} */
        double sup = hr;   /* coefficient of z_{i+1} */
        if (i == 0) {
            cp[i] = sup / diag;
            f[i] = f[i] / diag;
        } else {
            double den = diag - sub * cp[i - 1];
            cp[i] = sup / den;
            f[i] = (f[i] - sub * f[i - 1]) / den;
        }
    }
    for (int64_t i = mc - 2; i >= 0; i--) f[i] -= cp[i] * f[i + 1];
    free(cp);
    return 0;
}

enum { OP_MASSTRANS, OP_SOLVE, OP_PROLONG_MASS };

/* Apply a 1D operator to every fibre along dimension d of a packed array A
 * of shape sh, writing packed B whose size along d is m_out (the coarse size
 * for OP_MASSTRANS, the fine size for OP_PROLONG_MASS, sh[d] for OP_SOLVE). */
static int along_dim(const double* A, double* B, int nd, const int64_t* sh,
                     int d, int op, const double* y, int64_t m_out)
{
    int64_t outer = 1, inner = 1, m_in = sh[d];
    for (int e = 0; e < d; e++) outer *= sh[e];
    for (int e = d + 1; e < nd; e++) inner *= sh[e];
    int64_t mx = (m_in > m_out) ? m_in : m_out;
    int64_t nfib = outer * inner;
    int rc = 0;
    /* every fibre is independent: one per iteration, each thread with its
     * own two fibre buffers */
#pragma omp parallel num_threads(g_threads) if (g_threads > 1)
    {
        double* t0 = (double*)malloc(sizeof(double) * (size_t)mx);
        double* t1 = (double*)malloc(sizeof(double) * (size_t)mx);
        int lrc = (t0 && t1) ? 0 : 6;
#pragma omp for schedule(static)
        for (int64_t fb = 0; fb < nfib; fb++) {
            if (lrc) continue;
            int64_t o = fb / inner, in = fb % inner;
            for (int64_t j = 0; j < m_in; j++) t0[j] = A[(o * m_in + j) * inner + in];
            if (op == OP_MASSTRANS) {
                mass_mult(t0, t1, m_in, y);
                restrict_t(t1, t0, m_in, y);
            } else if (op == OP_SOLVE) {
                lrc = thomas(t0, m_in, y);
            } else {
                prolong(t0, t1, m_out, y);
                mass_mult(t1, t0, m_out, y);
            }
            for (int64_t i = 0; i < m_out; i++) B[(o * m_out + i) * inner + in] = t0[i];
        }
        free(t0);
        free(t1);
#pragma omp critical
        if (lrc && !rc) rc = lrc;
    }
    return rc;
}

/* ---- the four stages of one level step --------------------------------- */

/* Stage 1 (Sec. II-A.1): c(p) = u(p) - sum_q w(p,q) u(q) over the 2^t coarse
 * corners q of each fine-only node p (t = number of odd level indices of p),
 * w(p,q) the product of the 1D linear-interpolation weights.  Coarse values
 * are never modified, so updating in place is safe. */
static int stage_coefficients(double* u, const grid_t* g, int k)
{
    int nd = g->nd;
    int64_t m[MAXD], V = 1;
    double* y[MAXD] = {0};
    int rc = 0;
    for (int d = 0; d < nd; d++) {
        m[d] = lsize(g, d, k);
        V *= m[d];
        y[d] = level_coords(g, d, k);
        if (!y[d]) rc = 6;
    }
    if (rc == 0) {
        /* each node reads only coarse nodes, which this stage never writes,
         * so the nodes are independent */
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1)
        for (int64_t idx = 0; idx < V; idx++) {
            int64_t j[MAXD];
            index_of(nd, idx, m, j);
            int odd[MAXD], t = 0;
            for (int d = 0; d < nd; d++) { odd[d] = is_fine(j[d], m[d]); t += odd[d]; }
            if (t == 0) continue;
            double interp = 0.0;
            for (int mask = 0; mask < (1 << nd); mask++) {
                int skip = 0;
                double w = 1.0;
                int64_t q[MAXD];
                for (int d = 0; d < nd; d++) {
                    int up = (mask >> d) & 1;
                    if (!odd[d]) {
                        if (up) { skip = 1; break; }
                        q[d] = j[d];
                    } else {
                        double a = interp_a(y[d], j[d]);
                        q[d] = up ? j[d] + 1 : j[d] - 1;
                        w *= up ? a : (1.0 - a);
                    }
                }
                if (skip) continue;
                interp += w * u[offset_of(g, q, k)];
            }
            u[offset_of(g, j, k)] -= interp;
        }
    }
    for (int d = 0; d < nd; d++) free(y[d]);
    return rc;
}

/* Stage 2 (Sec. II-A.2): f = R M vec(C) with C the level grid holding the
 * coefficients at fine-only nodes and zeros at coarse nodes.  M and R are
 * tensor products; they are applied dimension by dimension, last first.
 * f is written packed, of size (m_d+1)/2 per dimension. */
static int stage_load_vector(const double* u, double* f, const grid_t* g, int k)
{
    int nd = g->nd;
    int64_t m[MAXD], j[MAXD] = {0, 0, 0, 0}, V = 1;
    for (int d = 0; d < nd; d++) { m[d] = lsize(g, d, k); V *= m[d]; }
    double* a = (double*)malloc(sizeof(double) * (size_t)V);
    double* b = (double*)malloc(sizeof(double) * (size_t)V);
    int rc = (a && b) ? 0 : 6;
    if (rc == 0) {
        int64_t idx = 0;
        do {
            int coarse = 1;
            for (int d = 0; d < nd; d++) if (is_fine(j[d], m[d])) coarse = 0;
            a[idx++] = coarse ? 0.0 : u[offset_of(g, j, k)];
        } while (next_index(nd, j, m));
        int64_t sh[MAXD];
        for (int d = 0; d < nd; d++) sh[d] = m[d];
        for (int d = nd - 1; d >= 0 && rc == 0; d--) {
            double* y = level_coords(g, d, k);
            if (!y) { rc = 6; break; }
            rc = along_dim(a, b, nd, sh, d, OP_MASSTRANS, y, sh[d] / 2 + 1);
            free(y);
            sh[d] = sh[d] / 2 + 1;
            double* t = a; a = b; b = t;
        }
        if (rc == 0) {
            int64_t Vc = 1;
            for (int d = 0; d < nd; d++) Vc *= sh[d];
            memcpy(f, a, sizeof(double) * (size_t)Vc);
        }
    }
    free(a);
    free(b);
    return rc;
}

/* Stage 3 (Sec. II-A.2, Sec. III-A.3): solve M_{l-1} z = f in place, where
 * M_{l-1} is the tensor product of the 1D mass matrices on the coarse level
 * coordinates; one Thomas solve per fibre, dimensions last first. */
static int stage_correction(double* f, const grid_t* g, int k, int reverse)
{
    int nd = g->nd;
    int64_t sh[MAXD], Vc = 1;
    for (int d = 0; d < nd; d++) { sh[d] = lsize(g, d, k + 1); Vc *= sh[d]; }
    double* tmp = (double*)malloc(sizeof(double) * (size_t)Vc);
    int rc = tmp ? 0 : 6;
    for (int s = 0; s < nd && rc == 0; s++) {
        int d = reverse ? s : nd - 1 - s;
        double* yc = level_coords(g, d, k + 1);
        if (!yc) { rc = 6; break; }
        rc = along_dim(f, tmp, nd, sh, d, OP_SOLVE, yc, sh[d]);
        free(yc);
        memcpy(f, tmp, sizeof(double) * (size_t)Vc);
    }
    free(tmp);
    return rc;
}

/* Adds sign * z (packed, coarse level shape) to the coarse nodes of the
 * level grid at step k. */
static void stage_apply(double* u, const double* z, const grid_t* g, int k, double sign)
{
    int nd = g->nd;
    int64_t mc[MAXD], j[MAXD] = {0, 0, 0, 0}, idx = 0;
    for (int d = 0; d < nd; d++) mc[d] = lsize(g, d, k + 1);
    do {
        u[offset_of(g, j, k + 1)] += sign * z[idx++];
    } while (next_index(nd, j, mc));
}

/* Recomposition stage: u(p) += sum_q w(p,q) u(q) at fine-only nodes p. */
static int stage_interpolate_add(double* u, const grid_t* g, int k)
{
    int nd = g->nd;
    int64_t m[MAXD], V = 1;
    double* y[MAXD] = {0};
    int rc = 0;
    for (int d = 0; d < nd; d++) {
        m[d] = lsize(g, d, k);
        V *= m[d];
        y[d] = level_coords(g, d, k);
        if (!y[d]) rc = 6;
    }
    if (rc == 0) {
        /* each node reads only coarse nodes, which this stage never writes,
         * so the nodes are independent */
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1)
        for (int64_t idx = 0; idx < V; idx++) {
            int64_t j[MAXD];
            index_of(nd, idx, m, j);
            int odd[MAXD], t = 0;
            for (int d = 0; d < nd; d++) { odd[d] = is_fine(j[d], m[d]); t += odd[d]; }
            if (t == 0) continue;
            double interp = 0.0;
            for (int mask = 0; mask < (1 << nd); mask++) {
                int skip = 0;
                double w = 1.0;
                int64_t q[MAXD];
                for (int d = 0; d < nd; d++) {
                    int up = (mask >> d) & 1;
                    if (!odd[d]) {
                        if (up) { skip = 1; break; }
                        q[d] = j[d];
                    } else {
                        double a = interp_a(y[d], j[d]);
                        q[d] = up ? j[d] + 1 : j[d] - 1;
                        w *= up ? a : (1.0 - a);
                    }
                }
                if (skip) continue;
                interp += w * u[offset_of(g, q, k)];
            }
            u[offset_of(g, j, k)] += interp;
        }
    }
    for (int d = 0; d < nd; d++) free(y[d]);
    return rc;
}

static int64_t coarse_count(const grid_t* g, int k)
{
    int64_t Vc = 1;
    for (int d = 0; d < g->nd; d++) Vc *= lsize(g, d, k + 1);
    return Vc;
}

/* ---- public entry points ------------------------------------------------ */

int oracle_decompose(double* u, int ndim, const int64_t* shape,
                     const double* const* coords, int nlevels)
{
    grid_t g;
    if (!u) return 1;
    int rc = setup(&g, ndim, shape, coords, &nlevels);
    if (rc) return rc;
    for (int k = 0; k < nlevels && rc == 0; k++) {
        double* f = (double*)malloc(sizeof(double) * (size_t)coarse_count(&g, k));
        if (!f) return 6;
        rc = stage_coefficients(u, &g, k);
        if (rc == 0) rc = stage_load_vector(u, f, &g, k);
        if (rc == 0) rc = stage_correction(f, &g, k, 0);
        if (rc == 0) stage_apply(u, f, &g, k, +1.0);
        free(f);
    }
    return rc;
}

int oracle_recompose(double* u, int ndim, const int64_t* shape,
                     const double* const* coords, int nlevels)
{
    grid_t g;
    if (!u) return 1;
    int rc = setup(&g, ndim, shape, coords, &nlevels);
    if (rc) return rc;
    for (int k = nlevels - 1; k >= 0 && rc == 0; k--) {
        double* f = (double*)malloc(sizeof(double) * (size_t)coarse_count(&g, k));
        if (!f) return 6;
        rc = stage_load_vector(u, f, &g, k);
        if (rc == 0) rc = stage_correction(f, &g, k, 0);
        if (rc == 0) stage_apply(u, f, &g, k, -1.0);
        if (rc == 0) rc = stage_interpolate_add(u, &g, k);
        free(f);
    }
    return rc;
}

/* Transpose of one decomposition step.  With c = x_f - Phi x_c (Phi the
 * multilinear interpolation), z = A c (A = M_c^{-1} R M E_f, E_f embedding
 * fine values with zeros at coarse nodes) and x_c' = x_c + z, the transpose
 * maps (g_c, g_f) to
 *     out_f = g_f + E_f^T M P M_c^{-1} g_c,
 *     out_c = g_c - Phi^T out_f,
 * using M, M_c symmetric and R = P^T.  Steps run coarse to fine. */
int oracle_decompose_adjoint(double* g_arr, int ndim, const int64_t* shape,
                             const double* const* coords, int nlevels)
{
    grid_t g;
    if (!g_arr) return 1;
    int rc = setup(&g, ndim, shape, coords, &nlevels);
    if (rc) return rc;
    int nd = g.nd;
    for (int k = nlevels - 1; k >= 0 && rc == 0; k--) {
        int64_t m[MAXD], mc[MAXD], V = 1, Vc = 1, j[MAXD] = {0, 0, 0, 0};
        for (int d = 0; d < nd; d++) {
            m[d] = lsize(&g, d, k);
            mc[d] = lsize(&g, d, k + 1);
            V *= m[d];
            Vc *= mc[d];
        }
        double* a = (double*)malloc(sizeof(double) * (size_t)V);
        double* b = (double*)malloc(sizeof(double) * (size_t)V);
        if (!a || !b) { free(a); free(b); return 6; }
        /* w = M_c^{-1} g_c */
        int64_t idx = 0;
        do { a[idx++] = g_arr[offset_of(&g, j, k + 1)]; } while (next_index(nd, j, mc));
        rc = stage_correction(a, &g, k, 1);
        /* t = (M P) w along every dimension (first to last). */
        int64_t sh[MAXD];
        for (int d = 0; d < nd; d++) sh[d] = mc[d];
        for (int d = 0; d < nd && rc == 0; d++) {
            double* y = level_coords(&g, d, k);
            if (!y) { rc = 6; break; }
            rc = along_dim(a, b, nd, sh, d, OP_PROLONG_MASS, y, m[d]);
            free(y);
            sh[d] = m[d];
            double* t = a; a = b; b = t;
        }
        if (rc == 0) {
            /* out_f = g_f + t at fine-only nodes. */
            double* y[MAXD] = {0};
            for (int d = 0; d < nd; d++) { y[d] = level_coords(&g, d, k); if (!y[d]) rc = 6; }
            if (rc == 0) {
                memset(j, 0, sizeof(j));
                idx = 0;
                do {
                    int fine = 0;
                    for (int d = 0; d < nd; d++) if (is_fine(j[d], m[d])) fine = 1;
                    if (fine) g_arr[offset_of(&g, j, k)] += a[idx];
                    idx++;
                } while (next_index(nd, j, m));
                /* out_c = g_c - Phi^T out_f: scatter each fine value to its
                 * coarse corners with the interpolation weights. */
                memset(j, 0, sizeof(j));
                do {
                    int odd[MAXD], t = 0;
                    for (int d = 0; d < nd; d++) { odd[d] = is_fine(j[d], m[d]); t += odd[d]; }
                    if (t == 0) continue;
                    double vf = g_arr[offset_of(&g, j, k)];
                    for (int mask = 0; mask < (1 << nd); mask++) {
                        int skip = 0;
                        double w = 1.0;
                        int64_t q[MAXD];
                        for (int d = 0; d < nd; d++) {
                            int up = (mask >> d) & 1;
                            if (!odd[d]) {
                                if (up) { skip = 1; break; }
                                q[d] = j[d];
                            } else {
                                double aa = interp_a(y[d], j[d]);
                                q[d] = up ? j[d] + 1 : j[d] - 1;
                                w *= up ? aa : (1.0 - aa);
                            }
                        }
                        if (skip) continue;
                        g_arr[offset_of(&g, q, k)] -= w * vf;
                    }
                } while (next_index(nd, j, m));
            }
            for (int d = 0; d < nd; d++) free(y[d]);
        }
        free(a);
        free(b);
    }
    return rc;
}

/* Transpose of the recomposition, i.e. the inverse transpose D^{-T} of the
 * decomposition (derived from Eq. (1)-(2); not in the paper).  Recomposition
 * step k maps (y_c, y_f) to x_c = y_c - A y_f, x_f = y_f + Phi x_c (A as for
 * the decomposition's transpose above), so its transpose maps (g_c, g_f) to
 *     g_c' = g_c + Phi^T g_f,
 *     g_f' = g_f - A^T g_c' = g_f - E_f^T M P M_c^{-1} g_c'.
 * Recomposition runs coarse to fine, so its transpose runs fine to coarse. */
int oracle_recompose_adjoint(double* g_arr, int ndim, const int64_t* shape,
                             const double* const* coords, int nlevels)
{
    grid_t g;
    if (!g_arr) return 1;
    int rc = setup(&g, ndim, shape, coords, &nlevels);
    if (rc) return rc;
    int nd = g.nd;
    for (int k = 0; k < nlevels && rc == 0; k++) {
        int64_t m[MAXD], mc[MAXD], V = 1, j[MAXD] = {0, 0, 0, 0};
        double* y[MAXD] = {0};
        for (int d = 0; d < nd; d++) {
            m[d] = lsize(&g, d, k);
            mc[d] = lsize(&g, d, k + 1);
            V *= m[d];
            y[d] = level_coords(&g, d, k);
            if (!y[d]) rc = 6;
        }
        double* a = (double*)malloc(sizeof(double) * (size_t)V);
        double* b = (double*)malloc(sizeof(double) * (size_t)V);
        if (!a || !b) rc = 6;
        if (rc == 0) {
            /* g_c' = g_c + Phi^T g_f: each fine-only value goes to its coarse
             * corners with the interpolation weights. */
            do {
                int odd[MAXD], t = 0;
                for (int d = 0; d < nd; d++) { odd[d] = is_fine(j[d], m[d]); t += odd[d]; }
                if (t == 0) continue;
                double vf = g_arr[offset_of(&g, j, k)];
                for (int mask = 0; mask < (1 << nd); mask++) {
                    int skip = 0;
                    double w = 1.0;
                    int64_t q[MAXD];
                    for (int d = 0; d < nd; d++) {
                        int up = (mask >> d) & 1;
                        if (!odd[d]) {
                            if (up) { skip = 1; break; }
                            q[d] = j[d];
                        } else {
                            double aa = interp_a(y[d], j[d]);
                            q[d] = up ? j[d] + 1 : j[d] - 1;
                            w *= up ? aa : (1.0 - aa);
                        }
                    }
                    if (skip) continue;
                    g_arr[offset_of(&g, q, k)] += w * vf;
                }
            } while (next_index(nd, j, m));
            /* w = M_c^{-1} g_c' */
            int64_t idx = 0;
            memset(j, 0, sizeof(j));
            do { a[idx++] = g_arr[offset_of(&g, j, k + 1)]; } while (next_index(nd, j, mc));
            rc = stage_correction(a, &g, k, 1);
            /* t = (M P) w along every dimension (first to last) */
            int64_t sh[MAXD];
            for (int d = 0; d < nd; d++) sh[d] = mc[d];
            for (int d = 0; d < nd && rc == 0; d++) {
                rc = along_dim(a, b, nd, sh, d, OP_PROLONG_MASS, y[d], m[d]);
                sh[d] = m[d];
                double* tt = a; a = b; b = tt;
            }
            /* g_f' = g_f - t at the fine-only nodes */
            if (rc == 0) {
                memset(j, 0, sizeof(j));
                idx = 0;
                do {
                    int fine = 0;
                    for (int d = 0; d < nd; d++) if (is_fine(j[d], m[d])) fine = 1;
                    if (fine) g_arr[offset_of(&g, j, k)] -= a[idx];
                    idx++;
                } while (next_index(nd, j, m));
            }
        }
        free(a);
        free(b);
        for (int d = 0; d < nd; d++) free(y[d]);
    }
    return rc;
}

int oracle_coefficients_level(double* u, int ndim, const int64_t* shape,
                              const double* const* coords, int k)
{
    grid_t g;
    int nl = -1;
    if (!u) return 1;
    int rc = setup(&g, ndim, shape, coords, &nl);
    if (rc) return rc;
    if (k < 0 || k > nl) return 3;
    return stage_coefficients(u, &g, k);
}

int oracle_load_vector_level(const double* u, double* f, int ndim,
                             const int64_t* shape, const double* const* coords,
                             int k)
{
    grid_t g;
    int nl = -1;
    if (!u || !f) return 1;
    int rc = setup(&g, ndim, shape, coords, &nl);
    if (rc) return rc;
    if (k < 0 || k > nl) return 3;
    return stage_load_vector(u, f, &g, k);
}

int oracle_correction_level(double* f, int ndim, const int64_t* shape,
                            const double* const* coords, int k)
{
    grid_t g;
    int nl = -1;
    if (!f) return 1;
    int rc = setup(&g, ndim, shape, coords, &nl);
    if (rc) return rc;
    if (k < 0 || k > nl) return 3;
    return stage_correction(f, &g, k, 0);
}

int oracle_class_map(int ndim, const int64_t* shape, int nlevels, uint8_t* out)
{
    grid_t g;
    if (!out) return 1;
    int rc = setup(&g, ndim, shape, NULL, &nlevels);
    if (rc) return rc;
    int64_t j[MAXD] = {0, 0, 0, 0}, idx = 0;
    do {
        /* Finest step k at which node j is a level-grid node that is not
         * coarse: the smallest 2-adic valuation over its indices. */
        int v = nlevels;
        for (int d = 0; d < g.nd; d++) {
            int vd = 0;
            /* the first and last nodes are on every level grid */
            if (j[d] == 0 || j[d] == g.n[d] - 1) continue;
            while (((j[d] >> vd) & 1) == 0) vd++;
            if (vd < v) v = vd;
        }
        out[idx++] = (uint8_t)((v >= nlevels) ? 0 : nlevels - v);
    } while (next_index(g.nd, j, g.n));
    return 0;
}

/* ---- quantisation of the classes (Sec. V, lossy compression) -------------
 * The paper moves MGARD's quantisation and dequantisation of the refactored
 * classes onto the GPU but does not state the quantiser.  Reading taken: a
 * uniform scalar quantiser per class.  An element y of class c (bin width
 * b_c > 0) gets the code q = round-half-even(y / b_c), computed in the
 * precision of the data (the bin width is first rounded to it), and is
 * dequantised to q * b_c in that precision.  A rounded quotient that is NaN
 * or outside +-(2^31 - 1) is clamped (NaN to 0) and counted.  In the
 * in-place layout the class of an element is that of its node; in the
 * class-packed layout it is the segment the element lies in. */

/* Class of every element of the chosen layout (malloc'd; NULL on failure). */
static uint8_t* element_classes(int ndim, const int64_t* shape, int nlevels, int packed, int64_t* total)
{
    grid_t g;
    if (setup(&g, ndim, shape, NULL, &nlevels)) return NULL;
    int64_t n = 1;
    for (int d = 0; d < ndim; d++) n *= shape[d];
    uint8_t* cls = (uint8_t*)malloc((size_t)n);
    if (!cls) return NULL;
    if (oracle_class_map(ndim, shape, nlevels, cls)) {
        free(cls);
        return NULL;
    }
    if (packed) {
        /* segment c holds as many elements as there are nodes of class c */
        int64_t count[256] = {0};
        for (int64_t i = 0; i < n; i++) count[cls[i]]++;
        int64_t i = 0;
        for (int c = 0; c <= nlevels; c++)
            for (int64_t k = 0; k < count[c]; k++) cls[i++] = (uint8_t)c;
    }
    *total = n;
    return cls;
}

static int bins_ok(const double* bins, int nclasses)
{
    if (!bins) return 0;
    for (int c = 0; c < nclasses; c++)
        if (!(bins[c] > 0.0) || !isfinite(bins[c])) return 0;
    return 1;
}

static int32_t clamp_code(double q, int64_t* nclamped)
{
    if (q != q) {
        (*nclamped)++;
        return 0;
    }
    if (q > 2147483647.0) {
        (*nclamped)++;
        return 2147483647;
    }
    if (q < -2147483647.0) {
        (*nclamped)++;
        return -2147483647;
    }
    return (int32_t)q;
}

int oracle_quantize(const void* y, int32_t* q, int dtype, int ndim, const int64_t* shape, int nlevels,
                    int packed, const double* bins, int64_t* nclamped)
{
    int64_t n = 0, clamped = 0;
    if (!y || !q || (dtype != 0 && dtype != 1)) return 1;
    if (nlevels < 0) nlevels = oracle_max_levels(ndim, shape);
    if (nlevels < 0) return 2;
    if (!bins_ok(bins, nlevels + 1)) return 1;
    uint8_t* cls = element_classes(ndim, shape, nlevels, packed, &n);
    if (!cls) return 6;
    for (int64_t i = 0; i < n; i++) {
        if (dtype == 0) {
            const float b = (float)bins[cls[i]];
            const float r = ((const float*)y)[i] / b;
            q[i] = clamp_code((double)rintf(r), &clamped);
        } else {
            const double b = bins[cls[i]];
            const double r = ((const double*)y)[i] / b;
            q[i] = clamp_code(rint(r), &clamped);
        }
    }
    free(cls);
    if (nclamped) *nclamped = clamped;
    return 0;
}

int oracle_dequantize(const int32_t* q, void* y, int dtype, int ndim, const int64_t* shape, int nlevels,
                      int packed, const double* bins)
{
    int64_t n = 0;
    if (!y || !q || (dtype != 0 && dtype != 1)) return 1;
    if (nlevels < 0) nlevels = oracle_max_levels(ndim, shape);
    if (nlevels < 0) return 2;
    if (!bins_ok(bins, nlevels + 1)) return 1;
    uint8_t* cls = element_classes(ndim, shape, nlevels, packed, &n);
    if (!cls) return 6;
    for (int64_t i = 0; i < n; i++) {
        if (dtype == 0)
            ((float*)y)[i] = (float)q[i] * (float)bins[cls[i]];
        else
            ((double*)y)[i] = (double)q[i] * bins[cls[i]];
    }
    free(cls);
    return 0;
}

/* Bin widths for a bound tol on the largest pointwise error of the
 * recomposition (exact arithmetic).  A change e of the class-0 values moves
 * the recomposed values by at most max|e|: the later steps only interpolate
 * it, with nonnegative weights that sum to one.  A change e of class l >= 1
 * moves them by (I - Q_{l-1}) applied to the level-l interpolant of e (the
 * correction subtracts the projection of the coefficients, Eq. (1)), then
 * interpolated again, so by at most (1 + |Q|) max|e|, where |Q| is the
 * largest row sum of the projection's nodal matrix: the tensor product of
 * one-dimensional projections onto piecewise-linear functions, each of which
 * has a max-norm bound of 3 on any mesh, so |Q| <= 3^d.  Splitting tol
 * evenly over the L + 1 classes with errors of half a bin:
 *   b_0 = 2 tol / (L + 1),   b_l = 2 tol / ((L + 1) (1 + 3^d)). */
int oracle_quant_bins(int ndim, int nlevels, double tol, double* bins)
{
    if (!bins || ndim < 1 || ndim > MAXD || nlevels < 0 || !(tol > 0.0) || !isfinite(tol)) return 1;
    double k = 1.0;
    for (int d = 0; d < ndim; d++) k *= 3.0;
    for (int c = 0; c <= nlevels; c++)
        bins[c] = 2.0 * tol / ((double)(nlevels + 1) * (c == 0 ? 1.0 : 1.0 + k));
    return 0;
}
