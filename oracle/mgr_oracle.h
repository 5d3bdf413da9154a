/*
 * mgr_oracle.h - plain FP64 CPU oracle for multigrid hierarchical data
 * refactoring (Chen et al., "Accelerating Multigrid-based Hierarchical
 * Scientific Data Refactoring on GPUs", arXiv 2007.04457).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU product path
 * never links, loads or calls it, and it shares no code with the GPU path.
 *
 * Conventions (all functions):
 *   u       : C-order array of prod(shape) doubles, transformed in place.
 *   ndim    : 1..4.
 *   shape   : shape[d] = 2^k_d + 1 with k_d >= 1.
 *   coords  : NULL, or coords[d] = NULL, means uniform node positions x = i;
 *             otherwise coords[d] points to shape[d] strictly increasing
 *             doubles (nonuniform structured grid, Sec. II-A).
 *   nlevels : number of decomposition steps L, 0..min_d k_d, or -1 for the
 *             full decomposition (L = min_d k_d - 1, coarsest min-dim 3).
 * Return value: 0 on success, a positive error code otherwise (1 argument,
 * 2 shape, 3 levels, 4 coordinates, 6 allocation).
 */
#ifndef MGR_ORACLE_H
#define MGR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int oracle_max_levels(int ndim, const int64_t* shape);

/* Threads for the loops over independent fibres and nodes (the library is
 * built with OpenMP); results are bitwise independent of the count.
 * Default 1.  Returns the previous value. */
int oracle_set_threads(int n);

/* Decomposition, Sec. II-A, Eq. (1)-(2): finest to coarsest level. */
int oracle_decompose(double* u, int ndim, const int64_t* shape,
                     const double* const* coords, int nlevels);
/* Recomposition: the exact inverse, coarsest to finest level (Sec. II-A). */
int oracle_recompose(double* u, int ndim, const int64_t* shape,
                     const double* const* coords, int nlevels);
/* Transpose of the decomposition map under the Euclidean inner product on
 * the in-place array (derived from Eq. (1)-(2); not in the paper). */
int oracle_decompose_adjoint(double* g, int ndim, const int64_t* shape,
                             const double* const* coords, int nlevels);

/* Transpose of the recomposition (= inverse transpose of the
 * decomposition) under the same inner product; fine to coarse. */
int oracle_recompose_adjoint(double* g, int ndim, const int64_t* shape,
                             const double* const* coords, int nlevels);

/* Per-stage entry points for one level step k (stride 2^k), Sec. II-A.
 * coefficients: step "compute coefficients" only, in place on u.
 * load_vector : f = R M vec(C) for the level step k, written packed to f
 *               (shape (m_d+1)/2 per dim, m_d the level-grid size); u is
 *               read only (its fine nodes must already hold coefficients).
 * correction  : solves M_{l-1} z = f in place on the packed f.            */
int oracle_coefficients_level(double* u, int ndim, const int64_t* shape,
                              const double* const* coords, int k);
int oracle_load_vector_level(const double* u, double* f, int ndim,
                             const int64_t* shape, const double* const* coords,
                             int k);
int oracle_correction_level(double* f, int ndim, const int64_t* shape,
                            const double* const* coords, int k);

/* Class id per node: 0 = coarsest nodal values, L = finest coefficients. */
int oracle_class_map(int ndim, const int64_t* shape, int nlevels,
                     uint8_t* out);

/* Quantisation of a refactored array (the quantisation stage of the lossy
 * compression workflow, Sec. V): per-class uniform scalar quantiser, code
 * q = round-half-even(y / b_c) in the data's precision (dtype 0 = float,
 * 1 = double; y is float* or double*), b_c = bins[class] rounded to that
 * precision, clamped to +-(2^31 - 1) (NaN to 0); *nclamped (may be NULL)
 * receives the number clamped.  packed = 0: y is in the in-place layout;
 * packed = 1: the class-packed layout (class c is the c-th segment).
 * bins: host, nlevels + 1 positive finite widths (nlevels -1 = full). */
int oracle_quantize(const void* y, int32_t* q, int dtype, int ndim, const int64_t* shape, int nlevels,
                    int packed, const double* bins, int64_t* nclamped);
/* y = q * b_c in the data's precision, same conventions. */
int oracle_dequantize(const int32_t* q, void* y, int dtype, int ndim, const int64_t* shape, int nlevels,
                      int packed, const double* bins);
/* Bin widths (nlevels + 1) for a bound tol on the pointwise error of the
 * recomposed field (exact arithmetic); see mgr_oracle.c. */
int oracle_quant_bins(int ndim, int nlevels, double tol, double* bins);

#ifdef __cplusplus
}
#endif
#endif
