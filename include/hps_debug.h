/*
 * hps_debug.h -- test hooks of libhps.so (not needed by applications).
 *
 * They expose single kernels and the operators a build stores, so tests can
 * check each stage of Algorithm 1 (leaf operators of Sec. 3, merge operators
 * of Sec. 4) separately.  Same error conventions as hps.h.
 */
#ifndef HPS_DEBUG_H
#define HPS_DEBUG_H

#include <stdint.h>

#include "hps.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C = alpha * A * B on the grouped FP64 MFMA GEMM kernel.  Device arrays,
 * column-major: A (M x K, lda), B (K x N, ldb), C (M x N, ldc). */
int hps_debug_gemm(int M, int N, int K, double alpha, const double *A, int lda,
                   const double *B, int ldb, double *C, int ldc, void *stream);

/* The same on one tile variant of the kernel (0: 64 x 64, 1: 128 x 64,
 * 2: 64 x 128, 3: 128 x 128, 4: 32 x 32, 5: 64 x 32, 6: 32 x 64 output tiles
 * with K chunks of 16; 7: 64 x 64 with K chunks of 8); every variant must
 * give bitwise the same C. */
int hps_debug_gemm_variant(int variant, int M, int N, int K, double alpha, const double *A,
                           int lda, const double *B, int ldb, double *C, int ldc, void *stream);

/* X_i = inverse(A_i) for `batch` column-major n x n matrices stored one after
 * another (device), by the Gauss-Jordan kernel the build uses for an
 * interface block of size n (register-resident for n <= 196, blocked above).
 * Returns HPS_ESINGULAR / HPS_ENONFINITE like hps_build. */
int hps_debug_invert(int n, int batch, const double *A, double *X, void *stream);

/* Bytes of solve work memory (work vectors and split-K partials) that
 * nrhs right-hand sides take on this handle; 0 for bad arguments. */
size_t hps_debug_solve_work_bytes(const hps_handle *h, int nrhs);

/* Number of boxes of a built handle and, per box (pre-order numbering,
 * parents before children): [is_leaf, leaf index or -1, parent, alpha, beta,
 * n_fin, n_nat, m] into host int32 out[n_boxes][8]. */
int hps_debug_boxes(const hps_handle *h, int *n_boxes, int32_t *out);

/* Global Gauss node ids of a box's boundary in its final order (n_fin
 * entries), its natural order (n_nat) or its interior edge (m), host out. */
int hps_debug_box_nodes(const hps_handle *h, int box, int which, int64_t *out);

/* Copy a stored operator to host memory (column-major):
 * which = 0 T (n_fin x n_fin), 1 X (m x m), 2 S (m x n_nat; leaves:
 * S_ci, (p-2)^2 x 4q), 3 F (leaves, (p-2)^2 x (p-2)^2), 4 H (leaves,
 * 4q x (p-2)^2).  Returns the element count through *count. */
int hps_debug_box_op(const hps_handle *h, int box, int which, double *out, int64_t *count);

/* GEMM tile variant the tuner chose for each GEMM step of the build
 * program, in program order, into host out[max_n]; *count receives the
 * number of GEMM steps. */
int hps_debug_gemm_choices(const hps_handle *h, int *out, int max_n, int *count);

/* Per-launch timing: when enabled, every kernel launch step of builds and
 * solves on this handle is bracketed by HIP events on the caller's stream.
 * hps_debug_profile_read waits for the device, returns (kind, ms, work)
 * triples of the steps recorded since the last read (kind = 16 * step type +
 * variant, the variant being the size class of an interface Gauss-Jordan
 * (GEMM: its tile variant) and 0 otherwise; types 0 GEMM,
 * 1 leaf Gauss-Jordan, 2 interface Gauss-Jordan,
 * 3 interface difference, 4 panel, 5 column permutation, 6 solve apply) and
 * clears them.  work is the launch's algorithmic flop count (GEMM,
 * Gauss-Jordan, panel) or the number of operator elements it applies to each
 * right-hand side (apply); `work` may be NULL.  Host arrays of max_n entries;
 * *count receives the number recorded. */
int hps_debug_profile(hps_handle *h, int enable);
int hps_debug_profile_read(hps_handle *h, int *kinds, double *ms, double *work, int max_n,
                           int *count);

#ifdef __cplusplus
}
#endif

#endif /* HPS_DEBUG_H */
