// Device sparse products for the B^N operators (N > 1) and for the
// smoothed-aggregation hierarchy of a moving body: launchers of the
// row-merge product kernels and their helpers (spgemm.hip).
#pragma once

#include "kernels.h"

namespace ibpm {

constexpr int kMergeMax = 32;   // longest left row a product kernel merges

// cnt[i] = distinct columns of row i of A[rows] * B, where row i of A[rows] is
// A's row rows[i] (or r0 + i when rows is null); *err = 1 when a left row
// has more than kMergeMax entries
void launch_spgemm_count(hipStream_t s, int nrows, int r0, const int32_t *rows, CSRView A, CSRView B,
                         int32_t *cnt, int *err);
// the same rows of the product, written from out_ptr[i] on (sorted columns)
void launch_spgemm_fill(hipStream_t s, int nrows, int r0, const int32_t *rows, CSRView A, CSRView B,
                        const int64_t *out_ptr, int32_t *out_col, double *out_val);
// C = diag(d) (I + X + Y), square n x n, X and Y sorted CSR
void launch_diag_sum_count(hipStream_t s, int n, CSRView X, CSRView Y, int32_t *cnt);
void launch_diag_sum_fill(hipStream_t s, int n, const double *d, CSRView X, CSRView Y, const int64_t *out_ptr,
                          int32_t *out_col, double *out_val);
// chunks of kMergeMax entries per row: cnt[i] = chunks of row i; from their
// offsets off (n + 1, exclusive scan of cnt) the chunk row starts cptr
// (off[n] + 1 entries) and the chunk-sum matrix (columns scol, unit values)
void launch_chunk_count(hipStream_t s, int n, const int32_t *ptr, int32_t *cnt);
void launch_chunk_fill(hipStream_t s, int n, const int32_t *ptr, const int32_t *off, int32_t *cptr, int32_t *scol,
                       double *sval);
// transpose: entries per column (cnt zeroed by the caller), then the fill
// from the column offsets tptr (cursor zeroed), then each row sorted
void launch_col_count(hipStream_t s, int64_t nnz, const int32_t *col, int32_t *cnt);
void launch_transpose_fill(hipStream_t s, CSRView A, const int32_t *tptr, int32_t *cursor, int32_t *tcol,
                           double *tval);
void launch_sort_rows(hipStream_t s, int n, const int32_t *ptr, int32_t *col, double *val);
// the tentative prolongator T of an aggregation (n x nagg, n + 1 row starts)
void launch_tentative(hipStream_t s, int n, const int32_t *agg, int32_t *ptr, int32_t *col, double *val);
// P = T - w D^-1 (A T) in place over the values of A T; *err = 1 when a
// diagonal entry is not positive
void launch_smooth_prolongator(hipStream_t s, int n, const int32_t *ptr, const int32_t *col, double *val,
                               const int32_t *agg, const double *diag, double w, int *err);
// y = a x + b y
void launch_axpby(hipStream_t s, int n, double a, const double *x, double b, double *y);
// y = base + alpha A x (base may be null)
void launch_csr_gemv(hipStream_t s, CSRView A, const double *x, double alpha, const double *base, double *y);

}  // namespace ibpm
