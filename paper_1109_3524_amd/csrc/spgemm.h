// Device sparse products for the B^N operators (N > 1): launchers of the
// row-merge product kernels (spgemm.hip).
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
// y = base + alpha A x (base may be null)
void launch_csr_gemv(hipStream_t s, CSRView A, const double *x, double alpha, const double *base, double *y);

}  // namespace ibpm
