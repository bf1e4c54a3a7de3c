// Sparse matrix products on the device, for the operators of B^N with
// N > 1 (Sec. 2, text after Eq. 11): B^N = dt Mf^{-1} sum_{k<N} S^k with
// S = (nu/2) L B^1, and the Poisson operator K = Q^T B^N Q formed slice by
// slice so that no full-size intermediate is ever held (the memory-bounded
// triple product of Sec. 4); and for the smoothed-aggregation hierarchy
// formed anew for a moving body (Sec. 4): P = (I - w D^-1 A) T, its
// transpose, and the Galerkin product P^T A P.
//
// Every product row is a k-way merge: the rows of the right operand named by
// the columns of one left row are walked together in column order, so the
// output row comes out sorted with each column once, and each output entry
// is summed in the left row's column order -- deterministic, no atomics and
// no hashing.  One thread per output row; the left rows are short (at most
// kMergeMax entries: 5 for S, 13 for S^2, 19 for B^3, <= 24 for a row of
// Q^T), the right rows a few tens.  This is set-up work, not on the time
// step.
#include "spgemm.h"

#include <climits>

namespace ibpm {

namespace {

// Products of rows[0..nrows) of A (row i of the product is A's row rows[i],
// or r0 + i when rows is null) with B: the number of distinct columns of
// each product row into cnt[i]; *err = 1 if a left row is longer than
// kMergeMax.
__global__ __launch_bounds__(kBlock) void k_spgemm_count(int nrows, int r0, const int32_t *rows, CSRView A,
                                                         CSRView B, int32_t *cnt, int *err) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= nrows) return;
    const int row = rows ? rows[i] : r0 + i;
    const int a0 = A.ptr[row], m = A.ptr[row + 1] - a0;
    if (m > kMergeMax) {
        *err = 1;
        cnt[i] = 0;
        return;
    }
    int pos[kMergeMax], end[kMergeMax];
    for (int t = 0; t < m; ++t) {
        const int k = A.col[a0 + t];
        pos[t] = B.ptr[k];
        end[t] = B.ptr[k + 1];
    }
    int count = 0;
    for (;;) {
        int jmin = INT_MAX;
        for (int t = 0; t < m; ++t)
            if (pos[t] < end[t]) jmin = min(jmin, B.col[pos[t]]);
        if (jmin == INT_MAX) break;
        ++count;
        for (int t = 0; t < m; ++t)
            if (pos[t] < end[t] && B.col[pos[t]] == jmin) ++pos[t];
    }
    cnt[i] = count;
}

// The product rows themselves, written at out_ptr[i] (slice-local offsets)
__global__ __launch_bounds__(kBlock) void k_spgemm_fill(int nrows, int r0, const int32_t *rows, CSRView A,
                                                        CSRView B, const int64_t *out_ptr, int32_t *out_col,
                                                        double *out_val) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= nrows) return;
    const int row = rows ? rows[i] : r0 + i;
    const int a0 = A.ptr[row], m = A.ptr[row + 1] - a0;
    if (m > kMergeMax) return;
    int pos[kMergeMax], end[kMergeMax];
    for (int t = 0; t < m; ++t) {
        const int k = A.col[a0 + t];
        pos[t] = B.ptr[k];
        end[t] = B.ptr[k + 1];
    }
    int64_t w = out_ptr[i];
    for (;;) {
        int jmin = INT_MAX;
        for (int t = 0; t < m; ++t)
            if (pos[t] < end[t]) jmin = min(jmin, B.col[pos[t]]);
        if (jmin == INT_MAX) break;
        double sum = 0.0;
        for (int t = 0; t < m; ++t)
            if (pos[t] < end[t] && B.col[pos[t]] == jmin) {
                sum += A.val[a0 + t] * B.val[pos[t]];
                ++pos[t];
            }
        out_col[w] = jmin;
        out_val[w] = sum;
        ++w;
    }
}

// Row i of C = D (I + X + Y) with D diagonal: the merge of row i of X and
// of Y with the unit diagonal, each entry d_i ((delta_ij + x_ij) + y_ij)
__global__ __launch_bounds__(kBlock) void k_diag_sum_count(int n, CSRView X, CSRView Y, int32_t *cnt) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int px = X.ptr[i], ex = X.ptr[i + 1], py = Y.ptr[i], ey = Y.ptr[i + 1];
    bool diag = true;
    int count = 0;
    for (;;) {
        int j = INT_MAX;
        if (px < ex) j = min(j, X.col[px]);
        if (py < ey) j = min(j, Y.col[py]);
        if (diag) j = min(j, i);
        if (j == INT_MAX) break;
        ++count;
        if (px < ex && X.col[px] == j) ++px;
        if (py < ey && Y.col[py] == j) ++py;
        if (diag && j == i) diag = false;
    }
    cnt[i] = count;
}

__global__ __launch_bounds__(kBlock) void k_diag_sum_fill(int n, const double *d, CSRView X, CSRView Y,
                                                          const int64_t *out_ptr, int32_t *out_col,
                                                          double *out_val) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int px = X.ptr[i], ex = X.ptr[i + 1], py = Y.ptr[i], ey = Y.ptr[i + 1];
    bool diag = true;
    int64_t w = out_ptr[i];
    for (;;) {
        int j = INT_MAX;
        if (px < ex) j = min(j, X.col[px]);
        if (py < ey) j = min(j, Y.col[py]);
        if (diag) j = min(j, i);
        if (j == INT_MAX) break;
        double v = 0.0;
        if (diag && j == i) {
            v = 1.0;
            diag = false;
        }
        if (px < ex && X.col[px] == j) v += X.val[px++];
        if (py < ey && Y.col[py] == j) v += Y.val[py++];
        out_col[w] = j;
        out_val[w] = d[i] * v;
        ++w;
    }
}

// y = base + alpha A x (base may be null), one thread per row, the row
// summed in column order
__global__ __launch_bounds__(kBlock) void k_csr_gemv(CSRView A, const double *x, double alpha, const double *base,
                                                     double *y) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= A.nrows) return;
    double s = 0.0;
    for (int p = A.ptr[i]; p < A.ptr[i + 1]; ++p) s += A.val[p] * x[A.col[p]];
    y[i] = base ? base[i] + alpha * s : alpha * s;
}

// Left rows longer than kMergeMax are taken in chunks of kMergeMax entries:
// chunk k of row i is a row of its own (A' shares A's columns and values),
// and the chunk products are summed by a second product whose left rows
// hold a unit entry per chunk.  cnt[i] = the chunks of row i.
__global__ __launch_bounds__(kBlock) void k_chunk_count(int n, const int32_t *ptr, int32_t *cnt) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) cnt[i] = (ptr[i + 1] - ptr[i] + kMergeMax - 1) / kMergeMax;
}

// A'.ptr (chunk starts, then nnz(A)) and the chunk-sum matrix S (row i:
// unit entries at the chunks of row i), from the chunk offsets off (n + 1)
__global__ __launch_bounds__(kBlock) void k_chunk_fill(int n, const int32_t *ptr, const int32_t *off,
                                                       int32_t *cptr, int32_t *scol, double *sval) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i > n) return;
    if (i == n) {
        cptr[off[n]] = ptr[n];
        return;
    }
    for (int k = off[i]; k < off[i + 1]; ++k) {
        cptr[k] = ptr[i] + (k - off[i]) * kMergeMax;
        scol[k] = k;
        sval[k] = 1.0;
    }
}

// Transpose: entries per column (atomic counts; the order of the fill below
// is then fixed by sorting each row on its column)
__global__ __launch_bounds__(kBlock) void k_col_count(int64_t nnz, const int32_t *col, int32_t *cnt) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < nnz) atomicAdd(&cnt[col[p]], 1);
}

__global__ __launch_bounds__(kBlock) void k_transpose_fill(CSRView A, const int32_t *tptr, int32_t *cursor,
                                                           int32_t *tcol, double *tval) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= A.nrows) return;
    for (int p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
        const int j = A.col[p];
        const int w = tptr[j] + atomicAdd(&cursor[j], 1);
        tcol[w] = i;
        tval[w] = A.val[p];
    }
}

// each row's entries sorted on their (distinct) columns
__global__ __launch_bounds__(kBlock) void k_sort_rows(int n, const int32_t *ptr, int32_t *col, double *val) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int p0 = ptr[i], p1 = ptr[i + 1];
    for (int a = p0 + 1; a < p1; ++a) {
        const int kc = col[a];
        const double kv = val[a];
        int b = a - 1;
        while (b >= p0 && col[b] > kc) {
            col[b + 1] = col[b];
            val[b + 1] = val[b];
            --b;
        }
        col[b + 1] = kc;
        val[b + 1] = kv;
    }
}

// T of the aggregation as CSR: row i holds a unit entry at aggregate agg[i]
__global__ __launch_bounds__(kBlock) void k_tentative(int n, const int32_t *agg, int32_t *ptr, int32_t *col,
                                                      double *val) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i > n) return;
    ptr[i] = i;
    if (i < n) {
        col[i] = agg[i];
        val[i] = 1.0;
    }
}

// P = T - w D^{-1} (A T) in place on the pattern of A T (which holds
// agg[i] in row i, from the diagonal of A); *err = 1 for a non-positive
// diagonal
__global__ __launch_bounds__(kBlock) void k_smooth_prolongator(int n, const int32_t *ptr, const int32_t *col,
                                                               double *val, const int32_t *agg, const double *diag,
                                                               double w, int *err) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double d = diag[i];
    if (!(d > 0)) *err = 1;
    const double dinv = 1.0 / d;
    for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
        const double t = col[p] == agg[i] ? 1.0 : 0.0;
        val[p] = t - w * (dinv * val[p]);
    }
}

// y = a x + b y
__global__ __launch_bounds__(kBlock) void k_axpby(int n, double a, const double *x, double b, double *y) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = a * x[i] + b * y[i];
}

int blocks_for(int n) { return (n + kBlock - 1) / kBlock; }

}  // namespace

#define LAUNCHS(kernel, grid, ...) hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, __VA_ARGS__)

void launch_spgemm_count(hipStream_t s, int nrows, int r0, const int32_t *rows, CSRView A, CSRView B,
                         int32_t *cnt, int *err) {
    if (nrows > 0) LAUNCHS(k_spgemm_count, blocks_for(nrows), nrows, r0, rows, A, B, cnt, err);
}

void launch_spgemm_fill(hipStream_t s, int nrows, int r0, const int32_t *rows, CSRView A, CSRView B,
                        const int64_t *out_ptr, int32_t *out_col, double *out_val) {
    if (nrows > 0) LAUNCHS(k_spgemm_fill, blocks_for(nrows), nrows, r0, rows, A, B, out_ptr, out_col, out_val);
}

void launch_diag_sum_count(hipStream_t s, int n, CSRView X, CSRView Y, int32_t *cnt) {
    if (n > 0) LAUNCHS(k_diag_sum_count, blocks_for(n), n, X, Y, cnt);
}

void launch_diag_sum_fill(hipStream_t s, int n, const double *d, CSRView X, CSRView Y, const int64_t *out_ptr,
                          int32_t *out_col, double *out_val) {
    if (n > 0) LAUNCHS(k_diag_sum_fill, blocks_for(n), n, d, X, Y, out_ptr, out_col, out_val);
}

void launch_chunk_count(hipStream_t s, int n, const int32_t *ptr, int32_t *cnt) {
    if (n > 0) LAUNCHS(k_chunk_count, blocks_for(n), n, ptr, cnt);
}

void launch_chunk_fill(hipStream_t s, int n, const int32_t *ptr, const int32_t *off, int32_t *cptr, int32_t *scol,
                       double *sval) {
    LAUNCHS(k_chunk_fill, blocks_for(n + 1), n, ptr, off, cptr, scol, sval);
}

void launch_col_count(hipStream_t s, int64_t nnz, const int32_t *col, int32_t *cnt) {
    if (nnz > 0) LAUNCHS(k_col_count, (int)((nnz + kBlock - 1) / kBlock), nnz, col, cnt);
}

void launch_transpose_fill(hipStream_t s, CSRView A, const int32_t *tptr, int32_t *cursor, int32_t *tcol,
                           double *tval) {
    if (A.nrows > 0) LAUNCHS(k_transpose_fill, blocks_for(A.nrows), A, tptr, cursor, tcol, tval);
}

void launch_sort_rows(hipStream_t s, int n, const int32_t *ptr, int32_t *col, double *val) {
    if (n > 0) LAUNCHS(k_sort_rows, blocks_for(n), n, ptr, col, val);
}

void launch_tentative(hipStream_t s, int n, const int32_t *agg, int32_t *ptr, int32_t *col, double *val) {
    LAUNCHS(k_tentative, blocks_for(n + 1), n, agg, ptr, col, val);
}

void launch_smooth_prolongator(hipStream_t s, int n, const int32_t *ptr, const int32_t *col, double *val,
                               const int32_t *agg, const double *diag, double w, int *err) {
    if (n > 0) LAUNCHS(k_smooth_prolongator, blocks_for(n), n, ptr, col, val, agg, diag, w, err);
}

void launch_axpby(hipStream_t s, int n, double a, const double *x, double b, double *y) {
    if (n > 0) LAUNCHS(k_axpby, blocks_for(n), n, a, x, b, y);
}

void launch_csr_gemv(hipStream_t s, CSRView A, const double *x, double alpha, const double *base, double *y) {
    if (A.nrows > 0) LAUNCHS(k_csr_gemv, blocks_for(A.nrows), A, x, alpha, base, y);
}

}  // namespace ibpm
