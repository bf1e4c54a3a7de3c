// Device rebuild of E and of K for a body in prescribed motion (moving.hip).
#pragma once

#include "kernels.h"

namespace ibpm {

constexpr int kEllE = 12;   // E row: the 4 x 3 (u) or 3 x 4 (v) faces nearest the point

// E rows (2 nb x kEllE, ascending face columns) for the points (xb, yb)
void launch_e_rows(hipStream_t s, GridView g, const double *xf, const double *yf, int nb, const double *xb,
                   const double *yb, int32_t *col, double *val);
// force rows of K: out_ptr null counts into len (2 nb), else fills at out_ptr
void launch_force_rows(hipStream_t s, GridView g, double dt, int nb, int pin, const int32_t *ecol, const double *eval,
                       const double *xb, const double *yb, double reach, int32_t *len, const int64_t *out_ptr,
                       int32_t *out_col, double *out_val);
// rows of the cells of the box [bi0, bi1] x [bj0, bj1] (row-major in the box)
void launch_box_rows(hipStream_t s, GridView g, const double *xf, const double *yf, double dt, int nb, int pin,
                     int bi0, int bi1, int bj0, int bj1, CSRView Kpp, const int32_t *ecol, const double *eval,
                     const double *xb, const double *yb, int32_t *len, const int64_t *out_ptr, int32_t *out_col,
                     double *out_val);
void launch_row_lengths(hipStream_t s, int nx, int n_cell, int nl, int bi0, int bi1, int bj0, int bj1, CSRView Kpp,
                        const int32_t *box_len, const int32_t *force_len, int32_t *len);
void launch_assemble(hipStream_t s, int nx, int n_cell, int nl, int bi0, int bi1, int bj0, int bj1, CSRView Kpp,
                     const int64_t *box_ptr, const int32_t *box_col, const double *box_val, const int64_t *force_ptr,
                     const int32_t *force_col, const double *force_val, const int32_t *ptr, int32_t *col,
                     double *val);
// diag[r] = k_rr and (wdinv non-null) wdinv[r] = omega / k_rr
void launch_diag_weights(hipStream_t s, CSRView K, double omega, double *diag, double *wdinv);
// exclusive scan of n int32 into out (n + 1 int64; out32, when non-null,
// gets the same as int32); tile_sums has scan_tiles_for(n) entries, total one
int scan_tiles_for(int n);
void launch_exclusive_scan(hipStream_t s, int n, const int32_t *in, int64_t *out, int32_t *out32,
                           int64_t *tile_sums, int64_t *total);
// q = q* - B^1 (G phi + E^T f~), E given as rows; only the faces of the
// cell box [bi0, bi1] x [bj0, bj1] meet a support
void launch_project_moving(hipStream_t s, GridView g, double dt, int nb, const int32_t *ecol, const double *eval,
                           int bi0, int bi1, int bj0, int bj1, const double *xf, const double *yf,
                           const double *xb, const double *yb, const double *qstar, const double *lam,
                           double *qout);

}  // namespace ibpm
