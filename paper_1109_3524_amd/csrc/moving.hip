// A body in prescribed motion (Sec. 6): the interpolation E and every row
// of K = Q^T B^1 Q that couples to the boundary forces are formed anew on
// the device for each set of point positions, and K is re-assembled in
// place as one CSR (Sec. 4: keep everything on the GPU).  With B^1 =
// dt Mf^{-1} diagonal, per face f with b_f = B^1_f:
//   K_fc[k, c] = sum_f E_kf b_f G_fc      (force rows, cell columns)
//   K_ff[k, l] = sum_f E_kf b_f E_lf      (force rows, force columns)
//   K_cf       = K_fc^T                   (the coupled cells' rows)
// and the pressure block G^T B^1 G does not change (its rows are kept).
// Every sum runs over faces in ascending index order, in the same
// expression (G b) e on both sides of the diagonal, so K stays bitwise
// symmetric; nothing is accumulated with atomics.
#include "moving.h"

#include <climits>

// no fused multiply-adds in this file: the force rows add products formed
// before the sum, the coupled cells' rows form them inside it, and both must
// round alike for K to stay symmetric bit for bit
#pragma clang fp contract(off)

namespace ibpm {

namespace {

// Eq. (6) for unit spacing, the inner branch including s = 0, zero from
// |s| = 1.5 on
__device__ __forceinline__ double phi_dev(double s) {
    s = fabs(s);
    if (s <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * (s * s))) / 3.0;
    if (s < 1.5) {
        const double t = 1.0 - s;
        return (5.0 - 3.0 * s - sqrt(1.0 - 3.0 * (t * t))) / 6.0;
    }
    return 0.0;
}

// index i with f[i] <= x < f[i+1] (f strictly increasing, n + 1 entries)
__device__ __forceinline__ int cell_index(const double *f, int n, double x) {
    int lo = 0, hi = n;   // f[lo] <= x < f[hi] kept
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (f[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// B^1 on a face (dt dy_j / Dx_i on u faces, dt dx_i / Dy_j on v faces)
__device__ __forceinline__ double b1_face(const GridView &g, double dt, int f) {
    const int nxm = g.nx - 1;
    if (f < g.n_u) {
        const int j = f / nxm, i = f - j * nxm + 1;
        return dt * g.dy[j] * g.iDx[i];
    }
    const int r = f - g.n_u, j = r / g.nx + 1, i = r - (j - 1) * g.nx;
    return dt * g.dx[i] * g.iDy[j];
}

// E rows (Eq. 7 in flux form, E = Ehat R^-1): row k (x force of point k)
// over the u faces (x_i, yc_j), row nb + k (y force) over the v faces
// (xc_i, y_j), the 4 x 3 (u) or 3 x 4 (v) faces nearest the point in
// ascending face order, weights zero outside the support
__global__ __launch_bounds__(kBlock) void k_e_rows(GridView g, const double *xf, const double *yf, int nb,
                                                   const double *xb, const double *yb, int32_t *col,
                                                   double *val) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= 2 * nb) return;
    const int k = t % nb;
    const bool vrow = t >= nb;
    const double X = xb[k], Y = yb[k];
    const int i0 = cell_index(xf, g.nx, X), j0 = cell_index(yf, g.ny, Y);
    const double hx = g.dx[i0], hy = g.dy[j0];
    int32_t *c = col + (size_t)t * kEllE;
    double *v = val + (size_t)t * kEllE;
    int s = 0;
    if (!vrow) {
        // u faces: x_i for i = i0-1 .. i0+2, cell centres yc_j for j = j0-1 .. j0+1
        for (int j = j0 - 1; j <= j0 + 1; ++j) {
            const double yc = 0.5 * (yf[j] + yf[j + 1]);
            const double wy = phi_dev((yc - Y) / hy) / hy;
            for (int i = i0 - 1; i <= i0 + 2; ++i) {
                const double wx = phi_dev((xf[i] - X) / hx) / hx;
                c[s] = j * (g.nx - 1) + (i - 1);
                v[s] = g.Dx[i] * wx * wy;
                ++s;
            }
        }
    } else {
        // v faces: cell centres xc_i for i = i0-1 .. i0+1, y_j for j = j0-1 .. j0+2
        for (int j = j0 - 1; j <= j0 + 2; ++j) {
            const double wy = phi_dev((yf[j] - Y) / hy) / hy;
            for (int i = i0 - 1; i <= i0 + 1; ++i) {
                const double xc = 0.5 * (xf[i] + xf[i + 1]);
                const double wx = phi_dev((xc - X) / hx) / hx;
                c[s] = g.n_u + (j - 1) * g.nx + i;
                v[s] = g.Dy[j] * wx * wy;
                ++s;
            }
        }
    }
}

// the cell pair of face f: (+1 cell, -1 cell) of G
__device__ __forceinline__ void face_cells(const GridView &g, int f, int &cp, int &cm) {
    const int nxm = g.nx - 1;
    if (f < g.n_u) {
        const int j = f / nxm, i = f - j * nxm + 1;
        cp = j * g.nx + i;
        cm = cp - 1;
    } else {
        const int r = f - g.n_u, j = r / g.nx + 1, i = r - (j - 1) * g.nx;
        cp = j * g.nx + i;
        cm = cp - g.nx;
    }
}

// Force row t of K (t < 2 nb): the cells it couples to (sorted, the pinned
// column left out) and then the force unknowns of the same component whose
// faces meet its own.  count: the row length into len[t]; fill: the row
// from out_ptr[t] on.
template <bool kFill>
__global__ __launch_bounds__(kBlock) void k_force_rows(GridView g, double dt, int nb, int pin, const int32_t *ecol,
                                                       const double *eval, const double *xb, const double *yb,
                                                       double reach, int32_t *len, const int64_t *out_ptr,
                                                       int32_t *out_col, double *out_val) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= 2 * nb) return;
    const int32_t *ck = ecol + (size_t)t * kEllE;
    const double *vk = eval + (size_t)t * kEllE;
    // (cell, term) pairs in slot order, then sorted by cell with a stable
    // insertion sort, so each cell's terms are summed in slot order
    int cc[2 * kEllE];
    double cv[2 * kEllE];
    int m = 0;
    for (int s = 0; s < kEllE; ++s) {
        const int f = ck[s];
        const double e = vk[s];
        if (e == 0.0) continue;
        const double b = b1_face(g, dt, f);
        int cp, cm;
        face_cells(g, f, cp, cm);
        cc[m] = cp;
        cv[m++] = (1.0 * b) * e;
        cc[m] = cm;
        cv[m++] = (-1.0 * b) * e;
    }
    for (int a = 1; a < m; ++a) {
        const int kc = cc[a];
        const double kv = cv[a];
        int b = a - 1;
        while (b >= 0 && cc[b] > kc) {
            cc[b + 1] = cc[b];
            cv[b + 1] = cv[b];
            --b;
        }
        cc[b + 1] = kc;
        cv[b + 1] = kv;
    }
    int64_t w = kFill ? out_ptr[t] : 0;
    int cnt = 0;
    for (int a = 0; a < m;) {
        const int c = cc[a];
        double sum = 0.0;
        while (a < m && cc[a] == c) sum += cv[a++];
        if (c == pin) continue;
        if (kFill) {
            out_col[w] = c;
            out_val[w] = sum;
            ++w;
        }
        ++cnt;
    }
    // force columns: the points of the same component near point k
    const int comp = t / nb, k = t % nb;
    const double X = xb[k], Y = yb[k];
    for (int l = 0; l < nb; ++l) {
        if (fabs(xb[l] - X) >= reach || fabs(yb[l] - Y) >= reach) continue;
        const int u = comp * nb + l;
        const int32_t *cl = ecol + (size_t)u * kEllE;
        const double *vl = eval + (size_t)u * kEllE;
        // both face lists ascend: walk them together
        double sum = 0.0;
        bool any = false;
        int p = 0, q = 0;
        while (p < kEllE && q < kEllE) {
            if (ck[p] < cl[q]) ++p;
            else if (ck[p] > cl[q]) ++q;
            else {
                if (vk[p] != 0.0 && vl[q] != 0.0) {
                    // b (e_k e_l): the same rounding for (k, l) and (l, k)
                    sum += b1_face(g, dt, ck[p]) * (vk[p] * vl[q]);
                    any = true;
                }
                ++p;
                ++q;
            }
        }
        if (!any) continue;
        if (kFill) {
            out_col[w] = g.n_cell + u;
            out_val[w] = sum;
            ++w;
        }
        ++cnt;
    }
    if (!kFill) len[t] = cnt;
}

// Row of a cell of the coupling box: its pressure entries (the fixed rows
// of G^T B^1 G) and then its coupling to every force unknown whose row
// meets one of its four faces
template <bool kFill>
__global__ __launch_bounds__(kBlock) void k_box_rows(GridView g, const double *xf, const double *yf, double dt,
                                                     int nb, int pin, int bi0, int bi1, int bj0, int bj1, CSRView Kpp,
                                                     const int32_t *ecol, const double *eval, const double *xb,
                                                     const double *yb, int32_t *len, const int64_t *out_ptr,
                                                     int32_t *out_col, double *out_val) {
    const int bw = bi1 - bi0 + 1;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= bw * (bj1 - bj0 + 1)) return;
    const int i = bi0 + t % bw, j = bj0 + t / bw;
    const int c = j * g.nx + i;
    int64_t w = kFill ? out_ptr[t] : 0;
    int cnt = 0;
    for (int p = Kpp.ptr[c]; p < Kpp.ptr[c + 1]; ++p) {
        if (kFill) {
            out_col[w] = Kpp.col[p];
            out_val[w] = Kpp.val[p];
            ++w;
        }
        ++cnt;
    }
    if (c != pin) {
        // the four faces of the cell in ascending index order with G_fc
        const int nxm = g.nx - 1;
        int fs[4];
        double gs[4];
        int nf = 0;
        if (i > 0) { fs[nf] = j * nxm + (i - 1); gs[nf++] = 1.0; }             // u(i, j): +1
        if (i < g.nx - 1) { fs[nf] = j * nxm + i; gs[nf++] = -1.0; }           // u(i+1, j): -1
        if (j > 0) { fs[nf] = g.n_u + (j - 1) * g.nx + i; gs[nf++] = 1.0; }    // v(i, j): +1
        if (j < g.ny - 1) { fs[nf] = g.n_u + j * g.nx + i; gs[nf++] = -1.0; }  // v(i, j+1): -1
        const double xc = 0.5 * (xf[i] + xf[i + 1]), yc = 0.5 * (yf[j] + yf[j + 1]);
        const double rx = 2.5 * g.dx[i], ry = 2.5 * g.dy[j];
        for (int u = 0; u < 2 * nb; ++u) {
            const int k = u % nb;
            // a support reaches 1.5 cells from its point, a face half a cell
            // from the cell centre: farther points cannot meet this cell
            if (fabs(xb[k] - xc) >= rx || fabs(yb[k] - yc) >= ry) continue;
            const int32_t *ck = ecol + (size_t)u * kEllE;
            const double *vk = eval + (size_t)u * kEllE;
            double sum = 0.0;
            bool any = false;
            for (int a = 0; a < nf; ++a)
                for (int s = 0; s < kEllE; ++s)
                    if (ck[s] == fs[a] && vk[s] != 0.0) {
                        sum += (gs[a] * b1_face(g, dt, fs[a])) * vk[s];
                        any = true;
                    }
            if (!any) continue;
            if (kFill) {
                out_col[w] = g.n_cell + u;
                out_val[w] = sum;
                ++w;
            }
            ++cnt;
        }
    }
    if (!kFill) len[t] = cnt;
}

// Row lengths of the whole K: a box cell's from its new row, a force row's
// likewise, every other cell's from the fixed pressure rows
__global__ __launch_bounds__(kBlock) void k_row_lengths(int nx, int n_cell, int nl, int bi0, int bi1, int bj0,
                                                        int bj1, CSRView Kpp, const int32_t *box_len,
                                                        const int32_t *force_len, int32_t *len) {
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= nl) return;
    if (r >= n_cell) {
        len[r] = force_len[r - n_cell];
        return;
    }
    const int j = r / nx, i = r - j * nx;
    if (i >= bi0 && i <= bi1 && j >= bj0 && j <= bj1)
        len[r] = box_len[(j - bj0) * (bi1 - bi0 + 1) + (i - bi0)];
    else
        len[r] = Kpp.ptr[r + 1] - Kpp.ptr[r];
}

// K's rows copied to their offsets (ptr from the scan of the lengths)
__global__ __launch_bounds__(kBlock) void k_assemble(int nx, int n_cell, int nl, int bi0, int bi1, int bj0, int bj1,
                                                     CSRView Kpp, const int64_t *box_ptr, const int32_t *box_col,
                                                     const double *box_val, const int64_t *force_ptr,
                                                     const int32_t *force_col, const double *force_val,
                                                     const int32_t *ptr, int32_t *col, double *val) {
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= nl) return;
    const int32_t *sc;
    const double *sv;
    int64_t p0, p1;
    if (r >= n_cell) {
        const int t = r - n_cell;
        p0 = force_ptr[t];
        p1 = force_ptr[t + 1];
        sc = force_col;
        sv = force_val;
    } else {
        const int j = r / nx, i = r - j * nx;
        if (i >= bi0 && i <= bi1 && j >= bj0 && j <= bj1) {
            const int t = (j - bj0) * (bi1 - bi0 + 1) + (i - bi0);
            p0 = box_ptr[t];
            p1 = box_ptr[t + 1];
            sc = box_col;
            sv = box_val;
        } else {
            p0 = Kpp.ptr[r];
            p1 = Kpp.ptr[r + 1];
            sc = Kpp.col;
            sv = Kpp.val;
        }
    }
    int32_t w = ptr[r];
    for (int64_t p = p0; p < p1; ++p, ++w) {
        col[w] = sc[p];
        val[w] = sv[p];
    }
}

// diagonal of K and the damped Jacobi weights omega / k_ii
__global__ __launch_bounds__(kBlock) void k_diag_weights(CSRView K, double omega, double *diag, double *wdinv) {
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= K.nrows) return;
    double d = 0.0;
    for (int p = K.ptr[r]; p < K.ptr[r + 1]; ++p)
        if (K.col[p] == r) d = K.val[p];
    diag[r] = d;
    if (wdinv) wdinv[r] = omega / d;
}

// Exclusive scan of n int32 values in three launches: block scans of
// kScanTile values, the scan of the block totals in one block, and the
// totals added back.  out has n + 1 entries (out[n] = the sum).
constexpr int kScanTile = 1024;

__global__ __launch_bounds__(kBlock) void k_scan_tiles(int n, const int32_t *in, int64_t *out, int64_t *tile_sums) {
    __shared__ int64_t sh[kScanTile];
    const int base = blockIdx.x * kScanTile;
    for (int k = threadIdx.x; k < kScanTile; k += kBlock) sh[k] = base + k < n ? (int64_t)in[base + k] : 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int k = 0; k < kScanTile; ++k) {
            const int64_t v = sh[k];
            sh[k] = acc;
            acc += v;
        }
        tile_sums[blockIdx.x] = acc;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kScanTile; k += kBlock)
        if (base + k < n) out[base + k] = sh[k];
}

__global__ __launch_bounds__(kBlock) void k_scan_sums(int ntiles, int64_t *tile_sums, int64_t *total) {
    if (threadIdx.x != 0) return;
    int64_t acc = 0;
    for (int k = 0; k < ntiles; ++k) {
        const int64_t v = tile_sums[k];
        tile_sums[k] = acc;
        acc += v;
    }
    *total = acc;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(int n, int64_t *out, const int64_t *tile_sums,
                                                     const int64_t *total, int32_t *out32) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k < n) {
        out[k] += tile_sums[k / kScanTile];
        if (out32) out32[k] = (int32_t)out[k];
    }
    if (k == n) {
        out[n] = *total;
        if (out32) out32[n] = (int32_t)*total;
    }
}

// q = q* - B^1 (G phi + E^T f~): the gradient from the two cells of the
// face, the spreading as a gather over the points whose rows reach the
// face (only faces of the box [bi0, bi1] x [bj0, bj1] can be reached; a
// point farther than two cell widths from the face cannot reach it)
__global__ __launch_bounds__(kBlock) void k_project_moving(GridView g, double dt, int nb, const int32_t *ecol,
                                                           const double *eval, int bi0, int bi1, int bj0, int bj1,
                                                           const double *xf, const double *yf, const double *xb,
                                                           const double *yb, const double *qstar,
                                                           const double *lam, double *qout) {
    const int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= g.n_q) return;
    int cp, cm;
    face_cells(g, f, cp, cm);
    double w = lam[cp] - lam[cm];
    const bool vface = f >= g.n_u;
    int i, j;
    double xfc, yfc;
    if (!vface) {
        j = f / (g.nx - 1);
        i = f - j * (g.nx - 1) + 1;
        xfc = xf[i];
        yfc = 0.5 * (yf[j] + yf[j + 1]);
    } else {
        const int r = f - g.n_u;
        j = r / g.nx + 1;
        i = r - (j - 1) * g.nx;
        xfc = 0.5 * (xf[i] + xf[i + 1]);
        yfc = yf[j];
    }
    const bool in_box = vface ? (i >= bi0 && i <= bi1 && j >= bj0 && j <= bj1 + 1)
                              : (i >= bi0 && i <= bi1 + 1 && j >= bj0 && j <= bj1);
    if (in_box) {
        const int comp = vface ? 1 : 0;
        const int ic = i < g.nx ? i : g.nx - 1, jc = j < g.ny ? j : g.ny - 1;
        const double rx = 2.0 * g.dx[ic], ry = 2.0 * g.dy[jc];
        for (int k = 0; k < nb; ++k) {
            if (fabs(xb[k] - xfc) >= rx || fabs(yb[k] - yfc) >= ry) continue;
            const int u = comp * nb + k;
            const int32_t *ck = ecol + (size_t)u * kEllE;
            const double *vk = eval + (size_t)u * kEllE;
            for (int s = 0; s < kEllE; ++s)
                if (ck[s] == f) w += vk[s] * lam[g.n_cell + u];
        }
    }
    qout[f] = qstar[f] - b1_face(g, dt, f) * w;
}

}  // namespace

#define LAUNCHM(kernel, grid, ...) hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, __VA_ARGS__)
inline int mblocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

void launch_e_rows(hipStream_t s, GridView g, const double *xf, const double *yf, int nb, const double *xb,
                   const double *yb, int32_t *col, double *val) {
    if (nb > 0) LAUNCHM(k_e_rows, mblocks(2 * nb), g, xf, yf, nb, xb, yb, col, val);
}

void launch_force_rows(hipStream_t s, GridView g, double dt, int nb, int pin, const int32_t *ecol, const double *eval,
                       const double *xb, const double *yb, double reach, int32_t *len, const int64_t *out_ptr,
                       int32_t *out_col, double *out_val) {
    if (nb == 0) return;
    if (!out_ptr)
        LAUNCHM(k_force_rows<false>, mblocks(2 * nb), g, dt, nb, pin, ecol, eval, xb, yb, reach, len, out_ptr,
                out_col, out_val);
    else
        LAUNCHM(k_force_rows<true>, mblocks(2 * nb), g, dt, nb, pin, ecol, eval, xb, yb, reach, len, out_ptr,
                out_col, out_val);
}

void launch_box_rows(hipStream_t s, GridView g, const double *xf, const double *yf, double dt, int nb, int pin,
                     int bi0, int bi1, int bj0, int bj1, CSRView Kpp, const int32_t *ecol, const double *eval,
                     const double *xb, const double *yb, int32_t *len, const int64_t *out_ptr, int32_t *out_col,
                     double *out_val) {
    const int64_t nbox = (int64_t)(bi1 - bi0 + 1) * (bj1 - bj0 + 1);
    if (nbox <= 0) return;
    if (!out_ptr)
        LAUNCHM(k_box_rows<false>, mblocks(nbox), g, xf, yf, dt, nb, pin, bi0, bi1, bj0, bj1, Kpp, ecol, eval, xb,
                yb, len, out_ptr, out_col, out_val);
    else
        LAUNCHM(k_box_rows<true>, mblocks(nbox), g, xf, yf, dt, nb, pin, bi0, bi1, bj0, bj1, Kpp, ecol, eval, xb,
                yb, len, out_ptr, out_col, out_val);
}

void launch_row_lengths(hipStream_t s, int nx, int n_cell, int nl, int bi0, int bi1, int bj0, int bj1, CSRView Kpp,
                        const int32_t *box_len, const int32_t *force_len, int32_t *len) {
    LAUNCHM(k_row_lengths, mblocks(nl), nx, n_cell, nl, bi0, bi1, bj0, bj1, Kpp, box_len, force_len, len);
}

void launch_assemble(hipStream_t s, int nx, int n_cell, int nl, int bi0, int bi1, int bj0, int bj1, CSRView Kpp,
                     const int64_t *box_ptr, const int32_t *box_col, const double *box_val, const int64_t *force_ptr,
                     const int32_t *force_col, const double *force_val, const int32_t *ptr, int32_t *col,
                     double *val) {
    LAUNCHM(k_assemble, mblocks(nl), nx, n_cell, nl, bi0, bi1, bj0, bj1, Kpp, box_ptr, box_col, box_val, force_ptr,
            force_col, force_val, ptr, col, val);
}

void launch_diag_weights(hipStream_t s, CSRView K, double omega, double *diag, double *wdinv) {
    LAUNCHM(k_diag_weights, mblocks(K.nrows), K, omega, diag, wdinv);
}

int scan_tiles_for(int n) { return (n + kScanTile - 1) / kScanTile; }

void launch_exclusive_scan(hipStream_t s, int n, const int32_t *in, int64_t *out, int32_t *out32,
                           int64_t *tile_sums, int64_t *total) {
    const int nt = scan_tiles_for(n);
    if (nt > 0) LAUNCHM(k_scan_tiles, nt, n, in, out, tile_sums);
    LAUNCHM(k_scan_sums, 1, nt, tile_sums, total);
    LAUNCHM(k_scan_add, mblocks(n + 1), n, out, tile_sums, total, out32);
}

void launch_project_moving(hipStream_t s, GridView g, double dt, int nb, const int32_t *ecol, const double *eval,
                           int bi0, int bi1, int bj0, int bj1, const double *xf, const double *yf,
                           const double *xb, const double *yb, const double *qstar, const double *lam,
                           double *qout) {
    LAUNCHM(k_project_moving, mblocks(g.n_q), g, dt, nb, ecol, eval, bi0, bi1, bj0, bj1, xf, yf, xb, yb, qstar,
            lam, qout);
}

}  // namespace ibpm
