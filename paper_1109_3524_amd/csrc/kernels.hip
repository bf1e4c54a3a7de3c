// HIP kernels for gfx950: the per-step stages of the immersed-boundary
// projection method and the pieces of the Krylov / AMG solvers.
//
// Every kernel is HBM-bound (sparse, stencil, vector).  Work is one row per
// thread in 256-thread blocks; a block handles a contiguous range of 256-row
// tiles and the block index is remapped so that each of the 8 XCDs owns a
// contiguous eighth of the rows (neighbour rows of a stencil then hit the
// same L2).  Reductions are deterministic: a fixed-order LDS tree per block,
// per-block partials, and the last block to finish (an integer atomic
// counter decides which) sums the partials in a fixed order.  No floating-
// point atomics are used anywhere.
//
// The solver kernels are templates on the vector precision T (double, or
// float for the mixed-precision inner solve); dot products always
// accumulate in double.
#include "kernels.h"

namespace ibpm {

namespace {

__device__ __forceinline__ int remap_block(int b, int G) {
    int per = G >> 3;
    if (b >= 8 * per) return b;
    return (b & 7) * per + (b >> 3);
}

struct Tiles {
    int t0, t1;
};

__device__ __forceinline__ Tiles my_tiles(int n) {
    int ntiles = (n + kBlock - 1) / kBlock;
    int G = gridDim.x;
    int l = remap_block(blockIdx.x, G);
    int T = (ntiles + G - 1) / G;
    int t0 = l * T;
    int t1 = min(t0 + T, ntiles);
    return {t0, t1};
}

inline int grid_for(int n) {
    int ntiles = (n + kBlock - 1) / kBlock;
    if (ntiles < 1) ntiles = 1;
    return ntiles < kMaxParts ? ntiles : kMaxParts;
}

template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N]) {
    __shared__ double sh[N][kBlock];
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < N; ++k) sh[k][t] = v[k];
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int k = 0; k < N; ++k) sh[k][t] += sh[k][t + s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = sh[k][0];
    __syncthreads();
}

// Per-block partial sums; returns true in every thread of the last block,
// where `tot` (valid in thread 0) holds the grid-wide sums in fixed order.
template <int N>
__device__ bool grid_sum(double (&v)[N], double *parts, SolveStatus *st, double (&tot)[N]) {
    block_sum<N>(v);
    __shared__ int is_last;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) parts[k * kMaxParts + blockIdx.x] = v[k];
        __threadfence();
        unsigned prev = atomicAdd(&st->counter, 1u);
        is_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    double acc[N];
#pragma unroll
    for (int k = 0; k < N; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) {
#pragma unroll
        for (int k = 0; k < N; ++k)
            acc[k] += __hip_atomic_load(&parts[k * kMaxParts + b], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    }
    block_sum<N>(acc);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) tot[k] = acc[k];
        st->counter = 0;
    }
    return true;
}

__device__ __forceinline__ bool bad(double v) { return !(v == v) || v > 1e300; }

// ---------------------------------------------------------------------------
// operator rows

// Row `row` of K = Q^T B^1 Q (pinned) in precision T.  x(c) gives the
// operand.  Also returns the diagonal.  Pressure rows: the 5-point stencil
// with coefficients B^1 = dt * dy_j / Dx_i (u faces) and dt * dx_i / Dy_j
// (v faces) on interior faces, plus the stored force coupling inside the box.
template <class T, class X>
__device__ __forceinline__ T k0_row(const K0T<T> &K, int row, X x, T &diag) {
    const GridT<T> &g = K.g;
    if (row < g.n_cell) {
        int j = row / g.nx;
        int i = row - j * g.nx;
        T bw = i > 0 ? K.dt * g.dy[j] * g.iDx[i] : T(0);
        T be = i < g.nx - 1 ? K.dt * g.dy[j] * g.iDx[i + 1] : T(0);
        T bs = j > 0 ? K.dt * g.dx[i] * g.iDy[j] : T(0);
        T bn = j < g.ny - 1 ? K.dt * g.dx[i] * g.iDy[j + 1] : T(0);
        diag = ((bw + be) + bs) + bn;
        T y = diag * x(row);
        if (row == 0) return y;
        if (j > 0 && row - g.nx != 0) y -= bs * x(row - g.nx);
        if (i > 0 && row - 1 != 0) y -= bw * x(row - 1);
        if (i < g.nx - 1) y -= be * x(row + 1);
        if (j < g.ny - 1) y -= bn * x(row + g.nx);
        if (i >= K.cb_i0 && i <= K.cb_i1 && j >= K.cb_j0 && j <= K.cb_j1) {
            int r = (j - K.cb_j0) * (K.cb_i1 - K.cb_i0 + 1) + (i - K.cb_i0);
            for (int p = K.cf.ptr[r]; p < K.cf.ptr[r + 1]; ++p)
                y += K.cf.val[p] * x(g.n_cell + K.cf.col[p]);
        }
        return y;
    }
    int k = row - g.n_cell;
    diag = K.kf_diag[k];
    T y = T(0);
    for (int p = K.kf.ptr[k]; p < K.kf.ptr[k + 1]; ++p) y += K.kf.val[p] * x(K.kf.col[p]);
    return y;
}

template <class T>
__device__ __forceinline__ T k0_diag(const K0T<T> &K, int row) {
    const GridT<T> &g = K.g;
    if (row < g.n_cell) {
        int j = row / g.nx;
        int i = row - j * g.nx;
        T bw = i > 0 ? K.dt * g.dy[j] * g.iDx[i] : T(0);
        T be = i < g.nx - 1 ? K.dt * g.dy[j] * g.iDx[i + 1] : T(0);
        T bs = j > 0 ? K.dt * g.dx[i] * g.iDy[j] : T(0);
        T bn = j < g.ny - 1 ? K.dt * g.dx[i] * g.iDy[j + 1] : T(0);
        return ((bw + be) + bs) + bn;
    }
    return K.kf_diag[row - g.n_cell];
}

// Row f of A = Mf/dt - (nu/2) M Lhat R^{-1} on interior faces (wall
// neighbours contribute through the right-hand side).
template <class X>
__device__ __forceinline__ double a_row(const AView &A, int f, X x, double &diag) {
    const GridView &g = A.g;
    if (f < g.n_u) {
        int nxm = g.nx - 1;
        int j = f / nxm;
        int i = f - j * nxm + 1;
        double idyj = g.idy[j];
        double u = x(f) * idyj;
        double uE = i < g.nx - 1 ? x(f + 1) * idyj : 0.0;
        double uW = i > 1 ? x(f - 1) * idyj : 0.0;
        double uN = j < g.ny - 1 ? x(f + nxm) * g.idy[j + 1] : 0.0;
        double uS = j > 0 ? x(f - nxm) * g.idy[j - 1] : 0.0;
        double lapx = ((uE - u) * g.idx[i] - (u - uW) * g.idx[i - 1]) * g.iDx[i];
        double lapy = ((uN - u) * g.iDy[j + 1] - (u - uS) * g.iDy[j]) * idyj;
        double mf = g.Dx[i] * idyj;
        diag = mf * A.idt + 0.5 * A.nu * ((g.idx[i] + g.idx[i - 1]) * idyj +
                                          g.Dx[i] * (g.iDy[j + 1] + g.iDy[j]) * idyj * idyj);
        return mf * A.idt * x(f) - 0.5 * A.nu * (g.Dx[i] * (lapx + lapy));
    }
    int r = f - g.n_u;
    int j = r / g.nx + 1;
    int i = r - (j - 1) * g.nx;
    double idxi = g.idx[i];
    double v = x(f) * idxi;
    double vE = i < g.nx - 1 ? x(f + 1) * g.idx[i + 1] : 0.0;
    double vW = i > 0 ? x(f - 1) * g.idx[i - 1] : 0.0;
    double vN = j < g.ny - 1 ? x(f + g.nx) * idxi : 0.0;
    double vS = j > 1 ? x(f - g.nx) * idxi : 0.0;
    double lapx = ((vE - v) * g.iDx[i + 1] - (v - vW) * g.iDx[i]) * idxi;
    double lapy = ((vN - v) * g.idy[j] - (v - vS) * g.idy[j - 1]) * g.iDy[j];
    double mf = g.Dy[j] * idxi;
    diag = mf * A.idt + 0.5 * A.nu * (g.Dy[j] * (g.iDx[i + 1] + g.iDx[i]) * idxi * idxi +
                                      (g.idy[j] + g.idy[j - 1]) * idxi);
    return mf * A.idt * x(f) - 0.5 * A.nu * (g.Dy[j] * (lapx + lapy));
}

__device__ __forceinline__ double a_diag(const AView &A, int f) {
    double d;
    a_row(A, f, [](int) { return 0.0; }, d);
    return d;
}

// overloads so the Krylov kernels can be written once
template <class T, class X>
__device__ __forceinline__ T op_row(const K0T<T> &K, int r, X x, T &d) {
    return k0_row(K, r, x, d);
}
template <class X>
__device__ __forceinline__ double op_row(const AView &A, int r, X x, double &d) {
    return a_row(A, r, x, d);
}
template <class T>
__device__ __forceinline__ T op_diag(const K0T<T> &K, int r) { return k0_diag(K, r); }
__device__ __forceinline__ double op_diag(const AView &A, int r) { return a_diag(A, r); }
template <class T>
__host__ __device__ inline int op_n(const K0T<T> &K) { return K.n; }
__host__ __device__ inline int op_n(const AView &A) { return A.g.n_q; }

// ---------------------------------------------------------------------------
// Krylov kernels

template <class Op, class T>
__global__ __launch_bounds__(kBlock) void k_pcg_init(Op op, const T *b, const T *x, T *r,
                                                     SolveStatus *st, double *parts, int jacobi,
                                                     double rtol2, int maxit) {
    const int n = op_n(op);
    Tiles Tl = my_tiles(n);
    double v[3] = {0.0, 0.0, 0.0};   // bb, rr, rz
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < n) {
            T d;
            T ax = op_row(op, row, [&](int c) { return x[c]; }, d);
            T bi = b[row];
            T ri = bi - ax;
            r[row] = ri;
            v[0] += (double)bi * (double)bi;
            v[1] += (double)ri * (double)ri;
            if (jacobi) v[2] += (double)ri * (double)ri / (double)d;
        }
    }
    double tot[3];
    if (grid_sum<3>(v, parts, st, tot) && threadIdx.x == 0) {
        st->bb = tot[0];
        st->rr = tot[1];
        st->tol2 = rtol2;
        st->maxit = maxit;
        st->iter = 0;
        st->beta = 0.0;
        st->first = 1;
        st->done = ST_RUNNING;
        if (tot[0] == 0.0) {
            st->done = ST_ZERO_RHS;
        } else if (bad(tot[1])) {
            st->done = ST_NAN;
        } else if (tot[1] <= rtol2 * tot[0]) {
            st->done = ST_CONVERGED;
        }
        if (jacobi) {
            st->rz = tot[2];
            st->first = 0;
        }
    }
}

// x = 0, r = b (initial guess zero; used by the inner mixed-precision solve)
template <class T>
__global__ __launch_bounds__(kBlock) void k_pcg_init_zero(int n, const T *b, T *x, T *r,
                                                          SolveStatus *st, double *parts,
                                                          double rtol2, int maxit) {
    Tiles Tl = my_tiles(n);
    double v[1] = {0.0};
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < n) {
            T bi = b[row];
            x[row] = T(0);
            r[row] = bi;
            v[0] += (double)bi * (double)bi;
        }
    }
    double tot[1];
    if (grid_sum<1>(v, parts, st, tot) && threadIdx.x == 0) {
        st->bb = tot[0];
        st->rr = tot[0];
        st->tol2 = rtol2;
        st->maxit = maxit;
        st->iter = 0;
        st->beta = 0.0;
        st->first = 1;
        st->done = tot[0] == 0.0 ? ST_ZERO_RHS : (bad(tot[0]) ? ST_NAN : ST_RUNNING);
    }
}

// p_new = z + beta p_old (z = D^{-1} r for Jacobi), q = op p_new, pq = p_new . q
template <class Op, class T>
__global__ __launch_bounds__(kBlock) void k_pcg_spmv(Op op, const T *src, const T *pold, T *pnew,
                                                     T *q, SolveStatus *st, double *parts,
                                                     int jacobi) {
    if (st->done) return;
    const int n = op_n(op);
    const T beta = (T)st->beta;
    Tiles Tl = my_tiles(n);
    double v[1] = {0.0};
    auto pval = [&](int c) {
        T z = jacobi ? src[c] / op_diag(op, c) : src[c];
        return z + beta * pold[c];
    };
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < n) {
            T d;
            T qi = op_row(op, row, pval, d);
            T pi = pval(row);
            pnew[row] = pi;
            q[row] = qi;
            v[0] += (double)pi * (double)qi;
        }
    }
    double tot[1];
    if (grid_sum<1>(v, parts, st, tot) && threadIdx.x == 0) st->pq = tot[0];
}

// x += alpha p, r -= alpha q; convergence test on ||r||^2
template <class Op, class T>
__global__ __launch_bounds__(kBlock) void k_pcg_update(Op op, T *x, T *r, const T *p, const T *q,
                                                       SolveStatus *st, double *parts, int jacobi) {
    if (st->done) return;
    const int n = op_n(op);
    const T alpha = (T)(st->rz / st->pq);
    Tiles Tl = my_tiles(n);
    double v[2] = {0.0, 0.0};
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < n) {
            x[row] += alpha * p[row];
            T ri = r[row] - alpha * q[row];
            r[row] = ri;
            v[0] += (double)ri * (double)ri;
            if (jacobi) v[1] += (double)ri * (double)ri / (double)op_diag(op, row);
        }
    }
    double tot[2];
    if (grid_sum<2>(v, parts, st, tot) && threadIdx.x == 0) {
        st->rr = tot[0];
        st->iter += 1;
        if (bad(tot[0])) st->done = ST_NAN;
        else if (tot[0] <= st->tol2 * st->bb) st->done = ST_CONVERGED;
        else if (st->iter >= st->maxit) st->done = ST_MAXIT;
        if (jacobi) {
            st->beta = tot[1] / st->rz;
            st->rz = tot[1];
        }
    }
}

template <class Op, class T>
__global__ __launch_bounds__(kBlock) void k_true_residual(Op op, const T *b, const T *x,
                                                          SolveStatus *st, double *parts) {
    const int n = op_n(op);
    Tiles Tl = my_tiles(n);
    double v[1] = {0.0};
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < n) {
            T d;
            T ri = b[row] - op_row(op, row, [&](int c) { return x[c]; }, d);
            v[0] += (double)ri * (double)ri;
        }
    }
    double tot[1];
    if (grid_sum<1>(v, parts, st, tot) && threadIdx.x == 0) st->true_rr = tot[0];
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_zero_if_zero_rhs(T *x, int n, const SolveStatus *st) {
    if (st->done != ST_ZERO_RHS) return;
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = T(0);
}

template <class Op, class T>
__global__ __launch_bounds__(kBlock) void k_apply(Op op, const T *x, T *y) {
    const int n = op_n(op);
    Tiles Tl = my_tiles(n);
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < n) {
            T d;
            y[row] = op_row(op, row, [&](int c) { return x[c]; }, d);
        }
    }
}

// r . z for the PCG when the preconditioner wrote z directly (one-level AMG)
template <class T>
__global__ __launch_bounds__(kBlock) void k_dot_rz(int n, const T *r, const T *z, SolveStatus *st,
                                                   double *parts) {
    if (st->done) return;
    Tiles Tl = my_tiles(n);
    double v[1] = {0.0};
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < n) v[0] += (double)r[row] * (double)z[row];
    }
    double tot[1];
    if (grid_sum<1>(v, parts, st, tot) && threadIdx.x == 0) {
        if (st->first) {
            st->beta = 0.0;
            st->first = 0;
        } else {
            st->beta = tot[0] / st->rz;
        }
        st->rz = tot[0];
    }
}

// ---------------------------------------------------------------------------
// V-cycle on level 0 (K0)

template <class T>
__global__ __launch_bounds__(kBlock) void k_k0_jacobi_first(K0T<T> K, T omega, const T *b, T *x,
                                                            const SolveStatus *st) {
    if (st->done) return;
    Tiles Tl = my_tiles(K.n);
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < K.n) x[row] = omega / k0_diag(K, row) * b[row];
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_k0_jacobi(K0T<T> K, T omega, const T *b, const T *xin,
                                                      T *xout, const SolveStatus *st) {
    if (st->done) return;
    Tiles Tl = my_tiles(K.n);
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < K.n) {
            T d;
            T ax = k0_row(K, row, [&](int c) { return xin[c]; }, d);
            xout[row] = xin[row] + omega / d * (b[row] - ax);
        }
    }
}

// last post-smoothing sweep: also forms r . z for the PCG (b is the PCG residual)
template <class T>
__global__ __launch_bounds__(kBlock) void k_k0_jacobi_rz(K0T<T> K, T omega, const T *b,
                                                         const T *xin, T *xout, SolveStatus *st,
                                                         double *parts) {
    if (st->done) return;
    Tiles Tl = my_tiles(K.n);
    double v[1] = {0.0};
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < K.n) {
            T d;
            T ax = k0_row(K, row, [&](int c) { return xin[c]; }, d);
            T bi = b[row];
            T z = xin[row] + omega / d * (bi - ax);
            xout[row] = z;
            v[0] += (double)bi * (double)z;
        }
    }
    double tot[1];
    if (grid_sum<1>(v, parts, st, tot) && threadIdx.x == 0) {
        if (st->first) {
            st->beta = 0.0;
            st->first = 0;
        } else {
            st->beta = tot[0] / st->rz;
        }
        st->rz = tot[0];
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_k0_residual(K0T<T> K, const T *b, const T *x, T *r,
                                                        const SolveStatus *st) {
    if (st->done) return;
    Tiles Tl = my_tiles(K.n);
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < K.n) {
            T d;
            r[row] = b[row] - k0_row(K, row, [&](int c) { return x[c]; }, d);
        }
    }
}

// ---------------------------------------------------------------------------
// V-cycle on coarse levels (CSR), one row per thread

template <class T>
__device__ __forceinline__ T csr_dot(const CSRT<T> &A, int row, const T *x) {
    T y = T(0);
    for (int p = A.ptr[row]; p < A.ptr[row + 1]; ++p) y += A.val[p] * x[A.col[p]];
    return y;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_csr_jacobi_first(CSRT<T> A, const T *wdinv, const T *b,
                                                             T *x, const SolveStatus *st) {
    if (st->done) return;
    Tiles Tl = my_tiles(A.nrows);
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < A.nrows) x[row] = wdinv[row] * b[row];
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_csr_jacobi(CSRT<T> A, const T *wdinv, const T *b,
                                                       const T *xin, T *xout,
                                                       const SolveStatus *st) {
    if (st->done) return;
    Tiles Tl = my_tiles(A.nrows);
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < A.nrows) xout[row] = xin[row] + wdinv[row] * (b[row] - csr_dot(A, row, xin));
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_csr_residual(CSRT<T> A, const T *b, const T *x, T *r,
                                                         const SolveStatus *st) {
    if (st->done) return;
    Tiles Tl = my_tiles(A.nrows);
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < A.nrows) r[row] = b[row] - csr_dot(A, row, x);
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_csr_spmv(CSRT<T> A, const T *x, T *y, int add,
                                                     const SolveStatus *st) {
    if (st && st->done) return;
    Tiles Tl = my_tiles(A.nrows);
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < A.nrows) {
            T v = csr_dot(A, row, x);
            y[row] = add ? y[row] + v : v;
        }
    }
}

// x = Ainv b with Ainv dense FP64, column-major (coalesced over rows);
// FP64 accumulation whatever T is (the coarsest solve stays FP64)
template <class T>
__global__ __launch_bounds__(kBlock) void k_dense_solve(int n, const double *inv, const T *b, T *x,
                                                        const SolveStatus *st) {
    if (st->done) return;
    __shared__ double sb[kBlock];
    int row = blockIdx.x * kBlock + threadIdx.x;
    double acc = 0.0;
    for (int c0 = 0; c0 < n; c0 += kBlock) {
        int c = c0 + threadIdx.x;
        sb[threadIdx.x] = c < n ? (double)b[c] : 0.0;
        __syncthreads();
        int m = min(kBlock, n - c0);
        if (row < n)
            for (int k = 0; k < m; ++k) acc += inv[(size_t)(c0 + k) * n + row] * sb[k];
        __syncthreads();
    }
    if (row < n) x[row] = (T)acc;
}

// ---------------------------------------------------------------------------
// mixed precision outer loop (FP64)

// r = b - K x in FP64, r32 = (float) r, ||r||^2 (and ||b||^2 when first)
__global__ __launch_bounds__(kBlock) void k_outer_residual(K0View K, const double *b,
                                                           const double *x, float *r32,
                                                           SolveStatus *st, double *parts,
                                                           int first) {
    Tiles Tl = my_tiles(K.n);
    double v[2] = {0.0, 0.0};
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < K.n) {
            double d;
            double bi = b[row];
            double ri = bi - k0_row(K, row, [&](int c) { return x[c]; }, d);
            r32[row] = (float)ri;
            v[0] += ri * ri;
            v[1] += bi * bi;
        }
    }
    double tot[2];
    if (grid_sum<2>(v, parts, st, tot) && threadIdx.x == 0) {
        st->rr = tot[0];
        if (first) {
            st->bb = tot[1];
            st->iter = 0;
        } else {
            st->iter += 1;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_add_correction(int n, double *x, const float *d) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] += (double)d[i];
}

// ---------------------------------------------------------------------------
// time-step stages

struct Vel {
    GridView g;
    const double *q;
    const double *w;
    WallOffsets o;
    // u velocity at face (i, j), i = 0..nx (walls at 0 and nx), j = 0..ny-1
    __device__ __forceinline__ double U(int i, int j) const {
        if (i == 0) return w[o.uL + j];
        if (i == g.nx) return w[o.uR + j];
        return q[(size_t)j * (g.nx - 1) + (i - 1)] * g.idy[j];
    }
    // v velocity at face (i, j), i = 0..nx-1, j = 0..ny (walls at 0 and ny)
    __device__ __forceinline__ double V(int i, int j) const {
        if (j == 0) return w[o.vB + i];
        if (j == g.ny) return w[o.vT + i];
        return q[g.n_u + (size_t)(j - 1) * g.nx + i] * g.idx[i];
    }
    // corner (x_i, y_j): u interpolated across the y line, walls on top / bottom
    __device__ __forceinline__ double Uc(int i, int j) const {
        if (j == 0) return w[o.uBt + i];
        if (j == g.ny) return w[o.uTt + i];
        double wlo = 0.5 * g.dy[j] * g.iDy[j];
        double whi = 0.5 * g.dy[j - 1] * g.iDy[j];
        return wlo * U(i, j - 1) + whi * U(i, j);
    }
    // corner (x_i, y_j): v interpolated across the x line, walls left / right
    __device__ __forceinline__ double Vc(int i, int j) const {
        if (i == 0) return w[o.vLt + j];
        if (i == g.nx) return w[o.vRt + j];
        double wle = 0.5 * g.dx[i] * g.iDx[i];
        double wri = 0.5 * g.dx[i - 1] * g.iDx[i];
        return wle * V(i - 1, j) + wri * V(i, j);
    }
};

// Right-hand side of the momentum equation (AB2 convection, Crank-Nicolson
// diffusion): r1 = Mf/dt q + nu/2 (M Lhat u^n incl. walls^n + M bc(walls^{n+1}))
//                 - 3/2 N(q^n) + 1/2 N(q^{n-1})
__global__ __launch_bounds__(kBlock) void k_momentum_rhs(GridView g, const double *q,
                                                         const double *conv_prev, double *conv_now,
                                                         double *r1, const double *w0,
                                                         const double *w1, double nu, double idt,
                                                         int first_step) {
    int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= g.n_q) return;
    WallOffsets o = WallOffsets::make(g.nx, g.ny);
    Vel V0{g, q, w0, o};
    double conv, lap, bcn1, mf, M;
    if (f < g.n_u) {
        int nxm = g.nx - 1;
        int j = f / nxm;
        int i = f - j * nxm + 1;
        double u = V0.U(i, j);
        double ucE = 0.5 * (u + V0.U(i + 1, j));
        double ucW = 0.5 * (V0.U(i - 1, j) + u);
        double uvN = V0.Uc(i, j + 1) * V0.Vc(i, j + 1);
        double uvS = V0.Uc(i, j) * V0.Vc(i, j);
        M = g.Dx[i];
        conv = (ucE * ucE - ucW * ucW) + M * g.idy[j] * (uvN - uvS);
        double uN = (j == g.ny - 1) ? w0[o.uTt + i] : V0.U(i, j + 1);
        double uS = (j == 0) ? w0[o.uBt + i] : V0.U(i, j - 1);
        double lapx = ((V0.U(i + 1, j) - u) * g.idx[i] - (u - V0.U(i - 1, j)) * g.idx[i - 1]) * g.iDx[i];
        double lapy = ((uN - u) * g.iDy[j + 1] - (u - uS) * g.iDy[j]) * g.idy[j];
        lap = M * (lapx + lapy);
        double b = 0.0;
        if (i == 1) b += w1[o.uL + j] * g.idx[0] * g.iDx[1];
        if (i == g.nx - 1) b += w1[o.uR + j] * g.idx[g.nx - 1] * g.iDx[g.nx - 1];
        if (j == 0) b += w1[o.uBt + i] * g.iDy[0] * g.idy[0];
        if (j == g.ny - 1) b += w1[o.uTt + i] * g.iDy[g.ny] * g.idy[g.ny - 1];
        bcn1 = M * b;
        mf = M * g.idy[j];
    } else {
        int r = f - g.n_u;
        int j = r / g.nx + 1;
        int i = r - (j - 1) * g.nx;
        double v = V0.V(i, j);
        double vcN = 0.5 * (v + V0.V(i, j + 1));
        double vcS = 0.5 * (V0.V(i, j - 1) + v);
        double uvE = V0.Uc(i + 1, j) * V0.Vc(i + 1, j);
        double uvW = V0.Uc(i, j) * V0.Vc(i, j);
        M = g.Dy[j];
        conv = M * g.idx[i] * (uvE - uvW) + (vcN * vcN - vcS * vcS);
        double vE = (i == g.nx - 1) ? w0[o.vRt + j] : V0.V(i + 1, j);
        double vW = (i == 0) ? w0[o.vLt + j] : V0.V(i - 1, j);
        double lapx = ((vE - v) * g.iDx[i + 1] - (v - vW) * g.iDx[i]) * g.idx[i];
        double lapy = ((V0.V(i, j + 1) - v) * g.idy[j] - (v - V0.V(i, j - 1)) * g.idy[j - 1]) * g.iDy[j];
        lap = M * (lapx + lapy);
        double b = 0.0;
        if (j == 1) b += w1[o.vB + i] * g.idy[0] * g.iDy[1];
        if (j == g.ny - 1) b += w1[o.vT + i] * g.idy[g.ny - 1] * g.iDy[g.ny - 1];
        if (i == 0) b += w1[o.vLt + j] * g.iDx[0] * g.idx[0];
        if (i == g.nx - 1) b += w1[o.vRt + j] * g.iDx[g.nx] * g.idx[g.nx - 1];
        bcn1 = M * b;
        mf = M * g.idx[i];
    }
    double prev = first_step ? conv : conv_prev[f];
    conv_now[f] = conv;
    r1[f] = mf * idt * q[f] + 0.5 * nu * (lap + bcn1) - 1.5 * conv + 0.5 * prev;
}

// Wall values n -> n+1: convective outflow on the right wall (explicit
// upwind in time), then a uniform shift of the outflow normal velocity so
// the net wall flux is zero.  One block.
__global__ __launch_bounds__(kBlock) void k_walls_update(GridView g, const double *w0, double *w1,
                                                         const double *q, double uconv, double dt,
                                                         double ly) {
    WallOffsets o = WallOffsets::make(g.nx, g.ny);
    const int t = threadIdx.x;
    for (int k = t; k < o.total; k += kBlock) w1[k] = w0[k];
    __syncthreads();
    const int nx = g.nx, ny = g.ny;
    const double dxl = g.dx[nx - 1];
    for (int j = t; j < ny; j += kBlock) {
        double uin = q[(size_t)j * (nx - 1) + (nx - 2)] * g.idy[j];
        double ub = w0[o.uR + j];
        w1[o.uR + j] = ub - uconv * dt * (ub - uin) / dxl;
    }
    for (int j = 1 + t; j < ny; j += kBlock) {
        double vin = q[g.n_u + (size_t)(j - 1) * nx + (nx - 1)] * g.idx[nx - 1];
        double vb = w0[o.vRt + j];
        w1[o.vRt + j] = vb - uconv * dt * (vb - vin) / (0.5 * dxl);
    }
    __syncthreads();
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = t; j < ny; j += kBlock) {
        v[0] += w1[o.uR + j] * g.dy[j];
        v[1] += w1[o.uL + j] * g.dy[j];
    }
    for (int i = t; i < nx; i += kBlock) {
        v[2] += w1[o.vT + i] * g.dx[i];
        v[3] += w1[o.vB + i] * g.dx[i];
    }
    block_sum<4>(v);
    double net = ((v[0] - v[1]) + v[2]) - v[3];
    for (int j = t; j < ny; j += kBlock) w1[o.uR + j] -= net / ly;
}

// [-D q* + bc2 ; E q* - u_B] with the n+1 walls; entry 0 (pinned) cleared
__global__ __launch_bounds__(kBlock) void k_poisson_rhs(GridView g, int nb, const double *qs,
                                                        const double *w1, CSRView E,
                                                        const double *ub, double *rhs) {
    int row = blockIdx.x * kBlock + threadIdx.x;
    if (row < g.n_cell) {
        WallOffsets o = WallOffsets::make(g.nx, g.ny);
        int j = row / g.nx;
        int i = row - j * g.nx;
        int nxm = g.nx - 1;
        double fe = i < g.nx - 1 ? qs[(size_t)j * nxm + i] : w1[o.uR + j] * g.dy[j];
        double fw = i > 0 ? qs[(size_t)j * nxm + i - 1] : w1[o.uL + j] * g.dy[j];
        double fn = j < g.ny - 1 ? qs[g.n_u + (size_t)j * g.nx + i] : w1[o.vT + i] * g.dx[i];
        double fs = j > 0 ? qs[g.n_u + (size_t)(j - 1) * g.nx + i] : w1[o.vB + i] * g.dx[i];
        rhs[row] = row == 0 ? 0.0 : -(((fe - fw) + fn) - fs);
    } else if (row < g.n_cell + 2 * nb) {
        int k = row - g.n_cell;
        double s = 0.0;
        for (int p = E.ptr[k]; p < E.ptr[k + 1]; ++p) s += E.val[p] * qs[E.col[p]];
        rhs[row] = s - ub[k];
    }
}

// q = q* - B^1 (G phi + E^T f~): pressure gradient and delta spreading,
// the spreading as a gather over the stored face -> point weights
__global__ __launch_bounds__(kBlock) void k_project(GridView g, double dt, int nb,
                                                    const double *qs, const double *lam,
                                                    double *qout, CSRView etu, int fu_i0, int fu_i1,
                                                    int fu_j0, int fu_j1, CSRView etv, int fv_i0,
                                                    int fv_i1, int fv_j0, int fv_j1) {
    int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= g.n_q) return;
    const double *phi = lam;
    double s, b1;
    if (f < g.n_u) {
        int nxm = g.nx - 1;
        int j = f / nxm;
        int i = f - j * nxm + 1;
        s = phi[j * g.nx + i] - phi[j * g.nx + i - 1];
        if (i >= fu_i0 && i <= fu_i1 && j >= fu_j0 && j <= fu_j1) {
            int r = (j - fu_j0) * (fu_i1 - fu_i0 + 1) + (i - fu_i0);
            const double *fx = lam + g.n_cell;
            for (int p = etu.ptr[r]; p < etu.ptr[r + 1]; ++p) s += etu.val[p] * fx[etu.col[p]];
        }
        b1 = dt * g.dy[j] * g.iDx[i];
    } else {
        int r = f - g.n_u;
        int j = r / g.nx + 1;
        int i = r - (j - 1) * g.nx;
        s = phi[j * g.nx + i] - phi[(j - 1) * g.nx + i];
        if (i >= fv_i0 && i <= fv_i1 && j >= fv_j0 && j <= fv_j1) {
            int rr = (j - fv_j0) * (fv_i1 - fv_i0 + 1) + (i - fv_i0);
            const double *fy = lam + g.n_cell + nb;
            for (int p = etv.ptr[rr]; p < etv.ptr[rr + 1]; ++p) s += etv.val[p] * fy[etv.col[p]];
        }
        b1 = dt * g.dx[i] * g.iDy[j];
    }
    qout[f] = qs[f] - b1 * s;
}

__global__ __launch_bounds__(kBlock) void k_forces(int n_cell, int nb, const double *lam,
                                                   SolveStatus *st) {
    double v[2] = {0.0, 0.0};
    for (int k = threadIdx.x; k < nb; k += kBlock) {
        v[0] += lam[n_cell + k];
        v[1] += lam[n_cell + nb + k];
    }
    block_sum<2>(v);
    if (threadIdx.x == 0) {
        st->fx = v[0];
        st->fy = v[1];
    }
}

__global__ __launch_bounds__(kBlock) void k_init_state(GridView g, double *q, double *conv,
                                                       double *lam, int n_lam, double U, double V) {
    int f = blockIdx.x * kBlock + threadIdx.x;
    if (f < g.n_q) {
        if (f < g.n_u) {
            int j = f / (g.nx - 1);
            q[f] = U * g.dy[j];
        } else {
            int i = (f - g.n_u) % g.nx;
            q[f] = V * g.dx[i];
        }
        conv[f] = 0.0;
    }
    if (f < n_lam) lam[f] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_fill_walls(GridView g, double *w, double U, double V) {
    WallOffsets o = WallOffsets::make(g.nx, g.ny);
    for (int k = threadIdx.x; k < o.total; k += kBlock) {
        bool is_u = (k < o.vB) || (k >= o.uBt && k < o.vLt);
        w[k] = is_u ? U : V;
    }
}


}  // namespace

// ---------------------------------------------------------------------------
// launchers

#define LAUNCH(kernel, grid, ...) hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, __VA_ARGS__)

void launch_walls_update(hipStream_t s, GridView g, const double *w0, double *w1, const double *q,
                         double uconv, double dt, double ly) {
    LAUNCH(k_walls_update, 1, g, w0, w1, q, uconv, dt, ly);
}

void launch_momentum_rhs(hipStream_t s, GridView g, const double *q, const double *conv_prev,
                         double *conv_now, double *r1, const double *w0, const double *w1,
                         double nu, double dt, int first_step) {
    LAUNCH(k_momentum_rhs, (g.n_q + kBlock - 1) / kBlock, g, q, conv_prev, conv_now, r1, w0, w1, nu,
           1.0 / dt, first_step);
}

void launch_poisson_rhs(hipStream_t s, GridView g, int nb, const double *qstar, const double *w1,
                        CSRView E, const double *ub, double *rhs) {
    int n = g.n_cell + 2 * nb;
    LAUNCH(k_poisson_rhs, (n + kBlock - 1) / kBlock, g, nb, qstar, w1, E, ub, rhs);
}

void launch_project(hipStream_t s, GridView g, double dt, int nb, const double *qstar,
                    const double *lam, double *qout, CSRView etu, int fu_i0, int fu_i1, int fu_j0,
                    int fu_j1, CSRView etv, int fv_i0, int fv_i1, int fv_j0, int fv_j1) {
    LAUNCH(k_project, (g.n_q + kBlock - 1) / kBlock, g, dt, nb, qstar, lam, qout, etu, fu_i0, fu_i1,
           fu_j0, fu_j1, etv, fv_i0, fv_i1, fv_j0, fv_j1);
}

void launch_forces(hipStream_t s, int n_cell, int nb, const double *lam, SolveStatus *st) {
    LAUNCH(k_forces, 1, n_cell, nb, lam, st);
}

void launch_init_state(hipStream_t s, GridView g, double *q, double *conv, double *lam, int n_lam,
                       double U, double V) {
    int n = g.n_q > n_lam ? g.n_q : n_lam;
    LAUNCH(k_init_state, (n + kBlock - 1) / kBlock, g, q, conv, lam, n_lam, U, V);
}

void launch_fill_walls(hipStream_t s, GridView g, double *w, double U, double V) {
    LAUNCH(k_fill_walls, 1, g, w, U, V);
}

void launch_apply_K0(hipStream_t s, const K0View &K, const double *x, double *y) {
    LAUNCH((k_apply<K0View, double>), grid_for(K.n), K, x, y);
}

void launch_apply_A(hipStream_t s, const AView &A, const double *x, double *y) {
    LAUNCH((k_apply<AView, double>), grid_for(A.g.n_q), A, x, y);
}

template <class Op, class T>
void launch_pcg_init(hipStream_t s, const Op &op, const T *b, const T *x, T *r, SolveStatus *st,
                     double *parts, bool jacobi, double rtol2, int maxit) {
    LAUNCH((k_pcg_init<Op, T>), grid_for(op_n(op)), op, b, x, r, st, parts, (int)jacobi, rtol2, maxit);
}

template <class T>
void launch_pcg_init_zero(hipStream_t s, int n, const T *b, T *x, T *r, SolveStatus *st,
                          double *parts, double rtol2, int maxit) {
    LAUNCH((k_pcg_init_zero<T>), grid_for(n), n, b, x, r, st, parts, rtol2, maxit);
}

template <class Op, class T>
void launch_pcg_spmv(hipStream_t s, const Op &op, const T *src, const T *pold, T *pnew, T *q,
                     SolveStatus *st, double *parts, bool jacobi) {
    LAUNCH((k_pcg_spmv<Op, T>), grid_for(op_n(op)), op, src, pold, pnew, q, st, parts, (int)jacobi);
}

template <class Op, class T>
void launch_pcg_update(hipStream_t s, const Op &op, T *x, T *r, const T *p, const T *q,
                       SolveStatus *st, double *parts, bool jacobi) {
    LAUNCH((k_pcg_update<Op, T>), grid_for(op_n(op)), op, x, r, p, q, st, parts, (int)jacobi);
}

template <class Op, class T>
void launch_true_residual(hipStream_t s, const Op &op, const T *b, const T *x, SolveStatus *st,
                          double *parts) {
    LAUNCH((k_true_residual<Op, T>), grid_for(op_n(op)), op, b, x, st, parts);
}

template <class T>
void launch_dot_rz(hipStream_t s, int n, const T *r, const T *z, SolveStatus *st, double *parts) {
    LAUNCH((k_dot_rz<T>), grid_for(n), n, r, z, st, parts);
}

template <class T>
void launch_zero_if_zero_rhs(hipStream_t s, T *x, int n, const SolveStatus *st) {
    LAUNCH((k_zero_if_zero_rhs<T>), (n + kBlock - 1) / kBlock, x, n, st);
}

template <class T>
void launch_k0_jacobi_first(hipStream_t s, const K0T<T> &K, double omega, const T *b, T *x,
                            const SolveStatus *st) {
    LAUNCH((k_k0_jacobi_first<T>), grid_for(K.n), K, (T)omega, b, x, st);
}

template <class T>
void launch_k0_jacobi(hipStream_t s, const K0T<T> &K, double omega, const T *b, const T *xin,
                      T *xout, const SolveStatus *st) {
    LAUNCH((k_k0_jacobi<T>), grid_for(K.n), K, (T)omega, b, xin, xout, st);
}

template <class T>
void launch_k0_jacobi_rz(hipStream_t s, const K0T<T> &K, double omega, const T *b, const T *xin,
                         T *xout, SolveStatus *st, double *parts) {
    LAUNCH((k_k0_jacobi_rz<T>), grid_for(K.n), K, (T)omega, b, xin, xout, st, parts);
}

template <class T>
void launch_k0_residual(hipStream_t s, const K0T<T> &K, const T *b, const T *x, T *r,
                        const SolveStatus *st) {
    LAUNCH((k_k0_residual<T>), grid_for(K.n), K, b, x, r, st);
}

template <class T>
void launch_csr_jacobi_first(hipStream_t s, CSRT<T> A, const T *wdinv, const T *b, T *x,
                             const SolveStatus *st) {
    LAUNCH((k_csr_jacobi_first<T>), grid_for(A.nrows), A, wdinv, b, x, st);
}

template <class T>
void launch_csr_jacobi(hipStream_t s, CSRT<T> A, const T *wdinv, const T *b, const T *xin,
                       T *xout, const SolveStatus *st) {
    LAUNCH((k_csr_jacobi<T>), grid_for(A.nrows), A, wdinv, b, xin, xout, st);
}

template <class T>
void launch_csr_residual(hipStream_t s, CSRT<T> A, const T *b, const T *x, T *r,
                         const SolveStatus *st) {
    LAUNCH((k_csr_residual<T>), grid_for(A.nrows), A, b, x, r, st);
}

template <class T>
void launch_csr_spmv(hipStream_t s, CSRT<T> A, const T *x, T *y, const SolveStatus *st) {
    LAUNCH((k_csr_spmv<T>), grid_for(A.nrows), A, x, y, 0, st);
}

template <class T>
void launch_csr_spmv_add(hipStream_t s, CSRT<T> A, const T *x, T *y, const SolveStatus *st) {
    LAUNCH((k_csr_spmv<T>), grid_for(A.nrows), A, x, y, 1, st);
}

template <class T>
void launch_dense_solve(hipStream_t s, int n, const double *inv, const T *b, T *x,
                        const SolveStatus *st) {
    LAUNCH((k_dense_solve<T>), (n + kBlock - 1) / kBlock, n, inv, b, x, st);
}

void launch_outer_residual(hipStream_t s, const K0View &K, const double *b, const double *x,
                           float *r32, SolveStatus *st, double *parts, int first) {
    LAUNCH(k_outer_residual, grid_for(K.n), K, b, x, r32, st, parts, first);
}

void launch_add_correction(hipStream_t s, int n, double *x, const float *d) {
    LAUNCH(k_add_correction, (n + kBlock - 1) / kBlock, n, x, d);
}

// explicit instantiations
#define INST_OP(OP, T)                                                                           \
    template void launch_pcg_init<OP, T>(hipStream_t, const OP &, const T *, const T *, T *,     \
                                         SolveStatus *, double *, bool, double, int);            \
    template void launch_pcg_spmv<OP, T>(hipStream_t, const OP &, const T *, const T *, T *, T *, \
                                         SolveStatus *, double *, bool);                         \
    template void launch_pcg_update<OP, T>(hipStream_t, const OP &, T *, T *, const T *,         \
                                           const T *, SolveStatus *, double *, bool);            \
    template void launch_true_residual<OP, T>(hipStream_t, const OP &, const T *, const T *,     \
                                              SolveStatus *, double *);
INST_OP(K0View, double)
INST_OP(AView, double)
INST_OP(K0T<float>, float)

#define INST_T(T)                                                                                \
    template void launch_pcg_init_zero<T>(hipStream_t, int, const T *, T *, T *, SolveStatus *,  \
                                          double *, double, int);                                \
    template void launch_dot_rz<T>(hipStream_t, int, const T *, const T *, SolveStatus *,        \
                                   double *);                                                    \
    template void launch_zero_if_zero_rhs<T>(hipStream_t, T *, int, const SolveStatus *);        \
    template void launch_k0_jacobi_first<T>(hipStream_t, const K0T<T> &, double, const T *, T *, \
                                            const SolveStatus *);                                \
    template void launch_k0_jacobi<T>(hipStream_t, const K0T<T> &, double, const T *, const T *, \
                                      T *, const SolveStatus *);                                 \
    template void launch_k0_jacobi_rz<T>(hipStream_t, const K0T<T> &, double, const T *,         \
                                         const T *, T *, SolveStatus *, double *);               \
    template void launch_k0_residual<T>(hipStream_t, const K0T<T> &, const T *, const T *, T *,  \
                                        const SolveStatus *);                                    \
    template void launch_csr_jacobi_first<T>(hipStream_t, CSRT<T>, const T *, const T *, T *,    \
                                             const SolveStatus *);                               \
    template void launch_csr_jacobi<T>(hipStream_t, CSRT<T>, const T *, const T *, const T *,    \
                                       T *, const SolveStatus *);                                \
    template void launch_csr_residual<T>(hipStream_t, CSRT<T>, const T *, const T *, T *,        \
                                         const SolveStatus *);                                   \
    template void launch_csr_spmv<T>(hipStream_t, CSRT<T>, const T *, T *, const SolveStatus *); \
    template void launch_csr_spmv_add<T>(hipStream_t, CSRT<T>, const T *, T *,                   \
                                         const SolveStatus *);                                   \
    template void launch_dense_solve<T>(hipStream_t, int, const double *, const T *, T *,        \
                                        const SolveStatus *);
INST_T(double)
INST_T(float)

}  // namespace ibpm
