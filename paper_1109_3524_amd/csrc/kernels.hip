// HIP kernels for gfx950: the per-step stages of the immersed-boundary
// projection method and the pieces of the Krylov / AMG solvers.
//
// Every kernel is HBM-bound (sparse, stencil, vector).  Work is one row per
// thread in 256-thread blocks; a block handles a contiguous range of 256-row
// tiles and the block index is remapped so that each of the 8 XCDs owns a
// contiguous eighth of the rows (neighbour rows of a stencil then hit the
// same L2).  Reductions are deterministic: a fixed-order tree per block
// (wave butterflies, then the block's waves in order) writes one partial
// per block, and the partials are summed in block order either by the
// kernel that consumes the scalar (when there are at most kFuseMaxParts of
// them) or by a one-block finalize launch.  No atomics are used.
//
// The solver kernels are templates on the vector precision T (double, or
// float for the mixed-precision inner solve); dot products always
// accumulate in double.
#include "kernels.h"

#include <algorithm>
#include <cstdlib>
#include <stdexcept>
#include <type_traits>

namespace ibpm {

LaunchShape &launch_shape() {
    static LaunchShape ls = [] {
        LaunchShape v;
        if (const char *e = std::getenv("IBPM_WALK_ROWS")) {
            int r = std::atoi(e);
            if (r == 1 || r == 2 || r == 4 || r == 8 || r == 16) v.walk_rows = r;
        }
        if (const char *e = std::getenv("IBPM_MAX_BLOCKS")) {
            int b = std::atoi(e);
            if (b >= 256 && b <= kMaxParts) v.max_blocks = b;
        }
        if (const char *e = std::getenv("IBPM_MAX_WALK_BLOCKS")) {
            int b = std::atoi(e);
            if (b >= 256 && b <= kMaxParts) v.max_walk_blocks = b;
        }
        return v;
    }();
    return ls;
}

namespace {


__device__ __forceinline__ int remap_block(int b, int G) {
    int per = G >> 3;
    if (b >= 8 * per) return b;
    return (b & 7) * per + (b >> 3);
}

struct Tiles {
    int t0, t1;
};

// Tiles of 256 elements of the block: the ntiles tiles are split in
// proportion over the G blocks in remapped order, so that XCD x takes the
// x-th eighth of the vector, the same elements its blocks take in every
// other kernel (the stencil walkers, the CSR kernels, the one-tile kernels):
// a vector written by one kernel is read from the same L2 by the next.
__device__ __forceinline__ Tiles my_tiles(int n) {
    const int ntiles = (n + kBlock - 1) / kBlock;
    const int G = gridDim.x;
    const long long l = remap_block(blockIdx.x, G);
    return {(int)(l * ntiles / G), (int)((l + 1) * ntiles / G)};
}

// first element of a one-tile-per-block kernel (grid = number of tiles)
__device__ __forceinline__ int tile_base() { return remap_block(blockIdx.x, gridDim.x) * kBlock; }

inline int grid_for(int n) {
    int ntiles = (n + kBlock - 1) / kBlock;
    if (ntiles < 1) ntiles = 1;
    const int cap = launch_shape().max_blocks;
    return ntiles < cap ? ntiles : cap;
}

template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N]) {
    // butterfly within each wave (no barriers), then the four wave sums in
    // wave order: a fixed summation order, so results are reproducible
    constexpr int kWaves = kBlock / 64;
    __shared__ double sh[N][kWaves];
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) sh[k][w] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double a = sh[k][0];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) a += sh[k][q];
        v[k] = a;
    }
    __syncthreads();
}

// acc[k] += the partials parts[k * kMaxParts + b], b = threadIdx.x, + kBlock, ...
// (b < G), for k < n, in increasing b; the loads of up to 8 rounds are issued
// before they are added (the partials come from other XCDs, so each round
// would otherwise wait a memory latency)
template <int N>
__device__ __forceinline__ void gather_parts(const double *parts, int G, int n, double (&acc)[N]) {
    constexpr int U = 8;
    for (int b0 = 0; b0 < G; b0 += U * kBlock) {
        double v[N][U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = b0 + u * kBlock + threadIdx.x;
#pragma unroll
            for (int k = 0; k < N; ++k) v[k][u] = (b < G && k < n) ? parts[k * kMaxParts + b] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < N; ++k) acc[k] += v[k][u];
    }
}

// acc[0] += the Ga partials in pa, acc[1] += the Gb partials in pb (first
// row of each buffer), as gather_parts does each, with the loads of both
// issued together
__device__ __forceinline__ void gather_parts2(const double *pa, int Ga, const double *pb, int Gb,
                                              double (&acc)[2]) {
    constexpr int U = 8;
    const int G = Ga > Gb ? Ga : Gb;
    for (int b0 = 0; b0 < G; b0 += U * kBlock) {
        double va[U], vb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = b0 + u * kBlock + threadIdx.x;
            va[u] = b < Ga ? pa[b] : 0.0;
            vb[u] = b < Gb ? pb[b] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            acc[0] += va[u];
            acc[1] += vb[u];
        }
    }
}

// Per-block partial sums of N values: block tree in LDS (fixed order), then
// one store per value.  The grid-wide sums are formed by k_finalize, a
// one-block kernel queued right after, which adds the partials in block
// order: deterministic, and with no fences or atomics between blocks.
template <int N>
__device__ __forceinline__ void write_parts(double (&v)[N], double *parts) {
    block_sum<N>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) parts[k * kMaxParts + blockIdx.x] = v[k];
    }
}

__device__ __forceinline__ bool bad(double v) { return !(v == v) || v > 1e300; }

// ---------------------------------------------------------------------------
// Level-0 operators as walks over tiles of 256 columns x R rows of cells
// (one thread per column, walking its R rows), in a 1-D grid remapped so
// that the tiles of one XCD are contiguous.  The rows of K with stored
// entries are taken by two bands of blocks at the start of the grid, so they
// are dispatched first: the 2 nb force rows (about 18 entries each) and the
// cells of the coupling box that meet a force unknown (up to 9 entries on
// the cylinder workloads), 8 lanes per row with a shuffle reduction.  The
// tiles skip those cells (one bit each), so a tile is the plain 5-point
// stencil with every operand load issued before the arithmetic; tiles of
// two or more rows (the large grids) form each operand once per column and
// exchange the east / west values through LDS.

constexpr int kForceLanes = 8;
static_assert(kKfW % kForceLanes == 0 && kCcW % kForceLanes == 0, "ELL widths must be multiples of 8");

template <class T>
__host__ __device__ inline int force_blocks(const K0T<T> &K) {
    return (2 * K.nb * kForceLanes + kBlock - 1) / kBlock;
}
// both bands, padded to a multiple of 8 blocks, so that block b of the
// tiles that follow runs on XCD b mod 8 (the XCD a block is sent to) and
// the tile remap keeps XCD x on the x-th eighth of the cells
template <class T>
__host__ __device__ inline int k0_band(const K0T<T> &K) {
    const int nbk = force_blocks(K) + (K.ncc * kForceLanes + kBlock - 1) / kBlock;
    return (nbk + 7) & ~7;
}

// 5-point part of the pressure row of cell (i, j), any position on the grid
template <class T, class XV>
__device__ __forceinline__ T k0_cell_stencil(const K0T<T> &K, int i, int j, XV xv, T &diag, T &xc) {
    const GridT<T> &g = K.g;
    const int nx = g.nx, ny = g.ny;
    const int row = j * nx + i;
    const T dt = K.dt;
    const T dxi = g.dx[i];
    const T dyj = g.dy[j];
    const T bw = i > 0 ? dt * g.iDx[i] * dyj : T(0);
    const T be = i < nx - 1 ? dt * g.iDx[i + 1] * dyj : T(0);
    const T bs = j > 0 ? dt * dxi * g.iDy[j] : T(0);
    const T bn = j < ny - 1 ? dt * dxi * g.iDy[j + 1] : T(0);
    xc = xv(row);
    const T xs = j > 0 ? xv(row - nx) : T(0);
    const T xn = j < ny - 1 ? xv(row + nx) : T(0);
    const T xw = i > 0 ? xv(row - 1) : T(0);
    const T xe = i < nx - 1 ? xv(row + 1) : T(0);
    diag = ((bw + be) + bs) + bn;
    T y = diag * xc;
    const int P = K.pin;
    if (row != P) {
        if (row - nx != P) y -= bs * xs;
        if (row - 1 != P) y -= bw * xw;
        if (row + 1 != P) y -= be * xe;
        if (row + nx != P) y -= bn * xn;
    }
    return y;
}

// sum of the row's stored entries over the 8 lanes of the row: from the ELL
// slots (all loads issued at once; a clamped row for the lanes past the
// last row, and the terms of empty slots dropped by a select) or, for rows
// longer than the width, from the CSR row
template <int W, class T, class XV>
__device__ __forceinline__ T band_row_sum(bool live, int q, int lane, bool ell, const int32_t *ecol,
                                          const T *eval, const CSRT<T> &csr, int crow, int col_off, XV xv) {
    T y = T(0);
    if (ell) {
        constexpr int kS = W / kForceLanes;
        const int base = (live ? q : 0) * W + lane;
        int cc[kS];
        T cv[kS], cx[kS];
#pragma unroll
        for (int k = 0; k < kS; ++k) {
            cc[k] = ecol[base + k * kForceLanes];
            cv[k] = eval[base + k * kForceLanes];
        }
#pragma unroll
        for (int k = 0; k < kS; ++k) cx[k] = xv(col_off + (cc[k] >= 0 ? cc[k] : 0));
#pragma unroll
        for (int k = 0; k < kS; ++k) {
            const T t = y + cv[k] * cx[k];
            y = (live && cc[k] >= 0) ? t : y;
        }
    } else if (live) {
        for (int p = csr.ptr[crow] + lane; p < csr.ptr[crow + 1]; p += kForceLanes)
            y += csr.val[p] * xv(col_off + csr.col[p]);
    }
#pragma unroll
    for (int o = kForceLanes / 2; o > 0; o >>= 1) y += __shfl_xor(y, o, kForceLanes);
    return y;
}

// is cell (i, j) one of the coupled cells (taken by the band)?
template <class T>
__device__ __forceinline__ bool k0_coupled(const K0T<T> &K, int i, int j) {
    if (i < K.cb_i0 || i > K.cb_i1 || j < K.cb_j0 || j > K.cb_j1) return false;
    const int rb = (j - K.cb_j0) * (K.cb_i1 - K.cb_i0 + 1) + (i - K.cb_i0);
    return (K.cc_bits[rb >> 5] >> (rb & 31)) & 1u;
}

// Interior tile of R rows (every row has a north neighbour): all operand
// loads of the R rows are issued before the arithmetic.  BOX: the tile
// meets the coupling box, and its coupled cells are left to the band.
template <int R, bool BOX, class T, class XV, class PF, class ACT>
__device__ __forceinline__ void k0_tile(const K0T<T> &K, int i, int j0, XV xv, PF pf, ACT act) {
    const GridT<T> &g = K.g;
    const int nx = g.nx;
    const T dt = K.dt;
    const T dxi = g.dx[i];
    const T cw = i > 0 ? dt * g.iDx[i] : T(0);
    const T ce = i < nx - 1 ? dt * g.iDx[i + 1] : T(0);
    const int row0 = j0 * nx + i;
    T xcol[R + 2], xwr[R], xer[R], dyr[R], iyr[R + 1];
    bool skip[R];
    xcol[0] = j0 > 0 ? xv(row0 - nx) : T(0);
#pragma unroll
    for (int k = 0; k <= R; ++k) xcol[k + 1] = xv(row0 + k * nx);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        xwr[r] = i > 0 ? xv(row0 + r * nx - 1) : T(0);
        xer[r] = i < nx - 1 ? xv(row0 + r * nx + 1) : T(0);
        dyr[r] = g.dy[j0 + r];
        skip[r] = BOX ? k0_coupled(K, i, j0 + r) : false;
    }
#pragma unroll
    for (int r = 0; r <= R; ++r) iyr[r] = g.iDy[j0 + r];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = j0 + r;
        const int row = row0 + r * nx;
        const T bw = cw * dyr[r], be = ce * dyr[r];
        const T bs = j > 0 ? dt * dxi * iyr[r] : T(0);
        const T bn = dt * dxi * iyr[r + 1];
        const T diag = ((bw + be) + bs) + bn;
        const T xc = xcol[r + 1];
        T y = diag * xc;
        if (row != K.pin) {
            if (row - nx != K.pin) y -= bs * xcol[r];
            if (row - 1 != K.pin) y -= bw * xwr[r];
            if (row + 1 != K.pin) y -= be * xer[r];
            if (row + nx != K.pin) y -= bn * xcol[r + 2];
        }
        if (!BOX || !skip[r]) act(row, y, diag, xc, pf(row));
    }
}

// Interior tile without coupled cells, east / west operands through LDS:
// every lane forms xv once at each of the R + 2 rows of its column, the R
// centre rows go to LDS, the two edge lanes form the halo columns, and the
// east / west values are read back after one barrier.  The operands the
// per-row action reads (pf) are loaded before the barrier too, so that a
// tile waits for memory once.  Every lane of the block calls this (lanes
// past the last column only take the barrier).
template <int R, class T, class XV, class PF, class ACT>
__device__ __forceinline__ void k0_tile_lds(const K0T<T> &K, int i, int j0, XV xv, PF pf, ACT act) {
    __shared__ T sh[R][kBlock + 2];
    const GridT<T> &g = K.g;
    const int nx = g.nx;
    const bool on = i < nx;
    const int ic = on ? i : nx - 1;
    const T dt = K.dt;
    const T dxi = g.dx[ic];
    const T cw = ic > 0 ? dt * g.iDx[ic] : T(0);
    const T ce = ic < nx - 1 ? dt * g.iDx[ic + 1] : T(0);
    const int row0 = j0 * nx + ic;
    T xcol[R + 2], dyr[R], iyr[R + 1];
    xcol[0] = j0 > 0 ? xv(row0 - nx) : T(0);
#pragma unroll
    for (int k = 0; k <= R; ++k) xcol[k + 1] = xv(row0 + k * nx);
    const int tx = threadIdx.x;
    T hw[R], he[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        dyr[r] = g.dy[j0 + r];
        hw[r] = (tx == 0 && ic > 0) ? xv(row0 + r * nx - 1) : T(0);
        he[r] = (tx == kBlock - 1 && ic < nx - 1) ? xv(row0 + r * nx + 1) : T(0);
    }
#pragma unroll
    for (int r = 0; r <= R; ++r) iyr[r] = g.iDy[j0 + r];
    using PV = decltype(pf(0));
    PV pv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) pv[r] = pf(row0 + r * nx);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        sh[r][tx + 1] = xcol[r + 1];
        if (tx == 0) sh[r][0] = hw[r];
        if (tx == kBlock - 1) sh[r][kBlock + 1] = he[r];
    }
    __syncthreads();
    if (!on) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = j0 + r;
        const int row = row0 + r * nx;
        // the neighbour past the last column of the grid is zero
        const T xw = ic > 0 ? sh[r][tx] : T(0);
        const T xe = ic < nx - 1 ? sh[r][tx + 2] : T(0);
        const T bw = cw * dyr[r], be = ce * dyr[r];
        const T bs = j > 0 ? dt * dxi * iyr[r] : T(0);
        const T bn = dt * dxi * iyr[r + 1];
        const T diag = ((bw + be) + bs) + bn;
        const T xc = xcol[r + 1];
        T y = diag * xc;
        if (row != K.pin) {
            if (row - nx != K.pin) y -= bs * xcol[r];
            if (row - 1 != K.pin) y -= bw * xw;
            if (row + 1 != K.pin) y -= be * xe;
            if (row + nx != K.pin) y -= bn * xcol[r + 2];
        }
        act(row, y, diag, xc, pv[r]);
    }
}

// The rows of K with stored entries, for block b of the bands at the start
// of a walker's grid: the force rows (blocks below force_blocks), then the
// coupled cells, 8 lanes per row.
template <class T, class XV, class PF, class ACT>
__device__ __forceinline__ void k0_band_rows(const K0T<T> &K, int b, XV xv, PF pf, ACT act) {
    const GridT<T> &g = K.g;
    const int nx = g.nx;
    const int fbk = force_blocks(K);
    if (b < fbk) {
        // force rows
        const int t = b * kBlock + threadIdx.x;
        const int fr = t / kForceLanes, lane = t % kForceLanes;
        const bool live = fr < 2 * K.nb;
        const T y = band_row_sum<kKfW>(live, fr, lane, K.kf_ell, K.kfe_col, K.kfe_val, K.kf, fr, 0, xv);
        if (live && lane == 0) act(g.n_cell + fr, y, K.kf_diag[fr], xv(g.n_cell + fr), pf(g.n_cell + fr));
    } else {
        // coupled cells: the stencil (every lane forms it, so its loads go
        // out with the coupling slots) plus the force coupling
        if (K.ncc == 0) return;
        const int t = (b - fbk) * kBlock + threadIdx.x;
        const int q = t / kForceLanes, lane = t % kForceLanes;
        const bool live = q < K.ncc;
        const int row = K.cc_row[live ? q : 0];
        const int j = row / nx, i = row - j * nx;
        T diag, xc;
        const T ys = k0_cell_stencil(K, i, j, xv, diag, xc);
        const int rb = (j - K.cb_j0) * (K.cb_i1 - K.cb_i0 + 1) + (i - K.cb_i0);
        const T yc = band_row_sum<kCcW>(live, q, lane, K.cc_ell, K.cce_col, K.cce_val, K.cf, rb,
                                        g.n_cell, xv);
        if (live && lane == 0) act(row, row != K.pin ? ys + yc : ys, diag, xc, pf(row));
    }
}

// Pressure and force rows of K = Q^T B^1 Q (pinned), precision T.
// act(row, Kx, diag, x_row, pf(row)) is called once per row; pf(row) loads
// what the action reads of the row besides x (before the tile's barrier).
template <int R, class T, class XV, class PF, class ACT>
__device__ __forceinline__ void k0_walk_pf(const K0T<T> &K, XV xv, PF pf, ACT act) {
    const GridT<T> &g = K.g;
    const int nx = g.nx, ny = g.ny;
    const int band = k0_band(K);
    const int b = (int)blockIdx.x;
    if (b >= band) {
        // tile of 256 columns x R rows; the tiles of one XCD are contiguous in
        // (row-band, column-chunk) order, so halos are shared through its L2
        const int cx_n = (nx + kBlock - 1) / kBlock;
        const int Gw = (int)gridDim.x - band;
        const int w = remap_block(b - band, Gw);
        const int cy = w / cx_n, cx = w - cy * cx_n;
        const int i = cx * kBlock + threadIdx.x;
        const int j0 = cy * R;
        // the same for every lane of the block
        const bool box_tile = K.ncc > 0 && j0 <= K.cb_j1 && j0 + R - 1 >= K.cb_j0 &&
                              cx * kBlock <= K.cb_i1 && cx * kBlock + kBlock - 1 >= K.cb_i0;
        if (j0 + R < ny && !box_tile && R >= 2) {
            // tiles of 2 or more rows (the large grids) exchange east / west
            // values through LDS; every lane of the block reaches its barrier
            k0_tile_lds<R>(K, i, j0, xv, pf, act);
        } else if (i < nx && j0 + R < ny) {
            if (box_tile)
                k0_tile<R, true>(K, i, j0, xv, pf, act);
            else
                k0_tile<R, false>(K, i, j0, xv, pf, act);
        } else if (i < nx && j0 < ny) {
            // top rows: one row at a time
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int j = j0 + r;
                if (j >= ny) break;
                if (box_tile && k0_coupled(K, i, j)) continue;
                T diag, xc;
                const T y = k0_cell_stencil(K, i, j, xv, diag, xc);
                act(j * nx + i, y, diag, xc, pf(j * nx + i));
            }
        }
    } else {
        k0_band_rows<T>(K, b, xv, pf, act);
    }
}

struct NoPrefetch {};

// what the update-and-sweep pass reads of its own row
template <class T>
struct UpdRow {
    T bi, w, x, p;
};

// the walk for actions that read nothing more of the row
template <int R, class T, class XV, class ACT>
__device__ __forceinline__ void k0_walk(const K0T<T> &K, XV xv, ACT act) {
    k0_walk_pf<R>(K, xv, [](int) { return NoPrefetch{}; },
                  [&](int row, T y, T d, T xc, NoPrefetch) { act(row, y, d, xc); });
}

// 1-D grid: the bands, then one block per 256 columns x R rows
template <int R, class T>
inline dim3 k0_grid(const K0T<T> &K) {
    const int cx_n = (K.g.nx + kBlock - 1) / kBlock;
    const int cy_n = (K.g.ny + R - 1) / R;
    return dim3(k0_band(K) + cx_n * cy_n);
}

// Velocity rows of A = Mf/dt - (nu/2) M Lhat R^{-1}: u faces (nx-1) x ny,
// then v faces nx x (ny-1).  Wall neighbours contribute through the
// right-hand side.
template <int R, class XV, class ACT>
__device__ __forceinline__ void a_walk(const AView &A, XV xv, ACT act) {
    const GridView &g = A.g;
    const int nx = g.nx, ny = g.ny, nxm = nx - 1;
    const double hnu = 0.5 * A.nu;
    // 1-D grid of 256-column x R-row tiles, u faces then v faces, the tiles
    // of one XCD contiguous
    const int cxu = (nxm + kBlock - 1) / kBlock, cyu = (ny + R - 1) / R;
    const int cxv = (nx + kBlock - 1) / kBlock;
    const int Gu = cxu * cyu;
    const int w = remap_block((int)blockIdx.x, (int)gridDim.x);
    if (w < Gu) {
        const int cy = w / cxu, cx = w - cy * cxu;
        const int i = cx * kBlock + threadIdx.x + 1;                   // 1..nx-1
        const int j0 = cy * R;
        if (R >= 2 && j0 + R < ny) {
            // east / west through LDS (every lane of the block comes here)
            __shared__ double sh[R][kBlock + 2];
            const int tx = threadIdx.x;
            const bool on = i <= nx - 1;
            const int ic = on ? i : nx - 1;
            const int f0 = j0 * nxm + (ic - 1);
            double xcol[R + 2];
            xcol[0] = j0 > 0 ? xv(f0 - nxm) : 0.0;
#pragma unroll
            for (int k = 0; k <= R; ++k) xcol[k + 1] = xv(f0 + k * nxm);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                sh[r][tx + 1] = xcol[r + 1];
                if (tx == 0) sh[r][0] = ic > 1 ? xv(f0 + r * nxm - 1) : 0.0;
                if (tx == kBlock - 1) sh[r][kBlock + 1] = ic < nx - 1 ? xv(f0 + r * nxm + 1) : 0.0;
            }
            const double idxi = g.idx[ic], idxm = g.idx[ic - 1], iDxi = g.iDx[ic], Dxi = g.Dx[ic];
            __syncthreads();
            if (!on) return;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int j = j0 + r;
                const double xe = ic < nx - 1 ? sh[r][tx + 2] : 0.0;
                const double xw = ic > 1 ? sh[r][tx] : 0.0;
                const double idyj = g.idy[j];
                const double xc = xcol[r + 1];
                const double uc = xc * idyj;
                const double us = j > 0 ? xcol[r] * g.idy[j - 1] : 0.0;
                const double un = xcol[r + 2] * g.idy[j + 1];
                const double uE = xe * idyj, uW = xw * idyj;
                const double lapx = ((uE - uc) * idxi - (uc - uW) * idxm) * iDxi;
                const double lapy = ((un - uc) * g.iDy[j + 1] - (uc - us) * g.iDy[j]) * idyj;
                const double mf = Dxi * idyj;
                const double diag = mf * A.idt + hnu * ((idxi + idxm) * idyj +
                                                         Dxi * (g.iDy[j + 1] + g.iDy[j]) * idyj * idyj);
                act(f0 + r * nxm, mf * A.idt * xc - hnu * (Dxi * (lapx + lapy)), diag, xc);
            }
            return;
        }
        if (i > nx - 1 || j0 >= ny) return;
        const double idxi = g.idx[i], idxm = g.idx[i - 1], iDxi = g.iDx[i], Dxi = g.Dx[i];
        const int f0 = j0 * nxm + (i - 1);
        if (j0 + R < ny) {
            double xcol[R + 2], xe[R], xw[R];
            xcol[0] = j0 > 0 ? xv(f0 - nxm) : 0.0;
#pragma unroll
            for (int k = 0; k <= R; ++k) xcol[k + 1] = xv(f0 + k * nxm);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                xe[r] = i < nx - 1 ? xv(f0 + r * nxm + 1) : 0.0;
                xw[r] = i > 1 ? xv(f0 + r * nxm - 1) : 0.0;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int j = j0 + r;
                const double idyj = g.idy[j];
                const double xc = xcol[r + 1];
                const double uc = xc * idyj;
                const double us = j > 0 ? xcol[r] * g.idy[j - 1] : 0.0;
                const double un = xcol[r + 2] * g.idy[j + 1];
                const double uE = xe[r] * idyj, uW = xw[r] * idyj;
                const double lapx = ((uE - uc) * idxi - (uc - uW) * idxm) * iDxi;
                const double lapy = ((un - uc) * g.iDy[j + 1] - (uc - us) * g.iDy[j]) * idyj;
                const double mf = Dxi * idyj;
                const double diag = mf * A.idt + hnu * ((idxi + idxm) * idyj +
                                                         Dxi * (g.iDy[j + 1] + g.iDy[j]) * idyj * idyj);
                act(f0 + r * nxm, mf * A.idt * xc - hnu * (Dxi * (lapx + lapy)), diag, xc);
            }
            return;
        }
        int f = f0;
        double us = j0 > 0 ? xv(f - nxm) * g.idy[j0 - 1] : 0.0;
        double xc = xv(f);
        double uc = xc * g.idy[j0];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int j = j0 + r;
            if (j >= ny) break;
            const double idyj = g.idy[j];
            const double xn = j < ny - 1 ? xv(f + nxm) : 0.0;
            const double un = j < ny - 1 ? xn * g.idy[j + 1] : 0.0;
            const double uE = i < nx - 1 ? xv(f + 1) * idyj : 0.0;
            const double uW = i > 1 ? xv(f - 1) * idyj : 0.0;
            const double lapx = ((uE - uc) * idxi - (uc - uW) * idxm) * iDxi;
            const double lapy = ((un - uc) * g.iDy[j + 1] - (uc - us) * g.iDy[j]) * idyj;
            const double mf = Dxi * idyj;
            const double diag = mf * A.idt + hnu * ((idxi + idxm) * idyj +
                                                     Dxi * (g.iDy[j + 1] + g.iDy[j]) * idyj * idyj);
            act(f, mf * A.idt * xc - hnu * (Dxi * (lapx + lapy)), diag, xc);
            us = uc;
            uc = un;
            xc = xn;
            f += nxm;
        }
    } else {
        const int wv = w - Gu;
        const int cy = wv / cxv, cx = wv - cy * cxv;
        const int i = cx * kBlock + threadIdx.x;                       // 0..nx-1
        const int j0 = cy * R + 1;                                     // 1..ny-1
        if (R >= 2 && j0 + R < ny) {
            // east / west through LDS (every lane of the block comes here)
            __shared__ double sh[R][kBlock + 2];
            const int tx = threadIdx.x;
            const bool on = i < nx;
            const int ic = on ? i : nx - 1;
            const int f0 = g.n_u + (j0 - 1) * nx + ic;
            double xcol[R + 2];
            xcol[0] = j0 > 1 ? xv(f0 - nx) : 0.0;
#pragma unroll
            for (int k = 0; k <= R; ++k) xcol[k + 1] = xv(f0 + k * nx);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                sh[r][tx + 1] = xcol[r + 1];
                if (tx == 0) sh[r][0] = ic > 0 ? xv(f0 + r * nx - 1) : 0.0;
                if (tx == kBlock - 1) sh[r][kBlock + 1] = ic < nx - 1 ? xv(f0 + r * nx + 1) : 0.0;
            }
            const double idxi = g.idx[ic], dxr = g.iDx[ic + 1], dxl = g.iDx[ic];
            const double idxe = ic < nx - 1 ? g.idx[ic + 1] : 0.0, idxw = ic > 0 ? g.idx[ic - 1] : 0.0;
            __syncthreads();
            if (!on) return;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int j = j0 + r;
                const double xe = ic < nx - 1 ? sh[r][tx + 2] : 0.0;
                const double xw = ic > 0 ? sh[r][tx] : 0.0;
                const double xc = xcol[r + 1];
                const double vc = xc * idxi, vs = xcol[r] * idxi, vn = xcol[r + 2] * idxi;
                const double vE = xe * idxe, vW = xw * idxw;
                const double lapx = ((vE - vc) * dxr - (vc - vW) * dxl) * idxi;
                const double lapy = ((vn - vc) * g.idy[j] - (vc - vs) * g.idy[j - 1]) * g.iDy[j];
                const double Dyj = g.Dy[j];
                const double mf = Dyj * idxi;
                const double diag = mf * A.idt + hnu * (Dyj * (dxr + dxl) * idxi * idxi +
                                                         (g.idy[j] + g.idy[j - 1]) * idxi);
                act(f0 + r * nx, mf * A.idt * xc - hnu * (Dyj * (lapx + lapy)), diag, xc);
            }
            return;
        }
        if (i >= nx || j0 > ny - 1) return;
        const double idxi = g.idx[i], dxr = g.iDx[i + 1], dxl = g.iDx[i];
        const double idxe = i < nx - 1 ? g.idx[i + 1] : 0.0, idxw = i > 0 ? g.idx[i - 1] : 0.0;
        const int f0 = g.n_u + (j0 - 1) * nx + i;
        if (j0 + R < ny) {
            double xcol[R + 2], xe[R], xw[R];
            xcol[0] = j0 > 1 ? xv(f0 - nx) : 0.0;
#pragma unroll
            for (int k = 0; k <= R; ++k) xcol[k + 1] = xv(f0 + k * nx);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                xe[r] = i < nx - 1 ? xv(f0 + r * nx + 1) : 0.0;
                xw[r] = i > 0 ? xv(f0 + r * nx - 1) : 0.0;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int j = j0 + r;
                const double xc = xcol[r + 1];
                const double vc = xc * idxi, vs = xcol[r] * idxi, vn = xcol[r + 2] * idxi;
                const double vE = xe[r] * idxe, vW = xw[r] * idxw;
                const double lapx = ((vE - vc) * dxr - (vc - vW) * dxl) * idxi;
                const double lapy = ((vn - vc) * g.idy[j] - (vc - vs) * g.idy[j - 1]) * g.iDy[j];
                const double Dyj = g.Dy[j];
                const double mf = Dyj * idxi;
                const double diag = mf * A.idt + hnu * (Dyj * (dxr + dxl) * idxi * idxi +
                                                         (g.idy[j] + g.idy[j - 1]) * idxi);
                act(f0 + r * nx, mf * A.idt * xc - hnu * (Dyj * (lapx + lapy)), diag, xc);
            }
            return;
        }
        int f = f0;
        double vs = j0 > 1 ? xv(f - nx) * idxi : 0.0;
        double xc = xv(f);
        double vc = xc * idxi;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int j = j0 + r;
            if (j > ny - 1) break;
            const double xn = j < ny - 1 ? xv(f + nx) : 0.0;
            const double vn = xn * idxi;
            const double vE = i < nx - 1 ? xv(f + 1) * idxe : 0.0;
            const double vW = i > 0 ? xv(f - 1) * idxw : 0.0;
            const double lapx = ((vE - vc) * dxr - (vc - vW) * dxl) * idxi;
            const double lapy = ((vn - vc) * g.idy[j] - (vc - vs) * g.idy[j - 1]) * g.iDy[j];
            const double Dyj = g.Dy[j];
            const double mf = Dyj * idxi;
            const double diag = mf * A.idt + hnu * (Dyj * (dxr + dxl) * idxi * idxi +
                                                     (g.idy[j] + g.idy[j - 1]) * idxi);
            act(f, mf * A.idt * xc - hnu * (Dyj * (lapx + lapy)), diag, xc);
            vs = vc;
            vc = vn;
            xc = xn;
            f += nx;
        }
    }
}

template <int R>
inline dim3 a_grid(const AView &A) {
    const int nx = A.g.nx, ny = A.g.ny;
    const int gu = ((nx - 1 + kBlock - 1) / kBlock) * ((ny + R - 1) / R);
    const int gv = ((nx + kBlock - 1) / kBlock) * ((ny - 1 + R - 1) / R);
    return dim3(gu + gv);
}

// diagonal of A for one face (used by elementwise kernels)
__device__ __forceinline__ double a_diag(const AView &A, int f) {
    const GridView &g = A.g;
    const double hnu = 0.5 * A.nu;
    if (f < g.n_u) {
        int nxm = g.nx - 1;
        int j = f / nxm;
        int i = f - j * nxm + 1;
        double idyj = g.idy[j];
        return g.Dx[i] * idyj * A.idt +
               hnu * ((g.idx[i] + g.idx[i - 1]) * idyj + g.Dx[i] * (g.iDy[j + 1] + g.iDy[j]) * idyj * idyj);
    }
    int r = f - g.n_u;
    int j = r / g.nx + 1;
    int i = r - (j - 1) * g.nx;
    double idxi = g.idx[i];
    return g.Dy[j] * idxi * A.idt +
           hnu * (g.Dy[j] * (g.iDx[i + 1] + g.iDx[i]) * idxi * idxi + (g.idy[j] + g.idy[j - 1]) * idxi);
}

template <class T>
__device__ __forceinline__ T k0_diag(const K0T<T> &K, int row) {
    const GridT<T> &g = K.g;
    if (row < g.n_cell) {
        int j = row / g.nx;
        int i = row - j * g.nx;
        T bw = i > 0 ? K.dt * g.iDx[i] * g.dy[j] : T(0);
        T be = i < g.nx - 1 ? K.dt * g.iDx[i + 1] * g.dy[j] : T(0);
        T bs = j > 0 ? K.dt * g.dx[i] * g.iDy[j] : T(0);
        T bn = j < g.ny - 1 ? K.dt * g.dx[i] * g.iDy[j + 1] : T(0);
        return ((bw + be) + bs) + bn;
    }
    return K.kf_diag[row - g.n_cell];
}

// walker dispatch over the operator type
template <int R, class T, class XV, class ACT>
__device__ __forceinline__ void op_walk(const K0T<T> &K, XV xv, ACT act) { k0_walk<R>(K, xv, act); }
template <int R, class XV, class ACT>
__device__ __forceinline__ void op_walk(const AView &A, XV xv, ACT act) { a_walk<R>(A, xv, act); }
template <class T>
__device__ __forceinline__ T op_diag(const K0T<T> &K, int r) { return k0_diag(K, r); }
__device__ __forceinline__ double op_diag(const AView &A, int r) { return a_diag(A, r); }
template <class T>
__host__ __device__ inline int op_n(const K0T<T> &K) { return K.n; }
__host__ __device__ inline int op_n(const AView &A) { return A.g.n_q; }
template <int R, class T>
inline dim3 op_grid(const K0T<T> &K) { return k0_grid<R>(K); }
template <int R>
inline dim3 op_grid(const AView &A) { return a_grid<R>(A); }

// rows r0 .. r1 - 1 of row block bi of M
template <class T>
__device__ __forceinline__ void block_rows(const CSRT<T> &M, int bi, int &r0, int &r1) {
    if (M.rpb > 0) {
        r0 = bi * M.rpb;
        r1 = min(r0 + M.rpb, M.nrows);
    } else {
        r0 = M.bst[bi];
        r1 = M.bst[bi + 1];
    }
}

// stored operator (the walk depth R does not apply): in its row blocks where
// it has them, as the CSR levels' kernels take them (every load coalesced,
// each row summed by the block's lanes), else one row per thread over the
// block's tiles, each row summed in column order
template <int R, class T, class XV, class ACT>
__device__ __forceinline__ void op_walk(const CsrOpT<T> &op, XV xv, ACT act) {
    const int n = op.A.nrows;
    if (op.A.nblk > 0) {
        __shared__ T lds[kStreamCap];
        int r0, r1;
        block_rows(op.A, remap_block(blockIdx.x, gridDim.x), r0, r1);
        const int base = op.A.ptr[r0], e = op.A.ptr[r1];
        for (int k = base + (int)threadIdx.x; k < e; k += kBlock) lds[k - base] = op.A.val[k] * xv(op.A.col[k]);
        __syncthreads();
        int L = 64;
        while (L > 1 && L * (r1 - r0) > kBlock) L >>= 1;
        const int row = r0 + (int)threadIdx.x / L, sub = (int)threadIdx.x & (L - 1);
        T sum = T(0);
        if (row < r1)
            for (int p = op.A.ptr[row] + sub; p < op.A.ptr[row + 1]; p += L) sum += lds[p - base];
        for (int o = L >> 1; o > 0; o >>= 1) sum += __shfl_xor(sum, o, L);
        if (row < r1 && sub == 0) act(row, sum, op.diag[row], xv(row));
        return;
    }
    const Tiles Tl = my_tiles(n);
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        const int row = t * kBlock + threadIdx.x;
        if (row < n) {
            T s = T(0);
            for (int p = op.A.ptr[row]; p < op.A.ptr[row + 1]; ++p) s += op.A.val[p] * xv(op.A.col[p]);
            act(row, s, op.diag[row], xv(row));
        }
    }
}
template <class T>
__device__ __forceinline__ T op_diag(const CsrOpT<T> &op, int r) { return op.diag[r]; }
template <class T>
__host__ __device__ inline int op_n(const CsrOpT<T> &op) { return op.A.nrows; }
template <int R, class T>
inline dim3 op_grid(const CsrOpT<T> &op) {
    if (op.A.nblk > 0) return dim3(op.A.nblk);
    return dim3(grid_for(op.A.nrows));
}

__device__ __forceinline__ int block_linear() { return blockIdx.y * gridDim.x + blockIdx.x; }

// Per-block partials at the linear block index (the 2-D grids)
template <int N>
__device__ __forceinline__ void write_parts2(double (&v)[N], double *parts) {
    block_sum<N>(v);
    if (threadIdx.x == 0) {
        const int b = block_linear();
#pragma unroll
        for (int k = 0; k < N; ++k) parts[k * kMaxParts + b] = v[k];
    }
}

// ---------------------------------------------------------------------------
// Krylov kernels on the level-0 operators (vectors of T; dots in FP64)

// r = b - op x; z = D^{-1} r for Jacobi; sums bb, rr, rz
template <int R, class Op, class T>
__global__ __launch_bounds__(kBlock) void k_pcg_init(Op op, const T *b, const T *x, T *r, T *z,
                                                     double *parts, int jacobi) {
    double v[3] = {0.0, 0.0, 0.0};
    op_walk<R>(op, [&](int c) { return x[c]; }, [&](int row, T ax, T d, T) {
        T bi = b[row];
        T ri = bi - ax;
        r[row] = ri;
        v[0] += (double)bi * (double)bi;
        v[1] += (double)ri * (double)ri;
        if (jacobi) {
            T zi = ri / d;
            z[row] = zi;
            v[2] += (double)ri * (double)zi;
        }
    });
    write_parts2<3>(v, parts);
}

// p_new = z + beta p_old, q = op p_new, pq = p_new . q
template <int R, class Op, class T>
__global__ __launch_bounds__(kBlock) void k_pcg_spmv(Op op, const T *__restrict__ z,
                                                     const T *__restrict__ pold,
                                                     T *__restrict__ pnew, T *__restrict__ q,
                                                     SolveStatus *st,
                                                     const double *__restrict__ rz_parts, int G_rz,
                                                     double *__restrict__ parts,
                                                     const double *__restrict__ rr_parts, int G_rr) {
    if (st->done) return;
    T beta;
    if (rz_parts) {
        // r . z of the new preconditioned residual from the preconditioner's
        // partials (every block sums them in the same order); st->rz and
        // st->first are only read here, the new value goes to st->rz_next
        const int first = st->first;
        const double rz_old = st->rz;
        double a[2] = {0.0, 0.0};
        if (rr_parts && !first) {
            gather_parts2(rz_parts, G_rz, rr_parts, G_rr, a);
        } else {
            double a0[1] = {0.0};
            gather_parts<1>(rz_parts, G_rz, 1, a0);
            a[0] = a0[0];
        }
        // with rr_parts: the stop test of the previous update (the same
        // decision in every block: it depends only on sums formed in a fixed
        // order and on fields no block of this kernel writes before reading)
        block_sum<2>(a);
        if (rr_parts && !first) {
            const double rr = a[1];
            const int stop = bad(rr) ? ST_NAN
                             : rr <= st->tol2 * st->bb ? ST_CONVERGED
                             : st->iter >= st->maxit ? ST_MAXIT : ST_RUNNING;
            if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
                st->rr = rr;
                if (stop != ST_RUNNING) st->done = stop;
            }
            if (stop != ST_RUNNING) return;
        }
        const double bt = first ? 0.0 : a[0] / rz_old;
        beta = (T)bt;
        if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
            st->rz_next = a[0];
            st->beta = bt;
        }
    } else {
        beta = (T)st->beta;
    }
    double v[1] = {0.0};
    op_walk<R>(op, [&](int c) { return z[c] + beta * pold[c]; }, [&](int row, T qi, T, T pi) {
        pnew[row] = pi;
        q[row] = qi;
        v[0] += (double)pi * (double)qi;
    });
    write_parts2<1>(v, parts);
}

// sum (b - op x)^2
template <int R, class Op, class T>
__global__ __launch_bounds__(kBlock) void k_true_residual(Op op, const T *b, const T *x,
                                                          double *parts) {
    double v[1] = {0.0};
    op_walk<R>(op, [&](int c) { return x[c]; }, [&](int row, T ax, T, T) {
        T ri = b[row] - ax;
        v[0] += (double)ri * (double)ri;
    });
    write_parts2<1>(v, parts);
}

template <int R, class Op, class T>
__global__ __launch_bounds__(kBlock) void k_apply(Op op, const T *x, T *y) {
    op_walk<R>(op, [&](int c) { return x[c]; }, [&](int row, T ax, T, T) { y[row] = ax; });
}

// x += alpha p, r -= alpha q (z = D^{-1} r for Jacobi); sums rr, rz
template <class Op, class T>
__global__ __launch_bounds__(kBlock) void k_pcg_update(Op op, T *__restrict__ x, T *__restrict__ r,
                                                       T *__restrict__ z, const T *__restrict__ p,
                                                       const T *__restrict__ q, SolveStatus *st,
                                                       const double *__restrict__ pq_parts, int G_pq,
                                                       double *__restrict__ parts, int flags) {
    if (st->done) return;
    // bit 0: Jacobi (z = D^-1 r here); bit 1: rz from the product (rz_next);
    // bit 2: deferred stop test (block 0 counts the iteration and moves
    // rz_next to rz: no block of this kernel reads iter, rz or first)
    const bool jacobi = flags & 1, fused_rz = flags & 2;
    const int n = op_n(op);
    // the status scalar and the operands of the block's first tile are read
    // before the p . q sum below, whose barriers would otherwise make every
    // later load wait for it (a clamped row where the block has none)
    const double rz = fused_rz ? st->rz_next : st->rz;
    const Tiles Tl = my_tiles(n);
    const int row0 = Tl.t0 * kBlock + threadIdx.x;
    const bool have0 = Tl.t0 < Tl.t1 && row0 < n;
    const int rc = have0 ? row0 : 0;
    const T x0 = x[rc], p0 = p[rc], r0 = r[rc], q0 = q[rc];
    // p . q from the partials of the product kernel, summed by every block in
    // the order the one-block finalize would use (so no separate launch)
    double pq;
    if (pq_parts) {
        double a[1] = {0.0};
        gather_parts<1>(pq_parts, G_pq, 1, a);
        block_sum<1>(a);
        pq = a[0];
        if (blockIdx.x == 0 && threadIdx.x == 0) st->pq = pq;
    } else {
        pq = st->pq;
    }
    const T alpha = (T)(rz / pq);
    if ((flags & 4) && blockIdx.x == 0 && threadIdx.x == 0) {
        st->iter += 1;
        st->rz = rz;
        st->first = 0;
    }
    double v[2] = {0.0, 0.0};
    auto one = [&](int row, T xi, T pi, T ri, T qi) {
        x[row] = xi + alpha * pi;
        ri = ri - alpha * qi;
        r[row] = ri;
        v[0] += (double)ri * (double)ri;
        if (jacobi) {
            T zi = ri / op_diag(op, row);
            z[row] = zi;
            v[1] += (double)ri * (double)zi;
        }
    };
    if (have0) one(row0, x0, p0, r0, q0);
    for (int t = Tl.t0 + 1; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < n) one(row, x[row], p[row], r[row], q[row]);
    }
    write_parts<2>(v, parts);
}

// ---------------------------------------------------------------------------
// V-cycle on level 0 (K0)

template <class T>
__global__ __launch_bounds__(kBlock) void k_k0_jacobi_first(K0T<T> K, T omega, const T *__restrict__ b, T *__restrict__ x,
                                                            const SolveStatus *st) {
    if (st->done) return;
    Tiles Tl = my_tiles(K.n);
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        int row = t * kBlock + threadIdx.x;
        if (row < K.n) x[row] = omega / k0_diag(K, row) * b[row];
    }
}

// coarse-grid correction on level 0 without the stored prolongator:
// x += P x1 with P = (I - w D^-1 K) T, i.e. x += t - w (K t) / d where
// t = x1[agg] is the piecewise-constant interpolation
template <int R, class T>
__global__ __launch_bounds__(kBlock) void k_k0_prolong_mf(K0T<T> K, const int *__restrict__ agg,
                                                          const T *__restrict__ x1, T w,
                                                          T *__restrict__ x, const SolveStatus *st) {
    if (st->done) return;
    k0_walk_pf<R>(K, [&](int c) { return x1[agg[c]]; }, [&](int row) { return x[row]; },
                  [&](int row, T kt, T d, T t, T xr) { x[row] = xr + (t - w * (kt / d)); });
}

// wd = omega / diag(K) on level 0
template <class T>
__global__ __launch_bounds__(kBlock) void k_k0_wdinv(K0T<T> K, T omega, T *__restrict__ wd) {
    const int row = blockIdx.x * kBlock + threadIdx.x;
    if (row < K.n) wd[row] = omega / k0_diag(K, row);
}

// the first two pre-smoothing sweeps in one pass: y = wd b (the sweep from
// zero) is formed wherever K y needs it, then x = y + wd (b - K y)
template <int R, class T>
__global__ __launch_bounds__(kBlock) void k_k0_presmooth2(K0T<T> K, const T *__restrict__ wd,
                                                          const T *__restrict__ b,
                                                          T *__restrict__ x,
                                                          const SolveStatus *st) {
    if (st->done) return;
    k0_walk<R>(K, [&](int c) { return wd[c] * b[c]; }, [&](int row, T ky, T, T yr) {
        x[row] = yr + wd[row] * (b[row] - ky);
    });
}

// The PCG update and the first two pre-smoothing sweeps of the V-cycle in
// one pass.  alpha = rz_next / (p . q), p . q summed from the product's
// partials; the new residual b = r_in - alpha q is formed wherever the sweep
// needs it and written to r_out (r_in stays intact: other blocks still read
// it), x += alpha p, xs = y + wd (b - K y) with y = wd b.  Partials of b . b
// go to parts (the next product takes the stop test), and block 0 counts
// the iteration and moves rz_next to rz (no block here reads those fields).
template <int R, class T>
__global__ __launch_bounds__(kBlock) void k_k0_update_presmooth2(
    K0T<T> K, const T *__restrict__ wd, T *__restrict__ x, const T *__restrict__ rin, T *__restrict__ rout,
    const T *__restrict__ p, const T *__restrict__ q, T *__restrict__ xs, SolveStatus *st,
    const double *__restrict__ pq_parts, int G_pq, double *__restrict__ parts) {
    if (st->done) return;
    const double rz = st->rz_next;
    double pq;
    if (pq_parts) {
        double a[1] = {0.0};
        gather_parts<1>(pq_parts, G_pq, 1, a);
        block_sum<1>(a);
        pq = a[0];
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->pq = pq;
            st->iter += 1;
            st->rz = rz;
            st->first = 0;
        }
    } else {
        // p . q and the bookkeeping from one-block finalizes around the pass
        pq = st->pq;
    }
    const T alpha = (T)(rz / pq);
    double v[1] = {0.0};
    k0_walk_pf<R>(
        K, [&](int c) { return wd[c] * (rin[c] - alpha * q[c]); },
        [&](int row) {
            UpdRow<T> u;
            u.bi = rin[row] - alpha * q[row];
            u.w = wd[row];
            u.x = x[row];
            u.p = p[row];
            return u;
        },
        [&](int row, T ky, T, T yr, UpdRow<T> u) {
            xs[row] = yr + u.w * (u.bi - ky);
            rout[row] = u.bi;
            x[row] = u.x + alpha * u.p;
            v[0] += (double)u.bi * (double)u.bi;
        });
    write_parts2<1>(v, parts);
}

// FP64 CG with an FP32 V-cycle: the FP64 update folded into the FP32 first
// pass.  b = r_in - alpha q in FP64 (to r_out, with x += alpha p and the
// partials of b . b), its FP32 rounding to r32, and the two FP32 sweeps
// from zero for it: exactly the rounding of b to FP32 followed by the FP32
// pass.
template <int R>
__global__ __launch_bounds__(kBlock) void k_k0_update_presmooth2_mixed(
    K0T<float> K, const float *__restrict__ wd, double *__restrict__ x, const double *__restrict__ rin,
    double *__restrict__ rout, const double *__restrict__ p, const double *__restrict__ q,
    float *__restrict__ xs, float *__restrict__ r32, SolveStatus *st, const double *__restrict__ pq_parts,
    int G_pq, double *__restrict__ parts) {
    if (st->done) return;
    const double rz = st->rz_next;
    double pq;
    if (pq_parts) {
        double a[1] = {0.0};
        gather_parts<1>(pq_parts, G_pq, 1, a);
        block_sum<1>(a);
        pq = a[0];
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->pq = pq;
            st->iter += 1;
            st->rz = rz;
            st->first = 0;
        }
    } else {
        pq = st->pq;
    }
    const double alpha = rz / pq;
    double v[1] = {0.0};
    k0_walk<R>(K, [&](int c) { return wd[c] * (float)(rin[c] - alpha * q[c]); },
               [&](int row, float ky, float, float yr) {
                   const double bi = rin[row] - alpha * q[row];
                   const float bf = (float)bi;
                   xs[row] = yr + wd[row] * (bf - ky);
                   r32[row] = bf;
                   rout[row] = bi;
                   x[row] += alpha * p[row];
                   v[0] += bi * bi;
               });
    write_parts2<1>(v, parts);
}

// The last FP32 post-sweep of that cycle with its result widened: z64 =
// FP64(x + omega/d (b - K x)), and the partials of r64 . z64 (the FP64
// residual), as the FP32 sweep followed by the widening would give.
template <int R>
__global__ __launch_bounds__(kBlock) void k_k0_jacobi_widen_rz(K0T<float> K, float omega,
                                                               const float *__restrict__ b,
                                                               const float *__restrict__ xin,
                                                               double *__restrict__ z64,
                                                               const double *__restrict__ r64,
                                                               const SolveStatus *st, double *parts) {
    if (st->done) return;
    double v[1] = {0.0};
    k0_walk<R>(K, [&](int c) { return xin[c]; }, [&](int row, float ax, float d, float xr) {
        const float z = xr + omega / d * (b[row] - ax);
        const double zd = (double)z;
        z64[row] = zd;
        v[0] += r64[row] * zd;
    });
    write_parts2<1>(v, parts);
}

template <int R, class T>
__global__ __launch_bounds__(kBlock) void k_k0_jacobi(K0T<T> K, T omega, const T *__restrict__ b, const T *__restrict__ xin,
                                                      T *__restrict__ xout, const SolveStatus *st) {
    if (st->done) return;
    k0_walk_pf<R>(K, [&](int c) { return xin[c]; }, [&](int row) { return b[row]; },
                  [&](int row, T ax, T d, T xr, T br) { xout[row] = xr + omega / d * (br - ax); });
}

// last post-smoothing sweep: also forms r . z for the PCG (b is the PCG residual)
template <int R, class T>
__global__ __launch_bounds__(kBlock) void k_k0_jacobi_rz(K0T<T> K, T omega, const T *__restrict__ b,
                                                         const T *__restrict__ xin, T *__restrict__ xout, SolveStatus *st,
                                                         double *parts) {
    if (st->done) return;
    double v[1] = {0.0};
    k0_walk_pf<R>(K, [&](int c) { return xin[c]; }, [&](int row) { return b[row]; },
                  [&](int row, T ax, T d, T xr, T bi) {
                      T z = xr + omega / d * (bi - ax);
                      xout[row] = z;
                      v[0] += (double)bi * (double)z;
                  });
    write_parts2<1>(v, parts);
}

template <int R, class T>
__global__ __launch_bounds__(kBlock) void k_k0_residual(K0T<T> K, const T *__restrict__ b, const T *__restrict__ x, T *__restrict__ r,
                                                        const SolveStatus *st) {
    if (st->done) return;
    k0_walk_pf<R>(K, [&](int c) { return x[c]; }, [&](int row) { return b[row]; },
                  [&](int row, T ax, T, T, T br) { r[row] = br - ax; });
}

// --- prolongation and the two post-smoothing sweeps in one pass ----------
//
// Strips: a wave takes 64 columns of cells (58 written, 3 recomputed on
// either side) and walks the RF rows of its block plus 3 above and below.
// At the step that brings in row jw it forms x' at row jw-1, y at row jw-2
// and z at row jw-3, each from the row above, the row itself and the row
// below of the previous result (kept per lane) and its east / west values
// (one lane over, by a cross-lane read): no LDS and no barrier.  The
// arithmetic of every result is that of the three passes.  Cells of the
// skipped box are left to the box passes; values the strip forms there (or
// past the grid) are dropped, and a result is only written where all it
// used lies outside the box coupled to the forces.

constexpr int kPostHalo = 3;
constexpr int kPostCols = 64 - 2 * kPostHalo;   // written columns of a wave
constexpr int kPostBlockCols = 4 * kPostCols;   // of a block
constexpr int kPostAhead = 3;                   // rows of operands in flight

// 5-point part of the pressure row `row` (the pinned row and column
// honoured), from the centre value and its south, west, east and north
// neighbours, with the same association as the walkers
template <class T>
__device__ __forceinline__ T k0_row5(int row, int nx, int pin, T diag, T bs, T bw, T be, T bn, T xc,
                                     T xs, T xw, T xe, T xn) {
    T y = diag * xc;
    if (row != pin) {
        if (row - nx != pin) y -= bs * xs;
        if (row - 1 != pin) y -= bw * xw;
        if (row + 1 != pin) y -= be * xe;
        if (row + nx != pin) y -= bn * xn;
    }
    return y;
}

// coefficients of the pressure row of cell (column with dxi, cw, ce; row j)
template <class T>
struct Row5 {
    T bs, bw, be, bn, diag;
};
template <class T>
__device__ __forceinline__ Row5<T> k0_coef(const GridT<T> &g, T dt, T dxi, T cw, T ce, int j) {
    Row5<T> c;
    const T dyj = g.dy[j];
    c.bw = cw * dyj;
    c.be = ce * dyj;
    c.bs = j > 0 ? dt * dxi * g.iDy[j] : T(0);
    c.bn = j < g.ny - 1 ? dt * dxi * g.iDy[j + 1] : T(0);
    c.diag = ((c.bw + c.be) + c.bs) + c.bn;
    return c;
}

__device__ __forceinline__ bool in_rect(const CellRect &r, int i, int j) {
    return i >= r.i0 && i <= r.i1 && j >= r.j0 && j <= r.j1;
}

// value of lane k (uniform k) of v
__device__ __forceinline__ double lane_value(double v, int k) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_value(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

// The level-0 rows of a rectangle of cells (one thread per cell; coupled
// cells are left to the band) and the band rows.
template <class T, class XV, class PF, class ACT>
__device__ __forceinline__ void k0_walk_rect(const K0T<T> &K, CellRect rc, XV xv, PF pf, ACT act) {
    const int band = k0_band(K);
    const int b = (int)blockIdx.x;
    if (b < band) {
        k0_band_rows<T>(K, b, xv, pf, act);
        return;
    }
    const int wdt = rc.i1 - rc.i0 + 1;
    const int idx = (b - band) * kBlock + threadIdx.x;
    if (wdt <= 0 || idx >= wdt * (rc.j1 - rc.j0 + 1)) return;
    const int j = rc.j0 + idx / wdt, i = rc.i0 + idx % wdt;
    if (k0_coupled(K, i, j)) return;
    T diag, xc;
    const T y = k0_cell_stencil(K, i, j, xv, diag, xc);
    const int row = j * K.g.nx + i;
    act(row, y, diag, xc, pf(row));
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_k0_jacobi_rect(K0T<T> K, CellRect rc, T omega,
                                                           const T *__restrict__ b, const T *__restrict__ xin,
                                                           T *__restrict__ xout, const SolveStatus *st) {
    if (st->done) return;
    k0_walk_rect(K, rc, [&](int c) { return xin[c]; }, [&](int row) { return b[row]; },
                 [&](int row, T ax, T d, T xr, T br) { xout[row] = xr + omega / d * (br - ax); });
}

template <int MODE, class T>
__global__ __launch_bounds__(kBlock) void k_k0_jacobi_last_rect(K0T<T> K, CellRect rc, T omega,
                                                                const T *__restrict__ b,
                                                                const T *__restrict__ xin, T *__restrict__ z,
                                                                double *__restrict__ z64,
                                                                const double *__restrict__ r64,
                                                                const SolveStatus *st, double *parts) {
    if (st->done) return;
    double v[1] = {0.0};
    k0_walk_rect(K, rc, [&](int c) { return xin[c]; }, [&](int row) { return b[row]; },
                 [&](int row, T ax, T d, T xr, T br) {
                     const T zz = xr + omega / d * (br - ax);
                     if constexpr (MODE == POST_WIDEN) {
                         const double zd = (double)zz;
                         z64[row] = zd;
                         v[0] += r64[row] * zd;
                     } else {
                         z[row] = zz;
                         if constexpr (MODE == POST_RZ) v[0] += (double)br * (double)zz;
                     }
                 });
    if constexpr (MODE != POST_PLAIN) write_parts2<1>(v, parts);
}

template <int RF, int MODE, class T>
__global__ __launch_bounds__(kBlock) void k_k0_prolong_post2(
    K0T<T> K, CellRect skip, const int *__restrict__ agg, const T *__restrict__ x1, T pw, T omega,
    const T *__restrict__ b, const T *__restrict__ a, T *__restrict__ z, double *__restrict__ z64,
    const double *__restrict__ r64, const SolveStatus *st, double *parts, CellRect r2, T *__restrict__ tmp,
    int G2) {
    constexpr int NS = RF + 2 * kPostHalo;       // rows walked
    constexpr int D = kPostAhead;
    static_assert(NS + 1 <= 64, "the row metrics of a walk are held one row per lane");
    if (st->done) return;
    if ((int)blockIdx.x < G2) {
        // the first G2 blocks (dispatched first: their rows reach through
        // gathers) form x' on the box grown by 5 and the force rows, into tmp
        k0_walk_rect(K, r2, [&](int c) { return x1[agg[c]]; }, [&](int row) { return a[row]; },
                     [&](int row, T kt, T d, T t, T ar) { tmp[row] = ar + (t - pw * (kt / d)); });
        return;
    }
    const GridT<T> &g = K.g;
    const int nx = g.nx, ny = g.ny, pin = K.pin;
    const int ncs = (nx + kPostBlockCols - 1) / kPostBlockCols;
    const int sb = (int)blockIdx.x - G2;         // strip block
    const int w = remap_block(sb, (int)gridDim.x - G2);
    const int cy = w / ncs, cx = w - cy * ncs;
    const int lane = threadIdx.x & 63;
    const int i = cx * kPostBlockCols + (threadIdx.x >> 6) * kPostCols - kPostHalo + lane;
    const int j0 = cy * RF;
    const int jt = j0 - kPostHalo;               // row of walk step 0
    const bool cin = i >= 0 && i < nx;
    const int ic = cin ? i : (i < 0 ? 0 : nx - 1);
    const T dt = K.dt;
    const T dxi = g.dx[ic];
    const T cw = (cin && i > 0) ? dt * g.iDx[ic] : T(0);
    const T ce = (cin && i < nx - 1) ? dt * g.iDx[ic + 1] : T(0);
    const T cs = dt * dxi;
    const bool wcol = cin && lane >= kPostHalo && lane < 64 - kPostHalo;
    // lane k holds dy and iDy of walk row k (clamped to the grid)
    T dyl, iyl;
    {
        const int jl = jt + lane;
        dyl = g.dy[jl < 0 ? 0 : (jl > ny - 1 ? ny - 1 : jl)];
        iyl = g.iDy[jl < 0 ? 0 : (jl > ny ? ny : jl)];
    }
    // Operand loads are unconditional, from the clamped cell, and zeroed
    // where they are used, so that no branch or copy makes a step wait for
    // loads still in flight: slot s % D holds the operands of walk row s,
    // issued D steps ahead, and the aggregates D steps before that.
    auto live = [&](int sr) { return cin && jt + sr >= 0 && jt + sr < ny; };
    auto rix = [&](int sr) {
        const int jr = jt + sr;
        return (jr < 0 ? 0 : (jr > ny - 1 ? ny - 1 : jr)) * nx + ic;
    };
    constexpr bool widen = MODE == POST_WIDEN;
    T ft[D], fa[D], fb[D];
    double fr[D];                                // widen: the FP64 residual
    int fg[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int rw = rix(k);
        ft[k] = x1[agg[rw]];
        fa[k] = a[rw];
        fb[k] = b[rw];
        fr[k] = widen ? r64[rw] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) fg[k] = agg[rix(D + k)];
    // per lane: t at rows jw-2, jw-1; a at jw-1; b at jw-1..jw-3; x' at
    // jw-2, jw-3; y at jw-3, jw-4 (zero outside the grid); the diagonal and
    // omega / diagonal of rows jw-2 and jw-3
    T tm2 = T(0), tm1 = T(0), am1 = T(0), bm1 = T(0), bm2 = T(0), bm3 = T(0);
    T pm2 = T(0), pm3 = T(0), qm3 = T(0), qm4 = T(0);
    T d2 = T(1), d3 = T(1), o2 = T(0), o3 = T(0);
    double rm1 = 0.0, rm2 = 0.0, rm3 = 0.0;     // widen: r64 at rows jw-1..jw-3
    double v = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int jw = jt + s;
        const int sl = s % D;
        const bool ls = live(s);
        const T t0 = ls ? ft[sl] : T(0), a0 = ls ? fa[sl] : T(0), b0 = ls ? fb[sl] : T(0);
        const double r0 = widen ? fr[sl] : 0.0;
        if (s + D < NS) {
            const int rw = rix(s + D);
            ft[sl] = x1[fg[sl]];
            fa[sl] = a[rw];
            fb[sl] = b[rw];
            if (widen) fr[sl] = r64[rw];
            if (s + 2 * D < NS) fg[sl] = agg[rix(s + 2 * D)];
        }
        const T tw = __shfl_up(tm1, 1, 64), te = __shfl_down(tm1, 1, 64);
        const T pwv = __shfl_up(pm2, 1, 64), pev = __shfl_down(pm2, 1, 64);
        const T qw = __shfl_up(qm3, 1, 64), qe = __shfl_down(qm3, 1, 64);
        // coefficients of walk row s - 1 (the walkers' association) and of
        // rows s - 2, s - 3 (their diagonals kept from earlier steps)
        auto coef = [&](int k, T &bs, T &bw, T &be, T &bn) {
            const int j = jt + k;
            const T dyj = lane_value(dyl, k);
            bw = cw * dyj;
            be = ce * dyj;
            bs = j > 0 ? cs * lane_value(iyl, k) : T(0);
            bn = j < ny - 1 ? cs * lane_value(iyl, k + 1) : T(0);
        };
        T p1 = T(0), d1 = T(1), o1 = T(0);
        if (s >= 1) {
            // x' = a + (t - pw (K t) / d) at row jw - 1
            T bs, bw, be, bn;
            coef(s - 1, bs, bw, be, bn);
            d1 = ((bw + be) + bs) + bn;
            o1 = omega / d1;
            const int j = jw - 1;
            const T kt = k0_row5(j * nx + i, nx, pin, d1, bs, bw, be, bn, tm1, tm2, tw, te, t0);
            const T pv = am1 + (tm1 - pw * (kt / d1));
            p1 = (cin && j >= 0 && j < ny) ? pv : T(0);
        }
        T q1 = T(0);
        if (s >= 2) {
            // y = x' + omega / d (b - K x') at row jw - 2
            T bs, bw, be, bn;
            coef(s - 2, bs, bw, be, bn);
            const int j = jw - 2;
            const T kp = k0_row5(j * nx + i, nx, pin, d2, bs, bw, be, bn, pm2, pm3, pwv, pev, p1);
            const T qv = pm2 + o2 * (bm2 - kp);
            q1 = (cin && j >= 0 && j < ny) ? qv : T(0);
        }
        if (s >= 3) {
            // z = y + omega / d (b - K y) at row jw - 3, written in the strip
            const int j = jw - 3;
            if (j >= j0 && wcol && j < ny && !in_rect(skip, i, j)) {
                T bs, bw, be, bn;
                coef(s - 3, bs, bw, be, bn);
                const int row = j * nx + i;
                const T kq = k0_row5(row, nx, pin, d3, bs, bw, be, bn, qm3, qm4, qw, qe, q1);
                const T zz = qm3 + o3 * (bm3 - kq);
                if constexpr (MODE == POST_WIDEN) {
                    const double zd = (double)zz;
                    z64[row] = zd;
                    v += rm3 * zd;
                } else {
                    z[row] = zz;
                    if constexpr (MODE == POST_RZ) v += (double)bm3 * (double)zz;
                }
            }
        }
        rm3 = rm2;
        rm2 = rm1;
        rm1 = r0;
        tm2 = tm1;
        tm1 = t0;
        am1 = a0;
        bm3 = bm2;
        bm2 = bm1;
        bm1 = b0;
        pm3 = pm2;
        pm2 = p1;
        qm4 = qm3;
        qm3 = q1;
        d3 = d2;
        d2 = d1;
        o3 = o2;
        o2 = o1;
    }
    if constexpr (MODE != POST_PLAIN) {
        double vv[1] = {v};
        block_sum<1>(vv);
        if (threadIdx.x == 0) parts[sb] = vv[0];
    }
}

// mixed precision outer loop: r = b - K x in FP64, r32 = (float) r, ||r||^2, ||b||^2
template <int R>
__global__ __launch_bounds__(kBlock) void k_outer_residual(K0View K, const double *b,
                                                           const double *x, float *r32,
                                                           double *parts) {
    double v[2] = {0.0, 0.0};
    k0_walk<R>(K, [&](int c) { return x[c]; }, [&](int row, double ax, double, double) {
        double bi = b[row];
        double ri = bi - ax;
        r32[row] = (float)ri;
        v[0] += ri * ri;
        v[1] += bi * bi;
    });
    write_parts2<2>(v, parts);
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
    write_parts<1>(v, parts);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_zero_if_zero_rhs(T *x, int n, const SolveStatus *st) {
    if (st->done != ST_ZERO_RHS) return;
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = T(0);
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
    write_parts<1>(v, parts);
}

// Grid-wide sums of the partials written by the previous kernel (G blocks)
// and the status update that goes with them.  One block.
enum : int {
    FIN_INIT = 0, FIN_INIT_ZERO, FIN_PQ, FIN_UPDATE, FIN_TRUE, FIN_RZ, FIN_OUTER,
    FIN_OMEGA, FIN_RZ_NEXT
};

__global__ __launch_bounds__(kBlock) void k_finalize(int kind, int G, const double *parts,
                                                     SolveStatus *st, int flag, double rtol2,
                                                     int maxit) {
    if ((kind == FIN_PQ || kind == FIN_UPDATE || kind == FIN_RZ || kind == FIN_RZ_NEXT) && st->done)
        return;
    const int N = (kind == FIN_INIT) ? 3
                  : (kind == FIN_UPDATE || kind == FIN_OUTER || kind == FIN_OMEGA)
                      ? 2
                      : 1;
    double acc[3] = {0.0, 0.0, 0.0};
    gather_parts<3>(parts, G, N, acc);
    block_sum<3>(acc);
    if (threadIdx.x != 0) return;
    switch (kind) {
    case FIN_INIT:   // acc = (bb, rr, rz); flag = jacobi
        st->bb = acc[0];
        st->rr = acc[1];
        st->tol2 = rtol2;
        st->maxit = maxit;
        st->iter = 0;
        st->beta = 0.0;
        st->first = 1;
        st->done = ST_RUNNING;
        if (acc[0] == 0.0) st->done = ST_ZERO_RHS;
        else if (bad(acc[1])) st->done = ST_NAN;
        else if (acc[1] <= rtol2 * acc[0]) st->done = ST_CONVERGED;
        if (flag) {
            st->rz = acc[2];
            st->first = 0;
        }
        break;
    case FIN_INIT_ZERO:   // acc = (bb)
        st->bb = acc[0];
        st->rr = acc[0];
        st->tol2 = rtol2;
        st->maxit = maxit;
        st->iter = 0;
        st->beta = 0.0;
        st->first = 1;
        st->done = acc[0] == 0.0 ? ST_ZERO_RHS : (bad(acc[0]) ? ST_NAN : ST_RUNNING);
        break;
    case FIN_PQ:
        st->pq = acc[0];
        break;
    case FIN_UPDATE:   // acc = (rr, rz); flag bit 0: Jacobi (rz here), bit 1: rz from the product
        st->rr = acc[0];
        st->iter += 1;
        if (bad(acc[0])) st->done = ST_NAN;
        else if (acc[0] <= st->tol2 * st->bb) st->done = ST_CONVERGED;
        else if (st->iter >= st->maxit) st->done = ST_MAXIT;
        if (flag & 1) {
            st->beta = acc[1] / st->rz;
            st->rz = acc[1];
        }
        if (flag & 2) {
            st->rz = st->rz_next;
            st->first = 0;
        }
        break;
    case FIN_TRUE:
        st->true_rr = acc[0];
        break;
    case FIN_RZ_NEXT:   // as the product kernel's own sum of the r . z partials
        st->beta = st->first ? 0.0 : acc[0] / st->rz;
        st->rz_next = acc[0];
        break;
    case FIN_RZ:
        if (st->first) {
            st->beta = 0.0;
            st->first = 0;
        } else {
            st->beta = acc[0] / st->rz;
        }
        st->rz = acc[0];
        break;
    case FIN_OMEGA: {  // acc = (d.r1, d.K d): energy-optimal weight of the learned correction
        double w = (acc[1] > 0.0 && !bad(acc[0]) && !bad(acc[1])) ? acc[0] / acc[1] : 0.0;
        st->beta = w;
        break;
    }
    case FIN_OUTER:   // acc = (rr, bb); flag = first outer residual
        st->rr = acc[0];
        if (flag) {
            st->bb = acc[1];
            st->iter = 0;
        } else {
            st->iter += 1;
        }
        break;
    }
}

// ---------------------------------------------------------------------------
// flexible CG with the learned stage

// --- FCG(m) -----------------------------------------------------------------

template <class T>
__global__ __launch_bounds__(kBlock) void k_fcg_multidot(int n, const T *__restrict__ z,
                                                         FcgVecs<T> Q, int cnt, FcgSlots sl,
                                                         const SolveStatus *st, double *parts) {
    if (st->done) return;
    Tiles Tl = my_tiles(n);
    double v[kFcgMax];
#pragma unroll
    for (int j = 0; j < kFcgMax; ++j) v[j] = 0.0;
    for (int t = Tl.t0; t < Tl.t1; ++t) {
        const int row = t * kBlock + threadIdx.x;
        if (row < n) {
            const double zr = (double)z[row];
#pragma unroll
            for (int j = 0; j < kFcgMax; ++j)
                if (j < cnt) v[j] += zr * (double)Q.v[sl.s[j]][row];
        }
    }
    write_parts<kFcgMax>(v, parts);
}

__global__ __launch_bounds__(kBlock) void k_fcg_betas_finalize(int G, int cnt, FcgSlots sl,
                                                               const double *parts, FcgRing *ring,
                                                               const SolveStatus *st) {
    if (st->done) return;
    double acc[kFcgMax];
#pragma unroll
    for (int j = 0; j < kFcgMax; ++j) acc[j] = 0.0;
    gather_parts<kFcgMax>(parts, G, cnt, acc);
    block_sum<kFcgMax>(acc);
    if (threadIdx.x == 0)
        for (int j = 0; j < cnt; ++j) {
            const double pq = ring->pq[sl.s[j]];
            ring->beta[j] = pq != 0.0 ? -acc[j] / pq : 0.0;
        }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_fcg_direction(int n, const T *__restrict__ z,
                                                          FcgVecs<T> P, int cnt, FcgSlots sl,
                                                          const FcgRing *ring, T *p,
                                                          const SolveStatus *st) {
    // p may be the slot of the oldest direction in the window: each element
    // is read before it is overwritten, by the same thread
    if (st->done) return;
    const int i = tile_base() + threadIdx.x;
    if (i >= n) return;
    T v = z[i];
    for (int j = 0; j < cnt; ++j) v += (T)ring->beta[j] * P.v[sl.s[j]][i];
    p[i] = v;
}

template <int R, class T>
__global__ __launch_bounds__(kBlock) void k_fcg_product(K0T<T> K, const T *__restrict__ p,
                                                        T *__restrict__ q, const T *__restrict__ r,
                                                        const SolveStatus *st, double *parts) {
    if (st->done) return;
    double v[2] = {0.0, 0.0};
    k0_walk<R>(K, [&](int c) { return p[c]; }, [&](int row, T qi, T, T pi) {
        q[row] = qi;
        v[0] += (double)pi * (double)qi;
        v[1] += (double)pi * (double)r[row];
    });
    write_parts2<2>(v, parts);
}

__global__ __launch_bounds__(kBlock) void k_fcg_pq_finalize(int G, const double *parts, int slot,
                                                            FcgRing *ring, SolveStatus *st) {
    if (st->done) return;
    double acc[2] = {0.0, 0.0};
    gather_parts<2>(parts, G, 2, acc);
    block_sum<2>(acc);
    if (threadIdx.x == 0) {
        st->pq = acc[0];
        st->rz = acc[1];
        ring->pq[slot] = acc[0];
    }
}

// sums d.r1 and d.(K d)
template <int R, class T>
__global__ __launch_bounds__(kBlock) void k_kd_dots(K0T<T> K, const T *__restrict__ d,
                                                    const T *__restrict__ r1, const SolveStatus *st,
                                                    double *parts) {
    if (st->done) return;
    double v[2] = {0.0, 0.0};
    k0_walk<R>(K, [&](int c) { return d[c]; }, [&](int row, T kd, T, T dr) {
        v[0] += (double)dr * (double)r1[row];
        v[1] += (double)dr * (double)kd;
    });
    write_parts2<2>(v, parts);
}

// z = z0 + omega d (omega from the learned-stage status); omega = 0 drops the
// correction altogether, so a non-finite network output never reaches z.
// z may be z0 (in-place update).
template <class T>
__global__ __launch_bounds__(kBlock) void k_axpy_omega(int n, const T *z0, const T *d,
                                                       const SolveStatus *stw, T *z,
                                                       const SolveStatus *st) {
    if (st->done) return;
    const int i = tile_base() + threadIdx.x;
    const T w = (T)stw->beta;
    if (i < n) z[i] = w != T(0) ? z0[i] + w * d[i] : z0[i];
}

// harvest: e1 = x* - x - z in FP32
__global__ __launch_bounds__(kBlock) void k_harvest_e1(int n, const double *xstar, const double *x,
                                                       const double *z, float *e1) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) e1[i] = (float)(xstar[i] - x[i] - z[i]);
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
// CSR with a subgroup of L lanes per row: lane k takes entries k, k+L, ...,
// then a butterfly over the subgroup (fixed order, so deterministic)

// sum over the row's entries [p0, e) of val * xv(col), L lanes per row:
// each lane takes entries lane, lane + L, ... two per round with both
// rounds' loads issued together (rows up to 2L long take one round), in the
// same order as one entry per round; then a butterfly over the L lanes
template <class T, int L, class XV>
__device__ __forceinline__ T csrv_sum(const CSRT<T> &A, int p0, int e, int lane, XV xv) {
    T y = T(0);
    for (int p = p0 + lane; p < e; p += 2 * L) {
        const bool h1 = p + L < e;
        const int q = h1 ? p + L : p;
        const int c0 = A.col[p], c1 = A.col[q];
        const T v0 = A.val[p], v1 = A.val[q];
        const T x0 = xv(c0), x1 = xv(c1);
        y += v0 * x0;
        const T y1 = y + v1 * x1;
        y = h1 ? y1 : y;
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) y += __shfl_xor(y, off, L);
    return y;
}

// The row's own operands are loaded by every lane of the row before the
// sum, so that their latency overlaps the gather's.
template <class T, int L>
__global__ __launch_bounds__(kBlock) void k_csrv_jacobi(CSRT<T> A, const T *__restrict__ wdinv, const T *__restrict__ b,
                                                        const T *__restrict__ xin, T *__restrict__ xout,
                                                        const SolveStatus *st) {
    if (st->done) return;
    const int row = remap_block(blockIdx.x, gridDim.x) * (kBlock / L) + threadIdx.x / L;
    const int lane = threadIdx.x % L;
    if (row >= A.nrows) return;
    const T xr = xin[row], wr = wdinv[row], br = b[row];
    const T ax = csrv_sum<T, L>(A, A.ptr[row], A.ptr[row + 1], lane, [&](int c) { return xin[c]; });
    if (lane == 0) xout[row] = xr + wr * (br - ax);
}

template <class T, int L>
__global__ __launch_bounds__(kBlock) void k_csrv_residual(CSRT<T> A, const T *__restrict__ b, const T *__restrict__ x, T *__restrict__ r,
                                                          const SolveStatus *st) {
    if (st->done) return;
    const int row = remap_block(blockIdx.x, gridDim.x) * (kBlock / L) + threadIdx.x / L;
    const int lane = threadIdx.x % L;
    if (row >= A.nrows) return;
    const T br = b[row];
    const T ax = csrv_sum<T, L>(A, A.ptr[row], A.ptr[row + 1], lane, [&](int c) { return x[c]; });
    if (lane == 0) r[row] = br - ax;
}

template <class T, int L>
__global__ __launch_bounds__(kBlock) void k_csrv_spmv(CSRT<T> A, const T *__restrict__ x, T *__restrict__ y, int add,
                                                      const SolveStatus *st) {
    if (st && st->done) return;
    const int row = remap_block(blockIdx.x, gridDim.x) * (kBlock / L) + threadIdx.x / L;
    const int lane = threadIdx.x % L;
    if (row >= A.nrows) return;
    const T yr = add ? y[row] : T(0);
    const T v = csrv_sum<T, L>(A, A.ptr[row], A.ptr[row + 1], lane, [&](int c) { return x[c]; });
    if (lane == 0) y[row] = add ? yr + v : v;
}

// the first two damped-Jacobi sweeps from zero in one pass on a CSR level:
// x = y + W (b - A y) with y = W b formed at every column
template <class T, int L>
__global__ __launch_bounds__(kBlock) void k_csrv_presmooth2(CSRT<T> A, const T *__restrict__ wdinv,
                                                            const T *__restrict__ b,
                                                            T *__restrict__ x,
                                                            const SolveStatus *st) {
    if (st->done) return;
    const int row = remap_block(blockIdx.x, gridDim.x) * (kBlock / L) + threadIdx.x / L;
    const int lane = threadIdx.x % L;
    if (row >= A.nrows) return;
    const T w = wdinv[row], bi = b[row];
    const T ay = csrv_sum<T, L>(A, A.ptr[row], A.ptr[row + 1], lane,
                                [&](int c) { return wdinv[c] * b[c]; });
    if (lane == 0) x[row] = w * bi + w * (bi - ay);
}

// Restriction with the residual folded in: b_c = (R b)_c - (R A x)_c, the
// two rows walked in one loop (L lanes per coarse row; entry k of each row
// taken by lane k mod L, both matrices' loads of a round issued together)
template <class T, int L>
__global__ __launch_bounds__(kBlock) void k_csrv_restrict(CSRT<T> R, CSRT<T> RA, const T *__restrict__ b,
                                                          const T *__restrict__ x, T *__restrict__ bc,
                                                          const SolveStatus *st) {
    if (st->done) return;
    const int row = remap_block(blockIdx.x, gridDim.x) * (kBlock / L) + threadIdx.x / L;
    const int lane = threadIdx.x % L;
    if (row >= R.nrows) return;
    const int r0 = R.ptr[row], nr = R.ptr[row + 1] - r0;
    const int a0 = RA.ptr[row], na = RA.ptr[row + 1] - a0;
    const int nm = nr > na ? nr : na;
    T sr = T(0), sa = T(0);
    for (int k = lane; k < nm; k += L) {
        // a slot past the end of its row reads entry 0 (every array holds
        // at least one element) and gathers column 0; its term is dropped
        const bool hr = k < nr, ha = k < na;
        const int pr = hr ? r0 + k : 0, pa = ha ? a0 + k : 0;
        const int cr0 = R.col[pr], ca0 = RA.col[pa];
        const int cr = hr ? cr0 : 0, ca = ha ? ca0 : 0;
        const T vr = R.val[pr], va = RA.val[pa];
        const T xr = b[cr], xa = x[ca];
        const T tr = sr + vr * xr, ta = sa + va * xa;
        sr = hr ? tr : sr;
        sa = ha ? ta : sa;
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) {
        sr += __shfl_xor(sr, off, L);
        sa += __shfl_xor(sa, off, L);
    }
    if (lane == 0) bc[row] = sr - sa;
}

// Prolongation and the first post-sweep in one pass:
// x_out = x + P e + W (b - A x - (A P) e), the three rows walked in one loop
template <class T, int L>
__global__ __launch_bounds__(kBlock) void k_csrv_prolong_jacobi(CSRT<T> A, CSRT<T> AP, CSRT<T> P,
                                                                const T *__restrict__ wdinv,
                                                                const T *__restrict__ b,
                                                                const T *__restrict__ x,
                                                                const T *__restrict__ e,
                                                                T *__restrict__ xout,
                                                                const SolveStatus *st) {
    if (st->done) return;
    const int row = remap_block(blockIdx.x, gridDim.x) * (kBlock / L) + threadIdx.x / L;
    const int lane = threadIdx.x % L;
    if (row >= A.nrows) return;
    const T xr = x[row], wr = wdinv[row], br = b[row];
    const int a0 = A.ptr[row], na = A.ptr[row + 1] - a0;
    const int q0 = AP.ptr[row], nq = AP.ptr[row + 1] - q0;
    const int p0 = P.ptr[row], np = P.ptr[row + 1] - p0;
    int nm = na > nq ? na : nq;
    nm = nm > np ? nm : np;
    T sa = T(0), sq = T(0), sp = T(0);
    for (int k = lane; k < nm; k += L) {
        // slots past the end of a row: entry 0 and column 0, term dropped
        const bool ha = k < na, hq = k < nq, hp = k < np;
        const int pa = ha ? a0 + k : 0, pq = hq ? q0 + k : 0, pp = hp ? p0 + k : 0;
        const int ca0 = A.col[pa], cq0 = AP.col[pq], cp0 = P.col[pp];
        const int ca = ha ? ca0 : 0, cq = hq ? cq0 : 0, cp = hp ? cp0 : 0;
        const T va = A.val[pa], vq = AP.val[pq], vp = P.val[pp];
        const T xa = x[ca], eq = e[cq], ep = e[cp];
        const T ta = sa + va * xa, tq = sq + vq * eq, tp = sp + vp * ep;
        sa = ha ? ta : sa;
        sq = hq ? tq : sq;
        sp = hp ? tp : sp;
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) {
        sa += __shfl_xor(sa, off, L);
        sq += __shfl_xor(sq, off, L);
        sp += __shfl_xor(sp, off, L);
    }
    if (lane == 0) xout[row] = (xr + sp) + wr * ((br - sa) - sq);
}

// ---------------------------------------------------------------------------
// Stored-operator kernels in row blocks (the CSR levels of the V-cycle): a
// block takes a run of consecutive rows (its row block, formed on the host:
// at most kBlock rows whose entries, of every matrix the kernel walks, fit
// kStreamCap), streams their entries -- all threads of the block over one
// contiguous range of the value and column arrays, so every load is
// coalesced -- multiplies each by the gathered operand into LDS, and then
// sums each row with L lanes, the largest power of two (at most 64) with L
// times the block's rows within kBlock: lane k adds the row's products k,
// k + L, ... and the lanes are combined by a butterfly, so every thread of
// the block takes part whatever the row length.

template <class T, class XV>
__device__ __forceinline__ void stream_fill(const CSRT<T> &A, int r0, int r1, T *lds, XV xv) {
    const int base = A.ptr[r0], e = A.ptr[r1];
    for (int k = base + (int)threadIdx.x; k < e; k += kBlock) lds[k - base] = A.val[k] * xv(A.col[k]);
}

// lanes per row and this thread's row and lane within it
struct StreamLane {
    int L, row, sub;
    bool live;
};

__device__ __forceinline__ StreamLane stream_lane(int r0, int r1) {
    StreamLane sl;
    sl.L = 64;
    while (sl.L > 1 && sl.L * (r1 - r0) > kBlock) sl.L >>= 1;
    sl.row = r0 + (int)threadIdx.x / sl.L;
    sl.sub = (int)threadIdx.x & (sl.L - 1);
    sl.live = sl.row < r1;
    return sl;
}

// the sum of a row's products (every lane of the block calls this)
template <class T>
__device__ __forceinline__ T stream_row(const CSRT<T> &A, const StreamLane &sl, int base, const T *lds) {
    T s = T(0);
    if (sl.live) {
        const int e = A.ptr[sl.row + 1];
        for (int p = A.ptr[sl.row] + sl.sub; p < e; p += sl.L) s += lds[p - base];
    }
    for (int o = sl.L >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, sl.L);
    return s;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_csrs_jacobi(CSRT<T> A, const T *__restrict__ wdinv,
                                                        const T *__restrict__ b, const T *__restrict__ xin,
                                                        T *__restrict__ xout, const SolveStatus *st) {
    if (st->done) return;
    __shared__ T lds[kStreamCap];
    int r0, r1;
    block_rows(A, remap_block(blockIdx.x, gridDim.x), r0, r1);
    stream_fill(A, r0, r1, lds, [&](int c) { return xin[c]; });
    __syncthreads();
    const StreamLane sl = stream_lane(r0, r1);
    const T ax = stream_row(A, sl, A.ptr[r0], lds);
    if (sl.live && sl.sub == 0) xout[sl.row] = xin[sl.row] + wdinv[sl.row] * (b[sl.row] - ax);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_csrs_residual(CSRT<T> A, const T *__restrict__ b,
                                                          const T *__restrict__ x, T *__restrict__ r,
                                                          const SolveStatus *st) {
    if (st->done) return;
    __shared__ T lds[kStreamCap];
    int r0, r1;
    block_rows(A, remap_block(blockIdx.x, gridDim.x), r0, r1);
    stream_fill(A, r0, r1, lds, [&](int c) { return x[c]; });
    __syncthreads();
    const StreamLane sl = stream_lane(r0, r1);
    const T ax = stream_row(A, sl, A.ptr[r0], lds);
    if (sl.live && sl.sub == 0) r[sl.row] = b[sl.row] - ax;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_csrs_spmv(CSRT<T> A, const T *__restrict__ x,
                                                      T *__restrict__ y, int add, const SolveStatus *st) {
    if (st && st->done) return;
    __shared__ T lds[kStreamCap];
    int r0, r1;
    block_rows(A, remap_block(blockIdx.x, gridDim.x), r0, r1);
    stream_fill(A, r0, r1, lds, [&](int c) { return x[c]; });
    __syncthreads();
    const StreamLane sl = stream_lane(r0, r1);
    const T v = stream_row(A, sl, A.ptr[r0], lds);
    if (sl.live && sl.sub == 0) y[sl.row] = add ? y[sl.row] + v : v;
}

// the first two damped-Jacobi sweeps from zero: x = y + W (b - A y), y = W b
template <class T>
__global__ __launch_bounds__(kBlock) void k_csrs_presmooth2(CSRT<T> A, const T *__restrict__ wdinv,
                                                            const T *__restrict__ b, T *__restrict__ x,
                                                            const SolveStatus *st) {
    if (st->done) return;
    __shared__ T lds[kStreamCap];
    int r0, r1;
    block_rows(A, remap_block(blockIdx.x, gridDim.x), r0, r1);
    stream_fill(A, r0, r1, lds, [&](int c) { return wdinv[c] * b[c]; });
    __syncthreads();
    const StreamLane sl = stream_lane(r0, r1);
    const T ay = stream_row(A, sl, A.ptr[r0], lds);
    if (sl.live && sl.sub == 0) {
        const T w = wdinv[sl.row], bi = b[sl.row];
        x[sl.row] = w * bi + w * (bi - ay);
    }
}

// b_c = R b - (R A) x: the block's entries of R, then of R A, in one buffer
template <class T>
__global__ __launch_bounds__(kBlock) void k_csrs_restrict(CSRT<T> R, CSRT<T> RA, const T *__restrict__ b,
                                                          const T *__restrict__ x, T *__restrict__ bc,
                                                          const SolveStatus *st) {
    if (st->done) return;
    __shared__ T lds[kStreamCap];
    int r0, r1;
    block_rows(RA, remap_block(blockIdx.x, gridDim.x), r0, r1);
    const int nr = R.ptr[r1] - R.ptr[r0];
    stream_fill(R, r0, r1, lds, [&](int c) { return b[c]; });
    stream_fill(RA, r0, r1, lds + nr, [&](int c) { return x[c]; });
    __syncthreads();
    const StreamLane sl = stream_lane(r0, r1);
    const T rb = stream_row(R, sl, R.ptr[r0], lds);
    const T rax = stream_row(RA, sl, RA.ptr[r0], lds + nr);
    if (sl.live && sl.sub == 0) bc[sl.row] = rb - rax;
}

// x_out = x + P e + W (b - A x - (A P) e): entries of A, A P and P in turn
template <class T>
__global__ __launch_bounds__(kBlock) void k_csrs_prolong_jacobi(CSRT<T> A, CSRT<T> AP, CSRT<T> P,
                                                                const T *__restrict__ wdinv,
                                                                const T *__restrict__ b,
                                                                const T *__restrict__ x,
                                                                const T *__restrict__ e,
                                                                T *__restrict__ xout,
                                                                const SolveStatus *st) {
    if (st->done) return;
    __shared__ T lds[kStreamCap];
    int r0, r1;
    block_rows(A, remap_block(blockIdx.x, gridDim.x), r0, r1);
    const int na = A.ptr[r1] - A.ptr[r0], nq = AP.ptr[r1] - AP.ptr[r0];
    stream_fill(A, r0, r1, lds, [&](int c) { return x[c]; });
    stream_fill(AP, r0, r1, lds + na, [&](int c) { return e[c]; });
    stream_fill(P, r0, r1, lds + na + nq, [&](int c) { return e[c]; });
    __syncthreads();
    const StreamLane sl = stream_lane(r0, r1);
    const T sa = stream_row(A, sl, A.ptr[r0], lds), sq = stream_row(AP, sl, AP.ptr[r0], lds + na);
    const T sp = stream_row(P, sl, P.ptr[r0], lds + na + nq);
    if (sl.live && sl.sub == 0) {
        const int row = sl.row;
        xout[row] = (x[row] + sp) + wdinv[row] * ((b[row] - sa) - sq);
    }
}

// ---------------------------------------------------------------------------
// the coarse part of the cycle as one dense matrix

// x = C b with one wave per row (C row-major FP64, FP64 accumulation; b and
// x in the precision of the cycle)
template <class T>
__global__ __launch_bounds__(kBlock) void k_coarse_dense(int n, const double *__restrict__ C,
                                                         const T *__restrict__ b,
                                                         T *__restrict__ x,
                                                         const SolveStatus *st) {
    if (st->done) return;
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const double *c = C + (size_t)row * n;
    double acc = 0.0;
    if (((size_t)row * n) % 2 == 0) {
        // the row starts on 16 bytes: pairs of entries per load, several
        // loads in flight per lane
        const int n2 = n & ~1;
        double a1 = 0.0;
#pragma unroll 4
        for (int k = 2 * lane; k < n2; k += 128) {
            const double2 cv = *(const double2 *)(c + k);
            acc += cv.x * (double)b[k];
            a1 += cv.y * (double)b[k + 1];
        }
        if ((n & 1) && lane == 0) acc += c[n - 1] * (double)b[n - 1];
        acc += a1;
    } else {
#pragma unroll 4
        for (int k = lane; k < n; k += 64) acc += c[k] * (double)b[k];
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) x[row] = (T)acc;
}

// y = x, two doubles per lane per step (grid-stride)
__global__ __launch_bounds__(kBlock) void k_stream_copy(size_t n2, const double2 *__restrict__ x,
                                                        double2 *__restrict__ y) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n2; i += (size_t)gridDim.x * kBlock)
        y[i] = x[i];
}

// ---------------------------------------------------------------------------
// mixed precision: x += d

// y = FP32(x) (predicated on the solve's status)
__global__ __launch_bounds__(kBlock) void k_to_f32(int n, const double *__restrict__ x,
                                                   float *__restrict__ y, const SolveStatus *st) {
    if (st->done) return;
    const int i = tile_base() + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

__global__ __launch_bounds__(kBlock) void k_add_correction(int n, double *x, const float *d) {
    int i = tile_base() + threadIdx.x;
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
                                                         const double *q, int convective,
                                                         double uconv, double dt, double ly) {
    WallOffsets o = WallOffsets::make(g.nx, g.ny);
    const int t = threadIdx.x;
    for (int k = t; k < o.total; k += kBlock) w1[k] = w0[k];
    // Dirichlet walls keep their values
    if (!convective) return;
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

// [-D q* + bc2 ; E q* - u_B] with the n+1 walls; the pinned entry cleared
__global__ __launch_bounds__(kBlock) void k_poisson_rhs(GridView g, int nb, int pin, const double *qs,
                                                        const double *w1, CSRView E,
                                                        const double *ub, double ub_scale, double *rhs) {
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
        rhs[row] = row == pin ? 0.0 : -(((fe - fw) + fn) - fs);
    } else if (row < g.n_cell + 2 * nb) {
        int k = row - g.n_cell;
        double s = 0.0;
        for (int p = E.ptr[k]; p < E.ptr[k + 1]; ++p) s += E.val[p] * qs[E.col[p]];
        rhs[row] = s - ub_scale * ub[k];
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

// every wall value from the side velocities (left, right, bottom, top)
__global__ __launch_bounds__(kBlock) void k_fill_walls(GridView g, double *w, WallSides ws) {
    WallOffsets o = WallOffsets::make(g.nx, g.ny);
    for (int k = threadIdx.x; k < o.total; k += kBlock) {
        double v;
        if (k < o.uR) v = ws.u[0];            // uL: normal, left
        else if (k < o.vB) v = ws.u[1];       // uR: normal, right
        else if (k < o.vT) v = ws.v[2];       // vB: normal, bottom
        else if (k < o.uBt) v = ws.v[3];      // vT: normal, top
        else if (k < o.uTt) v = ws.u[2];      // uBt: tangential, bottom
        else if (k < o.vLt) v = ws.u[3];      // uTt: tangential, top
        else if (k < o.vRt) v = ws.v[0];      // vLt: tangential, left
        else v = ws.v[1];                     // vRt: tangential, right
        w[k] = v;
    }
}


}  // namespace

// ---------------------------------------------------------------------------
// launchers

#define LAUNCH(kernel, grid, ...) hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, __VA_ARGS__)

void launch_walls_update(hipStream_t s, GridView g, const double *w0, double *w1, const double *q,
                         int convective, double uconv, double dt, double ly) {
    LAUNCH(k_walls_update, 1, g, w0, w1, q, convective, uconv, dt, ly);
}

void launch_momentum_rhs(hipStream_t s, GridView g, const double *q, const double *conv_prev,
                         double *conv_now, double *r1, const double *w0, const double *w1,
                         double nu, double dt, int first_step) {
    LAUNCH(k_momentum_rhs, (g.n_q + kBlock - 1) / kBlock, g, q, conv_prev, conv_now, r1, w0, w1, nu,
           1.0 / dt, first_step);
}

void launch_poisson_rhs(hipStream_t s, GridView g, int nb, int pin, const double *qstar,
                        const double *w1, CSRView E, const double *ub, double ub_scale, double *rhs) {
    int n = g.n_cell + 2 * nb;
    LAUNCH(k_poisson_rhs, (n + kBlock - 1) / kBlock, g, nb, pin, qstar, w1, E, ub, ub_scale, rhs);
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

void launch_fill_walls(hipStream_t s, GridView g, double *w, const WallSides &ws) {
    LAUNCH(k_fill_walls, 1, g, w, ws);
}


// walk depth: the smallest R in {1, 2, 4, 8, 16} that keeps the grid within
// launch_shape().max_walk_blocks (or the forced depth), never beyond the
// partial-sum buffer.  The K walkers, whose tiles read fewer streams than
// the velocity walker's, take half that grid (plus their bands): on the
// 2048^2 grid R = 4 instead of 2, 3-5 % faster per level-0 sweep.
template <class Op>
struct WalkCap {
    static long of(long max_blocks) { return max_blocks; }
};
template <class T>
struct WalkCap<K0T<T>> {
    static long of(long max_blocks) { return max_blocks / 2 + 128; }
};

template <class Op>
static long walk_blocks(const Op &op, int R) {
    dim3 gd = R == 1 ? op_grid<1>(op) : R == 2 ? op_grid<2>(op) : R == 4 ? op_grid<4>(op)
            : R == 8 ? op_grid<8>(op) : op_grid<16>(op);
    return (long)gd.x * gd.y;
}

template <class Op>
static int pick_R(const Op &op) {
    const LaunchShape &ls = launch_shape();
    int R = 16;
    if (ls.walk_rows > 0) {
        R = ls.walk_rows;
    } else {
        const long cap = WalkCap<Op>::of(ls.max_walk_blocks);
        for (int r : {1, 2, 4, 8})
            if (walk_blocks(op, r) <= cap) {
                R = r;
                break;
            }
    }
    while (R < 16 && walk_blocks(op, R) > kMaxParts) R *= 2;
    if (walk_blocks(op, R) > kMaxParts) throw std::runtime_error("grid too large for the reduction buffer");
    return R;
}

#define WALK_SWITCH(R, BODY)                                   \
    switch (R) {                                               \
    case 1: { constexpr int RR = 1; BODY; } break;             \
    case 2: { constexpr int RR = 2; BODY; } break;             \
    case 4: { constexpr int RR = 4; BODY; } break;             \
    case 8: { constexpr int RR = 8; BODY; } break;             \
    default: { constexpr int RR = 16; BODY; } break;           \
    }

#define LAUNCH2(kernel, grid, ...) hipLaunchKernelGGL(kernel, grid, dim3(kBlock), 0, s, __VA_ARGS__)

void launch_apply_K0(hipStream_t s, const K0View &K, const double *x, double *y) {
    WALK_SWITCH(pick_R(K), LAUNCH2((k_apply<RR, K0View, double>), op_grid<RR>(K), K, x, y))
}

void launch_apply_A(hipStream_t s, const AView &A, const double *x, double *y) {
    WALK_SWITCH(pick_R(A), LAUNCH2((k_apply<RR, AView, double>), op_grid<RR>(A), A, x, y))
}

template <class Op, class T>
void launch_pcg_init(hipStream_t s, const Op &op, const T *b, const T *x, T *r, T *z,
                     SolveStatus *st, double *parts, bool jacobi, double rtol2, int maxit) {
    int G = 0;
    WALK_SWITCH(pick_R(op), {
        dim3 gd = op_grid<RR>(op);
        G = gd.x * gd.y;
        LAUNCH2((k_pcg_init<RR, Op, T>), gd, op, b, x, r, z, parts, (int)jacobi);
    })
    LAUNCH(k_finalize, 1, (int)FIN_INIT, G, parts, st, (int)jacobi, rtol2, maxit);
}

template <class T>
void launch_pcg_init_zero(hipStream_t s, int n, const T *b, T *x, T *r, SolveStatus *st,
                          double *parts, double rtol2, int maxit) {
    int G = grid_for(n);
    LAUNCH((k_pcg_init_zero<T>), G, n, b, x, r, st, parts, rtol2, maxit);
    LAUNCH(k_finalize, 1, (int)FIN_INIT_ZERO, G, parts, st, 0, rtol2, maxit);
}

template <class Op>
static int walk_grid_blocks(const Op &op) {
    int G = 0;
    WALK_SWITCH(pick_R(op), {
        dim3 gd = op_grid<RR>(op);
        G = gd.x * gd.y;
    })
    return G;
}

int walk_blocks_of(const K0View &K) { return walk_grid_blocks(K); }
int walk_blocks_of(const K0T<float> &K) { return walk_grid_blocks(K); }
int update_blocks_of(int n) { return grid_for(n); }

template <class Op, class T>
void launch_pcg_spmv(hipStream_t s, const Op &op, const T *z, const T *pold, T *pnew, T *q,
                     SolveStatus *st, const double *rz_parts, int G_rz, double *parts,
                     const double *rr_parts, int G_rr) {
    if (rz_parts && (rz_parts == parts || G_rz < 1 || G_rz > kMaxParts))
        throw std::runtime_error("pcg product: bad partial buffers");
    if (rr_parts && (!rz_parts || rr_parts == parts || rr_parts == rz_parts || G_rz > kFuseMaxParts ||
                     G_rr < 1 || G_rr > kFuseMaxParts))
        throw std::runtime_error("pcg product: the deferred stop test needs fused sums");
    if (rz_parts && G_rz > kFuseMaxParts) {
        LAUNCH(k_finalize, 1, (int)FIN_RZ_NEXT, G_rz, rz_parts, st, 0, 0.0, 0);
        rz_parts = nullptr;
    }
    WALK_SWITCH(pick_R(op), {
        dim3 gd = op_grid<RR>(op);
        LAUNCH2((k_pcg_spmv<RR, Op, T>), gd, op, z, pold, pnew, q, st, rz_parts, G_rz, parts,
                rr_parts, G_rr);
    })
}

template <class Op, class T>
void launch_pcg_update(hipStream_t s, const Op &op, T *x, T *r, T *z, const T *p, const T *q,
                       SolveStatus *st, const double *pq_parts, double *parts, bool jacobi,
                       bool fused_rz, bool defer) {
    if (pq_parts == parts) throw std::runtime_error("pcg update: partial buffers must differ");
    if (defer && (jacobi || !fused_rz)) throw std::runtime_error("pcg update: deferred stop test needs r . z from the product");
    int G_pq = pq_parts ? walk_grid_blocks(op) : 0;
    if (pq_parts && G_pq > kFuseMaxParts) {
        LAUNCH(k_finalize, 1, (int)FIN_PQ, G_pq, pq_parts, st, 0, 0.0, 0);
        pq_parts = nullptr;
        G_pq = 0;
    }
    int G = grid_for(op_n(op));
    LAUNCH((k_pcg_update<Op, T>), G, op, x, r, z, p, q, st, pq_parts, G_pq, parts,
           (int)jacobi | (fused_rz ? 2 : 0) | (defer ? 4 : 0));
    if (!defer)
        LAUNCH(k_finalize, 1, (int)FIN_UPDATE, G, parts, st, (int)jacobi | (fused_rz ? 2 : 0), 0.0, 0);
}

void launch_finalize_pq(hipStream_t s, int G, const double *parts, SolveStatus *st) {
    LAUNCH(k_finalize, 1, (int)FIN_PQ, G, parts, st, 0, 0.0, 0);
}

void launch_finalize_update(hipStream_t s, int G, const double *parts, SolveStatus *st, int flag) {
    LAUNCH(k_finalize, 1, (int)FIN_UPDATE, G, parts, st, flag, 0.0, 0);
}

template <class Op, class T>
void launch_true_residual(hipStream_t s, const Op &op, const T *b, const T *x, SolveStatus *st,
                          double *parts) {
    int G = 0;
    WALK_SWITCH(pick_R(op), {
        dim3 gd = op_grid<RR>(op);
        G = gd.x * gd.y;
        LAUNCH2((k_true_residual<RR, Op, T>), gd, op, b, x, parts);
    })
    LAUNCH(k_finalize, 1, (int)FIN_TRUE, G, parts, st, 0, 0.0, 0);
}

template <class T>
int launch_dot_rz_parts(hipStream_t s, int n, const T *r, const T *z, SolveStatus *st, double *parts) {
    int G = grid_for(n);
    LAUNCH((k_dot_rz<T>), G, n, r, z, st, parts);
    return G;
}

template <class T>
void launch_zero_if_zero_rhs(hipStream_t s, T *x, int n, const SolveStatus *st) {
    LAUNCH((k_zero_if_zero_rhs<T>), (n + kBlock - 1) / kBlock, x, n, st);
}

template <class T>
void launch_k0_prolong_mf(hipStream_t s, const K0T<T> &K, const int *agg, const T *x1, double w,
                          T *x, const SolveStatus *st) {
    WALK_SWITCH(pick_R(K), LAUNCH2((k_k0_prolong_mf<RR, T>), op_grid<RR>(K), K, agg, x1, (T)w, x, st))
}

template <class T>
void launch_k0_wdinv(hipStream_t s, const K0T<T> &K, double omega, T *wd) {
    LAUNCH((k_k0_wdinv<T>), (K.n + kBlock - 1) / kBlock, K, (T)omega, wd);
}

int launch_k0_update_presmooth2_mixed(hipStream_t s, const K0T<float> &K, const float *wd, double *x,
                                      const double *rin, double *rout, const double *p, const double *q,
                                      float *xs, float *r32, SolveStatus *st, const double *pq_parts,
                                      double *parts) {
    if (rin == rout || pq_parts == parts) throw std::runtime_error("update + pre-smoothing: buffers must differ");
    const int G_pq = pq_parts ? walk_grid_blocks(K) : 0;
    if (G_pq > kFuseMaxParts) throw std::runtime_error("update + pre-smoothing: too many product partials");
    int G = 0;
    WALK_SWITCH(pick_R(K), {
        dim3 gd = op_grid<RR>(K);
        G = gd.x * gd.y;
        LAUNCH2((k_k0_update_presmooth2_mixed<RR>), gd, K, wd, x, rin, rout, p, q, xs, r32, st, pq_parts,
                G_pq, parts);
    })
    return G;
}

int launch_k0_jacobi_widen_rz(hipStream_t s, const K0T<float> &K, double omega, const float *b,
                              const float *xin, double *z64, const double *r64, const SolveStatus *st,
                              double *parts) {
    int G = 0;
    WALK_SWITCH(pick_R(K), {
        dim3 gd = op_grid<RR>(K);
        G = gd.x * gd.y;
        LAUNCH2((k_k0_jacobi_widen_rz<RR>), gd, K, (float)omega, b, xin, z64, r64, st, parts);
    })
    return G;
}

template <class T>
int launch_k0_update_presmooth2(hipStream_t s, const K0T<T> &K, const T *wd, T *x, const T *rin, T *rout,
                                const T *p, const T *q, T *xs, SolveStatus *st, const double *pq_parts,
                                double *parts) {
    if (rin == rout || pq_parts == parts) throw std::runtime_error("update + pre-smoothing: buffers must differ");
    const int G_pq = pq_parts ? walk_grid_blocks(K) : 0;
    if (G_pq > kFuseMaxParts) throw std::runtime_error("update + pre-smoothing: too many product partials");
    int G = 0;
    WALK_SWITCH(pick_R(K), {
        dim3 gd = op_grid<RR>(K);
        G = gd.x * gd.y;
        LAUNCH2((k_k0_update_presmooth2<RR, T>), gd, K, wd, x, rin, rout, p, q, xs, st, pq_parts, G_pq, parts);
    })
    return G;
}
template <class T>
void launch_k0_presmooth2(hipStream_t s, const K0T<T> &K, const T *wd, const T *b, T *x,
                          const SolveStatus *st) {
    WALK_SWITCH(pick_R(K), LAUNCH2((k_k0_presmooth2<RR, T>), op_grid<RR>(K), K, wd, b, x, st))
}

template <class T>
void launch_k0_jacobi_first(hipStream_t s, const K0T<T> &K, double omega, const T *b, T *x,
                            const SolveStatus *st) {
    LAUNCH((k_k0_jacobi_first<T>), grid_for(K.n), K, (T)omega, b, x, st);
}

template <class T>
void launch_k0_jacobi(hipStream_t s, const K0T<T> &K, double omega, const T *b, const T *xin,
                      T *xout, const SolveStatus *st) {
    WALK_SWITCH(pick_R(K), LAUNCH2((k_k0_jacobi<RR, T>), op_grid<RR>(K), K, (T)omega, b, xin, xout, st))
}

template <class T>
int launch_k0_jacobi_rz(hipStream_t s, const K0T<T> &K, double omega, const T *b, const T *xin,
                        T *xout, SolveStatus *st, double *parts) {
    int G = 0;
    WALK_SWITCH(pick_R(K), {
        dim3 gd = op_grid<RR>(K);
        G = gd.x * gd.y;
        LAUNCH2((k_k0_jacobi_rz<RR, T>), gd, K, (T)omega, b, xin, xout, st, parts);
    })
    return G;
}

template <class T>
int post2_rows(const K0T<T> &K) {
    // read at every call (the calls are queued once per recorded graph)
    const char *ef = std::getenv("IBPM_POST_FUSE");
    const int fuse = ef ? std::atoi(ef) : -1;
    const char *er = std::getenv("IBPM_POST_ROWS");
    const int rr = er ? std::atoi(er) : 0;
    const int forced = (rr == 8 || rr == 16 || rr == 32) ? rr : 0;
    // on by default from 2^22 cells: below that the three small box passes
    // (about 18 us, mostly latency) outweigh what the one pass saves
    if (fuse == 0 || (fuse < 0 && (long)K.g.nx * K.g.ny < (1L << 22))) return 0;
    if (forced) return forced;
    // the deepest strips that still give every CU four blocks
    const long ncs = (K.g.nx + kPostBlockCols - 1) / kPostBlockCols;
    for (int rf : {32, 16})
        if (ncs * ((K.g.ny + rf - 1) / rf) >= 1024) return rf;
    return 8;
}

// the box coupled to the forces grown by m cells, clipped to the grid
// (empty without a body)
template <class T>
static CellRect grown_box(const K0T<T> &K, int m) {
    if (K.nb == 0 || K.cb_i1 < K.cb_i0 || K.cb_j1 < K.cb_j0) return CellRect{0, -1, 0, -1};
    return CellRect{std::max(K.cb_i0 - m, 0), std::min(K.cb_i1 + m, K.g.nx - 1), std::max(K.cb_j0 - m, 0),
                    std::min(K.cb_j1 + m, K.g.ny - 1)};
}

template <class T>
static int rect_blocks(const K0T<T> &K, const CellRect &r) {
    const long cells = r.i1 < r.i0 ? 0L : (long)(r.i1 - r.i0 + 1) * (r.j1 - r.j0 + 1);
    return k0_band(K) + (int)((cells + kBlock - 1) / kBlock);
}

template <class T>
int launch_k0_prolong_post2(hipStream_t s, const K0T<T> &K, const int *agg, const T *x1, double pw,
                            double omega, const T *b, const T *a, T *tmp, T *tmp2, T *z, double *z64,
                            const double *r64, const SolveStatus *st, double *parts, int mode) {
    const int RF = post2_rows(K);
    if (RF == 0) throw std::runtime_error("prolongation + post-smoothing pass: off for this grid");
    if (mode == POST_WIDEN && !std::is_same<T, float>::value)
        throw std::runtime_error("prolongation + post-smoothing pass: widening needs the FP32 cycle");
    if (a == tmp || a == tmp2 || tmp == tmp2 || (z && (a == z || tmp == z || tmp2 == z)))
        throw std::runtime_error("prolongation + post-smoothing pass: buffers must differ");
    const CellRect skip = grown_box(K, kPostHalo), r1 = grown_box(K, kPostHalo + 1),
                   r2 = grown_box(K, kPostHalo + 2);
    const int ncs = (K.g.nx + kPostBlockCols - 1) / kPostBlockCols;
    const int Gf = ncs * ((K.g.ny + RF - 1) / RF);
    const int Gb = rect_blocks(K, skip);
    if (Gf + Gb > kMaxParts) throw std::runtime_error("prolongation + post-smoothing pass: grid too large");
    const T tw = (T)pw, to = (T)omega;
    // The box passes read a, x1 and b and write tmp, tmp2, z on the box and
    // the force rows and their own partials; the strips read the same and
    // write z elsewhere.
    const int G1 = rect_blocks(K, r1), G2 = rect_blocks(K, r2);
    auto box = [&](hipStream_t q) {
        // (x' on the box grown by 5 and the force rows is formed by the first
        // blocks of the strip launch) y on it grown by 4, then z on it grown
        // by 3
        if (G1 > 0) hipLaunchKernelGGL((k_k0_jacobi_rect<T>), dim3(G1), dim3(kBlock), 0, q, K, r1, to, b, (const T *)tmp, tmp2, st);
        if (Gb > 0) {
            double *pb = parts + Gf;
            if (mode == POST_RZ)
                hipLaunchKernelGGL((k_k0_jacobi_last_rect<POST_RZ, T>), dim3(Gb), dim3(kBlock), 0, q, K, skip, to, b,
                                   (const T *)tmp2, z, z64, r64, st, pb);
            else if (mode == POST_PLAIN)
                hipLaunchKernelGGL((k_k0_jacobi_last_rect<POST_PLAIN, T>), dim3(Gb), dim3(kBlock), 0, q, K, skip, to, b,
                                   (const T *)tmp2, z, z64, r64, st, pb);
            else if constexpr (std::is_same<T, float>::value)
                hipLaunchKernelGGL((k_k0_jacobi_last_rect<POST_WIDEN, T>), dim3(Gb), dim3(kBlock), 0, q, K, skip, to, b,
                                   (const T *)tmp2, z, z64, r64, st, pb);
        }
    };
    // the strips, after G2p blocks that form x' on the box (G2 padded to a
    // multiple of 8, so that the strips keep their XCD mapping)
    const int G2p = (G2 + 7) & ~7;
#define POST_STRIPS(RFV, MODEV)                                                                   \
    LAUNCH((k_k0_prolong_post2<RFV, MODEV, T>), G2p + Gf, K, skip, agg, x1, tw, to, b, a, z, z64, r64, st, \
           parts, r2, tmp, G2p)
#define POST_MODES(RFV)                                                                           \
    if (mode == POST_RZ) POST_STRIPS(RFV, POST_RZ);                                                \
    else if (mode == POST_PLAIN) POST_STRIPS(RFV, POST_PLAIN);                                     \
    else if constexpr (std::is_same<T, float>::value) POST_STRIPS(RFV, POST_WIDEN);
    if (RF == 8) { POST_MODES(8) }
    else if (RF == 16) { POST_MODES(16) }
    else { POST_MODES(32) }
#undef POST_MODES
#undef POST_STRIPS
    box(s);
    return mode == POST_PLAIN ? 0 : Gf + Gb;
}

template <class T>
void launch_k0_residual(hipStream_t s, const K0T<T> &K, const T *b, const T *x, T *r,
                        const SolveStatus *st) {
    WALK_SWITCH(pick_R(K), LAUNCH2((k_k0_residual<RR, T>), op_grid<RR>(K), K, b, x, r, st))
}

template <class T>
void launch_csr_jacobi_first(hipStream_t s, CSRT<T> A, const T *wdinv, const T *b, T *x,
                             const SolveStatus *st) {
    LAUNCH((k_csr_jacobi_first<T>), grid_for(A.nrows), A, wdinv, b, x, st);
}

template <class T>
void launch_dense_solve(hipStream_t s, int n, const double *inv, const T *b, T *x,
                        const SolveStatus *st) {
    LAUNCH((k_dense_solve<T>), (n + kBlock - 1) / kBlock, n, inv, b, x, st);
}

template <class T, int L>
static void csrv_dispatch_jacobi(hipStream_t s, CSRT<T> A, const T *wdinv, const T *b,
                                 const T *xin, T *xout, const SolveStatus *st) {
    int nb = (A.nrows + kBlock / L - 1) / (kBlock / L);
    LAUNCH((k_csrv_jacobi<T, L>), nb > 0 ? nb : 1, A, wdinv, b, xin, xout, st);
}
template <class T, int L>
static void csrv_dispatch_residual(hipStream_t s, CSRT<T> A, const T *b, const T *x, T *r,
                                   const SolveStatus *st) {
    int nb = (A.nrows + kBlock / L - 1) / (kBlock / L);
    LAUNCH((k_csrv_residual<T, L>), nb > 0 ? nb : 1, A, b, x, r, st);
}
template <class T, int L>
static void csrv_dispatch_spmv(hipStream_t s, CSRT<T> A, const T *x, T *y, int add,
                               const SolveStatus *st) {
    int nb = (A.nrows + kBlock / L - 1) / (kBlock / L);
    LAUNCH((k_csrv_spmv<T, L>), nb > 0 ? nb : 1, A, x, y, add, st);
}

#define CSRV_SWITCH(FN, ...)                              \
    switch (lanes) {                                      \
    case 1: FN<T, 1>(s, __VA_ARGS__); break;              \
    case 2: FN<T, 2>(s, __VA_ARGS__); break;              \
    case 4: FN<T, 4>(s, __VA_ARGS__); break;              \
    case 8: FN<T, 8>(s, __VA_ARGS__); break;              \
    case 16: FN<T, 16>(s, __VA_ARGS__); break;            \
    case 32: FN<T, 32>(s, __VA_ARGS__); break;            \
    default: FN<T, 64>(s, __VA_ARGS__); break;            \
    }

template <class T, int L>
static void csrv_dispatch_restrict(hipStream_t s, CSRT<T> R, CSRT<T> RA, const T *b, const T *x, T *bc,
                                   const SolveStatus *st) {
    int nb = (R.nrows + kBlock / L - 1) / (kBlock / L);
    LAUNCH((k_csrv_restrict<T, L>), nb > 0 ? nb : 1, R, RA, b, x, bc, st);
}
template <class T, int L>
static void csrv_dispatch_prolong_jacobi(hipStream_t s, CSRT<T> A, CSRT<T> AP, CSRT<T> P, const T *wdinv,
                                         const T *b, const T *x, const T *e, T *xout,
                                         const SolveStatus *st) {
    int nb = (A.nrows + kBlock / L - 1) / (kBlock / L);
    LAUNCH((k_csrv_prolong_jacobi<T, L>), nb > 0 ? nb : 1, A, AP, P, wdinv, b, x, e, xout, st);
}
template <class T, int L>
static void csrv_dispatch_presmooth2(hipStream_t s, CSRT<T> A, const T *wdinv, const T *b, T *x,
                                     const SolveStatus *st) {
    int nb = (A.nrows + kBlock / L - 1) / (kBlock / L);
    LAUNCH((k_csrv_presmooth2<T, L>), nb > 0 ? nb : 1, A, wdinv, b, x, st);
}
// `lanes` > 0: the row-vector kernels with that many lanes per row;
// `lanes` < 0: the row-block kernels over the row blocks of the shape's
// matrix (A, or R A and A P for the fused transfers)
template <class T>
static void need_blocks(const CSRT<T> &M) {
    if ((!M.bst && M.rpb < 1) || M.nblk < 1) throw std::runtime_error("row-block CSR kernel: the matrix has no row blocks");
}
template <class T>
void launch_csrv_presmooth2(hipStream_t s, CSRT<T> A, int lanes, const T *wdinv, const T *b, T *x,
                            const SolveStatus *st) {
    if (lanes < 0) {
        need_blocks(A);
        LAUNCH((k_csrs_presmooth2<T>), A.nblk, A, wdinv, b, x, st);
        return;
    }
    CSRV_SWITCH(csrv_dispatch_presmooth2, A, wdinv, b, x, st)
}
template <class T>
void launch_csrv_restrict(hipStream_t s, CSRT<T> R, CSRT<T> RA, int lanes, const T *b, const T *x, T *bc,
                          const SolveStatus *st) {
    if (R.nrows != RA.nrows) throw std::runtime_error("fused restriction: R and R A differ in rows");
    if (lanes < 0) {
        need_blocks(RA);
        LAUNCH((k_csrs_restrict<T>), RA.nblk, R, RA, b, x, bc, st);
        return;
    }
    CSRV_SWITCH(csrv_dispatch_restrict, R, RA, b, x, bc, st)
}
template <class T>
void launch_csrv_prolong_jacobi(hipStream_t s, CSRT<T> A, CSRT<T> AP, CSRT<T> P, int lanes,
                                const T *wdinv, const T *b, const T *x, const T *e, T *xout,
                                const SolveStatus *st) {
    if (A.nrows != AP.nrows || A.nrows != P.nrows || AP.ncols != P.ncols)
        throw std::runtime_error("fused prolongation: A, A P and P do not match");
    if (lanes < 0) {
        // the blocks of A P's shape (formed over A, A P and P together)
        need_blocks(AP);
        CSRT<T> Ab = A;
        Ab.bst = AP.bst;
        Ab.rpb = AP.rpb;
        Ab.nblk = AP.nblk;
        LAUNCH((k_csrs_prolong_jacobi<T>), AP.nblk, Ab, AP, P, wdinv, b, x, e, xout, st);
        return;
    }
    CSRV_SWITCH(csrv_dispatch_prolong_jacobi, A, AP, P, wdinv, b, x, e, xout, st)
}
template <class T>
void launch_csrv_jacobi(hipStream_t s, CSRT<T> A, int lanes, const T *wdinv, const T *b,
                        const T *xin, T *xout, const SolveStatus *st) {
    if (lanes < 0) {
        need_blocks(A);
        LAUNCH((k_csrs_jacobi<T>), A.nblk, A, wdinv, b, xin, xout, st);
        return;
    }
    CSRV_SWITCH(csrv_dispatch_jacobi, A, wdinv, b, xin, xout, st)
}
template <class T>
void launch_csrv_residual(hipStream_t s, CSRT<T> A, int lanes, const T *b, const T *x, T *r,
                          const SolveStatus *st) {
    if (lanes < 0) {
        need_blocks(A);
        LAUNCH((k_csrs_residual<T>), A.nblk, A, b, x, r, st);
        return;
    }
    CSRV_SWITCH(csrv_dispatch_residual, A, b, x, r, st)
}
template <class T>
void launch_csrv_spmv(hipStream_t s, CSRT<T> A, int lanes, const T *x, T *y, bool add,
                      const SolveStatus *st) {
    if (lanes < 0) {
        need_blocks(A);
        LAUNCH((k_csrs_spmv<T>), A.nblk, A, x, y, (int)add, st);
        return;
    }
    CSRV_SWITCH(csrv_dispatch_spmv, A, x, y, (int)add, st)
}

void launch_stream_copy(hipStream_t s, size_t n, const double *x, double *y) {
    if (n % 2) throw std::runtime_error("stream copy: odd length");
    LAUNCH(k_stream_copy, 8192, n / 2, (const double2 *)x, (double2 *)y);
}

template <class T>
void launch_coarse_dense(hipStream_t s, int n, const double *C, const T *b, T *x, const SolveStatus *st) {
    if (n < 1 || n > 8192 || !C || !b || !x)
        throw std::runtime_error("coarse cycle: bad size or operand");
    const int rows_per_block = kBlock / 64;
    LAUNCH((k_coarse_dense<T>), (n + rows_per_block - 1) / rows_per_block, n, C, b, x, st);
}

template <class T>
void launch_fcg_betas(hipStream_t s, int n, const T *z, FcgVecs<T> Q, int cnt, FcgSlots sl,
                      FcgRing *ring, const SolveStatus *st, double *parts) {
    if (cnt < 1) return;
    if (cnt > kFcgMax) throw std::runtime_error("fcg: too many directions");
    int G = grid_for(n);
    LAUNCH((k_fcg_multidot<T>), G, n, z, Q, cnt, sl, st, parts);
    LAUNCH(k_fcg_betas_finalize, 1, G, cnt, sl, (const double *)parts, ring, st);
}

template <class T>
void launch_fcg_direction(hipStream_t s, int n, const T *z, FcgVecs<T> P, int cnt, FcgSlots sl,
                          const FcgRing *ring, T *p, const SolveStatus *st) {
    if (cnt < 0 || cnt > kFcgMax) throw std::runtime_error("fcg: too many directions");
    LAUNCH((k_fcg_direction<T>), (n + kBlock - 1) / kBlock, n, z, P, cnt, sl, ring, p, st);
}

template <class T>
void launch_fcg_product(hipStream_t s, const K0T<T> &K, const T *p, T *q, const T *r, int slot,
                        FcgRing *ring, SolveStatus *st, double *parts) {
    int G = 0;
    WALK_SWITCH(pick_R(K), {
        dim3 gd = op_grid<RR>(K);
        G = gd.x * gd.y;
        LAUNCH2((k_fcg_product<RR, T>), gd, K, p, q, r, (const SolveStatus *)st, parts);
    })
    LAUNCH(k_fcg_pq_finalize, 1, G, (const double *)parts, slot, ring, st);
}

// the learned-stage weight is only computed while the solve runs (st), into stw
template <class T>
void launch_kd_omega(hipStream_t s, const K0T<T> &K, const T *d, const T *r1, SolveStatus *stw,
                     double *parts, const SolveStatus *st) {
    int G = 0;
    WALK_SWITCH(pick_R(K), {
        dim3 gd = op_grid<RR>(K);
        G = gd.x * gd.y;
        LAUNCH2((k_kd_dots<RR, T>), gd, K, d, r1, st, parts);
    })
    LAUNCH(k_finalize, 1, (int)FIN_OMEGA, G, parts, stw, 0, 0.0, 0);
}

template <class T>
void launch_axpy_omega(hipStream_t s, int n, const T *z0, const T *d, const SolveStatus *stw, T *z,
                       const SolveStatus *st) {
    LAUNCH((k_axpy_omega<T>), (n + kBlock - 1) / kBlock, n, z0, d, stw, z, st);
}

void launch_harvest_e1(hipStream_t s, int n, const double *xstar, const double *x, const double *z,
                       float *e1) {
    LAUNCH(k_harvest_e1, (n + kBlock - 1) / kBlock, n, xstar, x, z, e1);
}

void launch_outer_residual(hipStream_t s, const K0View &K, const double *b, const double *x,
                           float *r32, SolveStatus *st, double *parts, int first) {
    int G = 0;
    WALK_SWITCH(pick_R(K), {
        dim3 gd = op_grid<RR>(K);
        G = gd.x * gd.y;
        LAUNCH2((k_outer_residual<RR>), gd, K, b, x, r32, parts);
    })
    LAUNCH(k_finalize, 1, (int)FIN_OUTER, G, parts, st, first, 0.0, 0);
}

void launch_to_f32(hipStream_t s, int n, const double *x, float *y, const SolveStatus *st) {
    LAUNCH(k_to_f32, (n + kBlock - 1) / kBlock, n, x, y, st);
}
void launch_add_correction(hipStream_t s, int n, double *x, const float *d) {
    LAUNCH(k_add_correction, (n + kBlock - 1) / kBlock, n, x, d);
}

// explicit instantiations
#define INST_OP(OP, T)                                                                           \
    template void launch_pcg_init<OP, T>(hipStream_t, const OP &, const T *, const T *, T *, T *,\
                                         SolveStatus *, double *, bool, double, int);            \
    template void launch_pcg_spmv<OP, T>(hipStream_t, const OP &, const T *, const T *, T *, T *, \
                                         SolveStatus *, const double *, int, double *,           \
                                         const double *, int);                                   \
    template void launch_pcg_update<OP, T>(hipStream_t, const OP &, T *, T *, T *, const T *,    \
                                           const T *, SolveStatus *, const double *, double *,   \
                                           bool, bool, bool);                                          \
    template void launch_true_residual<OP, T>(hipStream_t, const OP &, const T *, const T *,     \
                                              SolveStatus *, double *);
INST_OP(K0View, double)
INST_OP(AView, double)
INST_OP(K0T<float>, float)
INST_OP(CsrOpView, double)

#define INST_T(T)                                                                                \
    template void launch_pcg_init_zero<T>(hipStream_t, int, const T *, T *, T *, SolveStatus *,  \
                                          double *, double, int);                                \
    template int launch_dot_rz_parts<T>(hipStream_t, int, const T *, const T *, SolveStatus *,   \
                                        double *);                                               \
    template void launch_zero_if_zero_rhs<T>(hipStream_t, T *, int, const SolveStatus *);        \
    template void launch_k0_wdinv<T>(hipStream_t, const K0T<T> &, double, T *);                   \
    template void launch_k0_prolong_mf<T>(hipStream_t, const K0T<T> &, const int *, const T *,    \
                                          double, T *, const SolveStatus *);                      \
    template void launch_k0_presmooth2<T>(hipStream_t, const K0T<T> &, const T *, const T *, T *,  \
                                          const SolveStatus *);                                   \
    template int launch_k0_update_presmooth2<T>(hipStream_t, const K0T<T> &, const T *, T *,       \
                                                const T *, T *, const T *, const T *, T *,          \
                                                SolveStatus *, const double *, double *);           \
    template void launch_k0_jacobi_first<T>(hipStream_t, const K0T<T> &, double, const T *, T *, \
                                            const SolveStatus *);                                \
    template void launch_k0_jacobi<T>(hipStream_t, const K0T<T> &, double, const T *, const T *, \
                                      T *, const SolveStatus *);                                 \
    template int launch_k0_jacobi_rz<T>(hipStream_t, const K0T<T> &, double, const T *,          \
                                        const T *, T *, SolveStatus *, double *);                \
    template void launch_k0_residual<T>(hipStream_t, const K0T<T> &, const T *, const T *, T *,  \
                                        const SolveStatus *);                                    \
    template int launch_k0_prolong_post2<T>(hipStream_t, const K0T<T> &, const int *, const T *,  \
                                            double, double, const T *, const T *, T *, T *, T *,  \
                                            double *, const double *, const SolveStatus *, double *, \
                                            int);                                                 \
    template int post2_rows<T>(const K0T<T> &);                                                  \
    template void launch_csr_jacobi_first<T>(hipStream_t, CSRT<T>, const T *, const T *, T *,    \
                                             const SolveStatus *);                               \
    template void launch_dense_solve<T>(hipStream_t, int, const double *, const T *, T *,        \
                                        const SolveStatus *);
INST_T(double)
INST_T(float)

#define INST_V(T)                                                                                \
    template void launch_csrv_jacobi<T>(hipStream_t, CSRT<T>, int, const T *, const T *,         \
                                        const T *, T *, const SolveStatus *);                    \
    template void launch_csrv_residual<T>(hipStream_t, CSRT<T>, int, const T *, const T *, T *,  \
                                          const SolveStatus *);                                  \
    template void launch_csrv_spmv<T>(hipStream_t, CSRT<T>, int, const T *, T *, bool,           \
                                      const SolveStatus *);                                      \
    template void launch_csrv_restrict<T>(hipStream_t, CSRT<T>, CSRT<T>, int, const T *, const T *, \
                                          T *, const SolveStatus *);                             \
    template void launch_csrv_prolong_jacobi<T>(hipStream_t, CSRT<T>, CSRT<T>, CSRT<T>, int,      \
                                                const T *, const T *, const T *, const T *, T *,  \
                                                const SolveStatus *);                             \
    template void launch_coarse_dense<T>(hipStream_t, int, const double *, const T *, T *,        \
                                         const SolveStatus *);
INST_V(double)
INST_V(float)

#define INST_F(T)                                                                                \
    template void launch_kd_omega<T>(hipStream_t, const K0T<T> &, const T *, const T *,          \
                                     SolveStatus *, double *, const SolveStatus *);              \
    template void launch_axpy_omega<T>(hipStream_t, int, const T *, const T *, const SolveStatus *,\
                                       T *, const SolveStatus *);
INST_F(double)
INST_F(float)

#define INST_P(T)                                                                                \
    template void launch_csrv_presmooth2<T>(hipStream_t, CSRT<T>, int, const T *, const T *, T *, \
                                            const SolveStatus *);

INST_P(double)
INST_P(float)

#define INST_M(T)                                                                                \
    template void launch_fcg_betas<T>(hipStream_t, int, const T *, FcgVecs<T>, int, FcgSlots,   \
                                      FcgRing *, const SolveStatus *, double *);                 \
    template void launch_fcg_direction<T>(hipStream_t, int, const T *, FcgVecs<T>, int, FcgSlots,\
                                          const FcgRing *, T *, const SolveStatus *);            \
    template void launch_fcg_product<T>(hipStream_t, const K0T<T> &, const T *, T *, const T *,  \
                                        int, FcgRing *, SolveStatus *, double *);
INST_M(double)
INST_M(float)

}  // namespace ibpm
