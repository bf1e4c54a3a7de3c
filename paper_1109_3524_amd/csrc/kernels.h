// Device data views and kernel launchers (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace ibpm {

constexpr int kBlock = 256;        // threads per block (4 wave64)
constexpr int kMaxParts = 32768;   // upper bound on blocks of a reducing kernel; a buffer of
                                   // partials holds one row of kMaxParts per summed value

// Launch shapes of the reducing kernels: the largest 2-D grid of the stencil
// walkers (the walk depth R grows until the grid fits; walk_rows > 0 forces
// R) and the largest 1-D grid of the elementwise kernels.  Set once per
// process (IBPM_WALK_ROWS, IBPM_MAX_BLOCKS override the defaults).
struct LaunchShape {
    int max_walk_blocks = 8448;
    int walk_rows = 0;
    int max_blocks = 2048;
};
LaunchShape &launch_shape();

// Tensor-product staggered grid; metric arrays live on the device.
template <class T>
struct GridT {
    int nx, ny;
    int n_u, n_v, n_q, n_cell;
    const T *dx, *dy, *Dx, *Dy;      // nx, ny, nx+1, ny+1
    const T *idx, *idy, *iDx, *iDy;  // reciprocals
};
using GridView = GridT<double>;

// Packed wall values: uL[ny] uR[ny] vB[nx] vT[nx] uBt[nx+1] uTt[nx+1] vLt[ny+1] vRt[ny+1]
struct WallOffsets {
    int uL, uR, vB, vT, uBt, uTt, vLt, vRt, total;
    __host__ __device__ static WallOffsets make(int nx, int ny) {
        WallOffsets o;
        o.uL = 0;
        o.uR = ny;
        o.vB = 2 * ny;
        o.vT = 2 * ny + nx;
        o.uBt = 2 * ny + 2 * nx;
        o.uTt = 2 * ny + 3 * nx + 1;
        o.vLt = 2 * ny + 4 * nx + 2;
        o.vRt = 3 * ny + 4 * nx + 3;
        o.total = 4 * ny + 4 * nx + 4;
        return o;
    }
};

// Velocity of each wall side, in the order left, right, bottom, top
struct WallSides {
    double u[4], v[4];
};

template <class T>
struct CSRT {
    int nrows, ncols;
    const int32_t *ptr, *col;
    const T *val;
    // the row blocks of the row-block kernels, nblk of them, each at most
    // kBlock rows whose entries (of every matrix the kernel walks) fit
    // kStreamCap: block k takes rows k rpb .. (k + 1) rpb - 1 (rpb > 0), or
    // bst[k] .. bst[k + 1] - 1; neither where the matrix has no row blocks
    const int32_t *bst = nullptr;
    int rpb = 0;
    int nblk = 0;
};
using CSRView = CSRT<double>;

// Rows of K with stored entries are taken by bands of blocks ahead of the
// stencil tiles, 8 lanes per row, from fixed-width (ELL) copies of the CSR
// rows so that a row's entries are fetched in one round of independent
// loads: slot k * 8 + l of a row is CSR entry k * 8 + l, taken by lane l;
// empty slots hold column -1 and value 0.  Rows longer than the width are
// read from the CSR instead (the ELL flag of the matrix is 0).
constexpr int kKfW = 24;   // slots per force row
constexpr int kStreamCap = 2048;   // entries one block of the row-block CSR kernels holds in LDS
constexpr int kCcW = 16;   // slots per coupled cell (force unknowns it meets)

// Level-0 Poisson operator K = Q^T B^1 Q (pinned), matrix-free pressure
// stencil plus stored coupling rows, in precision T.
template <class T>
struct K0T {
    GridT<T> g;
    T dt;
    int nb, n;                       // n = n_cell + 2 nb
    int pin;                         // pinned cell: row and column cleared but the diagonal
    int cb_i0, cb_i1, cb_j0, cb_j1;  // box of cells coupled to forces
    CSRT<T> cf;                      // box cells -> (force 0..2nb-1, value)
    CSRT<T> kf;                      // force rows, columns in lambda numbering
    const T *kf_diag;
    // ELL copies of the force rows ([row * kKfW + slot])
    int kf_ell;
    const int32_t *kfe_col;
    const T *kfe_val;
    // the ncc box cells with coupling entries: their cell indices, one bit
    // per box cell (row-major in the box) marking them, and the ELL copy of
    // their coupling ([q * kCcW + slot], columns 0..2nb-1)
    int ncc, cc_ell;
    const int32_t *cc_row;
    const uint32_t *cc_bits;
    const int32_t *cce_col;
    const T *cce_val;
};
using K0View = K0T<double>;

// A stored (CSR, sorted rows) operator for the Krylov kernels: the level-0
// Poisson operator K = Q^T B^N Q when N > 1, its diagonal kept apart.
template <class T>
struct CsrOpT {
    CSRT<T> A;   // with row blocks the Krylov kernels take them, else one row per thread
    const T *diag;
};
using CsrOpView = CsrOpT<double>;

// Velocity operator A = Mf/dt - (nu/2) L on interior faces (matrix-free, FP64).
struct AView {
    GridView g;
    double dt, idt, nu;
};

// Device-side state of one Krylov solve.  Written only by the last block
// of a reducing kernel; read by every later kernel of the stream.
enum : int { ST_RUNNING = 0, ST_CONVERGED = 1, ST_MAXIT = 2, ST_NAN = 3, ST_ZERO_RHS = 4 };
struct SolveStatus {
    double bb, rr, rz, pq, beta, tol2, true_rr;
    double rz_next;                  // r . z of the new preconditioned residual (fused path)
    double fx, fy;
    int iter, maxit, done, first;
    unsigned int counter;
    int pad;
};

// --- launchers (all asynchronous on `s`) ---------------------------------
// step stages (FP64)
void launch_walls_update(hipStream_t s, GridView g, const double *w0, double *w1,
                         const double *q, int convective, double uconv, double dt, double ly);
void launch_momentum_rhs(hipStream_t s, GridView g, const double *q, const double *conv_prev,
                         double *conv_now, double *r1, const double *w0, const double *w1,
                         double nu, double dt, int first_step);
void launch_poisson_rhs(hipStream_t s, GridView g, int nb, int pin, const double *qstar,
                        const double *w1, CSRView E, const double *ub, double ub_scale, double *rhs);
void launch_project(hipStream_t s, GridView g, double dt, int nb, const double *qstar,
                    const double *lam, double *qout, CSRView etu, int fu_i0, int fu_i1, int fu_j0,
                    int fu_j1, CSRView etv, int fv_i0, int fv_i1, int fv_j0, int fv_j1);
void launch_forces(hipStream_t s, int n_cell, int nb, const double *lam, SolveStatus *st);
void launch_init_state(hipStream_t s, GridView g, double *q, double *conv, double *lam, int n_lam,
                       double U, double V);
void launch_fill_walls(hipStream_t s, GridView g, double *w, const WallSides &ws);

// operators
void launch_apply_K0(hipStream_t s, const K0View &K, const double *x, double *y);
void launch_apply_A(hipStream_t s, const AView &A, const double *x, double *y);

// Krylov pieces.  Op is K0T<T> (vectors of T) or AView (vectors of double);
// dot products always accumulate in FP64.
// r = b - op x (and z = D^{-1} r for Jacobi preconditioning)
template <class Op, class T>
void launch_pcg_init(hipStream_t s, const Op &op, const T *b, const T *x, T *r, T *z,
                     SolveStatus *st, double *parts, bool jacobi, double rtol2, int maxit);
template <class T>
void launch_pcg_init_zero(hipStream_t s, int n, const T *b, T *x, T *r, SolveStatus *st,
                          double *parts, double rtol2, int maxit);
// restriction with the residual folded in: bc = R b - (R A) x
template <class T>
void launch_csrv_restrict(hipStream_t s, CSRT<T> R, CSRT<T> RA, int lanes, const T *b, const T *x, T *bc,
                          const SolveStatus *st);
// prolongation and the first post-sweep: xout = x + P e + W (b - A x - (A P) e)
template <class T>
void launch_csrv_prolong_jacobi(hipStream_t s, CSRT<T> A, CSRT<T> AP, CSRT<T> P, int lanes,
                                const T *wdinv, const T *b, const T *x, const T *e, T *xout,
                                const SolveStatus *st);
// the first two damped-Jacobi sweeps from zero on a CSR level in one pass
template <class T>
void launch_csrv_presmooth2(hipStream_t s, CSRT<T> A, int lanes, const T *wdinv, const T *b, T *x,
                            const SolveStatus *st);

// number of blocks (and of partials) of a level-0 stencil kernel
int walk_blocks_of(const K0View &K);
int walk_blocks_of(const K0T<float> &K);
// number of blocks (and of partials) of the PCG update on n unknowns
int update_blocks_of(int n);
// above this many partials a sum read by every block of the consumer costs
// more than a one-block finalize launch
constexpr int kFuseMaxParts = 2048;
// p_new = z + beta p_old; q = op p_new; per-block partials of p . q in parts
// (no finalize: the update below sums them).  beta is st->beta, or, when
// rz_parts is given (G_rz partials of r . z from the preconditioner's last
// kernel), beta = rz_new / st->rz (0 on the first iteration) with rz_new
// summed here and left in st->rz_next.  With rr_parts (the G_rr partials of
// r . r left by a deferred update, see below; needs rz_parts, both at most
// kFuseMaxParts) every block also sums r . r and, except on the first
// iteration, takes the stop decision the update's finalize would have taken
// (NaN, converged, iteration limit): then it does nothing else and block 0
// records it in st.
template <class Op, class T>
void launch_pcg_spmv(hipStream_t s, const Op &op, const T *z, const T *pold, T *pnew, T *q,
                     SolveStatus *st, const double *rz_parts, int G_rz, double *parts,
                     const double *rr_parts = nullptr, int G_rr = 0);
// x += alpha p; r -= alpha q (and z = D^{-1} r for Jacobi), alpha = rz / pq
// with pq summed from pq_parts (the product kernel's partials; another
// buffer than parts) or, when pq_parts is null, taken from st->pq; rz is
// st->rz_next after a product with rz_parts (fused_rz), else st->rz.
// Leaves the partials of r . r in parts; a one-block finalize then counts
// the iteration and takes the stop decision, unless defer is set (needs
// fused_rz, not Jacobi): then block 0 counts the iteration and moves
// rz_next to rz, and the next product kernel takes the decision.
template <class Op, class T>
void launch_pcg_update(hipStream_t s, const Op &op, T *x, T *r, T *z, const T *p, const T *q,
                       SolveStatus *st, const double *pq_parts, double *parts, bool jacobi,
                       bool fused_rz, bool defer = false);
template <class Op, class T>
void launch_true_residual(hipStream_t s, const Op &op, const T *b, const T *x, SolveStatus *st,
                          double *parts);
// per-block partials of r . z (no finalize); returns the number of partials
template <class T>
int launch_dot_rz_parts(hipStream_t s, int n, const T *r, const T *z, SolveStatus *st, double *parts);
template <class T>
void launch_zero_if_zero_rhs(hipStream_t s, T *x, int n, const SolveStatus *st);

// V-cycle pieces, predicated on st->done
// x += P x1 on level 0 with the smoothed prolongator applied matrix-free:
// P = (I - w D^-1 K) T, T the aggregates (agg[i] = aggregate of unknown i)
template <class T>
void launch_k0_prolong_mf(hipStream_t s, const K0T<T> &K, const int *agg, const T *x1, double w,
                          T *x, const SolveStatus *st);
// wd = omega / diag(K0)
template <class T>
void launch_k0_wdinv(hipStream_t s, const K0T<T> &K, double omega, T *wd);
// two damped-Jacobi sweeps from x = 0 in one pass: x = y + wd (b - K y), y = wd b
// one-block sums of partials into the status: p.q (FIN_PQ), and the stop
// test of an update (FIN_UPDATE; flag bit 0: Jacobi r.z in the second row,
// bit 1: r.z came from the product)
void launch_finalize_pq(hipStream_t s, int G, const double *parts, SolveStatus *st);
void launch_finalize_update(hipStream_t s, int G, const double *parts, SolveStatus *st, int flag);
// FP64 CG around an FP32 V-cycle: the FP64 update folded into the FP32
// first pass (b = r_in - alpha q in FP64 to r_out, x += alpha p, FP32(b) to
// r32, the two FP32 sweeps from zero to xs; partials of b.b), and the last
// FP32 post-sweep with its result widened to z64 and the partials of
// r64 . z64.  Both return the number of partials.
int launch_k0_update_presmooth2_mixed(hipStream_t s, const K0T<float> &K, const float *wd, double *x,
                                      const double *rin, double *rout, const double *p, const double *q,
                                      float *xs, float *r32, SolveStatus *st, const double *pq_parts,
                                      double *parts);
int launch_k0_jacobi_widen_rz(hipStream_t s, const K0T<float> &K, double omega, const float *b,
                              const float *xin, double *z64, const double *r64, const SolveStatus *st,
                              double *parts);
// the PCG update (alpha = st->rz_next / p.q) and the first two
// pre-smoothing sweeps on level 0 in one pass: b = r_in - alpha q to r_out,
// x += alpha p, xs = the two sweeps from zero for b; partials of b.b in
// parts.  With pq_parts, p.q is summed from the product's partials (at most
// kFuseMaxParts) and block 0 counts the iteration (the stop test deferred to
// the next product); with pq_parts null, p.q is read from the status and
// the caller finalizes (launch_finalize_pq before, launch_finalize_update
// after).  Returns the number of partials.
template <class T>
int launch_k0_update_presmooth2(hipStream_t s, const K0T<T> &K, const T *wd, T *x, const T *rin, T *rout,
                                const T *p, const T *q, T *xs, SolveStatus *st, const double *pq_parts,
                                double *parts);
template <class T>
void launch_k0_presmooth2(hipStream_t s, const K0T<T> &K, const T *wd, const T *b, T *x,
                          const SolveStatus *st);
template <class T>
void launch_k0_jacobi_first(hipStream_t s, const K0T<T> &K, double omega, const T *b, T *x,
                            const SolveStatus *st);
template <class T>
void launch_k0_jacobi(hipStream_t s, const K0T<T> &K, double omega, const T *b, const T *xin,
                      T *xout, const SolveStatus *st);
// The prolongation and both post-smoothing sweeps of the level-0 V-cycle
// (post = 2):  x' = a + P x1 (launch_k0_prolong_mf), y = x' + omega D^-1
// (b - K x'), z = y + omega D^-1 (b - K y), as those three passes compute
// them, cell for cell.  Away from the body it is one pass over strips of
// post2_rows(K) rows of cells per block, each wave recomputing x' and y
// three cells around its 58 columns; the cells within three of the box
// coupled to the forces and the force rows, whose rows reach past any
// strip, are done over that box grown by 2, 1 and 0 more cells: x' by the
// first blocks of the strip launch, y and z by two small launches after it,
// through the level-0 work vectors tmp (x') and tmp2 (y).  a is only read.
// mode 0: z in T and the partials of b . z; mode 1 (T = float): z widened to
// z64 and the partials of r64 . z64; mode 2: z only.  Returns the number of
// partials (the strip pass's, then the box pass's).
enum { POST_RZ = 0, POST_WIDEN = 1, POST_PLAIN = 2 };
// cells [i0, i1] x [j0, j1] of the level-0 grid (empty when i1 < i0)
struct CellRect {
    int i0, i1, j0, j1;
};
template <class T>
int launch_k0_prolong_post2(hipStream_t s, const K0T<T> &K, const int *agg, const T *x1, double pw,
                            double omega, const T *b, const T *a, T *tmp, T *tmp2, T *z, double *z64,
                            const double *r64, const SolveStatus *st, double *parts, int mode);
// rows of cells per block of that pass on this grid (8, 16 or 32); 0 when
// the pass is off for it (IBPM_POST_FUSE=0, or a grid below 2^22 cells
// unless IBPM_POST_FUSE=1; IBPM_POST_ROWS forces the depth)
template <class T>
int post2_rows(const K0T<T> &K);
// last post-sweep; per-block partials of b . xout in parts (no finalize:
// the next product kernel sums them); returns the number of partials
template <class T>
int launch_k0_jacobi_rz(hipStream_t s, const K0T<T> &K, double omega, const T *b, const T *xin,
                        T *xout, SolveStatus *st, double *parts);
template <class T>
void launch_k0_residual(hipStream_t s, const K0T<T> &K, const T *b, const T *x, T *r,
                        const SolveStatus *st);
template <class T>
void launch_csr_jacobi_first(hipStream_t s, CSRT<T> A, const T *wdinv, const T *b, T *x,
                             const SolveStatus *st);
template <class T>
void launch_dense_solve(hipStream_t s, int n, const double *inv_colmajor, const T *b, T *x,
                        const SolveStatus *st);

// CSR kernels with `lanes` threads per row (1, 2, 4, ..., 64; a power of two)
template <class T>
void launch_csrv_jacobi(hipStream_t s, CSRT<T> A, int lanes, const T *wdinv, const T *b,
                        const T *xin, T *xout, const SolveStatus *st);
template <class T>
void launch_csrv_residual(hipStream_t s, CSRT<T> A, int lanes, const T *b, const T *x, T *r,
                          const SolveStatus *st);
template <class T>
void launch_csrv_spmv(hipStream_t s, CSRT<T> A, int lanes, const T *x, T *y, bool add,
                      const SolveStatus *st);

// Coarse levels applied together as one dense map (levels lc .. L-1): the
// first level below level 0 with at most kCoarseRows unknowns starts it
// (kCoarseRowsMoving for a moving body, whose small levels and dense map are
// formed anew on the host at every refresh of the hierarchy).
constexpr int kCoarseRows = 4096;
constexpr int kCoarseRowsMoving = 1024;
constexpr int kMaxLevels = 16;
// the V-cycle on the small levels as one dense product x = C b, C row-major
// n x n in FP64 for either precision of the cycle
template <class T>
void launch_coarse_dense(hipStream_t s, int n, const double *C, const T *b, T *x,
                         const SolveStatus *st);

// y = x (n even), a plain streaming copy for bandwidth reference
void launch_stream_copy(hipStream_t s, size_t n, const double *x, double *y);

// Truncated flexible CG, FCG(m) (Notay): the new direction is made
// K-orthogonal to the last m directions.  Directions and their products are
// kept in a ring of m slots; ring->pq holds p_i . q_i of each slot.
constexpr int kFcgMax = 8;
struct FcgRing {
    double pq[kFcgMax];
    double beta[kFcgMax];
};
template <class T>
struct FcgVecs {
    T *v[kFcgMax];
};
struct FcgSlots {
    int s[kFcgMax];
};
//   beta_j = -(z . q_{slot j}) / pq_{slot j}, j < cnt (into ring->beta)
template <class T>
void launch_fcg_betas(hipStream_t s, int n, const T *z, FcgVecs<T> Q, int cnt, FcgSlots sl,
                      FcgRing *ring, const SolveStatus *st, double *parts);
//   p = z + sum_j beta_j P_{slot j}
template <class T>
void launch_fcg_direction(hipStream_t s, int n, const T *z, FcgVecs<T> P, int cnt, FcgSlots sl,
                          const FcgRing *ring, T *p, const SolveStatus *st);
//   q = K p; st->pq = p . q, st->rz = p . r, ring->pq[slot] = p . q
template <class T>
void launch_fcg_product(hipStream_t s, const K0T<T> &K, const T *p, T *q, const T *r, int slot,
                        FcgRing *ring, SolveStatus *st, double *parts);

// flexible CG with a learned stage (vectors of T, sums in FP64):
//   stw->beta = (d.r1) / (d.K d) (0 if not positive or not finite); the sums
//   are skipped once the solve with status st has finished
template <class T>
void launch_kd_omega(hipStream_t s, const K0T<T> &K, const T *d, const T *r1, SolveStatus *stw,
                     double *parts, const SolveStatus *st);
//   z = z0 + stw->beta d (z = z0 when the weight is 0)
template <class T>
void launch_axpy_omega(hipStream_t s, int n, const T *z0, const T *d, const SolveStatus *stw, T *z,
                       const SolveStatus *st);
// harvest: e1 = x* - x - z (FP32)
void launch_harvest_e1(hipStream_t s, int n, const double *xstar, const double *x, const double *z,
                       float *e1);

// mixed precision: FP64 outer residual r = b - K x (also cast to FP32) and x += d
void launch_outer_residual(hipStream_t s, const K0View &K, const double *b, const double *x,
                           float *r32, SolveStatus *st, double *parts, int first);
void launch_add_correction(hipStream_t s, int n, double *x, const float *d);
// FP64 CG with an FP32 V-cycle: y = FP32(x) (the residual on entry to the cycle)
void launch_to_f32(hipStream_t s, int n, const double *x, float *y, const SolveStatus *st);

}  // namespace ibpm
