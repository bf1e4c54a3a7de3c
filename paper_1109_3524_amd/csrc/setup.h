// Host-side assembly of the operators of the immersed-boundary projection
// method and of the smoothed-aggregation hierarchy.  Pure C++ (no HIP): the
// results are uploaded to the device by the context code.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ibpm {

// Compressed sparse rows, int32 indices.
struct CSR {
    int32_t nrows = 0, ncols = 0;
    std::vector<int32_t> ptr;   // nrows + 1
    std::vector<int32_t> col;
    std::vector<double> val;
    int64_t nnz() const { return (int64_t)col.size(); }
};

struct GridMetrics {
    int32_t nx = 0, ny = 0;
    std::vector<double> xf, yf;      // faces
    std::vector<double> dx, dy;      // cell widths
    std::vector<double> xc, yc;      // cell centres
    std::vector<double> Dx, Dy;      // nx+1 / ny+1 distances across face lines
    int64_t n_u = 0, n_v = 0, n_q = 0, n_cell = 0;
    int64_t uidx(int i, int j) const { return (int64_t)j * (nx - 1) + (i - 1); }
    int64_t vidx(int i, int j) const { return n_u + (int64_t)(j - 1) * nx + i; }
};

// Everything the device needs for the level-0 operators.
struct Model {
    GridMetrics g;
    int32_t nb = 0;
    int32_t pin = 0;                 // pinned pressure cell (row and column cleared)
    double nu = 0, dt = 0;
    std::vector<double> ub;          // 2nb prescribed body velocity (x then y)
    CSR E;                           // 2nb x n_q interpolation (flux form)
    // bounding boxes of the delta supports (inclusive), for gathers
    int32_t cb_i0 = 0, cb_i1 = -1, cb_j0 = 0, cb_j1 = -1;  // cells with force coupling
    CSR Kcf;                         // rows: bbox cells (row-major in the box), cols: force index 0..2nb-1
    CSR Kf;                          // 2nb force rows of K, cols in lambda numbering
    std::vector<double> Kf_diag;     // 2nb
    int32_t fu_i0 = 0, fu_i1 = -1, fu_j0 = 0, fu_j1 = -1;  // u faces touched by E
    int32_t fv_i0 = 0, fv_i1 = -1, fv_j0 = 0, fv_j1 = -1;  // v faces touched by E
    CSR Etu;                         // rows: u faces of the box, cols: force index 0..nb-1
    CSR Etv;                         // rows: v faces of the box, cols: force index 0..nb-1
    CSR K;                           // full pinned K (for the hierarchy setup)
    // delta weights between the points and the cell centres (learned stage):
    // phi((xc_i - xi_k)/h) phi((yc_j - eta_k)/h), cells of a box -> points and back
    int32_t dc_i0 = 0, dc_i1 = -1, dc_j0 = 0, dc_j1 = -1;
    CSR Dc2p;                        // rows: box cells, cols: point 0..nb-1
    CSR Dp2c;                        // rows: points, cols: cell index (j*nx + i)
    double hmin = 0;                 // smallest cell width
};

struct Level {
    CSR A;                           // operator of this level (level 0: copy of K)
    std::vector<double> wdinv;       // omega / a_ii
    double rho = 0;                  // spectral radius estimate of D^{-1} A
    double omega = 0;                // 4 / (3 rho)
    CSR P, R;                        // prolongator to this level from the next, and P^T
    CSR RA, AP;                      // R A and A P where the device fuses the
                                     // residual into the restriction and the
                                     // prolongation into the first post-sweep
    std::vector<int32_t> agg;
    double pomega = 0;               // P = (I - pomega D^-1 A) T (T: aggregates)
};

struct Hierarchy {
    std::vector<Level> levels;
    std::vector<double> coarse_inv;  // column-major inverse of the coarsest operator
    int32_t n_coarse = 0;
};

struct AmgParams {
    double theta = 0.0;
    int coarse_max = 256;
    int max_levels = 12;
};

// Throws std::runtime_error with a message on invalid input.
void build_grid(GridMetrics &g, int nx, int ny, const double *xf, const double *yf);
void build_model(Model &m, int nx, int ny, const double *xf, const double *yf, int nb,
                 const double *xb, const double *yb, const double *ubx, const double *uby,
                 double nu, double dt, int pin = 0);
void build_hierarchy(Hierarchy &h, const CSR &K, const AmgParams &p);
// The V-cycle restricted to levels lc..L-1 (pre >= 1 damped-Jacobi sweeps,
// the first from zero, restriction, recursion, exact solve on the coarsest
// level, prolongation, post sweeps) is a fixed linear map b -> x; returns its
// matrix, row-major n_lc x n_lc.
std::vector<double> coarse_cycle_matrix(const Hierarchy &h, int lc, int pre, int post);
// Levels from..L-1 formed anew from a new operator A of level `from`, with
// the aggregates and smoothing weights each level already holds: the
// Jacobi weights, P = (I - pomega D^-1 A) T, R = P^T, the Galerkin
// products and the inverse of the coarsest operator.
void regalerkin_from(Hierarchy &h, int from, CSR &&A);

// Operators of B^N for N > 1, built on the host for the device products:
// L = M Lhat R^-1 on the interior faces (n_q x n_q, rows sorted), the
// diagonal of B^1 = dt Mf^-1, Q^T = [G^T; E] (n_lambda x n_q), and a copy
// of K with row and column `pin` cleared except the diagonal.
CSR laplacian_csr(const GridMetrics &g);
std::vector<double> b1_diagonal(const GridMetrics &g, double dt);
CSR poisson_qt(const Model &m);
CSR pin_rows_cols(const CSR &K, int32_t pin);
// Throws unless every point's delta support lies on cells of its own width
// (Eq. 7) away from the domain edges: the test build_model makes
void check_points(const GridMetrics &g, int nb, const double *xb, const double *yb);

// helpers exposed for the host tests
double roma_phi(double s);
CSR csr_transpose(const CSR &A);

// The three-dimensional extension (the 7-point pressure stencil named as
// the next step in Sec. 7): Eqs. 6-11 carried over axis by axis.  Unknowns
// x fastest, then y, then z: u (faces x_1..x_{nx-1}) | v | w, then the
// cells and the 3 nb forces (x, y, z components) of lambda.  q = R u with
// R the face areas, M the centre-to-centre gaps across the faces,
// A = M R^-1 / dt - (nu/2) M Lhat R^-1 (7 points per row), B^1 = dt R M^-1,
// Q^T = [-D; E] with E = (control volume x product of three deltas) R^-1,
// K = Q^T B^1 Q with cell `pin` pinned.
struct Model3 {
    int32_t nx = 0, ny = 0, nz = 0, nb = 0, pin = 0;
    int64_t n_q = 0, n_cell = 0;
    CSR A, QT, Q, K;
    std::vector<double> b1;
};
void build_model3(Model3 &m, int nx, int ny, int nz, const double *xf, const double *yf, const double *zf, int nb,
                  const double *xb, const double *yb, const double *zb, double nu, double dt, int pin);
CSR csr_multiply(const CSR &A, const CSR &B);

}  // namespace ibpm
