// Host-side assembly: grid metrics, the regularised-delta interpolation E,
// the pinned matrix K = Q^T B^1 Q (stencil part, coupling rows), and the
// smoothed-aggregation hierarchy used by the AMG preconditioner.
//
// Discretisation (Sec. 2 of Layton, Krishnan & Barba; the symmetrising
// transformation it defers to Taira & Colonius is written out here):
//   q = R u with R = diag(dy_j | dx_i);  momentum rows scaled by
//   M = diag(Dx_i | Dy_j);  Mf = M R^{-1};  B^1 = dt Mf^{-1};
//   G = -D^T with D the interior-face divergence;  E = E^ R^{-1} with
//   E^_{k,i} = dA_i d_h(x_i - xi_k) d_h(y_i - eta_k)   (Eq. 7),
//   dA = Dx_i dy_j on u faces and dx_i Dy_j on v faces;
//   K = Q^T B^1 Q with Q = [G, E^T], one pressure cell pinned (row and
//   column cleared except the diagonal).
#include "setup.h"

#include <algorithm>
#include <thread>
#include <cmath>
#include <map>
#include <stdexcept>

namespace ibpm {

namespace {

void fail(const std::string &msg) { throw std::runtime_error(msg); }

// index of the cell [f[i], f[i+1]) holding x (clamped to the grid)
int cell_of(const std::vector<double> &f, double x) {
    int n = (int)f.size() - 1;
    int i = (int)(std::upper_bound(f.begin(), f.end(), x) - f.begin()) - 1;
    return std::min(std::max(i, 0), n - 1);
}

// width h of the cell holding x; every cell meeting the open support
// (x - 1.5h, x + 1.5h) -- the cells whose widths enter the weights -- must
// share it
double local_width(const std::vector<double> &f, const std::vector<double> &w, double x,
                   const char *axis) {
    int n = (int)w.size();
    int i0 = cell_of(f, x);
    if (i0 < 2 || i0 > n - 3)
        fail(std::string("Lagrangian point too close to the domain edge along ") + axis);
    double h = w[i0];
    // first cell with f[i+1] > x - 1.5h, last cell with f[i] < x + 1.5h
    const int first = (int)(std::upper_bound(f.begin(), f.end(), x - 1.5 * h) - f.begin()) - 1;
    const int last = (int)(std::lower_bound(f.begin(), f.end(), x + 1.5 * h) - f.begin()) - 1;
    for (int i = std::max(first, 0); i <= std::min(last, n - 1); ++i)
        if (std::fabs(w[i] - h) > 1e-9 * h)
            fail(std::string("grid is not uniform under the delta support along ") + axis);
    return h;
}

double delta_h(double r, double h) { return roma_phi(r / h) / h; }

}  // namespace

// Eq. (6): three-point regularised delta for unit spacing.  The inner
// branch is taken to include s = 0.
double roma_phi(double s) {
    s = std::fabs(s);
    if (s <= 0.5) return (1.0 + std::sqrt(1.0 - 3.0 * (s * s))) / 3.0;
    if (s <= 1.5) {
        double t = 1.0 - s;
        return (5.0 - 3.0 * s - std::sqrt(1.0 - 3.0 * (t * t))) / 6.0;
    }
    return 0.0;
}

void build_grid(GridMetrics &g, int nx, int ny, const double *xf, const double *yf) {
    if (nx < 4 || ny < 4) fail("need at least 4 cells per direction");
    if (!xf || !yf) fail("face arrays must not be NULL");
    g.nx = nx;
    g.ny = ny;
    g.xf.assign(xf, xf + nx + 1);
    g.yf.assign(yf, yf + ny + 1);
    g.dx.resize(nx);
    g.dy.resize(ny);
    g.xc.resize(nx);
    g.yc.resize(ny);
    for (int i = 0; i < nx; ++i) {
        g.dx[i] = g.xf[i + 1] - g.xf[i];
        if (!(g.dx[i] > 0)) fail("x faces must be strictly increasing");
        g.xc[i] = 0.5 * (g.xf[i] + g.xf[i + 1]);
    }
    for (int j = 0; j < ny; ++j) {
        g.dy[j] = g.yf[j + 1] - g.yf[j];
        if (!(g.dy[j] > 0)) fail("y faces must be strictly increasing");
        g.yc[j] = 0.5 * (g.yf[j] + g.yf[j + 1]);
    }
    g.Dx.resize(nx + 1);
    g.Dy.resize(ny + 1);
    g.Dx[0] = 0.5 * g.dx[0];
    for (int i = 1; i < nx; ++i) g.Dx[i] = 0.5 * (g.dx[i - 1] + g.dx[i]);
    g.Dx[nx] = 0.5 * g.dx[nx - 1];
    g.Dy[0] = 0.5 * g.dy[0];
    for (int j = 1; j < ny; ++j) g.Dy[j] = 0.5 * (g.dy[j - 1] + g.dy[j]);
    g.Dy[ny] = 0.5 * g.dy[ny - 1];
    g.n_u = (int64_t)(nx - 1) * ny;
    g.n_v = (int64_t)nx * (ny - 1);
    g.n_q = g.n_u + g.n_v;
    g.n_cell = (int64_t)nx * ny;
    if (g.n_q + 2 > INT32_MAX / 2) fail("grid too large for 32-bit indices");
}

namespace {

void build_E(Model &m, const double *xb, const double *yb) {
    const GridMetrics &g = m.g;
    int nb = m.nb;
    CSR &E = m.E;
    E.nrows = 2 * nb;
    E.ncols = (int32_t)g.n_q;
    E.ptr.assign(2 * nb + 1, 0);
    std::vector<std::vector<std::pair<int32_t, double>>> rows(2 * nb);
    for (int k = 0; k < nb; ++k) {
        double X = xb[k], Y = yb[k];
        double hx = local_width(g.xf, g.dx, X, "x");
        double hy = local_width(g.yf, g.dy, Y, "y");
        int i0 = cell_of(g.xf, X), j0 = cell_of(g.yf, Y);
        // u row k: faces x_i (i = 1..nx-1) at yc_j
        for (int j = std::max(0, j0 - 2); j <= std::min(g.ny - 1, j0 + 2); ++j) {
            if (!(std::fabs(g.yc[j] - Y) < 1.5 * hy)) continue;
            for (int i = std::max(1, i0 - 2); i <= std::min(g.nx - 1, i0 + 3); ++i) {
                if (!(std::fabs(g.xf[i] - X) < 1.5 * hx)) continue;
                double w = g.Dx[i] * g.dy[j] * delta_h(g.xf[i] - X, hx) * delta_h(g.yc[j] - Y, hy);
                rows[k].push_back({(int32_t)g.uidx(i, j), w * (1.0 / g.dy[j])});
            }
        }
        // v row nb+k: faces y_j (j = 1..ny-1) at xc_i
        for (int j = std::max(1, j0 - 2); j <= std::min(g.ny - 1, j0 + 3); ++j) {
            if (!(std::fabs(g.yf[j] - Y) < 1.5 * hy)) continue;
            for (int i = std::max(0, i0 - 2); i <= std::min(g.nx - 1, i0 + 2); ++i) {
                if (!(std::fabs(g.xc[i] - X) < 1.5 * hx)) continue;
                double w = g.dx[i] * g.Dy[j] * delta_h(g.xc[i] - X, hx) * delta_h(g.yf[j] - Y, hy);
                rows[nb + k].push_back({(int32_t)g.vidx(i, j), w * (1.0 / g.dx[i])});
            }
        }
    }
    for (int r = 0; r < 2 * nb; ++r) {
        std::sort(rows[r].begin(), rows[r].end());
        for (auto &e : rows[r]) {
            E.col.push_back(e.first);
            E.val.push_back(e.second);
        }
        E.ptr[r + 1] = (int32_t)E.col.size();
    }
}

// decode a flux index into (is_v, i, j)
inline void face_of(const GridMetrics &g, int64_t f, bool &is_v, int &i, int &j) {
    if (f < g.n_u) {
        is_v = false;
        j = (int)(f / (g.nx - 1));
        i = (int)(f % (g.nx - 1)) + 1;
    } else {
        is_v = true;
        int64_t r = f - g.n_u;
        j = (int)(r / g.nx) + 1;
        i = (int)(r % g.nx);
    }
}

// B^1 on a face: dt / (M / R)
inline double b1_face(const Model &m, bool is_v, int i, int j) {
    const GridMetrics &g = m.g;
    double Mf = is_v ? g.Dy[j] / g.dx[i] : g.Dx[i] / g.dy[j];
    return m.dt / Mf;
}

void build_coupling(Model &m) {
    const GridMetrics &g = m.g;
    int nb = m.nb;
    int64_t nc = g.n_cell;
    const CSR &E = m.E;
    // cell -> (force, value) for K_{phi f} = G^T B^1 E^T (pinned cell dropped)
    std::map<int64_t, std::map<int32_t, double>> cf;
    // face -> list of (force row, E value), for K_ff and for E^T gathers
    std::map<int64_t, std::vector<std::pair<int32_t, double>>> ft;
    for (int k = 0; k < 2 * nb; ++k) {
        for (int p = E.ptr[k]; p < E.ptr[k + 1]; ++p) {
            int64_t f = E.col[p];
            double e = E.val[p];
            bool is_v;
            int i, j;
            face_of(g, f, is_v, i, j);
            double t = b1_face(m, is_v, i, j) * e;
            // G^T: a face adds +1 to the cell on its high side, -1 to the low side
            int64_t c_hi = (int64_t)j * g.nx + i;
            int64_t c_lo = is_v ? (int64_t)(j - 1) * g.nx + i : (int64_t)j * g.nx + (i - 1);
            if (c_hi != m.pin) cf[c_hi][k] += t;
            if (c_lo != m.pin) cf[c_lo][k] -= t;
            ft[f].push_back({k, e});
        }
    }
    // bounding box of coupled cells
    m.cb_i0 = g.nx; m.cb_i1 = -1; m.cb_j0 = g.ny; m.cb_j1 = -1;
    for (auto &kv : cf) {
        int i = (int)(kv.first % g.nx), j = (int)(kv.first / g.nx);
        m.cb_i0 = std::min(m.cb_i0, i); m.cb_i1 = std::max(m.cb_i1, i);
        m.cb_j0 = std::min(m.cb_j0, j); m.cb_j1 = std::max(m.cb_j1, j);
    }
    if (cf.empty()) { m.cb_i0 = 0; m.cb_i1 = -1; m.cb_j0 = 0; m.cb_j1 = -1; }
    int bw = m.cb_i1 - m.cb_i0 + 1, bh = m.cb_j1 - m.cb_j0 + 1;
    m.Kcf = CSR();
    m.Kcf.nrows = std::max(0, bw * bh);
    m.Kcf.ncols = 2 * nb;
    m.Kcf.ptr.assign(m.Kcf.nrows + 1, 0);
    for (int jj = 0; jj < bh; ++jj)
        for (int ii = 0; ii < bw; ++ii) {
            int r = jj * bw + ii;
            int64_t c = (int64_t)(m.cb_j0 + jj) * g.nx + (m.cb_i0 + ii);
            auto it = cf.find(c);
            if (it != cf.end())
                for (auto &e : it->second) {
                    m.Kcf.col.push_back(e.first);
                    m.Kcf.val.push_back(e.second);
                }
            m.Kcf.ptr[r + 1] = (int32_t)m.Kcf.col.size();
        }
    // force rows: K_{f phi} (transpose of the cell coupling) and K_ff
    std::vector<std::map<int64_t, double>> frow(2 * nb);
    for (auto &kv : cf)
        for (auto &e : kv.second) frow[e.first][kv.first] = e.second;
    for (auto &kv : ft) {
        bool is_v;
        int i, j;
        face_of(g, kv.first, is_v, i, j);
        double b1 = b1_face(m, is_v, i, j);
        for (auto &a : kv.second)
            for (auto &b : kv.second) frow[a.first][nc + b.first] += (a.second * b1) * b.second;
    }
    m.Kf = CSR();
    m.Kf.nrows = 2 * nb;
    m.Kf.ncols = (int32_t)(nc + 2 * nb);
    m.Kf.ptr.assign(2 * nb + 1, 0);
    m.Kf_diag.assign(2 * nb, 0.0);
    for (int k = 0; k < 2 * nb; ++k) {
        for (auto &e : frow[k]) {
            m.Kf.col.push_back((int32_t)e.first);
            m.Kf.val.push_back(e.second);
            if (e.first == nc + k) m.Kf_diag[k] = e.second;
        }
        m.Kf.ptr[k + 1] = (int32_t)m.Kf.col.size();
    }
    // E^T gathers by face, u and v separately, over the face boxes
    m.fu_i0 = g.nx; m.fu_i1 = -1; m.fu_j0 = g.ny; m.fu_j1 = -1;
    m.fv_i0 = g.nx; m.fv_i1 = -1; m.fv_j0 = g.ny; m.fv_j1 = -1;
    for (auto &kv : ft) {
        bool is_v;
        int i, j;
        face_of(g, kv.first, is_v, i, j);
        if (!is_v) {
            m.fu_i0 = std::min(m.fu_i0, i); m.fu_i1 = std::max(m.fu_i1, i);
            m.fu_j0 = std::min(m.fu_j0, j); m.fu_j1 = std::max(m.fu_j1, j);
        } else {
            m.fv_i0 = std::min(m.fv_i0, i); m.fv_i1 = std::max(m.fv_i1, i);
            m.fv_j0 = std::min(m.fv_j0, j); m.fv_j1 = std::max(m.fv_j1, j);
        }
    }
    auto make_gather = [&](CSR &out, bool want_v, int i0, int i1, int j0, int j1) {
        out = CSR();
        int w = i1 - i0 + 1, h = j1 - j0 + 1;
        out.nrows = std::max(0, w * h);
        out.ncols = nb;
        out.ptr.assign(out.nrows + 1, 0);
        for (int jj = 0; jj < h; ++jj)
            for (int ii = 0; ii < w; ++ii) {
                int i = i0 + ii, j = j0 + jj;
                int64_t f = want_v ? g.vidx(i, j) : g.uidx(i, j);
                auto it = ft.find(f);
                if (it != ft.end()) {
                    std::vector<std::pair<int32_t, double>> es = it->second;
                    std::sort(es.begin(), es.end());
                    for (auto &e : es) {
                        out.col.push_back(want_v ? e.first - nb : e.first);
                        out.val.push_back(e.second);
                    }
                }
                out.ptr[jj * w + ii + 1] = (int32_t)out.col.size();
            }
    };
    if (m.fu_i1 < 0) { m.fu_i0 = 1; m.fu_i1 = 0; m.fu_j0 = 0; m.fu_j1 = -1; }
    if (m.fv_i1 < 0) { m.fv_i0 = 0; m.fv_i1 = -1; m.fv_j0 = 1; m.fv_j1 = 0; }
    make_gather(m.Etu, false, m.fu_i0, m.fu_i1, m.fu_j0, m.fu_j1);
    make_gather(m.Etv, true, m.fv_i0, m.fv_i1, m.fv_j0, m.fv_j1);
}

// Full pinned K in CSR (pressure stencil + coupling + force rows).
void build_full_K(Model &m) {
    const GridMetrics &g = m.g;
    int nx = g.nx, ny = g.ny;
    int64_t nc = g.n_cell;
    int nb = m.nb;
    CSR &K = m.K;
    K = CSR();
    K.nrows = K.ncols = (int32_t)(nc + 2 * nb);
    K.ptr.assign(K.nrows + 1, 0);
    K.col.reserve(5 * nc + m.Kcf.nnz() + m.Kf.nnz());
    K.val.reserve(K.col.capacity());
    int bw = m.cb_i1 - m.cb_i0 + 1;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int64_t c = (int64_t)j * nx + i;
            // B^1 on the four faces (0 where the face is a wall)
            double bw_ = i > 0 ? b1_face(m, false, i, j) : 0.0;
            double be_ = i < nx - 1 ? b1_face(m, false, i + 1, j) : 0.0;
            double bs_ = j > 0 ? b1_face(m, true, i, j) : 0.0;
            double bn_ = j < ny - 1 ? b1_face(m, true, i, j + 1) : 0.0;
            double diag = ((bw_ + be_) + bs_) + bn_;
            auto push = [&](int64_t col, double v) {
                K.col.push_back((int32_t)col);
                K.val.push_back(v);
            };
            if (c == m.pin) {
                push(c, diag);
            } else {
                if (j > 0 && c - nx != m.pin) push(c - nx, -bs_);
                if (i > 0 && c - 1 != m.pin) push(c - 1, -bw_);
                push(c, diag);
                if (i < nx - 1 && c + 1 != m.pin) push(c + 1, -be_);
                if (j < ny - 1 && c + nx != m.pin) push(c + nx, -bn_);
                if (i >= m.cb_i0 && i <= m.cb_i1 && j >= m.cb_j0 && j <= m.cb_j1) {
                    int r = (j - m.cb_j0) * bw + (i - m.cb_i0);
                    for (int p = m.Kcf.ptr[r]; p < m.Kcf.ptr[r + 1]; ++p)
                        push(nc + m.Kcf.col[p], m.Kcf.val[p]);
                }
            }
            K.ptr[c + 1] = (int32_t)K.col.size();
        }
    for (int k = 0; k < 2 * nb; ++k) {
        for (int p = m.Kf.ptr[k]; p < m.Kf.ptr[k + 1]; ++p) {
            K.col.push_back(m.Kf.col[p]);
            K.val.push_back(m.Kf.val[p]);
        }
        K.ptr[nc + k + 1] = (int32_t)K.col.size();
    }
}

// Delta weights at cell centres for the learned stage's force channels.
void build_cell_delta(Model &m, const double *xb, const double *yb) {
    const GridMetrics &g = m.g;
    int nb = m.nb;
    std::vector<std::vector<std::pair<int64_t, double>>> rows(nb);
    int i0 = g.nx, i1 = -1, j0 = g.ny, j1 = -1;
    for (int k = 0; k < nb; ++k) {
        double X = xb[k], Y = yb[k];
        double hx = local_width(g.xf, g.dx, X, "x");
        double hy = local_width(g.yf, g.dy, Y, "y");
        int ic = cell_of(g.xf, X), jc = cell_of(g.yf, Y);
        for (int j = std::max(0, jc - 2); j <= std::min(g.ny - 1, jc + 2); ++j) {
            if (!(std::fabs(g.yc[j] - Y) < 1.5 * hy)) continue;
            for (int i = std::max(0, ic - 2); i <= std::min(g.nx - 1, ic + 2); ++i) {
                if (!(std::fabs(g.xc[i] - X) < 1.5 * hx)) continue;
                double w = roma_phi((g.xc[i] - X) / hx) * roma_phi((g.yc[j] - Y) / hy);
                rows[k].push_back({(int64_t)j * g.nx + i, w});
                i0 = std::min(i0, i); i1 = std::max(i1, i);
                j0 = std::min(j0, j); j1 = std::max(j1, j);
            }
        }
    }
    m.Dp2c = CSR();
    m.Dp2c.nrows = nb;
    m.Dp2c.ncols = (int32_t)g.n_cell;
    m.Dp2c.ptr.assign(nb + 1, 0);
    for (int k = 0; k < nb; ++k) {
        for (auto &e : rows[k]) {
            m.Dp2c.col.push_back((int32_t)e.first);
            m.Dp2c.val.push_back(e.second);
        }
        m.Dp2c.ptr[k + 1] = (int32_t)m.Dp2c.col.size();
    }
    if (i1 < 0) { i0 = 0; i1 = -1; j0 = 0; j1 = -1; }
    m.dc_i0 = i0; m.dc_i1 = i1; m.dc_j0 = j0; m.dc_j1 = j1;
    int bw = i1 - i0 + 1, bh = j1 - j0 + 1;
    std::vector<std::vector<std::pair<int32_t, double>>> cells(std::max(0, bw * bh));
    for (int k = 0; k < nb; ++k)
        for (auto &e : rows[k]) {
            int i = (int)(e.first % g.nx), j = (int)(e.first / g.nx);
            cells[(j - j0) * bw + (i - i0)].push_back({k, e.second});
        }
    m.Dc2p = CSR();
    m.Dc2p.nrows = std::max(0, bw * bh);
    m.Dc2p.ncols = nb;
    m.Dc2p.ptr.assign(m.Dc2p.nrows + 1, 0);
    for (int r = 0; r < m.Dc2p.nrows; ++r) {
        for (auto &e : cells[r]) {
            m.Dc2p.col.push_back(e.first);
            m.Dc2p.val.push_back(e.second);
        }
        m.Dc2p.ptr[r + 1] = (int32_t)m.Dc2p.col.size();
    }
    m.hmin = *std::min_element(g.dx.begin(), g.dx.end());
    m.hmin = std::min(m.hmin, *std::min_element(g.dy.begin(), g.dy.end()));
}

}  // namespace

void build_model(Model &m, int nx, int ny, const double *xf, const double *yf, int nb,
                 const double *xb, const double *yb, const double *ubx, const double *uby,
                 double nu, double dt, int pin) {
    build_grid(m.g, nx, ny, xf, yf);
    if (pin < 0 || (int64_t)pin >= m.g.n_cell) fail("pin_cell must be a cell index in 0..nx*ny-1");
    m.pin = pin;
    if (nb < 0) fail("nb must be >= 0");
    if (nb > 0 && (!xb || !yb)) fail("body point arrays must not be NULL");
    if (!(nu > 0) || !(dt > 0)) fail("nu and dt must be positive");
    m.nb = nb;
    m.nu = nu;
    m.dt = dt;
    m.ub.assign(2 * nb, 0.0);
    for (int k = 0; k < nb; ++k) {
        if (ubx) m.ub[k] = ubx[k];
        if (uby) m.ub[nb + k] = uby[k];
    }
    build_E(m, xb, yb);
    build_coupling(m);
    build_full_K(m);
    build_cell_delta(m, xb, yb);
}

// ---------------------------------------------------------------------------
// sparse helpers

// ---------------------------------------------------------------------------
// Operators of B^N for N > 1 (Sec. 2, text after Eq. 11)

namespace {
// one row of a CSR under construction: entries appended in any order, then
// sorted by column (the columns of a row are distinct)
void push_row(CSR &M, std::vector<std::pair<int32_t, double>> &row) {
    std::sort(row.begin(), row.end());
    for (const auto &e : row) {
        M.col.push_back(e.first);
        M.val.push_back(e.second);
    }
    M.ptr.push_back((int32_t)M.col.size());
    row.clear();
}
}  // namespace

CSR laplacian_csr(const GridMetrics &g) {
    // L = M Lhat R^-1 on the interior faces: Lhat the 3-point second
    // difference per direction with the gaps of the staggered grid, the
    // wall values left out (they enter the right-hand side)
    const int nx = g.nx, ny = g.ny;
    CSR L;
    L.nrows = L.ncols = (int32_t)g.n_q;
    L.ptr.reserve(g.n_q + 1);
    L.ptr.push_back(0);
    L.col.reserve(5 * g.n_q);
    L.val.reserve(5 * g.n_q);
    std::vector<std::pair<int32_t, double>> row;
    for (int j = 0; j < ny; ++j)
        for (int i = 1; i < nx; ++i) {
            // u at (x_i, yc_j): row weight Dx_i, unknown scale dy
            const double lo_x = 1.0 / (g.dx[i - 1] * g.Dx[i]), hi_x = 1.0 / (g.dx[i] * g.Dx[i]);
            const double lo_y = 1.0 / (g.Dy[j] * g.dy[j]), hi_y = 1.0 / (g.Dy[j + 1] * g.dy[j]);
            const double m = g.Dx[i];
            row.push_back({(int32_t)g.uidx(i, j), -m * (lo_x + hi_x + lo_y + hi_y) / g.dy[j]});
            if (i > 1) row.push_back({(int32_t)g.uidx(i - 1, j), m * lo_x / g.dy[j]});
            if (i < nx - 1) row.push_back({(int32_t)g.uidx(i + 1, j), m * hi_x / g.dy[j]});
            if (j > 0) row.push_back({(int32_t)g.uidx(i, j - 1), m * lo_y / g.dy[j - 1]});
            if (j < ny - 1) row.push_back({(int32_t)g.uidx(i, j + 1), m * hi_y / g.dy[j + 1]});
            push_row(L, row);
        }
    for (int j = 1; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            // v at (xc_i, y_j): row weight Dy_j, unknown scale dx
            const double lo_x = 1.0 / (g.Dx[i] * g.dx[i]), hi_x = 1.0 / (g.Dx[i + 1] * g.dx[i]);
            const double lo_y = 1.0 / (g.dy[j - 1] * g.Dy[j]), hi_y = 1.0 / (g.dy[j] * g.Dy[j]);
            const double m = g.Dy[j];
            row.push_back({(int32_t)g.vidx(i, j), -m * (lo_x + hi_x + lo_y + hi_y) / g.dx[i]});
            if (i > 0) row.push_back({(int32_t)g.vidx(i - 1, j), m * lo_x / g.dx[i - 1]});
            if (i < nx - 1) row.push_back({(int32_t)g.vidx(i + 1, j), m * hi_x / g.dx[i + 1]});
            if (j > 1) row.push_back({(int32_t)g.vidx(i, j - 1), m * lo_y / g.dx[i]});
            if (j < ny - 1) row.push_back({(int32_t)g.vidx(i, j + 1), m * hi_y / g.dx[i]});
            push_row(L, row);
        }
    return L;
}

std::vector<double> b1_diagonal(const GridMetrics &g, double dt) {
    // B^1 = dt Mf^-1, Mf = M R^-1: dt dy_j / Dx_i on u faces, dt dx_i / Dy_j on v faces
    std::vector<double> b((size_t)g.n_q);
    for (int j = 0; j < g.ny; ++j)
        for (int i = 1; i < g.nx; ++i) b[g.uidx(i, j)] = dt * g.dy[j] / g.Dx[i];
    for (int j = 1; j < g.ny; ++j)
        for (int i = 0; i < g.nx; ++i) b[g.vidx(i, j)] = dt * g.dx[i] / g.Dy[j];
    return b;
}

CSR poisson_qt(const Model &m) {
    // Q^T = [G^T; E] (n_lambda x n_q): G^T = -D on the cells (interior faces
    // only), then the interpolation rows
    const GridMetrics &g = m.g;
    const int nx = g.nx, ny = g.ny;
    CSR Q;
    Q.nrows = (int32_t)(g.n_cell + 2 * m.nb);
    Q.ncols = (int32_t)g.n_q;
    Q.ptr.push_back(0);
    std::vector<std::pair<int32_t, double>> row;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (i > 0) row.push_back({(int32_t)g.uidx(i, j), 1.0});
            if (i < nx - 1) row.push_back({(int32_t)g.uidx(i + 1, j), -1.0});
            if (j > 0) row.push_back({(int32_t)g.vidx(i, j), 1.0});
            if (j < ny - 1) row.push_back({(int32_t)g.vidx(i, j + 1), -1.0});
            push_row(Q, row);
        }
    for (int k = 0; k < m.E.nrows; ++k) {
        for (int p = m.E.ptr[k]; p < m.E.ptr[k + 1]; ++p) row.push_back({m.E.col[p], m.E.val[p]});
        push_row(Q, row);
    }
    return Q;
}

void check_points(const GridMetrics &g, int nb, const double *xb, const double *yb) {
    for (int k = 0; k < nb; ++k) {
        if (!std::isfinite(xb[k]) || !std::isfinite(yb[k])) fail("point positions must be finite");
        (void)local_width(g.xf, g.dx, xb[k], "x");
        (void)local_width(g.yf, g.dy, yb[k], "y");
    }
}

CSR pin_rows_cols(const CSR &K, int32_t pin) {
    // clear row and column `pin` except the diagonal entry
    CSR out;
    out.nrows = K.nrows;
    out.ncols = K.ncols;
    out.ptr.reserve(K.nrows + 1);
    out.ptr.push_back(0);
    out.col.reserve(K.col.size());
    out.val.reserve(K.val.size());
    for (int32_t r = 0; r < K.nrows; ++r) {
        for (int32_t p = K.ptr[r]; p < K.ptr[r + 1]; ++p) {
            const int32_t c = K.col[p];
            if ((r == pin || c == pin) && r != c) continue;
            out.col.push_back(c);
            out.val.push_back(K.val[p]);
        }
        out.ptr.push_back((int32_t)out.col.size());
    }
    return out;
}

CSR csr_transpose(const CSR &A) {
    CSR T;
    T.nrows = A.ncols;
    T.ncols = A.nrows;
    T.ptr.assign(T.nrows + 1, 0);
    for (int32_t c : A.col) T.ptr[c + 1]++;
    for (int r = 0; r < T.nrows; ++r) T.ptr[r + 1] += T.ptr[r];
    T.col.resize(A.col.size());
    T.val.resize(A.val.size());
    std::vector<int32_t> pos(T.ptr.begin(), T.ptr.end() - 1);
    for (int r = 0; r < A.nrows; ++r)
        for (int p = A.ptr[r]; p < A.ptr[r + 1]; ++p) {
            int32_t q = pos[A.col[p]]++;
            T.col[q] = r;
            T.val[q] = A.val[p];
        }
    return T;
}

// Gustavson product with a dense accumulator; output rows sorted.
CSR csr_multiply(const CSR &A, const CSR &B) {
    if (A.ncols != B.nrows) fail("csr_multiply: shape mismatch");
    CSR C;
    C.nrows = A.nrows;
    C.ncols = B.ncols;
    C.ptr.assign(C.nrows + 1, 0);
    std::vector<double> acc(B.ncols, 0.0);
    std::vector<int32_t> mark(B.ncols, -1);
    std::vector<int32_t> cols;
    for (int r = 0; r < A.nrows; ++r) {
        cols.clear();
        for (int p = A.ptr[r]; p < A.ptr[r + 1]; ++p) {
            int32_t k = A.col[p];
            double a = A.val[p];
            for (int q = B.ptr[k]; q < B.ptr[k + 1]; ++q) {
                int32_t c = B.col[q];
                if (mark[c] != r) {
                    mark[c] = r;
                    acc[c] = a * B.val[q];
                    cols.push_back(c);
                } else {
                    acc[c] += a * B.val[q];
                }
            }
        }
        std::sort(cols.begin(), cols.end());
        for (int32_t c : cols) {
            C.col.push_back(c);
            C.val.push_back(acc[c]);
        }
        C.ptr[r + 1] = (int32_t)C.col.size();
    }
    return C;
}

// ---------------------------------------------------------------------------
// smoothed aggregation (Sec. 3: PCG with a smoothed-aggregation AMG
// preconditioner).  Reading of the unstated parameters: strength
// |a_ij| >= max(theta, 1e-12) sqrt(|a_ii a_jj|); three greedy aggregation
// passes in natural order; constant tentative prolongator; one damped
// Jacobi smoothing step of it with weight 4 / (3 rho); Galerkin coarse
// operator.  rho estimates the spectral radius of D^{-1} A (the scaling of
// the Jacobi weights in Cusp's smoothed aggregation, which Sec. 3 uses): the
// largest Ritz value of a fixed number of Lanczos steps on D^{-1/2} A D^{-1/2}
// from a fixed pseudo-random start.  A row-sum (Gershgorin) bound is no
// substitute on the coupled system: the pressure rows next to the force
// unknowns push it several times above rho.

namespace {

double diag_of(const CSR &A, int r) {
    for (int p = A.ptr[r]; p < A.ptr[r + 1]; ++p)
        if (A.col[p] == r) return A.val[p];
    return 0.0;
}

// splitmix64 output for counter k (Steele, Lea & Flood, OOPSLA 2014): the
// state advanced k times by the golden-ratio increment, then mixed
uint64_t splitmix64_at(uint64_t k) {
    uint64_t z = k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Number of eigenvalues of the symmetric tridiagonal (a, b) below x
// (Sturm sequence of the LDL^T pivots).
int sturm_below(const std::vector<double> &a, const std::vector<double> &b, double x) {
    int cnt = 0;
    double q = 1.0;
    for (size_t i = 0; i < a.size(); ++i) {
        double off = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
        q = (a[i] - x) - (i > 0 ? off / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// Largest eigenvalue of the symmetric tridiagonal (a, b) by bisection
// between its Gershgorin limits.
double tridiag_max_eig(const std::vector<double> &a, const std::vector<double> &b) {
    const size_t k = a.size();
    double lo = a[0], hi = a[0];
    for (size_t i = 0; i < k; ++i) {
        double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_below(a, b, mid) == (int)k) hi = mid;   // every eigenvalue below mid
        else lo = mid;
    }
    return hi;
}

constexpr int kLanczosSteps = 20;

// Spectral radius estimate of D^{-1} A (A symmetric, positive diagonal d):
// Lanczos on S = D^{-1/2} A D^{-1/2}, which is similar to D^{-1} A, from the
// start v_i = u(i) - 1/2 with u(i) the top 53 bits of splitmix64(i + 1)
// over 2^53; each new vector is orthogonalised twice against all earlier
// ones (classical Gram-Schmidt, repeated), and the iteration ends early when
// what is left of it is below 1e-12 of |S v| (an invariant Krylov space);
// the estimate is the largest eigenvalue of the Lanczos tridiagonal.
double lanczos_rho(const CSR &A, const std::vector<double> &d) {
    const int n = A.nrows;
    const int k = std::min(kLanczosSteps, n);
    std::vector<double> s(n);
    for (int i = 0; i < n; ++i) s[i] = 1.0 / std::sqrt(d[i]);
    std::vector<std::vector<double>> V;
    std::vector<double> v(n), w(n), sv(n), h;
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) {
        v[i] = (double)(splitmix64_at((uint64_t)i + 1) >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        nrm += v[i] * v[i];
    }
    nrm = std::sqrt(nrm);
    for (int i = 0; i < n; ++i) v[i] /= nrm;
    std::vector<double> alpha, beta;
    for (int j = 0; j < k; ++j) {
        V.push_back(v);
        for (int i = 0; i < n; ++i) sv[i] = s[i] * v[i];
        double a = 0.0;
        for (int r = 0; r < n; ++r) {
            double t = 0.0;
            for (int p = A.ptr[r]; p < A.ptr[r + 1]; ++p) t += A.val[p] * sv[A.col[p]];
            w[r] = s[r] * t;
            a += v[r] * w[r];
        }
        alpha.push_back(a);
        double wn = 0.0;
        for (int i = 0; i < n; ++i) wn += w[i] * w[i];
        wn = std::sqrt(wn);
        for (int pass = 0; pass < 2; ++pass) {
            h.assign(V.size(), 0.0);
            for (size_t m = 0; m < V.size(); ++m) {
                double t = 0.0;
                for (int i = 0; i < n; ++i) t += V[m][i] * w[i];
                h[m] = t;
            }
            for (size_t m = 0; m < V.size(); ++m)
                for (int i = 0; i < n; ++i) w[i] -= h[m] * V[m][i];
        }
        double b = 0.0;
        for (int i = 0; i < n; ++i) b += w[i] * w[i];
        b = std::sqrt(b);
        if (j == k - 1 || b <= 1e-12 * wn) break;
        beta.push_back(b);
        for (int i = 0; i < n; ++i) v[i] = w[i] / b;
    }
    beta.resize(alpha.size() > 0 ? alpha.size() - 1 : 0);
    return tridiag_max_eig(alpha, beta);
}

// strong-neighbour lists (sorted, excluding the diagonal)
void strength_graph(const CSR &A, const std::vector<double> &d, double theta,
                    std::vector<int32_t> &sptr, std::vector<int32_t> &sidx) {
    double thr = std::max(theta, 1e-12);
    sptr.assign(A.nrows + 1, 0);
    sidx.clear();
    for (int r = 0; r < A.nrows; ++r) {
        for (int p = A.ptr[r]; p < A.ptr[r + 1]; ++p) {
            int c = A.col[p];
            if (c == r) continue;
            if (std::fabs(A.val[p]) >= thr * std::sqrt(std::fabs(d[r] * d[c]))) sidx.push_back(c);
        }
        sptr[r + 1] = (int32_t)sidx.size();
    }
}

int32_t aggregate(int n, const std::vector<int32_t> &sptr, const std::vector<int32_t> &sidx,
                  std::vector<int32_t> &agg) {
    agg.assign(n, -1);
    int32_t nagg = 0;
    // pass 1: a node whose strong neighbours are all free roots an aggregate
    for (int i = 0; i < n; ++i) {
        if (agg[i] != -1) continue;
        bool free_nbhd = true;
        for (int p = sptr[i]; p < sptr[i + 1]; ++p)
            if (agg[sidx[p]] != -1) { free_nbhd = false; break; }
        if (!free_nbhd) continue;
        agg[i] = nagg;
        for (int p = sptr[i]; p < sptr[i + 1]; ++p) agg[sidx[p]] = nagg;
        ++nagg;
    }
    std::vector<int32_t> pass1 = agg;
    // pass 2: join the aggregate of the lowest-index neighbour taken in pass 1
    for (int i = 0; i < n; ++i) {
        if (agg[i] != -1) continue;
        for (int p = sptr[i]; p < sptr[i + 1]; ++p)
            if (pass1[sidx[p]] != -1) { agg[i] = pass1[sidx[p]]; break; }
    }
    // pass 3: remaining nodes root aggregates with their free neighbours
    for (int i = 0; i < n; ++i) {
        if (agg[i] != -1) continue;
        agg[i] = nagg;
        for (int p = sptr[i]; p < sptr[i + 1]; ++p)
            if (agg[sidx[p]] == -1) agg[sidx[p]] = nagg;
        ++nagg;
    }
    return nagg;
}

// P = T - w D^{-1} A T with T_{i,agg(i)} = 1
CSR smoothed_prolongator(const CSR &A, const std::vector<double> &d,
                         const std::vector<int32_t> &agg, int32_t nagg, double w) {
    CSR P;
    P.nrows = A.nrows;
    P.ncols = nagg;
    P.ptr.assign(A.nrows + 1, 0);
    std::vector<double> acc(nagg, 0.0);
    std::vector<int32_t> mark(nagg, -1);
    std::vector<int32_t> cols;
    for (int r = 0; r < A.nrows; ++r) {
        cols.clear();
        for (int p = A.ptr[r]; p < A.ptr[r + 1]; ++p) {
            int32_t a = agg[A.col[p]];
            if (mark[a] != r) { mark[a] = r; acc[a] = A.val[p]; cols.push_back(a); }
            else acc[a] += A.val[p];
        }
        if (mark[agg[r]] != r) { mark[agg[r]] = r; acc[agg[r]] = 0.0; cols.push_back(agg[r]); }
        std::sort(cols.begin(), cols.end());
        double dinv = 1.0 / d[r];
        for (int32_t a : cols) {
            double t = (a == agg[r]) ? 1.0 : 0.0;
            P.col.push_back(a);
            P.val.push_back(t - w * (dinv * acc[a]));
        }
        P.ptr[r + 1] = (int32_t)P.col.size();
    }
    return P;
}

void finish_level(Level &L) {
    int n = L.A.nrows;
    std::vector<double> d(n);
    for (int r = 0; r < n; ++r) {
        d[r] = diag_of(L.A, r);
        if (!(d[r] > 0)) fail("AMG: non-positive diagonal");
    }
    L.rho = lanczos_rho(L.A, d);
    if (!(L.rho > 0) || !std::isfinite(L.rho)) fail("AMG: spectral radius estimate failed");
    L.omega = 4.0 / (3.0 * L.rho);
    L.wdinv.resize(n);
    for (int r = 0; r < n; ++r) L.wdinv[r] = L.omega / d[r];
}

// dense Cholesky (lower) and explicit inverse, column-major output
void dense_spd_inverse(const CSR &A, std::vector<double> &inv) {
    int n = A.nrows;
    std::vector<double> M((size_t)n * n, 0.0);   // row-major
    for (int r = 0; r < n; ++r)
        for (int p = A.ptr[r]; p < A.ptr[r + 1]; ++p) M[(size_t)r * n + A.col[p]] = A.val[p];
    // Cholesky in place (lower)
    for (int j = 0; j < n; ++j) {
        double s = M[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= M[(size_t)j * n + k] * M[(size_t)j * n + k];
        if (!(s > 0)) fail("AMG: coarsest operator is not positive definite");
        double ljj = std::sqrt(s);
        M[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = M[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= M[(size_t)i * n + k] * M[(size_t)j * n + k];
            M[(size_t)i * n + j] = t / ljj;
        }
    }
    inv.assign((size_t)n * n, 0.0);
    std::vector<double> y(n);
    for (int c = 0; c < n; ++c) {
        // L y = e_c
        for (int i = 0; i < n; ++i) {
            double t = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) t -= M[(size_t)i * n + k] * y[k];
            y[i] = t / M[(size_t)i * n + i];
        }
        // L^T x = y
        for (int i = n - 1; i >= 0; --i) {
            double t = y[i];
            for (int k = i + 1; k < n; ++k) t -= M[(size_t)k * n + i] * y[k];
            y[i] = t / M[(size_t)i * n + i];
        }
        for (int i = 0; i < n; ++i) inv[(size_t)c * n + i] = y[i];
    }
}

}  // namespace

void build_hierarchy(Hierarchy &h, const CSR &K, const AmgParams &prm) {
    h.levels.clear();
    h.levels.emplace_back();
    h.levels[0].A = K;
    finish_level(h.levels[0]);
    while (h.levels.back().A.nrows > prm.coarse_max && (int)h.levels.size() < prm.max_levels) {
        Level &L = h.levels.back();
        int n = L.A.nrows;
        std::vector<double> d(n);
        for (int r = 0; r < n; ++r) d[r] = diag_of(L.A, r);
        std::vector<int32_t> sptr, sidx;
        strength_graph(L.A, d, prm.theta, sptr, sidx);
        std::vector<int32_t> agg;
        int32_t nagg = aggregate(n, sptr, sidx, agg);
        if (nagg >= n) break;
        double w = L.omega;
        CSR P = smoothed_prolongator(L.A, d, agg, nagg, w);
        CSR R = csr_transpose(P);
        CSR RA = csr_multiply(R, L.A);
        CSR Ac = csr_multiply(RA, P);
        L.P = std::move(P);
        L.R = std::move(R);
        L.agg = std::move(agg);
        L.pomega = w;
        h.levels.emplace_back();
        h.levels.back().A = std::move(Ac);
        finish_level(h.levels.back());
    }
    const CSR &Ac = h.levels.back().A;
    if (Ac.nrows > 4096) fail("AMG: coarsest level too large for a dense solve");
    h.n_coarse = Ac.nrows;
    dense_spd_inverse(Ac, h.coarse_inv);
}

// ---------------------------------------------------------------------------
// Three dimensions

namespace {

struct Axis {
    std::vector<double> f, w, c, D;   // faces, widths, centres, centre-to-centre gaps (n + 1)
    int n = 0;
};

Axis make_axis(int n, const double *f, const char *name) {
    Axis a;
    if (n < 2) fail(std::string("need at least 2 cells along ") + name);
    a.n = n;
    a.f.assign(f, f + n + 1);
    a.w.resize(n);
    a.c.resize(n);
    for (int i = 0; i < n; ++i) {
        a.w[i] = a.f[i + 1] - a.f[i];
        if (!(a.w[i] > 0) || !std::isfinite(a.w[i])) fail(std::string("faces must be finite and increasing along ") + name);
        a.c[i] = 0.5 * (a.f[i] + a.f[i + 1]);
    }
    a.D.resize(n + 1);
    a.D[0] = 0.5 * a.w[0];
    a.D[n] = 0.5 * a.w[n - 1];
    for (int i = 1; i < n; ++i) a.D[i] = 0.5 * (a.w[i - 1] + a.w[i]);
    return a;
}

}  // namespace

void build_model3(Model3 &m, int nx, int ny, int nz, const double *xf, const double *yf, const double *zf, int nb,
                  const double *xb, const double *yb, const double *zb, double nu, double dt, int pin) {
    if (!xf || !yf || !zf) fail("face arrays are NULL");
    if (nb < 0 || (nb > 0 && (!xb || !yb || !zb))) fail("bad body points");
    if (!(nu > 0) || !(dt > 0)) fail("nu and dt must be positive");
    const Axis ax[3] = {make_axis(nx, xf, "x"), make_axis(ny, yf, "y"), make_axis(nz, zf, "z")};
    m = Model3();
    m.nx = nx;
    m.ny = ny;
    m.nz = nz;
    m.nb = nb;
    m.n_cell = (int64_t)nx * ny * nz;
    if (pin < 0 || pin >= m.n_cell) fail("pin_cell out of range");
    m.pin = pin;
    // component a: counts per axis and offset in q
    int64_t cnt[3][3], off[3];
    int64_t tot = 0;
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) cnt[a][b] = ax[b].n - (a == b ? 1 : 0);
        off[a] = tot;
        tot += cnt[a][0] * cnt[a][1] * cnt[a][2];
    }
    m.n_q = tot;
    const int64_t n_l = m.n_cell + 3 * (int64_t)nb;
    if (tot >= INT32_MAX || n_l >= INT32_MAX) fail("grid too large");
    // index of component a at per-axis indices (the own axis counted from
    // the first interior face line)
    auto fidx = [&](int a, const int64_t *id) {
        return off[a] + (id[2] * cnt[a][1] + id[1]) * cnt[a][0] + id[0];
    };
    // per-unknown metrics: M (gap across the face), R (face area)
    m.b1.resize(tot);
    std::vector<double> Mv(tot), Rv(tot);
    for (int a = 0; a < 3; ++a)
        for (int64_t k = 0; k < cnt[a][2]; ++k)
            for (int64_t j = 0; j < cnt[a][1]; ++j)
                for (int64_t i = 0; i < cnt[a][0]; ++i) {
                    const int64_t id[3] = {i, j, k};
                    const int64_t f = fidx(a, id);
                    double M = 1.0, R = 1.0;
                    for (int b = 0; b < 3; ++b) {
                        if (b == a) M = ax[b].D[id[b] + 1];
                        else R *= ax[b].w[id[b]];
                    }
                    Mv[f] = M;
                    Rv[f] = R;
                    m.b1[f] = dt * R / M;
                }
    // A: 7 points per row, columns in increasing order (z-, y-, x-, centre, x+, y+, z+)
    {
        CSR &A = m.A;
        A.nrows = A.ncols = (int32_t)tot;
        A.ptr.assign(1, 0);
        A.col.reserve(7 * tot);
        A.val.reserve(7 * tot);
        for (int a = 0; a < 3; ++a)
            for (int64_t k = 0; k < cnt[a][2]; ++k)
                for (int64_t j = 0; j < cnt[a][1]; ++j)
                    for (int64_t i = 0; i < cnt[a][0]; ++i) {
                        const int64_t id[3] = {i, j, k};
                        const int64_t f = fidx(a, id);
                        double lo[3], hi[3];
                        bool has_lo[3], has_hi[3];
                        double diag_l = 0.0;
                        for (int b = 0; b < 3; ++b) {
                            double cg, lg, rg;
                            if (b == a) {   // nodes on face lines 1..n-1: gaps are cell widths
                                const int64_t t = id[b] + 1;
                                cg = ax[b].D[t];
                                lg = ax[b].w[t - 1];
                                rg = ax[b].w[t];
                            } else {        // nodes at cell centres: gaps are centre distances
                                const int64_t t = id[b];
                                cg = ax[b].w[t];
                                lg = ax[b].D[t];
                                rg = ax[b].D[t + 1];
                            }
                            lo[b] = 1.0 / (lg * cg);
                            hi[b] = 1.0 / (rg * cg);
                            diag_l -= lo[b] + hi[b];
                            has_lo[b] = id[b] > 0;
                            has_hi[b] = id[b] < cnt[a][b] - 1;
                        }
                        const double Mf = Mv[f] / Rv[f];
                        auto push = [&](int64_t g, double lhat) {
                            // L = M Lhat R^-1: row weight M_f, column scale 1 / R_g
                            A.col.push_back((int32_t)g);
                            A.val.push_back(-0.5 * nu * (Mv[f] * lhat / Rv[g]));
                        };
                        const int64_t stride[3] = {1, cnt[a][0], cnt[a][0] * cnt[a][1]};
                        for (int b = 2; b >= 0; --b)
                            if (has_lo[b]) push(f - stride[b], lo[b]);
                        A.col.push_back((int32_t)f);
                        A.val.push_back(Mf / dt - 0.5 * nu * (Mv[f] * diag_l / Rv[f]));
                        for (int b = 0; b < 3; ++b)
                            if (has_hi[b]) push(f + stride[b], hi[b]);
                        A.ptr.push_back((int32_t)A.col.size());
                    }
    }
    // Q^T = [-D; E]
    CSR &QT = m.QT;
    QT.nrows = (int32_t)n_l;
    QT.ncols = (int32_t)tot;
    QT.ptr.assign(1, 0);
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t cid[3] = {i, j, k};
                for (int a = 0; a < 3; ++a) {
                    // low face (outward flux -q): -D gives +1; high face: -1
                    if (cid[a] >= 1) {
                        int64_t id[3] = {i, j, k};
                        id[a] -= 1;
                        QT.col.push_back((int32_t)fidx(a, id));
                        QT.val.push_back(1.0);
                    }
                    if (cid[a] <= ax[a].n - 2) {
                        QT.col.push_back((int32_t)fidx(a, cid));
                        QT.val.push_back(-1.0);
                    }
                }
                QT.ptr.push_back((int32_t)QT.col.size());
            }
    const double *P[3] = {xb, yb, zb};
    std::vector<double> h(3 * (size_t)nb);
    std::vector<int> cell(3 * (size_t)nb);
    for (int p = 0; p < nb; ++p)
        for (int b = 0; b < 3; ++b) {
            if (!std::isfinite(P[b][p])) fail("point positions must be finite");
            static const char *const names[3] = {"x", "y", "z"};
            h[3 * p + b] = local_width(ax[b].f, ax[b].w, P[b][p], names[b]);
            cell[3 * p + b] = cell_of(ax[b].f, P[b][p]);
        }
    for (int a = 0; a < 3; ++a)
        for (int p = 0; p < nb; ++p) {
            // candidate indices per axis (own axis: face lines 1..n-1, as
            // component indices 0..n-2; others: cells 0..n-1)
            std::vector<int64_t> near[3];
            std::vector<double> wt[3];
            for (int b = 0; b < 3; ++b) {
                const double X = P[b][p], hb = h[3 * p + b];
                const int c0 = cell[3 * p + b];
                for (int t = c0 - 2; t <= c0 + 3; ++t) {
                    double pos;
                    int64_t idx;
                    if (b == a) {
                        if (t < 1 || t > ax[b].n - 1) continue;
                        pos = ax[b].f[t];
                        idx = t - 1;
                    } else {
                        if (t < 0 || t > ax[b].n - 1) continue;
                        pos = ax[b].c[t];
                        idx = t;
                    }
                    if (!(std::fabs(pos - X) < 1.5 * hb)) continue;
                    near[b].push_back(idx);
                    wt[b].push_back(delta_h(pos - X, hb));
                }
            }
            for (size_t kk = 0; kk < near[2].size(); ++kk)
                for (size_t jj = 0; jj < near[1].size(); ++jj)
                    for (size_t ii = 0; ii < near[0].size(); ++ii) {
                        const int64_t id[3] = {near[0][ii], near[1][jj], near[2][kk]};
                        const int64_t f = fidx(a, id);
                        // control volume M R times the three deltas, then R^-1
                        const double v = (Mv[f] * Rv[f]) * (wt[0][ii] * wt[1][jj] * wt[2][kk]);
                        QT.col.push_back((int32_t)f);
                        QT.val.push_back(v * (1.0 / Rv[f]));
                    }
            QT.ptr.push_back((int32_t)QT.col.size());
        }
    m.Q = csr_transpose(QT);
    // K = Q^T (B^1 Q), pinned
    CSR BQ = m.Q;
    for (int32_t r = 0; r < BQ.nrows; ++r)
        for (int32_t q = BQ.ptr[r]; q < BQ.ptr[r + 1]; ++q) BQ.val[q] *= m.b1[r];
    m.K = pin_rows_cols(csr_multiply(QT, BQ), pin);
}

void regalerkin_from(Hierarchy &h, int from, CSR &&A) {
    const int L = (int)h.levels.size();
    if (from < 0 || from >= L) fail("hierarchy refresh: bad level");
    h.levels[from].A = std::move(A);
    for (int l = from; l < L; ++l) {
        Level &lv = h.levels[l];
        const int n = lv.A.nrows;
        std::vector<double> d(n);
        for (int r = 0; r < n; ++r) {
            d[r] = diag_of(lv.A, r);
            if (!(d[r] > 0)) fail("AMG: non-positive diagonal");
        }
        lv.wdinv.resize(n);
        for (int r = 0; r < n; ++r) lv.wdinv[r] = lv.omega / d[r];
        if (l == L - 1) break;
        CSR P = smoothed_prolongator(lv.A, d, lv.agg, h.levels[l + 1].A.nrows, lv.pomega);
        CSR R = csr_transpose(P);
        CSR RA = csr_multiply(R, lv.A);
        h.levels[l + 1].A = csr_multiply(RA, P);
        lv.P = std::move(P);
        lv.R = std::move(R);
    }
    dense_spd_inverse(h.levels.back().A, h.coarse_inv);
}

namespace {

void csr_apply(const CSR &A, const double *x, double *y) {
    for (int i = 0; i < A.nrows; ++i) {
        double s = 0.0;
        for (int p = A.ptr[i]; p < A.ptr[i + 1]; ++p) s += A.val[p] * x[A.col[p]];
        y[i] = s;
    }
}

// x = cycle_l(b) on levels l..L-1 (x has n_l entries)
void cycle_from(const Hierarchy &h, int l, int pre, int post, const std::vector<double> &b,
                std::vector<double> &x) {
    const int L = (int)h.levels.size();
    const Level &lv = h.levels[l];
    const int n = lv.A.nrows;
    x.assign(n, 0.0);
    if (l == L - 1) {
        const int nc = h.n_coarse;
        for (int k = 0; k < nc; ++k)
            for (int i = 0; i < nc; ++i) x[i] += h.coarse_inv[(size_t)k * nc + i] * b[k];
        return;
    }
    std::vector<double> ax(n), r(n);
    auto sweep = [&]() {
        csr_apply(lv.A, x.data(), ax.data());
        for (int i = 0; i < n; ++i) x[i] += lv.wdinv[i] * (b[i] - ax[i]);
    };
    for (int i = 0; i < n; ++i) x[i] = lv.wdinv[i] * b[i];
    for (int k = 1; k < pre; ++k) sweep();
    csr_apply(lv.A, x.data(), ax.data());
    for (int i = 0; i < n; ++i) r[i] = b[i] - ax[i];
    std::vector<double> bc(lv.R.nrows), xc, px(n);
    csr_apply(lv.R, r.data(), bc.data());
    cycle_from(h, l + 1, pre, post, bc, xc);
    csr_apply(lv.P, xc.data(), px.data());
    for (int i = 0; i < n; ++i) x[i] += px[i];
    for (int k = 0; k < post; ++k) sweep();
}

}  // namespace

std::vector<double> coarse_cycle_matrix(const Hierarchy &h, int lc, int pre, int post) {
    if (lc < 0 || lc >= (int)h.levels.size() || pre < 1) fail("coarse cycle: bad level or sweep count");
    const int n = h.levels[lc].A.nrows;
    std::vector<double> C((size_t)n * n);
    // the columns are independent cycles on unit vectors: a few host threads
    // take interleaved columns
    auto cols = [&](int j0, int step) {
        std::vector<double> e(n, 0.0), x;
        for (int j = j0; j < n; j += step) {
            e[j] = 1.0;
            cycle_from(h, lc, pre, post, e, x);
            e[j] = 0.0;
            for (int i = 0; i < n; ++i) C[(size_t)i * n + j] = x[i];
        }
    };
    const unsigned hw = std::thread::hardware_concurrency();
    const int nt = n < 256 ? 1 : (int)std::min<unsigned>(hw > 0 ? hw : 1, 8);
    std::vector<std::thread> ts;
    for (int t = 1; t < nt; ++t) ts.emplace_back(cols, t, nt);
    cols(0, nt);
    for (std::thread &t : ts) t.join();
    return C;
}

}  // namespace ibpm
