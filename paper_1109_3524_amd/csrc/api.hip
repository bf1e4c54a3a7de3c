// C ABI of the library: context set-up, the time-step driver and the
// Krylov / AMG drivers that queue the kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ibpm.h"
#include "kernels.h"
#include "setup.h"

using namespace ibpm;

namespace {

struct HipError : std::runtime_error {
    using std::runtime_error::runtime_error;
};
struct InvalidArg : std::runtime_error {
    using std::runtime_error::runtime_error;
};

#define HIPCHECK(call)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            throw HipError(std::string(#call) + ": " + hipGetErrorString(e_));              \
    } while (0)

struct DevCSR {
    int nrows = 0, ncols = 0;
    int32_t *ptr = nullptr, *col = nullptr;
    double *val = nullptr;
    CSRView view() const { return CSRView{nrows, ncols, ptr, col, val}; }
};

struct DevLevel {
    int n = 0;
    DevCSR A, P, R;         // A unused on level 0 (matrix-free K0)
    double *wdinv = nullptr;
    double omega = 0;
    double *b = nullptr, *xa = nullptr, *xb = nullptr, *r = nullptr;
};

}  // namespace

struct ibpm_ctx {
    std::string err;
    hipStream_t stream = nullptr;
    ibpm_params prm{};
    Model m;
    Hierarchy h;
    bool amg = false;
    std::vector<void *> allocs;
    GridView g{};
    K0View K0{};
    AView A{};
    double ly = 0;
    double *walls[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t step = 0;
    DevCSR E, Etu, Etv;
    double *ub = nullptr;
    std::vector<DevLevel> lev;
    double *coarse_inv = nullptr;
    // work vectors
    double *vr = nullptr, *vp[2] = {nullptr, nullptr}, *vq = nullptr;      // velocity PCG (n_q)
    double *pr = nullptr, *pp[2] = {nullptr, nullptr}, *pq = nullptr, *pz = nullptr;  // Poisson PCG
    double *r1 = nullptr, *rhs2 = nullptr;
    SolveStatus *st_vel = nullptr, *st_poi = nullptr, *st_misc = nullptr, *st_bench = nullptr;
    double *parts = nullptr;
    SolveStatus *host_st = nullptr;   // pinned
    int est_vel = 8, est_poi = 32;

    template <class T>
    T *dalloc(size_t n) {
        void *p = nullptr;
        if (n == 0) n = 1;
        hipError_t e = hipMalloc(&p, n * sizeof(T));
        if (e != hipSuccess) throw std::bad_alloc();
        allocs.push_back(p);
        return (T *)p;
    }
    template <class T>
    T *upload(const std::vector<T> &v) {
        T *p = dalloc<T>(v.size());
        if (!v.empty()) {
            // the source may be a temporary: wait for the copy before returning
            HIPCHECK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, stream));
            HIPCHECK(hipStreamSynchronize(stream));
        }
        return p;
    }
    DevCSR upload(const CSR &c) {
        DevCSR d;
        d.nrows = c.nrows;
        d.ncols = c.ncols;
        d.ptr = upload(c.ptr.empty() ? std::vector<int32_t>{0} : c.ptr);
        d.col = upload(c.col);
        d.val = upload(c.val);
        return d;
    }
    void read_status(SolveStatus *st) {
        HIPCHECK(hipMemcpyAsync(host_st, st, sizeof(SolveStatus), hipMemcpyDeviceToHost, stream));
        HIPCHECK(hipStreamSynchronize(stream));
    }
    ~ibpm_ctx() {
        if (stream) (void)hipStreamSynchronize(stream);
        for (void *p : allocs) (void)hipFree(p);
        if (host_st) (void)hipHostFree(host_st);
    }
};

namespace {

int fail(ibpm_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

template <class F>
int guarded(ibpm_ctx *c, F &&f) {
    if (!c) return IBPM_EINVAL;
    try {
        c->err.clear();
        return f();
    } catch (const InvalidArg &e) {
        return fail(c, IBPM_EINVAL, e.what());
    } catch (const HipError &e) {
        return fail(c, IBPM_EHIP, e.what());
    } catch (const std::bad_alloc &) {
        return fail(c, IBPM_ENOMEM, "out of memory");
    } catch (const std::exception &e) {
        return fail(c, IBPM_EINVAL, e.what());
    }
}

// ---------------------------------------------------------------------------
// V-cycle: z = M r (symmetric, zero initial guess per level), last
// post-smoothing sweep forms r . z.  Every kernel is predicated on st->done.

void enqueue_vcycle(ibpm_ctx *c, const double *r, double *z, SolveStatus *st) {
    hipStream_t s = c->stream;
    const int pre = c->prm.amg_pre, post = c->prm.amg_post;
    const int L = (int)c->lev.size();
    if (L == 1) {
        launch_dense_solve(s, c->K0.n, c->coarse_inv, r, z, st);
        launch_dot_rz(s, c->K0.n, r, z, st, c->parts);
        return;
    }
    std::vector<double *> cur(L);
    // level 0 down
    {
        DevLevel &l0 = c->lev[0];
        double *a = l0.xa, *b = l0.xb;
        launch_k0_jacobi_first(s, c->K0, l0.omega, r, a, st);
        for (int k = 1; k < pre; ++k) {
            launch_k0_jacobi(s, c->K0, l0.omega, r, a, b, st);
            std::swap(a, b);
        }
        cur[0] = a;
        launch_k0_residual(s, c->K0, r, a, l0.r, st);
        launch_csr_spmv(s, l0.R.view(), l0.r, c->lev[1].b, st);
    }
    for (int l = 1; l < L - 1; ++l) {
        DevLevel &lv = c->lev[l];
        double *a = lv.xa, *b = lv.xb;
        launch_csr_jacobi_first(s, lv.A.view(), lv.wdinv, lv.b, a, st);
        for (int k = 1; k < pre; ++k) {
            launch_csr_jacobi(s, lv.A.view(), lv.wdinv, lv.b, a, b, st);
            std::swap(a, b);
        }
        cur[l] = a;
        launch_csr_residual(s, lv.A.view(), lv.b, a, lv.r, st);
        launch_csr_spmv(s, lv.R.view(), lv.r, c->lev[l + 1].b, st);
    }
    DevLevel &lc = c->lev[L - 1];
    launch_dense_solve(s, lc.n, c->coarse_inv, lc.b, lc.xa, st);
    cur[L - 1] = lc.xa;
    for (int l = L - 2; l >= 1; --l) {
        DevLevel &lv = c->lev[l];
        double *a = cur[l];
        double *b = (a == lv.xa) ? lv.xb : lv.xa;
        launch_csr_spmv_add(s, lv.P.view(), cur[l + 1], a, st);
        for (int k = 0; k < post; ++k) {
            launch_csr_jacobi(s, lv.A.view(), lv.wdinv, lv.b, a, b, st);
            std::swap(a, b);
        }
        cur[l] = a;
    }
    {
        DevLevel &l0 = c->lev[0];
        double *a = cur[0];
        double *b = (a == l0.xa) ? l0.xb : l0.xa;
        launch_csr_spmv_add(s, l0.P.view(), cur[1], a, st);
        for (int k = 0; k < post - 1; ++k) {
            launch_k0_jacobi(s, c->K0, l0.omega, r, a, b, st);
            std::swap(a, b);
        }
        launch_k0_jacobi_rz(s, c->K0, l0.omega, r, a, z, st, c->parts);
    }
}

// Generic PCG driver.  Iterations are queued in chunks; every kernel of an
// iteration is predicated on the device status, so iterations queued past
// convergence do nothing.  The chunk length is estimated from the observed
// residual decay so few empty iterations are queued.
template <class Op>
int pcg_drive(ibpm_ctx *c, const Op &op, int n, bool jacobi, const double *b, double *x, double *r,
              double *z, double **p, double *q, SolveStatus *st, double rtol, int maxit, int &est,
              ibpm_solve_stats *out) {
    hipStream_t s = c->stream;
    auto t0 = std::chrono::steady_clock::now();
    launch_pcg_init(s, op, b, x, r, st, c->parts, jacobi, rtol * rtol, maxit);
    if (!jacobi) enqueue_vcycle(c, r, z, st);
    int curp = 0;
    int chunk = std::max(1, (int)(0.8 * est));
    int queued = 0;
    double last_rr = -1;
    int last_it = 0;
    for (;;) {
        for (int k = 0; k < chunk; ++k) {
            launch_pcg_spmv(s, op, jacobi ? r : z, p[curp], p[1 - curp], q, st, c->parts, jacobi);
            curp = 1 - curp;
            launch_pcg_update(s, op, x, r, p[curp], q, st, c->parts, jacobi);
            if (!jacobi) enqueue_vcycle(c, r, z, st);
        }
        queued += chunk;
        c->read_status(st);
        const SolveStatus &h = *c->host_st;
        if (h.done != ST_RUNNING || queued > maxit + 1) break;
        // estimate the remaining iterations from the decay so far
        int rem = 8;
        if (last_rr > 0 && h.iter > last_it && h.rr < last_rr) {
            double rate = std::log(h.rr / last_rr) / (h.iter - last_it);
            double need = std::log(h.tol2 * h.bb / h.rr);
            if (rate < 0) rem = (int)std::ceil(need / rate);
        } else if (h.iter > 0 && h.rr > 0 && h.bb > 0) {
            double rate = std::log(h.rr / h.bb) / h.iter;
            double need = std::log(h.tol2 * h.bb / h.rr);
            if (rate < 0) rem = (int)std::ceil(need / rate);
        }
        last_rr = h.rr;
        last_it = h.iter;
        chunk = std::min(std::max(rem, 1), 64);
    }
    launch_zero_if_zero_rhs(s, x, n, st);
    launch_true_residual(s, op, b, x, st, c->parts);
    c->read_status(st);
    const SolveStatus &h = *c->host_st;
    auto t1 = std::chrono::steady_clock::now();
    if (h.iter > 0) est = h.iter;
    int code = IBPM_OK;
    if (h.done == ST_NAN || !(h.true_rr == h.true_rr)) code = IBPM_ENAN;
    else if (h.done == ST_MAXIT || h.done == ST_RUNNING) code = IBPM_ENOTCONV;
    if (out) {
        out->iters = h.iter;
        out->status = code;
        out->relres = h.bb > 0 ? std::sqrt(h.true_rr / h.bb) : 0.0;
        out->ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    if (code == IBPM_ENAN) c->err = "residual became NaN";
    else if (code == IBPM_ENOTCONV) c->err = "iteration limit reached";
    return code;
}

int solve_poisson_impl(ibpm_ctx *c, const double *rhs, double *lam, ibpm_solve_stats *out) {
    bool jacobi = !c->amg;
    return pcg_drive(c, c->K0, c->K0.n, jacobi, rhs, lam, c->pr, c->pz, c->pp, c->pq, c->st_poi,
                     c->prm.poisson_rtol, c->prm.poisson_maxit, c->est_poi, out);
}

int solve_velocity_impl(ibpm_ctx *c, const double *rhs, double *q, ibpm_solve_stats *out) {
    return pcg_drive(c, c->A, c->g.n_q, true, rhs, q, c->vr, nullptr, c->vp, c->vq, c->st_vel,
                     c->prm.vel_rtol, c->prm.vel_maxit, c->est_vel, out);
}

void stage_walls(ibpm_ctx *c, const double *q) {
    double uconv = c->prm.uinf * std::cos(c->prm.alpha);
    launch_walls_update(c->stream, c->g, c->walls[c->cur], c->walls[1 - c->cur], q, uconv,
                        c->prm.dt, c->ly);
}

void stage_rhs1(ibpm_ctx *c, const double *q, const double *conv_prev, double *r1,
                double *conv_now) {
    launch_momentum_rhs(c->stream, c->g, q, conv_prev, conv_now, r1, c->walls[c->cur],
                        c->walls[1 - c->cur], c->prm.nu, c->prm.dt, c->step == 0 ? 1 : 0);
}

void stage_rhs2(ibpm_ctx *c, const double *qstar, double *rhs) {
    launch_poisson_rhs(c->stream, c->g, c->m.nb, qstar, c->walls[1 - c->cur], c->E.view(), c->ub,
                       rhs);
}

void stage_project(ibpm_ctx *c, const double *qstar, const double *lam, double *qout) {
    const Model &m = c->m;
    launch_project(c->stream, c->g, c->prm.dt, m.nb, qstar, lam, qout, c->Etu.view(), m.fu_i0,
                   m.fu_i1, m.fu_j0, m.fu_j1, c->Etv.view(), m.fv_i0, m.fv_i1, m.fv_j0, m.fv_j1);
    launch_forces(c->stream, (int)m.g.n_cell, m.nb, lam, c->st_misc);
}

void check_params(const ibpm_params *p) {
    if (!p) throw InvalidArg("params is NULL");
    if (p->bn_order != 1) throw InvalidArg("only B^N with N = 1 is supported");
    if (!(p->vel_rtol > 0) || !(p->poisson_rtol > 0)) throw InvalidArg("tolerances must be > 0");
    if (p->vel_maxit < 1 || p->poisson_maxit < 1) throw InvalidArg("maxit must be >= 1");
    if (p->poisson_solver != IBPM_SOLVER_JACOBI_PCG && p->poisson_solver != IBPM_SOLVER_AMG_PCG)
        throw InvalidArg("Poisson solver not available in this build");
    if (p->poisson_solver == IBPM_SOLVER_AMG_PCG) {
        if (p->amg_pre < 1 || p->amg_post < 1) throw InvalidArg("AMG needs >= 1 pre and post sweep");
        if (p->amg_coarse_max < 1 || p->amg_max_levels < 1) throw InvalidArg("bad AMG limits");
        if (!(p->amg_theta >= 0)) throw InvalidArg("amg_theta must be >= 0");
    }
}

void build(ibpm_ctx *c, const ibpm_params *p) {
    check_params(p);
    c->prm = *p;
    c->prm.xf = c->prm.yf = c->prm.xb = c->prm.yb = c->prm.ubx = c->prm.uby = nullptr;
    Model &m = c->m;
    try {
        build_model(m, p->nx, p->ny, p->xf, p->yf, p->nb, p->xb, p->yb, p->ubx, p->uby, p->nu, p->dt);
    } catch (const std::runtime_error &e) {
        throw InvalidArg(e.what());
    }
    c->amg = p->poisson_solver != IBPM_SOLVER_JACOBI_PCG;
    if (c->amg) {
        AmgParams ap;
        ap.theta = p->amg_theta;
        ap.coarse_max = p->amg_coarse_max;
        ap.max_levels = p->amg_max_levels;
        try {
            build_hierarchy(c->h, m.K, ap);
        } catch (const std::runtime_error &e) {
            throw InvalidArg(e.what());
        }
    }
    const GridMetrics &G = m.g;
    int nx = G.nx, ny = G.ny;
    // metrics and reciprocals in one upload
    std::vector<double> met;
    auto put = [&](const std::vector<double> &v, bool recip) {
        for (double d : v) met.push_back(recip ? 1.0 / d : d);
    };
    put(G.dx, false); put(G.dy, false); put(G.Dx, false); put(G.Dy, false);
    put(G.dx, true); put(G.dy, true); put(G.Dx, true); put(G.Dy, true);
    double *dm = c->upload(met);
    size_t o = 0;
    GridView &g = c->g;
    g.nx = nx; g.ny = ny;
    g.n_u = (int)G.n_u; g.n_v = (int)G.n_v; g.n_q = (int)G.n_q; g.n_cell = (int)G.n_cell;
    g.dx = dm + o; o += nx;
    g.dy = dm + o; o += ny;
    g.Dx = dm + o; o += nx + 1;
    g.Dy = dm + o; o += ny + 1;
    g.idx = dm + o; o += nx;
    g.idy = dm + o; o += ny;
    g.iDx = dm + o; o += nx + 1;
    g.iDy = dm + o; o += ny + 1;
    c->ly = 0;
    for (double d : G.dy) c->ly += d;
    WallOffsets wo = WallOffsets::make(nx, ny);
    c->walls[0] = c->dalloc<double>(wo.total);
    c->walls[1] = c->dalloc<double>(wo.total);
    c->E = c->upload(m.E);
    c->Etu = c->upload(m.Etu);
    c->Etv = c->upload(m.Etv);
    c->ub = c->upload(m.ub);
    DevCSR cf = c->upload(m.Kcf), kf = c->upload(m.Kf);
    double *kfd = c->upload(m.Kf_diag);
    K0View &K = c->K0;
    K.g = g;
    K.dt = p->dt;
    K.nb = m.nb;
    K.n = (int)G.n_cell + 2 * m.nb;
    K.cb_i0 = m.cb_i0; K.cb_i1 = m.cb_i1; K.cb_j0 = m.cb_j0; K.cb_j1 = m.cb_j1;
    K.cf = cf.view();
    K.kf = kf.view();
    K.kf_diag = kfd;
    c->A.g = g;
    c->A.dt = p->dt;
    c->A.idt = 1.0 / p->dt;
    c->A.nu = p->nu;
    // hierarchy
    if (c->amg) {
        int L = (int)c->h.levels.size();
        c->lev.resize(L);
        for (int l = 0; l < L; ++l) {
            const Level &hl = c->h.levels[l];
            DevLevel &dl = c->lev[l];
            dl.n = hl.A.nrows;
            dl.omega = hl.omega;
            if (l > 0) {
                dl.A = c->upload(hl.A);
                dl.wdinv = c->upload(hl.wdinv);
                dl.b = c->dalloc<double>(dl.n);
            }
            if (l < L - 1) {
                dl.P = c->upload(hl.P);
                dl.R = c->upload(hl.R);
                dl.r = c->dalloc<double>(dl.n);
            }
            dl.xa = c->dalloc<double>(dl.n);
            dl.xb = c->dalloc<double>(dl.n);
        }
        c->coarse_inv = c->upload(c->h.coarse_inv);
        // keep only what the host API still needs (sizes, aggregates)
        for (auto &hl : c->h.levels) {
            hl.P = CSR();
            hl.R = CSR();
            hl.wdinv.clear();
        }
    }
    int nq = g.n_q, nl = K.n;
    c->vr = c->dalloc<double>(nq);
    c->vp[0] = c->dalloc<double>(nq);
    c->vp[1] = c->dalloc<double>(nq);
    c->vq = c->dalloc<double>(nq);
    c->pr = c->dalloc<double>(nl);
    c->pp[0] = c->dalloc<double>(nl);
    c->pp[1] = c->dalloc<double>(nl);
    c->pq = c->dalloc<double>(nl);
    c->pz = c->dalloc<double>(nl);
    c->r1 = c->dalloc<double>(nq);
    c->rhs2 = c->dalloc<double>(nl);
    for (double *v : {c->vp[0], c->vp[1]}) HIPCHECK(hipMemsetAsync(v, 0, nq * sizeof(double), c->stream));
    for (double *v : {c->pp[0], c->pp[1]}) HIPCHECK(hipMemsetAsync(v, 0, nl * sizeof(double), c->stream));
    SolveStatus *sts = c->dalloc<SolveStatus>(4);
    HIPCHECK(hipMemsetAsync(sts, 0, 4 * sizeof(SolveStatus), c->stream));
    c->st_vel = sts;
    c->st_poi = sts + 1;
    c->st_misc = sts + 2;
    c->st_bench = sts + 3;
    c->parts = c->dalloc<double>(4 * kMaxParts);
    HIPCHECK(hipHostMalloc((void **)&c->host_st, sizeof(SolveStatus), hipHostMallocDefault));
    double U = p->uinf * std::cos(p->alpha), V = p->uinf * std::sin(p->alpha);
    launch_fill_walls(c->stream, g, c->walls[0], U, V);
    launch_fill_walls(c->stream, g, c->walls[1], U, V);
    HIPCHECK(hipStreamSynchronize(c->stream));
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

int ibpm_build_operators(const ibpm_params *p, void *stream, ibpm_ctx **out) {
    if (!out) return IBPM_EINVAL;
    *out = nullptr;
    ibpm_ctx *c = new (std::nothrow) ibpm_ctx();
    if (!c) return IBPM_ENOMEM;
    c->stream = (hipStream_t)stream;
    int rc = guarded(c, [&] {
        build(c, p);
        return IBPM_OK;
    });
    *out = c;   // returned even on failure so that ibpm_last_error can report
    return rc;
}

int ibpm_destroy(ibpm_ctx *ctx) {
    delete ctx;
    return IBPM_OK;
}

const char *ibpm_last_error(const ibpm_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

int ibpm_sizes(const ibpm_ctx *c, int64_t *nq, int64_t *nl) {
    if (!c || c->g.nx == 0) return IBPM_EINVAL;
    if (nq) *nq = c->g.n_q;
    if (nl) *nl = c->K0.n;
    return IBPM_OK;
}

int ibpm_init_state(ibpm_ctx *c, double *q, double *conv, double *lam) {
    return guarded(c, [&] {
        if (!q || !conv || !lam) throw InvalidArg("NULL vector");
        double U = c->prm.uinf * std::cos(c->prm.alpha), V = c->prm.uinf * std::sin(c->prm.alpha);
        launch_init_state(c->stream, c->g, q, conv, lam, c->K0.n, U, V);
        launch_fill_walls(c->stream, c->g, c->walls[0], U, V);
        launch_fill_walls(c->stream, c->g, c->walls[1], U, V);
        c->cur = 0;
        c->step = 0;
        return IBPM_OK;
    });
}

int ibpm_step(ibpm_ctx *c, int32_t nsteps, double *q, double *conv, double *lam,
              ibpm_step_stats *stats) {
    return guarded(c, [&] {
        if (!q || !conv || !lam) throw InvalidArg("NULL vector");
        if (nsteps < 0) throw InvalidArg("nsteps < 0");
        auto t0 = std::chrono::steady_clock::now();
        ibpm_step_stats acc{};
        int worst = IBPM_OK;
        for (int s = 0; s < nsteps; ++s) {
            stage_walls(c, q);
            stage_rhs1(c, q, conv, c->r1, conv);
            ibpm_solve_stats vs{}, ps{};
            int rc1 = solve_velocity_impl(c, c->r1, q, &vs);
            stage_rhs2(c, q, c->rhs2);
            int rc2 = solve_poisson_impl(c, c->rhs2, lam, &ps);
            stage_project(c, q, lam, q);
            c->cur = 1 - c->cur;
            c->step += 1;
            acc.steps += 1;
            acc.vel_iters += vs.iters;
            acc.poisson_iters += ps.iters;
            acc.last_vel_iters = vs.iters;
            acc.last_poisson_iters = ps.iters;
            acc.vel_relres_max = std::max(acc.vel_relres_max, vs.relres);
            acc.poisson_relres_max = std::max(acc.poisson_relres_max, ps.relres);
            acc.vel_ms += vs.ms;
            acc.poisson_ms += ps.ms;
            for (int rc : {rc1, rc2})
                if (rc != IBPM_OK && (worst == IBPM_OK || rc == IBPM_ENAN)) worst = rc;
        }
        if (stats) {
            c->read_status(c->st_misc);
            acc.fx = c->host_st->fx;
            acc.fy = c->host_st->fy;
            auto t1 = std::chrono::steady_clock::now();
            acc.ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
            *stats = acc;
        }
        if (worst != IBPM_OK && c->err.empty()) c->err = "a solve did not converge";
        return worst;
    });
}

int ibpm_solve_poisson(ibpm_ctx *c, const double *rhs, double *lam, ibpm_solve_stats *stats) {
    return guarded(c, [&] {
        if (!rhs || !lam) throw InvalidArg("NULL vector");
        return solve_poisson_impl(c, rhs, lam, stats);
    });
}

int ibpm_solve_velocity(ibpm_ctx *c, const double *rhs, double *q, ibpm_solve_stats *stats) {
    return guarded(c, [&] {
        if (!rhs || !q) throw InvalidArg("NULL vector");
        return solve_velocity_impl(c, rhs, q, stats);
    });
}

int ibpm_apply_K(ibpm_ctx *c, const double *x, double *y) {
    return guarded(c, [&] {
        if (!x || !y || x == y) throw InvalidArg("x and y must be distinct device vectors");
        launch_apply_K0(c->stream, c->K0, x, y);
        return IBPM_OK;
    });
}

int ibpm_apply_A(ibpm_ctx *c, const double *x, double *y) {
    return guarded(c, [&] {
        if (!x || !y || x == y) throw InvalidArg("x and y must be distinct device vectors");
        launch_apply_A(c->stream, c->A, x, y);
        return IBPM_OK;
    });
}

int ibpm_stage_walls(ibpm_ctx *c, const double *q) {
    return guarded(c, [&] {
        if (!q) throw InvalidArg("NULL vector");
        stage_walls(c, q);
        return IBPM_OK;
    });
}

int ibpm_stage_rhs1(ibpm_ctx *c, const double *q, const double *conv_prev, double *r1,
                    double *conv_now) {
    return guarded(c, [&] {
        if (!q || !conv_prev || !r1 || !conv_now) throw InvalidArg("NULL vector");
        stage_rhs1(c, q, conv_prev, r1, conv_now);
        return IBPM_OK;
    });
}

int ibpm_stage_rhs2(ibpm_ctx *c, const double *qstar, double *rhs) {
    return guarded(c, [&] {
        if (!qstar || !rhs) throw InvalidArg("NULL vector");
        stage_rhs2(c, qstar, rhs);
        return IBPM_OK;
    });
}

int ibpm_stage_project(ibpm_ctx *c, const double *qstar, const double *lam, double *qout) {
    return guarded(c, [&] {
        if (!qstar || !lam || !qout) throw InvalidArg("NULL vector");
        stage_project(c, qstar, lam, qout);
        return IBPM_OK;
    });
}

int ibpm_get_walls(ibpm_ctx *c, int32_t which, double *host) {
    return guarded(c, [&] {
        if (!host || (which != 0 && which != 1)) throw InvalidArg("bad arguments");
        WallOffsets wo = WallOffsets::make(c->g.nx, c->g.ny);
        const double *src = c->walls[which == 0 ? c->cur : 1 - c->cur];
        HIPCHECK(hipMemcpyAsync(host, src, wo.total * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(hipStreamSynchronize(c->stream));
        return IBPM_OK;
    });
}

int ibpm_set_walls(ibpm_ctx *c, int32_t which, const double *host) {
    return guarded(c, [&] {
        if (!host || (which != 0 && which != 1)) throw InvalidArg("bad arguments");
        WallOffsets wo = WallOffsets::make(c->g.nx, c->g.ny);
        double *dst = c->walls[which == 0 ? c->cur : 1 - c->cur];
        HIPCHECK(hipMemcpyAsync(dst, host, wo.total * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIPCHECK(hipStreamSynchronize(c->stream));
        return IBPM_OK;
    });
}

int ibpm_get_step(const ibpm_ctx *c, int64_t *step) {
    if (!c || !step) return IBPM_EINVAL;
    *step = c->step;
    return IBPM_OK;
}

int ibpm_set_step(ibpm_ctx *c, int64_t step) {
    if (!c || step < 0) return IBPM_EINVAL;
    c->step = step;
    return IBPM_OK;
}

int ibpm_get_forces(ibpm_ctx *c, double *fx, double *fy) {
    return guarded(c, [&] {
        c->read_status(c->st_misc);
        if (fx) *fx = c->host_st->fx;
        if (fy) *fy = c->host_st->fy;
        return IBPM_OK;
    });
}

int ibpm_hierarchy_info(const ibpm_ctx *c, int32_t *levels, int64_t *sizes, int64_t *nnz) {
    if (!c || !levels) return IBPM_EINVAL;
    if (!c->amg) {
        *levels = 0;
        return IBPM_OK;
    }
    *levels = (int32_t)c->h.levels.size();
    for (size_t l = 0; l < c->h.levels.size(); ++l) {
        if (sizes) sizes[l] = c->h.levels[l].A.nrows;
        if (nnz) nnz[l] = c->h.levels[l].A.nnz();
    }
    return IBPM_OK;
}

int ibpm_get_aggregates(const ibpm_ctx *c, int32_t level, int32_t *agg) {
    if (!c || !agg || !c->amg) return IBPM_EINVAL;
    if (level < 0 || level + 1 >= (int)c->h.levels.size()) return IBPM_EINVAL;
    const std::vector<int32_t> &a = c->h.levels[level].agg;
    std::copy(a.begin(), a.end(), agg);
    return IBPM_OK;
}

int ibpm_time_kernel(ibpm_ctx *c, int32_t kernel, int32_t reps, double *avg_ms, double *bytes) {
    return guarded(c, [&] {
        if (reps < 1 || !avg_ms) throw InvalidArg("bad arguments");
        const bool needs_amg = kernel == IBPM_KERNEL_K0_JACOBI || kernel == IBPM_KERNEL_K0_RESIDUAL ||
                               kernel == IBPM_KERNEL_RESTRICT0 || kernel == IBPM_KERNEL_PROLONG0;
        if (needs_amg && (!c->amg || c->lev.size() < 2)) throw InvalidArg("kernel needs an AMG hierarchy");
        hipStream_t s = c->stream;
        const K0View &K = c->K0;
        const int n = K.n, nq = c->g.n_q;
        const Model &m = c->m;
        // compulsory bytes of the coupling part of K and of the grid metrics
        const double b_metric = 2.0 * 8.0 * (2.0 * m.g.nx + 2.0 * m.g.ny + 2.0);
        const double b_coupling = 12.0 * (double)(m.Kcf.nnz() + m.Kf.nnz()) +
                                  4.0 * (double)(m.Kcf.nrows + m.Kf.nrows + 2) + 8.0 * 2 * m.nb;
        double by = 0;
        SolveStatus zero{};
        HIPCHECK(hipMemcpyAsync(c->st_bench, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
        HIPCHECK(hipStreamSynchronize(s));
        // operands: fill with something finite
        HIPCHECK(hipMemsetAsync(c->pr, 0, n * sizeof(double), s));
        HIPCHECK(hipMemsetAsync(c->pz, 0, n * sizeof(double), s));
        HIPCHECK(hipMemsetAsync(c->vr, 0, nq * sizeof(double), s));
        std::function<void()> launch;
        switch (kernel) {
        case IBPM_KERNEL_K0_JACOBI: {
            DevLevel &l0 = c->lev[0];
            launch = [&] { launch_k0_jacobi(s, K, l0.omega, c->pr, l0.xa, l0.xb, c->st_bench); };
            by = 24.0 * n + b_coupling + b_metric;
            break;
        }
        case IBPM_KERNEL_K0_PCG_SPMV:
            launch = [&] { launch_pcg_spmv(s, K, c->pz, c->pp[0], c->pp[1], c->pq, c->st_bench, c->parts, false); };
            by = 32.0 * n + b_coupling + b_metric;
            break;
        case IBPM_KERNEL_A_PCG_SPMV:
            launch = [&] { launch_pcg_spmv(s, c->A, c->vr, c->vp[0], c->vp[1], c->vq, c->st_bench, c->parts, true); };
            by = 32.0 * nq + b_metric;
            break;
        case IBPM_KERNEL_K0_RESIDUAL: {
            DevLevel &l0 = c->lev[0];
            launch = [&] { launch_k0_residual(s, K, c->pr, l0.xa, l0.r, c->st_bench); };
            by = 24.0 * n + b_coupling + b_metric;
            break;
        }
        case IBPM_KERNEL_RESTRICT0: {
            DevLevel &l0 = c->lev[0];
            const DevCSR &R = l0.R;
            launch = [&] { launch_csr_spmv(s, R.view(), l0.r, c->lev[1].b, c->st_bench); };
            by = 4.0 * (R.nrows + 1) + 8.0 * R.ncols + 8.0 * R.nrows;
            break;
        }
        case IBPM_KERNEL_PROLONG0: {
            DevLevel &l0 = c->lev[0];
            const DevCSR &P = l0.P;
            launch = [&] { launch_csr_spmv_add(s, P.view(), c->lev[1].xa, l0.xa, c->st_bench); };
            by = 4.0 * (P.nrows + 1) + 8.0 * P.ncols + 16.0 * P.nrows;
            break;
        }
        case IBPM_KERNEL_PCG_UPDATE_K:
            launch = [&] { launch_pcg_update(s, K, c->pp[1], c->pr, c->pp[0], c->pq, c->st_bench, c->parts, false); };
            by = 48.0 * n;
            break;
        default:
            throw InvalidArg("unknown kernel id");
        }
        if (kernel == IBPM_KERNEL_RESTRICT0 || kernel == IBPM_KERNEL_PROLONG0) {
            // stored matrix bytes: 4 (column) + 8 (value) per non-zero
            const DevCSR &M = kernel == IBPM_KERNEL_RESTRICT0 ? c->lev[0].R : c->lev[0].P;
            int nnz = 0;
            HIPCHECK(hipMemcpy(&nnz, M.ptr + M.nrows, sizeof(int), hipMemcpyDeviceToHost));
            by += 12.0 * nnz;
        }
        launch();   // warm the caches and the code object
        hipEvent_t e0, e1;
        HIPCHECK(hipEventCreate(&e0));
        HIPCHECK(hipEventCreate(&e1));
        HIPCHECK(hipEventRecord(e0, s));
        for (int k = 0; k < reps; ++k) launch();
        HIPCHECK(hipEventRecord(e1, s));
        HIPCHECK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *avg_ms = ms / reps;
        if (bytes) *bytes = by;
        return IBPM_OK;
    });
}

}  // extern "C"
