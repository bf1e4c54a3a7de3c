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

// Device CSR in precision T; `lanes` threads per row for the CSR kernels
template <class T>
struct DevCSRT {
    int nrows = 0, ncols = 0, lanes = 1;
    int64_t nnz = 0;
    int32_t *ptr = nullptr, *col = nullptr;
    T *val = nullptr;
    CSRT<T> view() const { return CSRT<T>{nrows, ncols, ptr, col, val}; }
};
using DevCSR = DevCSRT<double>;

// lanes per row: the power of two nearest above 2/3 of the mean row length
int lanes_for(int64_t nnz, int nrows) {
    double m = nrows > 0 ? (double)nnz / nrows : 1.0;
    int L = 1;
    while (L < 64 && L * 1.5 < m) L *= 2;
    return L;
}

// One AMG level in precision T (level 0 uses the matrix-free K0 for A)
template <class T>
struct DevLevelT {
    int n = 0;
    double omega = 0;
    DevCSRT<T> A, P, R;
    T *wdinv = nullptr;
    T *b = nullptr, *xa = nullptr, *xb = nullptr, *r = nullptr;
};

// Everything one precision needs for the Poisson solve
template <class T>
struct PrecSet {
    K0T<T> K0{};
    std::vector<DevLevelT<T>> lev;
    CoarseLevel<T> *coarse_dev = nullptr;
    int lc = 1;                        // first level solved by the one-work-group coarse cycle
    // PCG work vectors (n_lambda)
    T *r = nullptr, *z = nullptr, *p[2] = {nullptr, nullptr}, *q = nullptr;
};

}  // namespace

struct ibpm_ctx {
    std::string err;
    hipStream_t stream = nullptr;
    ibpm_params prm{};
    Model m;
    Hierarchy h;
    bool amg = false, mixed = false;
    std::vector<void *> allocs;
    GridView g{};
    AView A{};
    double ly = 0;
    double *walls[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t step = 0;
    DevCSR E, Etu, Etv;
    double *ub = nullptr;
    PrecSet<double> p64;
    PrecSet<float> p32;
    float *rin32 = nullptr, *d32 = nullptr;          // mixed: inner right-hand side and correction
    double *coarse_inv = nullptr;
    // velocity PCG (n_q)
    double *vr = nullptr, *vz = nullptr, *vp[2] = {nullptr, nullptr}, *vq = nullptr;
    double *r1 = nullptr, *rhs2 = nullptr;
    SolveStatus *st_vel = nullptr, *st_poi = nullptr, *st_misc = nullptr, *st_bench = nullptr,
                *st_out = nullptr;
    double *parts = nullptr;
    SolveStatus *host_st = nullptr;   // pinned
    int est_vel = 8, est_poi = 32, est_inner = 32;

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
    template <class T>
    DevCSRT<T> upload_csr(const CSR &c) {
        DevCSRT<T> d;
        d.nrows = c.nrows;
        d.ncols = c.ncols;
        d.nnz = c.nnz();
        d.lanes = lanes_for(d.nnz, d.nrows);
        d.ptr = upload(c.ptr.empty() ? std::vector<int32_t>{0} : c.ptr);
        d.col = upload(c.col);
        d.val = upload(std::vector<T>(c.val.begin(), c.val.end()));
        return d;
    }
    // FP32 copy of the values of an uploaded FP64 matrix (indices shared)
    DevCSRT<float> values32(const DevCSR &d, const CSR &c) {
        DevCSRT<float> f;
        f.nrows = d.nrows;
        f.ncols = d.ncols;
        f.nnz = d.nnz;
        f.lanes = d.lanes;
        f.ptr = d.ptr;
        f.col = d.col;
        f.val = upload(std::vector<float>(c.val.begin(), c.val.end()));
        return f;
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
// V-cycle: z = M r (symmetric, zero initial guess per level), the last
// post-smoothing sweep forms r . z.  Levels lc.. run in one work-group.
// Every kernel is predicated on st->done.

template <class T>
void enqueue_vcycle(ibpm_ctx *c, PrecSet<T> &P, const T *r, T *z, SolveStatus *st) {
    hipStream_t s = c->stream;
    const int pre = c->prm.amg_pre, post = c->prm.amg_post;
    const int L = (int)P.lev.size();
    const K0T<T> &K = P.K0;
    if (L == 1) {
        launch_dense_solve(s, K.n, c->coarse_inv, r, z, st);
        launch_dot_rz(s, K.n, r, z, st, c->parts);
        return;
    }
    std::vector<T *> cur(L);
    {
        DevLevelT<T> &l0 = P.lev[0];
        T *a = l0.xa, *b = l0.xb;
        launch_k0_jacobi_first(s, K, l0.omega, r, a, st);
        for (int k = 1; k < pre; ++k) {
            launch_k0_jacobi(s, K, l0.omega, r, a, b, st);
            std::swap(a, b);
        }
        cur[0] = a;
        launch_k0_residual(s, K, r, (const T *)a, l0.r, st);
        launch_csrv_spmv(s, l0.R.view(), l0.R.lanes, (const T *)l0.r, P.lev[1].b, false, st);
    }
    for (int l = 1; l < P.lc; ++l) {
        DevLevelT<T> &lv = P.lev[l];
        T *a = lv.xa, *b = lv.xb;
        launch_csr_jacobi_first(s, lv.A.view(), (const T *)lv.wdinv, (const T *)lv.b, a, st);
        for (int k = 1; k < pre; ++k) {
            launch_csrv_jacobi(s, lv.A.view(), lv.A.lanes, (const T *)lv.wdinv, (const T *)lv.b,
                               (const T *)a, b, st);
            std::swap(a, b);
        }
        cur[l] = a;
        launch_csrv_residual(s, lv.A.view(), lv.A.lanes, (const T *)lv.b, (const T *)a, lv.r, st);
        launch_csrv_spmv(s, lv.R.view(), lv.R.lanes, (const T *)lv.r, P.lev[l + 1].b, false, st);
    }
    launch_coarse_cycle(s, (const CoarseLevel<T> *)P.coarse_dev, P.lc, L, pre, post, c->coarse_inv,
                        P.lev[L - 1].n, st);
    cur[P.lc] = P.lev[P.lc].xa;
    for (int l = P.lc - 1; l >= 1; --l) {
        DevLevelT<T> &lv = P.lev[l];
        T *a = cur[l];
        T *b = (a == lv.xa) ? lv.xb : lv.xa;
        launch_csrv_spmv(s, lv.P.view(), lv.P.lanes, (const T *)cur[l + 1], a, true, st);
        for (int k = 0; k < post; ++k) {
            launch_csrv_jacobi(s, lv.A.view(), lv.A.lanes, (const T *)lv.wdinv, (const T *)lv.b,
                               (const T *)a, b, st);
            std::swap(a, b);
        }
        cur[l] = a;
    }
    {
        DevLevelT<T> &l0 = P.lev[0];
        T *a = cur[0];
        T *b = (a == l0.xa) ? l0.xb : l0.xa;
        launch_csrv_spmv(s, l0.P.view(), l0.P.lanes, (const T *)cur[1], a, true, st);
        for (int k = 0; k < post - 1; ++k) {
            launch_k0_jacobi(s, K, l0.omega, r, (const T *)a, b, st);
            std::swap(a, b);
        }
        launch_k0_jacobi_rz(s, K, l0.omega, r, (const T *)a, z, st, c->parts);
    }
}

// Generic PCG driver.  Iterations are queued in chunks; every kernel of an
// iteration is predicated on the device status, so iterations queued past
// convergence do nothing.  The chunk length is estimated from the observed
// residual decay so few empty iterations are queued.
//   precond(r, z): queue z = M r (with the r . z reduction); null for Jacobi
template <class Op, class T>
int pcg_drive(ibpm_ctx *c, const Op &op, int n, bool jacobi,
              const std::function<void(const T *, T *)> &precond, const T *b, T *x, T *r, T *z,
              T **p, T *q, SolveStatus *st, double rtol, int maxit, int &est, bool zero_guess,
              bool true_residual, ibpm_solve_stats *out) {
    hipStream_t s = c->stream;
    auto t0 = std::chrono::steady_clock::now();
    if (zero_guess) launch_pcg_init_zero(s, n, b, x, r, st, c->parts, rtol * rtol, maxit);
    else launch_pcg_init(s, op, b, (const T *)x, r, z, st, c->parts, jacobi, rtol * rtol, maxit);
    if (!jacobi) precond(r, z);
    int curp = 0;
    int chunk = std::max(1, (int)(0.8 * est));
    int queued = 0;
    double last_rr = -1;
    int last_it = 0;
    for (;;) {
        for (int k = 0; k < chunk; ++k) {
            launch_pcg_spmv(s, op, (const T *)z, (const T *)p[curp], p[1 - curp], q, st, c->parts);
            curp = 1 - curp;
            launch_pcg_update(s, op, x, r, z, (const T *)p[curp], (const T *)q, st, c->parts, jacobi);
            if (!jacobi) precond(r, z);
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
    if (true_residual) {
        launch_true_residual(s, op, b, (const T *)x, st, c->parts);
        c->read_status(st);
    }
    const SolveStatus &h = *c->host_st;
    auto t1 = std::chrono::steady_clock::now();
    if (h.iter > 0) est = h.iter;
    int code = IBPM_OK;
    if (h.done == ST_NAN || (true_residual && !(h.true_rr == h.true_rr))) code = IBPM_ENAN;
    else if (h.done == ST_MAXIT || h.done == ST_RUNNING) code = IBPM_ENOTCONV;
    if (out) {
        out->iters = h.iter;
        out->status = code;
        out->relres = h.bb > 0 ? std::sqrt((true_residual ? h.true_rr : h.rr) / h.bb) : 0.0;
        out->ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        out->outer_iters = 1;
        out->fallbacks = 0;
    }
    if (code == IBPM_ENAN) c->err = "residual became NaN";
    else if (code == IBPM_ENOTCONV) c->err = "iteration limit reached";
    return code;
}

int solve_poisson_fp64(ibpm_ctx *c, const double *rhs, double *lam, ibpm_solve_stats *out) {
    bool jacobi = !c->amg;
    PrecSet<double> &P = c->p64;
    std::function<void(const double *, double *)> pre = [c](const double *r, double *z) {
        enqueue_vcycle(c, c->p64, r, z, c->st_poi);
    };
    return pcg_drive<K0View, double>(c, P.K0, P.K0.n, jacobi, pre, rhs, lam, P.r, P.z, P.p, P.q,
                                     c->st_poi, c->prm.poisson_rtol, c->prm.poisson_maxit,
                                     c->est_poi, false, true, out);
}

// Mixed precision: FP64 iterative refinement around an FP32 AMG-PCG.  The
// outer residual, its norm, the correction update and the coarsest-level
// solve are FP64; the inner SpMV, V-cycle and vectors are FP32 with FP64
// dot products.  Each inner solve is asked for the reduction the outer
// tolerance still needs (at least 1e-5, about what FP32 can deliver).
int solve_poisson_mixed(ibpm_ctx *c, const double *rhs, double *lam, ibpm_solve_stats *out) {
    hipStream_t s = c->stream;
    auto t0 = std::chrono::steady_clock::now();
    const K0View &K = c->p64.K0;
    const int n = K.n;
    const double rtol = c->prm.poisson_rtol;
    launch_outer_residual(s, K, rhs, lam, c->rin32, c->st_out, c->parts, 1);
    c->read_status(c->st_out);
    double bb = c->host_st->bb, rr = c->host_st->rr;
    int inner_total = 0, outer = 0, code = IBPM_OK;
    PrecSet<float> &P = c->p32;
    std::function<void(const float *, float *)> pre = [c](const float *r, float *z) {
        enqueue_vcycle(c, c->p32, r, z, c->st_poi);
    };
    if (bb == 0.0) {
        HIPCHECK(hipMemsetAsync(lam, 0, n * sizeof(double), s));
        rr = 0.0;
    }
    while (bb > 0.0 && rr > rtol * rtol * bb) {
        if (!(rr == rr)) {
            code = IBPM_ENAN;
            break;
        }
        if (outer >= 30 || inner_total >= c->prm.poisson_maxit) {
            code = IBPM_ENOTCONV;
            break;
        }
        double need = rtol * std::sqrt(bb / rr);
        double tol_in = std::max(0.5 * need, 1e-5);
        ibpm_solve_stats is{};
        int rc = pcg_drive<K0T<float>, float>(c, P.K0, n, false, pre, c->rin32, c->d32, P.r, P.z,
                                              P.p, P.q, c->st_poi, tol_in,
                                              c->prm.poisson_maxit - inner_total, c->est_inner,
                                              true, false, &is);
        inner_total += is.iters;
        if (rc == IBPM_ENAN) {
            code = IBPM_ENAN;
            break;
        }
        launch_add_correction(s, n, lam, c->d32);
        launch_outer_residual(s, K, rhs, lam, c->rin32, c->st_out, c->parts, 0);
        c->read_status(c->st_out);
        rr = c->host_st->rr;
        ++outer;
    }
    auto t1 = std::chrono::steady_clock::now();
    if (out) {
        out->iters = inner_total;
        out->status = code;
        out->relres = bb > 0 ? std::sqrt(rr / bb) : 0.0;
        out->ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        out->outer_iters = outer;
        out->fallbacks = 0;
    }
    if (code == IBPM_ENAN) c->err = "residual became NaN";
    else if (code == IBPM_ENOTCONV) c->err = "iteration limit reached";
    return code;
}

int solve_poisson_impl(ibpm_ctx *c, const double *rhs, double *lam, ibpm_solve_stats *out) {
    if (c->mixed) return solve_poisson_mixed(c, rhs, lam, out);
    return solve_poisson_fp64(c, rhs, lam, out);
}

int solve_velocity_impl(ibpm_ctx *c, const double *rhs, double *q, ibpm_solve_stats *out) {
    std::function<void(const double *, double *)> none;
    return pcg_drive<AView, double>(c, c->A, c->g.n_q, true, none, rhs, q, c->vr, c->vz, c->vp,
                                    c->vq, c->st_vel, c->prm.vel_rtol, c->prm.vel_maxit, c->est_vel,
                                    false, true, out);
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
    if (p->poisson_solver != IBPM_SOLVER_JACOBI_PCG && p->poisson_solver != IBPM_SOLVER_AMG_PCG &&
        p->poisson_solver != IBPM_SOLVER_AMG_PCG_MIXED)
        throw InvalidArg("Poisson solver not available in this build");
    if (p->poisson_solver != IBPM_SOLVER_JACOBI_PCG) {
        if (p->amg_pre < 1 || p->amg_post < 1) throw InvalidArg("AMG needs >= 1 pre and post sweep");
        if (p->amg_coarse_max < 1 || p->amg_max_levels < 1) throw InvalidArg("bad AMG limits");
        if (p->amg_max_levels > kMaxLevels) throw InvalidArg("amg_max_levels too large");
        if (!(p->amg_theta >= 0)) throw InvalidArg("amg_theta must be >= 0");
    }
}

// K0 view in precision T over device metric / coupling arrays
template <class T>
K0T<T> make_k0(const GridT<T> &g, double dt, const Model &m, const DevCSRT<T> &cf,
               const DevCSRT<T> &kf, const T *kfd) {
    K0T<T> K;
    K.g = g;
    K.dt = (T)dt;
    K.nb = m.nb;
    K.n = (int)m.g.n_cell + 2 * m.nb;
    K.cb_i0 = m.cb_i0; K.cb_i1 = m.cb_i1; K.cb_j0 = m.cb_j0; K.cb_j1 = m.cb_j1;
    K.cf = cf.view();
    K.kf = kf.view();
    K.kf_diag = kfd;
    return K;
}

template <class T>
GridT<T> make_grid(ibpm_ctx *c, const GridMetrics &G) {
    std::vector<T> met;
    auto put = [&](const std::vector<double> &v, bool recip) {
        for (double d : v) met.push_back((T)(recip ? 1.0 / d : d));
    };
    put(G.dx, false); put(G.dy, false); put(G.Dx, false); put(G.Dy, false);
    put(G.dx, true); put(G.dy, true); put(G.Dx, true); put(G.Dy, true);
    T *dm = c->upload(met);
    int nx = G.nx, ny = G.ny;
    size_t o = 0;
    GridT<T> g;
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
    return g;
}

// Upload the hierarchy in precision T (values converted from FP64)
template <class T>
void upload_levels(ibpm_ctx *c, PrecSet<T> &P) {
    int L = (int)c->h.levels.size();
    P.lev.resize(L);
    for (int l = 0; l < L; ++l) {
        const Level &hl = c->h.levels[l];
        DevLevelT<T> &dl = P.lev[l];
        dl.n = hl.A.nrows;
        dl.omega = hl.omega;
        if (l > 0) {
            dl.A = c->upload_csr<T>(hl.A);
            dl.wdinv = c->upload(std::vector<T>(hl.wdinv.begin(), hl.wdinv.end()));
            dl.b = c->dalloc<T>(dl.n);
        }
        if (l < L - 1) {
            dl.P = c->upload_csr<T>(hl.P);
            dl.R = c->upload_csr<T>(hl.R);
            dl.r = c->dalloc<T>(dl.n);
        }
        dl.xa = c->dalloc<T>(dl.n);
        dl.xb = c->dalloc<T>(dl.n);
    }
    // the one-work-group coarse cycle takes every level from the first with
    // at most kCoarseRows unknowns (never level 0, which is matrix-free); a
    // single work-group is latency-bound, so only the tiny levels go there
    P.lc = L - 1;
    for (int l = 1; l < L; ++l)
        if (P.lev[l].n <= kCoarseRows) {
            P.lc = l;
            break;
        }
    std::vector<CoarseLevel<T>> cl(L);
    for (int l = 0; l < L; ++l) {
        DevLevelT<T> &dl = P.lev[l];
        CoarseLevel<T> &x = cl[l];
        x.n = dl.n;
        x.A = dl.A.view();
        x.wdinv = dl.wdinv;
        x.P = dl.P.view();
        x.R = dl.R.view();
        x.b = dl.b;
        x.xa = dl.xa;
        x.xb = dl.xb;
        x.r = dl.r;
    }
    std::vector<char> raw(sizeof(CoarseLevel<T>) * L);
    std::memcpy(raw.data(), cl.data(), raw.size());
    P.coarse_dev = (CoarseLevel<T> *)c->upload(raw);
}

template <class T>
void alloc_pcg(ibpm_ctx *c, PrecSet<T> &P, int n) {
    P.r = c->dalloc<T>(n);
    P.z = c->dalloc<T>(n);
    P.p[0] = c->dalloc<T>(n);
    P.p[1] = c->dalloc<T>(n);
    P.q = c->dalloc<T>(n);
    for (T *v : {P.p[0], P.p[1]}) HIPCHECK(hipMemsetAsync(v, 0, n * sizeof(T), c->stream));
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
    c->mixed = p->poisson_solver == IBPM_SOLVER_AMG_PCG_MIXED;
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
    c->g = make_grid<double>(c, G);
    c->ly = 0;
    for (double d : G.dy) c->ly += d;
    WallOffsets wo = WallOffsets::make(G.nx, G.ny);
    c->walls[0] = c->dalloc<double>(wo.total);
    c->walls[1] = c->dalloc<double>(wo.total);
    c->E = c->upload_csr<double>(m.E);
    c->Etu = c->upload_csr<double>(m.Etu);
    c->Etv = c->upload_csr<double>(m.Etv);
    c->ub = c->upload(m.ub);
    DevCSR cf = c->upload_csr<double>(m.Kcf), kf = c->upload_csr<double>(m.Kf);
    double *kfd = c->upload(m.Kf_diag);
    c->p64.K0 = make_k0<double>(c->g, p->dt, m, cf, kf, kfd);
    c->A.g = c->g;
    c->A.dt = p->dt;
    c->A.idt = 1.0 / p->dt;
    c->A.nu = p->nu;
    const int nq = c->g.n_q, nl = c->p64.K0.n;
    if (c->amg) {
        upload_levels<double>(c, c->p64);
        c->coarse_inv = c->upload(c->h.coarse_inv);
    }
    if (c->mixed) {
        GridT<float> g32 = make_grid<float>(c, G);
        DevCSRT<float> cf32 = c->values32(cf, m.Kcf), kf32 = c->values32(kf, m.Kf);
        float *kfd32 = c->upload(std::vector<float>(m.Kf_diag.begin(), m.Kf_diag.end()));
        c->p32.K0 = make_k0<float>(g32, p->dt, m, cf32, kf32, kfd32);
        upload_levels<float>(c, c->p32);
        alloc_pcg(c, c->p32, nl);
        c->rin32 = c->dalloc<float>(nl);
        c->d32 = c->dalloc<float>(nl);
    }
    if (c->amg) {
        // host copies are needed only for sizes and aggregates from now on
        for (auto &hl : c->h.levels) {
            hl.P = CSR();
            hl.R = CSR();
            hl.wdinv.clear();
        }
    }
    c->vr = c->dalloc<double>(nq);
    c->vz = c->dalloc<double>(nq);
    c->vp[0] = c->dalloc<double>(nq);
    c->vp[1] = c->dalloc<double>(nq);
    c->vq = c->dalloc<double>(nq);
    for (double *v : {c->vp[0], c->vp[1]}) HIPCHECK(hipMemsetAsync(v, 0, nq * sizeof(double), c->stream));
    alloc_pcg(c, c->p64, nl);
    c->r1 = c->dalloc<double>(nq);
    c->rhs2 = c->dalloc<double>(nl);
    SolveStatus *sts = c->dalloc<SolveStatus>(5);
    HIPCHECK(hipMemsetAsync(sts, 0, 5 * sizeof(SolveStatus), c->stream));
    c->st_vel = sts;
    c->st_poi = sts + 1;
    c->st_misc = sts + 2;
    c->st_bench = sts + 3;
    c->st_out = sts + 4;
    c->parts = c->dalloc<double>(4 * kMaxParts);
    HIPCHECK(hipHostMalloc((void **)&c->host_st, sizeof(SolveStatus), hipHostMallocDefault));
    double U = p->uinf * std::cos(p->alpha), V = p->uinf * std::sin(p->alpha);
    launch_fill_walls(c->stream, c->g, c->walls[0], U, V);
    launch_fill_walls(c->stream, c->g, c->walls[1], U, V);
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
    if (nl) *nl = c->p64.K0.n;
    return IBPM_OK;
}

int ibpm_init_state(ibpm_ctx *c, double *q, double *conv, double *lam) {
    return guarded(c, [&] {
        if (!q || !conv || !lam) throw InvalidArg("NULL vector");
        double U = c->prm.uinf * std::cos(c->prm.alpha), V = c->prm.uinf * std::sin(c->prm.alpha);
        launch_init_state(c->stream, c->g, q, conv, lam, c->p64.K0.n, U, V);
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
        launch_apply_K0(c->stream, c->p64.K0, x, y);
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
                               kernel == IBPM_KERNEL_RESTRICT0 || kernel == IBPM_KERNEL_PROLONG0 ||
                               kernel == IBPM_KERNEL_COARSE_CYCLE;
        PrecSet<double> &P = c->p64;
        if (needs_amg && (!c->amg || P.lev.size() < 2)) throw InvalidArg("kernel needs an AMG hierarchy");
        hipStream_t s = c->stream;
        const K0View &K = P.K0;
        const int n = K.n, nq = c->g.n_q;
        const Model &m = c->m;
        // compulsory bytes of the coupling part of K and of the grid metrics
        const double b_metric = 2.0 * 8.0 * (2.0 * m.g.nx + 2.0 * m.g.ny + 2.0);
        const double b_coupling = 12.0 * (double)(m.Kcf.nnz() + m.Kf.nnz()) +
                                  4.0 * (double)(m.Kcf.nrows + m.Kf.nrows + 2) + 8.0 * 2 * m.nb;
        auto csr_bytes = [](const DevCSR &M, bool add) {
            return 12.0 * (double)M.nnz + 4.0 * (M.nrows + 1) + 8.0 * M.ncols +
                   (add ? 16.0 : 8.0) * M.nrows;
        };
        // a status that never converges and keeps every scalar finite
        SolveStatus st0{};
        st0.bb = 1.0;
        st0.tol2 = -1.0;
        st0.rz = 1.0;
        st0.pq = 1.0;
        st0.maxit = 0x7fffffff;
        HIPCHECK(hipMemcpyAsync(c->st_bench, &st0, sizeof(st0), hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemsetAsync(P.r, 0, n * sizeof(double), s));
        HIPCHECK(hipMemsetAsync(P.z, 0, n * sizeof(double), s));
        HIPCHECK(hipMemsetAsync(P.q, 0, n * sizeof(double), s));
        HIPCHECK(hipMemsetAsync(c->vr, 0, nq * sizeof(double), s));
        HIPCHECK(hipMemsetAsync(c->vz, 0, nq * sizeof(double), s));
        HIPCHECK(hipStreamSynchronize(s));
        SolveStatus *sb = c->st_bench;
        double by = 0;
        std::function<void()> launch;
        switch (kernel) {
        case IBPM_KERNEL_K0_JACOBI: {
            DevLevelT<double> &l0 = P.lev[0];
            launch = [&] { launch_k0_jacobi(s, K, l0.omega, (const double *)P.r, (const double *)l0.xa, l0.xb, sb); };
            by = 24.0 * n + b_coupling + b_metric;
            break;
        }
        case IBPM_KERNEL_K0_PCG_SPMV:
            launch = [&] { launch_pcg_spmv(s, K, (const double *)P.z, (const double *)P.p[0], P.p[1], P.q, sb, c->parts); };
            by = 32.0 * n + b_coupling + b_metric;
            break;
        case IBPM_KERNEL_A_PCG_SPMV:
            launch = [&] { launch_pcg_spmv(s, c->A, (const double *)c->vz, (const double *)c->vp[0], c->vp[1], c->vq, sb, c->parts); };
            by = 32.0 * nq + b_metric;
            break;
        case IBPM_KERNEL_K0_RESIDUAL: {
            DevLevelT<double> &l0 = P.lev[0];
            launch = [&] { launch_k0_residual(s, K, (const double *)P.r, (const double *)l0.xa, l0.r, sb); };
            by = 24.0 * n + b_coupling + b_metric;
            break;
        }
        case IBPM_KERNEL_RESTRICT0: {
            DevLevelT<double> &l0 = P.lev[0];
            launch = [&] { launch_csrv_spmv(s, l0.R.view(), l0.R.lanes, (const double *)l0.r, P.lev[1].b, false, sb); };
            by = csr_bytes(l0.R, false);
            break;
        }
        case IBPM_KERNEL_PROLONG0: {
            DevLevelT<double> &l0 = P.lev[0];
            launch = [&] { launch_csrv_spmv(s, l0.P.view(), l0.P.lanes, (const double *)P.lev[1].xa, l0.xa, true, sb); };
            by = csr_bytes(l0.P, true);
            break;
        }
        case IBPM_KERNEL_PCG_UPDATE_K:
            launch = [&] { launch_pcg_update(s, K, P.p[1], P.r, P.z, (const double *)P.p[0], (const double *)P.q, sb, c->parts, false); };
            by = 48.0 * n;
            break;
        case IBPM_KERNEL_COARSE_CYCLE: {
            int L = (int)P.lev.size();
            launch = [&] { launch_coarse_cycle(s, (const CoarseLevel<double> *)P.coarse_dev, P.lc, L, c->prm.amg_pre, c->prm.amg_post, c->coarse_inv, P.lev[L - 1].n, sb); };
            by = 0.0;
            for (int l = P.lc; l < L; ++l) by += (l < L - 1 ? csr_bytes(P.lev[l].A, false) : 0.0);
            break;
        }
        default:
            throw InvalidArg("unknown kernel id");
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
