// C ABI of the library: context set-up, the time-step driver and the
// Krylov / AMG drivers that queue the kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <functional>
#include <initializer_list>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/ibpm.h"
#include "kernels.h"
#include "nn.h"
#include "setup.h"
#include "spgemm.h"
#include "moving.h"

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
    int32_t *bst = nullptr;            // row blocks of the row-block kernels (nblk + 1 row starts),
    int rpb = 0;                       // or rpb rows each
    int nblk = 0;
    CSRT<T> view() const { return CSRT<T>{nrows, ncols, ptr, col, val, bst, rpb, nblk}; }
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
    DevCSRT<T> RA, AP;                 // fused transfers (nrows 0 where not formed)
    T *wdinv = nullptr;
    T *b = nullptr, *xa = nullptr, *xb = nullptr, *r = nullptr;
    int32_t *agg = nullptr;            // level 0: aggregates (matrix-free prolongation)
    double pomega = 0;                 // level 0: prolongator smoothing weight
};

// Everything one precision needs for the Poisson solve
template <class T>
struct PrecSet {
    K0T<T> K0{};
    std::vector<DevLevelT<T>> lev;
    double *coarseC = nullptr;         // cycle on levels lc.. as a dense FP64 matrix
    int lc = 1;                        // first level of the dense coarse cycle
    // PCG work vectors (n_lambda)
    T *r = nullptr, *z = nullptr, *p[2] = {nullptr, nullptr}, *q = nullptr;
    T *r2 = nullptr;                   // second residual (the update folded into the cycle)
};

// The residual-to-correction network (weights, Adam moments, activations)
struct NNState {
    bool ready = false, train_ready = false;
    int H = 0, W = 0;
    int cin[kNNLayers] = {kNNInPad, 32, 32, 32, 32, 32};
    int kp[kNNLayers] = {};
    float *master[kNNLayers] = {}, *grad[kNNLayers] = {}, *m[kNNLayers] = {}, *v[kNNLayers] = {};
    bf16 *fwd[kNNLayers] = {}, *bwd[kNNLayers] = {};
    bf16 *act[kNNLayers] = {};        // act[0]: features [H][W][8]; act[l]: output of layer l-1
    float *y32 = nullptr;             // network output [H][W][32]
    float *g[2] = {nullptr, nullptr}; // gradients [H][W][32]
    float *partials = nullptr, *fdiff = nullptr;
    double *scale = nullptr, *sparts = nullptr, *losses = nullptr;
    double *d = nullptr, *r1 = nullptr, *z0 = nullptr;   // learned-stage work vectors (FP64)
    float *d32 = nullptr, *r132 = nullptr, *z032 = nullptr;   // and FP32 (mixed inner solve)
    SolveStatus *st = nullptr;
    CellDelta cd{};
    int adam_t = 0;
    double inv_hmin = 1.0;
    int max_losses = 0;
};

// ring of FCG(m) directions for precision T (allocated on first use)
template <class T> struct FcgStore { FcgVecs<T> P{}, Q{}; int m = 0; };

}  // namespace

struct ibpm_ctx {
    std::string err;
    hipStream_t stream = nullptr;
    ibpm_params prm{};
    Model m;
    Hierarchy h;
    bool amg = false, mixed = false, mixed_precond = false;
    bool guess_learned = false;        // solver 6: learned initial guess before the FP32-cycle CG
    double *static_work = nullptr;     // device address of the file-scope work array on this
                                       // context's device (ibpm_solve_velocity_static)
    // B^N with N > 1: the operator B^N and Q (device CSR) for the projection,
    // the stored level-0 K = Q^T B^N Q with its diagonal, and Q lambda
    int bn = 1;
    DevCSR Bn{}, Qd{}, K0c{};
    CsrOpView K0op{};
    // a body in prescribed motion: the level-0 K is stored and re-assembled
    // on the device at every move (moving.hip); stored0 = the level-0
    // operator is a stored CSR (B^N with N > 1, or a moving body)
    bool moving = false, stored0 = false;
    int64_t moves = 0, K_cap = 0;
    DevCSR Kpp{};                                   // fixed pressure rows
    double *xf_d = nullptr, *yf_d = nullptr, *xb_d = nullptr, *yb_d = nullptr;
    int32_t *ecol = nullptr, *eptr = nullptr;       // E rows, kEllE entries each
    double *eval = nullptr;
    int32_t *len_all = nullptr, *force_len = nullptr, *box_len = nullptr;
    int64_t *ptr64 = nullptr, *scan_tiles = nullptr, *scan_total = nullptr, *force_ptr = nullptr,
            *box_ptr = nullptr;
    int32_t *force_col = nullptr, *box_col = nullptr;
    double *force_val = nullptr, *box_val = nullptr;
    int64_t force_cap = 0, box_cap = 0, box_rows_cap = 0;
    int box[4] = {0, -1, 0, -1};                    // cells whose faces E reaches (i0, i1, j0, j1)
    double *K0diag = nullptr;
    // the three-dimensional extension: stored A (with its diagonal), Q,
    // Q^T and B^1 (as a diagonal CSR) for the linear algebra of a step
    bool three_d = false;
    DevCSR A3{}, Q3{}, QT3{}, B3{};
    CsrOpView A3op{};
    int64_t n_q3 = 0;
    std::vector<int32_t *> agg_d;                   // aggregates of the levels formed on the device
    std::vector<int64_t> level_nnz;                 // entries of each level's operator
    int64_t refreshes = 0;
    double *wq = nullptr;
    int64_t bn_peak_bytes = 0, bn_unsliced_bytes = 0;
    std::vector<void *> allocs;
    GridView g{};
    AView A{};
    double ly = 0;
    WallSides wall_init{};             // wall velocities at the start (per side)
    int convective = 0;                // 1: the right wall is a convective outflow
    double *walls[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t step = 0;
    DevCSR E, Etu, Etv;
    double *ub = nullptr;
    PrecSet<double> p64;
    PrecSet<float> p32;
    float *rin32 = nullptr, *d32 = nullptr;          // mixed: inner right-hand side and correction
    double *coarse_inv = nullptr;
    std::vector<double> coarse_C;      // host copy of the dense coarse-cycle matrix
    double *coarse_C_dev = nullptr;    // its device copy (shared by both precisions)
    double *copy_x = nullptr, *copy_y = nullptr;   // bandwidth reference buffers
    FcgStore<double> fcg64;                        // FCG(m) direction rings
    FcgStore<float> fcg32;
    FcgRing *fcg_ring = nullptr;
    int coarse_C_lc = -1;
    // velocity PCG (n_q)
    double *vr = nullptr, *vz = nullptr, *vp[2] = {nullptr, nullptr}, *vq = nullptr;
    double *r1 = nullptr, *rhs2 = nullptr;
    SolveStatus *st_vel = nullptr, *st_poi = nullptr, *st_misc = nullptr, *st_bench = nullptr,
                *st_out = nullptr;
    double *parts = nullptr;
    double *parts2 = nullptr;          // second partial-sum buffer (read by the next kernel)
    double *parts3 = nullptr;          // r . r partials of a deferred PCG update
    int rz_G = 0;                      // partials of r . z left in parts by the last V-cycle
    SolveStatus *host_st = nullptr;   // pinned
    int est_vel = 8, est_poi = 32;
    int est_inner[32];                 // iterations of the k-th inner solve of a refinement
    ibpm_ctx() { for (int &e : est_inner) e = 32; }
    bool learned = false;
    NNState nn;

    template <class T>
    T *dalloc(size_t n) {
        void *p = nullptr;
        if (n == 0) n = 1;
        hipError_t e = hipMalloc(&p, n * sizeof(T));
        if (e != hipSuccess) throw std::bad_alloc();
        allocs.push_back(p);
        return (T *)p;
    }
    // device memory that does not live as long as the context (set-up
    // temporaries): released by dfree
    template <class T>
    T *dtemp(size_t n) {
        void *p = nullptr;
        if (n == 0) n = 1;
        if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) throw std::bad_alloc();
        return (T *)p;
    }
    void dfree(const void *p) {
        if (p) (void)hipFree(const_cast<void *>(p));
    }
    // free memory taken with dalloc before the context ends
    void release(const void *p) {
        if (!p) return;
        auto it = std::find(allocs.begin(), allocs.end(), const_cast<void *>(p));
        if (it != allocs.end()) {
            allocs.erase(it);
            (void)hipFree(const_cast<void *>(p));
        }
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
    // HIP graphs of two PCG iterations, one per solve kind (velocity,
    // Poisson FP64, inner FP32), with the operand addresses they were made for
    struct IterGraph {
        hipGraphExec_t exec = nullptr;
        std::vector<const void *> key;
    };
    IterGraph graphs[3];
    hipStream_t cap_stream = nullptr;  // used only to record the graphs
    ~ibpm_ctx() {
        if (stream) (void)hipStreamSynchronize(stream);
        for (IterGraph &g : graphs)
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (void *p : allocs) (void)hipFree(p);
        if (host_st) (void)hipHostFree(host_st);
    }
};

namespace {

int fail(ibpm_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

// the entry points of the two-dimensional time step refuse a 3-D context
void need2d(const ibpm_ctx *c) {
    if (c->three_d) throw InvalidArg("a two-dimensional entry point called on a three-dimensional context");
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

// A PCG update left for the preconditioner's first kernel to apply:
// alpha = st->rz_next / (p . q) with p . q summed from pq_parts, x += alpha p,
// r_out = r_in - alpha q (the residual the preconditioner is applied to)
template <class T>
struct UpdArgs {
    T *x;
    const T *r_in;
    T *r_out;
    const T *p, *q;
    const double *pq_parts;
};

// An FP32 cycle inside FP64 CG: the residual r64 (FP64) and its FP32 copy
// r32, the FP64 result z64; u, when given, is the FP64 update folded into
// the first pass (which then writes r32).
struct MixedIO {
    const UpdArgs<double> *u;
    const double *r64;
    double *z64;
    float *r32;
};

// With u, the cycle starts with the update (folded into the first two
// pre-smoothing sweeps) and is applied to u->r_out; the partials of the new
// r . r go to c->parts3 (one per block of the level-0 walker grid).  With mx
// (an FP32 cycle) the last sweep writes mx->z64 and the partials of
// r64 . z64 instead of z.
template <class T>
void enqueue_vcycle(ibpm_ctx *c, PrecSet<T> &P, const T *r, T *z, SolveStatus *st,
                    bool with_rz = true, const UpdArgs<T> *u = nullptr, const MixedIO *mx = nullptr) {
    hipStream_t s = c->stream;
    const int pre = c->prm.amg_pre, post = c->prm.amg_post;
    const int L = (int)P.lev.size();
    const K0T<T> &K = P.K0;
    constexpr bool f32 = std::is_same<T, float>::value;
    if ((u || (mx && mx->u)) && (L == 1 || pre < 2))
        throw std::runtime_error("V-cycle: the update folds into two pre-sweeps only");
    if (mx && (!f32 || u || L == 1)) throw std::runtime_error("V-cycle: bad mixed-precision request");
    if (u) r = u->r_out;
    if (mx && mx->u) r = (const T *)mx->r32;
    if (L == 1) {
        launch_dense_solve(s, K.n, c->coarse_inv, r, z, st);
        if (with_rz) c->rz_G = launch_dot_rz_parts(s, K.n, r, z, st, c->parts);
        return;
    }
    std::vector<T *> cur(L);
    {
        DevLevelT<T> &l0 = P.lev[0];
        T *a = l0.xa, *b = l0.xb;
        int k = 1;
        // on grids whose product has more partials than a block gathers, p.q
        // and the update's stop test come from one-block finalizes
        const int G_pq = walk_blocks_of(K);
        const bool fin = G_pq > kFuseMaxParts;
        if (u) {
            if (fin) launch_finalize_pq(s, G_pq, u->pq_parts, st);
            const int G = launch_k0_update_presmooth2(s, K, (const T *)l0.wdinv, u->x, u->r_in, u->r_out, u->p,
                                                      u->q, a, st, fin ? nullptr : u->pq_parts, c->parts3);
            if (fin) launch_finalize_update(s, G, c->parts3, st, 2);
            k = 2;
        } else if (mx && mx->u) {
            if constexpr (f32) {
                const UpdArgs<double> *v = mx->u;
                if (fin) launch_finalize_pq(s, G_pq, v->pq_parts, st);
                const int G = launch_k0_update_presmooth2_mixed(s, K, (const float *)l0.wdinv, v->x, v->r_in,
                                                                v->r_out, v->p, v->q, a, mx->r32, st,
                                                                fin ? nullptr : v->pq_parts, c->parts3);
                if (fin) launch_finalize_update(s, G, c->parts3, st, 2);
            }
            k = 2;
        } else if (pre >= 2) {
            launch_k0_presmooth2(s, K, (const T *)l0.wdinv, r, a, st);
            k = 2;
        } else {
            launch_k0_jacobi_first(s, K, l0.omega, r, a, st);
        }
        for (; k < pre; ++k) {
            launch_k0_jacobi(s, K, l0.omega, r, a, b, st);
            std::swap(a, b);
        }
        cur[0] = a;
        if (l0.RA.nrows > 0) {
            launch_csrv_restrict(s, l0.R.view(), l0.RA.view(), l0.RA.lanes, r, (const T *)a, P.lev[1].b, st);
        } else {
            launch_k0_residual(s, K, r, (const T *)a, l0.r, st);
            launch_csrv_spmv(s, l0.R.view(), l0.R.lanes, (const T *)l0.r, P.lev[1].b, false, st);
        }
    }
    for (int l = 1; l < P.lc; ++l) {
        DevLevelT<T> &lv = P.lev[l];
        T *a = lv.xa, *b = lv.xb;
        int k = 1;
        if (pre >= 2) {
            launch_csrv_presmooth2(s, lv.A.view(), lv.A.lanes, (const T *)lv.wdinv, (const T *)lv.b, a, st);
            k = 2;
        } else {
            launch_csr_jacobi_first(s, lv.A.view(), (const T *)lv.wdinv, (const T *)lv.b, a, st);
        }
        for (; k < pre; ++k) {
            launch_csrv_jacobi(s, lv.A.view(), lv.A.lanes, (const T *)lv.wdinv, (const T *)lv.b,
                               (const T *)a, b, st);
            std::swap(a, b);
        }
        cur[l] = a;
        if (lv.RA.nrows > 0) {
            launch_csrv_restrict(s, lv.R.view(), lv.RA.view(), lv.RA.lanes, (const T *)lv.b, (const T *)a,
                                 P.lev[l + 1].b, st);
        } else {
            launch_csrv_residual(s, lv.A.view(), lv.A.lanes, (const T *)lv.b, (const T *)a, lv.r, st);
            launch_csrv_spmv(s, lv.R.view(), lv.R.lanes, (const T *)lv.r, P.lev[l + 1].b, false, st);
        }
    }
    launch_coarse_dense(s, P.lev[P.lc].n, (const double *)P.coarseC, (const T *)P.lev[P.lc].b,
                        P.lev[P.lc].xa, st);
    cur[P.lc] = P.lev[P.lc].xa;
    for (int l = P.lc - 1; l >= 1; --l) {
        DevLevelT<T> &lv = P.lev[l];
        T *a = cur[l];
        T *b = (a == lv.xa) ? lv.xb : lv.xa;
        int k = 0;
        if (lv.AP.nrows > 0) {
            // prolongation and the first post-sweep in one pass
            launch_csrv_prolong_jacobi(s, lv.A.view(), lv.AP.view(), lv.P.view(), lv.AP.lanes,
                                       (const T *)lv.wdinv, (const T *)lv.b, (const T *)a,
                                       (const T *)cur[l + 1], b, st);
            std::swap(a, b);
            k = 1;
        } else {
            launch_csrv_spmv(s, lv.P.view(), lv.P.lanes, (const T *)cur[l + 1], a, true, st);
        }
        for (; k < post; ++k) {
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
        if (post == 2 && post2_rows(K) > 0) {
            // the prolongation and both post-sweeps in one pass
            if (mx) {
                if constexpr (f32)
                    c->rz_G = launch_k0_prolong_post2(s, K, (const int *)l0.agg, (const T *)cur[1], l0.pomega,
                                                      l0.omega, r, (const T *)a, b, l0.r, (T *)nullptr, mx->z64,
                                                      mx->r64, st, c->parts, POST_WIDEN);
            } else {
                const int G = launch_k0_prolong_post2(s, K, (const int *)l0.agg, (const T *)cur[1], l0.pomega,
                                                      l0.omega, r, (const T *)a, b, l0.r, z, nullptr, nullptr, st,
                                                      c->parts, with_rz ? POST_RZ : POST_PLAIN);
                if (with_rz) c->rz_G = G;
            }
            return;
        }
        launch_k0_prolong_mf(s, K, (const int *)l0.agg, (const T *)cur[1], l0.pomega, a, st);
        for (int k = 0; k < post - 1; ++k) {
            launch_k0_jacobi(s, K, l0.omega, r, (const T *)a, b, st);
            std::swap(a, b);
        }
        if (mx) {
            if constexpr (f32)
                c->rz_G = launch_k0_jacobi_widen_rz(s, K, l0.omega, r, (const float *)a, mx->z64, mx->r64, st,
                                                    c->parts);
        } else if (with_rz) {
            c->rz_G = launch_k0_jacobi_rz(s, K, l0.omega, r, (const T *)a, z, st, c->parts);
        } else {
            launch_k0_jacobi(s, K, l0.omega, r, (const T *)a, z, st);
        }
    }
}

// A preconditioner that can start with the pending PCG update (see
// UpdArgs): fn(u, z) queues the update and z = M u.r_out; r2 is the second
// residual buffer; G_pq and G_rr are the partial counts of the product and
// of the folded update (both at most kFuseMaxParts for it to be used).
template <class T>
struct FusedPre {
    std::function<void(const UpdArgs<T> &, T *)> fn;
    T *r2;
    int G_pq, G_rr;
};

// CG iterations per recorded graph (even: the direction and residual
// buffers swap every iteration, so a replay leaves them as it found them)
constexpr int kGraphIters = 8;

// Generic PCG driver.  Iterations are queued in chunks; every kernel of an
// iteration is predicated on the device status, so iterations queued past
// convergence do nothing.  The chunk length is estimated from the observed
// residual decay so few empty iterations are queued.
//   precond(r, z): queue z = M r (with the r . z reduction); null for Jacobi
template <class Op, class T>
int pcg_drive(ibpm_ctx *c, const Op &op, int n, bool jacobi,
              const std::function<void(const T *, T *)> &precond, const T *b, T *x, T *r, T *z,
              T **p, T *q, SolveStatus *st, double rtol, int maxit, int &est, bool zero_guess,
              bool true_residual, ibpm_solve_stats *out, int graph_slot = -1,
              const FusedPre<T> *fpre = nullptr) {
    hipStream_t s = c->stream;
    auto t0 = std::chrono::steady_clock::now();
    if (zero_guess) launch_pcg_init_zero(s, n, b, x, r, st, c->parts, rtol * rtol, maxit);
    else launch_pcg_init(s, op, b, (const T *)x, r, z, st, c->parts, jacobi, rtol * rtol, maxit);
    if (!jacobi) precond(r, z);
    int curp = 0;
    // With a preconditioner whose r . z partials the product sums itself,
    // the update's stop test moves into the next product (no finalize
    // launch per iteration): the update leaves its r . r partials in parts3
    // and the preconditioner runs once more after the converged update, on
    // a residual no later kernel uses.
    // With a preconditioner that starts with the update, the update kernel
    // goes too: the residual then alternates between r and fpre->r2.  With
    // the deferred stop test the folded pass gathers the product's partials
    // itself; where it cannot (large grids) one-block finalizes around the
    // pass give it p.q and take the stop test, and the fold is kept: it
    // saves a whole pass, the deferred test only a one-block launch.
    const bool fuse = fpre != nullptr;
    const bool defer = !jacobi && c->rz_G <= kFuseMaxParts && update_blocks_of(n) <= kFuseMaxParts &&
                       (!fuse || (fpre->G_pq <= kFuseMaxParts && fpre->G_rr <= kFuseMaxParts));
    const int G_rr = fuse ? fpre->G_rr : update_blocks_of(n);
    T *rcur = r, *rnext = fuse ? fpre->r2 : nullptr;
    auto iteration = [&]() {
        // with the V-cycle the product sums its r . z partials (in parts)
        launch_pcg_spmv(s, op, (const T *)z, (const T *)p[curp], p[1 - curp], q, st,
                        jacobi ? (const double *)nullptr : (const double *)c->parts, c->rz_G,
                        c->parts2, defer ? (const double *)c->parts3 : (const double *)nullptr,
                        defer ? G_rr : 0);
        curp = 1 - curp;
        if (fuse) {
            const UpdArgs<T> u{x, (const T *)rcur, rnext, (const T *)p[curp], (const T *)q,
                               (const double *)c->parts2};
            fpre->fn(u, z);
            std::swap(rcur, rnext);
        } else {
            launch_pcg_update(s, op, x, rcur, z, (const T *)p[curp], (const T *)q, st,
                              (const double *)c->parts2, defer ? c->parts3 : c->parts, jacobi, !jacobi,
                              defer);
            if (!jacobi) precond(rcur, z);
        }
    };
    // the iterations are identical launches (the two direction buffers swap
    // every iteration), so a graph of kGraphIters of them is replayed
    hipGraphExec_t gexec = nullptr;
    if (c->prm.use_graphs && graph_slot >= 0) {
        ibpm_ctx::IterGraph &G = c->graphs[graph_slot];
        std::vector<const void *> key = {&op, b, x, r, z, p[0], p[1], q, st,
                                         (const void *)(intptr_t)jacobi,
                                         (const void *)(intptr_t)c->rz_G, rnext};
        if (!G.exec || G.key != key) {
            if (G.exec) (void)hipGraphExecDestroy(G.exec);
            G.exec = nullptr;
            // capture on the context's own capture stream (the caller's
            // stream may be the legacy default stream, which cannot be
            // captured); the graph is then launched on the caller's stream
            if (!c->cap_stream) HIPCHECK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
            hipGraph_t graph = nullptr;
            HIPCHECK(hipStreamSynchronize(s));
            const hipStream_t user = c->stream;
            c->stream = c->cap_stream;
            s = c->cap_stream;
            HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            try {
                for (int k = 0; k < kGraphIters; ++k) iteration();
            } catch (...) {
                (void)hipStreamEndCapture(s, &graph);
                if (graph) (void)hipGraphDestroy(graph);
                c->stream = user;
                s = user;
                throw;
            }
            hipError_t ec = hipStreamEndCapture(s, &graph);
            c->stream = user;
            s = user;
            if (ec != hipSuccess) throw HipError(std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
            hipError_t e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                G.exec = nullptr;
                throw HipError(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
            G.key = key;
        }
        gexec = G.exec;
    }
    int chunk = std::max(1, (int)(0.8 * est));
    int queued = 0;
    double last_rr = -1;
    int last_it = 0;
    for (;;) {
        if (gexec) {
            chunk = (chunk + kGraphIters - 1) / kGraphIters * kGraphIters;
            for (int k = 0; k < chunk; k += kGraphIters) HIPCHECK(hipGraphLaunch(gexec, s));
        } else {
            for (int k = 0; k < chunk; ++k) iteration();
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

void enqueue_vcycle_csr(ibpm_ctx *c, PrecSet<double> &P, const double *r, double *z, SolveStatus *st);

FcgStore<double> &fcg_store(ibpm_ctx *c, double *) { return c->fcg64; }
FcgStore<float> &fcg_store(ibpm_ctx *c, float *) { return c->fcg32; }

int solve_poisson_fp64(ibpm_ctx *c, const double *rhs, double *lam, ibpm_solve_stats *out) {
    bool jacobi = !c->amg;
    if (c->stored0) {
        // B^N with N > 1 or a moving body: the stored K and the all-CSR V-cycle
        std::function<void(const double *, double *)> pre = [c](const double *r, double *z) {
            enqueue_vcycle_csr(c, c->p64, r, z, c->st_poi);
        };
        PrecSet<double> &P = c->p64;
        return pcg_drive<CsrOpView, double>(c, c->K0op, c->K0op.A.nrows, jacobi, pre, rhs, lam, P.r, P.z, P.p,
                                            P.q, c->st_poi, c->prm.poisson_rtol, c->prm.poisson_maxit,
                                            c->est_poi, false, true, out, 1, nullptr);
    }
    PrecSet<double> &P = c->p64;
    std::function<void(const double *, double *)> pre = [c](const double *r, double *z) {
        enqueue_vcycle(c, c->p64, r, z, c->st_poi);
    };
    FusedPre<double> fpre{[c](const UpdArgs<double> &u, double *z) {
                              enqueue_vcycle(c, c->p64, (const double *)u.r_out, z, c->st_poi, true, &u);
                          },
                          P.r2, walk_blocks_of(P.K0), walk_blocks_of(P.K0)};
    const bool can_fuse = !jacobi && P.lev.size() > 1 && c->prm.amg_pre >= 2;
    return pcg_drive<K0View, double>(c, P.K0, P.K0.n, jacobi, pre, rhs, lam, P.r, P.z, P.p, P.q,
                                     c->st_poi, c->prm.poisson_rtol, c->prm.poisson_maxit,
                                     c->est_poi, false, true, out, 1, can_fuse ? &fpre : nullptr);
}

// Mixed precision: FP64 iterative refinement around an FP32 AMG-PCG.  The
// outer residual, its norm, the correction update and the coarsest-level
// solve are FP64; the inner SpMV, V-cycle and vectors are FP32 with FP64
// dot products.  Each inner solve is asked for the reduction the outer
// tolerance still needs (at least 1e-5, about what FP32 can deliver).
template <class T>
SolveStatus fcg_learned_drive(ibpm_ctx *c, PrecSet<T> &P, const T *b, T *x, SolveStatus *st,
                              double rtol, int maxit, int &est, bool zero_guess, bool *stall);
void learned_guess(ibpm_ctx *c, const double *b, double *x, SolveStatus *st);

// FP64 iterative refinement: r = b - K x in FP64, an FP32 inner solve of
// K d = r to a relative tolerance that aims at the outer one, x += d.  The
// inner solve is AMG-PCG, or with the learned stage flexible CG with the
// network (falling back to AMG-PCG for the remaining inner solves once a
// learned inner solve stalls or breaks down).
int solve_poisson_mixed(ibpm_ctx *c, const double *rhs, double *lam, ibpm_solve_stats *out) {
    hipStream_t s = c->stream;
    auto t0 = std::chrono::steady_clock::now();
    const K0View &K = c->p64.K0;
    const int n = K.n;
    const double rtol = c->prm.poisson_rtol;
    const bool learned = c->learned;
    if (learned && !c->nn.ready)
        throw InvalidArg("the learned solver needs network weights (ibpm_nn_init or ibpm_nn_set_weights)");
    if (learned) learned_guess(c, rhs, lam, c->st_poi);
    launch_outer_residual(s, K, rhs, lam, c->rin32, c->st_out, c->parts, 1);
    c->read_status(c->st_out);
    double bb = c->host_st->bb, rr = c->host_st->rr;
    int inner_total = 0, outer = 0, code = IBPM_OK, fallbacks = 0;
    bool plain = !learned;
    PrecSet<float> &P = c->p32;
    std::function<void(const float *, float *)> pre = [c](const float *r, float *z) {
        enqueue_vcycle(c, c->p32, r, z, c->st_poi);
    };
    FusedPre<float> fpre{[c](const UpdArgs<float> &u, float *z) {
                             enqueue_vcycle(c, c->p32, (const float *)u.r_out, z, c->st_poi, true, &u);
                         },
                         P.r2, walk_blocks_of(K), walk_blocks_of(K)};
    const bool can_fuse = P.lev.size() > 1 && c->prm.amg_pre >= 2;
    if (bb == 0.0) {
        HIPCHECK(hipMemsetAsync(lam, 0, n * sizeof(double), s));
        rr = 0.0;
    }
    const double floor_in = c->prm.inner_rtol > 0 ? c->prm.inner_rtol : 1e-5;
    while (bb > 0.0 && rr > rtol * rtol * bb) {
        if (!(rr == rr)) {
            code = IBPM_ENAN;
            break;
        }
        if (outer >= 30 || inner_total >= c->prm.poisson_maxit) {
            code = IBPM_ENOTCONV;
            break;
        }
        // the inner solve aims at a tenth of the outer tolerance, so the last
        // outer step ends well inside it: the force unknowns (and the drag)
        // carry the slowest modes, and a residual just under rtol leaves them
        // further from the FP64 solution than the FP64 solver's own stop does
        double need = rtol * std::sqrt(bb / rr);
        double tol_in = std::max(0.1 * need, floor_in);
        const int maxit_in = c->prm.poisson_maxit - inner_total;
        bool add = true;
        if (!plain) {
            bool stall = false;
            SolveStatus h = fcg_learned_drive<float>(c, P, c->rin32, c->d32, c->st_poi, tol_in,
                                                     maxit_in, c->est_inner[std::min(outer, 31)], true, &stall);
            inner_total += h.iter;
            if (h.done == ST_NAN) add = false;
            if (stall || h.done == ST_NAN) {
                plain = true;
                fallbacks = 1;
            }
        } else {
            ibpm_solve_stats is{};
            int rc = pcg_drive<K0T<float>, float>(c, P.K0, n, false, pre, c->rin32, c->d32, P.r,
                                                  P.z, P.p, P.q, c->st_poi, tol_in, maxit_in,
                                                  c->est_inner[std::min(outer, 31)], true, false, &is, 2,
                                                  can_fuse ? &fpre : nullptr);
            inner_total += is.iters;
            if (rc == IBPM_ENAN) {
                code = IBPM_ENAN;
                break;
            }
        }
        if (add) launch_add_correction(s, n, lam, c->d32);
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
        out->fallbacks = fallbacks;
    }
    if (code == IBPM_ENAN) c->err = "residual became NaN";
    else if (code == IBPM_ENOTCONV) c->err = "iteration limit reached";
    return code;
}

// ---------------------------------------------------------------------------
// residual-to-correction network

size_t img(const NNState &N, int ch) { return (size_t)N.H * N.W * ch; }

void nn_alloc(ibpm_ctx *c) {
    NNState &N = c->nn;
    if (N.ready) return;
    const Model &m = c->m;
    N.H = m.g.ny;
    N.W = m.g.nx;
    for (int l = 0; l < kNNLayers; ++l) {
        N.kp[l] = conv_kp(N.cin[l]);
        size_t np = (size_t)32 * N.kp[l];
        N.master[l] = c->dalloc<float>(np);
        N.fwd[l] = c->dalloc<bf16>(np);
        N.bwd[l] = c->dalloc<bf16>((size_t)32 * conv_kp(32));
        N.act[l] = c->dalloc<bf16>(img(N, l == 0 ? kNNInPad : 32));
    }
    N.y32 = c->dalloc<float>(img(N, 32));
    N.scale = c->dalloc<double>(2);
    N.sparts = c->dalloc<double>(1024);
    const int n = c->p64.K0.n;
    N.d = c->dalloc<double>(n);
    N.r1 = c->dalloc<double>(n);
    N.z0 = c->dalloc<double>(n);
    if (c->mixed) {
        N.d32 = c->dalloc<float>(n);
        N.r132 = c->dalloc<float>(n);
        N.z032 = c->dalloc<float>(n);
    }
    N.st = c->dalloc<SolveStatus>(1);
    HIPCHECK(hipMemsetAsync(N.st, 0, sizeof(SolveStatus), c->stream));
    DevCSR c2p = c->upload_csr<double>(m.Dc2p), p2c = c->upload_csr<double>(m.Dp2c);
    N.cd.i0 = m.dc_i0; N.cd.i1 = m.dc_i1; N.cd.j0 = m.dc_j0; N.cd.j1 = m.dc_j1;
    N.cd.c2p = c2p.view();
    N.cd.p2c = p2c.view();
    N.inv_hmin = 1.0 / m.hmin;
    N.ready = true;
}

void nn_alloc_training(ibpm_ctx *c) {
    NNState &N = c->nn;
    if (N.train_ready) return;
    for (int l = 0; l < kNNLayers; ++l) {
        size_t np = (size_t)32 * N.kp[l];
        N.grad[l] = c->dalloc<float>(np);
        N.m[l] = c->dalloc<float>(np);
        N.v[l] = c->dalloc<float>(np);
        HIPCHECK(hipMemsetAsync(N.m[l], 0, np * sizeof(float), c->stream));
        HIPCHECK(hipMemsetAsync(N.v[l], 0, np * sizeof(float), c->stream));
    }
    N.g[0] = c->dalloc<float>(img(N, 32));
    N.g[1] = c->dalloc<float>(img(N, 32));
    N.partials = c->dalloc<float>((size_t)conv_dw_blocks(N.H, N.W) * 32 * conv_kp(32));
    N.fdiff = c->dalloc<float>(2 * c->m.nb + 1);
    N.train_ready = true;
}

void nn_pack(ibpm_ctx *c) {
    NNState &N = c->nn;
    for (int l = 0; l < kNNLayers; ++l)
        launch_pack_weights(c->stream, N.cin[l], 32, N.master[l], N.fwd[l], N.bwd[l]);
}

// real channel counts of layer l (the stored tensors are padded)
int nn_cin_real(int l) { return l == 0 ? kNNIn : kNNWidth; }
int nn_cout_real(int l) { return l == kNNLayers - 1 ? kNNOut : kNNWidth; }
int64_t nn_param_count() {
    int64_t n = 0;
    for (int l = 0; l < kNNLayers; ++l) n += (int64_t)nn_cout_real(l) * nn_cin_real(l) * 9;
    return n;
}

// weights given as [out][in][3][3] per layer (layers concatenated) <-> master [32][kp]
void nn_set_master(ibpm_ctx *c, const float *pt) {
    NNState &N = c->nn;
    int64_t off = 0;
    for (int l = 0; l < kNNLayers; ++l) {
        std::vector<float> mst((size_t)32 * N.kp[l], 0.0f);
        int ci = nn_cin_real(l), co = nn_cout_real(l);
        for (int o = 0; o < co; ++o)
            for (int cc = 0; cc < ci; ++cc)
                for (int t = 0; t < 9; ++t) mst[(size_t)o * N.kp[l] + t * N.cin[l] + cc] = pt[off + ((int64_t)o * ci + cc) * 9 + t];
        off += (int64_t)co * ci * 9;
        HIPCHECK(hipMemcpyAsync(N.master[l], mst.data(), mst.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
        HIPCHECK(hipStreamSynchronize(c->stream));
    }
    nn_pack(c);
    N.adam_t = 0;
    if (N.train_ready)
        for (int l = 0; l < kNNLayers; ++l) {
            size_t np = (size_t)32 * N.kp[l];
            HIPCHECK(hipMemsetAsync(N.m[l], 0, np * sizeof(float), c->stream));
            HIPCHECK(hipMemsetAsync(N.v[l], 0, np * sizeof(float), c->stream));
        }
}

void nn_get_master(ibpm_ctx *c, float *pt) {
    NNState &N = c->nn;
    int64_t off = 0;
    for (int l = 0; l < kNNLayers; ++l) {
        std::vector<float> mst((size_t)32 * N.kp[l]);
        HIPCHECK(hipMemcpyAsync(mst.data(), N.master[l], mst.size() * sizeof(float), hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(hipStreamSynchronize(c->stream));
        int ci = nn_cin_real(l), co = nn_cout_real(l);
        for (int o = 0; o < co; ++o)
            for (int cc = 0; cc < ci; ++cc)
                for (int t = 0; t < 9; ++t) pt[off + ((int64_t)o * ci + cc) * 9 + t] = mst[(size_t)o * N.kp[l] + t * N.cin[l] + cc];
        off += (int64_t)co * ci * 9;
    }
}

// He-normal initial weights from a counter-based generator (splitmix64 +
// Box-Muller), so an initialisation is reproducible from its seed
void nn_init_weights(ibpm_ctx *c, uint64_t seed) {
    std::vector<float> pt((size_t)nn_param_count());
    uint64_t ctr = 0;
    auto next = [&]() {
        uint64_t z = (seed + 0x9e3779b97f4a7c15ULL * (++ctr));
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        z ^= z >> 31;
        return ((z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    };
    int64_t off = 0;
    for (int l = 0; l < kNNLayers; ++l) {
        int ci = nn_cin_real(l), co = nn_cout_real(l);
        double sd = std::sqrt(2.0 / (9.0 * ci));
        for (int64_t k = 0; k < (int64_t)co * ci * 9; ++k) {
            double u1 = next(), u2 = next();
            pt[off + k] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
        }
        off += (int64_t)co * ci * 9;
    }
    nn_set_master(c, pt.data());
}

// forward pass from the features in act[0]; the output goes to y32, ys
// channels per cell (32 for training, whose gradient takes every channel;
// kOutRow at inference, where only the kNNOut output channels are read)
constexpr int kOutRow = 4;
void nn_forward(ibpm_ctx *c, int ys = 32) {
    NNState &N = c->nn;
    hipStream_t s = c->stream;
    for (int l = 0; l < kNNLayers; ++l) {
        const bool last = l == kNNLayers - 1;
        float *y32 = last ? N.y32 : nullptr;
        bf16 *y16 = last ? nullptr : N.act[l + 1];
        if (N.cin[l] == kNNInPad)
            launch_conv3x3<bf16, kNNInPad>(s, N.H, N.W, N.act[l], nullptr, N.fwd[l], y32, y16, last ? 0 : 1, ys);
        else
            launch_conv3x3<bf16, 32>(s, N.H, N.W, N.act[l], nullptr, N.fwd[l], y32, y16, last ? 0 : 1, ys);
    }
}

// e = correction for the residual r (lambda layout): scale, features,
// network, output (pressure and interpolated forces) times scale / dt
template <class T>
void nn_apply(ibpm_ctx *c, const T *r, T *e) {
    NNState &N = c->nn;
    hipStream_t s = c->stream;
    const Model &m = c->m;
    launch_nn_scale(s, c->p64.K0.n, r, N.sparts, N.scale);
    launch_nn_features(s, c->g, m.nb, r, (const double *)N.scale, N.inv_hmin, N.cd, N.act[0]);
    nn_forward(c, kOutRow);
    launch_nn_output(s, (int)m.g.n_cell, m.nb, N.y32, N.scale, 1.0 / c->prm.dt, N.cd, e, kOutRow);
}

// loss of one (residual, error) pair and its gradient, added to N.grad;
// the loss value is copied to the device double `loss`
void nn_sample_grad(ibpm_ctx *c, const float *r, const float *t, double *loss) {
    NNState &N = c->nn;
    hipStream_t s = c->stream;
    const Model &m = c->m;
    const int n = c->p64.K0.n;
    launch_nn_scale(s, n, r, N.sparts, N.scale);
    launch_nn_features(s, c->g, m.nb, r, (const double *)N.scale, N.inv_hmin, N.cd, N.act[0]);
    nn_forward(c);
    launch_nn_energy_loss(s, c->p64.K0, m.nb, N.y32, r, t, N.scale, c->prm.dt, N.cd, N.d, N.z0,
                          N.g[0], c->parts, N.st);
    HIPCHECK(hipMemcpyAsync(loss, &N.st->rr, sizeof(double), hipMemcpyDeviceToDevice, s));
    int cur = 0;
    for (int l = kNNLayers - 1; l >= 0; --l) {
        // the ReLU derivative of this layer's output masks the incoming gradient
        const bf16 *mask = (l == kNNLayers - 1) ? nullptr : N.act[l + 1];
        const int blocks = conv_dw_blocks(N.H, N.W);
        if (N.cin[l] == kNNInPad)
            launch_conv3x3_dw<kNNInPad>(s, N.H, N.W, N.act[l], N.g[cur], mask, N.partials);
        else
            launch_conv3x3_dw<32>(s, N.H, N.W, N.act[l], N.g[cur], mask, N.partials);
        launch_dw_reduce(s, blocks, 32 * N.kp[l], N.partials, N.grad[l]);
        if (l > 0) {
            launch_conv3x3<float, 32>(s, N.H, N.W, N.g[cur], mask, N.bwd[l], N.g[1 - cur], nullptr, 0);
            cur = 1 - cur;
        }
    }
}

// master-layout [32][kp] gradients -> [out][in][3][3] per layer (host)
void nn_get_grads(ibpm_ctx *c, float *pt) {
    NNState &N = c->nn;
    int64_t off = 0;
    for (int l = 0; l < kNNLayers; ++l) {
        std::vector<float> g((size_t)32 * N.kp[l]);
        HIPCHECK(hipMemcpyAsync(g.data(), N.grad[l], g.size() * sizeof(float), hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(hipStreamSynchronize(c->stream));
        int ci = nn_cin_real(l), co = nn_cout_real(l);
        for (int o = 0; o < co; ++o)
            for (int cc = 0; cc < ci; ++cc)
                for (int t = 0; t < 9; ++t) pt[off + ((int64_t)o * ci + cc) * 9 + t] = g[(size_t)o * N.kp[l] + t * N.cin[l] + cc];
        off += (int64_t)co * ci * 9;
    }
}

// one training pass over `order` (indices into the sample set) in batches
double nn_train(ibpm_ctx *c, const float *r1, const float *e1, int S, const int32_t *order,
                int nord, int batch, float lr) {
    NNState &N = c->nn;
    nn_alloc_training(c);
    hipStream_t s = c->stream;
    const Model &m = c->m;
    const int n = c->p64.K0.n;
    if (N.max_losses < nord) {
        N.losses = c->dalloc<double>(nord);
        N.max_losses = nord;
    }
    for (int b0 = 0; b0 < nord; b0 += batch) {
        const int b1 = std::min(nord, b0 + batch);
        for (int l = 0; l < kNNLayers; ++l)
            HIPCHECK(hipMemsetAsync(N.grad[l], 0, (size_t)32 * N.kp[l] * sizeof(float), s));
        for (int q = b0; q < b1; ++q) {
            const int idx = order[q];
            if (idx < 0 || idx >= S) throw InvalidArg("sample index out of range");
            nn_sample_grad(c, r1 + (size_t)idx * n, e1 + (size_t)idx * n, N.losses + q);
        }
        // Adam on the summed batch gradient (its step does not depend on the
        // gradient's scale, so the sum serves as well as the mean)
        N.adam_t += 1;
        for (int l = 0; l < kNNLayers; ++l)
            launch_adam(s, 32 * N.kp[l], N.master[l], N.grad[l], N.m[l], N.v[l], N.adam_t, lr, 0.9f,
                        0.999f, 1e-8f);
        nn_pack(c);
    }
    std::vector<double> h(nord);
    HIPCHECK(hipMemcpyAsync(h.data(), N.losses, nord * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    double mean = 0;
    for (double v : h) mean += v;
    return nord ? mean / nord : 0.0;
}

// Flexible CG (one-term recurrence) with the preconditioner
//   M(r) = z0 + w d,  z0 = V(r),  r1 = r - K z0,  d = network(r1),
//   w = (d . r1) / (d . K d)  (energy-optimal; 0 if the direction is useless)
// in precision T (the V-cycle, K and the vectors; the network runs in BF16
// with FP32 accumulation either way).
template <class T> struct LearnedVecs { T *d, *r1, *z0; };
LearnedVecs<double> learned_vecs(NNState &N, double *) { return {N.d, N.r1, N.z0}; }
LearnedVecs<float> learned_vecs(NNState &N, float *) { return {N.d32, N.r132, N.z032}; }

template <class T>
void learned_precond(ibpm_ctx *c, PrecSet<T> &P, const T *r, T *z, SolveStatus *st) {
    NNState &N = c->nn;
    hipStream_t s = c->stream;
    LearnedVecs<T> w = learned_vecs(N, (T *)nullptr);
    enqueue_vcycle(c, P, r, w.z0, st, false);
    launch_k0_residual(s, P.K0, r, (const T *)w.z0, w.r1, st);
    nn_apply<T>(c, (const T *)w.r1, w.d);
    launch_kd_omega<T>(s, P.K0, w.d, w.r1, N.st, c->parts, st);
    launch_axpy_omega<T>(s, P.K0.n, w.z0, w.d, N.st, z, st);
}

// Learned initial guess for K x = b from x: x += w N(b - K x) with the
// energy-optimal w (x unchanged when w = 0).  FP64.
void learned_guess(ibpm_ctx *c, const double *b, double *x, SolveStatus *st) {
    NNState &N = c->nn;
    hipStream_t s = c->stream;
    PrecSet<double> &P = c->p64;
    // a status that stays running (tolerance 0) so the predicated kernels act
    launch_pcg_init(s, P.K0, b, (const double *)x, N.r1, (double *)nullptr, st, c->parts, false, 0.0, 1);
    nn_apply<double>(c, (const double *)N.r1, N.d);
    launch_kd_omega<double>(s, P.K0, N.d, N.r1, N.st, c->parts, st);
    launch_axpy_omega<double>(s, P.K0.n, (const double *)x, N.d, N.st, x, st);
}

// The flexible-CG loop (iterations queued in predicated chunks as in
// pcg_drive).  Returns the host copy of the final status; *stall is set when
// ||r|| has not fallen 5 % below its value at the last such fall for at
// least 16 iterations (the residual 2-norm of CG is not monotone, so one
// short flat stretch is no stall).
FcgStore<double> &fcg_store(ibpm_ctx *c, double *);
FcgStore<float> &fcg_store(ibpm_ctx *c, float *);

template <class T>
FcgStore<T> &fcg_ring(ibpm_ctx *c, int m, int n) {
    FcgStore<T> &F = fcg_store(c, (T *)nullptr);
    for (int j = F.m; j < m; ++j) {
        F.P.v[j] = c->dalloc<T>(n);
        F.Q.v[j] = c->dalloc<T>(n);
    }
    if (m > F.m) F.m = m;
    return F;
}

template <class T>
SolveStatus fcg_learned_drive(ibpm_ctx *c, PrecSet<T> &P, const T *b, T *x, SolveStatus *st,
                              double rtol, int maxit, int &est, bool zero_guess, bool *stall) {
    hipStream_t s = c->stream;
    const K0T<T> &K = P.K0;
    const int n = K.n;
    const int m = std::min(kFcgMax, c->prm.fcg_depth > 0 ? c->prm.fcg_depth : 4);
    FcgStore<T> &F = fcg_ring<T>(c, m, n);
    if (!c->fcg_ring) c->fcg_ring = c->dalloc<FcgRing>(1);
    FcgRing *ring = c->fcg_ring;
    if (zero_guess) launch_pcg_init_zero(s, n, b, x, P.r, st, c->parts, rtol * rtol, maxit);
    else launch_pcg_init(s, K, b, (const T *)x, P.r, (T *)nullptr, st, c->parts, false, rtol * rtol, maxit);
    // the network runs on every `every`-th preconditioner application, the
    // plain V-cycle on the others (flexible CG allows the change)
    const int every = std::max(1, c->prm.learned_every);
    long napp = 0;
    auto precond = [&](const T *r, T *z) {
        if (napp++ % every == 0) learned_precond<T>(c, P, r, z, st);
        else enqueue_vcycle(c, P, r, z, st, false);
    };
    long k = 0;   // iterations queued so far (direction k goes to slot k % m)
    auto iteration = [&]() {
        precond(P.r, P.z);
        const int cnt = (int)std::min<long>(k, m);
        FcgSlots sl{};
        for (int j = 0; j < cnt; ++j) sl.s[j] = (int)((k - cnt + j) % m);
        launch_fcg_betas<T>(s, n, P.z, F.Q, cnt, sl, ring, st, c->parts);
        const int slot = (int)(k % m);
        launch_fcg_direction<T>(s, n, P.z, F.P, cnt, sl, ring, F.P.v[slot], st);
        launch_fcg_product<T>(s, K, F.P.v[slot], F.Q.v[slot], P.r, slot, ring, st, c->parts);
        launch_pcg_update(s, K, x, P.r, (T *)nullptr, (const T *)F.P.v[slot], (const T *)F.Q.v[slot],
                          st, (const double *)nullptr, c->parts, false, false);
        ++k;
    };
    int chunk = std::max(1, (int)(0.8 * est)), queued = 0;
    double last_rr = -1, mark_rr = -1;
    int last_it = 0, mark_it = 0;
    const double fall = c->prm.fcg_stall_fall > 0 ? c->prm.fcg_stall_fall : 0.05;
    const double keep2 = (1.0 - fall) * (1.0 - fall);   // rr is the squared norm
    *stall = false;
    for (;;) {
        for (int i = 0; i < chunk; ++i) iteration();
        queued += chunk;
        c->read_status(st);
        const SolveStatus &h = *c->host_st;
        if (h.done != ST_RUNNING || queued > maxit + 1) break;
        // stall: 16 or more iterations since ||r|| last fell by `fall` below the mark
        if (mark_rr < 0 || h.rr < keep2 * mark_rr) {
            mark_rr = h.rr;
            mark_it = h.iter;
        } else if (h.iter - mark_it >= 16) {
            *stall = true;
            break;
        }
        int rem = 8;
        if (last_rr > 0 && h.iter > last_it && h.rr < last_rr) {
            double rate = std::log(h.rr / last_rr) / (h.iter - last_it);
            double need = std::log(h.tol2 * h.bb / h.rr);
            if (rate < 0) rem = (int)std::ceil(need / rate);
        }
        last_rr = h.rr;
        last_it = h.iter;
        chunk = std::min(std::max(rem, 8), 64);
    }
    if (c->host_st->iter > 0 && !*stall) est = c->host_st->iter;
    return *c->host_st;
}

int solve_poisson_learned(ibpm_ctx *c, const double *rhs, double *lam, ibpm_solve_stats *out) {
    if (!c->nn.ready) throw InvalidArg("the learned solver needs network weights (ibpm_nn_init or ibpm_nn_set_weights)");
    hipStream_t s = c->stream;
    auto t0 = std::chrono::steady_clock::now();
    PrecSet<double> &P = c->p64;
    const K0View &K = P.K0;
    const int n = K.n;
    SolveStatus *st = c->st_poi;
    learned_guess(c, rhs, lam, st);
    bool stall = false;
    SolveStatus h = fcg_learned_drive<double>(c, P, rhs, lam, st, c->prm.poisson_rtol,
                                              c->prm.poisson_maxit, c->est_poi, false, &stall);
    const int fcg_iters = h.iter;
    const bool nan = h.done == ST_NAN;
    int code = IBPM_OK, fallbacks = 0;
    ibpm_solve_stats fb{};
    if (stall || nan) {
        // plain AMG-PCG from the current iterate (from zero if it is not finite)
        if (nan) HIPCHECK(hipMemsetAsync(lam, 0, n * sizeof(double), s));
        fallbacks = 1;
        code = solve_poisson_fp64(c, rhs, lam, &fb);
    } else {
        launch_zero_if_zero_rhs(s, lam, n, st);
        launch_true_residual(s, K, rhs, (const double *)lam, st, c->parts);
        c->read_status(st);
        const SolveStatus &hh = *c->host_st;
        if (hh.done == ST_MAXIT || hh.done == ST_RUNNING) code = IBPM_ENOTCONV;
        fb.relres = hh.bb > 0 ? std::sqrt(hh.true_rr / hh.bb) : 0.0;
    }
    auto t1 = std::chrono::steady_clock::now();
    if (out) {
        out->iters = fcg_iters + fb.iters;
        out->status = code;
        out->relres = fb.relres;
        out->ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        out->outer_iters = 1;
        out->fallbacks = fallbacks;
    }
    if (code == IBPM_ENOTCONV && c->err.empty()) c->err = "iteration limit reached";
    return code;
}

// FP64 CG (product, update, dot products and the iterate in FP64) with the
// V-cycle in FP32: r is rounded to FP32, the FP32 cycle gives z32, and z is
// its FP64 value, so the preconditioner is a fixed linear map
int solve_poisson_mixed_precond(ibpm_ctx *c, const double *rhs, double *lam, ibpm_solve_stats *out) {
    PrecSet<double> &P = c->p64;
    const int n = P.K0.n;
    if (c->guess_learned) {
        if (!c->nn.ready) throw InvalidArg("the learned initial guess needs network weights (ibpm_nn_init or ibpm_nn_set_weights)");
        learned_guess(c, rhs, lam, c->st_poi);
    }
    // the residual goes to FP32 on entry to the cycle and the cycle's result
    // back to FP64 in its last sweep (with r . z); in the iterations the
    // FP64 update is folded into the FP32 first pass
    std::function<void(const double *, double *)> pre = [c, n](const double *r, double *z) {
        launch_to_f32(c->stream, n, r, c->rin32, c->st_poi);
        const MixedIO mx{nullptr, r, z, c->rin32};
        enqueue_vcycle(c, c->p32, (const float *)c->rin32, c->d32, c->st_poi, false, (const UpdArgs<float> *)nullptr, &mx);
    };
    FusedPre<double> fpre{[c](const UpdArgs<double> &u, double *z) {
                              const MixedIO mx{&u, u.r_out, z, c->rin32};
                              enqueue_vcycle(c, c->p32, (const float *)c->rin32, c->d32, c->st_poi, false,
                                             (const UpdArgs<float> *)nullptr, &mx);
                          },
                          P.r2, walk_blocks_of(P.K0), walk_blocks_of(P.K0)};
    const bool can_fuse = c->p32.lev.size() > 1 && c->prm.amg_pre >= 2;
    return pcg_drive<K0View, double>(c, P.K0, n, false, pre, rhs, lam, P.r, P.z, P.p, P.q,
                                     c->st_poi, c->prm.poisson_rtol, c->prm.poisson_maxit,
                                     c->est_poi, false, true, out, 1, can_fuse ? &fpre : nullptr);
}

int solve_poisson_impl(ibpm_ctx *c, const double *rhs, double *lam, ibpm_solve_stats *out) {
    if (c->mixed_precond) return solve_poisson_mixed_precond(c, rhs, lam, out);
    if (c->mixed) return solve_poisson_mixed(c, rhs, lam, out);
    if (c->learned) return solve_poisson_learned(c, rhs, lam, out);
    return solve_poisson_fp64(c, rhs, lam, out);
}

int solve_velocity_impl(ibpm_ctx *c, const double *rhs, double *q, ibpm_solve_stats *out) {
    std::function<void(const double *, double *)> none;
    return pcg_drive<AView, double>(c, c->A, c->g.n_q, true, none, rhs, q, c->vr, c->vz, c->vp,
                                    c->vq, c->st_vel, c->prm.vel_rtol, c->prm.vel_maxit, c->est_vel,
                                    false, true, out, 0);
}

void stage_walls(ibpm_ctx *c, const double *q) {
    double uconv = c->prm.uinf * std::cos(c->prm.alpha);
    launch_walls_update(c->stream, c->g, c->walls[c->cur], c->walls[1 - c->cur], q, c->convective,
                        uconv, c->prm.dt, c->ly);
}

void stage_rhs1(ibpm_ctx *c, const double *q, const double *conv_prev, double *r1,
                double *conv_now) {
    launch_momentum_rhs(c->stream, c->g, q, conv_prev, conv_now, r1, c->walls[c->cur],
                        c->walls[1 - c->cur], c->prm.nu, c->prm.dt, c->step == 0 ? 1 : 0);
}

// share of the prescribed body velocity at the time the current step
// advances to (the start-up ramp of ibpm_params.body_ramp)
double body_velocity_scale(const ibpm_ctx *c) {
    const double T = c->prm.body_ramp;
    if (!(T > 0)) return 1.0;
    const double t = (double)(c->step + 1) * c->prm.dt;
    if (t >= T) return 1.0;
    const double sn = std::sin(0.5 * M_PI * t / T);
    return sn * sn;
}

void stage_rhs2(ibpm_ctx *c, const double *qstar, double *rhs) {
    launch_poisson_rhs(c->stream, c->g, c->m.nb, c->m.pin, qstar, c->walls[1 - c->cur], c->E.view(), c->ub,
                       body_velocity_scale(c), rhs);
}

void stage_project(ibpm_ctx *c, const double *qstar, const double *lam, double *qout) {
    const Model &m = c->m;
    if (c->moving) {
        launch_project_moving(c->stream, c->g, c->prm.dt, m.nb, c->ecol, c->eval, c->box[0], c->box[1],
                              c->box[2], c->box[3], c->xf_d, c->yf_d, c->xb_d, c->yb_d, qstar, lam, qout);
        launch_forces(c->stream, (int)m.g.n_cell, m.nb, lam, c->st_misc);
        return;
    }
    if (c->bn > 1) {
        // q = q* - B^N (Q lambda) as a pair of sparse products (Sec. 4)
        launch_csr_gemv(c->stream, c->Qd.view(), lam, -1.0, nullptr, c->wq);
        launch_csr_gemv(c->stream, c->Bn.view(), c->wq, 1.0, qstar, qout);
        launch_forces(c->stream, (int)m.g.n_cell, m.nb, lam, c->st_misc);
        return;
    }
    launch_project(c->stream, c->g, c->prm.dt, m.nb, qstar, lam, qout, c->Etu.view(), m.fu_i0,
                   m.fu_i1, m.fu_j0, m.fu_j1, c->Etv.view(), m.fv_i0, m.fv_i1, m.fv_j0, m.fv_j1);
    launch_forces(c->stream, (int)m.g.n_cell, m.nb, lam, c->st_misc);
}

// Wall velocities at the start from the wall kinds: a Dirichlet side keeps
// (bc_u, bc_v), the convective right side starts at the freestream.  Without
// a convective wall nothing can balance the wall fluxes, so the Dirichlet
// walls must carry zero net flux (else the pinned system has no solution).
void set_walls_spec(ibpm_ctx *c, const GridMetrics &G) {
    const ibpm_params &p = c->prm;
    const double U = p.uinf * std::cos(p.alpha), V = p.uinf * std::sin(p.alpha);
    c->convective = 0;
    for (int side = 0; side < 4; ++side) {
        if (p.bc_kind[side] == IBPM_BC_CONVECTIVE) {
            c->convective = 1;
            c->wall_init.u[side] = U;
            c->wall_init.v[side] = V;
        } else {
            c->wall_init.u[side] = p.bc_u[side];
            c->wall_init.v[side] = p.bc_v[side];
        }
    }
    if (!c->convective) {
        const double lx = G.xf[G.nx] - G.xf[0], ly = G.yf[G.ny] - G.yf[0];
        const WallSides &w = c->wall_init;
        const double net = (w.u[1] - w.u[0]) * ly + (w.v[3] - w.v[2]) * lx;
        const double scale = (std::fabs(w.u[1]) + std::fabs(w.u[0])) * ly +
                             (std::fabs(w.v[3]) + std::fabs(w.v[2])) * lx;
        if (std::fabs(net) > 1e-12 * scale)
            throw InvalidArg("Dirichlet walls (bc_u, bc_v) must carry zero net flux when no wall is convective");
    }
}

void check_params(const ibpm_params *p) {
    if (!p) throw InvalidArg("params is NULL");
    // N = 2 is left out: B^2 = B^1 (I + S) is indefinite wherever (nu dt / 2) rho(L Mf^-1) > 1
    // (already on the 512^2 grid), while 1 + s + s^2 > 0 keeps B^3 positive definite
    if (p->bn_order != 1 && p->bn_order != 3) throw InvalidArg("bn_order must be 1 or 3 (B^1 or B^3)");
    if (p->bn_order > 1 && p->poisson_solver != IBPM_SOLVER_JACOBI_PCG && p->poisson_solver != IBPM_SOLVER_AMG_PCG)
        throw InvalidArg("B^N with N > 1 supports the Jacobi-PCG and AMG-PCG Poisson solvers only");
    if (!(p->vel_rtol > 0) || !(p->poisson_rtol > 0)) throw InvalidArg("tolerances must be > 0");
    if (p->vel_maxit < 1 || p->poisson_maxit < 1) throw InvalidArg("maxit must be >= 1");
    if (p->poisson_solver < IBPM_SOLVER_JACOBI_PCG || p->poisson_solver > IBPM_SOLVER_AMG_PCG_FP32_CYCLE_GUESS)
        throw InvalidArg("unknown Poisson solver");
    if (!(p->inner_rtol >= 0) || p->inner_rtol >= 1) throw InvalidArg("inner_rtol must be in [0, 1)");
    if (p->learned_every < 0) throw InvalidArg("learned_every must be >= 0");
    if (p->fcg_depth < 0 || p->fcg_depth > kFcgMax) throw InvalidArg("fcg_depth must be in [0, 8]");
    if (p->fuse_transfers != 0 && p->fuse_transfers != 1) throw InvalidArg("fuse_transfers must be 0 or 1");
    if (!(p->fcg_stall_fall >= 0 && p->fcg_stall_fall <= 1)) throw InvalidArg("fcg_stall_fall must be in [0, 1]");
    if (!(p->body_ramp >= 0) || !std::isfinite(p->body_ramp)) throw InvalidArg("body_ramp must be finite and >= 0");
    if (p->moving_body != 0 && p->moving_body != 1) throw InvalidArg("moving_body must be 0 or 1");
    if (p->amg_rebuild_every < 0) throw InvalidArg("amg_rebuild_every must be >= 0");
    if (p->moving_body && p->nb < 1) throw InvalidArg("a moving body needs at least one point");
    if (p->moving_body && (p->bn_order != 1 || (p->poisson_solver != IBPM_SOLVER_JACOBI_PCG &&
                                                p->poisson_solver != IBPM_SOLVER_AMG_PCG)))
        throw InvalidArg("a moving body supports B^1 with the Jacobi-PCG and AMG-PCG Poisson solvers only");
    for (int side = 0; side < 4; ++side) {
        const int k = p->bc_kind[side];
        if (k != IBPM_BC_DIRICHLET && k != IBPM_BC_CONVECTIVE) throw InvalidArg("unknown wall kind (bc_kind)");
        if (k == IBPM_BC_CONVECTIVE && side != 1)
            throw InvalidArg("a convective wall (bc_kind) is supported on the right side only");
        if (k == IBPM_BC_DIRICHLET && (!std::isfinite(p->bc_u[side]) || !std::isfinite(p->bc_v[side])))
            throw InvalidArg("Dirichlet wall velocities (bc_u, bc_v) must be finite");
    }
    if (p->poisson_solver != IBPM_SOLVER_JACOBI_PCG) {
        if (p->amg_pre < 1 || p->amg_post < 1) throw InvalidArg("AMG needs >= 1 pre and post sweep");
        if (p->amg_coarse_max < 1 || p->amg_max_levels < 1) throw InvalidArg("bad AMG limits");
        if (p->amg_max_levels > kMaxLevels) throw InvalidArg("amg_max_levels too large");
        if (!(p->amg_theta >= 0)) throw InvalidArg("amg_theta must be >= 0");
    }
}

// The stored rows of level-0 K as the walker's bands take them: fixed-width
// (ELL) copies of the force rows and of the coupled cells' rows (slot q of
// a row is CSR entry q; empty slots hold column -1 and value 0), the list of
// coupled cells (box cells with at least one coupling entry) and one bit per
// box cell marking them.
struct BandHost {
    bool kf_ok = true, cc_ok = true;
    std::vector<int32_t> kf_col, cc_row, cc_col;
    std::vector<double> kf_val, cc_val;
    std::vector<uint32_t> bits;
};

BandHost make_bands(const Model &m) {
    BandHost h;
    const CSR &kf = m.Kf, &cf = m.Kcf;
    h.kf_col.assign((size_t)kKfW * kf.nrows, -1);
    h.kf_val.assign((size_t)kKfW * kf.nrows, 0.0);
    for (int r = 0; r < kf.nrows; ++r) {
        const int p0 = kf.ptr[r], len = kf.ptr[r + 1] - p0;
        if (len > kKfW) {
            h.kf_ok = false;
            continue;
        }
        for (int q = 0; q < len; ++q) {
            h.kf_col[(size_t)r * kKfW + q] = kf.col[p0 + q];
            h.kf_val[(size_t)r * kKfW + q] = kf.val[p0 + q];
        }
    }
    const int bw = m.cb_i1 - m.cb_i0 + 1;
    h.bits.assign(((size_t)cf.nrows + 31) / 32, 0u);
    for (int rb = 0; rb < cf.nrows; ++rb) {
        const int p0 = cf.ptr[rb], len = cf.ptr[rb + 1] - p0;
        if (len == 0) continue;
        h.bits[rb >> 5] |= 1u << (rb & 31);
        const int q = (int)h.cc_row.size();
        h.cc_row.push_back((m.cb_j0 + rb / bw) * m.g.nx + (m.cb_i0 + rb % bw));
        h.cc_col.resize((size_t)(q + 1) * kCcW, -1);
        h.cc_val.resize((size_t)(q + 1) * kCcW, 0.0);
        if (len > kCcW) {
            h.cc_ok = false;
            continue;
        }
        for (int k = 0; k < len; ++k) {
            h.cc_col[(size_t)q * kCcW + k] = cf.col[p0 + k];
            h.cc_val[(size_t)q * kCcW + k] = cf.val[p0 + k];
        }
    }
    return h;
}

// device copies of the band arrays in precision T (indices shared)
template <class T>
struct BandDev {
    int kf_ok = 0, cc_ok = 0, ncc = 0;
    const int32_t *kf_col = nullptr, *cc_row = nullptr, *cc_col = nullptr;
    const uint32_t *bits = nullptr;
    const T *kf_val = nullptr, *cc_val = nullptr;
};

// K0 view in precision T over device metric / coupling arrays
template <class T>
K0T<T> make_k0(const GridT<T> &g, double dt, const Model &m, const DevCSRT<T> &cf,
               const DevCSRT<T> &kf, const T *kfd, const BandDev<T> &bd) {
    K0T<T> K;
    K.g = g;
    K.dt = (T)dt;
    K.nb = m.nb;
    K.pin = m.pin;
    K.n = (int)m.g.n_cell + 2 * m.nb;
    K.cb_i0 = m.cb_i0; K.cb_i1 = m.cb_i1; K.cb_j0 = m.cb_j0; K.cb_j1 = m.cb_j1;
    K.cf = cf.view();
    K.kf = kf.view();
    K.kf_diag = kfd;
    K.kf_ell = bd.kf_ok;
    K.kfe_col = bd.kf_col;
    K.kfe_val = bd.kf_val;
    K.ncc = bd.ncc;
    K.cc_ell = bd.cc_ok;
    K.cc_row = bd.cc_row;
    K.cc_bits = bd.bits;
    K.cce_col = bd.cc_col;
    K.cce_val = bd.cc_val;
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

// First level of the dense coarse cycle: the first level below level 0 with
// at most `rows` unknowns (the coarsest if none)
int dense_level(const Hierarchy &h, int rows) {
    const int L = (int)h.levels.size();
    for (int l = 1; l < L; ++l)
        if (h.levels[l].A.nrows <= rows) return l;
    return L - 1;
}

// Where a V-cycle kernel is bound by launch and memory latency rather than
// by bandwidth, two launches per level are saved with products formed once:
//   restriction  b_{l+1} = R (b - A x) = R b - (R A) x   (one gather kernel)
//   prolongation and first post-sweep
//     x'' = x + P e + W (b - A x - (A P) e)             (one gather kernel)
// R A is formed on every CSR level, where it holds fewer entries than A, and
// on level 0 (whose K is applied matrix-free, so R A adds stored entries)
// only up to kFuseRows0 unknowns; A P adds entries to the sweep and is
// formed up to kFuseRowsP unknowns.  R A is dropped where a row of R and R A
// together would not fit the row-block kernels' LDS buffer (the 3-D levels
// whose coarse rows gather thousands of entries): there one wave per row
// took 36 us where the residual in row blocks and R take 20.
constexpr int kFuseRows0 = 600000;
constexpr int kFuseRowsP = 200000;

void fused_transfer_products(Hierarchy &h) {
    const int L = (int)h.levels.size();
    if (L < 2) return;
    const int lc = dense_level(h, kCoarseRows);
    for (int l = 0; l < lc; ++l) {
        Level &lv = h.levels[l];
        if (l > 0 || lv.A.nrows <= kFuseRows0) {
            lv.RA = csr_multiply(lv.R, lv.A);
            bool fits = true;
            for (int32_t r = 0; r < lv.R.nrows && fits; ++r)
                fits = (lv.R.ptr[r + 1] - lv.R.ptr[r]) + (lv.RA.ptr[r + 1] - lv.RA.ptr[r]) <= kStreamCap;
            if (!fits) lv.RA = CSR();
        }
        if (l > 0 && lv.A.nrows <= kFuseRowsP) lv.AP = csr_multiply(lv.A, lv.P);
    }
}

// Upload the hierarchy in precision T (values converted from FP64)
// Row blocks of the row-block CSR kernels for the matrices one kernel walks
// together.  The plain partition takes rpb rows per block, rpb the largest
// power of two up to kBlock for which every block's entries (in all the
// matrices) fit kStreamCap.  Where a few long rows force rpb far below what
// the other rows allow (the force rows of the three-dimensional K: 16 rows
// per block where 256 cell rows fit), the blocks are formed greedily
// instead: runs of at most kBlock rows whose entries fit kStreamCap, each
// as long as that allows; this is taken when it needs under half the
// blocks (on the 96^3 K it halved the time of a solve; runs of at most 64
// rows gained only half as much).  Returns the plain rows per block (and no
// row starts: the kernels form them) or the greedy row starts (rpb 0).
// Empty when a single row does not fit (then the row-vector kernels run),
// or when IBPM_CSR_STREAM=0 selects the row-vector kernels everywhere.
std::vector<int32_t> stream_blocks_of(std::initializer_list<const CSR *> ms, int &rpb_out) {
    static const bool off = [] {
        const char *e = std::getenv("IBPM_CSR_STREAM");
        return e && e[0] == '0';
    }();
    std::vector<int32_t> bst;
    rpb_out = 0;
    if (off || ms.size() == 0) return bst;
    const int n = (*ms.begin())->nrows;
    for (const CSR *m : ms)
        if (m->nrows != n || (int)m->ptr.size() != n + 1) return bst;
    auto entries = [&](int r0, int r1) {
        int64_t tot = 0;
        for (const CSR *m : ms) tot += m->ptr[r1] - m->ptr[r0];
        return tot;
    };
    int rpb = 0;
    for (int r = kBlock; r >= 1 && rpb == 0; r /= 2) {
        bool ok = true;
        for (int r0 = 0; r0 < n && ok; r0 += r) ok = entries(r0, std::min(r0 + r, n)) <= kStreamCap;
        if (ok) rpb = r;
    }
    if (rpb == 0) return bst;
    std::vector<int32_t> greedy{0};
    for (int r0 = 0; r0 < n;) {
        int r1 = r0;
        while (r1 < n && r1 - r0 < kBlock && entries(r0, r1 + 1) <= kStreamCap) ++r1;
        greedy.push_back(r1);
        r0 = r1;
    }
    const int64_t plain = n > 0 ? ((int64_t)n + rpb - 1) / rpb : 1;
    if (n > 0 && 2 * ((int64_t)greedy.size() - 1) < plain) return greedy;
    rpb_out = rpb;
    return bst;
}

// Give a device matrix the row-block shape for the matrices its kernels
// walk (lanes = -1 and its row blocks), or keep its row-vector lanes.
template <class T>
void set_stream_shape(ibpm_ctx *c, DevCSRT<T> &d, std::initializer_list<const CSR *> ms) {
    int rpb = 0;
    std::vector<int32_t> bst = stream_blocks_of(ms, rpb);
    if (rpb > 0) {
        const int64_t nb = std::max<int64_t>(1, ((int64_t)d.nrows + rpb - 1) / rpb);
        if (nb > kMaxParts) return;
        d.rpb = rpb;
        d.nblk = (int)nb;
    } else {
        if (bst.empty() || (int64_t)bst.size() - 1 > kMaxParts) return;
        d.bst = c->upload(bst);
        d.nblk = (int)bst.size() - 1;
    }
    d.lanes = -1;
}

template <class T>
void upload_levels(ibpm_ctx *c, PrecSet<T> &P) {
    int L = (int)c->h.levels.size();
    P.lev.resize(L);
    for (int l = 0; l < L; ++l) {
        const Level &hl = c->h.levels[l];
        DevLevelT<T> &dl = P.lev[l];
        dl.n = hl.A.nrows;
        dl.omega = hl.omega;
        const bool stored = l > 0 || c->stored0;   // level 0 is matrix-free for a fixed body and B^1
        if (stored) {
            bool shared = false;
            if constexpr (std::is_same<T, double>::value) {
                if (l == 0 && c->stored0) {
                    dl.A = c->K0c;   // the finest operator is the stored K, uploaded once
                    shared = true;
                }
            }
            if (!shared) dl.A = c->upload_csr<T>(hl.A);
            dl.wdinv = c->upload(std::vector<T>(hl.wdinv.begin(), hl.wdinv.end()));
            if (l > 0) dl.b = c->dalloc<T>(dl.n);
        } else {
            // level 0 is matrix-free; its smoother weights omega / k_ii are
            // formed on the device from the same stencil, and its prolongator
            // is applied from the aggregates and the stencil
            dl.wdinv = c->dalloc<T>(dl.n);
            launch_k0_wdinv(c->stream, P.K0, hl.omega, dl.wdinv);
            if (L > 1) {
                dl.agg = c->upload(hl.agg);
                dl.pomega = hl.pomega;
            }
        }
        if (l < L - 1) {
            // level 0 applies its prolongator matrix-free (aggregates + stencil)
            if (stored) dl.P = c->upload_csr<T>(hl.P);
            dl.R = c->upload_csr<T>(hl.R);
            dl.r = c->dalloc<T>(dl.n);
            if (hl.RA.nrows > 0) dl.RA = c->upload_csr<T>(hl.RA);
            if (hl.AP.nrows > 0) dl.AP = c->upload_csr<T>(hl.AP);
        }
        // launch shapes (the fused kernels walk their matrices together);
        // a moving body changes the rows, so its levels keep row-vector shapes
        if (c->moving) {
            dl.xa = c->dalloc<T>(dl.n);
            dl.xb = c->dalloc<T>(dl.n);
            continue;
        }
        if (dl.A.nrows > 0) set_stream_shape(c, dl.A, {&hl.A});
        if (dl.R.nrows > 0) set_stream_shape(c, dl.R, {&hl.R});
        if (dl.P.nrows > 0) set_stream_shape(c, dl.P, {&hl.P});
        if (dl.RA.nrows > 0) set_stream_shape(c, dl.RA, {&hl.R, &hl.RA});
        if (dl.AP.nrows > 0) set_stream_shape(c, dl.AP, {&hl.A, &hl.AP, &hl.P});
        dl.xa = c->dalloc<T>(dl.n);
        dl.xb = c->dalloc<T>(dl.n);
    }
    // levels from the first with at most kCoarseRows unknowns (never level 0,
    // which may be matrix-free) down to the coarsest are applied as one dense
    // product: the cycle there is a fixed linear map, formed once on the host
    P.lc = dense_level(c->h, c->moving ? kCoarseRowsMoving : kCoarseRows);
    if (c->coarse_C_lc != P.lc) {
        c->coarse_C = coarse_cycle_matrix(c->h, P.lc, c->prm.amg_pre, c->prm.amg_post);
        c->coarse_C_lc = P.lc;
    }
    if (!c->coarse_C_dev) c->coarse_C_dev = c->upload(c->coarse_C);
    P.coarseC = c->coarse_C_dev;
}

template <class T>
void alloc_pcg(ibpm_ctx *c, PrecSet<T> &P, int n) {
    P.r = c->dalloc<T>(n);
    P.z = c->dalloc<T>(n);
    P.p[0] = c->dalloc<T>(n);
    P.p[1] = c->dalloc<T>(n);
    P.q = c->dalloc<T>(n);
    P.r2 = c->dalloc<T>(n);
    for (T *v : {P.p[0], P.p[1]}) HIPCHECK(hipMemsetAsync(v, 0, n * sizeof(T), c->stream));
}

// ---------------------------------------------------------------------------
// B^N with N > 1 (Sec. 2, text after Eq. 11): B^N = B^1 (I + S + ... + S^{N-1})
// with S = (nu/2) L B^1, formed on the device by row-merge products, and
// K = Q^T B^N Q formed slice by slice (Sec. 4, triple matrix product): for a
// slice of K's rows, the faces F its rows of Q^T touch, Y_F = B^N[F, :] Q
// and then K_slice = Q^T[slice, F] Y_F; only one slice's Y_F and K_slice
// are held at a time.  K comes back to the host (the smoothed-aggregation
// set-up needs it there) and is pinned there.

constexpr int kSliceRows = 1 << 18;   // rows of K per slice

// A device CSR built by the product kernels, owned by the caller until
// free_dev_csr (temporaries) or kept (c->allocs)
struct ProdCSR {
    DevCSR m{};
    int64_t bytes = 0;
};

DevCSR upload_temp_csr(ibpm_ctx *c, const CSR &h) {
    DevCSR d;
    d.nrows = h.nrows;
    d.ncols = h.ncols;
    d.nnz = h.nnz();
    d.lanes = lanes_for(d.nnz, d.nrows);
    d.ptr = c->dtemp<int32_t>(h.ptr.size());
    d.col = c->dtemp<int32_t>(h.col.size());
    d.val = c->dtemp<double>(h.val.size());
    HIPCHECK(hipMemcpyAsync(d.ptr, h.ptr.data(), h.ptr.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    if (!h.col.empty()) {
        HIPCHECK(hipMemcpyAsync(d.col, h.col.data(), h.col.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                c->stream));
        HIPCHECK(hipMemcpyAsync(d.val, h.val.data(), h.val.size() * sizeof(double), hipMemcpyHostToDevice,
                                c->stream));
    }
    HIPCHECK(hipStreamSynchronize(c->stream));
    return d;
}

void free_temp_csr(ibpm_ctx *c, DevCSR &d) {
    c->dfree(d.ptr);
    c->dfree(d.col);
    c->dfree(d.val);
    d = DevCSR();
}

// row counts (device) -> host offsets -> device CSR arrays of the product
// rows; `fill` launches the fill kernel with the 64-bit offsets
template <class Count, class Fill>
ProdCSR product_rows(ibpm_ctx *c, int nrows, int ncols, Count count, Fill fill, bool keep) {
    hipStream_t s = c->stream;
    ProdCSR out;
    out.m.nrows = nrows;
    out.m.ncols = ncols;
    int32_t *cnt = nrows > 0 ? c->dtemp<int32_t>(nrows) : nullptr;
    int *err = c->dtemp<int>(1);
    HIPCHECK(hipMemsetAsync(err, 0, sizeof(int), s));
    count(cnt, err);
    std::vector<int32_t> h(nrows);
    int herr = 0;
    if (nrows > 0) HIPCHECK(hipMemcpyAsync(h.data(), cnt, nrows * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    c->dfree(cnt);
    c->dfree(err);
    if (herr) throw InvalidArg("a row of a B^N product has more than 32 left entries");
    std::vector<int64_t> off(nrows + 1, 0);
    for (int i = 0; i < nrows; ++i) off[i + 1] = off[i] + h[i];
    const int64_t nnz = off[nrows];
    if (nnz >= INT32_MAX) throw InvalidArg("a B^N product has more than 2^31 entries");
    std::vector<int32_t> p32(off.begin(), off.end());
    int64_t *off_d = c->dtemp<int64_t>(nrows + 1);
    HIPCHECK(hipMemcpyAsync(off_d, off.data(), (nrows + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    int32_t *ptr = keep ? c->dalloc<int32_t>(nrows + 1) : c->dtemp<int32_t>(nrows + 1);
    int32_t *col = keep ? c->dalloc<int32_t>(nnz) : c->dtemp<int32_t>(nnz);
    double *val = keep ? c->dalloc<double>(nnz) : c->dtemp<double>(nnz);
    HIPCHECK(hipMemcpyAsync(ptr, p32.data(), (nrows + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    fill(off_d, col, val);
    HIPCHECK(hipStreamSynchronize(s));
    c->dfree(off_d);
    out.m.ptr = ptr;
    out.m.col = col;
    out.m.val = val;
    out.m.nnz = nnz;
    out.m.lanes = lanes_for(nnz, nrows);
    out.bytes = 12 * nnz + 4 * (int64_t)(nrows + 1);
    return out;
}

void free_prod(ibpm_ctx *c, ProdCSR &p) {
    free_temp_csr(c, p.m);
    p = ProdCSR();
}

// C = A[rows] B (rows null: all rows of A)
ProdCSR spgemm(ibpm_ctx *c, const DevCSR &A, const int32_t *rows, int nrows, const DevCSR &B, bool keep) {
    hipStream_t s = c->stream;
    const CSRView Av = A.view(), Bv = B.view();
    return product_rows(
        c, nrows, B.ncols,
        [&](int32_t *cnt, int *err) { launch_spgemm_count(s, nrows, 0, rows, Av, Bv, cnt, err); },
        [&](const int64_t *off, int32_t *col, double *val) {
            launch_spgemm_fill(s, nrows, 0, rows, Av, Bv, off, col, val);
        },
        keep);
}

void form_bn_operators(ibpm_ctx *c) {
    Model &m = c->m;
    const ibpm_params &p = c->prm;
    hipStream_t s = c->stream;
    const GridMetrics &g = m.g;
    const int nq = (int)g.n_q, nl = (int)(g.n_cell + 2 * m.nb);
    // host: L, B^1, S = (nu/2) L B^1, Q^T and Q
    CSR S = laplacian_csr(g);
    const std::vector<double> b1 = b1_diagonal(g, p.dt);
    for (size_t k = 0; k < S.val.size(); ++k) S.val[k] = 0.5 * p.nu * S.val[k] * b1[S.col[k]];
    const CSR QT = poisson_qt(m);
    const CSR Qh = csr_transpose(QT);
    // device: B^N = B^1 (I + X + Y) with X = S and Y = S^2 (N = 3) or empty (N = 2)
    DevCSR Sd = upload_temp_csr(c, S);
    double *b1d = c->dtemp<double>(b1.size());
    HIPCHECK(hipMemcpyAsync(b1d, b1.data(), b1.size() * sizeof(double), hipMemcpyHostToDevice, s));
    ProdCSR S2;
    DevCSR Y{};
    if (p.bn_order >= 3) {
        S2 = spgemm(c, Sd, nullptr, nq, Sd, false);
        Y = S2.m;
    } else {
        Y.nrows = Y.ncols = nq;
        Y.ptr = c->dtemp<int32_t>(nq + 1);
        HIPCHECK(hipMemsetAsync(Y.ptr, 0, (nq + 1) * sizeof(int32_t), s));
    }
    const CSRView Xv = Sd.view(), Yv = Y.view();
    ProdCSR Bn = product_rows(
        c, nq, nq, [&](int32_t *cnt, int *) { launch_diag_sum_count(s, nq, Xv, Yv, cnt); },
        [&](const int64_t *off, int32_t *col, double *val) {
            launch_diag_sum_fill(s, nq, b1d, Xv, Yv, off, col, val);
        },
        true);
    if (p.bn_order >= 3) free_prod(c, S2);
    else c->dfree(Y.ptr);
    c->Bn = Bn.m;
    c->Qd = c->upload_csr<double>(Qh);
    // K = Q^T B^N Q in slices of rows
    CSR K;
    K.nrows = K.ncols = nl;
    K.ptr.assign(1, 0);
    std::vector<int32_t> local(nq, -1);
    int64_t peak = 0, unsliced_y = 0;
    std::vector<std::pair<int, int>> slices;
    for (int r0 = 0; r0 < (int)g.n_cell; r0 += kSliceRows) slices.push_back({r0, std::min<int>(r0 + kSliceRows, (int)g.n_cell)});
    if (m.nb > 0) slices.push_back({(int)g.n_cell, nl});
    for (const auto &sl : slices) {
        const int r0 = sl.first, r1 = sl.second, nr = r1 - r0;
        // the faces these rows of Q^T touch, and the rows with local columns
        std::vector<int32_t> F;
        for (int32_t q = QT.ptr[r0]; q < QT.ptr[r1]; ++q) F.push_back(QT.col[q]);
        std::sort(F.begin(), F.end());
        F.erase(std::unique(F.begin(), F.end()), F.end());
        for (size_t k = 0; k < F.size(); ++k) local[F[k]] = (int32_t)k;
        CSR QTs;
        QTs.nrows = nr;
        QTs.ncols = (int32_t)F.size();
        QTs.ptr.assign(1, 0);
        for (int r = r0; r < r1; ++r) {
            for (int32_t q = QT.ptr[r]; q < QT.ptr[r + 1]; ++q) {
                QTs.col.push_back(local[QT.col[q]]);
                QTs.val.push_back(QT.val[q]);
            }
            QTs.ptr.push_back((int32_t)QTs.col.size());
        }
        for (int32_t f : F) local[f] = -1;
        int32_t *Fd = c->dtemp<int32_t>(F.size());
        HIPCHECK(hipMemcpyAsync(Fd, F.data(), F.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        DevCSR QTd = upload_temp_csr(c, QTs);
        ProdCSR YF = spgemm(c, c->Bn, Fd, (int)F.size(), c->Qd, false);
        ProdCSR Ks = spgemm(c, QTd, nullptr, nr, YF.m, false);
        peak = std::max<int64_t>(peak, YF.bytes + Ks.bytes + 12 * QTs.nnz() + 4 * (int64_t)(F.size() + nr + 1));
        unsliced_y += YF.bytes;
        // back to the host, appended to K
        std::vector<int32_t> kp(nr + 1), kc(Ks.m.nnz);
        std::vector<double> kv(Ks.m.nnz);
        HIPCHECK(hipMemcpyAsync(kp.data(), Ks.m.ptr, (nr + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipMemcpyAsync(kc.data(), Ks.m.col, Ks.m.nnz * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipMemcpyAsync(kv.data(), Ks.m.val, Ks.m.nnz * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        const int32_t base = K.ptr.back();
        for (int i = 1; i <= nr; ++i) K.ptr.push_back(base + kp[i]);
        K.col.insert(K.col.end(), kc.begin(), kc.end());
        K.val.insert(K.val.end(), kv.begin(), kv.end());
        free_prod(c, Ks);
        free_prod(c, YF);
        free_temp_csr(c, QTd);
        c->dfree(Fd);
    }
    c->bn_peak_bytes = peak;
    c->bn_unsliced_bytes = unsliced_y;
    m.K = pin_rows_cols(K, m.pin);
    free_temp_csr(c, Sd);
    c->dfree(b1d);
}

// The V-cycle of Sec. 3 on a hierarchy whose finest level is stored too
// (B^N with N > 1): every level runs the CSR kernels; the last post-sweep on
// the finest level writes z, and r . z is summed after it.
void enqueue_vcycle_csr(ibpm_ctx *c, PrecSet<double> &P, const double *r, double *z, SolveStatus *st) {
    hipStream_t s = c->stream;
    const int pre = c->prm.amg_pre, post = c->prm.amg_post;
    const int L = (int)P.lev.size();
    if (L == 1) {
        launch_dense_solve(s, P.lev[0].n, c->coarse_inv, r, z, st);
        c->rz_G = launch_dot_rz_parts(s, P.lev[0].n, r, z, st, c->parts);
        return;
    }
    std::vector<double *> cur(L);
    for (int l = 0; l < P.lc; ++l) {
        DevLevelT<double> &lv = P.lev[l];
        const double *b = l == 0 ? r : lv.b;
        double *a = lv.xa, *bb = lv.xb;
        int k = 1;
        if (pre >= 2) {
            launch_csrv_presmooth2(s, lv.A.view(), lv.A.lanes, (const double *)lv.wdinv, b, a, st);
            k = 2;
        } else {
            launch_csr_jacobi_first(s, lv.A.view(), (const double *)lv.wdinv, b, a, st);
        }
        for (; k < pre; ++k) {
            launch_csrv_jacobi(s, lv.A.view(), lv.A.lanes, (const double *)lv.wdinv, b, (const double *)a, bb, st);
            std::swap(a, bb);
        }
        cur[l] = a;
        if (lv.RA.nrows > 0) {
            launch_csrv_restrict(s, lv.R.view(), lv.RA.view(), lv.RA.lanes, b, (const double *)a, P.lev[l + 1].b, st);
        } else {
            launch_csrv_residual(s, lv.A.view(), lv.A.lanes, b, (const double *)a, lv.r, st);
            launch_csrv_spmv(s, lv.R.view(), lv.R.lanes, (const double *)lv.r, P.lev[l + 1].b, false, st);
        }
    }
    launch_coarse_dense(s, P.lev[P.lc].n, (const double *)P.coarseC, (const double *)P.lev[P.lc].b,
                        P.lev[P.lc].xa, st);
    cur[P.lc] = P.lev[P.lc].xa;
    for (int l = P.lc - 1; l >= 0; --l) {
        DevLevelT<double> &lv = P.lev[l];
        const double *b = l == 0 ? r : lv.b;
        double *a = cur[l];
        double *bb = (a == lv.xa) ? lv.xb : lv.xa;
        int k = 0;
        if (lv.AP.nrows > 0) {
            launch_csrv_prolong_jacobi(s, lv.A.view(), lv.AP.view(), lv.P.view(), lv.AP.lanes,
                                       (const double *)lv.wdinv, b, (const double *)a,
                                       (const double *)cur[l + 1], bb, st);
            std::swap(a, bb);
            k = 1;
        } else {
            launch_csrv_spmv(s, lv.P.view(), lv.P.lanes, (const double *)cur[l + 1], a, true, st);
        }
        for (; k < post; ++k) {
            double *dst = (l == 0 && k == post - 1) ? z : bb;
            launch_csrv_jacobi(s, lv.A.view(), lv.A.lanes, (const double *)lv.wdinv, b, (const double *)a, dst, st);
            if (dst == z) a = z;
            else std::swap(a, bb);
        }
        if (l == 0 && a != z) HIPCHECK(hipMemcpyAsync(z, a, P.lev[0].n * sizeof(double), hipMemcpyDeviceToDevice, s));
        cur[l] = a;
    }
    c->rz_G = launch_dot_rz_parts(s, P.lev[0].n, r, z, st, c->parts);
}

// ---------------------------------------------------------------------------
// A body in prescribed motion (Sec. 4 and 6).  E and every row of K that
// couples to the forces are formed anew on the device at each move; the
// level-0 K is a stored CSR rewritten in place.  The SA hierarchy is kept
// for a number of moves and then formed anew on the device from the
// current K: the aggregates and the smoothing weights of the first set-up
// are kept (the aggregation follows the sparsity pattern, which a rigid
// motion leaves as it was up to the cells near the body), the prolongators
// P = (I - w D^-1 A) T, their transposes and the Galerkin products
// P^T A P are recomputed down to the first level of the dense coarse cycle,
// whose small levels and dense map are formed on the host.

void invalidate_graphs(ibpm_ctx *c) {
    HIPCHECK(hipStreamSynchronize(c->stream));
    for (ibpm_ctx::IterGraph &G : c->graphs) {
        if (G.exec) (void)hipGraphExecDestroy(G.exec);
        G.exec = nullptr;
        G.key.clear();
    }
}

// exclusive scan of cnt (n values) on the device into off64 (n + 1) and,
// when non-null, off32; returns the total (read back)
int64_t device_scan(ibpm_ctx *c, int n, const int32_t *cnt, int64_t *off64, int32_t *off32) {
    hipStream_t s = c->stream;
    int64_t *tiles = c->dtemp<int64_t>(scan_tiles_for(n) + 1);
    int64_t *total = tiles + scan_tiles_for(n);
    launch_exclusive_scan(s, n, cnt, off64, off32, tiles, total);
    int64_t h = 0;
    HIPCHECK(hipMemcpyAsync(&h, total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    c->dfree(tiles);
    return h;
}

// product rows with the offsets scanned on the device; `count` may raise
// *err (a left row longer than the merge allows), which is returned
template <class Count, class Fill>
bool product_rows_dev(ibpm_ctx *c, int nrows, int ncols, Count count, Fill fill, bool keep, DevCSR &out) {
    hipStream_t s = c->stream;
    int32_t *cnt = c->dtemp<int32_t>(nrows);
    int *err = c->dtemp<int>(1);
    HIPCHECK(hipMemsetAsync(err, 0, sizeof(int), s));
    count(cnt, err);
    int64_t *off = c->dtemp<int64_t>(nrows + 1);
    int32_t *ptr = keep ? c->dalloc<int32_t>(nrows + 1) : c->dtemp<int32_t>(nrows + 1);
    const int64_t nnz = device_scan(c, nrows, cnt, off, ptr);
    int herr = 0;
    HIPCHECK(hipMemcpy(&herr, err, sizeof(int), hipMemcpyDeviceToHost));
    c->dfree(cnt);
    c->dfree(err);
    if (herr || nnz >= INT32_MAX) {
        c->dfree(off);
        if (keep) c->release(ptr);
        else c->dfree(ptr);
        if (!herr) throw InvalidArg("a hierarchy product has more than 2^31 entries");
        return false;
    }
    out = DevCSR();
    out.nrows = nrows;
    out.ncols = ncols;
    out.nnz = nnz;
    out.lanes = lanes_for(nnz, nrows);
    out.ptr = ptr;
    out.col = keep ? c->dalloc<int32_t>(nnz) : c->dtemp<int32_t>(nnz);
    out.val = keep ? c->dalloc<double>(nnz) : c->dtemp<double>(nnz);
    fill(off, out.col, out.val);
    HIPCHECK(hipStreamSynchronize(s));
    c->dfree(off);
    return true;
}

void drop_csr(ibpm_ctx *c, DevCSR &d, bool keep) {
    if (keep) {
        c->release(d.ptr);
        c->release(d.col);
        c->release(d.val);
    } else {
        free_temp_csr(c, d);
    }
    d = DevCSR();
}

// C = A B for left rows of any length: rows longer than kMergeMax are split
// into chunks whose products are summed by a second product
DevCSR spgemm_any(ibpm_ctx *c, const DevCSR &A, const DevCSR &B, bool keep) {
    hipStream_t s = c->stream;
    const CSRView Av = A.view(), Bv = B.view();
    const int n = A.nrows;
    DevCSR C;
    if (product_rows_dev(
            c, n, B.ncols, [&](int32_t *cnt, int *err) { launch_spgemm_count(s, n, 0, nullptr, Av, Bv, cnt, err); },
            [&](const int64_t *off, int32_t *col, double *val) {
                launch_spgemm_fill(s, n, 0, nullptr, Av, Bv, off, col, val);
            },
            keep, C))
        return C;
    int32_t *cnt = c->dtemp<int32_t>(n);
    launch_chunk_count(s, n, A.ptr, cnt);
    int64_t *off64 = c->dtemp<int64_t>(n + 1);
    int32_t *off32 = c->dtemp<int32_t>(n + 1);
    const int64_t nch = device_scan(c, n, cnt, off64, off32);
    c->dfree(cnt);
    c->dfree(off64);
    DevCSR Ac{}, S{};
    Ac.nrows = (int)nch;
    Ac.ncols = A.ncols;
    Ac.ptr = c->dtemp<int32_t>(nch + 1);
    Ac.col = A.col;
    Ac.val = A.val;
    S.nrows = n;
    S.ncols = (int)nch;
    S.ptr = off32;
    S.col = c->dtemp<int32_t>(nch);
    S.val = c->dtemp<double>(nch);
    launch_chunk_fill(s, n, A.ptr, off32, Ac.ptr, S.col, S.val);
    DevCSR Z;
    const CSRView Acv = Ac.view();
    const int ncr = (int)nch;
    if (!product_rows_dev(
            c, ncr, B.ncols, [&](int32_t *cc, int *err) { launch_spgemm_count(s, ncr, 0, nullptr, Acv, Bv, cc, err); },
            [&](const int64_t *off, int32_t *col, double *val) {
                launch_spgemm_fill(s, ncr, 0, nullptr, Acv, Bv, off, col, val);
            },
            false, Z))
        throw InvalidArg("hierarchy product: a chunk row exceeds the merge width");
    const CSRView Sv = S.view(), Zv = Z.view();
    const bool ok = product_rows_dev(
        c, n, B.ncols, [&](int32_t *cc, int *err) { launch_spgemm_count(s, n, 0, nullptr, Sv, Zv, cc, err); },
        [&](const int64_t *off, int32_t *col, double *val) {
            launch_spgemm_fill(s, n, 0, nullptr, Sv, Zv, off, col, val);
        },
        keep, C);
    free_temp_csr(c, Z);
    c->dfree(Ac.ptr);
    c->dfree(S.col);
    c->dfree(S.val);
    c->dfree(off32);
    if (!ok) throw InvalidArg("hierarchy product: a row has more than kMergeMax^2 entries");
    return C;
}

// A^T (rows sorted) in memory that lives as long as the context
DevCSR transpose_dev(ibpm_ctx *c, const DevCSR &A) {
    hipStream_t s = c->stream;
    const int m = A.ncols;
    int32_t *cnt = c->dtemp<int32_t>(m);
    HIPCHECK(hipMemsetAsync(cnt, 0, (size_t)m * sizeof(int32_t), s));
    launch_col_count(s, A.nnz, A.col, cnt);
    DevCSR T;
    T.nrows = m;
    T.ncols = A.nrows;
    T.ptr = c->dalloc<int32_t>(m + 1);
    int64_t *off = c->dtemp<int64_t>(m + 1);
    T.nnz = device_scan(c, m, cnt, off, T.ptr);
    c->dfree(off);
    if (T.nnz != A.nnz) throw HipError("transpose: entry count mismatch");
    T.col = c->dalloc<int32_t>(T.nnz);
    T.val = c->dalloc<double>(T.nnz);
    HIPCHECK(hipMemsetAsync(cnt, 0, (size_t)m * sizeof(int32_t), s));
    launch_transpose_fill(s, A.view(), T.ptr, cnt, T.col, T.val);
    launch_sort_rows(s, m, T.ptr, T.col, T.val);
    HIPCHECK(hipStreamSynchronize(s));
    c->dfree(cnt);
    T.lanes = lanes_for(T.nnz, T.nrows);
    return T;
}

// Form the hierarchy anew from the current level-0 K (see above)
void refresh_hierarchy(ibpm_ctx *c) {
    hipStream_t s = c->stream;
    PrecSet<double> &P = c->p64;
    Hierarchy &h = c->h;
    const int L = (int)P.lev.size();
    if (L < 2) {
        // one level: the dense solve of the moved K
        const DevCSR &D = c->K0c;
        CSR A;
        A.nrows = D.nrows;
        A.ncols = D.ncols;
        A.ptr.resize(D.nrows + 1);
        A.col.resize(D.nnz);
        A.val.resize(D.nnz);
        HIPCHECK(hipStreamSynchronize(s));
        HIPCHECK(hipMemcpy(A.ptr.data(), D.ptr, A.ptr.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(A.col.data(), D.col, A.col.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(A.val.data(), D.val, A.val.size() * sizeof(double), hipMemcpyDeviceToHost));
        try {
            regalerkin_from(h, 0, std::move(A));
        } catch (const std::runtime_error &e) {
            throw InvalidArg(e.what());
        }
        HIPCHECK(hipMemcpy(c->coarse_inv, h.coarse_inv.data(), h.coarse_inv.size() * sizeof(double),
                           hipMemcpyHostToDevice));
        h.levels[0].wdinv.clear();
        c->refreshes++;
        invalidate_graphs(c);
        return;
    }
    const int lc = P.lc;
    double *diag = c->dtemp<double>(P.lev[0].n);
    int *err = c->dtemp<int>(1);
    HIPCHECK(hipMemsetAsync(err, 0, sizeof(int), s));
    for (int l = 0; l < lc; ++l) {
        DevLevelT<double> &lv = P.lev[l];
        const Level &hl = h.levels[l];
        const DevCSR &A = lv.A;
        launch_diag_weights(s, A.view(), hl.omega, diag, lv.wdinv);
        const int nc = P.lev[l + 1].n;
        DevCSR T{};
        T.nrows = lv.n;
        T.ncols = nc;
        T.nnz = lv.n;
        T.ptr = c->dtemp<int32_t>(lv.n + 1);
        T.col = c->dtemp<int32_t>(lv.n);
        T.val = c->dtemp<double>(lv.n);
        launch_tentative(s, lv.n, c->agg_d[l], T.ptr, T.col, T.val);
        DevCSR Pn = spgemm_any(c, A, T, true);
        free_temp_csr(c, T);
        launch_smooth_prolongator(s, lv.n, Pn.ptr, Pn.col, Pn.val, c->agg_d[l], diag, hl.pomega, err);
        DevCSR Rn = transpose_dev(c, Pn);
        DevCSR AP = spgemm_any(c, A, Pn, false);
        DevCSR Ac = spgemm_any(c, Rn, AP, true);
        free_temp_csr(c, AP);
        drop_csr(c, lv.P, true);
        drop_csr(c, lv.R, true);
        lv.P = Pn;
        lv.R = Rn;
        drop_csr(c, P.lev[l + 1].A, true);
        P.lev[l + 1].A = Ac;
    }
    int herr = 0;
    HIPCHECK(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    c->dfree(err);
    c->dfree(diag);
    if (herr) throw InvalidArg("AMG: non-positive diagonal in the moved operator");
    // the small levels on the host: A_lc back, the levels below it and the
    // dense coarse cycle formed there
    const DevCSR &Alc = P.lev[lc].A;
    CSR A;
    A.nrows = Alc.nrows;
    A.ncols = Alc.ncols;
    A.ptr.resize(Alc.nrows + 1);
    A.col.resize(Alc.nnz);
    A.val.resize(Alc.nnz);
    HIPCHECK(hipMemcpy(A.ptr.data(), Alc.ptr, A.ptr.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(A.col.data(), Alc.col, A.col.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(A.val.data(), Alc.val, A.val.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int l = 0; l < lc; ++l) c->level_nnz[l + 1] = P.lev[l + 1].A.nnz;
    try {
        regalerkin_from(h, lc, std::move(A));
    } catch (const std::runtime_error &e) {
        throw InvalidArg(e.what());
    }
    for (int l = lc + 1; l < L; ++l) c->level_nnz[l] = h.levels[l].A.nnz();
    c->coarse_C = coarse_cycle_matrix(h, lc, c->prm.amg_pre, c->prm.amg_post);
    HIPCHECK(hipMemcpy(c->coarse_C_dev, c->coarse_C.data(), c->coarse_C.size() * sizeof(double),
                       hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(c->coarse_inv, h.coarse_inv.data(), h.coarse_inv.size() * sizeof(double),
                       hipMemcpyHostToDevice));
    for (int l = lc; l < L; ++l) {
        Level &hl = h.levels[l];
        hl.P = CSR();
        hl.R = CSR();
        hl.wdinv.clear();
    }
    c->refreshes++;
    invalidate_graphs(c);
}

// K's level-0 storage with room for `cap` entries (the row starts stay)
void grow_k0(ibpm_ctx *c, int64_t cap) {
    HIPCHECK(hipStreamSynchronize(c->stream));
    c->release(c->K0c.col);
    c->release(c->K0c.val);
    c->K0c.col = c->dalloc<int32_t>(cap);
    c->K0c.val = c->dalloc<double>(cap);
    c->K_cap = cap;
    c->K0op.A = c->K0c.view();
    if (!c->p64.lev.empty()) {
        c->p64.lev[0].A.col = c->K0c.col;
        c->p64.lev[0].A.val = c->K0c.val;
    }
    invalidate_graphs(c);
}

// room for `need` entries of a (col, val) pair of row buffers
void grow_pair(ibpm_ctx *c, int32_t *&col, double *&val, int64_t &cap, int64_t need) {
    if (col && need <= cap) return;
    HIPCHECK(hipStreamSynchronize(c->stream));
    c->release(col);
    c->release(val);
    cap = std::max<int64_t>({need, cap + cap / 2, 1});
    col = c->dalloc<int32_t>(cap);
    val = c->dalloc<double>(cap);
}

// E and K for the point positions in xb_d / yb_d (host copies xb, yb)
void assemble_moving(ibpm_ctx *c, const double *xb, const double *yb) {
    hipStream_t s = c->stream;
    const Model &m = c->m;
    const GridMetrics &G = m.g;
    const int nb = m.nb, nx = G.nx, ny = G.ny;
    const int n_cell = (int)G.n_cell, nl = n_cell + 2 * nb;
    // the cells whose faces the E rows reach: the point's cell +- 2
    auto cell = [](const std::vector<double> &f, double x) {
        return (int)(std::upper_bound(f.begin(), f.end(), x) - f.begin()) - 1;
    };
    int i0 = INT_MAX, i1 = INT_MIN, j0 = INT_MAX, j1 = INT_MIN;
    double hmax = 0.0;
    for (int k = 0; k < nb; ++k) {
        const int i = cell(G.xf, xb[k]), j = cell(G.yf, yb[k]);
        i0 = std::min(i0, i - 2);
        i1 = std::max(i1, i + 2);
        j0 = std::min(j0, j - 2);
        j1 = std::max(j1, j + 2);
        hmax = std::max({hmax, G.dx[i], G.dy[j]});
    }
    i0 = std::max(i0, 0);
    j0 = std::max(j0, 0);
    i1 = std::min(i1, nx - 1);
    j1 = std::min(j1, ny - 1);
    c->box[0] = i0;
    c->box[1] = i1;
    c->box[2] = j0;
    c->box[3] = j1;
    const int nbox = (i1 - i0 + 1) * (j1 - j0 + 1);
    launch_e_rows(s, c->g, c->xf_d, c->yf_d, nb, c->xb_d, c->yb_d, c->ecol, c->eval);
    const double reach = 3.5 * hmax;
    const double dt = c->prm.dt;
    const int pin = m.pin;
    // force rows: lengths, offsets, rows
    launch_force_rows(s, c->g, dt, nb, pin, c->ecol, c->eval, c->xb_d, c->yb_d, reach, c->force_len, nullptr,
                      nullptr, nullptr);
    const int64_t nf = device_scan(c, 2 * nb, c->force_len, c->force_ptr, nullptr);
    grow_pair(c, c->force_col, c->force_val, c->force_cap, nf);
    launch_force_rows(s, c->g, dt, nb, pin, c->ecol, c->eval, c->xb_d, c->yb_d, reach, nullptr, c->force_ptr,
                      c->force_col, c->force_val);
    // rows of the box cells
    if (nbox > c->box_rows_cap) {
        HIPCHECK(hipStreamSynchronize(s));
        c->release(c->box_len);
        c->release(c->box_ptr);
        c->box_rows_cap = nbox;
        c->box_len = c->dalloc<int32_t>(nbox);
        c->box_ptr = c->dalloc<int64_t>(nbox + 1);
    }
    const CSRView Kpp = c->Kpp.view();
    launch_box_rows(s, c->g, c->xf_d, c->yf_d, dt, nb, pin, i0, i1, j0, j1, Kpp, c->ecol, c->eval, c->xb_d, c->yb_d,
                    c->box_len, nullptr, nullptr, nullptr);
    const int64_t nbx = device_scan(c, nbox, c->box_len, c->box_ptr, nullptr);
    grow_pair(c, c->box_col, c->box_val, c->box_cap, nbx);
    launch_box_rows(s, c->g, c->xf_d, c->yf_d, dt, nb, pin, i0, i1, j0, j1, Kpp, c->ecol, c->eval, c->xb_d, c->yb_d,
                    nullptr, c->box_ptr, c->box_col, c->box_val);
    // the whole K: lengths, row starts, rows
    launch_row_lengths(s, nx, n_cell, nl, i0, i1, j0, j1, Kpp, c->box_len, c->force_len, c->len_all);
    const int64_t nnz = device_scan(c, nl, c->len_all, c->ptr64, c->K0c.ptr);
    if (nnz >= INT32_MAX) throw InvalidArg("K has more than 2^31 entries");
    if (nnz > c->K_cap) grow_k0(c, nnz + nnz / 8);
    launch_assemble(s, nx, n_cell, nl, i0, i1, j0, j1, Kpp, c->box_ptr, c->box_col, c->box_val, c->force_ptr,
                    c->force_col, c->force_val, c->K0c.ptr, c->K0c.col, c->K0c.val);
    c->K0c.nnz = nnz;
    if (!c->p64.lev.empty()) c->p64.lev[0].A.nnz = nnz;
    c->level_nnz[0] = nnz;
    const double w0 = c->amg ? c->h.levels[0].omega : 1.0;
    launch_diag_weights(s, c->K0c.view(), w0, c->K0diag, c->amg ? c->p64.lev[0].wdinv : nullptr);
    HIPCHECK(hipStreamSynchronize(s));
}

void upload_points(ibpm_ctx *c, const double *xb, const double *yb, const double *ubx, const double *uby) {
    const int nb = c->m.nb;
    if (nb == 0) return;
    hipStream_t s = c->stream;
    HIPCHECK(hipMemcpyAsync(c->xb_d, xb, nb * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(c->yb_d, yb, nb * sizeof(double), hipMemcpyHostToDevice, s));
    if (ubx && uby) {
        HIPCHECK(hipMemcpyAsync(c->ub, ubx, nb * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(c->ub + nb, uby, nb * sizeof(double), hipMemcpyHostToDevice, s));
    }
    HIPCHECK(hipStreamSynchronize(s));
}

// Device storage of the moving-body path, then E and K at the first
// positions; called after the hierarchy is on the device
void moving_setup(ibpm_ctx *c, const ibpm_params *p) {
    const Model &m = c->m;
    const GridMetrics &G = m.g;
    const int nb = m.nb, n_cell = (int)G.n_cell, nl = n_cell + 2 * nb;
    c->xf_d = c->upload(G.xf);
    c->yf_d = c->upload(G.yf);
    c->xb_d = c->dalloc<double>(nb);
    c->yb_d = c->dalloc<double>(nb);
    c->ecol = c->dalloc<int32_t>((size_t)2 * nb * kEllE);
    c->eval = c->dalloc<double>((size_t)2 * nb * kEllE);
    std::vector<int32_t> ep(2 * nb + 1);
    for (int t = 0; t <= 2 * nb; ++t) ep[t] = t * kEllE;
    c->eptr = c->upload(ep);
    // E as a CSR view over its fixed-width rows (zero weights included)
    c->E.nrows = 2 * nb;
    c->E.ncols = (int)G.n_q;
    c->E.nnz = (int64_t)2 * nb * kEllE;
    c->E.ptr = c->eptr;
    c->E.col = c->ecol;
    c->E.val = c->eval;
    // the pressure rows of K (cell rows, cell columns), fixed
    CSR Kpp;
    Kpp.nrows = n_cell;
    Kpp.ncols = n_cell;
    Kpp.ptr.assign(1, 0);
    for (int r = 0; r < n_cell; ++r) {
        for (int32_t q = m.K.ptr[r]; q < m.K.ptr[r + 1]; ++q)
            if (m.K.col[q] < n_cell) {
                Kpp.col.push_back(m.K.col[q]);
                Kpp.val.push_back(m.K.val[q]);
            }
        Kpp.ptr.push_back((int32_t)Kpp.col.size());
    }
    c->Kpp = c->upload_csr<double>(Kpp);
    c->len_all = c->dalloc<int32_t>(nl);
    c->ptr64 = c->dalloc<int64_t>(nl + 1);
    c->force_len = c->dalloc<int32_t>(std::max(1, 2 * nb));
    c->force_ptr = c->dalloc<int64_t>(2 * nb + 1);
    c->level_nnz.assign(std::max<size_t>(1, c->h.levels.size()), 0);
    for (size_t l = 0; l < c->h.levels.size(); ++l) c->level_nnz[l] = c->h.levels[l].A.nnz();
    if (c->amg) {
        const int lc = c->p64.lc;
        c->agg_d.assign(lc, nullptr);
        for (int l = 0; l < lc; ++l) c->agg_d[l] = c->upload(c->h.levels[l].agg);
    }
    upload_points(c, p->xb, p->yb, nullptr, nullptr);
    assemble_moving(c, p->xb, p->yb);
}

void move_body(ibpm_ctx *c, const double *xb, const double *yb, const double *ubx, const double *uby) {
    if (!c->moving) throw InvalidArg("the context was built for a fixed body (moving_body = 0)");
    const int nb = c->m.nb;
    if (nb > 0 && (!xb || !yb || !ubx || !uby)) throw InvalidArg("NULL point array");
    for (int k = 0; k < nb; ++k)
        if (!std::isfinite(xb[k]) || !std::isfinite(yb[k]) || !std::isfinite(ubx[k]) || !std::isfinite(uby[k]))
            throw InvalidArg("point positions and velocities must be finite");
    try {
        check_points(c->m.g, nb, xb, yb);
    } catch (const std::runtime_error &e) {
        throw InvalidArg(e.what());
    }
    upload_points(c, xb, yb, ubx, uby);
    assemble_moving(c, xb, yb);
    ++c->moves;
    if (c->amg && c->prm.amg_rebuild_every > 0 && c->moves % c->prm.amg_rebuild_every == 0) refresh_hierarchy(c);
}

// Work memory of the allocation-free velocity solve: the five PCG vectors
// (r, z, two directions, q) of at most kStaticMaxNq values each, three
// buffers of per-block partial sums (three rows of kMaxParts each, as many
// as one reduction writes) and the solve status, in one file-scope device
// array.  Each device that loads the library holds its own copy until the
// process ends; its address is looked up once per device.
constexpr int64_t kStaticMaxNq = (int64_t)1 << 20;
constexpr size_t kStaticVec = (size_t)kStaticMaxNq;
constexpr size_t kStaticParts = (size_t)3 * kMaxParts;
constexpr size_t kStaticStatus = (sizeof(SolveStatus) + sizeof(double) - 1) / sizeof(double);
constexpr size_t kStaticDoubles = 5 * kStaticVec + 3 * kStaticParts + kStaticStatus;
static __device__ __align__(256) double scratch[kStaticDoubles];

constexpr int kStaticMaxDevices = 64;
std::mutex g_static_mu;
double *g_static_ptr[kStaticMaxDevices] = {};

// device address of `scratch` on the current device (host code never uses
// the array's own name as an address)
double *static_work_address() {
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kStaticMaxDevices) throw std::runtime_error("device index out of range");
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            throw HipError(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_static_ptr[dev] = (double *)ptr;
    }
    return g_static_ptr[dev];
}

__global__ void k_clear_words(double *w, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = 0.0;
}

// the solve vectors (velocity n_q, Poisson n_lambda), statuses, partial
// sums and the pinned status copy
void alloc_work(ibpm_ctx *c, int nq, int nl) {
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
    // partial sums of up to kFcgMax components per block (FCG multi-dot)
    c->parts = c->dalloc<double>((size_t)kFcgMax * kMaxParts);
    c->parts2 = c->dalloc<double>((size_t)kFcgMax * kMaxParts);
    // the update writes two rows of partials (r . r and, for Jacobi, r . z)
    c->parts3 = c->dalloc<double>((size_t)kFcgMax * kMaxParts);
    HIPCHECK(hipHostMalloc((void **)&c->host_st, sizeof(SolveStatus), hipHostMallocDefault));
}

// a device CSR and its diagonal as a stored operator for the Krylov kernels
CsrOpView stored_op(ibpm_ctx *c, const CSR &M, DevCSR &dev) {
    dev = c->upload_csr<double>(M);
    std::vector<double> d((size_t)M.nrows, 0.0);
    for (int32_t r = 0; r < M.nrows; ++r)
        for (int32_t q = M.ptr[r]; q < M.ptr[r + 1]; ++q)
            if (M.col[q] == r) d[r] = M.val[q];
    set_stream_shape(c, dev, {&M});
    CsrOpView op{};
    op.A = dev.view();
    op.diag = c->upload(d);
    return op;
}

void check_params3(const ibpm3d_params *p) {
    if (!p) throw InvalidArg("params is NULL");
    if (!(p->vel_rtol > 0) || !(p->poisson_rtol > 0)) throw InvalidArg("tolerances must be > 0");
    if (p->vel_maxit < 1 || p->poisson_maxit < 1) throw InvalidArg("maxit must be >= 1");
    if (p->poisson_solver != IBPM_SOLVER_JACOBI_PCG && p->poisson_solver != IBPM_SOLVER_AMG_PCG)
        throw InvalidArg("3-D: the Jacobi-PCG and AMG-PCG Poisson solvers only");
    if (p->poisson_solver == IBPM_SOLVER_AMG_PCG) {
        if (p->amg_pre < 1 || p->amg_post < 1) throw InvalidArg("AMG needs >= 1 pre and post sweep");
        if (p->amg_coarse_max < 1 || p->amg_max_levels < 1 || p->amg_max_levels > kMaxLevels)
            throw InvalidArg("bad AMG limits");
        if (!(p->amg_theta >= 0)) throw InvalidArg("amg_theta must be >= 0");
    }
    if (p->use_graphs != 0 && p->use_graphs != 1) throw InvalidArg("use_graphs must be 0 or 1");
}

// Operators of the three-dimensional extension on the host, then stored on
// the device: K (level 0 of an all-CSR hierarchy), A, Q, Q^T and B^1
void build3(ibpm_ctx *c, const ibpm3d_params *p) {
    check_params3(p);
    Model3 m3;
    try {
        build_model3(m3, p->nx, p->ny, p->nz, p->xf, p->yf, p->zf, p->nb, p->xb, p->yb, p->zb, p->nu, p->dt,
                     p->pin_cell);
    } catch (const std::runtime_error &e) {
        throw InvalidArg(e.what());
    }
    // the solver settings are kept in the fields of the 2-D parameter block
    ibpm_params &q = c->prm;
    q = ibpm_params{};
    q.nu = p->nu;
    q.dt = p->dt;
    q.bn_order = 1;
    q.vel_rtol = p->vel_rtol;
    q.vel_maxit = p->vel_maxit;
    q.poisson_solver = p->poisson_solver;
    q.poisson_rtol = p->poisson_rtol;
    q.poisson_maxit = p->poisson_maxit;
    q.amg_theta = p->amg_theta;
    q.amg_pre = p->amg_pre;
    q.amg_post = p->amg_post;
    q.amg_coarse_max = p->amg_coarse_max;
    q.amg_max_levels = p->amg_max_levels;
    q.use_graphs = p->use_graphs;
    q.fuse_transfers = 1;
    q.pin_cell = p->pin_cell;
    c->three_d = true;
    c->stored0 = true;
    c->amg = p->poisson_solver == IBPM_SOLVER_AMG_PCG;
    c->n_q3 = m3.n_q;
    const int nq = (int)m3.n_q, nl = m3.K.nrows;
    if (c->amg) {
        AmgParams ap;
        ap.theta = p->amg_theta;
        ap.coarse_max = p->amg_coarse_max;
        ap.max_levels = p->amg_max_levels;
        try {
            build_hierarchy(c->h, m3.K, ap);
        } catch (const std::runtime_error &e) {
            throw InvalidArg(e.what());
        }
        fused_transfer_products(c->h);
    }
    c->K0op = stored_op(c, m3.K, c->K0c);
    c->A3op = stored_op(c, m3.A, c->A3);
    c->QT3 = c->upload_csr<double>(m3.QT);
    c->Q3 = c->upload_csr<double>(m3.Q);
    {
        // B^1 as a diagonal CSR, for the projection's product
        CSR B;
        B.nrows = B.ncols = nq;
        B.ptr.resize(nq + 1);
        B.col.resize(nq);
        for (int f = 0; f <= nq; ++f) B.ptr[f] = f;
        for (int f = 0; f < nq; ++f) B.col[f] = f;
        B.val = m3.b1;
        c->B3 = c->upload_csr<double>(B);
    }
    if (c->amg) {
        upload_levels<double>(c, c->p64);
        c->coarse_inv = c->upload(c->h.coarse_inv);
        for (auto &hl : c->h.levels) {
            hl.P = CSR();
            hl.R = CSR();
            hl.RA = CSR();
            hl.AP = CSR();
            hl.wdinv.clear();
        }
    }
    c->wq = c->dalloc<double>(nq);
    alloc_work(c, nq, nl);
    HIPCHECK(hipStreamSynchronize(c->stream));
}

// q* = solution of A q* = rhs (Jacobi-PCG from q)
int solve_velocity3(ibpm_ctx *c, const double *rhs, double *q, ibpm_solve_stats *out) {
    std::function<void(const double *, double *)> none;
    return pcg_drive<CsrOpView, double>(c, c->A3op, (int)c->n_q3, true, none, rhs, q, c->vr, c->vz, c->vp,
                                        c->vq, c->st_vel, c->prm.vel_rtol, c->prm.vel_maxit, c->est_vel, false,
                                        true, out, 0);
}

// rhs = Q^T q* - r2, the pinned entry cleared
void poisson_rhs3(ibpm_ctx *c, const double *qstar, const double *r2, double *rhs) {
    hipStream_t s = c->stream;
    launch_csr_gemv(s, c->QT3.view(), qstar, 1.0, nullptr, rhs);
    launch_axpby(s, c->QT3.nrows, -1.0, r2, 1.0, rhs);
    HIPCHECK(hipMemsetAsync(rhs + c->prm.pin_cell, 0, sizeof(double), s));
}

// qout = q* - B^1 (Q lambda)
void project3(ibpm_ctx *c, const double *qstar, const double *lam, double *qout) {
    hipStream_t s = c->stream;
    launch_csr_gemv(s, c->Q3.view(), lam, -1.0, nullptr, c->wq);
    launch_csr_gemv(s, c->B3.view(), c->wq, 1.0, qstar, qout);
}

void need3d(const ibpm_ctx *c) {
    if (!c->three_d) throw InvalidArg("a three-dimensional entry point called on a two-dimensional context");
}

void build(ibpm_ctx *c, const ibpm_params *p) {
    check_params(p);
    c->prm = *p;
    c->prm.xf = c->prm.yf = c->prm.xb = c->prm.yb = c->prm.ubx = c->prm.uby = nullptr;
    Model &m = c->m;
    try {
        build_model(m, p->nx, p->ny, p->xf, p->yf, p->nb, p->xb, p->yb, p->ubx, p->uby, p->nu, p->dt,
                    p->pin_cell);
    } catch (const std::runtime_error &e) {
        throw InvalidArg(e.what());
    }
    set_walls_spec(c, m.g);
    c->amg = p->poisson_solver != IBPM_SOLVER_JACOBI_PCG;
    c->mixed = p->poisson_solver == IBPM_SOLVER_AMG_PCG_MIXED ||
               p->poisson_solver == IBPM_SOLVER_AMG_FCG_MIXED_LEARNED ||
               p->poisson_solver == IBPM_SOLVER_AMG_PCG_FP32_CYCLE ||
               p->poisson_solver == IBPM_SOLVER_AMG_PCG_FP32_CYCLE_GUESS;
    c->mixed_precond = p->poisson_solver == IBPM_SOLVER_AMG_PCG_FP32_CYCLE ||
                       p->poisson_solver == IBPM_SOLVER_AMG_PCG_FP32_CYCLE_GUESS;
    c->guess_learned = p->poisson_solver == IBPM_SOLVER_AMG_PCG_FP32_CYCLE_GUESS;
    c->learned = p->poisson_solver == IBPM_SOLVER_AMG_FCG_LEARNED ||
                 p->poisson_solver == IBPM_SOLVER_AMG_FCG_MIXED_LEARNED;
    // every parameter is valid: from here on the device is used
    c->static_work = static_work_address();
    c->bn = p->bn_order;
    c->moving = p->moving_body != 0;
    c->stored0 = c->bn > 1 || c->moving;
    if (c->bn > 1) form_bn_operators(c);   // replaces m.K by the pinned Q^T B^N Q
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
        // the fused products hold K, which a moving body changes
        if (p->fuse_transfers && !c->moving) fused_transfer_products(c->h);
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
    {
        const long nbox = m.cb_i1 >= m.cb_i0 && m.cb_j1 >= m.cb_j0
                              ? (long)(m.cb_i1 - m.cb_i0 + 1) * (m.cb_j1 - m.cb_j0 + 1) : 0;
        if (nbox != (long)m.Kcf.nrows) throw std::runtime_error("coupling rows do not match the coupling box");
    }
    const BandHost bh = make_bands(m);
    BandDev<double> bd64;
    bd64.kf_ok = bh.kf_ok;
    bd64.cc_ok = bh.cc_ok;
    bd64.ncc = (int)bh.cc_row.size();
    bd64.kf_col = c->upload(bh.kf_col);
    bd64.cc_row = c->upload(bh.cc_row);
    bd64.cc_col = c->upload(bh.cc_col);
    bd64.bits = c->upload(bh.bits);
    bd64.kf_val = c->upload(bh.kf_val);
    bd64.cc_val = c->upload(bh.cc_val);
    c->p64.K0 = make_k0<double>(c->g, p->dt, m, cf, kf, kfd, bd64);
    c->A.g = c->g;
    c->A.dt = p->dt;
    c->A.idt = 1.0 / p->dt;
    c->A.nu = p->nu;
    const int nq = c->g.n_q, nl = c->p64.K0.n;
    if (c->bn > 1) {
        // the stored level-0 operator and its diagonal
        c->K0c = c->upload_csr<double>(m.K);
        set_stream_shape(c, c->K0c, {&m.K});
        std::vector<double> dg((size_t)m.K.nrows, 0.0);
        for (int32_t r = 0; r < m.K.nrows; ++r)
            for (int32_t q = m.K.ptr[r]; q < m.K.ptr[r + 1]; ++q)
                if (m.K.col[q] == r) dg[r] = m.K.val[q];
        c->K0op.A = c->K0c.view();
        c->K0op.diag = c->upload(dg);
        c->wq = c->dalloc<double>(nq);
    }
    if (c->moving) {
        // the stored level-0 K with room for the rows of the moved body
        const int64_t nnz = m.K.nnz();
        c->K_cap = nnz + std::max<int64_t>(4096, (int64_t)256 * m.nb);
        c->K0c.nrows = c->K0c.ncols = nl;
        c->K0c.nnz = nnz;
        c->K0c.lanes = lanes_for(nnz, nl);
        c->K0c.bst = nullptr;
        c->K0c.rpb = 0;
        c->K0c.nblk = 0;
        c->K0c.ptr = c->upload(m.K.ptr);
        c->K0c.col = c->dalloc<int32_t>(c->K_cap);
        c->K0c.val = c->dalloc<double>(c->K_cap);
        HIPCHECK(hipMemcpy(c->K0c.col, m.K.col.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPCHECK(hipMemcpy(c->K0c.val, m.K.val.data(), nnz * sizeof(double), hipMemcpyHostToDevice));
        c->K0diag = c->dalloc<double>(nl);
        c->K0op.A = c->K0c.view();
        c->K0op.diag = c->K0diag;   // no row blocks: its rows change with every move
    }
    if (c->amg) {
        upload_levels<double>(c, c->p64);
        c->coarse_inv = c->upload(c->h.coarse_inv);
    }
    if (c->mixed) {
        GridT<float> g32 = make_grid<float>(c, G);
        DevCSRT<float> cf32 = c->values32(cf, m.Kcf), kf32 = c->values32(kf, m.Kf);
        float *kfd32 = c->upload(std::vector<float>(m.Kf_diag.begin(), m.Kf_diag.end()));
        BandDev<float> bd32;
        bd32.kf_ok = bd64.kf_ok;
        bd32.cc_ok = bd64.cc_ok;
        bd32.ncc = bd64.ncc;
        bd32.kf_col = bd64.kf_col;
        bd32.cc_row = bd64.cc_row;
        bd32.cc_col = bd64.cc_col;
        bd32.bits = bd64.bits;
        bd32.kf_val = c->upload(std::vector<float>(bh.kf_val.begin(), bh.kf_val.end()));
        bd32.cc_val = c->upload(std::vector<float>(bh.cc_val.begin(), bh.cc_val.end()));
        c->p32.K0 = make_k0<float>(g32, p->dt, m, cf32, kf32, kfd32, bd32);
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
            hl.RA = CSR();
            hl.AP = CSR();
            hl.wdinv.clear();
        }
    }
    alloc_work(c, nq, nl);
    launch_fill_walls(c->stream, c->g, c->walls[0], c->wall_init);
    launch_fill_walls(c->stream, c->g, c->walls[1], c->wall_init);
    if (c->moving) moving_setup(c, p);
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

int ibpm3d_build_operators(const ibpm3d_params *p, void *stream, ibpm_ctx **out) {
    if (!out) return IBPM_EINVAL;
    *out = nullptr;
    ibpm_ctx *c = new (std::nothrow) ibpm_ctx();
    if (!c) return IBPM_ENOMEM;
    c->stream = (hipStream_t)stream;
    int rc = guarded(c, [&] {
        build3(c, p);
        return IBPM_OK;
    });
    *out = c;
    return rc;
}

int ibpm3d_solve_velocity(ibpm_ctx *c, const double *rhs, double *q, ibpm_solve_stats *stats) {
    return guarded(c, [&] {
        need3d(c);
        if (!rhs || !q) throw InvalidArg("NULL vector");
        return solve_velocity3(c, rhs, q, stats);
    });
}

int ibpm3d_apply_A(ibpm_ctx *c, const double *x, double *y) {
    return guarded(c, [&] {
        need3d(c);
        if (!x || !y || x == y) throw InvalidArg("x and y must be distinct device vectors");
        launch_csr_gemv(c->stream, c->A3.view(), x, 1.0, nullptr, y);
        return IBPM_OK;
    });
}

int ibpm3d_poisson_rhs(ibpm_ctx *c, const double *qstar, const double *r2, double *rhs) {
    return guarded(c, [&] {
        need3d(c);
        if (!qstar || !r2 || !rhs || rhs == r2) throw InvalidArg("NULL or aliased vector");
        poisson_rhs3(c, qstar, r2, rhs);
        return IBPM_OK;
    });
}

int ibpm3d_project(ibpm_ctx *c, const double *qstar, const double *lam, double *qout) {
    return guarded(c, [&] {
        need3d(c);
        if (!qstar || !lam || !qout) throw InvalidArg("NULL vector");
        project3(c, qstar, lam, qout);
        return IBPM_OK;
    });
}

int ibpm3d_linear_step(ibpm_ctx *c, const double *r1, const double *r2, double *q, double *lam,
                       ibpm_solve_stats *vel_stats, ibpm_solve_stats *poisson_stats) {
    return guarded(c, [&] {
        need3d(c);
        if (!r1 || !r2 || !q || !lam) throw InvalidArg("NULL vector");
        int rc = solve_velocity3(c, r1, q, vel_stats);
        if (rc != IBPM_OK) return rc;
        poisson_rhs3(c, q, r2, c->rhs2);
        rc = solve_poisson_impl(c, c->rhs2, lam, poisson_stats);
        if (rc != IBPM_OK) return rc;
        project3(c, q, lam, q);
        HIPCHECK(hipStreamSynchronize(c->stream));
        return IBPM_OK;
    });
}

int ibpm_destroy(ibpm_ctx *ctx) {
    delete ctx;
    return IBPM_OK;
}

const char *ibpm_last_error(const ibpm_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

int ibpm_sizes(const ibpm_ctx *c, int64_t *nq, int64_t *nl) {
    if (c && c->three_d) {
        if (nq) *nq = c->n_q3;
        if (nl) *nl = c->K0c.nrows;
        return IBPM_OK;
    }
    if (!c || c->g.nx == 0) return IBPM_EINVAL;
    if (nq) *nq = c->g.n_q;
    if (nl) *nl = c->p64.K0.n;
    return IBPM_OK;
}

int ibpm_init_state(ibpm_ctx *c, double *q, double *conv, double *lam) {
    return guarded(c, [&] {
        need2d(c);
        if (!q || !conv || !lam) throw InvalidArg("NULL vector");
        double U = c->prm.uinf * std::cos(c->prm.alpha), V = c->prm.uinf * std::sin(c->prm.alpha);
        launch_init_state(c->stream, c->g, q, conv, lam, c->p64.K0.n, U, V);
        launch_fill_walls(c->stream, c->g, c->walls[0], c->wall_init);
        launch_fill_walls(c->stream, c->g, c->walls[1], c->wall_init);
        c->cur = 0;
        c->step = 0;
        return IBPM_OK;
    });
}

int ibpm_step(ibpm_ctx *c, int32_t nsteps, double *q, double *conv, double *lam,
              ibpm_step_stats *stats) {
    return guarded(c, [&] {
        need2d(c);
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
        need2d(c);
        if (!rhs || !q) throw InvalidArg("NULL vector");
        return solve_velocity_impl(c, rhs, q, stats);
    });
}

int ibpm_solve_velocity_static(ibpm_ctx *c, const double *rhs, double *q, ibpm_solve_stats *stats) {
    return guarded(c, [&] {
        need2d(c);
        if (!rhs || !q) throw InvalidArg("NULL vector");
        const int64_t nq = c->g.n_q;
        if (nq > kStaticMaxNq)
            throw InvalidArg("n_q = " + std::to_string(nq) + " exceeds the " + std::to_string(kStaticMaxNq) +
                             " flux unknowns the static work array holds");
        double *base = c->static_work;
        if (!base) throw std::runtime_error("static work array not set up");
        double *r = base, *z = base + kStaticVec, *qq = base + 4 * kStaticVec;
        double *dirs[2] = {base + 2 * kStaticVec, base + 3 * kStaticVec};
        double *parts = base + 5 * kStaticVec;
        SolveStatus *st = (SolveStatus *)(parts + 3 * kStaticParts);
        // the array keeps the last call's contents: the status starts cleared
        // (the vectors and partial sums are written before they are read)
        hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, c->stream, (double *)st, (int)kStaticStatus);
        HIPCHECK(hipGetLastError());
        // the solver's kernels take their partial-sum buffers from the
        // context; point them at the array for this call only
        struct Restore {
            ibpm_ctx *c;
            double *a, *b, *d;
            ~Restore() { c->parts = a; c->parts2 = b; c->parts3 = d; }
        } restore{c, c->parts, c->parts2, c->parts3};
        c->parts = parts;
        c->parts2 = parts + kStaticParts;
        c->parts3 = parts + 2 * kStaticParts;
        std::function<void(const double *, double *)> none;
        // launched one by one: recording a graph would allocate
        return pcg_drive<AView, double>(c, c->A, (int)nq, true, none, rhs, q, r, z, dirs, qq, st,
                                        c->prm.vel_rtol, c->prm.vel_maxit, c->est_vel, false, true, stats, -1);
    });
}

int ibpm_apply_K(ibpm_ctx *c, const double *x, double *y) {
    return guarded(c, [&] {
        if (!x || !y || x == y) throw InvalidArg("x and y must be distinct device vectors");
        if (c->stored0) launch_csr_gemv(c->stream, c->K0c.view(), x, 1.0, nullptr, y);
        else launch_apply_K0(c->stream, c->p64.K0, x, y);
        return IBPM_OK;
    });
}

int ibpm_apply_A(ibpm_ctx *c, const double *x, double *y) {
    return guarded(c, [&] {
        need2d(c);
        if (!x || !y || x == y) throw InvalidArg("x and y must be distinct device vectors");
        launch_apply_A(c->stream, c->A, x, y);
        return IBPM_OK;
    });
}

int ibpm_get_poisson_matrix(ibpm_ctx *c, int64_t *nnz, int32_t *ptr, int32_t *col, double *val) {
    return guarded(c, [&] {
        if (!nnz) throw InvalidArg("nnz is NULL");
        if (c->moving || c->three_d) {
            // the device K of the current positions
            const DevCSR &D = c->K0c;
            *nnz = D.nnz;
            HIPCHECK(hipStreamSynchronize(c->stream));
            if (ptr) HIPCHECK(hipMemcpy(ptr, D.ptr, (D.nrows + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
            if (col) HIPCHECK(hipMemcpy(col, D.col, D.nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
            if (val) HIPCHECK(hipMemcpy(val, D.val, D.nnz * sizeof(double), hipMemcpyDeviceToHost));
            return IBPM_OK;
        }
        const CSR &K = c->m.K;
        *nnz = K.nnz();
        if (ptr) std::memcpy(ptr, K.ptr.data(), K.ptr.size() * sizeof(int32_t));
        if (col) std::memcpy(col, K.col.data(), K.col.size() * sizeof(int32_t));
        if (val) std::memcpy(val, K.val.data(), K.val.size() * sizeof(double));
        return IBPM_OK;
    });
}

int ibpm_bn_info(const ibpm_ctx *cc, int64_t *nnz_K, int64_t *nnz_B, int64_t *peak_bytes,
                 int64_t *unsliced_bytes) {
    ibpm_ctx *c = const_cast<ibpm_ctx *>(cc);
    return guarded(c, [&] {
        if (nnz_K) *nnz_K = c->moving ? c->K0c.nnz : c->m.K.nnz();
        if (nnz_B) *nnz_B = c->bn > 1 ? c->Bn.nnz : (int64_t)c->g.n_q;
        if (peak_bytes) *peak_bytes = c->bn_peak_bytes;
        if (unsliced_bytes) *unsliced_bytes = c->bn_unsliced_bytes;
        return IBPM_OK;
    });
}

int ibpm_move_body(ibpm_ctx *c, const double *xb, const double *yb, const double *ubx, const double *uby) {
    return guarded(c, [&] {
        need2d(c);
        move_body(c, xb, yb, ubx, uby);
        return IBPM_OK;
    });
}

int ibpm_moving_info(const ibpm_ctx *cc, int64_t *moves, int64_t *refreshes, int32_t *box) {
    ibpm_ctx *c = const_cast<ibpm_ctx *>(cc);
    return guarded(c, [&] {
        if (!c->moving) throw InvalidArg("the context was built for a fixed body (moving_body = 0)");
        if (moves) *moves = c->moves;
        if (refreshes) *refreshes = c->refreshes;
        if (box)
            for (int k = 0; k < 4; ++k) box[k] = c->box[k];
        return IBPM_OK;
    });
}

int ibpm_stage_walls(ibpm_ctx *c, const double *q) {
    return guarded(c, [&] {
        need2d(c);
        if (!q) throw InvalidArg("NULL vector");
        stage_walls(c, q);
        return IBPM_OK;
    });
}

int ibpm_stage_rhs1(ibpm_ctx *c, const double *q, const double *conv_prev, double *r1,
                    double *conv_now) {
    return guarded(c, [&] {
        need2d(c);
        if (!q || !conv_prev || !r1 || !conv_now) throw InvalidArg("NULL vector");
        stage_rhs1(c, q, conv_prev, r1, conv_now);
        return IBPM_OK;
    });
}

int ibpm_stage_rhs2(ibpm_ctx *c, const double *qstar, double *rhs) {
    return guarded(c, [&] {
        need2d(c);
        if (!qstar || !rhs) throw InvalidArg("NULL vector");
        stage_rhs2(c, qstar, rhs);
        return IBPM_OK;
    });
}

int ibpm_stage_project(ibpm_ctx *c, const double *qstar, const double *lam, double *qout) {
    return guarded(c, [&] {
        need2d(c);
        if (!qstar || !lam || !qout) throw InvalidArg("NULL vector");
        stage_project(c, qstar, lam, qout);
        return IBPM_OK;
    });
}

int ibpm_get_walls(ibpm_ctx *c, int32_t which, double *host) {
    return guarded(c, [&] {
        need2d(c);
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
        need2d(c);
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
        if (nnz) nnz[l] = c->moving ? c->level_nnz[l] : c->h.levels[l].A.nnz();
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

int ibpm_plan_hierarchy(const ibpm_params *p, int32_t cap, int32_t *levels, int64_t *sizes,
                        int64_t *nnz, double *rho, int32_t agg_level, int32_t *agg,
                        double *seconds, char *err, int32_t errlen) {
    auto report = [&](int code, const char *msg) {
        if (err && errlen > 0) {
            std::strncpy(err, msg, (size_t)errlen - 1);
            err[errlen - 1] = '\0';
        }
        return code;
    };
    try {
        check_params(p);
        if (p->poisson_solver == IBPM_SOLVER_JACOBI_PCG) throw InvalidArg("no hierarchy: the Poisson solver is Jacobi-PCG");
        if (p->bn_order > 1) throw InvalidArg("Q^T B^N Q with N > 1 is formed on the device: build a context");
        const auto t0 = std::chrono::steady_clock::now();
        Model m;
        try {
            build_model(m, p->nx, p->ny, p->xf, p->yf, p->nb, p->xb, p->yb, p->ubx, p->uby, p->nu, p->dt,
                        p->pin_cell);
        } catch (const std::runtime_error &e) {
            throw InvalidArg(e.what());
        }
        AmgParams ap;
        ap.theta = p->amg_theta;
        ap.coarse_max = p->amg_coarse_max;
        ap.max_levels = p->amg_max_levels;
        Hierarchy h;
        try {
            build_hierarchy(h, m.K, ap);
        } catch (const std::runtime_error &e) {
            throw InvalidArg(e.what());
        }
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        const int L = (int)h.levels.size();
        if (levels) *levels = L;
        if ((sizes || nnz || rho) && cap < L) throw InvalidArg("cap is below the level count");
        for (int l = 0; l < L; ++l) {
            if (sizes) sizes[l] = h.levels[l].A.nrows;
            if (nnz) nnz[l] = h.levels[l].A.nnz();
            if (rho) rho[l] = h.levels[l].rho;
        }
        if (agg) {
            if (agg_level < 0 || agg_level + 1 >= L) throw InvalidArg("agg_level out of range");
            const std::vector<int32_t> &a = h.levels[agg_level].agg;
            std::copy(a.begin(), a.end(), agg);
        }
        if (seconds) *seconds = secs;
        return report(IBPM_OK, "");
    } catch (const InvalidArg &e) {
        return report(IBPM_EINVAL, e.what());
    } catch (const std::bad_alloc &) {
        return report(IBPM_ENOMEM, "out of memory");
    } catch (const std::exception &e) {
        return report(IBPM_EINVAL, e.what());
    }
}

int ibpm_time_kernel(ibpm_ctx *c, int32_t kernel, int32_t reps, int64_t min_footprint, double *avg_ms,
                     double *bytes) {
    return guarded(c, [&] {
        need2d(c);
        if (reps < 1 || !avg_ms || min_footprint < 0) throw InvalidArg("bad arguments");
        if (c->stored0 && kernel != IBPM_KERNEL_A_PCG_SPMV && kernel != IBPM_KERNEL_STREAM_COPY &&
            kernel != IBPM_KERNEL_COPY_LEVEL0)
            throw InvalidArg("the level-0 kernels time the matrix-free operator of B^1 only");
        const bool needs_amg = kernel == IBPM_KERNEL_K0_JACOBI || kernel == IBPM_KERNEL_K0_RESIDUAL ||
                               kernel == IBPM_KERNEL_RESTRICT0 || kernel == IBPM_KERNEL_PROLONG0 ||
                               kernel == IBPM_KERNEL_COARSE_CYCLE || kernel == IBPM_KERNEL_PRESMOOTH0 ||
                               kernel == IBPM_KERNEL_UPDATE_PRESMOOTH0 || kernel == IBPM_KERNEL_L1_JACOBI ||
                               kernel == IBPM_KERNEL_PROLONG_POST0;
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
        st0.rz_next = 1.0;
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
        // Vector operands of the timed kernel: each is a slot with the
        // solver's own buffer; with min_footprint > 0 every slot gets one
        // copy per operand set, the sets together spanning at least
        // min_footprint bytes, and consecutive launches take consecutive sets
        // (so a launch finds none of its vectors in the caches).  Matrices,
        // aggregates, metrics and partial sums stay shared.
        std::vector<double *> own;
        std::vector<size_t> len;
        auto slot = [&](double *p, size_t cnt) {
            own.push_back(p);
            len.push_back(cnt);
            return (int)own.size() - 1;
        };
        int sets = 1;
        size_t per = 0;
        std::vector<size_t> off;
        double *pool = nullptr;
        auto at = [&](int sl, int k) -> double * {
            if (!pool) return own[sl];
            return pool + (size_t)(k % sets) * per + off[sl];
        };
        std::function<void(int)> launch;
        // every launch below captures its arguments by value (the slot
        // indices) and takes the buffers of set k through `at`: the lambda
        // runs after the switch, when block-scoped locals no longer exist
        const K0View K0 = K;
        double *parts = c->parts;
        switch (kernel) {
        case IBPM_KERNEL_K0_JACOBI: {
            const DevLevelT<double> &l0 = P.lev[0];
            const double omega = l0.omega;
            const int r = slot(P.r, n), xa = slot(l0.xa, n), xb = slot(l0.xb, n);
            launch = [=, &at](int k) { launch_k0_jacobi(s, K0, omega, at(r, k), at(xa, k), at(xb, k), sb); };
            by = 24.0 * n + b_coupling + b_metric;
            break;
        }
        case IBPM_KERNEL_K0_PCG_SPMV: {
            const int z = slot(P.z, n), p0 = slot(P.p[0], n), p1 = slot(P.p[1], n), q = slot(P.q, n);
            launch = [=, &at](int k) {
                launch_pcg_spmv(s, K0, at(z, k), at(p0, k), at(p1, k), at(q, k), sb, (const double *)nullptr, 0,
                                parts);
            };
            by = 32.0 * n + b_coupling + b_metric;
            break;
        }
        case IBPM_KERNEL_A_PCG_SPMV: {
            const AView A = c->A;
            const int z = slot(c->vz, nq), p0 = slot(c->vp[0], nq), p1 = slot(c->vp[1], nq), q = slot(c->vq, nq);
            launch = [=, &at](int k) {
                launch_pcg_spmv(s, A, at(z, k), at(p0, k), at(p1, k), at(q, k), sb, (const double *)nullptr, 0,
                                parts);
            };
            by = 32.0 * nq + b_metric;
            break;
        }
        case IBPM_KERNEL_K0_RESIDUAL: {
            const DevLevelT<double> &l0 = P.lev[0];
            const int r = slot(P.r, n), xa = slot(l0.xa, n), out = slot(l0.r, n);
            launch = [=, &at](int k) { launch_k0_residual(s, K0, at(r, k), at(xa, k), at(out, k), sb); };
            by = 24.0 * n + b_coupling + b_metric;
            break;
        }
        case IBPM_KERNEL_RESTRICT0: {
            const DevLevelT<double> &l0 = P.lev[0];
            const CSRView R0 = l0.R.view();
            const int b1 = slot(P.lev[1].b, P.lev[1].n);
            if (l0.RA.nrows > 0) {
                // the residual folded into the restriction: R b - (R A) x
                const CSRView RA0 = l0.RA.view();
                const int lanes = l0.RA.lanes;
                const int b0 = slot(P.r, n), x0 = slot(l0.xa, n);
                launch = [=, &at](int k) { launch_csrv_restrict(s, R0, RA0, lanes, at(b0, k), at(x0, k), at(b1, k), sb); };
                by = csr_bytes(l0.R, false) + csr_bytes(l0.RA, false) - 8.0 * l0.RA.nrows;
            } else {
                const int lanes = l0.R.lanes;
                const int r = slot(l0.r, n);
                launch = [=, &at](int k) { launch_csrv_spmv(s, R0, lanes, at(r, k), at(b1, k), false, sb); };
                by = csr_bytes(l0.R, false);
            }
            break;
        }
        case IBPM_KERNEL_PROLONG0: {
            const DevLevelT<double> &l0 = P.lev[0];
            const int *agg = l0.agg;
            const double w = l0.pomega;
            const int x1 = slot(P.lev[1].xa, P.lev[1].n), x0 = slot(l0.xa, n);
            launch = [=, &at](int k) { launch_k0_prolong_mf(s, K0, agg, at(x1, k), w, at(x0, k), sb); };
            // aggregates, x read and written, the coarse vector, coupling and metrics
            by = 4.0 * n + 16.0 * n + 8.0 * P.lev[1].n + b_coupling + b_metric;
            break;
        }
        case IBPM_KERNEL_PROLONG_POST0: {
            if (post2_rows(K0) == 0) throw InvalidArg("the prolongation + post-smoothing pass is off for this grid");
            const DevLevelT<double> &l0 = P.lev[0];
            const int *agg = l0.agg;
            const double pw = l0.pomega, omega = l0.omega;
            const int x1 = slot(P.lev[1].xa, P.lev[1].n), a = slot(l0.xa, n), tmp = slot(l0.xb, n),
                      tmp2 = slot(l0.r, n), r = slot(P.r, n), z = slot(P.z, n);
            launch = [=, &at](int k) {
                launch_k0_prolong_post2(s, K0, agg, (const double *)at(x1, k), pw, omega, (const double *)at(r, k),
                                        (const double *)at(a, k), at(tmp, k), at(tmp2, k), at(z, k), nullptr,
                                        nullptr, sb, parts, POST_RZ);
            };
            // aggregates, a and b read, z written, the coarse vector, the
            // coupling rows and the metrics (each once)
            by = 4.0 * n + 24.0 * n + 8.0 * P.lev[1].n + b_coupling + b_metric;
            break;
        }
        case IBPM_KERNEL_PCG_UPDATE_K: {
            const int x = slot(P.p[1], n), r = slot(P.r, n), z = slot(P.z, n), p0 = slot(P.p[0], n),
                      q = slot(P.q, n);
            // p . q partials for the update to sum: 1/G each, so p . q = 1 and the
            // status stays finite over the repetitions
            {
                const int G_pq = walk_blocks_of(K0);
                std::vector<double> ones(G_pq, 1.0 / G_pq);
                HIPCHECK(hipMemcpyAsync(c->parts2, ones.data(), G_pq * sizeof(double), hipMemcpyHostToDevice, s));
                HIPCHECK(hipStreamSynchronize(s));
            }
            const double *pq_parts = c->parts2;
            // as the AMG-PCG iteration launches it: alone, the stop test
            // deferred to the next product (the status never stops here)
            launch = [=, &at](int k) {
                launch_pcg_update(s, K0, at(x, k), at(r, k), at(z, k), at(p0, k), at(q, k), sb, pq_parts, parts,
                                  false, true, true);
            };
            by = 48.0 * n;
            break;
        }
        case IBPM_KERNEL_COARSE_CYCLE: {
            const int nlc = P.lev[P.lc].n;
            const double *C = P.coarseC;
            const int b = slot(P.lev[P.lc].b, nlc), x = slot(P.lev[P.lc].xa, nlc);
            launch = [=, &at](int k) { launch_coarse_dense(s, nlc, C, at(b, k), at(x, k), sb); };
            by = 8.0 * nlc * (double)nlc + 16.0 * nlc;
            break;
        }
        case IBPM_KERNEL_PRESMOOTH0: {
            const DevLevelT<double> &l0 = P.lev[0];
            const double *wd = l0.wdinv;
            const int r = slot(P.r, n), xa = slot(l0.xa, n);
            launch = [=, &at](int k) { launch_k0_presmooth2(s, K0, wd, at(r, k), at(xa, k), sb); };
            by = 24.0 * n + b_coupling + b_metric;
            break;
        }
        case IBPM_KERNEL_UPDATE_PRESMOOTH0: {
            const DevLevelT<double> &l0 = P.lev[0];
            const double *wd = l0.wdinv;
            const int x = slot(P.p[1], n), rin = slot(P.r, n), rout = slot(P.r2, n), p0 = slot(P.p[0], n),
                      q = slot(P.q, n), xs = slot(l0.xa, n);
            // p.q from the product's partials where a block gathers them,
            // else from the status (the solver finalizes it beforehand)
            const int G_pq = walk_blocks_of(K0);
            const bool gather = G_pq <= kFuseMaxParts;
            if (gather) {
                std::vector<double> ones(G_pq, 1.0 / G_pq);
                HIPCHECK(hipMemcpyAsync(c->parts2, ones.data(), G_pq * sizeof(double), hipMemcpyHostToDevice, s));
                HIPCHECK(hipStreamSynchronize(s));
            }
            const double *pq_parts = gather ? c->parts2 : nullptr;
            double *rr_parts = c->parts3;
            launch = [=, &at](int k) {
                launch_k0_update_presmooth2(s, K0, wd, at(x, k), at(rin, k), at(rout, k), at(p0, k), at(q, k),
                                            at(xs, k), sb, pq_parts, rr_parts);
            };
            // r, q, W, x, p read; r', x, x_s written
            by = 64.0 * n + b_coupling + b_metric;
            break;
        }
        case IBPM_KERNEL_L1_JACOBI: {
            if (P.lc < 2) throw InvalidArg("level 1 is part of the dense coarse cycle on this grid");
            const DevLevelT<double> &l1 = P.lev[1];
            const CSRView A1 = l1.A.view();
            const int lanes = l1.A.lanes, n1 = l1.n;
            const double *wd = l1.wdinv;
            const int b = slot(l1.b, n1), xa = slot(l1.xa, n1), xb = slot(l1.xb, n1);
            launch = [=, &at](int k) { launch_csrv_jacobi(s, A1, lanes, wd, at(b, k), at(xa, k), at(xb, k), sb); };
            // the operator, the damped inverse diagonal, b and x read, x written
            by = csr_bytes(l1.A, false) + 16.0 * n1;
            break;
        }
        case IBPM_KERNEL_STREAM_COPY: {
            const size_t nc = (size_t)1 << 25;
            if (!c->copy_x) {
                c->copy_x = c->dalloc<double>(nc);
                c->copy_y = c->dalloc<double>(nc);
                HIPCHECK(hipMemsetAsync(c->copy_x, 0, nc * sizeof(double), s));
            }
            const int x = slot(c->copy_x, nc), y = slot(c->copy_y, nc);
            launch = [=, &at](int k) { launch_stream_copy(s, nc, at(x, k), at(y, k)); };
            by = 16.0 * nc;
            break;
        }
        case IBPM_KERNEL_COPY_LEVEL0: {
            const size_t nc = (size_t)(n & ~1);
            const int x = slot(P.r, n), y = slot(P.z, n);
            launch = [=, &at](int k) { launch_stream_copy(s, nc, at(x, k), at(y, k)); };
            by = 16.0 * (double)nc;
            break;
        }
        default:
            throw InvalidArg("unknown kernel id");
        }
        for (size_t cnt : len) {
            off.push_back(per);
            per += (cnt + 31) / 32 * 32;   // 256-byte aligned slots
        }
        if (min_footprint > 0) {
            // at most 256 sets: a kernel whose vectors are that small is not
            // bound by HBM anyway
            sets = (int)std::min<int64_t>(256, std::max<int64_t>(2, (min_footprint + (int64_t)(8 * per) - 1) /
                                                                        (int64_t)(8 * per)));
            void *pp = nullptr;
            if (hipMalloc(&pp, (size_t)sets * per * sizeof(double)) != hipSuccess) throw std::bad_alloc();
            pool = (double *)pp;
            (void)hipMemsetAsync(pool, 0, (size_t)sets * per * sizeof(double), s);
            reps = std::max(reps, sets);
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        auto cleanup = [&] {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (pool) {
                (void)hipStreamSynchronize(s);
                (void)hipFree(pool);
                pool = nullptr;
            }
        };
        try {
            launch(0);   // warm the code object (and, with one set, the caches)
            HIPCHECK(hipEventCreate(&e0));
            HIPCHECK(hipEventCreate(&e1));
            HIPCHECK(hipEventRecord(e0, s));
            for (int k = 0; k < reps; ++k) launch(k + 1);
            HIPCHECK(hipEventRecord(e1, s));
            HIPCHECK(hipEventSynchronize(e1));
            float ms = 0;
            HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
            *avg_ms = ms / reps;
        } catch (...) {
            cleanup();
            throw;
        }
        cleanup();
        if (bytes) *bytes = by;
        return IBPM_OK;
    });
}

int ibpm_iteration_launches(const ibpm_ctx *cc, int32_t ncounts, int32_t *counts) {
    ibpm_ctx *c = const_cast<ibpm_ctx *>(cc);
    return guarded(c, [&] {
        if (!counts || ncounts < 0) throw InvalidArg("bad arguments");
        if (c->stored0) throw InvalidArg("launch counts are given for the matrix-free iteration only");
        PrecSet<double> &P = c->p64;
        if (!c->amg || P.lev.size() < 2) throw InvalidArg("needs an AMG hierarchy of two or more levels");
        int32_t k[IBPM_NUM_KERNELS] = {};
        const int pre = c->prm.amg_pre, post = c->prm.amg_post;
        // as pcg_drive and solve_poisson_fp64 decide: the update folds into
        // the first two sweeps (with one-block finalizes of p.q and of the
        // stop test around it where the partials exceed what a block gathers)
        const bool fuse = pre >= 2;
        k[IBPM_KERNEL_K0_PCG_SPMV] = 1;
        if (fuse) {
            k[IBPM_KERNEL_UPDATE_PRESMOOTH0] = 1;
        } else {
            k[IBPM_KERNEL_PCG_UPDATE_K] = 1;
            if (pre >= 2) k[IBPM_KERNEL_PRESMOOTH0] = 1;
        }
        // single sweeps on level 0: the pre-sweeps beyond the fused pair and
        // every post-sweep (the last one also forms r . z), unless the
        // prolongation and both post-sweeps go in one pass
        const bool post_fused = post == 2 && post2_rows(P.K0) > 0;
        k[IBPM_KERNEL_K0_JACOBI] = (pre >= 2 ? pre - 2 : pre) + (post_fused ? 0 : post);
        const DevLevelT<double> &l0 = P.lev[0];
        if (l0.RA.nrows == 0) k[IBPM_KERNEL_K0_RESIDUAL] = 1;
        k[IBPM_KERNEL_RESTRICT0] = 1;
        if (post_fused) k[IBPM_KERNEL_PROLONG_POST0] = 1;
        else k[IBPM_KERNEL_PROLONG0] = 1;
        k[IBPM_KERNEL_COARSE_CYCLE] = 1;
        if (P.lc >= 2) {
            // the plain sweeps of level 1: the pre-sweeps beyond the fused
            // pair and the post-sweeps (less the first where it carries the
            // prolongation)
            const DevLevelT<double> &l1 = P.lev[1];
            k[IBPM_KERNEL_L1_JACOBI] = (pre >= 2 ? pre - 2 : pre - 1) + (l1.AP.nrows > 0 ? post - 1 : post);
        }
        for (int i = 0; i < ncounts; ++i) counts[i] = i < IBPM_NUM_KERNELS ? k[i] : 0;
        return IBPM_OK;
    });
}

int ibpm_nn_init(ibpm_ctx *c, uint64_t seed) {
    return guarded(c, [&] {
        need2d(c);
        nn_alloc(c);
        nn_init_weights(c, seed);
        HIPCHECK(hipStreamSynchronize(c->stream));
        return IBPM_OK;
    });
}

int ibpm_nn_get_weights(ibpm_ctx *c, float *host, int64_t n) {
    return guarded(c, [&] {
        if (!c->nn.ready) throw InvalidArg("network not initialised");
        if (!host || n != nn_param_count()) throw InvalidArg("wrong weight count");
        nn_get_master(c, host);
        return IBPM_OK;
    });
}

int ibpm_nn_set_weights(ibpm_ctx *c, const float *host, int64_t n) {
    return guarded(c, [&] {
        need2d(c);
        if (!host || n != nn_param_count()) throw InvalidArg("wrong weight count");
        nn_alloc(c);
        nn_set_master(c, host);
        HIPCHECK(hipStreamSynchronize(c->stream));
        return IBPM_OK;
    });
}

int ibpm_nn_layer(ibpm_ctx *c, int32_t layer, int32_t mode, const float *x, const float *dy,
                  const float *mask, float *out) {
    return guarded(c, [&] {
        need2d(c);
        NNState &N = c->nn;
        if (!N.ready) throw InvalidArg("network not initialised");
        if (layer < 0 || layer >= kNNLayers || mode < 0 || mode > 2 || !out) throw InvalidArg("bad arguments");
        if ((mode != 1 && !x) || (mode != 0 && !dy)) throw InvalidArg("missing operand");
        hipStream_t s = c->stream;
        const int cin = N.cin[layer];
        bf16 *xb = N.act[1], *mb = mask ? N.act[2] : nullptr;
        if (x) launch_to_bf16(s, img(N, cin), x, xb);
        if (mask) launch_to_bf16(s, img(N, 32), mask, mb);
        if (mode == 0) {
            if (cin == kNNInPad) launch_conv3x3<bf16, kNNInPad>(s, N.H, N.W, xb, nullptr, N.fwd[layer], out, nullptr, 0);
            else launch_conv3x3<bf16, 32>(s, N.H, N.W, xb, nullptr, N.fwd[layer], out, nullptr, 0);
        } else if (mode == 1) {
            launch_conv3x3<float, 32>(s, N.H, N.W, dy, mb, N.bwd[layer], out, nullptr, 0);
        } else {
            nn_alloc_training(c);
            const int blocks = conv_dw_blocks(N.H, N.W);
            if (cin == kNNInPad) launch_conv3x3_dw<kNNInPad>(s, N.H, N.W, xb, dy, mb, N.partials);
            else launch_conv3x3_dw<32>(s, N.H, N.W, xb, dy, mb, N.partials);
            HIPCHECK(hipMemsetAsync(N.grad[layer], 0, (size_t)32 * N.kp[layer] * sizeof(float), s));
            launch_dw_reduce(s, blocks, 32 * N.kp[layer], N.partials, N.grad[layer]);
            std::vector<float> mst((size_t)32 * N.kp[layer]);
            HIPCHECK(hipMemcpyAsync(mst.data(), N.grad[layer], mst.size() * sizeof(float), hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
            const int ci = nn_cin_real(layer), co = nn_cout_real(layer);
            std::vector<float> pt((size_t)co * ci * 9);
            for (int o = 0; o < co; ++o)
                for (int cc = 0; cc < ci; ++cc)
                    for (int t = 0; t < 9; ++t) pt[((size_t)o * ci + cc) * 9 + t] = mst[(size_t)o * N.kp[layer] + t * cin + cc];
            HIPCHECK(hipMemcpyAsync(out, pt.data(), pt.size() * sizeof(float), hipMemcpyHostToDevice, s));
        }
        HIPCHECK(hipStreamSynchronize(s));
        return IBPM_OK;
    });
}

int ibpm_nn_apply(ibpm_ctx *c, const double *r, double *e) {
    return guarded(c, [&] {
        need2d(c);
        if (!c->nn.ready) throw InvalidArg("network not initialised");
        if (!r || !e) throw InvalidArg("NULL vector");
        nn_apply(c, r, e);
        return IBPM_OK;
    });
}

int ibpm_nn_train(ibpm_ctx *c, const float *r1, const float *e1, int32_t nsamples,
                  const int32_t *order, int32_t norder, int32_t batch, float lr, double *mean_loss) {
    return guarded(c, [&] {
        need2d(c);
        if (!c->nn.ready) throw InvalidArg("network not initialised");
        if (!r1 || !e1 || !order || nsamples < 1 || norder < 1 || batch < 1 || !(lr > 0))
            throw InvalidArg("bad arguments");
        double l = nn_train(c, r1, e1, nsamples, order, norder, batch, lr);
        if (mean_loss) *mean_loss = l;
        return IBPM_OK;
    });
}

int ibpm_nn_adam_step(ibpm_ctx *c, const float *grad, float lr) {
    return guarded(c, [&] {
        need2d(c);
        NNState &N = c->nn;
        if (!N.ready) throw InvalidArg("network not initialised");
        if (!grad || !(lr > 0)) throw InvalidArg("bad arguments");
        nn_alloc_training(c);
        // the gradient into the padded master layout (zeros in the padding,
        // where the update is then zero as well)
        int64_t off = 0;
        for (int l = 0; l < kNNLayers; ++l) {
            std::vector<float> g((size_t)32 * N.kp[l], 0.0f);
            const int ci = nn_cin_real(l), co = nn_cout_real(l);
            for (int o = 0; o < co; ++o)
                for (int cc = 0; cc < ci; ++cc)
                    for (int t = 0; t < 9; ++t)
                        g[(size_t)o * N.kp[l] + t * N.cin[l] + cc] = grad[off + ((int64_t)o * ci + cc) * 9 + t];
            off += (int64_t)co * ci * 9;
            HIPCHECK(hipMemcpyAsync(N.grad[l], g.data(), g.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
            HIPCHECK(hipStreamSynchronize(c->stream));
        }
        N.adam_t += 1;
        for (int l = 0; l < kNNLayers; ++l)
            launch_adam(c->stream, 32 * N.kp[l], N.master[l], N.grad[l], N.m[l], N.v[l], N.adam_t, lr, 0.9f,
                        0.999f, 1e-8f);
        nn_pack(c);
        HIPCHECK(hipStreamSynchronize(c->stream));
        return IBPM_OK;
    });
}

int ibpm_nn_loss_grad(ibpm_ctx *c, const float *r1, const float *e1, double *loss, float *grad) {
    return guarded(c, [&] {
        need2d(c);
        NNState &N = c->nn;
        if (!N.ready) throw InvalidArg("network not initialised");
        if (!r1 || !e1 || !loss || !grad) throw InvalidArg("NULL argument");
        nn_alloc_training(c);
        if (N.max_losses < 1) {
            N.losses = c->dalloc<double>(1);
            N.max_losses = 1;
        }
        for (int l = 0; l < kNNLayers; ++l)
            HIPCHECK(hipMemsetAsync(N.grad[l], 0, (size_t)32 * N.kp[l] * sizeof(float), c->stream));
        nn_sample_grad(c, r1, e1, N.losses);
        HIPCHECK(hipMemcpyAsync(loss, N.losses, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        nn_get_grads(c, grad);
        return IBPM_OK;
    });
}

int ibpm_harvest(ibpm_ctx *c, const double *rhs, double *x, const double *xstar, int32_t npairs,
                 float *r1_out, float *e1_out, int32_t *nout) {
    return guarded(c, [&] {
        need2d(c);
        if (!c->amg) throw InvalidArg("harvesting needs an AMG context");
        if (!rhs || !x || !xstar || !r1_out || !e1_out || npairs < 1) throw InvalidArg("bad arguments");
        hipStream_t s = c->stream;
        PrecSet<double> &P = c->p64;
        const K0View &K = P.K0;
        const int n = K.n;
        SolveStatus *st = c->st_poi;
        const double rtol = c->prm.poisson_rtol;
        launch_pcg_init(s, K, rhs, (const double *)x, P.r, (double *)nullptr, st, c->parts, false, rtol * rtol, c->prm.poisson_maxit);
        enqueue_vcycle(c, P, (const double *)P.r, P.z, st);
        int k = 0, curp = 0;
        for (; k < npairs; ++k) {
            c->read_status(st);
            if (c->host_st->done != ST_RUNNING) break;
            // r1 = r - K V(r) (FP32) and e1 = x* - x - V(r)
            launch_outer_residual(s, K, P.r, P.z, r1_out + (size_t)k * n, c->st_bench, c->parts, 1);
            launch_harvest_e1(s, n, xstar, x, P.z, e1_out + (size_t)k * n);
            launch_pcg_spmv(s, K, (const double *)P.z, (const double *)P.p[curp], P.p[1 - curp], P.q, st,
                            (const double *)c->parts, c->rz_G, c->parts2);
            curp = 1 - curp;
            launch_pcg_update(s, K, x, P.r, (double *)nullptr, (const double *)P.p[curp], (const double *)P.q, st,
                              (const double *)c->parts2, c->parts, false, true);
            enqueue_vcycle(c, P, (const double *)P.r, P.z, st);
        }
        HIPCHECK(hipStreamSynchronize(s));
        if (nout) *nout = k;
        return IBPM_OK;
    });
}

}  // extern "C"
