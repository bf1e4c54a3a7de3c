// Residual-to-correction network on the matrix cores of gfx950.
//
// A 3x3 convolution is an implicit GEMM: M = pixels, N = output channels
// (32), K = 9 taps x input channels.  One block takes 128 pixels of one image
// row (4 waves x 32 pixels); the three input rows it needs (with a one-pixel
// halo, zero outside the image) and the packed weights are staged in LDS,
// and every wave accumulates its 32 x 32 output tile with
// v_mfma_f32_32x32x16_bf16 (BF16 operands, FP32 accumulation), 16 of K per
// instruction.  Operand layout of that instruction (checked on the device):
// lane l supplies A[l % 32][8 (l / 32) + i] and B[8 (l / 32) + i][l % 32],
// i = 0..7, and receives C[8 (j / 4) + 4 (l / 32) + j % 4][l % 32] in its
// j-th accumulator.  The weight gradient is the GEMM dW[n][k] = sum_p
// dY[p][n] X[p + tap][c] with K = pixels: each block writes its 32 x K_pad
// partial and a reduction kernel adds the blocks in a fixed order, so
// training is deterministic.
#include "nn.h"

namespace ibpm {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kTW = kConvTile + 2;      // staged row width with halo
constexpr int kDS = kConvTile + 8;      // row stride of the transposed dY tile

__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(__bf16 v) { return (float)v; }

// stage NR image rows from ytop, pixels x0-1..x0+128 of an H x W x CIN image
// into LDS (zero outside the image; where mask <= 0 the value is taken as 0)
template <class TIn, int CIN, int NR>
__device__ __forceinline__ void stage_rows(__bf16 *xs, const TIn *X, const __bf16 *mask, int H,
                                           int W, int x0, int ytop) {
    constexpr int CH = CIN / 8;
    for (int e = threadIdx.x; e < NR * kTW * CH; e += kBlock) {
        int dy = e / (kTW * CH);
        int rem = e - dy * kTW * CH;
        int px = rem / CH;
        int cg = rem - px * CH;
        int gy = ytop + dy, gx = x0 + px - 1;
        bf16x8 v;
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = (__bf16)0.0f;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
            size_t base = ((size_t)gy * W + gx) * CIN + cg * 8;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                float f = to_f(X[base + k]);
                if (mask && (float)mask[base + k] <= 0.0f) f = 0.0f;
                v[k] = (__bf16)f;
            }
        }
        *(bf16x8 *)&xs[(dy * kTW + px) * CIN + cg * 8] = v;
    }
}

// One block: 128 pixels x kConvRows rows.  Each wave keeps the B fragments
// of every K step (its 32 x K_pad slice of the weights) in registers for all
// the rows of the tile; the input rows with their halo are staged once.
template <class TIn, int CIN>
__global__ __launch_bounds__(kBlock) void k_conv3x3(int H, int W, const TIn *X, const __bf16 *mask,
                                                    const __bf16 *Wp, float *Y32, __bf16 *Y16,
                                                    int relu, int ys) {
    constexpr int KP = conv_kp(CIN);
    constexpr int NS = KP / 16;
    __shared__ __attribute__((aligned(16))) __bf16 xs[(kConvRows + 2) * kTW * CIN];
    const int x0 = blockIdx.x * kConvTile, y0 = blockIdx.y * kConvRows;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int kh = (l >> 5) * 8;
    bf16x8 bw[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) bw[s] = *(const bf16x8 *)&Wp[(l & 31) * KP + s * 16 + kh];
    stage_rows<TIn, CIN, kConvRows + 2>(xs, X, mask, H, W, x0, y0 - 1);
    __syncthreads();
    const int pl = w * 32 + (l & 31);
    const int n = l & 31;
    for (int r = 0; r < kConvRows; ++r) {
        const int y = y0 + r;
        if (y >= H) break;
        f32x16 acc;
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = 0.0f;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int k0 = s * 16 + kh;
            const int tap = k0 / CIN, c0 = k0 - tap * CIN;
            bf16x8 a;
            if (tap < 9) {
                const int dy = tap / 3, dx = tap - dy * 3;
                a = *(const bf16x8 *)&xs[((r + dy) * kTW + pl + dx) * CIN + c0];
            } else {
#pragma unroll
                for (int k = 0; k < 8; ++k) a[k] = (__bf16)0.0f;
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bw[s], acc, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int p = w * 32 + 8 * (j >> 2) + 4 * (l >> 5) + (j & 3);
            const int gx = x0 + p;
            if (gx < W) {
                const size_t px = (size_t)y * W + gx;
                const float v = acc[j];
                if (Y32 && n < ys) Y32[px * ys + n] = v;
                if (Y16) Y16[px * 32 + n] = (__bf16)(relu ? fmaxf(v, 0.0f) : v);
            }
        }
    }
}

template <int CIN>
__global__ __launch_bounds__(kBlock) void k_conv3x3_dw(int H, int W, const __bf16 *X,
                                                       const float *dY, const __bf16 *mask,
                                                       float *partials) {
    constexpr int KP = conv_kp(CIN);
    constexpr int NC = (KP + 31) / 32;
    __shared__ __attribute__((aligned(16))) __bf16 xs[3 * kTW * CIN];
    __shared__ __attribute__((aligned(16))) __bf16 dyt[32 * kDS];
    const int x0 = blockIdx.x * kConvTile, y = blockIdx.y;
    stage_rows<__bf16, CIN, 3>(xs, X, nullptr, H, W, x0, y - 1);
    for (int e = threadIdx.x; e < kConvTile * 32; e += kBlock) {
        const int p = e >> 5, n = e & 31;
        const int gx = x0 + p;
        float v = 0.0f;
        if (gx < W) {
            const size_t o = ((size_t)y * W + gx) * 32 + n;
            v = dY[o];
            if (mask && (float)mask[o] <= 0.0f) v = 0.0f;
        }
        dyt[n * kDS + p] = (__bf16)v;
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const size_t blk = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    for (int cc = w; cc < NC; cc += 4) {
        const int kcol = cc * 32 + (l & 31);
        const bool kvalid = kcol < 9 * CIN;
        const int tap = kvalid ? kcol / CIN : 0;
        const int c = kcol - tap * CIN;
        const int dy = tap / 3, dx = tap - dy * 3;
        f32x16 acc;
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = 0.0f;
#pragma unroll
        for (int ks = 0; ks < kConvTile / 16; ++ks) {
            const int p0 = ks * 16 + (l >> 5) * 8;
            const bf16x8 a = *(const bf16x8 *)&dyt[(l & 31) * kDS + p0];
            bf16x8 b;
#pragma unroll
            for (int i = 0; i < 8; ++i)
                b[i] = kvalid ? xs[(dy * kTW + p0 + i + dx) * CIN + c] : (__bf16)0.0f;
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        const int col = cc * 32 + (l & 31);
        if (col < KP) {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int n = 8 * (j >> 2) + 4 * (l >> 5) + (j & 3);
                partials[blk * 32 * KP + n * KP + col] = acc[j];
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_dw_reduce(int blocks, int nk, const float *partials,
                                                      float *grad) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= nk) return;
    float s = 0.0f;
    for (int b = 0; b < blocks; ++b) s += partials[(size_t)b * nk + i];
    grad[i] += s;
}

// master [32][kp(cin)] (k = tap*cin + c) -> fwd BF16 same layout; bwd BF16
// [32][kp(32)] with bwd[c][(8 - tap)*32 + o] = master[o][tap*cin + c]
__global__ __launch_bounds__(kBlock) void k_pack_weights(int cin, const float *master, __bf16 *fwd,
                                                         __bf16 *bwd) {
    const int kpf = conv_kp(cin), kpb = conv_kp(32);
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < 32 * kpf) fwd[i] = (__bf16)master[i];
    if (bwd && i < 32 * kpb) {
        const int c = i / kpb, kb = i - c * kpb;
        float v = 0.0f;
        if (kb < 9 * 32 && c < cin) {
            const int tb = kb / 32, o = kb - tb * 32;
            const int tap = 8 - tb;
            v = master[o * kpf + tap * cin + c];
        }
        bwd[i] = (__bf16)v;
    }
}

__global__ __launch_bounds__(kBlock) void k_adam(int n, float *w, const float *g, float *m,
                                                 float *v, float b1t, float b2t, float lr,
                                                 float beta1, float beta2, float eps) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - b1t), vh = vi / (1.0f - b2t);
    w[i] -= lr * mh / (sqrtf(vh) + eps);
}

// sum of squares of a lambda vector (the RMS scale of the network input)
template <class T>
__global__ __launch_bounds__(kBlock) void k_sumsq(int n, const T *r, double *parts) {
    double v = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        v += (double)r[i] * (double)r[i];
    __shared__ double sh[kBlock];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kBlock) void k_scale_finalize(int G, int n, const double *parts,
                                                           double *scale) {
    __shared__ double sh[kBlock];
    double v = 0.0;
    for (int b = threadIdx.x; b < G; b += kBlock) v += parts[b];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double rms = sqrt(sh[0] / (double)n);
        scale[0] = rms > 0.0 ? rms : 1.0;
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_nn_features(GridView g, int nb, const T *r,
                                                        const double *scale, double inv_hmin,
                                                        CellDelta cd, __bf16 *X) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= g.n_cell) return;
    const int j = p / g.nx, i = p - j * g.nx;
    const double is = 1.0 / scale[0];
    double fx = 0.0, fy = 0.0;
    if (i >= cd.i0 && i <= cd.i1 && j >= cd.j0 && j <= cd.j1) {
        const int rb = (j - cd.j0) * (cd.i1 - cd.i0 + 1) + (i - cd.i0);
        for (int e = cd.c2p.ptr[rb]; e < cd.c2p.ptr[rb + 1]; ++e) {
            const int k = cd.c2p.col[e];
            const double wgt = cd.c2p.val[e];
            fx += wgt * (double)r[g.n_cell + k];
            fy += wgt * (double)r[g.n_cell + nb + k];
        }
    }
    bf16x8 v;
    v[0] = (__bf16)(float)((double)r[p] * is);
    v[1] = (__bf16)(float)(fx * is);
    v[2] = (__bf16)(float)(fy * is);
    v[3] = (__bf16)(float)log(g.dx[i] * inv_hmin);
    v[4] = (__bf16)(float)log(g.dy[j] * inv_hmin);
    v[5] = (__bf16)0.0f;
    v[6] = (__bf16)0.0f;
    v[7] = (__bf16)0.0f;
    *(bf16x8 *)&X[(size_t)p * 8] = v;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_nn_output(int n_cell, int nb, const float *Y32,
                                                      const double *scale, double inv_dt,
                                                      CellDelta cd, T *e, int ys) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const double sc = scale[0] * inv_dt;
    if (t < n_cell) {
        e[t] = (T)(sc * (double)Y32[(size_t)t * ys]);
    } else if (t < n_cell + 2 * nb) {
        const int k = t - n_cell;
        const int pk = k < nb ? k : k - nb;
        const int ch = k < nb ? 1 : 2;
        double s = 0.0;
        for (int q = cd.p2c.ptr[pk]; q < cd.p2c.ptr[pk + 1]; ++q)
            s += cd.p2c.val[q] * (double)Y32[(size_t)cd.p2c.col[q] * ys + ch];
        e[t] = (T)(sc * s);
    }
}

// Energy loss of a correction d (lambda layout, FP64) for a training pair
// (r1, e1) with K e1 = r1:  loss = -(d.r1)^2 / ((d.Kd)(r1.e1)).  Partial sums
// of d.r1, d.Kd and r1.e1 per block, then one block forms the loss and the
// two coefficients of its gradient  dL/dd = coef (r1 - ratio K d).
__global__ __launch_bounds__(kBlock) void k_energy_sums(int n, const double *d, const double *Kd,
                                                        const float *r1, const float *e1,
                                                        double *parts) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double ri = (double)r1[i];
        v[0] += d[i] * ri;
        v[1] += d[i] * Kd[i];
        v[2] += ri * (double)e1[i];
    }
    __shared__ double sh[3][kBlock];
    for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) parts[k * kMaxParts + blockIdx.x] = sh[k][0];
}

// st->rr = loss, st->beta = coef, st->pq = ratio (all 0 when d.Kd <= 0 or
// r1.e1 <= 0 or a sum is not finite)
__global__ __launch_bounds__(kBlock) void k_energy_finalize(int G, const double *parts,
                                                            SolveStatus *st) {
    __shared__ double sh[3][kBlock];
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < G; b += kBlock)
        for (int k = 0; k < 3; ++k) v[k] += parts[k * kMaxParts + b];
    for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double a = sh[0][0], b = sh[1][0], c = sh[2][0];
        const bool ok = b > 0.0 && c > 0.0 && isfinite(a) && isfinite(b) && isfinite(c);
        st->rr = ok ? -a * a / (b * c) : 0.0;
        st->beta = ok ? -2.0 * a / (b * c) : 0.0;
        st->pq = ok ? a / b : 0.0;
    }
}

// gd = coef (r1 - ratio K d), in place of d
__global__ __launch_bounds__(kBlock) void k_energy_grad(int n, const float *r1, const double *Kd,
                                                        const SolveStatus *st, double *gd) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) gd[i] = st->beta * ((double)r1[i] - st->pq * Kd[i]);
}

// dL/dY of the output map e = (s/dt) [Y0; D^T Y1; D^T Y2]:
// channel 0 = (s/dt) gd_cell, channels 1, 2 = (s/dt) D gd_force, others 0
__global__ __launch_bounds__(kBlock) void k_output_adjoint(GridView g, int nb, const double *gd,
                                                           const double *scale, double inv_dt,
                                                           CellDelta cd, float *dY) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= g.n_cell) return;
    const int j = p / g.nx, i = p - j * g.nx;
    const double sc = scale[0] * inv_dt;
    float out[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) out[k] = 0.0f;
    out[0] = (float)(sc * gd[p]);
    if (i >= cd.i0 && i <= cd.i1 && j >= cd.j0 && j <= cd.j1) {
        const int rb = (j - cd.j0) * (cd.i1 - cd.i0 + 1) + (i - cd.i0);
        double gx = 0.0, gy = 0.0;
        for (int e = cd.c2p.ptr[rb]; e < cd.c2p.ptr[rb + 1]; ++e) {
            const int k = cd.c2p.col[e];
            gx += cd.c2p.val[e] * gd[g.n_cell + k];
            gy += cd.c2p.val[e] * gd[g.n_cell + nb + k];
        }
        out[1] = (float)(sc * gx);
        out[2] = (float)(sc * gy);
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) dY[(size_t)p * 32 + k] = out[k];
}

__global__ __launch_bounds__(kBlock) void k_to_bf16(size_t n, const float *x, __bf16 *y) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = (__bf16)x[i];
}

}  // namespace

#define LAUNCH(kernel, grid, ...) hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, __VA_ARGS__)

template <class TIn, int CIN>
void launch_conv3x3(hipStream_t s, int H, int W, const TIn *X, const bf16 *mask, const bf16 *Wp,
                    float *Y32, bf16 *Y16, int relu, int ys) {
    if (ys < 1 || ys > 32) throw std::runtime_error("conv3x3: bad channel stride of the FP32 output");
    dim3 grid((W + kConvTile - 1) / kConvTile, (H + kConvRows - 1) / kConvRows);
    hipLaunchKernelGGL((k_conv3x3<TIn, CIN>), grid, dim3(kBlock), 0, s, H, W, X, mask, Wp, Y32, Y16,
                       relu, ys);
}

void launch_to_bf16(hipStream_t s, size_t n, const float *x, bf16 *y) {
    LAUNCH(k_to_bf16, (unsigned)((n + kBlock - 1) / kBlock), n, x, y);
}

int conv_dw_blocks(int H, int W) { return ((W + kConvTile - 1) / kConvTile) * H; }

template <int CIN>
void launch_conv3x3_dw(hipStream_t s, int H, int W, const bf16 *X, const float *dY,
                       const bf16 *mask, float *partials) {
    dim3 grid((W + kConvTile - 1) / kConvTile, H);
    hipLaunchKernelGGL((k_conv3x3_dw<CIN>), grid, dim3(kBlock), 0, s, H, W, X, dY, mask, partials);
}

void launch_dw_reduce(hipStream_t s, int blocks, int nk, const float *partials, float *grad) {
    LAUNCH(k_dw_reduce, (nk + kBlock - 1) / kBlock, blocks, nk, partials, grad);
}

void launch_pack_weights(hipStream_t s, int cin, int cout, const float *master, bf16 *fwd,
                         bf16 *bwd) {
    (void)cout;
    int n = 32 * (conv_kp(cin) > conv_kp(32) ? conv_kp(cin) : conv_kp(32));
    LAUNCH(k_pack_weights, (n + kBlock - 1) / kBlock, cin, master, fwd, bwd);
}

void launch_adam(hipStream_t s, int n, float *w, const float *g, float *m, float *v, int t,
                 float lr, float beta1, float beta2, float eps) {
    float b1t = powf(beta1, (float)t), b2t = powf(beta2, (float)t);
    LAUNCH(k_adam, (n + kBlock - 1) / kBlock, n, w, g, m, v, b1t, b2t, lr, beta1, beta2, eps);
}

template <class T>
void launch_nn_scale(hipStream_t s, int n, const T *r, double *parts, double *scale) {
    int G = (n + kBlock - 1) / kBlock;
    if (G > 1024) G = 1024;
    LAUNCH((k_sumsq<T>), G, n, r, parts);
    LAUNCH(k_scale_finalize, 1, G, n, parts, scale);
}

template <class T>
void launch_nn_features(hipStream_t s, GridView g, int nb, const T *r, const double *scale,
                        double inv_hmin, CellDelta cd, bf16 *X) {
    LAUNCH((k_nn_features<T>), (g.n_cell + kBlock - 1) / kBlock, g, nb, r, scale, inv_hmin, cd, X);
}

template <class T>
void launch_nn_output(hipStream_t s, int n_cell, int nb, const float *Y32, const double *scale,
                      double inv_dt, CellDelta cd, T *e, int ys) {
    int n = n_cell + 2 * nb;
    if (ys < kNNOut || ys > 32) throw std::runtime_error("nn output: bad channel stride");
    LAUNCH((k_nn_output<T>), (n + kBlock - 1) / kBlock, n_cell, nb, Y32, scale, inv_dt, cd, e, ys);
}

void launch_nn_energy_loss(hipStream_t s, const K0View &K, int nb, const float *Y32,
                           const float *r1, const float *e1, const double *scale, double dt,
                           CellDelta cd, double *d, double *Kd, float *dY, double *parts,
                           SolveStatus *st) {
    const int n = K.n;
    launch_nn_output<double>(s, K.g.n_cell, nb, Y32, scale, 1.0 / dt, cd, d);
    launch_apply_K0(s, K, (const double *)d, Kd);
    int G = (n + kBlock - 1) / kBlock;
    if (G > 1024) G = 1024;
    LAUNCH(k_energy_sums, G, n, (const double *)d, (const double *)Kd, r1, e1, parts);
    LAUNCH(k_energy_finalize, 1, G, (const double *)parts, st);
    LAUNCH(k_energy_grad, (n + kBlock - 1) / kBlock, n, r1, (const double *)Kd,
           (const SolveStatus *)st, d);
    LAUNCH(k_output_adjoint, (K.g.n_cell + kBlock - 1) / kBlock, K.g, nb, (const double *)d, scale,
           1.0 / dt, cd, dY);
}

template void launch_conv3x3<bf16, 8>(hipStream_t, int, int, const bf16 *, const bf16 *,
                                      const bf16 *, float *, bf16 *, int, int);
template void launch_conv3x3<bf16, 32>(hipStream_t, int, int, const bf16 *, const bf16 *,
                                       const bf16 *, float *, bf16 *, int, int);
template void launch_conv3x3<float, 32>(hipStream_t, int, int, const float *, const bf16 *,
                                        const bf16 *, float *, bf16 *, int, int);
template void launch_conv3x3<float, 8>(hipStream_t, int, int, const float *, const bf16 *,
                                       const bf16 *, float *, bf16 *, int, int);
template void launch_conv3x3_dw<8>(hipStream_t, int, int, const bf16 *, const float *,
                                   const bf16 *, float *);
template void launch_conv3x3_dw<32>(hipStream_t, int, int, const bf16 *, const float *,
                                    const bf16 *, float *);
template void launch_nn_scale<double>(hipStream_t, int, const double *, double *, double *);
template void launch_nn_scale<float>(hipStream_t, int, const float *, double *, double *);
template void launch_nn_features<double>(hipStream_t, GridView, int, const double *,
                                         const double *, double, CellDelta, bf16 *);
template void launch_nn_features<float>(hipStream_t, GridView, int, const float *,
                                        const double *, double, CellDelta, bf16 *);

template void launch_nn_output<double>(hipStream_t, int, int, const float *, const double *, double,
                                       CellDelta, double *, int);
template void launch_nn_output<float>(hipStream_t, int, int, const float *, const double *, double,
                                      CellDelta, float *, int);

}  // namespace ibpm
