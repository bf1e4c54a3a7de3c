// Residual-to-correction network: 3x3 convolutions on the cell grid with
// BF16 operands and FP32 accumulation on the gfx950 matrix cores.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <stdexcept>

#include "kernels.h"

namespace ibpm {

using bf16 = __bf16;

constexpr int kNNLayers = 6;
constexpr int kNNWidth = 32;        // hidden channels (and padded output channels)
constexpr int kNNIn = 5;            // input channels (padded to 8)
constexpr int kNNInPad = 8;
constexpr int kNNOut = 3;           // output channels (padded to 32)
constexpr int kConvTile = 128;      // pixels of one image row per block (4 waves x 32)
constexpr int kConvRows = 4;        // image rows per block of the convolution

// K of the implicit GEMM padded to the MFMA step (16)
__host__ __device__ constexpr int conv_kp(int cin) { return ((9 * cin + 15) / 16) * 16; }

// Cell-centre delta weights between Lagrangian points and cells (for the
// force channels): both directions as CSR (cells of the box -> points and
// points -> cells), weights phi((xc - xi)/h) phi((yc - eta)/h).
struct CellDelta {
    int i0, i1, j0, j1;         // box of cells
    CSRView c2p;                // box cell -> (point, weight)
    CSRView p2c;                // point -> (cell index, weight)
};

// One 3x3 convolution layer: Y = conv(X, W) on an H x W image, HWC layout.
//   X      input, CIN channels (8 or 32), BF16 (TIn = bf16) or FP32 (TIn = float)
//   mask   optional BF16 [H][W][CIN]; where mask <= 0 the input is read as 0
//          (the ReLU derivative in the backward pass)
//   Wp     packed weights [32][conv_kp(CIN)] BF16 (out channel major, k = tap*CIN + c)
//   Y32    optional FP32 [H][W][ys] pre-activation output (output channels
//          0 .. ys-1; ys = 32 keeps them all, the network's last layer at
//          inference keeps its kNNOut channels in rows of 4)
//   Y16    optional BF16 [H][W][32] output after ReLU (relu != 0) or as is
template <class TIn, int CIN>
void launch_conv3x3(hipStream_t s, int H, int W, const TIn *X, const bf16 *mask, const bf16 *Wp,
                    float *Y32, bf16 *Y16, int relu, int ys = 32);

// Weight gradient of one layer for one image: per-block partials
// [blocks][32][kp] of dW[n][k] = sum_p dY[p][n] X[p + tap][c]; dY is FP32
// [H][W][32] masked by `mask` (BF16 [H][W][32], > 0 keeps) when given.
template <int CIN>
void launch_conv3x3_dw(hipStream_t s, int H, int W, const bf16 *X, const float *dY,
                       const bf16 *mask, float *partials);
int conv_dw_blocks(int H, int W);
// grad[n][k] += sum over blocks of partials (fixed order)
void launch_dw_reduce(hipStream_t s, int blocks, int nk, const float *partials, float *grad);

// Master FP32 weights [32][kp] -> BF16 packed forward weights and the
// flipped / transposed weights used by the input-gradient convolution.
void launch_pack_weights(hipStream_t s, int cin, int cout, const float *master, bf16 *fwd,
                         bf16 *bwd);

// y = BF16(x), n values
void launch_to_bf16(hipStream_t s, size_t n, const float *x, bf16 *y);

// Adam step on n FP32 parameters (bias-corrected, step t >= 1)
void launch_adam(hipStream_t s, int n, float *w, const float *g, float *m, float *v, int t,
                 float lr, float beta1, float beta2, float eps);

// RMS scale of a lambda vector: scale[0] = sqrt(sum r^2 / n) (1 if zero);
// parts needs 1024 doubles
template <class T>
void launch_nn_scale(hipStream_t s, int n, const T *r, double *parts, double *scale);

// features: residual r (lambda layout) scaled by 1/scale -> X [H][W][8] BF16
//   ch0 pressure residual, ch1/ch2 force residuals spread to cell centres,
//   ch3/ch4 log of the cell widths over the finest width, ch5-7 zero
template <class T>
void launch_nn_features(hipStream_t s, GridView g, int nb, const T *r, const double *scale,
                        double inv_hmin, CellDelta cd, bf16 *X);
// network output Y32 [H][W][ys] -> correction e (lambda layout, T) times
// scale/dt: pressure from channel 0, forces interpolated from channels 1, 2
template <class T>
void launch_nn_output(hipStream_t s, int n_cell, int nb, const float *Y32, const double *scale,
                      double inv_dt, CellDelta cd, T *e, int ys = 32);
// training loss of the correction d = output map of Y32 for the pair (r1,
// e1) (FP32, lambda layout, K e1 = r1): the share of the energy-norm error
// that the optimally scaled d removes, -(d.r1)^2 / ((d.Kd)(r1.e1)), into
// st->rr, and dL/dY32 into dY ([H][W][32] FP32).  d and Kd are FP64 work
// vectors of n entries; parts holds 3 x 1024 partial sums.
void launch_nn_energy_loss(hipStream_t s, const K0View &K, int nb, const float *Y32,
                           const float *r1, const float *e1, const double *scale, double dt,
                           CellDelta cd, double *d, double *Kd, float *dY, double *parts,
                           SolveStatus *st);

}  // namespace ibpm
