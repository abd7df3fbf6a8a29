// mfma_internal.h - constants of the MFMA (precision-form) measurement.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace shw {

constexpr int kPrecBf16 = 1;
constexpr int kPrecBf16x3 = 2;
constexpr int kPrecFp16x3 = 3;

// Constant matrices, in 16x16 tiles, in B-operand lane order: lane `lane` of a tile owns the
// four values M[16 b + 4 (lane / 16) + r][16 c + lane % 16], r = 0..3, each split into a hi and
// a lo half.  N = 40, c0 = 39/2; in-band column j < 19 stands for the frequency k(j) = j (j <= 9)
// or j - 19 (j >= 10); rows and columns beyond a matrix are zero.
constexpr int kTabWr = 0;       // W^T, 16 x 48 (3 tiles): W^T[x][u] = exp(-2 pi i (u - c0) x / N), x < 10
constexpr int kTabWi = 3;
constexpr int kTabWiNeg = 6;
constexpr int kTabDr = 9;       // D^T, 48 x 32 (3 x 2 tiles): D^T[v][j] = exp(-2 pi i k(j) v / N)
constexpr int kTabDi = 15;
constexpr int kTabDiNeg = 21;
constexpr int kTabMvr = 27;     // Mv^T, 16 x 16: Mv^T[j][p] = c_j (1/N) sum_v Wb[p][v] exp(2 pi i k(j) v / N),
constexpr int kTabMvi = 28;     //   j < 10, c_0 = 1, c_j = 2 (the rows of negative frequency folded in)
constexpr int kTabMviNeg = 29;
constexpr int kTabMur = 30;     // Mu^T, 32 x 16 (2 tiles): Mu^T[j][q] = (1/N) sum_u Wb[q][u] exp(2 pi i k(j) u / N)
constexpr int kTabMuiNeg = 32;
constexpr int kMfmaTableTiles = 34;

// The table the kernels read holds ready B operands of the 16x16x32 products: operand `op` of
// lane `lane` is the 16-byte entry op * 64 + lane, the 4 halves of one tile part followed by the
// 4 halves of another, so that each operand is one LDS read into consecutive registers.
// [A|B] hi = (A hi, B hi); a hi operand is always followed by its lo operand.
constexpr int kOpW = 0;      // + 4 c (c < 3): [Wr|WiNeg] hi, lo; [Wi|Wr] hi, lo of column tile c
constexpr int kOpD = 12;     // + 4 t (t = 2 tb + tc < 6): [Dr|DiNeg] hi, lo; [Di|Dr] hi, lo
constexpr int kOpDre = 36;   // + tv (tv < 3): (Dr lo, Dr hi) of tile 2 tv; + 3 + tv: (Di lo, Di hi)
constexpr int kOpMv = 42;    // [Mvr|MviNeg] hi, lo; [Mvi|Mvr] hi, lo
constexpr int kOpMu = 46;    // + 2 tb (tb < 2): [Mur|MuiNeg] hi, lo
constexpr int kMfmaOps = 50;

bool mfma_shape_supported(int npx, int fft_n, int conv_n, int det_n, int prec);
// Detector values of items [a.item0, a.total) into a.det_ws (chunks of a.det_ws_items items), each
// chunk followed by det_noise_kernel (photometry, noise, centroid).
hipError_t launch_wfs_mfma(int prec, bool lgs, const WfsLaunch& a, const uint4* ops, hipStream_t st);

}  // namespace shw
