// mfma_internal.h - constants of the MFMA (precision-form) measurement.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace shw {

constexpr int kPrecBf16 = 1;
constexpr int kPrecBf16x3 = 2;
constexpr int kPrecFp16x3 = 3;

// Constant matrices, in 16x16 tiles, in B-operand lane order: entry (tile, lane) holds the
// four values M[16 b + 4 (lane / 16) + r][16 c + lane % 16], r = 0..3, as hi halves (8 bytes)
// then lo halves (8 bytes).  Tile offsets:
constexpr int kTabWr = 0;       // W^T real, 16 x 48 (3 tiles); W[u][x] = exp(-2 pi i (u - 39/2) x / 40)
constexpr int kTabWi = 3;       // W^T imaginary
constexpr int kTabWiNeg = 6;    // -W^T imaginary
constexpr int kTabC = 9;        // cos(2 pi k v / 40), 48 x 48 (9 tiles)
constexpr int kTabS = 18;       // sin(2 pi k v / 40)
constexpr int kTabSNeg = 27;    // -sin
constexpr int kTabWb = 36;      // rebin Wb^T, 48 x 16 (3 tiles)
constexpr int kMfmaTableTiles = 39;

bool mfma_shape_supported(int npx, int fft_n, int conv_n, int det_n, int prec);
hipError_t launch_wfs_mfma(int prec, bool lgs, const WfsLaunch& a, const uint2* tables, hipStream_t st);

}  // namespace shw
