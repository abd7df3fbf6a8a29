// big_internal.h - arguments of the large-sub-aperture (FFT 512) passes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace shw {

struct BigLaunch {
  const float* opd;
  int64_t row_pitch, wfs_stride, frame_stride;
  const int32_t* valid_idx;
  float* slopes;
  float* images;
  uint8_t* flags;
  int32_t n_valid, n_wfs, n_subap, npx, det_n, pad0;
  double inv_lambda;
  float r2_outer, r2_inner, half_n;
  float ph_scale, ron, thr;
  int32_t noise;
  uint32_t key0, key1, frame0;
  const FrameWork* list;  // nullable: per-frame buffers and keys
};

bool big_shape_supported(int npx, int fft_n, int conv_n, int det_n, int lgs);

// Items [item0, item0 + nitems): T holds nitems * npx * 512 complex, Jr nitems * det_n * 512 floats.
hipError_t launch_big(const BigLaunch& a, int64_t item0, int64_t nitems, float2* T, float* Jr, hipStream_t st);

}  // namespace shw
