// psf_internal.h - PSF kernel arguments shared by the host library and psf_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shw {

struct PsfLaunch {
  const float* opd;        // OPD metres, star s frame f at opd + s * star_stride + f * frame_stride
  int64_t row_pitch, frame_stride, star_stride;
  int64_t acc_stride;      // accumulator of star s at acc + s * acc_stride
  int32_t n_frames;        // frames per star in the call (Strehl index s * n_frames + f)
  int32_t pupil_n, pad0;
  double inv_lambda;
  float r2_outer, r2_inner, half_n;
  float inv_norm;          // 1 / (sum A)^2
};

bool psf_size_supported(int fft_m, int pupil_n);

// Row pass over frames [f0, f0 + nf) of stars [0, n_stars) into T (n_stars * nf * pupil_n * fft_m
// complex), and the column pass that reads T and adds the frames' PSFs to the accumulators.
hipError_t launch_psf_rows(const PsfLaunch& a, int n_stars, int64_t f0, int nf, float2* T, hipStream_t st);
hipError_t launch_psf_cols(const PsfLaunch& a, int n_stars, int64_t f0, int nf, const float2* T, float* acc,
                           float* strehl, hipStream_t st);

}  // namespace shw
