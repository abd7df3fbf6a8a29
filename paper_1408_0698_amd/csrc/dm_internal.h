// dm_internal.h - DM surface and residual kernel arguments.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shw {

constexpr int kMaxDm = 4;
constexpr int kResidualChunk = 32;  // outputs per launch (origins travel in the kernel arguments)

struct DmLaunch {
  const int* grid;   // [(2m+1)^2] actuator index of grid cell (gy, gx), -1 if none; device
  int32_t m;         // grid indices run over [-m, m]
  int32_t pitch;     // pixels
  int32_t size;      // surface side
  int32_t half_patch;
  float inv_2s2;     // 1 / (2 sigma^2)
};

struct ResidualLaunch {
  const float* screen;
  int64_t screen_pitch;
  const float* surf[kMaxDm];
  int32_t surf_size[kMaxDm];
  int32_t n_dm;
  int32_t pupil_n;
  int32_t scr_origin[kResidualChunk][2];
  int32_t dm_origin[kResidualChunk][kMaxDm][2];
  int64_t out_pitch, out_stride;
};

hipError_t launch_dm_surface(const DmLaunch& a, const float* coefs, float* surf, hipStream_t st);

// out[k][y][x] = amp[k] * IF of actuator act[k] at surface pixel (row0 + y, col0 + x); act_xy [n_act][2] device.
struct InfluenceLaunch {
  const float* act_xy;   // (x, y) pixels from the DM centre, FP32, device
  const int32_t* act;    // [n] actuator indices, device
  const float* amp;      // [n] amplitudes, device
  int32_t n, n_act, size, half_patch, row0, col0, pupil_n, pad0;
  float inv_2s2;
  int64_t out_pitch, out_stride;
};
hipError_t launch_influence_opd(const InfluenceLaunch& a, float* out, hipStream_t st);

// im[s * ld + m] = (slopes[2m][s] - slopes[2m+1][s]) * scale for m < n_modes, s < n_slopes.
hipError_t launch_push_pull(const float* slopes, int32_t n_modes, int32_t n_slopes, float scale, float* im,
                            int64_t ld, hipStream_t st);
hipError_t launch_residual(const ResidualLaunch& a, int n_out, float* out, hipStream_t st);

}  // namespace shw
