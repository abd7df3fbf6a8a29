// dm_kernels.hip - DM surfaces and residual OPD (Sec. 3 closed-loop block: residual =
// open-loop wavefront minus the DM; Sec. 2 DM mode counts; analytic influence functions).
//
// Surface: gather form, one lane per surface pixel.  The actuators sit on a
// square grid of pitch P, so the actuators whose patch covers a pixel form a
// small index box; a grid-index table maps each box entry to its actuator
// (or -1 outside the metapupil).  Residual: one lane per output pixel,
// coalesced rows of the screen and of every DM window.
#include <hip/hip_runtime.h>

#include "dm_internal.h"

namespace shw {

namespace {

__device__ __forceinline__ int floor_div(int a, int b) {  // b > 0
  int q = a / b;
  return (a % b != 0 && a < 0) ? q - 1 : q;
}

__global__ __launch_bounds__(256) void dm_surface_kernel(const DmLaunch a, const float* __restrict__ coefs,
                                                         float* __restrict__ surf) {
  const int j = blockIdx.x * 16 + (threadIdx.x & 15);
  const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (i >= a.size || j >= a.size) return;
  const int half = a.size / 2;
  // actuator grid index g (position g * pitch from the centre) covers pixel j iff
  // half + g*pitch - h <= j < half + g*pitch + h
  const int gx0 = floor_div(j - half - a.half_patch, a.pitch) + 1;
  const int gx1 = floor_div(j - half + a.half_patch, a.pitch);
  const int gy0 = floor_div(i - half - a.half_patch, a.pitch) + 1;
  const int gy1 = floor_div(i - half + a.half_patch, a.pitch);
  const float px = (float)j + 0.5f - (float)half;
  const float py = (float)i + 0.5f - (float)half;
  float acc = 0.0f;
  for (int gy = max(gy0, -a.m); gy <= min(gy1, a.m); ++gy) {
    const float dy = py - (float)(gy * a.pitch);
    const int* row = a.grid + (gy + a.m) * (2 * a.m + 1) + a.m;
    for (int gx = max(gx0, -a.m); gx <= min(gx1, a.m); ++gx) {
      const int k = row[gx];
      if (k < 0) continue;
      const float dx = px - (float)(gx * a.pitch);
      acc += coefs[k] * expf(-(dx * dx + dy * dy) * a.inv_2s2);
    }
  }
  surf[(int64_t)i * a.size + j] = acc;
}

__global__ __launch_bounds__(256) void residual_kernel(const ResidualLaunch a, float* __restrict__ out) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  const int k = blockIdx.z;
  if (x >= a.pupil_n) return;
  float v = a.screen[(int64_t)(a.scr_origin[k][0] + y) * a.screen_pitch + a.scr_origin[k][1] + x];
  for (int d = 0; d < a.n_dm; ++d)
    v -= a.surf[d][(int64_t)(a.dm_origin[k][d][0] + y) * a.surf_size[d] + a.dm_origin[k][d][1] + x];
  out[(int64_t)k * a.out_stride + (int64_t)y * a.out_pitch + x] = v;
}

}  // namespace

hipError_t launch_dm_surface(const DmLaunch& a, const float* coefs, float* surf, hipStream_t st) {
  dim3 grid((a.size + 15) / 16, (a.size + 15) / 16);
  hipLaunchKernelGGL(dm_surface_kernel, grid, dim3(256), 0, st, a, coefs, surf);
  return hipGetLastError();
}

hipError_t launch_residual(const ResidualLaunch& a, int n_out, float* out, hipStream_t st) {
  dim3 grid((a.pupil_n + 255) / 256, a.pupil_n, n_out);
  hipLaunchKernelGGL(residual_kernel, grid, dim3(256), 0, st, a, out);
  return hipGetLastError();
}

}  // namespace shw
