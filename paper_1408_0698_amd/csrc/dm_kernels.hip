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

// One lane per output pixel; the pixel is inside the actuator's patch or the value is 0.
__global__ __launch_bounds__(256) void influence_kernel(const InfluenceLaunch a, float* __restrict__ out) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  const int k = blockIdx.z;
  if (x >= a.pupil_n) return;
  const int act = a.act[k];
  if (act < 0 || act >= a.n_act) {  // an index off the grid yields a NaN frame, never a stray read
    out[(int64_t)k * a.out_stride + (int64_t)y * a.out_pitch + x] = __builtin_nanf("");
    return;
  }
  const float ax = a.act_xy[2 * act], ay = a.act_xy[2 * act + 1];
  const int half = a.size / 2;
  const int i = a.row0 + y, j = a.col0 + x;  // surface pixel
  const int cx = half + (int)ax, cy = half + (int)ay;
  float v = 0.0f;
  if (j >= cx - a.half_patch && j < cx + a.half_patch && i >= cy - a.half_patch && i < cy + a.half_patch) {
    const float dx = (float)j + 0.5f - (float)half - ax;
    const float dy = (float)i + 0.5f - (float)half - ay;
    v = a.amp[k] * expf(-(dx * dx + dy * dy) * a.inv_2s2);
  }
  out[(int64_t)k * a.out_stride + (int64_t)y * a.out_pitch + x] = v;
}

// Interaction-matrix columns from push/pull slope pairs: a 32 x 32 tile transpose through LDS.
__global__ __launch_bounds__(256) void push_pull_kernel(const float* __restrict__ slopes, int32_t n_modes,
                                                        int32_t n_slopes, float scale, float* __restrict__ im,
                                                        int64_t ld) {
  __shared__ float tile[32][33];
  const int s0 = blockIdx.x * 32, m0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int m = m0 + r, s = s0 + tx;
    float v = 0.0f;
    if (m < n_modes && s < n_slopes)
      v = (slopes[(int64_t)(2 * m) * n_slopes + s] - slopes[(int64_t)(2 * m + 1) * n_slopes + s]) * scale;
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int s = s0 + r, m = m0 + tx;
    if (s < n_slopes && m < n_modes) im[(int64_t)s * ld + m] = tile[tx][r];
  }
}

}  // namespace

hipError_t launch_influence_opd(const InfluenceLaunch& a, float* out, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  dim3 grid((a.pupil_n + 255) / 256, a.pupil_n, a.n);
  hipLaunchKernelGGL(influence_kernel, grid, dim3(256), 0, st, a, out);
  return hipGetLastError();
}

hipError_t launch_push_pull(const float* slopes, int32_t n_modes, int32_t n_slopes, float scale, float* im,
                            int64_t ld, hipStream_t st) {
  if (n_modes <= 0 || n_slopes <= 0) return hipSuccess;
  dim3 grid((n_slopes + 31) / 32, (n_modes + 31) / 32);
  hipLaunchKernelGGL(push_pull_kernel, grid, dim3(256), 0, st, slopes, n_modes, n_slopes, scale, im, ld);
  return hipGetLastError();
}

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
