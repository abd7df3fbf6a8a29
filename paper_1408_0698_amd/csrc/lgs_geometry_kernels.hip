// lgs_geometry_kernels.hip - open-loop wavefronts of finite-altitude sources (the cone effect)
// and the uplink tip-tilt of laser guide stars.
//
// Sec. 4 (open-loop generation): the shifted phase screens are piled up per source direction;
// for an LGS each sodium sub-layer is a source at its own altitude, whose beam crosses a layer
// at altitude h on a pupil footprint shrunk by (1 - h/H) and moved by h theta, and the spot on
// the sodium layer is displaced by the tip-tilt the laser beam picks up on its way up.
#include <hip/hip_runtime.h>

#include "geom_internal.h"

namespace shw {

// Bilinear sample of layer L at screen pixel coordinates (X, Y); the caller keeps (X, Y) inside
// [0, cols - 1] x [0, rows - 1] (the host checks the extremes), the clamp only guards rounding.
__device__ __forceinline__ double layer_sample(const LayerDesc& L, double X, double Y) {
  int ix = (int)floor(X), iy = (int)floor(Y);
  ix = ix < 0 ? 0 : (ix > L.cols - 2 ? L.cols - 2 : ix);
  iy = iy < 0 ? 0 : (iy > L.rows - 2 ? L.rows - 2 : iy);
  const double fx = X - ix, fy = Y - iy;
  const float* r0 = L.screen + (int64_t)iy * L.pitch + ix;
  const float* r1 = r0 + L.pitch;
  const double top = (1.0 - fx) * (double)r0[0] + fx * (double)r0[1];
  const double bot = (1.0 - fx) * (double)r1[0] + fx * (double)r1[1];
  return (1.0 - fy) * top + fy * bot;
}

// Sum over the layers of the OPD seen from pupil point (x, y) metres toward direction theta of a
// source at inverse altitude inv_h (0: infinity).  Layers go four at a time: the reads of a group
// are issued first and blended afterwards, so that they are in flight together.
__device__ __forceinline__ double piled_opd(const LayerSet& S, double x, double y, double tx, double ty,
                                            double inv_h) {
  double acc = 0.0;
  for (int l0 = 0; l0 < S.n_layers; l0 += 4) {
    float t00[4], t01[4], t10[4], t11[4];
    double fx[4], fy[4], use[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // past the last layer the group re-reads the last one (in bounds) and gives it weight 0:
      // no branch, so nothing waits for a read before the next one is issued
      const int l = l0 + q < S.n_layers ? l0 + q : S.n_layers - 1;
      use[q] = l0 + q < S.n_layers ? 1.0 : 0.0;
      const LayerDesc& L = S.layer[l];
      const double s = 1.0 - L.alt_m * inv_h;  // footprint scale of the cone at this altitude
      const double inv_p = 1.0 / L.pitch_m;
      const double X = L.x0 + (s * x + L.alt_m * tx) * inv_p, Y = L.y0 + (s * y + L.alt_m * ty) * inv_p;
      int ix = (int)floor(X), iy = (int)floor(Y);
      ix = ix < 0 ? 0 : (ix > L.cols - 2 ? L.cols - 2 : ix);
      iy = iy < 0 ? 0 : (iy > L.rows - 2 ? L.rows - 2 : iy);
      fx[q] = X - ix;
      fy[q] = Y - iy;
      const float* r0 = L.screen + (int64_t)iy * L.pitch + ix;
      t00[q] = r0[0];
      t01[q] = r0[1];
      t10[q] = r0[L.pitch];
      t11[q] = r0[L.pitch + 1];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double top = (1.0 - fx[q]) * (double)t00[q] + fx[q] * (double)t01[q];
      const double bot = (1.0 - fx[q]) * (double)t10[q] + fx[q] * (double)t11[q];
      acc += use[q] * ((1.0 - fy[q]) * top + fy[q] * bot);
    }
  }
  return acc;
}

__global__ __launch_bounds__(256) void project_layers_kernel(const ProjectLaunch a) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int i = blockIdx.y;
  const int t = blockIdx.z;
  if (j >= a.pupil_n) return;
  const double x = ((double)j + 0.5 - 0.5 * a.pupil_n) * a.dx;
  const double y = ((double)i + 0.5 - 0.5 * a.pupil_n) * a.dx;
  double opd = piled_opd(a.L, x, y, a.theta[t][0], a.theta[t][1], a.inv_h[t]);
  if (a.tilt) opd += a.tilt[2 * t] * x + a.tilt[2 * t + 1] * y;
  a.out[t * a.out_stride + (int64_t)i * a.out_pitch + j] = (float)opd;
}

hipError_t launch_project_layers(const ProjectLaunch& a, hipStream_t st) {
  const dim3 grid((unsigned)((a.pupil_n + 255) / 256), (unsigned)a.pupil_n, (unsigned)a.n_t);
  hipLaunchKernelGGL(project_layers_kernel, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

// One block per LGS: samples of the launch beam, FP64 sums reduced in a fixed order.
__global__ __launch_bounds__(256) void uplink_tilt_kernel(const UplinkLaunch a) {
  __shared__ double red[3][256];
  const int k = blockIdx.x;
  const double* g = a.lgs[k];
  const double lx = g[0], ly = g[1], tx = g[2], ty = g[3], H = g[4];
  const double step = a.d / a.n_s, r2 = 0.25 * a.d * a.d;
  double sxo = 0.0, syo = 0.0, sxx = 0.0;
  for (int e = threadIdx.x; e < a.n_s * a.n_s; e += 256) {
    const int si = e / a.n_s, sj = e - si * a.n_s;
    const double sx = ((double)sj + 0.5 - 0.5 * a.n_s) * step;
    const double sy = ((double)si + 0.5 - 0.5 * a.n_s) * step;
    if (sx * sx + sy * sy > r2) continue;
    // the beam centre at altitude h: launcher (1 - h/H) + h theta; the beam keeps its diameter
    double opd = 0.0;
    for (int l = 0; l < a.L.n_layers; ++l) {
      const LayerDesc& L = a.L.layer[l];
      const double f = L.alt_m / H;
      const double cx = lx * (1.0 - f) + L.alt_m * tx, cy = ly * (1.0 - f) + L.alt_m * ty;
      const double inv_p = 1.0 / L.pitch_m;
      opd += layer_sample(L, L.x0 + (cx + sx) * inv_p, L.y0 + (cy + sy) * inv_p);
    }
    sxo += sx * opd;
    syo += sy * opd;
    sxx += sx * sx;  // the sample set is symmetric: sum sy^2 = sum sx^2, sum sx = sum sy = sum sx sy = 0
  }
  red[0][threadIdx.x] = sxo;
  red[1][threadIdx.x] = syo;
  red[2][threadIdx.x] = sxx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double den = red[2][0];
    a.tilt[2 * k] = den > 0.0 ? red[0][0] / den : 0.0;
    a.tilt[2 * k + 1] = den > 0.0 ? red[1][0] / den : 0.0;
  }
}

hipError_t launch_uplink_tilt(const UplinkLaunch& a, hipStream_t st) {
  hipLaunchKernelGGL(uplink_tilt_kernel, dim3((unsigned)a.n), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace shw
