// psf_extras_kernels.hip - encircled energy of a PSF and resampling of a PSF to another
// wavelength's angular grid (Sec. 3 PSF block: PSFs at one or several wavelengths weighted by
// the object's colour; Strehl ratio and encircled energy in a chosen radius).
#include <hip/hip_runtime.h>

#include <mutex>

#include "geom_internal.h"

namespace shw {

// Workspace of the allocation-free encircled-energy entry point: one copy of this array per GPU,
// held until the process ends.  In host code the name stands for a host-side shadow, not a device
// address; kernels receive the address from ee_scratch_device() below.
static __device__ __align__(256) double scratch[kEeScratchDoubles];

// Largest integer w with w^2 <= q (q >= 0).
__device__ __forceinline__ int isqrt_floor(double q) {
  int w = (int)floor(sqrt(q));
  while ((double)(w + 1) * (w + 1) <= q) ++w;
  while (w > 0 && (double)w * w > q) --w;
  return w;
}

// Pass 1: block (g, s) takes rows g, g + G, ... of PSF s.  For a row at dv from the centre, the
// pixels within radius r form the run |u - c| <= w, w = floor(sqrt(r^2 - dv^2)): the row's share
// is a difference of its FP64 prefix sums.  Thread k < n_r keeps radius k's sum over the block's
// rows, thread n_r the rows' totals.
__global__ __launch_bounds__(256) void ee_rows_kernel(const EeLaunch a) {
  __shared__ double pre[4096 + 1];
  __shared__ double part[256];
  const int g = blockIdx.x, s = blockIdx.y, M = a.m, c = M / 2;
  const float* P = a.psf + s * a.psf_stride;
  const int per = (M + 255) / 256;  // consecutive pixels per thread
  double acc = 0.0;
  for (int v = g; v < M; v += kEeGroups) {
    const float* row = P + (int64_t)v * M;
    // thread-local run sums, then an exclusive scan of the 256 run sums in a fixed order
    const int u0 = threadIdx.x * per;
    double run = 0.0;
    for (int q = 0; q < per; ++q)
      if (u0 + q < M) run += (double)row[u0 + q];
    part[threadIdx.x] = run;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const double add = threadIdx.x >= off ? part[threadIdx.x - off] : 0.0;
      __syncthreads();
      part[threadIdx.x] += add;
      __syncthreads();
    }
    // pre[u + 1] = sum of row[0 .. u]
    double x = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0.0;
    if (threadIdx.x == 0) pre[0] = 0.0;
    for (int q = 0; q < per; ++q)
      if (u0 + q < M) {
        x += (double)row[u0 + q];
        pre[u0 + q + 1] = x;
      }
    __syncthreads();
    const double dv = (double)(v - c);
    if (threadIdx.x < a.n_r) {
      const double rem = a.r2[threadIdx.x] - dv * dv;
      if (rem >= 0.0) {
        const int w = isqrt_floor(rem);
        const int lo = c - w < 0 ? 0 : c - w;
        const int hi = c + w > M - 1 ? M - 1 : c + w;
        acc += pre[hi + 1] - pre[lo];
      }
    } else if (threadIdx.x == a.n_r) {
      acc += pre[M];
    }
    __syncthreads();  // pre and part are rewritten by the next row
  }
  if (threadIdx.x <= a.n_r) a.ws[((int64_t)s * kEeGroups + g) * (a.n_r + 1) + threadIdx.x] = acc;
}

// Pass 2: the groups of PSF s added in order; ee = inside / total.
__global__ __launch_bounds__(64) void ee_final_kernel(const EeLaunch a) {
  const int s = blockIdx.x, k = threadIdx.x;
  if (k >= a.n_r) return;
  const double* w = a.ws + (int64_t)s * kEeGroups * (a.n_r + 1);
  double in = 0.0, tot = 0.0;
  for (int g = 0; g < kEeGroups; ++g) {
    in += w[g * (a.n_r + 1) + k];
    tot += w[g * (a.n_r + 1) + a.n_r];
  }
  a.ee[(int64_t)s * a.n_r + k] = tot > 0.0 ? in / tot : 0.0;
}

hipError_t launch_encircled_energy(const EeLaunch& a, hipStream_t st) {
  hipLaunchKernelGGL(ee_rows_kernel, dim3(kEeGroups, (unsigned)a.n_psf), dim3(256), 0, st, a);
  hipLaunchKernelGGL(ee_final_kernel, dim3((unsigned)a.n_psf), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t ee_scratch_device(int device, double** out) {
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    // the caller has made `device` current; each GPU holds its own copy at its own address
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = static_cast<double*>(p);
  }
  *out = addr[device];
  return hipSuccess;
}

// dst[v][u] += w * src sampled bilinearly at (c + (v - c) s, c + (u - c) s), c = M/2; samples
// outside [0, M - 1]^2 add nothing.
__global__ __launch_bounds__(256) void psf_resample_kernel(const float* __restrict__ src, int32_t m, double s, float w,
                                                           float* __restrict__ dst) {
  const int u = blockIdx.x * 256 + threadIdx.x, v = blockIdx.y;
  if (u >= m) return;
  const int c = m / 2;
  const double X = c + (u - c) * s, Y = c + (v - c) * s;
  if (X < 0.0 || Y < 0.0 || X > (double)(m - 1) || Y > (double)(m - 1)) return;
  int ix = (int)floor(X), iy = (int)floor(Y);
  ix = ix > m - 2 ? m - 2 : ix;
  iy = iy > m - 2 ? m - 2 : iy;
  const double fx = X - ix, fy = Y - iy;
  const float* r0 = src + (int64_t)iy * m + ix;
  const float* r1 = r0 + m;
  const double top = (1.0 - fx) * (double)r0[0] + fx * (double)r0[1];
  const double bot = (1.0 - fx) * (double)r1[0] + fx * (double)r1[1];
  dst[(int64_t)v * m + u] += (float)((double)w * ((1.0 - fy) * top + fy * bot));
}

hipError_t launch_psf_resample(const float* src, int32_t m, double s, float w, float* dst, hipStream_t st) {
  hipLaunchKernelGGL(psf_resample_kernel, dim3((unsigned)((m + 255) / 256), (unsigned)m), dim3(256), 0, st, src, m,
                     s, w, dst);
  return hipGetLastError();
}

}  // namespace shw
