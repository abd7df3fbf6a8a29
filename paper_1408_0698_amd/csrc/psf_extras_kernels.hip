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

// Pass 1: block (g, s) takes rows g, g + G, ... of PSF s, one row per wavefront at a time.  For a
// row at dv from the centre, the pixels within radius r form the run |u - c| <= w, w =
// floor(sqrt(r^2 - dv^2)), whose share is pre(hi + 1) - pre(lo) of the row's FP64 prefix sums
// pre.  The wavefront stages the row in LDS with coalesced loads; lane l sums its run of R
// consecutive pixels (R a multiple of 8, 64 R >= M) in chunks of 8, a scan over the lanes gives the
// runs' offsets, and the lanes write pre at every 8th pixel; a prefix is then one of those plus at
// most 7 staged pixels.  Lane k < n_r keeps radius k's sum over the wavefront's rows, every lane
// the rows' total; the block's wavefronts are added in a fixed order at the end.
// LDS per wavefront: 65 doubles (the end), the row (pixel u at u + u/32, so that the lanes' runs
// start in different banks), and pre at every 8th pixel (ceil(M/8) doubles).
__device__ __forceinline__ void ee_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__host__ __device__ constexpr int ee_row_slot(int u) { return u + (u >> 5); }

__host__ __device__ constexpr size_t ee_wave_lds(int m) {
  return 65 * sizeof(double) + (size_t)((ee_row_slot(m) + 3) & ~3) * sizeof(float) +
         (size_t)((m + 7) / 8) * sizeof(double);
}

constexpr int kEeMaxChunks = 8;  // chunks of 8 pixels per lane: 64 x 64 >= M for M <= 4096
static_assert(kMaxRadii <= 64, "one lane per radius, entry n_r of the 65-double areas for the total");

__global__ __launch_bounds__(256) void ee_rows_kernel(const EeLaunch a) {
  extern __shared__ __align__(16) unsigned char ee_smem[];
  const int M = a.m, c = M / 2;
  const int R = ((M + 511) / 512) * 8;  // pixels per lane, a multiple of 8
  const int nw = blockDim.x >> 6, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = blockIdx.x, s = blockIdx.y;
  unsigned char* mine = ee_smem + (size_t)wave * ee_wave_lds(M);
  double* fin = reinterpret_cast<double*>(mine);
  float* srow = reinterpret_cast<float*>(mine + 65 * sizeof(double));
  double* pre8 =
      reinterpret_cast<double*>(mine + 65 * sizeof(double) + (size_t)((ee_row_slot(M) + 3) & ~3) * sizeof(float));
  const float* P = a.psf + s * a.psf_stride;
  const int u0 = lane * R;
  double acc = 0.0, tot = 0.0;
  for (int v = g + wave * kEeGroups; v < M; v += nw * kEeGroups) {
    const float* row = P + (int64_t)v * M;
    for (int u = lane; u < M; u += 64) srow[ee_row_slot(u)] = row[u];
    ee_wave_sync();
    double ch[kEeMaxChunks];
    double run = 0.0;
#pragma unroll
    for (int i = 0; i < kEeMaxChunks; ++i) {
      const int k = u0 + 8 * i;
      double cs = 0.0;
      if (8 * i < R && k < M) {
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (k + t < M) cs += (double)srow[ee_row_slot(k + t)];
      }
      ch[i] = cs;
      run += cs;
    }
    double inc = run;  // inclusive scan over the lanes, the same tree for every row
    for (int off = 1; off < 64; off <<= 1) {
      const double t = __shfl_up(inc, off);
      if (lane >= off) inc += t;
    }
    const double row_tot = __shfl(inc, 63);
    double x = inc - run;  // pre at the lane's chunk starts
#pragma unroll
    for (int i = 0; i < kEeMaxChunks; ++i) {
      const int k = u0 + 8 * i;
      if (8 * i < R && k < M) pre8[k >> 3] = x;
      x += ch[i];
    }
    ee_wave_sync();
    tot += row_tot;
    if (lane < a.n_r) {
      const double dv = (double)(v - c);
      const double rem = a.r2[lane] - dv * dv;
      if (rem >= 0.0) {
        const int w = isqrt_floor(rem);
        const int lo = c - w < 0 ? 0 : c - w;
        const int hi = c + w > M - 1 ? M - 1 : c + w;
        auto prefix = [&](int p) -> double {  // pre(p), 0 <= p <= M
          if (p == M) return row_tot;
          const int k = p & ~7;
          double y = pre8[k >> 3];
#pragma unroll
          for (int t = 0; t < 7; ++t)
            if (k + t < p) y += (double)srow[ee_row_slot(k + t)];
          return y;
        };
        acc += prefix(hi + 1) - prefix(lo);
      }
    }
    ee_wave_sync();  // the staged row and pre8 are rewritten for the next row
  }
  // the wavefronts' sums in LDS, then added in wavefront order
  if (lane < a.n_r) fin[lane] = acc;
  if (lane == 0) fin[a.n_r] = tot;
  __syncthreads();
  if ((int)threadIdx.x <= a.n_r) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += reinterpret_cast<const double*>(ee_smem + (size_t)w * ee_wave_lds(M))[threadIdx.x];
    a.ws[((int64_t)s * kEeGroups + g) * (a.n_r + 1) + threadIdx.x] = t;
  }
}

// Pass 2: block s adds the groups of PSF s and divides by the total.  Wavefront w takes entries
// k = w, w + 4, ... <= n_r; lane l adds groups l, l + 64, ... in order, then a fixed tree over
// the lanes.
__global__ __launch_bounds__(256) void ee_final_kernel(const EeLaunch a) {
  __shared__ double s_tot[kMaxRadii + 1];
  const int s = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double* w = a.ws + (int64_t)s * kEeGroups * (a.n_r + 1);
  for (int k = wave; k <= a.n_r; k += 4) {
    double x = 0.0;
    for (int gi = lane; gi < kEeGroups; gi += 64) x += w[gi * (a.n_r + 1) + k];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    if (lane == 0) s_tot[k] = x;
  }
  __syncthreads();
  if ((int)threadIdx.x < a.n_r) {
    const double tot = s_tot[a.n_r], in = s_tot[threadIdx.x];
    a.ee[(int64_t)s * a.n_r + threadIdx.x] = tot > 0.0 ? in / tot : 0.0;
  }
}

hipError_t launch_encircled_energy(const EeLaunch& a, hipStream_t st) {
  // 4 wavefronts per block when their LDS fits in 64 KB (M <= 3100 or so), else 2 (M <= 4096)
  const int nw = 4 * ee_wave_lds(a.m) <= 65536 ? 4 : 2;
  hipLaunchKernelGGL(ee_rows_kernel, dim3(kEeGroups, (unsigned)a.n_psf), dim3(64 * nw), nw * ee_wave_lds(a.m), st, a);
  hipLaunchKernelGGL(ee_final_kernel, dim3((unsigned)a.n_psf), dim3(256), 0, st, a);
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
