// recon_kernels.hip - control-matrix product and pure integrator of the closed loop (Sec. 3:
// the slope vectors are multiplied by the control matrix, the modal increments integrated).
//
// The product streams the whole matrix from HBM once; it is bandwidth-bound.  A block owns a
// tile of 64 rows x 4096 columns: the 16 KB slope chunk is staged in LDS once per block, each
// wave streams 16 rows with 16-byte loads (64 lanes cover 1 KB of a row per step, 16 loads in
// flight per lane), and per-row sums are reduced across the wave.  Chunk sums go to a
// partial buffer and a second pass adds them in a fixed order, so results do not depend on
// scheduling.
#include <hip/hip_runtime.h>

#include "recon_internal.h"

namespace shw {
namespace {

constexpr int kRowsPerWave = kReconRows / 4;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(256) void recon_partial_kernel(const float* __restrict__ cm, int64_t ld, int32_t n_modes,
                                                            int32_t n_slopes, const float* __restrict__ slopes,
                                                            float* __restrict__ partial) {
  __shared__ float4 s_sl[kReconCols / 4];
  const int chunk = blockIdx.x;
  const int64_t c0 = (int64_t)chunk * kReconCols;
  const int ncol = (int)((int64_t)n_slopes - c0 < kReconCols ? (int64_t)n_slopes - c0 : kReconCols);
  for (int k = threadIdx.x; k < kReconCols / 4; k += 256) {
    float v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (4 * k + e < ncol) ? slopes[c0 + 4 * k + e] : 0.0f;
    s_sl[k] = make_float4(v[0], v[1], v[2], v[3]);
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row0 = blockIdx.y * kReconRows + wave * kRowsPerWave;
  float acc[kRowsPerWave];
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) acc[r] = 0.0f;
  const int nfull = ncol / 4;  // float4 columns entirely inside the matrix
  for (int k = lane; k < nfull; k += 64) {
    const float4 x = s_sl[k];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
      const int m = row0 + r;
      if (m < n_modes) {
        const float4 a = *reinterpret_cast<const float4*>(cm + (int64_t)m * ld + c0 + 4 * k);
        acc[r] += a.x * x.x + a.y * x.y + a.z * x.z + a.w * x.w;
      }
    }
  }
  // ragged tail of the last chunk: at most 3 columns, one lane each
  if (lane < ncol - 4 * nfull) {
    const int c = 4 * nfull + lane;
    const float x = slopes[c0 + c];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
      const int m = row0 + r;
      if (m < n_modes) acc[r] += cm[(int64_t)m * ld + c0 + c] * x;
    }
  }
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    const float s = wave_sum(acc[r]);
    const int m = row0 + r;
    if (lane == 0 && m < n_modes) partial[(int64_t)chunk * n_modes + m] = s;
  }
}

__global__ __launch_bounds__(256) void recon_integrate_kernel(const float* __restrict__ partial, int32_t n_chunks,
                                                              int32_t n_modes, float gain, float* __restrict__ coefs,
                                                              float* __restrict__ delta_out) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= n_modes) return;
  float d = 0.0f;
  for (int c = 0; c < n_chunks; ++c) d += partial[(int64_t)c * n_modes + m];
  coefs[m] += gain * d;
  if (delta_out) delta_out[m] = d;
}

}  // namespace

hipError_t launch_recon_partial(const float* cm, int64_t ld, int32_t n_modes, int32_t n_slopes, const float* slopes,
                                float* partial, hipStream_t st) {
  if (n_modes <= 0 || n_slopes <= 0) return hipSuccess;
  dim3 grid((unsigned)recon_chunks(n_slopes), (unsigned)((n_modes + kReconRows - 1) / kReconRows));
  hipLaunchKernelGGL(recon_partial_kernel, grid, dim3(256), 0, st, cm, ld, n_modes, n_slopes, slopes, partial);
  return hipGetLastError();
}

hipError_t launch_recon_integrate(const float* partial, int32_t n_chunks, int32_t n_modes, float gain, float* coefs,
                                  float* delta_out, hipStream_t st) {
  if (n_modes <= 0) return hipSuccess;
  hipLaunchKernelGGL(recon_integrate_kernel, dim3((unsigned)((n_modes + 255) / 256)), dim3(256), 0, st, partial,
                     n_chunks, n_modes, gain, coefs, delta_out);
  return hipGetLastError();
}

}  // namespace shw
