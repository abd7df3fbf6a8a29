// psf_kernels.hip - science PSF accumulation (Sec. 3 PSF block, Sec. 5 Strehl).
//
// P(v,u) = |sum_{y,x} A e^{i phi} e^{-2 pi i ((u - M/2) x + (v - M/2) y) / M}|^2 / (sum A)^2
// with M = 1600 = 40 x 40, computed as a row pass then a column pass.
// Each M-point transform is the four-step split n = 40 n1 + n2,
// k = k1 + 40 k2: 40-point transforms over n1 (one per lane n2), the twiddle
// W_M^(n2 k1), a transpose through LDS, 40-point transforms over n2 (one
// per lane k1).  Only the first pupil_n <= M/2 inputs are non-zero, so the
// first 40-point transforms see n1 < 20 only and run as two 20-point
// transforms.  The fftshift centring (-1)^(x+y) is folded into the FP64
// phase as (x + y)/2 waves.
//
// Row pass: 8 rows per block of 320 lanes, intermediate T[f][y][u] (complex
// FP32).  Column pass: 8 columns per block, frames accumulated in registers,
// one read-modify-write of the accumulator per call; the on-axis sample of
// each frame is the Strehl ratio.
#include <hip/hip_runtime.h>

#include "psf_internal.h"
#include "regfft.h"

namespace shw {

namespace {

constexpr int kM = 1600;
constexpr int kQ = 40;        // M = kQ * kQ
constexpr int kNZ = kM / 2 / kQ;  // non-zero n1 (20)
constexpr int kLines = 8;      // transforms per block
constexpr int kST = kQ + 1;    // odd LDS stride

// Y[k1] *= W_M^(n2 k1) = exp(-2 pi i n2 k1 / M); exact angles every 8 steps, products in between.
__device__ __forceinline__ void four_step_twiddle(float2* Y, int n2) {
  float ss, cs;
  sincospif(-2.0f * (float)n2 / (float)kM, &ss, &cs);
  const float2 step = make_float2(cs, ss);
#pragma unroll
  for (int a = 0; a < kQ / 8; ++a) {
    const int m = (n2 * 8 * a) % kM;
    float sb, cb;
    sincospif(-2.0f * (float)m / (float)kM, &sb, &cb);
    float2 t = make_float2(cb, sb);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int k1 = 8 * a + b;
      if (k1 != 0) Y[k1] = cmul(Y[k1], t);
      t = cmul(t, step);
    }
  }
}

// First step on lane n2: inputs v[n1] (n1 < kNZ, zero beyond), output Y[k1], k1 < 40, twiddled.
__device__ __forceinline__ void first_step(const float2* v, float2* Y, int n2) {
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    float2 z[kNZ];
#pragma unroll
    for (int n1 = 0; n1 < kNZ; ++n1) z[n1] = twiddle_mul<kQ, -1>(v[n1], n1 * r);
    RegFFT<kNZ, -1>::run(z);
#pragma unroll
    for (int k = 0; k < kNZ; ++k) Y[2 * k + r] = z[k];
  }
  four_step_twiddle(Y, n2);
}

// Transpose one 40 x 40 complex tile of a line through one float plane: lane n2 holds
// Y[k1]; afterwards lane k1 holds z[n2] = Y_(lane n2)[k1].  Real parts, then imaginary.
__device__ __forceinline__ void transpose_tile(float* pl, const float2* Y, float2* z, int lane) {
#pragma unroll
  for (int k1 = 0; k1 < kQ; ++k1) pl[k1 * kST + lane] = Y[k1].x;
  __syncthreads();
#pragma unroll
  for (int n2 = 0; n2 < kQ; ++n2) z[n2].x = pl[lane * kST + n2];
  __syncthreads();
#pragma unroll
  for (int k1 = 0; k1 < kQ; ++k1) pl[k1 * kST + lane] = Y[k1].y;
  __syncthreads();
#pragma unroll
  for (int n2 = 0; n2 < kQ; ++n2) z[n2].y = pl[lane * kST + n2];
  __syncthreads();
}

}  // namespace

__global__ __launch_bounds__(kLines * kQ) void psf_rows_kernel(const PsfLaunch a, int64_t f0, int nf, int64_t nrows,
                                                               float2* __restrict__ T) {
  __shared__ float s_pl[kLines * kQ * kST];
  const int tid = threadIdx.x;
  const int line = tid / kQ, lane = tid - line * kQ;
  const int64_t row = (int64_t)blockIdx.x * kLines + line;  // (star * nf + frame - f0) * pupil_n + y
  const bool active = row < nrows;
  const int64_t sf = active ? row / a.pupil_n : 0;
  const int y = active ? (int)(row - sf * a.pupil_n) : 0;
  const int64_t star = sf / nf, fl = sf - star * nf;
  float* pl = s_pl + line * kQ * kST;
  float2 v[kNZ];
  {
    const float* src = a.opd + star * a.star_stride + (f0 + fl) * a.frame_stride + (int64_t)y * a.row_pitch;
    const float by = (float)y + 0.5f - a.half_n;
    const float by2 = by * by;
#pragma unroll
    for (int n1 = 0; n1 < kNZ; ++n1) {
      const int x = kQ * n1 + lane;
      float2 e = make_float2(0.0f, 0.0f);
      if (active && x < a.pupil_n) {
        const float bx = (float)x + 0.5f - a.half_n;
        const float r2 = bx * bx + by2;
        if (r2 <= a.r2_outer && r2 >= a.r2_inner) {
          double wv = (double)src[x] * a.inv_lambda + 0.5 * (double)(x + y);
          wv -= floor(wv);
          float sn, c;
          sincospif(2.0f * (float)wv, &sn, &c);
          e = make_float2(c, sn);
        }
      }
      v[n1] = e;
    }
  }
  float2 Y[kQ];
  first_step(v, Y, lane);
  float2 z[kQ];
  transpose_tile(pl, Y, z, lane);
  RegFFT<kQ, -1>::run(z);
  if (active) {
    float2* dst = T + row * kM;
#pragma unroll
    for (int k2 = 0; k2 < kQ; ++k2) dst[lane + kQ * k2] = z[k2];
  }
}

__global__ __launch_bounds__(kLines * kQ) void psf_cols_kernel(const PsfLaunch a, int64_t f0, int nf,
                                                               const float2* __restrict__ T, float* __restrict__ acc,
                                                               float* __restrict__ strehl) {
  __shared__ float s_pl[kLines * kQ * kST];
  const int tid = threadIdx.x;
  const int line = tid / kQ, lane = tid - line * kQ;
  const int star = blockIdx.x / (kM / kLines);
  const int u = (blockIdx.x - star * (kM / kLines)) * kLines + line;  // column of this star
  float* pl = s_pl + line * kQ * kST;
  float sum[kQ];
#pragma unroll
  for (int k2 = 0; k2 < kQ; ++k2) sum[k2] = 0.0f;
  for (int fl = 0; fl < nf; ++fl) {
    const float2* src = T + ((int64_t)star * nf + fl) * a.pupil_n * kM + u;
    float2 v[kNZ];
#pragma unroll
    for (int n1 = 0; n1 < kNZ; ++n1) {
      const int y = kQ * n1 + lane;
      v[n1] = y < a.pupil_n ? src[(int64_t)y * kM] : make_float2(0.0f, 0.0f);
    }
    float2 Y[kQ];
    first_step(v, Y, lane);
    float2 z[kQ];
    transpose_tile(pl, Y, z, lane);
    RegFFT<kQ, -1>::run(z);
#pragma unroll
    for (int k2 = 0; k2 < kQ; ++k2) {
      const float p = (z[k2].x * z[k2].x + z[k2].y * z[k2].y) * a.inv_norm;
      sum[k2] += p;
      // on-axis sample: v = u = M/2, i.e. lane 0, k2 = 20 of column M/2
      if (strehl && u == kM / 2 && lane == 0 && k2 == kM / 2 / kQ) strehl[(int64_t)star * a.n_frames + f0 + fl] = p;
    }
  }
#pragma unroll
  for (int k2 = 0; k2 < kQ; ++k2) {
    const int v = lane + kQ * k2;
    acc[star * a.acc_stride + (int64_t)v * kM + u] += sum[k2];
  }
}

bool psf_size_supported(int fft_m, int pupil_n) { return fft_m == kM && pupil_n >= 1 && pupil_n <= kM / 2; }

hipError_t launch_psf_chunk(const PsfLaunch& a, int n_stars, int64_t f0, int nf, float2* T, float* acc,
                            float* strehl, hipStream_t st) {
  const int64_t nrows = (int64_t)n_stars * nf * a.pupil_n;
  const int64_t rb = (nrows + kLines - 1) / kLines;
  hipLaunchKernelGGL(psf_rows_kernel, dim3((unsigned)rb), dim3(kLines * kQ), 0, st, a, f0, nf, nrows, T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(psf_cols_kernel, dim3((unsigned)(n_stars * (kM / kLines))), dim3(kLines * kQ), 0, st, a, f0, nf,
                     (const float2*)T, acc, strehl);
  return hipGetLastError();
}

}  // namespace shw
