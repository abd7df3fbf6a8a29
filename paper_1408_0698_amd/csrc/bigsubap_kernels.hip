// bigsubap_kernels.hip - Shack-Hartmann measurement for large sub-apertures (FFT 512).
//
// Same model as the fused kernel (Sec. 4: sub-aperture field, spot by FFT,
// rebin, noise, centroid) for sub-apertures too large to hold in one
// lane group: 400 x 400-pixel sub-apertures padded to 512 for the low-order
// NGS sensors.  Three passes per batch of work items:
//   rows  : field of one row (FP64 phase reduction, FP32 sincos, centring
//           ramp folded in) -> 512-point transform -> T[item][y][u]
//   cols  : 512-point transform of column u over the npx non-zero rows ->
//           |F|^2 / N^2 -> rebin along the column -> Jr[item][p][u]
//   detect: rebin along the row, photometry, noise, threshold, FP64 centroid
// The 512-point transform is a Stockham autosort radix-8 FFT (three passes
// with strides 1, 8, 64) on 64 lanes, ping-ponging between two LDS buffers.
#include <hip/hip_runtime.h>

#include "big_internal.h"
#include "noise.h"
#include "regfft.h"

namespace shw {

namespace {

constexpr int kN = 512;
constexpr int kLanes = 64;           // lanes per transform
constexpr int kLines = 8;            // transforms per block
constexpr int kBlock = kLines * kLanes;

struct Line {
  float* are;
  float* aim;
  float* bre;
  float* bim;
};

// One 512-point forward transform.  On entry lane j holds v[i] = x[j + 64 i];
// on return the result is in the b planes in natural order.  All kBlock
// lanes of the block must call this (it contains block barriers).
__device__ __forceinline__ void fft512(Line ln, const float2* __restrict__ tw, int j, float2* v) {
  // pass 0 (Ns = 1): no twiddle
  RegFFT<8, -1>::run(v);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    ln.bre[j * 8 + i] = v[i].x;
    ln.bim[j * 8 + i] = v[i].y;
  }
  __syncthreads();
  // pass 1 (Ns = 8): b -> a
  {
    const int k = j & 7;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = make_float2(ln.bre[j + 64 * i], ln.bim[j + 64 * i]);
#pragma unroll
    for (int i = 1; i < 8; ++i) v[i] = cmul(v[i], tw[(i * k * 8) & (kN - 1)]);
    RegFFT<8, -1>::run(v);
    const int d = (j >> 3) * 64 + k;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      ln.are[d + 8 * i] = v[i].x;
      ln.aim[d + 8 * i] = v[i].y;
    }
  }
  __syncthreads();
  // pass 2 (Ns = 64): a -> b
  {
    const int k = j;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = make_float2(ln.are[j + 64 * i], ln.aim[j + 64 * i]);
#pragma unroll
    for (int i = 1; i < 8; ++i) v[i] = cmul(v[i], tw[(i * k) & (kN - 1)]);
    RegFFT<8, -1>::run(v);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      ln.bre[k + 64 * i] = v[i].x;
      ln.bim[k + 64 * i] = v[i].y;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void fill_twiddles(float2* tw) {
  for (int m = threadIdx.x; m < kN; m += kBlock) {
    float s, c;
    sincospif(-2.0f * (float)m / (float)kN, &s, &c);
    tw[m] = make_float2(c, s);
  }
}

__device__ __forceinline__ void item_coords(const BigLaunch& a, int64_t item, int& f, int& w, int& i) {
  const int64_t per_frame = (int64_t)a.n_wfs * a.n_valid;
  f = (int)(item / per_frame);
  const int rem = (int)(item - (int64_t)f * per_frame);
  w = rem / a.n_valid;
  i = rem - w * a.n_valid;
}

}  // namespace

// Line r of the launch = row y of item item0 + r / npx.
__global__ __launch_bounds__(kBlock) void big_rows_kernel(const BigLaunch a, int64_t item0, int64_t nlines,
                                                          float2* __restrict__ T) {
  __shared__ float s_pl[kLines * 4 * kN];
  __shared__ float2 s_tw[kN];
  fill_twiddles(s_tw);
  const int line = threadIdx.x / kLanes, j = threadIdx.x % kLanes;
  const int64_t r = (int64_t)blockIdx.x * kLines + line;
  const bool active = r < nlines;
  const int64_t rr = active ? r : 0;
  const int64_t il = rr / a.npx;
  const int y = (int)(rr - il * a.npx);
  int f, w, i;
  item_coords(a, item0 + il, f, w, i);
  const int sidx = a.valid_idx[i];
  const int sa = sidx / a.n_subap, sb = sidx - (sidx / a.n_subap) * a.n_subap;
  const int prow = sa * a.npx + y;
  const float* src = a.list ? a.list[f].opd + (int64_t)w * a.list[f].wfs_stride + (int64_t)prow * a.list[f].row_pitch
                            : a.opd + (int64_t)f * a.frame_stride + (int64_t)w * a.wfs_stride +
                                  (int64_t)prow * a.row_pitch;
  src += (int64_t)sb * a.npx;
  const float ay = (float)prow + 0.5f - a.half_n;
  float2 v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int x = j + 64 * q;
    float2 e = make_float2(0.0f, 0.0f);
    if (active && x < a.npx) {
      const float ax = (float)(sb * a.npx + x) + 0.5f - a.half_n;
      const float r2 = ax * ax + ay * ay;
      if (r2 <= a.r2_outer && r2 >= a.r2_inner) {
        const double ramp = (double)((kN - 1) * (x + y)) / (2.0 * kN);
        double wv = (double)src[x] * a.inv_lambda + ramp;
        wv = __builtin_amdgcn_fract(wv);  // wv - floor(wv), one instruction
        // hardware sine and cosine take revolutions: exp(2 pi i wv) after the FP64 reduction
        const float fw = (float)wv;
        e = make_float2(__builtin_amdgcn_cosf(fw), __builtin_amdgcn_sinf(fw));
      }
    }
    v[q] = e;
  }
  __syncthreads();  // twiddles ready
  float* base = s_pl + line * 4 * kN;
  Line ln{base, base + kN, base + 2 * kN, base + 3 * kN};
  fft512(ln, s_tw, j, v);
  if (active) {
    float2* dst = T + rr * kN;
#pragma unroll
    for (int q = 0; q < 8; ++q) dst[j + 64 * q] = make_float2(ln.bre[j + 64 * q], ln.bim[j + 64 * q]);
  }
}

// Line c of the launch = column u = c % 512 of item item0 + c / 512.  Lanes are
// interleaved (line = t % 8) so that a wave reads 8 adjacent columns per row.
__global__ __launch_bounds__(kBlock) void big_cols_kernel(const BigLaunch a, int64_t nitems,
                                                          const float2* __restrict__ T, float* __restrict__ Jr) {
  __shared__ float s_pl[kLines * 4 * kN];
  __shared__ float2 s_tw[kN];
  fill_twiddles(s_tw);
  const int line = threadIdx.x % kLines, j = threadIdx.x / kLines;
  const int64_t c = (int64_t)blockIdx.x * kLines + line;
  const bool active = c < nitems * kN;
  const int64_t cc = active ? c : 0;
  const int64_t il = cc / kN;
  const int u = (int)(cc - il * kN);
  const float2* src = T + il * a.npx * kN + u;
  float2 v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int y = j + 64 * q;
    v[q] = (active && y < a.npx) ? src[(int64_t)y * kN] : make_float2(0.0f, 0.0f);
  }
  __syncthreads();
  float* base = s_pl + line * 4 * kN;
  Line ln{base, base + kN, base + 2 * kN, base + 3 * kN};
  fft512(ln, s_tw, j, v);
  // intensity into the a plane, then rebin along the column: b = 512 / det_n rows per pixel
  const float inv_n2 = 1.0f / ((float)kN * (float)kN);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int vv = j + 64 * q;
    const float re = ln.bre[vv], im = ln.bim[vv];
    ln.are[vv] = (re * re + im * im) * inv_n2;
  }
  __syncthreads();
  if (active && j < a.det_n) {
    const int b = kN / a.det_n;
    float s = 0.0f;
    for (int k = 0; k < b; ++k) s += ln.are[j * b + k];
    Jr[(il * a.det_n + j) * kN + u] = s;
  }
}

// One block per work item: detector pixel = row-rebinned sum, photometry, noise, centroid.
__global__ __launch_bounds__(256) void big_detect_kernel(const BigLaunch a, int64_t item0,
                                                         const float* __restrict__ Jr) {
  __shared__ double red[3][256];
  const int64_t il = blockIdx.x;
  const int64_t item = item0 + il;
  int f, w, i;
  item_coords(a, item, f, w, i);
  const int npix = a.det_n * a.det_n;
  const int b = kN / a.det_n;
  const float cd = 0.5f * (float)(a.det_n - 1);
  const uint32_t gsub = (uint32_t)(w * a.n_valid + i);
  uint32_t frame = a.frame0 + (uint32_t)f, key0 = a.key0, key1 = a.key1;
  float* slopes_fw = a.slopes + ((int64_t)f * a.n_wfs + w) * 2 * a.n_valid;
  float* images_it = a.images ? a.images + item * (int64_t)(a.det_n * a.det_n) : nullptr;
  if (a.list) {
    const FrameWork& fw = a.list[f];
    frame = (uint32_t)fw.frame;
    key0 = (uint32_t)(fw.seed & 0xFFFFFFFFu);
    key1 = (uint32_t)(fw.seed >> 32);
    slopes_fw = fw.slopes + (int64_t)w * 2 * a.n_valid;
    images_it = fw.images ? fw.images + ((int64_t)w * a.n_valid + i) * (a.det_n * a.det_n) : nullptr;
  }
  double s0 = 0.0, sx = 0.0, sy = 0.0;
  for (int pix = threadIdx.x; pix < npix; pix += 256) {
    const int p = pix / a.det_n, q = pix - p * a.det_n;
    const float* row = Jr + (il * a.det_n + p) * kN + q * b;
    float det = 0.0f;
    for (int k = 0; k < b; ++k) det += row[k];
    float img = det;
    if (a.ph_scale > 0.0f) {
      const float lam = a.ph_scale * det;
      img = a.noise ? noisy_pixel(lam, a.ron, (uint32_t)pix, (uint32_t)npix, gsub, frame, key0, key1) : lam;
    }
    if (images_it) images_it[pix] = img;
    const double t = (double)fmaxf(img - a.thr, 0.0f);
    s0 += t;
    sx += (double)((float)q - cd) * t;
    sy += (double)((float)p - cd) * t;
  }
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = sx;
  red[2][threadIdx.x] = sy;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double t0 = red[0][0];
    const bool empty = !(t0 > 0.0);
    slopes_fw[i] = empty ? 0.0f : (float)(red[1][0] / t0);
    slopes_fw[a.n_valid + i] = empty ? 0.0f : (float)(red[2][0] / t0);
    if (a.flags && !a.list) a.flags[item] = empty ? 1 : 0;
  }
}

bool big_shape_supported(int npx, int fft_n, int conv_n, int det_n, int lgs) {
  return fft_n == kN && conv_n == kN && npx >= 1 && npx <= kN && lgs == 0 && det_n >= 1 && det_n <= 256 &&
         kN % det_n == 0 && det_n * det_n <= 65536;
}

hipError_t launch_big(const BigLaunch& a, int64_t item0, int64_t nitems, float2* T, float* Jr, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  const int64_t rows = nitems * a.npx;
  hipLaunchKernelGGL(big_rows_kernel, dim3((unsigned)((rows + kLines - 1) / kLines)), dim3(kBlock), 0, st, a, item0,
                     rows, T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t cols = nitems * kN;
  hipLaunchKernelGGL(big_cols_kernel, dim3((unsigned)((cols + kLines - 1) / kLines)), dim3(kBlock), 0, st, a, nitems,
                     (const float2*)T, Jr);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(big_detect_kernel, dim3((unsigned)nitems), dim3(256), 0, st, a, item0, (const float*)Jr);
  return hipGetLastError();
}

}  // namespace shw
