// bigsubap_kernels.hip - Shack-Hartmann measurement for large sub-apertures (FFT 512).
//
// Same model as the fused kernel (Sec. 4: sub-aperture field, spot by FFT,
// rebin, noise, centroid) for sub-apertures too large to hold in one
// lane group: 400 x 400-pixel sub-apertures padded to 512 for the low-order
// NGS sensors.  Three passes per batch of work items:
//   rows  : field of one row (FP64 phase reduction, FP32 sincos, centring
//           ramp folded in) -> 512-point transform; 8 rows per block are
//           transposed through LDS and stored column-major, T[item][u][y],
//           so that each column's npx values are contiguous
//   cols  : 512-point transform of column u over its npx non-zero rows (one
//           contiguous read) -> |F|^2 / N^2 -> rebin along the column ->
//           Jr[item][u][p], the det_n values of a column contiguous
//   detect: rebin along the row, photometry, noise, threshold, FP64 centroid
// Every 512-point transform runs inside one wavefront: with n = j + 64 i
// and k = k1 + 8 k2, lane j first transforms its 8 samples over i, then
// multiplies by W_512^(j k1); the 64-point transforms over j that remain
// (one per k1) split again as 8 x 8, through two LDS transposes within the
// wavefront.  Lane L ends with X[L + 64 b], b = 0..7.
#include <hip/hip_runtime.h>

#include "big_internal.h"
#include "noise.h"
#include "regfft.h"

namespace shw {

namespace {

constexpr int kN = 512;
constexpr int kRowWaves = 8;         // rows per block of the row pass (one wavefront each), a power of two
constexpr int kColWaves = 4;         // columns per block of the column pass
// LDS strides of the in-wave transposes, in complex values.  First transpose: [k1][j] with row
// stride 72; second: [h][k2a][g] with g contiguous, k2a stride 8 and h stride 66.  With these, the
// 16 lanes served together by a 64-bit LDS access touch 16 different bank pairs in every read
// and write of the transform.
constexpr int kS1 = 72;
constexpr int kS4 = 66;
constexpr int kWaveArea = 8 * kS1;   // complex values per wavefront (>= 8 * kS4)
static_assert(8 * kS4 <= kWaveArea, "second transpose fits the wavefront's area");
constexpr int kTileStride = kRowWaves + 1;  // row pass: [u][row] tile, odd stride

// W_512^m, m < 512, rounded to FP32 from FP64 values at compile time
__constant__ const TwiddleTable<kN> kTw{};

__device__ __forceinline__ void fill_twiddles(float2* tw, int tid, int nthreads) {
  for (int m = tid; m < kN; m += nthreads) tw[m] = make_float2(kTw.c[m], -kTw.s[m]);
}

// One forward 512-point transform in one wavefront.  On entry lane j holds v[i] = x[j + 64 i];
// on return lane j holds v[b] = X[j + 64 b].  area: the wavefront's kWaveArea complex values;
// tw: W_512^m, m < 512.  Every lane of the block must call it (block barriers).
__device__ __forceinline__ void fft512_wave(float2 (&v)[8], float2* area, const float2* tw, int j) {
  // over i: 8-point transforms, then the twiddle W_512^(j k1)
  RegFFT<8, -1>::run(v);
#pragma unroll
  for (int k1 = 1; k1 < 8; ++k1) v[k1] = cmul(v[k1], tw[j * k1]);
#pragma unroll
  for (int k1 = 0; k1 < 8; ++k1) area[k1 * kS1 + j] = v[k1];
  __syncthreads();
  // lane (g, h) = (j >> 3, j & 7): samples y[h + 8 m] of the 64-point transform of k1 = g
  const int g = j >> 3, h = j & 7;
  float2 w[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) w[m] = area[g * kS1 + h + 8 * m];
  RegFFT<8, -1>::run(w);
#pragma unroll
  for (int a = 1; a < 8; ++a) w[a] = cmul(w[a], tw[8 * h * a]);  // W_64^(h a)
  __syncthreads();  // every lane has read the first transpose
#pragma unroll
  for (int a = 0; a < 8; ++a) area[h * kS4 + a * 8 + g] = w[a];
  __syncthreads();
  // lane (a, g') = (j >> 3, j & 7): the 8-point transform over h of k1 = g', k2a = a gives
  // X[g' + 8 a + 64 b] = X[j + 64 b]
  const int a2 = j >> 3, g2 = j & 7;
#pragma unroll
  for (int hh = 0; hh < 8; ++hh) v[hh] = area[hh * kS4 + a2 * 8 + g2];
  RegFFT<8, -1>::run(v);
}

__device__ __forceinline__ void item_coords(const BigLaunch& a, int64_t item, int& f, int& w, int& i) {
  const int64_t per_frame = (int64_t)a.n_wfs * a.n_valid;
  f = (int)(item / per_frame);
  const int rem = (int)(item - (int64_t)f * per_frame);
  w = rem / a.n_valid;
  i = rem - w * a.n_valid;
}

}  // namespace

// Row r of the launch = row y = r % npx of item item0 + r / npx; wavefront t of block b takes
// row 16 b + t.  T[(il * 512 + u) * npx + y] = X_y[u].
__global__ __launch_bounds__(kRowWaves * 64) void big_rows_kernel(const BigLaunch a, int64_t item0, int64_t nlines,
                                                                  float2* __restrict__ T) {
  // the wavefronts' transform areas, later reused as the [u][row] tile of the block
  constexpr int kAreas = kRowWaves * kWaveArea;
  constexpr int kTile = kN * kTileStride;
  __shared__ float2 s_buf[kAreas > kTile ? kAreas : kTile];
  __shared__ float2 s_tw[kN];
  const int tid = threadIdx.x;
  fill_twiddles(s_tw, tid, kRowWaves * 64);
  // the wavefront index is uniform: through readfirstlane the row's item arithmetic is scalar
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), j = tid & 63;
  const int64_t r = (int64_t)blockIdx.x * kRowWaves + wv;
  const bool active = r < nlines;
  const int64_t rr = active ? r : 0;
  const int64_t il = rr / a.npx;
  const int y = (int)(rr - il * a.npx);
  int f, w, i;
  item_coords(a, item0 + il, f, w, i);
  const int sidx = a.valid_idx[i];
  const int sa = sidx / a.n_subap, sb = sidx - sa * a.n_subap;
  const int prow = sa * a.npx + y;
  const float* src = a.list ? a.list[f].opd + (int64_t)w * a.list[f].wfs_stride + (int64_t)prow * a.list[f].row_pitch
                            : a.opd + (int64_t)f * a.frame_stride + (int64_t)w * a.wfs_stride +
                                  (int64_t)prow * a.row_pitch;
  src += (int64_t)sb * a.npx;
  // every sample of the row is loaded before any is used, unlit ones masked by amplitude
  float ov[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int x = j + 64 * q;
    ov[q] = (active && x < a.npx) ? src[x] : 0.0f;
  }
  const float ay = (float)prow + 0.5f - a.half_n;
  const float ay2 = ay * ay;
  float2 v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int x = j + 64 * q;
    const float ax = (float)(sb * a.npx + x) + 0.5f - a.half_n;
    const float r2 = ax * ax + ay2;
    const bool lit = active && x < a.npx && r2 <= a.r2_outer && r2 >= a.r2_inner;
    // waves: OPD / lambda + centring ramp (N - 1)(x + y) / (2 N), exact in FP64
    double wvs = (double)ov[q] * a.inv_lambda + (double)((kN - 1) * (x + y)) * (1.0 / (2.0 * kN));
    wvs = __builtin_amdgcn_fract(wvs);  // wvs - floor(wvs), one instruction
    // hardware sine and cosine take revolutions: exp(2 pi i wvs) after the FP64 reduction
    const float fw = (float)wvs;
    const float amp = lit ? 1.0f : 0.0f;
    v[q] = make_float2(amp * __builtin_amdgcn_cosf(fw), amp * __builtin_amdgcn_sinf(fw));
  }
  __syncthreads();  // twiddles ready
  fft512_wave(v, s_buf + wv * kWaveArea, s_tw, j);
  __syncthreads();  // every wavefront has read its area: the tile overwrites them
#pragma unroll
  for (int b = 0; b < 8; ++b) s_buf[(j + 64 * b) * kTileStride + wv] = v[b];
  __syncthreads();
  // write-out: kRowWaves consecutive threads store the block's rows of one column u, contiguous in
  // T when the rows belong to one item.  Thread tid always takes row t = tid % kRowWaves (the
  // block's thread count is a multiple of kRowWaves) and columns u = tid / kRowWaves + 64 k.
  const int t = tid & (kRowWaves - 1);
  const int64_t r0 = (int64_t)blockIdx.x * kRowWaves;
  const int64_t row = r0 + t;
  if (row < nlines) {
    // item and row of row r0 + t from those of r0 (uniform): at most kRowWaves steps when npx is small
    const int64_t il0 = r0 / a.npx;
    int64_t ilt = il0;
    int yt = (int)(r0 - il0 * a.npx) + t;
    while (yt >= a.npx) {
      yt -= a.npx;
      ++ilt;
    }
    float2* dst = T + ilt * kN * a.npx + yt;
    const int u0 = tid / kRowWaves;
#pragma unroll
    for (int k = 0; k < kN / 64; ++k) {
      const int u = u0 + 64 * k;
      dst[(int64_t)u * a.npx] = s_buf[u * kTileStride + t];
    }
  }
}

// Detector of item item0 + il: rebin along the row (b = 512 / det_n columns per pixel), photometry,
// noise, threshold, FP64 centroid.  All 256 threads of the calling block take part (barriers);
// red: 3 * 256 doubles of LDS.
__device__ __forceinline__ void detect_item(const BigLaunch& a, int64_t item0, int64_t il, const float* Jr, int tid,
                                            double (*red)[256]) {
  const int64_t item = item0 + il;
  int f, w, i;
  item_coords(a, item, f, w, i);
  const int dn = a.det_n;
  const int npix = dn * dn;
  const int b = kN / dn;
  const float cd = 0.5f * (float)(dn - 1);
  const uint32_t gsub = (uint32_t)(w * a.n_valid + i);
  uint32_t frame = a.frame0 + (uint32_t)f, key0 = a.key0, key1 = a.key1;
  float* slopes_fw = a.slopes + ((int64_t)f * a.n_wfs + w) * 2 * a.n_valid;
  float* images_it = a.images ? a.images + item * (int64_t)npix : nullptr;
  if (a.list) {
    const FrameWork& fw = a.list[f];
    frame = (uint32_t)fw.frame;
    key0 = (uint32_t)(fw.seed & 0xFFFFFFFFu);
    key1 = (uint32_t)(fw.seed >> 32);
    slopes_fw = fw.slopes + (int64_t)w * 2 * a.n_valid;
    images_it = fw.images ? fw.images + ((int64_t)w * a.n_valid + i) * npix : nullptr;
  }
  const float* jr = Jr + il * kN * dn;
  double s0 = 0.0, sx = 0.0, sy = 0.0;
  // thread t takes pixel (p, q) = (t % det_n, t / det_n): consecutive threads read consecutive p
  for (int t = tid; t < npix; t += 256) {
    const int q = t / dn, p = t - q * dn;
    const int pix = p * dn + q;
    const float* col = jr + (int64_t)q * b * dn + p;
    // b = 512 / det_n is a power of two: for b >= 8, eight loads in flight per step (partial sums
    // in a fixed order), not one load per dependent addition
    float det = 0.0f;
    if (b >= 8) {
      float ps[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
      for (int k0 = 0; k0 < b; k0 += 8) {
#pragma unroll
        for (int r = 0; r < 8; ++r) ps[r] += col[(k0 + r) * dn];
      }
      det = ((ps[0] + ps[1]) + (ps[2] + ps[3])) + ((ps[4] + ps[5]) + (ps[6] + ps[7]));
    } else {
      for (int k = 0; k < b; ++k) det += col[k * dn];
    }
    float img = det;
    if (a.ph_scale > 0.0f) {
      const float lam = a.ph_scale * det;
      img = a.noise ? noisy_pixel(lam, a.ron, (uint32_t)pix, (uint32_t)npix, gsub, frame, key0, key1) : lam;
    }
    if (images_it) images_it[pix] = img;
    const double tt = (double)fmaxf(img - a.thr, 0.0f);
    s0 += tt;
    sx += (double)((float)q - cd) * tt;
    sy += (double)((float)p - cd) * tt;
  }
  red[0][tid] = s0;
  red[1][tid] = sx;
  red[2][tid] = sy;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st)
      for (int c = 0; c < 3; ++c) red[c][tid] += red[c][tid + st];
    __syncthreads();
  }
  if (tid == 0) {
    const double t0 = red[0][0];
    const bool empty = !(t0 > 0.0);
    slopes_fw[i] = empty ? 0.0f : (float)(red[1][0] / t0);
    slopes_fw[a.n_valid + i] = empty ? 0.0f : (float)(red[2][0] / t0);
    if (a.flags && !a.list) a.flags[item] = empty ? 1 : 0;
  }
}

// Column c of the launch = column u = c % 512 of item c / 512, one wavefront each:
// Jr[(il * 512 + u) * det_n + p] = sum over the b = 512 / det_n rows v of pixel p of |X_u[v]|^2 / N^2.
__global__ __launch_bounds__(kColWaves * 64) void big_cols_kernel(const BigLaunch a, int64_t nitems,
                                                                  const float2* __restrict__ T, float* __restrict__ Jr) {
  __shared__ __align__(16) float2 s_area[kColWaves * kWaveArea];  // 16-byte reads in the rebin
  __shared__ float2 s_tw[kN];
  const int tid = threadIdx.x;
  fill_twiddles(s_tw, tid, kColWaves * 64);
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), j = tid & 63;
  const int64_t c = (int64_t)blockIdx.x * kColWaves + wv;
  const bool active = c < nitems * kN;
  const int64_t cc = active ? c : 0;
  const int64_t il = cc / kN;
  const int u = (int)(cc - il * kN);
  const float2* src = T + (il * kN + u) * a.npx;
  float2 v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int y = j + 64 * q;
    v[q] = (active && y < a.npx) ? src[y] : make_float2(0.0f, 0.0f);
  }
  __syncthreads();  // twiddles ready
  float2* area = s_area + wv * kWaveArea;
  fft512_wave(v, area, s_tw, j);
  // intensity of row v = j + 64 b into the wavefront's area (as floats), then the column rebin
  const float inv_n2 = 1.0f / ((float)kN * (float)kN);
  float* ia = reinterpret_cast<float*>(area);
  __syncthreads();  // every lane has read the second transpose
#pragma unroll
  for (int b = 0; b < 8; ++b) ia[j + 64 * b] = (v[b].x * v[b].x + v[b].y * v[b].y) * inv_n2;
  __syncthreads();
  if (active) {
    const int bsz = kN / a.det_n;  // rows per detector pixel, a power of two
    if (bsz >= 8) {
      // lane j sums rows 8j .. 8j+7 (two 16-byte reads), then groups of bsz / 8 lanes add up by
      // butterflies; the group's first lane holds pixel p = 8 j / bsz
      const float4 q0 = reinterpret_cast<const float4*>(ia)[2 * j];
      const float4 q1 = reinterpret_cast<const float4*>(ia)[2 * j + 1];
      float sum = ((q0.x + q0.y) + (q0.z + q0.w)) + ((q1.x + q1.y) + (q1.z + q1.w));
      const int gl = bsz >> 3;  // lanes per pixel, <= 64
      for (int off = 1; off < gl; off <<= 1) sum += __shfl_xor(sum, off, 64);
      if ((j & (gl - 1)) == 0) Jr[(il * kN + u) * a.det_n + j / gl] = sum;
    } else {
      for (int p = j; p < a.det_n; p += 64) {
        float sum = 0.0f;
        for (int k = 0; k < bsz; ++k) sum += ia[p * bsz + k];
        Jr[(il * kN + u) * a.det_n + p] = sum;
      }
    }
  }
}

// One block per work item: the detector stage.
__global__ __launch_bounds__(256) void big_detect_kernel(const BigLaunch a, int64_t item0,
                                                         const float* __restrict__ Jr) {
  __shared__ double red[3][256];
  detect_item(a, item0, blockIdx.x, Jr, threadIdx.x, red);
}

bool big_shape_supported(int npx, int fft_n, int conv_n, int det_n, int lgs) {
  return fft_n == kN && conv_n == kN && npx >= 1 && npx <= kN && lgs == 0 && det_n >= 1 && det_n <= 256 &&
         kN % det_n == 0 && det_n * det_n <= 65536;
}

hipError_t launch_big(const BigLaunch& a, int64_t item0, int64_t nitems, float2* T, float* Jr, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  const int64_t rows = nitems * a.npx;
  hipLaunchKernelGGL(big_rows_kernel, dim3((unsigned)((rows + kRowWaves - 1) / kRowWaves)), dim3(kRowWaves * 64), 0,
                     st, a, item0, rows, T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t cols = nitems * kN;
  hipLaunchKernelGGL(big_cols_kernel, dim3((unsigned)((cols + kColWaves - 1) / kColWaves)), dim3(kColWaves * 64), 0,
                     st, a, nitems, (const float2*)T, Jr);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(big_detect_kernel, dim3((unsigned)nitems), dim3(256), 0, st, a, item0, (const float*)Jr);
  return hipGetLastError();
}

}  // namespace shw
