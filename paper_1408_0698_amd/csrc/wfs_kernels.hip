// wfs_kernels.hip - fused Shack-Hartmann measurement for gfx950.
//
// One work item = one valid sub-aperture of one sensor in one frame
// (Sec. 4 LGS SH module: split into sub-apertures, spot by FFT, Gaussian
// convolution for the sodium extent, noise, centroid).  A block holds SPB
// items; each item owns CONV_N consecutive lanes, and each lane keeps one
// row or one column of the item's grid in registers, where it runs a
// whole 1-D transform (regfft.h).  LDS is used only to transpose between
// the row and the column passes, as two float planes (real, imaginary)
// with an odd row stride so that both passes are free of bank conflicts.
//
// Per item:
//  A  row pass of the spot transform.  Only NPX of the FFT_N rows carry
//     field, and the padded transform of length FFT_N = R * NPX splits into
//     R transforms of length NPX on twiddled inputs; lane (y, k2) builds
//     its NPX field values with the twiddle, the half-pixel centring ramp
//     and the phase folded into one FP64 phase reduced to [0, 1) waves
//     before the FP32 sincos, then runs one NPX-point transform.
//  A' column pass, same pruning, then I = |F|^2 / FFT_N^2: lane u holds
//     column u of the spot, embedded in the CONV_N grid.
//  B  (LGS) real column transform, per-row transform x K^ x inverse row
//     transform, inverse column transform: J = I (*) k.
//  C  rebin along the column in registers, then along the row via LDS.
//  D  photometry, Poisson + read noise, threshold, centre of gravity with
//     FP64 sums, reduced over the item's lanes.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "noise.h"
#include "regfft.h"

namespace shw {

constexpr double ct_floor(double x) {
  long i = (long)x;
  return (double)i > x ? (double)(i - 1) : (double)i;
}
// Area overlap of input pixel [k, k+1) with output pixel [b p, b (p+1)), b = CN / DN.
constexpr float rebin_weight(int CN, int DN, int p, int k) {
  const double b = (double)CN / (double)DN;
  const double lo = (double)k > b * p ? (double)k : b * p;
  const double hi = (double)(k + 1) < b * (p + 1) ? (double)(k + 1) : b * (p + 1);
  return hi > lo ? (float)(hi - lo) : 0.0f;
}

template <int NPX, int FFT_N, int CONV_N, int DET_N, bool LGS, int SPB>
__global__ __launch_bounds__(SPB * CONV_N) void wfs_fused_kernel(const WfsLaunch a) {
  constexpr int L = CONV_N;                  // lanes per item
  constexpr int R = FFT_N / NPX;             // column residues of the row pass
  constexpr int H = CONV_N / 2 + 1;          // stored half spectrum rows
  constexpr int ST = CONV_N + 1;             // odd LDS row stride (floats)
  constexpr int ROWS0 = NPX > H ? NPX : H;
  constexpr int ROWS = ROWS0 > DET_N ? ROWS0 : DET_N;
  constexpr int PLANE = ((ROWS * ST) + 1) & ~1;  // even: the imaginary plane is reused for doubles
  constexpr int OFF = (CONV_N - FFT_N) / 2;  // spot offset in the convolution grid
  constexpr float INV_N2 = 1.0f / (float)(FFT_N * FFT_N);
  constexpr int NPIX = DET_N * DET_N;
  constexpr int PIX_ITERS = (NPIX + L - 1) / L;
  static_assert(FFT_N % NPX == 0 && CONV_N >= FFT_N && (CONV_N - FFT_N) % 2 == 0, "shape");
  static_assert(3 * L * 2 <= PLANE, "reduction space");

  __shared__ __align__(16) float s_re[SPB * PLANE];
  __shared__ __align__(16) float s_im[SPB * PLANE];

  const int tid = threadIdx.x;
  const int s = tid / L;
  const int l = tid - s * L;
  const int64_t item = (int64_t)blockIdx.x * SPB + s;
  const bool active = item < a.total;
  const int64_t per_frame = (int64_t)a.n_wfs * a.n_valid;
  const int64_t it = active ? item : 0;
  const int f = (int)(it / per_frame);
  const int rem = (int)(it - (int64_t)f * per_frame);
  const int w = rem / a.n_valid;
  const int i = rem - w * a.n_valid;
  const int sidx = a.valid_idx[i];
  const int sa = sidx / a.n_subap;
  const int sb = sidx - sa * a.n_subap;
  float* re = s_re + s * PLANE;
  float* im = s_im + s * PLANE;

  // ---------------------------------------------------------------- A: row pass
  if (active && l < FFT_N) {
    const int y = l / R;
    const int k2 = l - y * R;
    const int prow = sa * NPX + y;
    const float* src = a.opd + (int64_t)f * a.frame_stride + (int64_t)w * a.wfs_stride +
                       (int64_t)prow * a.row_pitch + (int64_t)sb * NPX;
    const float ay = (float)prow + 0.5f - a.half_n;
    const float ay2 = ay * ay;
    float2 z[NPX];
#pragma unroll
    for (int x = 0; x < NPX; ++x) {
      const float ax = (float)(sb * NPX + x) + 0.5f - a.half_n;
      const float r2 = ax * ax + ay2;
      const bool lit = (r2 <= a.r2_outer) && (r2 >= a.r2_inner);
      // waves: OPD / lambda + centring ramp (FFT_N-1)(x+y)/(2 FFT_N) - x k2 / FFT_N
      const double ramp = (double)((FFT_N - 1) * (x + y)) / (2.0 * FFT_N) - (double)(x * k2) / (double)FFT_N;
      double wv = (double)src[x] * a.inv_lambda + ramp;
      wv -= floor(wv);
      float sn, cs;
      sincospif(2.0f * (float)wv, &sn, &cs);
      z[x] = lit ? make_float2(cs, sn) : make_float2(0.0f, 0.0f);
    }
    RegFFT<NPX, -1>::run(z);
#pragma unroll
    for (int k1 = 0; k1 < NPX; ++k1) {
      re[y * ST + k2 + R * k1] = z[k1].x;
      im[y * ST + k2 + R * k1] = z[k1].y;
    }
  }
  __syncthreads();

  // ---------------------------------------------------------------- A': column pass, |F|^2
  float col[CONV_N];
#pragma unroll
  for (int v = 0; v < CONV_N; ++v) col[v] = 0.0f;
  {
    const int u = l - OFF;
    if (active && u >= 0 && u < FFT_N) {
      float2 g[NPX];
#pragma unroll
      for (int y = 0; y < NPX; ++y) g[y] = make_float2(re[y * ST + u], im[y * ST + u]);
#pragma unroll
      for (int k2 = 0; k2 < R; ++k2) {
        float2 z[NPX];
#pragma unroll
        for (int y = 0; y < NPX; ++y) z[y] = twiddle_mul<FFT_N, -1>(g[y], y * k2);
        RegFFT<NPX, -1>::run(z);
#pragma unroll
        for (int k1 = 0; k1 < NPX; ++k1) col[OFF + k2 + R * k1] = (z[k1].x * z[k1].x + z[k1].y * z[k1].y) * INV_N2;
      }
    }
  }

  // ---------------------------------------------------------------- B: convolution with k
  if constexpr (LGS) {
    __syncthreads();  // every lane has read the row-pass plane
    {
      float2 z[CONV_N];
#pragma unroll
      for (int v = 0; v < CONV_N; ++v) z[v] = make_float2(col[v], 0.0f);
      RegFFT<CONV_N, -1>::run(z);
#pragma unroll
      for (int k = 0; k < H; ++k) {
        re[k * ST + l] = z[k].x;
        im[k * ST + l] = z[k].y;
      }
    }
    __syncthreads();
    if (active && l < H) {
      float2 z[CONV_N];
#pragma unroll
      for (int u = 0; u < CONV_N; ++u) z[u] = make_float2(re[l * ST + u], im[l * ST + u]);
      RegFFT<CONV_N, -1>::run(z);
      const float* kh = a.khat + ((int64_t)(w * a.n_valid + i) * H + l) * CONV_N;
#pragma unroll
      for (int u = 0; u < CONV_N; ++u) z[u] = cscale(z[u], kh[u]);
      RegFFT<CONV_N, 1>::run(z);
#pragma unroll
      for (int u = 0; u < CONV_N; ++u) {
        re[l * ST + u] = z[u].x;
        im[l * ST + u] = z[u].y;
      }
    }
    __syncthreads();
    {
      float2 z[CONV_N];
#pragma unroll
      for (int k = 0; k < H; ++k) z[k] = make_float2(re[k * ST + l], im[k * ST + l]);
#pragma unroll
      for (int k = 1; k < CONV_N / 2; ++k) z[CONV_N - k] = cconj(z[k]);
      RegFFT<CONV_N, 1>::run(z);
#pragma unroll
      for (int v = 0; v < CONV_N; ++v) col[v] = z[v].x;
    }
  }

  // ---------------------------------------------------------------- C: rebin
  __syncthreads();  // the planes are free
#pragma unroll
  for (int p = 0; p < DET_N; ++p) {
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < CONV_N; ++k) {
      const float wgt = rebin_weight(CONV_N, DET_N, p, k);
      if (wgt != 0.0f) acc += wgt * col[k];
    }
    re[p * ST + l] = acc;
  }
  __syncthreads();

  // ---------------------------------------------------------------- D: photometry, noise, centroid
  constexpr float B = (float)CONV_N / (float)DET_N;
  constexpr float CD = 0.5f * (float)(DET_N - 1);
  double s0 = 0.0, sx = 0.0, sy = 0.0;
  const uint32_t gsub = (uint32_t)(w * a.n_valid + i);
  const uint32_t frame = a.frame0 + (uint32_t)f;
  if (active) {
#pragma unroll 1
    for (int j = 0; j < PIX_ITERS; ++j) {
      const int pix = l + L * j;
      if (pix >= NPIX) break;
      const int p = pix / DET_N;
      const int q = pix - p * DET_N;
      const float lo = B * (float)q, hi = B * (float)(q + 1);
      const int kb = (int)floorf(lo);
      const int ke = min((int)ceilf(hi), CONV_N);
      float det = 0.0f;
      for (int k = kb; k < ke; ++k) {
        const float wgt = fminf((float)(k + 1), hi) - fmaxf((float)k, lo);
        if (wgt > 0.0f) det += wgt * re[p * ST + k];
      }
      float img = det;
      if (a.ph_scale > 0.0f) {
        const float lam = a.ph_scale * det;
        img = a.noise ? noisy_pixel(lam, a.ron, (uint32_t)pix, gsub, frame, a.key0, a.key1) : lam;
      }
      if (a.images) a.images[item * NPIX + pix] = img;
      const double t = (double)fmaxf(img - a.thr, 0.0f);
      s0 += t;
      sx += (double)((float)q - CD) * t;
      sy += (double)((float)p - CD) * t;
    }
  }
  double* red = reinterpret_cast<double*>(im);
  red[l] = s0;
  red[L + l] = sx;
  red[2 * L + l] = sy;
  __syncthreads();
  if (active && l == 0) {
    double t0 = 0.0, tx = 0.0, ty = 0.0;
    for (int j = 0; j < L; ++j) {
      t0 += red[j];
      tx += red[L + j];
      ty += red[2 * L + j];
    }
    const int64_t fw = item / a.n_valid;
    const bool empty = !(t0 > 0.0);
    a.slopes[(fw * 2) * a.n_valid + i] = empty ? 0.0f : (float)(tx / t0);
    a.slopes[(fw * 2 + 1) * a.n_valid + i] = empty ? 0.0f : (float)(ty / t0);
    if (a.flags) a.flags[item] = empty ? 1 : 0;
  }
}

// Items per block: the smallest count whose lanes fill whole 64-wide waves, at least 256 lanes.
constexpr int items_per_block(int lanes) {
  int spb = 1;
  while ((spb * lanes) % 64 != 0 || spb * lanes < 256) ++spb;
  return spb;
}

template <int NPX, int FFT_N, int CONV_N, int DET_N, bool LGS>
static hipError_t launch_one(const WfsLaunch& a, hipStream_t st) {
  constexpr int SPB = items_per_block(CONV_N);
  const int64_t blocks = (a.total + SPB - 1) / SPB;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((wfs_fused_kernel<NPX, FFT_N, CONV_N, DET_N, LGS, SPB>), dim3((unsigned)blocks),
                     dim3(SPB * CONV_N), 0, st, a);
  return hipGetLastError();
}

#define SHW_WFS_SHAPES(X)     \
  X(8, 16, 16, 8, false)      \
  X(8, 16, 16, 8, true)       \
  X(8, 16, 16, 16, false)     \
  X(10, 40, 40, 16, true)     \
  X(10, 40, 40, 16, false)    \
  X(10, 40, 40, 40, false)    \
  X(10, 20, 40, 16, true)     \
  X(10, 20, 20, 10, false)

bool wfs_shape_supported(const WfsShape& s) {
#define X(np, fn, cn, dn, lg) \
  if (s.npx == np && s.fft_n == fn && s.conv_n == cn && s.det_n == dn && (s.lgs != 0) == lg) return true;
  SHW_WFS_SHAPES(X)
#undef X
  return false;
}

hipError_t launch_wfs_fused(const WfsShape& s, const WfsLaunch& a, hipStream_t st) {
#define X(np, fn, cn, dn, lg) \
  if (s.npx == np && s.fft_n == fn && s.conv_n == cn && s.det_n == dn && (s.lgs != 0) == lg) \
    return launch_one<np, fn, cn, dn, lg>(a, st);
  SHW_WFS_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- kernel spectra (plan setup)
// One block per sub-aperture: k on the CONV_N grid summed over the symmetric
// lattice window |tx|, |ty| <= 3 CONV_N, normalised to unit sum, then the real
// part of its 2-D DFT by two real separable passes, all in FP64.
template <int CN>
__global__ __launch_bounds__(256) void lgs_spectra_kernel(const double* __restrict__ params, int64_t n,
                                                         float* __restrict__ out) {
  constexpr int H = CN / 2 + 1;
  __shared__ double kk[CN * CN];
  __shared__ double t1[CN * CN];
  __shared__ double t2[CN * CN];
  __shared__ double cs[CN], sn[CN];
  __shared__ double part[256];
  const int64_t idx = blockIdx.x;
  if (idx >= n) return;
  const double sp = params[3 * idx], sq = params[3 * idx + 1], psi = params[3 * idx + 2];
  const double c = cos(psi), s = sin(psi);
  const double ip2 = 1.0 / (sp * sp), iq2 = 1.0 / (sq * sq);
  const int tid = threadIdx.x;
  double mine = 0.0;
  for (int e = tid; e < CN * CN; e += 256) {
    const int r = e / CN, col = e - r * CN;
    double acc = 0.0;
    for (int my = -4; my <= 4; ++my) {
      const int ty = r + my * CN;
      if (ty < -3 * CN || ty > 3 * CN) continue;
      for (int mx = -4; mx <= 4; ++mx) {
        const int tx = col + mx * CN;
        if (tx < -3 * CN || tx > 3 * CN) continue;
        const double along = tx * c + ty * s;
        const double across = -tx * s + ty * c;
        acc += exp(-0.5 * (along * along * ip2 + across * across * iq2));
      }
    }
    kk[e] = acc;
    mine += acc;
  }
  if (tid < CN) {
    double sv, cv;
    sincospi(2.0 * tid / CN, &sv, &cv);
    cs[tid] = cv;
    sn[tid] = sv;
  }
  part[tid] = mine;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  const double inv_tot = 1.0 / part[0];
  // t1[r][l] = sum_j k[r][j] cos(2 pi l j / CN), t2 with sin
  for (int e = tid; e < CN * CN; e += 256) {
    const int r = e / CN, l = e - r * CN;
    double a1 = 0.0, a2 = 0.0;
    for (int j = 0; j < CN; ++j) {
      const int m = (l * j) % CN;
      a1 += kk[r * CN + j] * cs[m];
      a2 += kk[r * CN + j] * sn[m];
    }
    t1[e] = a1;
    t2[e] = a2;
  }
  __syncthreads();
  const double scale = inv_tot / ((double)CN * (double)CN);
  for (int e = tid; e < H * CN; e += 256) {
    const int k = e / CN, l = e - k * CN;
    double acc = 0.0;
    for (int r = 0; r < CN; ++r) {
      const int m = (k * r) % CN;
      acc += cs[m] * t1[r * CN + l] - sn[m] * t2[r * CN + l];
    }
    out[idx * H * CN + e] = (float)(acc * scale);
  }
}

hipError_t launch_lgs_spectra(int conv_n, const double* d_params, int64_t n, float* d_out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  switch (conv_n) {
    case 16:
      hipLaunchKernelGGL(lgs_spectra_kernel<16>, dim3((unsigned)n), dim3(256), 0, st, d_params, n, d_out);
      break;
    case 20:
      hipLaunchKernelGGL(lgs_spectra_kernel<20>, dim3((unsigned)n), dim3(256), 0, st, d_params, n, d_out);
      break;
    case 40:
      hipLaunchKernelGGL(lgs_spectra_kernel<40>, dim3((unsigned)n), dim3(256), 0, st, d_params, n, d_out);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace shw
