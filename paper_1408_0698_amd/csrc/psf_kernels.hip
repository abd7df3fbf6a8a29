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
// Every line (a row in the row pass, a column in the column pass) is
// transformed by 40 lane pairs (q, h).  First step: lane (n2 = q, h) runs the
// 20-point transform of residue h of the pruned 40-point transform over n1,
// giving Y[k1] for k1 = 2k + h, and applies its four-step twiddles.  After a
// transpose through LDS, lane (k1 = q, h) holds the samples n2 = 2t + h of
// row k1, and the 40-point transform over n2 is split radix-2 across the
// pair: 20-point transforms, twiddle, butterfly with the partner through
// DPP; lane h ends with outputs k2 = c + 20 h.  A lane thus keeps 20 complex
// values instead of 40, which keeps the kernels free of register spills.
//
// Row pass: 4 rows per block of 320 lanes; each lane of a pair computes half
// of the row's phases (all its OPD loads issued first) and swaps them with its partner.  The intermediate is
// stored in column blocks of 8: element (frame f, row y, column u) of T sits
// at ((f * M/8 + u/8) * pupil_n + y) * 8 + u % 8, so that rows write whole
// 64-byte runs and the 8 columns of a column block are one contiguous region.
// Column pass: 4 columns per block; the 8 blocks of a 32-column group (one
// 128-byte line of every accumulator row, and four column blocks of the
// intermediate) are launched 8 apart, so the dispatcher places them on one
// XCD and its L2 merges their reads of the intermediate and their writes of
// the accumulator.  Frames are accumulated in LDS (each lane owns its 20
// outputs, so no barrier), then one read-modify-write of the accumulator per
// call, 16 bytes (the block's 4 columns) per row; the on-axis sample of each
// frame is the Strehl ratio.  A 4-waves-per-
// SIMD register target (128 VGPRs) lets 3 blocks share a CU.
// Both passes have a form for pupil_n = M/2 (the Nyquist-sampled PSF), where
// every sample of the pruned transforms lies in the pupil grid, so its loads
// need no bounds masks.
#include <hip/hip_runtime.h>

#include "psf_internal.h"
#include "regfft.h"

namespace shw {

namespace {

constexpr int kM = 1600;
constexpr int kQ = 40;            // M = kQ * kQ
constexpr int kNZ = kM / 2 / kQ;  // non-zero n1 (20) = outputs per lane of the second step
constexpr int kP = 2 * kQ;        // lanes per line
constexpr int kLines = 4;         // lines per block
constexpr int kST = kQ + 1;       // odd LDS stride
constexpr int kCB = 8;            // columns per block of the intermediate
constexpr int kGroupCols = 32;    // columns per 128-byte accumulator line (8 column-pass blocks)

// Offset of element (star-frame sf, row y, column u) of the intermediate.
__device__ __forceinline__ int64_t t_index(int64_t sf, int pupil_n, int y, int u) {
  return ((sf * (kM / kCB) + (u >> 3)) * pupil_n + y) * kCB + (u & (kCB - 1));
}

// Value of the same register in the partner lane t ^ 1 (DPP quad permutation 1, 0, 3, 2).
__device__ __forceinline__ float pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float2 pair_swap(float2 v) { return make_float2(pair_swap(v.x), pair_swap(v.y)); }

// One M-point transform of a line with at most M/2 non-zero inputs v[n1] (sample 40 n1 + q),
// on lane pair (q, h) of the line; pl is the line's LDS plane.  On return lane (q, h) holds
// X[q + 40 (c + 20 h)] in x[c], c < 20.  Every lane of the block must call it.
__device__ __forceinline__ void line_transform(const float2 (&v)[kNZ], float2 (&x)[kNZ], float* pl, int q, int h) {
  float2 z[kNZ];
#pragma unroll
  for (int n1 = 0; n1 < kNZ; ++n1) z[n1] = h ? twiddle_mul<kQ, -1>(v[n1], n1) : v[n1];
  RegFFT<kNZ, -1>::run(z);
  // four-step twiddle W_M^(n2 k1), k1 = 2k + h: exact every 4 steps, products of W_M^(2 n2) between
  {
    const int n2 = q;
    constexpr float kInvM = 1.0f / (float)kM;
    const float sr = -(float)(2 * n2) * kInvM;  // 2 n2 < M
    const float2 step = make_float2(__builtin_amdgcn_cosf(sr), __builtin_amdgcn_sinf(sr));
#pragma unroll
    for (int b = 0; b < kNZ / 4; ++b) {
      const float rev = -(float)(n2 * (8 * b + h)) * kInvM;  // n2 (8 b + h) < M
      float2 t = make_float2(__builtin_amdgcn_cosf(rev), __builtin_amdgcn_sinf(rev));
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        z[4 * b + e] = cmul(z[4 * b + e], t);
        t = cmul(t, step);
      }
    }
  }
  // transpose: lane (n2, h) holds Y[2k + h]; lane (k1, h) takes samples n2 = 2t + h
#pragma unroll
  for (int k = 0; k < kNZ; ++k) pl[(2 * k + h) * kST + q] = z[k].x;
  __syncthreads();
#pragma unroll
  for (int t = 0; t < kNZ; ++t) x[t].x = pl[q * kST + 2 * t + h];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kNZ; ++k) pl[(2 * k + h) * kST + q] = z[k].y;
  __syncthreads();
#pragma unroll
  for (int t = 0; t < kNZ; ++t) x[t].y = pl[q * kST + 2 * t + h];
  __syncthreads();
  RegFFT<kNZ, -1>::run(x);
  if (h) {
#pragma unroll
    for (int c = 0; c < kNZ; ++c) x[c] = twiddle_mul<kQ, -1>(x[c], c);
  }
#pragma unroll
  for (int c = 0; c < kNZ; ++c) {
    const float2 o = pair_swap(x[c]);
    // h = 0: X[c] = E + W O (partner holds W O); h = 1: X[c + 20] = E (partner) - W O
    x[c] = h ? csub(o, x[c]) : cadd(x[c], o);
  }
}

}  // namespace

// FULL: pupil_n = M / 2, so every sample 40 n1 + q (n1 < 20) lies inside the grid.
template <bool FULL>
__global__ __launch_bounds__(kLines * kP) void psf_rows_kernel(const PsfLaunch a, int64_t f0, int nf, int64_t nrows,
                                                               float2* __restrict__ T) {
  __shared__ float s_pl[kLines * kQ * kST];
  const int tid = threadIdx.x;
  const int line = tid / kP, j = tid - line * kP;
  const int q = j >> 1, h = j & 1;
  const int64_t row = (int64_t)blockIdx.x * kLines + line;  // (star * nf + frame - f0) * pupil_n + y
  const bool active = row < nrows;
  const int64_t sf = active ? row / a.pupil_n : 0;
  const int y = active ? (int)(row - sf * a.pupil_n) : 0;
  const int64_t star = sf / nf, fl = sf - star * nf;
  float* pl = s_pl + line * kQ * kST;
  // field samples x = 40 n1 + q; lane h computes those with n1 = h (mod 2), then the pair swaps
  float2 v[kNZ];
  {
    const float* src = a.opd + star * a.star_stride + (f0 + fl) * a.frame_stride + (int64_t)y * a.row_pitch;
    const float by = (float)y + 0.5f - a.half_n;
    const float by2 = by * by;
    // every load is issued before any is used (at a clamped address), and the samples outside
    // the pupil, the annulus or the last block's rows are masked afterwards
    float ov[kNZ / 2];
#pragma unroll
    for (int i = 0; i < kNZ / 2; ++i) ov[i] = src[FULL ? kQ * (2 * i + h) + q : min(kQ * (2 * i + h) + q, a.pupil_n - 1)];
#pragma unroll
    for (int i = 0; i < kNZ / 2; ++i) {
      const int n1 = 2 * i + h;
      const int x = kQ * n1 + q;
      const float bx = (float)x + 0.5f - a.half_n;
      const float r2 = bx * bx + by2;
      const bool lit = active & (FULL || x < a.pupil_n) & (r2 <= a.r2_outer) & (r2 >= a.r2_inner);
      double wv = (double)ov[i] * a.inv_lambda + 0.5 * (double)(x + y);
      wv = __builtin_amdgcn_fract(wv);  // wv - floor(wv), one instruction
      // hardware sine and cosine take revolutions: exp(2 pi i wv) after the FP64 reduction
      const float fw = (float)wv;
      // a select, not a product with a 0/1 amplitude: samples outside the pupil may hold anything
      const float cw = __builtin_amdgcn_cosf(fw), sw = __builtin_amdgcn_sinf(fw);
      const float2 e = make_float2(lit ? cw : 0.0f, lit ? sw : 0.0f);
      const float2 o = pair_swap(e);  // the partner's sample 2 i + (1 - h)
      v[2 * i] = h ? o : e;
      v[2 * i + 1] = h ? e : o;
    }
  }
  float2 x[kNZ];
  line_transform(v, x, pl, q, h);
  if (active) {
    // column q + 40 (c + 20 h): its column block advances by 5 per c and its place in the block
    // stays q % 8, so the outputs are 40 pupil_n elements apart
    float2* dst = T + t_index(sf, a.pupil_n, y, q + kQ * kNZ * h);
    const int64_t step = (int64_t)(kQ / kCB) * a.pupil_n * kCB;
#pragma unroll
    for (int c = 0; c < kNZ; ++c) dst[c * step] = x[c];
  }
}

// Column pass.  Block b = 64 j + 8 m + x takes columns 4 m .. 4 m + 3 of the 32-column group
// g = 8 j + x (groups past the last one leave at once).
template <bool FULL>
__global__ __launch_bounds__(kLines * kP) __attribute__((amdgpu_waves_per_eu(4))) void psf_cols_kernel(const PsfLaunch a, int64_t f0, int nf,
                                                               int n_groups, const float2* __restrict__ T,
                                                               float* __restrict__ acc, float* __restrict__ strehl) {
  __shared__ float s_pl[kLines * kQ * kST];
  // per-line sums over the frames: lane (q, h) owns entries q + 40 (c + 20 h), c < 20 (no barrier)
  __shared__ float s_sum[kLines][kM];
  const int tid = threadIdx.x;
  const int line = tid / kP, j = tid - line * kP;
  const int q = j >> 1, h = j & 1;
  const int b = blockIdx.x;
  const int m = (b >> 3) & 7;
  const int g = (b >> 6) * 8 + (b & 7);
  if (g >= n_groups) return;  // the whole block
  constexpr int kGroups = kM / kGroupCols;
  const int star = g / kGroups;
  const int u0 = (g - star * kGroups) * kGroupCols + m * kLines;  // first column of the block
  const int u = u0 + line;
  float* pl = s_pl + line * kQ * kST;
  float* sum = s_sum[line];
#pragma unroll
  for (int c = 0; c < kNZ; ++c) sum[q + kQ * (c + kNZ * h)] = 0.0f;
  for (int fl = 0; fl < nf; ++fl) {
    const int64_t sf = (int64_t)star * nf + fl;
    // rows 40 n1 + q of column u, 40 x 8 elements apart; with FULL every row is inside the pupil
    const float2* src = T + t_index(sf, a.pupil_n, q, u);
    float2 v[kNZ];
#pragma unroll
    for (int n1 = 0; n1 < kNZ; ++n1)
      v[n1] = FULL || kQ * n1 + q < a.pupil_n ? src[n1 * kQ * kCB] : make_float2(0.0f, 0.0f);
    float2 x[kNZ];
    line_transform(v, x, pl, q, h);
#pragma unroll
    for (int c = 0; c < kNZ; ++c) {
      const float p = (x[c].x * x[c].x + x[c].y * x[c].y) * a.inv_norm;
      sum[q + kQ * (c + kNZ * h)] += p;
      // on-axis sample: v = u = M/2, i.e. k1 = 0, k2 = 20 (c = 0, h = 1) of column M/2
      if (strehl && u == kM / 2 && q == 0 && h == 1 && c == 0) strehl[(int64_t)star * a.n_frames + f0 + fl] = p;
    }
  }
  __syncthreads();  // every line's sums are in LDS
  // accumulator rows v, columns u0 .. u0 + 3: one 16-byte read-modify-write per row when the
  // accumulator allows it (u0 is a multiple of 4), else four 4-byte ones
  float* ac = acc + star * a.acc_stride + u0;
  if ((reinterpret_cast<uintptr_t>(ac) & 15) == 0) {
    for (int vv = tid; vv < kM; vv += kLines * kP) {
      float4* pa = reinterpret_cast<float4*>(ac + (int64_t)vv * kM);
      float4 o = *pa;
      o.x += s_sum[0][vv];
      o.y += s_sum[1][vv];
      o.z += s_sum[2][vv];
      o.w += s_sum[3][vv];
      *pa = o;
    }
  } else {
    for (int e = tid; e < kM * kLines; e += kLines * kP) {
      const int vv = e >> 2, l = e & 3;
      ac[(int64_t)vv * kM + l] += s_sum[l][vv];
    }
  }
}

bool psf_size_supported(int fft_m, int pupil_n) { return fft_m == kM && pupil_n >= 1 && pupil_n <= kM / 2; }

hipError_t launch_psf_rows(const PsfLaunch& a, int n_stars, int64_t f0, int nf, float2* T, hipStream_t st) {
  const int64_t nrows = (int64_t)n_stars * nf * a.pupil_n;
  const int64_t rb = (nrows + kLines - 1) / kLines;
  if (a.pupil_n == kM / 2)
    hipLaunchKernelGGL(psf_rows_kernel<true>, dim3((unsigned)rb), dim3(kLines * kP), 0, st, a, f0, nf, nrows, T);
  else
    hipLaunchKernelGGL(psf_rows_kernel<false>, dim3((unsigned)rb), dim3(kLines * kP), 0, st, a, f0, nf, nrows, T);
  return hipGetLastError();
}

hipError_t launch_psf_cols(const PsfLaunch& a, int n_stars, int64_t f0, int nf, const float2* T, float* acc,
                           float* strehl, hipStream_t st) {
  static_assert(kGroupCols == 8 * kLines && kM % kGroupCols == 0, "8 blocks per 32-column group");
  const int n_groups = n_stars * (kM / kGroupCols);
  const dim3 cg((unsigned)(((n_groups + 7) / 8) * 64));
  if (a.pupil_n == kM / 2)
    hipLaunchKernelGGL(psf_cols_kernel<true>, cg, dim3(kLines * kP), 0, st, a, f0, nf, n_groups, T, acc, strehl);
  else
    hipLaunchKernelGGL(psf_cols_kernel<false>, cg, dim3(kLines * kP), 0, st, a, f0, nf, n_groups, T, acc, strehl);
  return hipGetLastError();
}

}  // namespace shw
