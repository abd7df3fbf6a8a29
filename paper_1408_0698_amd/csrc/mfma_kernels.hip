// mfma_kernels.hip - the sub-aperture transforms as DFT-matrix GEMMs on MFMA (precision form).
//
// Same measurement as the fused kernel (Sec. 4: field, spot by Fourier
// transform, Gaussian convolution, rebin, noise, centroid), with every
// transform written as a product of small dense matrices:
//   F = W e W^T            (centred 40x10 DFT W; e the 10x10 field)
//   I = |F|^2 / 40^2
//   X = G I G^T, Y = X . K^, J = Re(conj(G) Y conj(G)^T)   (G the 40-point DFT)
//   Det = Wb J Wb^T        (area-overlap rebin, 16x40)
// padded to 48 (three 16-row tiles).  One wavefront owns one sub-aperture
// and keeps each matrix in registers in the MFMA accumulator layout
// (lane l, register r of tile (ti, tj) holds X[16 ti + 4 (l / 16) + r][16 tj + l % 16]).
// That layout is the A-operand layout of the transposed matrix, so every
// step is R = X^T M with M a constant matrix in the B-operand layout (equal
// to the accumulator layout), and W e W^T = (e^T W^T)^T W^T needs no
// transpose through memory.  The constant matrices are split into hi + lo
// parts in FP64 on the host and staged in LDS; the data operand is split
// on the fly.  Precision variants:
//   BF16   : A_hi B_hi
//   BF16X3 : A_hi B_hi + A_hi B_lo + A_lo B_hi (bf16 hi, bf16 of the residual)
//   FP16X3 : A_hi B_hi + 2^-11 (A_hi B_lo' + A_lo' B_hi) with lo' = fp16(2^11 residual)
// with FP32 accumulation; the phase reduction and the centroid sums stay FP64.
#include <hip/hip_runtime.h>

#include "mfma_internal.h"
#include "noise.h"

namespace shw {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kT = 3;        // 48 = 3 tiles of 16
constexpr int kWaves = 4;    // sub-apertures per block

__device__ __forceinline__ short bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);  // round to nearest even
}
__device__ __forceinline__ float bf16_float(short b) { return __uint_as_float(((uint32_t)(uint16_t)b) << 16); }

// Data operand, split for the precision variant.
template <int PREC>
struct Op;
template <>
struct Op<kPrecBf16> {
  s4 hi;
};
template <>
struct Op<kPrecBf16x3> {
  s4 hi, lo;
};
template <>
struct Op<kPrecFp16x3> {
  h4 hi, lo;
};

template <int PREC>
__device__ __forceinline__ Op<PREC> split(f4 x) {
  Op<PREC> o;
  if constexpr (PREC == kPrecFp16x3) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // below the fp16 normal range the whole value goes to the scaled low part, so that
      // no subnormal half reaches the matrix unit
      const _Float16 h = fabsf(x[r]) < 6.103515625e-05f ? (_Float16)0.0f : (_Float16)x[r];
      o.hi[r] = h;
      o.lo[r] = (_Float16)((x[r] - (float)h) * 2048.0f);
    }
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const short h = bf16_bits(x[r]);
      o.hi[r] = h;
      if constexpr (PREC == kPrecBf16x3) o.lo[r] = bf16_bits(x[r] - bf16_float(h));
    }
  }
  return o;
}

// Accumulator of one output tile (FP16X3 keeps the scaled correction apart).
template <int PREC>
struct Acc {
  f4 c;
};
template <>
struct Acc<kPrecFp16x3> {
  f4 c, corr;
};

template <int PREC>
__device__ __forceinline__ void acc_zero(Acc<PREC>& a) {
  a.c = f4{0.f, 0.f, 0.f, 0.f};
  if constexpr (PREC == kPrecFp16x3) a.corr = f4{0.f, 0.f, 0.f, 0.f};
}
template <int PREC>
__device__ __forceinline__ f4 acc_value(const Acc<PREC>& a) {
  if constexpr (PREC == kPrecFp16x3)
    return a.c + a.corr * (1.0f / 2048.0f);
  else
    return a.c;
}

// acc += A * B for one 16x16x16 step; B comes from an LDS table entry (hi, lo halves).
template <int PREC>
__device__ __forceinline__ void mma(Acc<PREC>& acc, const Op<PREC>& a, const uint2* __restrict__ bt) {
  if constexpr (PREC == kPrecFp16x3) {
    const uint4 b = *reinterpret_cast<const uint4*>(bt);
    h4 bhi, blo;
    __builtin_memcpy(&bhi, &b.x, 8);
    __builtin_memcpy(&blo, &b.z, 8);
    acc.c = __builtin_amdgcn_mfma_f32_16x16x16f16(a.hi, bhi, acc.c, 0, 0, 0);
    acc.corr = __builtin_amdgcn_mfma_f32_16x16x16f16(a.hi, blo, acc.corr, 0, 0, 0);
    acc.corr = __builtin_amdgcn_mfma_f32_16x16x16f16(a.lo, bhi, acc.corr, 0, 0, 0);
  } else {
    const uint4 b = *reinterpret_cast<const uint4*>(bt);
    s4 bhi;
    __builtin_memcpy(&bhi, &b.x, 8);
    acc.c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, bhi, acc.c, 0, 0, 0);
    if constexpr (PREC == kPrecBf16x3) {
      s4 blo;
      __builtin_memcpy(&blo, &b.z, 8);
      acc.c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, blo, acc.c, 0, 0, 0);
      acc.c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.lo, bhi, acc.c, 0, 0, 0);
    }
  }
}

// Table entry of constant matrix m, tile (b, c), for this lane (16 bytes: 4 hi + 4 lo halves).
__device__ __forceinline__ const uint2* tab(const uint2* t, int m_off, int tiles_c, int b, int c, int lane) {
  return t + ((size_t)(m_off + b * tiles_c + c) * 64 + lane) * 2;
}

}  // namespace

template <int PREC, bool LGS>
__global__ __launch_bounds__(64 * kWaves) void wfs_mfma_kernel(const WfsLaunch a, const uint2* __restrict__ tables) {
  __shared__ uint2 s_tab[kMfmaTableTiles * 64 * 2];
  // stage the constant tables (hi, lo per lane and tile) in LDS
  for (int e = threadIdx.x; e < kMfmaTableTiles * 64 * 2; e += 64 * kWaves) s_tab[e] = tables[e];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t item = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (item >= a.total) return;  // no block barrier below this point
  const int64_t per_frame = (int64_t)a.n_wfs * a.n_valid;
  const int f = (int)(item / per_frame);
  const int rem = (int)(item - (int64_t)f * per_frame);
  const int w = rem / a.n_valid;
  const int i = rem - w * a.n_valid;
  const int sidx = a.valid_idx[i];
  const int sa = sidx / a.n_subap, sb = sidx - sa * a.n_subap;
  const int lr = 4 * (lane >> 4);  // first row of this lane inside a tile
  const int lc = lane & 15;        // column of this lane inside a tile

  // ---------------------------------------------------------------- field e (16 x 16 tile)
  f4 er, ei;
  {
    const float* src = a.opd + (int64_t)f * a.frame_stride + (int64_t)w * a.wfs_stride;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int y = lr + r, x = lc;
      float cr = 0.0f, ci = 0.0f;
      if (y < 10 && x < 10) {
        const int prow = sa * 10 + y, pcol = sb * 10 + x;
        const float ay = (float)prow + 0.5f - a.half_n, ax = (float)pcol + 0.5f - a.half_n;
        const float r2 = ax * ax + ay * ay;
        if (r2 <= a.r2_outer && r2 >= a.r2_inner) {
          double wv = (double)src[(int64_t)prow * a.row_pitch + pcol] * a.inv_lambda;
          wv = __builtin_amdgcn_fract(wv);  // wv - floor(wv), one instruction
          float sn, cs;
          sincospif(2.0f * (float)wv, &sn, &cs);
          cr = cs;
          ci = sn;
        }
      }
      er[r] = cr;
      ei[r] = ci;
    }
  }
  // ---------------------------------------------------------------- spot: R1 = e^T W^T (16 x 48), F = R1^T W^T
  f4 Fr[kT][kT], Fi[kT][kT];
  {
    const Op<PREC> xr = split<PREC>(er), xi = split<PREC>(ei);
    f4 R1r[kT], R1i[kT];
#pragma unroll
    for (int c = 0; c < kT; ++c) {
      Acc<PREC> ar, ai;
      acc_zero(ar);
      acc_zero(ai);
      mma(ar, xr, tab(s_tab, kTabWr, kT, 0, c, lane));
      mma(ar, xi, tab(s_tab, kTabWiNeg, kT, 0, c, lane));
      mma(ai, xr, tab(s_tab, kTabWi, kT, 0, c, lane));
      mma(ai, xi, tab(s_tab, kTabWr, kT, 0, c, lane));
      R1r[c] = acc_value(ar);
      R1i[c] = acc_value(ai);
    }
#pragma unroll
    for (int ta = 0; ta < kT; ++ta) {
      const Op<PREC> yr = split<PREC>(R1r[ta]), yi = split<PREC>(R1i[ta]);
#pragma unroll
      for (int c = 0; c < kT; ++c) {
        Acc<PREC> ar, ai;
        acc_zero(ar);
        acc_zero(ai);
        mma(ar, yr, tab(s_tab, kTabWr, kT, 0, c, lane));
        mma(ar, yi, tab(s_tab, kTabWiNeg, kT, 0, c, lane));
        mma(ai, yr, tab(s_tab, kTabWi, kT, 0, c, lane));
        mma(ai, yi, tab(s_tab, kTabWr, kT, 0, c, lane));
        Fr[ta][c] = acc_value(ar);
        Fi[ta][c] = acc_value(ai);
      }
    }
  }
  // ---------------------------------------------------------------- I = |F|^2 / N^2
  f4 J[kT][kT];
#pragma unroll
  for (int ta = 0; ta < kT; ++ta)
#pragma unroll
    for (int tc = 0; tc < kT; ++tc) J[ta][tc] = (Fr[ta][tc] * Fr[ta][tc] + Fi[ta][tc] * Fi[ta][tc]) * (1.0f / 1600.0f);

  if constexpr (LGS) {
    // T = I^T G^T: Tr = I^T C, Ti = -I^T S     (G = C - i S, symmetric)
    f4 Tr[kT][kT], Ti[kT][kT];
    {
      Op<PREC> in[kT][kT];
#pragma unroll
      for (int b = 0; b < kT; ++b)
#pragma unroll
        for (int ta = 0; ta < kT; ++ta) in[b][ta] = split<PREC>(J[b][ta]);
#pragma unroll
      for (int ta = 0; ta < kT; ++ta)
#pragma unroll
        for (int c = 0; c < kT; ++c) {
          Acc<PREC> ar, ai;
          acc_zero(ar);
          acc_zero(ai);
#pragma unroll
          for (int b = 0; b < kT; ++b) {
            mma(ar, in[b][ta], tab(s_tab, kTabC, kT, b, c, lane));
            mma(ai, in[b][ta], tab(s_tab, kTabSNeg, kT, b, c, lane));
          }
          Tr[ta][c] = acc_value(ar);
          Ti[ta][c] = acc_value(ai);
        }
    }
    // X = T^T G^T = (Tr^T C + Ti^T S) + i (Ti^T C - Tr^T S); Y = X . K^
    f4 Yr[kT][kT], Yi[kT][kT];
    {
      Op<PREC> tr[kT][kT], ti[kT][kT];
#pragma unroll
      for (int b = 0; b < kT; ++b)
#pragma unroll
        for (int ta = 0; ta < kT; ++ta) {
          tr[b][ta] = split<PREC>(Tr[b][ta]);
          ti[b][ta] = split<PREC>(Ti[b][ta]);
        }
      const float* kh = a.khat + (int64_t)(w * a.n_valid + i) * 21 * 40;
#pragma unroll
      for (int ta = 0; ta < kT; ++ta)
#pragma unroll
        for (int c = 0; c < kT; ++c) {
          Acc<PREC> ar, ai;
          acc_zero(ar);
          acc_zero(ai);
#pragma unroll
          for (int b = 0; b < kT; ++b) {
            mma(ar, tr[b][ta], tab(s_tab, kTabC, kT, b, c, lane));
            mma(ar, ti[b][ta], tab(s_tab, kTabS, kT, b, c, lane));
            mma(ai, ti[b][ta], tab(s_tab, kTabC, kT, b, c, lane));
            mma(ai, tr[b][ta], tab(s_tab, kTabSNeg, kT, b, c, lane));
          }
          const f4 xr = acc_value(ar), xi = acc_value(ai);
          // K^(k, l) from the stored half spectrum (rows 0..20), K^(k, l) = K^(-k, -l)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int k = 16 * ta + lr + r, l = 16 * c + lc;
            float kv = 0.0f;
            if (k < 40 && l < 40) kv = k <= 20 ? kh[k * 40 + l] : kh[(40 - k) * 40 + (40 - l) % 40];
            Yr[ta][c][r] = xr[r] * kv;
            Yi[ta][c][r] = xi[r] * kv;
          }
        }
    }
    // U = Y^T conj(G)^T = (Yr^T C - Yi^T S) + i (Yr^T S + Yi^T C)
    f4 Ur[kT][kT], Ui[kT][kT];
    {
      Op<PREC> yr[kT][kT], yi[kT][kT];
#pragma unroll
      for (int b = 0; b < kT; ++b)
#pragma unroll
        for (int ta = 0; ta < kT; ++ta) {
          yr[b][ta] = split<PREC>(Yr[b][ta]);
          yi[b][ta] = split<PREC>(Yi[b][ta]);
        }
#pragma unroll
      for (int ta = 0; ta < kT; ++ta)
#pragma unroll
        for (int c = 0; c < kT; ++c) {
          Acc<PREC> ar, ai;
          acc_zero(ar);
          acc_zero(ai);
#pragma unroll
          for (int b = 0; b < kT; ++b) {
            mma(ar, yr[b][ta], tab(s_tab, kTabC, kT, b, c, lane));
            mma(ar, yi[b][ta], tab(s_tab, kTabSNeg, kT, b, c, lane));
            mma(ai, yr[b][ta], tab(s_tab, kTabS, kT, b, c, lane));
            mma(ai, yi[b][ta], tab(s_tab, kTabC, kT, b, c, lane));
          }
          Ur[ta][c] = acc_value(ar);
          Ui[ta][c] = acc_value(ai);
        }
    }
    // J = Re(U^T conj(G)^T) = Ur^T C - Ui^T S   (K^ carries the 1/N^2)
    {
      Op<PREC> ur[kT][kT], ui[kT][kT];
#pragma unroll
      for (int b = 0; b < kT; ++b)
#pragma unroll
        for (int ta = 0; ta < kT; ++ta) {
          ur[b][ta] = split<PREC>(Ur[b][ta]);
          ui[b][ta] = split<PREC>(Ui[b][ta]);
        }
#pragma unroll
      for (int ta = 0; ta < kT; ++ta)
#pragma unroll
        for (int c = 0; c < kT; ++c) {
          Acc<PREC> ar;
          acc_zero(ar);
#pragma unroll
          for (int b = 0; b < kT; ++b) {
            mma(ar, ur[b][ta], tab(s_tab, kTabC, kT, b, c, lane));
            mma(ar, ui[b][ta], tab(s_tab, kTabSNeg, kT, b, c, lane));
          }
          J[ta][c] = acc_value(ar);
        }
    }
  }
  // ---------------------------------------------------------------- rebin: V = J^T Wb^T (48 x 16), Det = V^T Wb^T
  f4 det;
  {
    Op<PREC> jo[kT][kT];
#pragma unroll
    for (int b = 0; b < kT; ++b)
#pragma unroll
      for (int ta = 0; ta < kT; ++ta) jo[b][ta] = split<PREC>(J[b][ta]);
    f4 V[kT];
#pragma unroll
    for (int ta = 0; ta < kT; ++ta) {
      Acc<PREC> ar;
      acc_zero(ar);
#pragma unroll
      for (int b = 0; b < kT; ++b) mma(ar, jo[b][ta], tab(s_tab, kTabWb, 1, b, 0, lane));
      V[ta] = acc_value(ar);
    }
    Acc<PREC> ad;
    acc_zero(ad);
#pragma unroll
    for (int b = 0; b < kT; ++b) mma(ad, split<PREC>(V[b]), tab(s_tab, kTabWb, 1, b, 0, lane));
    det = acc_value(ad);
  }
  // ---------------------------------------------------------------- photometry, noise, centroid (4 pixels per lane)
  const uint32_t gsub = (uint32_t)(w * a.n_valid + i);
  const uint32_t frame = a.frame0 + (uint32_t)f;
  double s0 = 0.0, sx = 0.0, sy = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int p = lr + r, q = lc, pix = p * 16 + q;
    float img = det[r];
    if (a.ph_scale > 0.0f) {
      const float lam = a.ph_scale * det[r];
      img = a.noise ? noisy_pixel(lam, a.ron, (uint32_t)pix, 256u, gsub, frame, a.key0, a.key1) : lam;
    }
    if (a.images) a.images[item * 256 + pix] = img;
    const double t = (double)fmaxf(img - a.thr, 0.0f);
    s0 += t;
    sx += (double)((float)q - 7.5f) * t;
    sy += (double)((float)p - 7.5f) * t;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_xor(s0, off);
    sx += __shfl_xor(sx, off);
    sy += __shfl_xor(sy, off);
  }
  if (lane == 0) {
    const int64_t fw = (int64_t)f * a.n_wfs + w;
    const bool empty = !(s0 > 0.0);
    a.slopes[(fw * 2) * a.n_valid + i] = empty ? 0.0f : (float)(sx / s0);
    a.slopes[(fw * 2 + 1) * a.n_valid + i] = empty ? 0.0f : (float)(sy / s0);
    if (a.flags) a.flags[item] = empty ? 1 : 0;
  }
}

bool mfma_shape_supported(int npx, int fft_n, int conv_n, int det_n, int prec) {
  return npx == 10 && fft_n == 40 && conv_n == 40 && det_n == 16 && prec >= kPrecBf16 && prec <= kPrecFp16x3;
}

hipError_t launch_wfs_mfma(int prec, bool lgs, const WfsLaunch& a, const uint2* tables, hipStream_t st) {
  const int64_t blocks = (a.total + kWaves - 1) / kWaves;
  if (blocks <= 0) return hipSuccess;
  const dim3 g((unsigned)blocks), b(64 * kWaves);
#define L(P, G)                                                                   \
  if (prec == P && lgs == G) {                                                    \
    hipLaunchKernelGGL((wfs_mfma_kernel<P, G>), g, b, 0, st, a, tables);          \
    return hipGetLastError();                                                     \
  }
  L(kPrecBf16, true)
  L(kPrecBf16x3, true)
  L(kPrecFp16x3, true)
  L(kPrecBf16, false)
  L(kPrecBf16x3, false)
  L(kPrecFp16x3, false)
#undef L
  return hipErrorInvalidValue;
}

}  // namespace shw
