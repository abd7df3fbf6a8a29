// mfma_kernels.hip - the sub-aperture transforms as small DFT GEMMs on MFMA (precision form).
//
// Same measurement as the fused kernel (Sec. 4: field, spot by Fourier
// transform, Gaussian convolution, rebin; noise and centroid then run in
// det_noise_kernel), with every transform a product of small dense matrices
// on the matrix cores.  With N = 40, e the 10 x 10 field and W the centred
// 40 x 10 DFT:
//   F = W e W^T,  I = |F|^2 / N^2                                  (spot)
//   I^ = D I D^T on the 19 x 19 in-band frequencies k, |k| <= 9     (D: 19 x 40 DFT rows)
//   J^ = I^ . K^                                                    (sodium kernel; 1 for an NGS)
//   Det = Re(Mv J^ Mu^T),  M[p][k] = (1/N) sum_v Wb[p][v] e^{2 pi i k v / N}
// The spot of a 10-pixel field has no spectrum beyond 9 samples from zero
// (its transform is the field's autocorrelation), so I^ outside the band is
// zero and the last line equals rebin(Re IDFT(DFT(I) . K^)) exactly.  I is
// real, so I^ is Hermitian: only the 10 rows of non-negative frequency are
// formed, and Mv weighs rows 1..9 by 2 to stand for their mirror rows.
//
// One wavefront owns one sub-aperture and keeps each matrix in the MFMA
// accumulator layout (lane l, register r of tile (ti, tj) holds
// X[16 ti + 4 (l / 16) + r][16 tj + l % 16]), which is the A-operand layout
// of X^T: every step is Out = In^T M with M a constant matrix in the
// B-operand layout (tables built on the host in FP64, split into hi + lo
// there and staged in LDS); the data operand is split on the fly with the
// packed conversion instructions.  102 16x16x16 products per sub-aperture
// (12 + 36 for the spot, 18 + 24 for the band spectrum, 8 + 4 for the map),
// each taken once (BF16) or three times (split variants):
//   BF16   : A_hi B_hi
//   BF16X3 : A_hi B_hi + A_hi B_lo + A_lo B_hi (bf16 hi, bf16 of the residual)
//   FP16X3 : A_hi B_hi + 2^-11 (A_hi B_lo' + A_lo' B_hi) with lo' = fp16(2^11 residual)
// with FP32 accumulation; the phase reduction stays FP64.  The products run
// as 16x16x32 steps, two 16x16x16 products side by side along k (the
// full-rate form of gfx950's matrix cores), from a table of ready B operands
// that the host builds and each block stages in LDS once.
#include <hip/hip_runtime.h>

#include "mfma_internal.h"

namespace shw {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));

// det_noise_kernel over the items of a (wfs_kernels.hip)
hipError_t launch_det_noise16(const WfsLaunch& a, hipStream_t st);

namespace {

constexpr int kWaves = 8;    // sub-apertures per block
constexpr int kN = 40;

// Two floats to packed halves (round to nearest even), as 32 bits: element 0 in the low half.
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  const b2v v = __builtin_convertvector((f2v){a, b}, b2v);
  uint32_t u;
  __builtin_memcpy(&u, &v, 4);
  return u;
}
__device__ __forceinline__ uint32_t pk_f16(float a, float b) {
  const h2v v = __builtin_convertvector((f2v){a, b}, h2v);
  uint32_t u;
  __builtin_memcpy(&u, &v, 4);
  return u;
}
__device__ __forceinline__ float2 unpk_f16(uint32_t u) {
  h2v v;
  __builtin_memcpy(&v, &u, 4);
  return make_float2((float)v[0], (float)v[1]);
}

// Operands.  A complex data tile is one group of 8 halves per lane for each precision part,
// [re(4) | im(4)], and a real tile one group [hi(4) | lo(4)] (4 VGPRs each), so that every
// 16x16x32 product reads its A operand from contiguous registers.  A 16x16x32 step sums over 32
// values of k; two 16x16x16 products with the same output tile become one such step when their
// k runs are put side by side in both operands: lane group g holds k = 4 g .. 4 g + 3 of the
// first product in elements 0..3 and of the second in elements 4..7, for A and B alike (any
// common order of k leaves the sum unchanged).
template <int PREC>
struct Cx;
template <>
struct Cx<kPrecBf16> {
  uint4 hi;  // [re | im], bf16
};
template <>
struct Cx<kPrecBf16x3> {
  uint4 hi, lo;  // [re_hi | im_hi], [re_lo | im_lo], bf16; lo = bf16 of the residual
};
template <>
struct Cx<kPrecFp16x3> {
  uint4 hi, lo;  // fp16; lo = fp16 of 2^11 x the residual
};
template <int PREC>
struct Re;
template <>
struct Re<kPrecBf16> {
  uint2 hi;
};
template <>
struct Re<kPrecBf16x3> {
  uint4 hl;  // [hi | lo]
};
template <>
struct Re<kPrecFp16x3> {
  uint4 hl;
};

// x split into 4 packed hi halves (h) and 4 packed lo halves (l) for the precision variant.
template <int PREC>
__device__ __forceinline__ void split4(f4 x, uint2& h, uint2& l) {
  if constexpr (PREC == kPrecFp16x3) {
    // below the fp16 normal range the whole value goes to the scaled low part, so that no
    // subnormal half reaches the matrix unit
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = fabsf(x[r]) < 6.103515625e-05f ? 0.0f : x[r];
    const uint32_t p0 = pk_f16(v[0], v[1]), p1 = pk_f16(v[2], v[3]);
    const float2 b0 = unpk_f16(p0), b1 = unpk_f16(p1);
    h = make_uint2(p0, p1);
    l = make_uint2(pk_f16((x[0] - b0.x) * 2048.0f, (x[1] - b0.y) * 2048.0f),
                   pk_f16((x[2] - b1.x) * 2048.0f, (x[3] - b1.y) * 2048.0f));
  } else {
    const uint32_t p0 = pk_bf16(x[0], x[1]), p1 = pk_bf16(x[2], x[3]);
    h = make_uint2(p0, p1);
    if constexpr (PREC == kPrecBf16x3) {
      // the hi halves back as floats: a bf16 is the high 16 bits of its float
      const float b0 = __uint_as_float(p0 << 16), b1 = __uint_as_float(p0 & 0xFFFF0000u);
      const float b2 = __uint_as_float(p1 << 16), b3 = __uint_as_float(p1 & 0xFFFF0000u);
      l = make_uint2(pk_bf16(x[0] - b0, x[1] - b1), pk_bf16(x[2] - b2, x[3] - b3));
    }
  }
}

template <int PREC>
__device__ __forceinline__ Cx<PREC> split_cx(f4 re, f4 im) {
  uint2 rh, rl, ih, il;
  split4<PREC>(re, rh, rl);
  split4<PREC>(im, ih, il);
  Cx<PREC> o;
  o.hi = make_uint4(rh.x, rh.y, ih.x, ih.y);
  if constexpr (PREC != kPrecBf16) o.lo = make_uint4(rl.x, rl.y, il.x, il.y);
  return o;
}

template <int PREC>
__device__ __forceinline__ Re<PREC> split_re(f4 x) {
  uint2 h, l;
  split4<PREC>(x, h, l);
  Re<PREC> o;
  if constexpr (PREC == kPrecBf16)
    o.hi = h;
  else
    o.hl = make_uint4(h.x, h.y, l.x, l.y);
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

// One 16x16x32 step (A, B: 8 halves each) and one 16x16x16 step (4 halves each).
template <bool F16>
__device__ __forceinline__ f4 k32(f4 c, uint4 a, uint4 b) {
  if constexpr (F16) {
    h8v av, bv;
    __builtin_memcpy(&av, &a, 16);
    __builtin_memcpy(&bv, &b, 16);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, c, 0, 0, 0);
  } else {
    b8v av, bv;
    __builtin_memcpy(&av, &a, 16);
    __builtin_memcpy(&bv, &b, 16);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  }
}
template <bool F16>
__device__ __forceinline__ f4 k16(f4 c, uint2 a, uint2 b) {
  if constexpr (F16) {
    h4 av, bv;
    __builtin_memcpy(&av, &a, 8);
    __builtin_memcpy(&bv, &b, 8);
    return __builtin_amdgcn_mfma_f32_16x16x16f16(av, bv, c, 0, 0, 0);
  } else {
    s4 av, bv;
    __builtin_memcpy(&av, &a, 8);
    __builtin_memcpy(&bv, &b, 8);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, c, 0, 0, 0);
  }
}

// acc += x.re T1 + x.im T2 for constant tiles T1, T2: o points at this lane's [T1|T2] hi
// operand, whose lo operand is 64 entries on.
template <int PREC>
__device__ __forceinline__ void cx_mac(Acc<PREC>& acc, const Cx<PREC>& x, uint4 bh, uint4 bl) {
  constexpr bool F16 = PREC == kPrecFp16x3;
  acc.c = k32<F16>(acc.c, x.hi, bh);
  if constexpr (PREC == kPrecBf16x3) {
    acc.c = k32<F16>(acc.c, x.hi, bl);  // hi x lo
    acc.c = k32<F16>(acc.c, x.lo, bh);  // lo x hi
  } else if constexpr (PREC == kPrecFp16x3) {
    acc.corr = k32<F16>(acc.corr, x.hi, bl);
    acc.corr = k32<F16>(acc.corr, x.lo, bh);
  }
}
template <int PREC>
__device__ __forceinline__ void cx_mac(Acc<PREC>& acc, const Cx<PREC>& x, const uint4* o) {
  cx_mac(acc, x, o[0], PREC == kPrecBf16 ? o[0] : o[64]);
}

// acc + h += x T for a real data tile x and constant tile T: o points at this lane's (T lo, T hi).
// The 16x16x16 (hi x hi) products go to their own accumulator h: a chain that alternates
// 16x16x32 and 16x16x16 steps on one accumulator gave wrong sums.
template <int PREC>
__device__ __forceinline__ void re_mac(Acc<PREC>& acc, f4& h, const Re<PREC>& x, const uint4* o) {
  constexpr bool F16 = PREC == kPrecFp16x3;
  const uint4 b = o[0];
  const uint2 bh = make_uint2(b.z, b.w);
  if constexpr (PREC == kPrecBf16) {
    h = k16<F16>(h, x.hi, bh);
  } else {
    h = k16<F16>(h, make_uint2(x.hl.x, x.hl.y), bh);  // hi x hi
    if constexpr (PREC == kPrecBf16x3)
      acc.c = k32<F16>(acc.c, x.hl, b);  // hi x lo + lo x hi
    else
      acc.corr = k32<F16>(acc.corr, x.hl, b);
  }
}

// Value of a real-operand product: its 16x16x32 accumulator plus its 16x16x16 accumulator.
template <int PREC>
__device__ __forceinline__ f4 re_value(const Acc<PREC>& acc, f4 h) {
  if constexpr (PREC == kPrecBf16)
    return h;
  else if constexpr (PREC == kPrecBf16x3)
    return acc.c + h;
  else
    return h + acc.corr * (1.0f / 2048.0f);
}

// Scheduling fence between steps: without it the compiler issues the operand reads of every
// later step at once, and the live operands (and copies into aligned register quads) cost
// spills and about 170 moves per sub-aperture.
__device__ __forceinline__ void step_fence() { __builtin_amdgcn_sched_barrier(0); }

// This lane's entry of constant operand `op`.
__device__ __forceinline__ const uint4* opnd(const uint4* t, int op, int lane) { return t + op * 64 + lane; }

// Frequency of in-band column j (j < 19): 0..9, then -9..-1.
__device__ __forceinline__ int band_k(int j) { return j <= 9 ? j : j - 19; }

}  // namespace

template <int PREC, bool LGS>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(4))) void wfs_mfma_kernel(const WfsLaunch a, const uint4* __restrict__ ops) {
  __shared__ uint4 s_tab[kMfmaOps * 64];
  // stage the constant operands in LDS
  for (int e = threadIdx.x; e < kMfmaOps * 64; e += 64 * kWaves) s_tab[e] = ops[e];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: item arithmetic on the scalar unit
  const int64_t item = a.item0 + (int64_t)blockIdx.x * kWaves + wave;
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
    // the four samples are loaded before any is used; unlit and padding pixels masked by amplitude
    float ov[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int y = lr + r, x = lc;
      const int prow = sa * 10 + (y < 10 ? y : 0), pcol = sb * 10 + (x < 10 ? x : 0);
      ov[r] = src[(int64_t)prow * a.row_pitch + pcol];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int y = lr + r, x = lc;
      const int prow = sa * 10 + y, pcol = sb * 10 + x;
      const float ay = (float)prow + 0.5f - a.half_n, ax = (float)pcol + 0.5f - a.half_n;
      const float r2 = ax * ax + ay * ay;
      const bool lit = y < 10 && x < 10 && r2 <= a.r2_outer && r2 >= a.r2_inner;
      double wv = (double)ov[r] * a.inv_lambda;
      wv = __builtin_amdgcn_fract(wv);  // wv - floor(wv), one instruction
      // hardware sine and cosine take revolutions: exp(2 pi i wv) after the FP64 reduction
      const float fw = (float)wv;
      const float amp = lit ? 1.0f : 0.0f;
      er[r] = amp * __builtin_amdgcn_cosf(fw);
      ei[r] = amp * __builtin_amdgcn_sinf(fw);
    }
  }
  // ---------------------------------------------------------------- spot: P1 = e^T W^T (16 x 48), F = P1^T W^T
  // I = |F|^2 / N^2, split as soon as each tile is formed
  Re<PREC> Is[3][3];
  {
    const Cx<PREC> x = split_cx<PREC>(er, ei);
    f4 P1r[3], P1i[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      step_fence();
      Acc<PREC> ar, ai;
      acc_zero(ar);
      acc_zero(ai);
      cx_mac(ar, x, opnd(s_tab, kOpW + 4 * c, lane));
      cx_mac(ai, x, opnd(s_tab, kOpW + 4 * c + 2, lane));
      P1r[c] = acc_value(ar);
      P1i[c] = acc_value(ai);
    }
    Cx<PREC> y[3];
#pragma unroll
    for (int tv = 0; tv < 3; ++tv) y[tv] = split_cx<PREC>(P1r[tv], P1i[tv]);
#pragma unroll
    for (int tu = 0; tu < 3; ++tu) {
      step_fence();
      // the four operands of column tile tu, read once for the three row tiles
      const uint4* ow = opnd(s_tab, kOpW + 4 * tu, lane);
      const uint4 rh = ow[0], rl = PREC == kPrecBf16 ? rh : ow[64];
      const uint4 ih = ow[128], il = PREC == kPrecBf16 ? ih : ow[192];
#pragma unroll
      for (int tv = 0; tv < 3; ++tv) {
        Acc<PREC> ar, ai;
        acc_zero(ar);
        acc_zero(ai);
        cx_mac(ar, y[tv], rh, rl);
        cx_mac(ai, y[tv], ih, il);
        const f4 fr = acc_value(ar), fi = acc_value(ai);
        Is[tv][tu] = split_re<PREC>((fr * fr + fi * fi) * (1.0f / (float)(kN * kN)));
      }
    }
  }
  // ---------------------------------------------------------------- band spectrum: P3 = I^T D^T (48 x 16: columns
  // j < 16 only, the rows of P4 that are used), P4 = P3^T D^T (16 x 32) = I^[k(j1)][k(j2)]
  f4 Hr[2], Hi[2];
  {
    Cx<PREC> p3[3];
#pragma unroll
    for (int tu = 0; tu < 3; ++tu) {
      step_fence();
      Acc<PREC> ar, ai;
      acc_zero(ar);
      acc_zero(ai);
      f4 hr = {0.f, 0.f, 0.f, 0.f}, hi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int tv = 0; tv < 3; ++tv) {
        re_mac(ar, hr, Is[tv][tu], opnd(s_tab, kOpDre + tv, lane));
        re_mac(ai, hi, Is[tv][tu], opnd(s_tab, kOpDre + 3 + tv, lane));
      }
      p3[tu] = split_cx<PREC>(re_value(ar, hr), re_value(ai, hi));
    }
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
      step_fence();
      Acc<PREC> ar, ai;
      acc_zero(ar);
      acc_zero(ai);
#pragma unroll
      for (int tu = 0; tu < 3; ++tu) {
        cx_mac(ar, p3[tu], opnd(s_tab, kOpD + 4 * (2 * tu + tj), lane));
        cx_mac(ai, p3[tu], opnd(s_tab, kOpD + 4 * (2 * tu + tj) + 2, lane));
      }
      Hr[tj] = acc_value(ar);
      Hi[tj] = acc_value(ai);
    }
  }
  // ---------------------------------------------------------------- J^ = I^ . K^ (rows j1 < 10; other rows and
  // columns j2 >= 19 meet zero rows of the map tables)
  if constexpr (LGS) {
    // rows k = 0..20 of the stored half spectrum, which carries the 1/N^2 of a full inverse
    // transform; the map tables carry their own 1/N each, so the stored value is scaled by N^2
    const float* kh = a.khat + (int64_t)(w * a.n_valid + i) * 21 * kN;
    float kv[2][4];
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j1 = lr + r, j2 = 16 * tj + lc;
        const bool in = j1 < 10 && j2 < 19;
        const int col = (band_k(j2) + kN) % kN;
        kv[tj][r] = in ? (float)(kN * kN) * kh[j1 * kN + col] : 0.0f;
      }
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Hr[tj][r] *= kv[tj][r];
        Hi[tj][r] *= kv[tj][r];
      }
  }
  // ---------------------------------------------------------------- map: P5 = J^^T Mv^T (32 x 16), Det = Re(P5^T Mu^T)
  f4 det;
  {
    Cx<PREC> p5[2];
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
      step_fence();
      const Cx<PREC> jv = split_cx<PREC>(Hr[tj], Hi[tj]);
      Acc<PREC> ar, ai;
      acc_zero(ar);
      acc_zero(ai);
      cx_mac(ar, jv, opnd(s_tab, kOpMv, lane));
      cx_mac(ai, jv, opnd(s_tab, kOpMv + 2, lane));
      p5[tj] = split_cx<PREC>(acc_value(ar), acc_value(ai));
    }
    Acc<PREC> ad;
    acc_zero(ad);
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) cx_mac(ad, p5[tj], opnd(s_tab, kOpMu + 2 * tj, lane));
    det = acc_value(ad);
  }
  // ---------------------------------------------------------------- detector values for det_noise_kernel
  float* dst = a.det_ws + (item - a.item0) * 256;
#pragma unroll
  for (int r = 0; r < 4; ++r) dst[(lr + r) * 16 + lc] = det[r];
}

bool mfma_shape_supported(int npx, int fft_n, int conv_n, int det_n, int prec) {
  return npx == 10 && fft_n == 40 && conv_n == 40 && det_n == 16 && prec >= kPrecBf16 && prec <= kPrecFp16x3;
}

hipError_t launch_wfs_mfma(int prec, bool lgs, const WfsLaunch& a0, const uint4* ops, hipStream_t st) {
  const int64_t step = a0.det_ws_items;
  if (!a0.det_ws || step <= 0) return hipErrorInvalidValue;
  for (int64_t i0 = a0.item0; i0 < a0.total; i0 += step) {
    WfsLaunch a = a0;
    a.item0 = i0;
    a.total = a0.total - i0 < step ? a0.total : i0 + step;
    const int64_t blocks = (a.total - a.item0 + kWaves - 1) / kWaves;
    const dim3 g((unsigned)blocks), b(64 * kWaves);
    bool launched = false;
#define L(P, G)                                                          \
  if (!launched && prec == P && lgs == G) {                              \
    hipLaunchKernelGGL((wfs_mfma_kernel<P, G>), g, b, 0, st, a, ops); \
    launched = true;                                                     \
  }
    L(kPrecBf16, true)
    L(kPrecBf16x3, true)
    L(kPrecFp16x3, true)
    L(kPrecBf16, false)
    L(kPrecBf16x3, false)
    L(kPrecFp16x3, false)
#undef L
    if (!launched) return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_det_noise16(a, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace shw
