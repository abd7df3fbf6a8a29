// noise.h - counter-based photon and read noise for detector pixels.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As
// Easy as 1, 2, 3", SC'11); Poisson counts by sequential-search inversion
// below mean 20 and by the transformed rejection with squeeze (PTRS) of
// W. Hormann, "The transformed rejection method for generating Poisson
// random variables" (1993) from mean 20; Gaussian read noise by
// Box-Muller.  The integer decisions are taken in FP32 with contraction
// off, operation by operation in the order written.
//
// Counters (key = seed), for an image of n pixels, h = ceil(n / 2), global
// sub-aperture g, frame f: the pair block (0, b, g, f), b < h, serves pixels
// b and b + h: words x and y are their inversion uniforms, and Box-Muller on
// words z and w gives r cos(theta) to pixel b and r sin(theta) to pixel b + h.
// Rejection-sampler trial t >= 1 of pixel p draws block (t, p, g, f).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shw {

// ln(k!) for k < 256, FP64 at compile time (ln x = 2 atanh((x-1)/(x+1)) after
// scaling into [0.75, 1.5]), rounded to FP32.
constexpr double ct_log(double x) {
  int e = 0;
  while (x > 1.5) {
    x *= 0.5;
    ++e;
  }
  while (x < 0.75) {
    x *= 2.0;
    --e;
  }
  const double t = (x - 1.0) / (x + 1.0), t2 = t * t;
  double term = t, sum = 0.0;
  for (int n = 1; n < 80; n += 2) {
    sum += term / n;
    term *= t2;
  }
  return 2.0 * sum + e * 0.693147180559945309417232121458;
}
struct LogFactorialTable {
  float v[256];
  constexpr LogFactorialTable() : v() {
    double acc = 0.0;
    for (int k = 1; k < 256; ++k) {
      acc += ct_log((double)k);
      v[k] = (float)acc;
    }
  }
};
__constant__ const LogFactorialTable kLogFactorial = LogFactorialTable();

__device__ __forceinline__ float log_factorial(float k) {
  return k < 256.0f ? kLogFactorial.v[(int)k] : lgammaf(k + 1.0f);
}

// a ^ b ^ c as one three-input bitwise operation (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32 x 32 -> 64-bit product per multiplier (v_mad_u64_u32), split into hi and lo words
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    if (r < 2) {
      // the counters used here have wavefront-uniform words z and w (and x), which keep parts
      // of the first rounds on the scalar unit: plain XORs leave them there
      c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
    } else {
      c = make_uint4(xor3((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1, xor3((uint32_t)(p0 >> 32), c.w, k1),
                     (uint32_t)p0);
    }
  }
  return c;
}

// ((x >> 9) + 1/2) * 2^-23: exact in FP32, never 0 or 1.  Formed as 1 + (x >> 9) 2^-23 (the
// high 23 bits as the mantissa of a number in [1, 2)) minus (1 - 2^-24): both operands and the
// difference (2 (x >> 9) + 1) 2^-24 are exact.
__device__ __forceinline__ float u01(uint32_t x) {
  return __uint_as_float((x >> 9) | 0x3F800000u) - 0.999999940395355224609375f;
}

// 1/k rounded to FP32 (index 0 unused): the inversion multiplies by it instead of dividing.
struct RcpTable {
  float v[128];  // at least kInversionMaxK + 3 entries (the search reads one pass ahead)
  constexpr RcpTable() : v() {
    for (int k = 1; k < 128; ++k) v[k] = (float)(1.0 / (double)k);
  }
};
__constant__ const RcpTable kRcp = RcpTable();
constexpr int kInversionMaxK = 100;
static_assert(kInversionMaxK + 3 <= 128, "reciprocal table size");
// Means below the split take the inversion, the others PTRS.  On the GPU the inversion's steps
// cost less than a rejection trial's logarithms up to means of about 20-30 (measured), and in
// FP32 e^-20 and the search up to its cap stay well within range.
constexpr float kPoissonSplit = 20.0f;

// e^-lam for 0 <= lam < 87 (a normal result), without the out-of-range branches of expf: with
// the Cody-Waite split of the exponent, -lam log2(e) = n + r, n = rint(h) for the rounded product
// h, r = (h - n) + l where l (FMA) carries the product's rounding error and the low part of
// log2(e); then e^-lam = 2^n 2^r with the hardware base-2 exponential of r (|r| <= 1/2 + 1e-6).
__device__ __forceinline__ float exp_neg(float lam) {
#pragma clang fp contract(off)  // h - n must be the exact difference of the rounded h and n
  constexpr float kLog2E = 1.44269502162933349609375f;       // log2(e) rounded to FP32
  constexpr float kLog2ELo = 1.925963033500011079e-8f;      // log2(e) - kLog2E
  const float h = -lam * kLog2E;
  const float l = fmaf(-lam, kLog2ELo, fmaf(-lam, kLog2E, -h));
  const float n = rintf(h);
  return ldexpf(__builtin_amdgcn_exp2f((h - n) + l), (int)n);
}

// Sequential search from p0 = exp(-lam): p_k = (p_{k-1} lam) (1/k), F_k = F_{k-1} + p_k; the
// smallest k with u <= F_k (at most kInversionMaxK).  The FP32 sum saturates a few 1e-7 below 1
// for some lam, so the search also stops at the first k whose term leaves F_k unchanged (the
// mass beyond it is below the sum's rounding) rather than running on to the cap.  The step
// counter is the loop counter, the same in every lane still searching, so 1/k is a scalar load.
// Two steps per pass (kInversionMaxK is even): both sums are formed, then compared with u in
// step order, which halves the loop's scalar bookkeeping and table loads.
__device__ __forceinline__ int poisson_inversion_from(float lam, float u, float p0) {
#pragma clang fp contract(off)
  static_assert(kInversionMaxK % 2 == 0, "two steps per pass");
  float p = p0;
  float F = p;
  if (!(u > F)) return 0;
  // u > F_{kk-1} on entry to a pass, which forms F_kk (Fa) and F_{kk+1} (F); the pass loads the
  // next pass's reciprocals (index at most kInversionMaxK + 2, inside the table) before its own
  // arithmetic, so that the load's latency is not waited out at the top of the pass
  float Fa;
  int kk = 1;
  float ra = kRcp.v[1], rb = kRcp.v[2];
  do {
    const float na = kRcp.v[kk + 2], nb = kRcp.v[kk + 3];
    const float pa = (p * lam) * ra;
    Fa = F + pa;
    p = (pa * lam) * rb;
    F = Fa + p;
    ra = na;
    rb = nb;
    kk += 2;
  } while (u > F && kk < kInversionMaxK);
  if (!(u > F)) return kk - 2 + (u > Fa ? 1 : 0);  // F >= Fa: u <= Fa ends at step kk - 2
  // The sum grows until its terms fall below its rounding and then never again, so a search
  // that ran out of steps with u still above the sum saturated: its count is the first step
  // that left the sum unchanged (found by replaying the steps; this happens about once in 1e9).
  p = p0;
  F = p0;
#pragma unroll 1
  for (kk = 1; kk <= kInversionMaxK; ++kk) {
    p = (p * lam) * kRcp.v[kk];
    const float Fn = F + p;
    if (!(Fn > F)) return kk;
    F = Fn;
  }
  return kInversionMaxK;
}

// The same with p0 = exp(-lam) computed here (0 < lam < kPoissonSplit).
__device__ __forceinline__ int poisson_inversion(float lam, float u) {
  return poisson_inversion_from(lam, u, exp_neg(lam));
}

// The first STEPS steps of NJ independent inversions, advanced in lockstep with the arithmetic
// of poisson_inversion: the searches of a lane overlap instead of running one after another.
// Entries with use[j] false keep k[j] = 0.  more[j] is set for an entry still searching after
// STEPS steps; poisson_inversion_from run on it from the start (with p0[j] = exp(-lam[j])) then
// gives its count (the same steps).
// The head leaves out the stop where the sum no longer grows: an entry that reaches such a step
// has u above the sum and stays searching, so it goes to poisson_inversion, which applies it.
template <int NJ, int STEPS>
__device__ __forceinline__ void poisson_inversion_head(const float (&lam)[NJ], const float (&u)[NJ],
                                                       const bool (&use)[NJ], int (&k)[NJ], bool (&more)[NJ],
                                                       float (&p0)[NJ]) {
#pragma clang fp contract(off)
  static_assert(STEPS < kInversionMaxK, "head steps");
  float p[NJ], F[NJ];
  bool act[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    p[j] = use[j] ? exp_neg(lam[j]) : 0.0f;
    p0[j] = p[j];
    F[j] = p[j];
    k[j] = 0;
    act[j] = use[j] && u[j] > F[j];
  }
  // Branch-free steps: p and F advance for every entry, which leaves the finished ones finished
  // (F only grows), and k takes the step number while the entry is still searching.
#pragma unroll
  for (int kk = 1; kk <= STEPS; ++kk) {
    const float r = kRcp.v[kk];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      k[j] = act[j] ? kk : k[j];
      p[j] = (p[j] * lam[j]) * r;
      F[j] = F[j] + p[j];
      act[j] = act[j] && u[j] > F[j];
    }
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j) more[j] = act[j];
}

// PTRS for mean lam >= kPoissonSplit (the method holds from 10) at pixel pix: trial t = 1 .. 64
// takes the uniforms (u, v) from words x and y of block (t, pix, gsub, frame); after 64
// rejections, floor(lam + 1/2).
__device__ __forceinline__ int poisson_ptrs(float lam, uint32_t pix, uint32_t gsub, uint32_t frame, uint32_t k0,
                                            uint32_t k1) {
#pragma clang fp contract(off)
  const float slam = sqrtf(lam);
  const float loglam = logf(lam);
  const float b = 0.931f + 2.53f * slam;
  const float a = -0.059f + 0.02483f * b;
  const float invalpha = 1.1239f + 1.1328f / (b - 3.4f);
  const float vr = 0.9277f - 3.6224f / (b - 2.0f);
  for (uint32_t t = 1; t <= 64u; ++t) {
    const uint4 w = philox4x32_10(make_uint4(t, pix, gsub, frame), k0, k1);
    const float U = u01(w.x) - 0.5f;
    const float V = u01(w.y);
    const float us = 0.5f - fabsf(U);
    const float kf = floorf((2.0f * a / us + b) * U + lam + 0.43f);
    if (us >= 0.07f && V <= vr) return kf > 0.0f ? (int)kf : 0;
    if (kf < 0.0f || (us < 0.013f && V > us)) continue;
    const float lhs = logf(V) + logf(invalpha) - logf(a / (us * us) + b);
    const float rhs = -lam + kf * loglam - log_factorial(kf);
    if (lhs <= rhs) return (int)kf;
  }
  return (int)floorf(lam + 0.5f);
}

// Pair block b of an image (serves pixels b and b + h).
__device__ __forceinline__ uint4 pair_block(uint32_t b, uint32_t gsub, uint32_t frame, uint32_t k0, uint32_t k1) {
  return philox4x32_10(make_uint4(0u, b, gsub, frame), k0, k1);
}

// The two standard normals of a pair block (Box-Muller on words z and w): x for the first pixel
// of the pair, y for the second.  No integer decision depends on them, so the hardware sine and
// cosine (argument in revolutions), log2 and square root are used: their ~1e-6 relative error is
// far below the read-noise tolerance.
__device__ __forceinline__ float2 read_noise_pair(uint4 w) {
  // -2 ln u = -2 ln(2) log2(u); u >= 2^-24 is a normal number, so the raw log2 needs no scaling
  const float r = __builtin_amdgcn_sqrtf(-1.38629436111989061f * __builtin_amdgcn_logf(u01(w.z)));
  const float t = u01(w.w);
  return make_float2(r * __builtin_amdgcn_cosf(t), r * __builtin_amdgcn_sinf(t));
}

// Electrons of pixel pix of an npix-pixel image with mean lam: Poisson count + ron * N(0, 1).
// Computes the pixel's pair block itself (kernels that hold both pixels of a pair share it).
__device__ __forceinline__ float noisy_pixel(float lam, float ron, uint32_t pix, uint32_t npix, uint32_t gsub,
                                             uint32_t frame, uint32_t k0, uint32_t k1) {
  const uint32_t h = (npix + 1u) >> 1;
  const bool second = pix >= h;
  const uint4 w = pair_block(second ? pix - h : pix, gsub, frame, k0, k1);
  int k = 0;
  if (lam > 0.0f) {
    if (lam < kPoissonSplit)
      k = poisson_inversion(lam, u01(second ? w.y : w.x));
    else
      k = poisson_ptrs(lam, pix, gsub, frame, k0, k1);
  }
  const float2 z = read_noise_pair(w);
  return (float)k + ron * (second ? z.y : z.x);
}

}  // namespace shw
