// noise.h - counter-based photon and read noise for detector pixels.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As
// Easy as 1, 2, 3", SC'11); Poisson counts by sequential-search inversion
// below mean 10 and by the transformed rejection with squeeze (PTRS) of
// W. Hormann, "The transformed rejection method for generating Poisson
// random variables" (1993) from mean 10; Gaussian read noise by
// Box-Muller.  The integer decisions are taken in FP32 with contraction
// off, operation by operation in the order written.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shw {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

// ((x >> 9) + 1/2) * 2^-23: exact in FP32, never 0 or 1.
__device__ __forceinline__ float u01(uint32_t x) {
  return ((float)(x >> 9) + 0.5f) * 1.1920928955078125e-07f;
}

__device__ __noinline__ int poisson_inversion(float lam, float u) {
#pragma clang fp contract(off)
  float p = expf(-lam);
  float F = p;
  int k = 0;
  while (u > F && k < 100) {
    ++k;
    p = (p * lam) / (float)k;
    F = F + p;
  }
  return k;
}

__device__ __noinline__ int poisson_ptrs(float lam, float u0, float v0, uint32_t pix, uint32_t gsub,
                                         uint32_t frame, uint32_t k0, uint32_t k1) {
#pragma clang fp contract(off)
  const float slam = sqrtf(lam);
  const float loglam = logf(lam);
  const float b = 0.931f + 2.53f * slam;
  const float a = -0.059f + 0.02483f * b;
  const float invalpha = 1.1239f + 1.1328f / (b - 3.4f);
  const float vr = 0.9277f - 3.6224f / (b - 2.0f);
  float u = u0, v = v0;
  for (uint32_t t = 0; t < 64u; ++t) {
    if (t) {
      const uint4 w = philox4x32_10(make_uint4(t, pix, gsub, frame), k0, k1);
      u = u01(w.x);
      v = u01(w.y);
    }
    const float U = u - 0.5f;
    const float V = v;
    const float us = 0.5f - fabsf(U);
    const float kf = floorf((2.0f * a / us + b) * U + lam + 0.43f);
    if (us >= 0.07f && V <= vr) return kf > 0.0f ? (int)kf : 0;
    if (kf < 0.0f || (us < 0.013f && V > us)) continue;
    const float lhs = logf(V) + logf(invalpha) - logf(a / (us * us) + b);
    const float rhs = -lam + kf * loglam - lgammaf(kf + 1.0f);
    if (lhs <= rhs) return (int)kf;
  }
  return (int)floorf(lam + 0.5f);
}

// Electrons of one pixel with mean lam: Poisson counts + ron * N(0, 1).
__device__ __forceinline__ float noisy_pixel(float lam, float ron, uint32_t pix, uint32_t gsub, uint32_t frame,
                                             uint32_t k0, uint32_t k1) {
  const uint4 w = philox4x32_10(make_uint4(0u, pix, gsub, frame), k0, k1);
  int k = 0;
  if (lam > 0.0f) {
    if (lam < 10.0f)
      k = poisson_inversion(lam, u01(w.x));
    else
      k = poisson_ptrs(lam, u01(w.x), u01(w.y), pix, gsub, frame, k0, k1);
  }
  float s, c;
  sincospif(2.0f * u01(w.w), &s, &c);
  const float z = sqrtf(-2.0f * logf(u01(w.z))) * c;
  return (float)k + ron * z;
}

}  // namespace shw
