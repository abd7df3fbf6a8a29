// band_rebin.h - the band-limited inverse column transform and column rebin of the LGS spot as
// one real linear map (the detector values of a column from its in-band spectrum values).
#pragma once

#include <hip/hip_runtime.h>

#include "regfft.h"

namespace shw {

// Band-limited column inverse transform and column rebin as one real linear map: for a column
// whose spectrum R (Hermitian, length N) is zero outside k < NB and k > N - NB, the rebinned
// values D[p] = sum_u W[p][u] J[u] of J[u] = sum_k R[k] e^(2 pi i u k / N) are
// D[p] = Re sum_{k<NB} c_k R[k] M[p][k], M[p][k] = sum_u W[p][u] e^(2 pi i u k / N), c_0 = 1, else 2.
// With two detector pixels per S = 2N/DN samples, pixel 2m + s is pixel s shifted by m S samples,
// so M[2m + s][k] = M[s][k] e^(2 pi i m k / G), G = DN/2: D[2m + s] = Re sum_j B_s[j] e^(2 pi i m j / G)
// with B_s[j] the sum of c_k R[k] M[s][k] over k = j mod G.  The real parts of the two G-point
// inverse transforms come from one complex transform of Z = H_0 + i H_1, H_s[j] = (B_s[j] +
// conj B_s[-j]) / 2 (Hermitian, so each transform alone would be real).  The table holds
// f_k c_k M[s][k], f_k = 1/2 except for j = 0 and G/2, where H_s[j] = Re B_s[j]: FP64 sums rounded
// to FP32 at compile time.
template <int N, int DN, int NB>
struct BandRebinPairs {
  static constexpr int G = DN / 2;
  float mr[2][NB];
  float mi[2][NB];
  constexpr BandRebinPairs() : mr(), mi() {
    const double bn = (double)N / (double)DN;
    for (int sp = 0; sp < 2; ++sp)
      for (int k = 0; k < NB; ++k) {
        double re = 0.0, im = 0.0;
        for (int u = 0; u < N; ++u) {
          const double lo = (double)u > bn * sp ? (double)u : bn * sp;
          const double hi = (double)(u + 1) < bn * (sp + 1) ? (double)(u + 1) : bn * (sp + 1);
          if (hi > lo) {
            re += (hi - lo) * ct_cos_frac((long)u * k, N);
            im += (hi - lo) * ct_sin_frac((long)u * k, N);
          }
        }
        const int j = k % G;
        const double f = (k == 0 ? 1.0 : 2.0) * ((j == 0 || 2 * j == G) ? 1.0 : 0.5);
        mr[sp][k] = (float)(f * re);
        mi[sp][k] = (float)(f * im);
      }
  }
};

// The rebinned detector values col[0 .. DN-1] of one column from its spectrum values R[k] =
// zr[k] + i zi[k], k < NB (zi[0] = 0; the others follow by Hermitian symmetry), by the map above:
// the two pixel phases s = 0, 1 accumulate B_s[j], the Hermitian parts H_s combine into Z = H_0 +
// i H_1, and one G-point inverse transform gives pixel 2m in Re and 2m + 1 in Im.
template <int N, int DN, int NB>
SHW_HD void band_rebin_column(const float (&zr)[NB], const float (&zi)[NB], float* col) {
  static_assert(2 * N % DN == 0 && DN % 2 == 0, "two detector pixels per whole number of samples");
  using BP = BandRebinPairs<N, DN, NB>;
  constexpr int G = BP::G;
  constexpr BP bm{};
  float2 bs[2][G];
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
#pragma unroll
    for (int j = 0; j < G; ++j) bs[sp][j] = make_float2(0.0f, 0.0f);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int j = k % G;
      const float ar = bm.mr[sp][k], ai = bm.mi[sp][k];
      bs[sp][j].x = fmaf(zr[k], ar, bs[sp][j].x);
      if (k > 0) bs[sp][j].x = fmaf(-zi[k], ai, bs[sp][j].x);
      if (j != 0 && 2 * j != G) {  // only the real part is used at j = 0 and G/2
        bs[sp][j].y = fmaf(zr[k], ai, bs[sp][j].y);
        if (k > 0) bs[sp][j].y = fmaf(zi[k], ar, bs[sp][j].y);
      }
    }
  }
  float2 zz[G];
  zz[0] = make_float2(bs[0][0].x, bs[1][0].x);
  zz[G / 2] = make_float2(bs[0][G / 2].x, bs[1][G / 2].x);
#pragma unroll
  for (int j = 1; j < G / 2; ++j) {
    const float2 h0 = make_float2(bs[0][j].x + bs[0][G - j].x, bs[0][j].y - bs[0][G - j].y);
    const float2 h1 = make_float2(bs[1][j].x + bs[1][G - j].x, bs[1][j].y - bs[1][G - j].y);
    zz[j] = make_float2(h0.x - h1.y, h0.y + h1.x);      // H_0 + i H_1
    zz[G - j] = make_float2(h0.x + h1.y, h1.x - h0.y);  // conj H_0 + i conj H_1
  }
  RegFFT<G, 1>::run(zz);
#pragma unroll
  for (int m = 0; m < G; ++m) {
    col[2 * m] = zz[m].x;
    col[2 * m + 1] = zz[m].y;
  }
}

}  // namespace shw
