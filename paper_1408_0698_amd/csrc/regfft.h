// regfft.h - small complex FFTs held entirely in one lane's registers.
//
// Lengths with a power-of-two factor and an odd factor (10, 20, 40, ...)
// use the Good-Thomas prime-factor mapping, which needs no twiddle
// factors; the others textbook mixed-radix decimation-in-time Cooley-Tukey:
// an N-point transform is R transforms of N/R points on the decimated
// sequences, twiddles W_N^(r k1), then N/R radix-R butterflies.  All loops are fully
// unrolled, so every index and every twiddle is a compile-time constant;
// the twiddle tables are constexpr objects evaluated by the compiler.
//
// DIR = -1: forward, X[k] = sum x[n] exp(-2 pi i n k / N)
// DIR = +1: inverse without the 1/N factor.
#pragma once

#include <hip/hip_runtime.h>

#define SHW_HD __host__ __device__ __forceinline__

namespace shw {

// ---------------------------------------------------------------- compile-time sin/cos
constexpr double kPi = 3.14159265358979323846264338327950288;

// Taylor series after reduction to [-pi/4, pi/4] by octant; |error| < 1e-17.
constexpr double ct_poly_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int n = 1; n < 14; ++n) {
    term *= -x2 / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ct_poly_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int n = 1; n < 14; ++n) {
    term *= -x2 / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi j / n for integers j, n > 0, exact octant symmetry.
constexpr double ct_cos_frac(long j, long n) {
  j %= n;
  if (j < 0) j += n;
  // angle = 2 pi j / n; octant o = floor(8 j / n)
  long o = (8 * j) / n;
  double rem = 2.0 * kPi * (double)(8 * j - o * n) / (8.0 * (double)n);  // in [0, pi/4)
  switch (o) {
    case 0: return ct_poly_cos(rem);
    case 1: return ct_poly_sin(kPi / 4 - rem);
    case 2: return -ct_poly_sin(rem);
    case 3: return -ct_poly_cos(kPi / 4 - rem);
    case 4: return -ct_poly_cos(rem);
    case 5: return -ct_poly_sin(kPi / 4 - rem);
    case 6: return ct_poly_sin(rem);
    default: return ct_poly_cos(kPi / 4 - rem);
  }
}
// sin(2 pi j / n) = cos(2 pi (4 j - n) / (4 n))
constexpr double ct_sin_frac(long j, long n) { return ct_cos_frac(4 * j - n, 4 * n); }

template <int N>
struct TwiddleTable {
  float c[N];
  float s[N];
  constexpr TwiddleTable() : c(), s() {
    for (int j = 0; j < N; ++j) {
      c[j] = (float)ct_cos_frac(j, N);
      s[j] = (float)ct_sin_frac(j, N);
    }
  }
};

// ---------------------------------------------------------------- complex helpers
// The arithmetic of the transforms is written operation by operation, the fused multiply-adds
// explicit and contraction off, so that a transform rounds the same way in every kernel that
// inlines it, whatever the surrounding code lets the compiler fuse.
SHW_HD float2 cadd(float2 a, float2 b) {
#pragma clang fp contract(off)
  return make_float2(a.x + b.x, a.y + b.y);
}
SHW_HD float2 csub(float2 a, float2 b) {
#pragma clang fp contract(off)
  return make_float2(a.x - b.x, a.y - b.y);
}
SHW_HD float2 cmul(float2 a, float2 b) {
#pragma clang fp contract(off)
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
SHW_HD float2 cscale(float2 a, float s) {
#pragma clang fp contract(off)
  return make_float2(a.x * s, a.y * s);
}
// multiply by i*DIR
template <int DIR>
SHW_HD float2 cmul_i(float2 a) {
  return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
SHW_HD float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// x * W_N^(DIR * j): exp(DIR * 2 pi i j / N), with the trivial angles special-cased.
template <int N, int DIR>
SHW_HD float2 twiddle_mul(float2 x, int j) {
  j %= N;
  if (j == 0) return x;
  if (4 * j == N) return cmul_i<DIR>(x);
  if (2 * j == N) return make_float2(-x.x, -x.y);
  if (4 * j == 3 * N) return cmul_i<-DIR>(x);
  constexpr TwiddleTable<N> tw{};
  const float c = tw.c[j];
  const float s = DIR > 0 ? tw.s[j] : -tw.s[j];
  return cmul(x, make_float2(c, s));
}

// ---------------------------------------------------------------- butterflies
template <int N, int DIR>
struct RegFFT;

template <int DIR>
struct RegFFT<1, DIR> {
  static SHW_HD void run(float2*) {}
};

template <int DIR>
struct RegFFT<2, DIR> {
  static SHW_HD void run(float2* x) {
    float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <int DIR>
struct RegFFT<4, DIR> {
  static SHW_HD void run(float2* x) {
    float2 s02 = cadd(x[0], x[2]), d02 = csub(x[0], x[2]);
    float2 s13 = cadd(x[1], x[3]), d13 = cmul_i<DIR>(csub(x[1], x[3]));
    x[0] = cadd(s02, s13);
    x[2] = csub(s02, s13);
    x[1] = cadd(d02, d13);
    x[3] = csub(d02, d13);
  }
};

template <int DIR>
struct RegFFT<5, DIR> {
  static SHW_HD void run(float2* x) {
#pragma clang fp contract(off)
    constexpr float c1 = (float)ct_cos_frac(1, 5), c2 = (float)ct_cos_frac(2, 5);
    constexpr float s1 = (float)ct_sin_frac(1, 5), s2 = (float)ct_sin_frac(2, 5);
    float2 a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
    float2 a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
    float2 x0 = x[0];
    float2 t1 = make_float2(fmaf(c2, a2.x, fmaf(c1, a1.x, x0.x)), fmaf(c2, a2.y, fmaf(c1, a1.y, x0.y)));
    float2 t2 = make_float2(fmaf(c1, a2.x, fmaf(c2, a1.x, x0.x)), fmaf(c1, a2.y, fmaf(c2, a1.y, x0.y)));
    float2 u1 = cmul_i<DIR>(make_float2(fmaf(s2, b2.x, s1 * b1.x), fmaf(s2, b2.y, s1 * b1.y)));
    float2 u2 = cmul_i<DIR>(make_float2(fmaf(-s1, b2.x, s2 * b1.x), fmaf(-s1, b2.y, s2 * b1.y)));
    x[0] = cadd(x0, cadd(a1, a2));
    x[1] = cadd(t1, u1);
    x[4] = csub(t1, u1);
    x[2] = cadd(t2, u2);
    x[3] = csub(t2, u2);
  }
};

constexpr int first_radix(int n) {
  return (n % 4 == 0 && n != 8) ? 4 : (n % 2 == 0 ? 2 : (n % 5 == 0 ? 5 : (n % 3 == 0 ? 3 : n)));
}
// Largest power of two dividing n, and the inverse of a modulo m (gcd(a, m) = 1, m > 1).
constexpr int pow2_part(int n) {
  int p = 1;
  while (n % 2 == 0) {
    n /= 2;
    p *= 2;
  }
  return p;
}
constexpr int inv_mod(int a, int m) {
  for (int t = 1; t < m; ++t)
    if ((a * t) % m == 1) return t;
  return 1;
}

// Composite N.  When N = P Q with P a power of two and Q > 1 odd (coprime factors), the
// Good-Thomas prime-factor mapping: input n = (Q n1 + P n2) mod N, output k = (TP k1 + TQ k2) mod N
// with TP = 1 mod P, 0 mod Q and TQ = 0 mod P, 1 mod Q (Chinese remainders) make W_N^(n k) =
// W_P^(n1 k1) W_Q^(n2 k2): Q transforms of P points, then P transforms of Q points, and no twiddle
// factors between them.  Otherwise N = R M, decimation in time with twiddles W_N^(r k1).
template <int N, int DIR>
struct RegFFT {
  static constexpr int P = pow2_part(N);
  static constexpr bool kPrimeFactor = P > 1 && P < N;
  static constexpr int R = first_radix(N);
  static constexpr int M = N / R;
  static_assert(R * M == N && M > 1, "unsupported register FFT size");
  static SHW_HD void run(float2* x) {
    if constexpr (kPrimeFactor) {
      constexpr int Q = N / P;
      constexpr int TP = Q * inv_mod(Q % P, P);
      constexpr int TQ = P * inv_mod(P % Q, Q);
      static_assert(TP % P == 1 % P && TP % Q == 0 && TQ % P == 0 && TQ % Q == 1, "prime-factor indices");
      float2 sub[Q][P];
#pragma unroll
      for (int n2 = 0; n2 < Q; ++n2)
#pragma unroll
        for (int n1 = 0; n1 < P; ++n1) sub[n2][n1] = x[(Q * n1 + P * n2) % N];
#pragma unroll
      for (int n2 = 0; n2 < Q; ++n2) RegFFT<P, DIR>::run(sub[n2]);
#pragma unroll
      for (int k1 = 0; k1 < P; ++k1) {
        float2 t[Q];
#pragma unroll
        for (int n2 = 0; n2 < Q; ++n2) t[n2] = sub[n2][k1];
        RegFFT<Q, DIR>::run(t);
#pragma unroll
        for (int k2 = 0; k2 < Q; ++k2) x[(TP * k1 + TQ * k2) % N] = t[k2];
      }
    } else {
      float2 sub[R][M];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int m = 0; m < M; ++m) sub[r][m] = x[m * R + r];
#pragma unroll
      for (int r = 0; r < R; ++r) RegFFT<M, DIR>::run(sub[r]);
#pragma unroll
      for (int k1 = 0; k1 < M; ++k1) {
        float2 t[R];
#pragma unroll
        for (int r = 0; r < R; ++r) t[r] = twiddle_mul<N, DIR>(sub[r][k1], r * k1);
        RegFFT<R, DIR>::run(t);
#pragma unroll
        for (int k2 = 0; k2 < R; ++k2) x[k1 + M * k2] = t[k2];
      }
    }
  }
};

}  // namespace shw
