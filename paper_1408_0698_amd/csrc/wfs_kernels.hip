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
//     With sodium sub-layers (SUB) A and A' repeat per sub-layer, each with
//     its own wavefront, its perspective tip-tilt and defocus added to the
//     FP64 phase, and its profile weight; the weighted spots are summed.
//     The following Gaussian convolution is linear, so summing before it
//     equals convolving every sub-layer spot and piling them up.
//  B  (LGS) real column transform, per-row transform x K^ x inverse row
//     transform, inverse column transform: J = I (*) k.
//     Band-limited variants (BL, FFT_N = CONV_N): the spot of an NPX-pixel
//     sub-aperture has no spectrum beyond NPX - 1 samples from zero (the
//     transfer function of the sub-aperture is its autocorrelation), so the
//     column spectrum of I is computed directly as the autocorrelation of
//     each row-pass column over its NPX samples, only rows 0 .. NPX-1 of the
//     half spectrum are filtered, and the inverse column transform reads
//     only those rows: the column pass, the real column transform and half
//     of the row filtering are not needed.  Their inverse column transform
//     and column rebin are one compile-time linear map (BandRebinPairs).
//  C  rebin along the column in registers (band-limited: done in B), then
//     along the row via LDS.
//  D  photometry, Poisson + read noise, threshold, centre of gravity with
//     FP64 sums, reduced over the item's lanes.  Detector-split variants
//     stop after C, write the detector values to a workspace and run D in
//     det_noise_kernel: one wavefront per item and few registers, so many
//     more waves hide the latency of the Philox chains; its centroid sums
//     are FP32 (a lane's few pixels, then a six-level tree over the lanes).
#include <hip/hip_runtime.h>

#include "band_rebin.h"
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

// 1/sqrt(n) rounded to FP32 (Newton iterations in FP64 at compile time).
template <int N>
constexpr float kBandAmp() {
  double r = 1.0 / (double)N;  // below the root, where the iteration rises monotonically to it
  for (int i = 0; i < 100; ++i) r = r * (1.5 - 0.5 * (double)N * r * r);
  return (float)r;
}

// Detector pixels per lane in the final stage: the smallest divisor QB of det_n such that
// det_n^2 / QB pixels fit on the item's lanes and conv_n QB / det_n is an integer.
constexpr int det_block(int conv_n, int det_n, int lanes) {
  for (int qb = 1; qb <= det_n; ++qb)
    if (det_n % qb == 0 && det_n * (det_n / qb) <= lanes && (conv_n * qb) % det_n == 0) return qb;
  return det_n;
}

// Value of the same register in the partner lane t ^ 1 (DPP quad permutation 1, 0, 3, 2).
__device__ __forceinline__ float pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ float2 pair_swap(float2 v) { return make_float2(pair_swap(v.x), pair_swap(v.y)); }

// Value of the same register in lane t ^ 2 (DPP quad permutation 2, 3, 0, 1).
__device__ __forceinline__ float quad_swap2(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
}
__device__ __forceinline__ float2 quad_swap2(float2 v) { return make_float2(quad_swap2(v.x), quad_swap2(v.y)); }


// floor(n / d) for n < 2^31, with (m, s) from div_magic(d).
__device__ __forceinline__ uint32_t udiv_magic(uint32_t n, uint32_t m, uint32_t s) {
  return (__umulhi(n, m) + n) >> s;
}

// v + (v of the lane selected by the DPP control) in the rows enabled by ROWS; the other rows
// add zero and keep v.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_add_f32(float v) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
// Sum over the 64 lanes of a wavefront (all lanes active), in every lane (read from lane 63): a six-level tree of pairs
// and quads (quad permutations), rows of 16 (rotations by 4 and 8), then row 0 into row 1 and row
// 2 into row 3 (broadcast of lane 15 to the next row) and rows 0-1 into row 3 (broadcast of lane
// 31).  Each value takes part in six additions, so the rounding error is at most about
// 6 * 2^-24 times the sum of the magnitudes.
__device__ __forceinline__ float wave_sum_tree(float v) {
  v = dpp_add_f32<0xB1, 0xF>(v);   // quad_perm 1, 0, 3, 2
  v = dpp_add_f32<0x4E, 0xF>(v);   // quad_perm 2, 3, 0, 1
  v = dpp_add_f32<0x124, 0xF>(v);  // row_ror 4
  v = dpp_add_f32<0x128, 0xF>(v);  // row_ror 8
  v = dpp_add_f32<0x142, 0xA>(v);  // row_bcast 15 into rows 1 and 3
  v = dpp_add_f32<0x143, 0xC>(v);  // row_bcast 31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Centroid num / den (den > 0) from the FP64 sums: FP32 operands times the hardware reciprocal,
// a relative error of a few 1e-7, far below a slope's tolerance, for a handful of instructions
// instead of an FP64 division.
__device__ __forceinline__ float centroid_ratio(double num, double den) {
  return (float)num * __builtin_amdgcn_rcpf((float)den);
}

// Per-item output buffers and noise key: from the work list, or the launch-wide layout.
struct ItemRef {
  int f, w, i;
  const float* opd_f;
  int64_t row_pitch, wfs_stride;
  float* slopes_fw;  // this frame and sensor: [2][n_valid]
  float* images_it;  // this item: [det][det] or null
  uint32_t key0, key1, frame;
};

__device__ __forceinline__ ItemRef resolve_item(const WfsLaunch& a, int64_t it, uint32_t frame_base, int npix) {
  ItemRef r;
  const int64_t per_frame = (int64_t)a.n_wfs * a.n_valid;
  if (it < (int64_t)0x80000000) {
    const uint32_t n = (uint32_t)it;
    r.f = (int)udiv_magic(n, a.dm_frame_m, a.dm_frame_s);
    const uint32_t rem = n - (uint32_t)r.f * (uint32_t)per_frame;
    r.w = (int)udiv_magic(rem, a.dm_valid_m, a.dm_valid_s);
    r.i = (int)rem - r.w * a.n_valid;
  } else {
    r.f = (int)(it / per_frame);
    const int rem = (int)(it - (int64_t)r.f * per_frame);
    r.w = rem / a.n_valid;
    r.i = rem - r.w * a.n_valid;
  }
  r.key0 = a.key0;
  r.key1 = a.key1;
  r.frame = frame_base + (uint32_t)r.f;
  if (a.list) {
    const FrameWork& fw = a.list[r.f];
    r.opd_f = fw.opd;
    r.row_pitch = fw.row_pitch;
    r.wfs_stride = fw.wfs_stride;
    r.slopes_fw = fw.slopes + (int64_t)r.w * 2 * a.n_valid;
    r.images_it = fw.images ? fw.images + ((int64_t)r.w * a.n_valid + r.i) * npix : nullptr;
    r.key0 = (uint32_t)(fw.seed & 0xFFFFFFFFu);
    r.key1 = (uint32_t)(fw.seed >> 32);
    r.frame = (uint32_t)fw.frame;
  } else {
    r.opd_f = a.opd + (int64_t)r.f * a.frame_stride;
    r.row_pitch = a.row_pitch;
    r.wfs_stride = a.wfs_stride;
    r.slopes_fw = a.slopes + ((int64_t)r.f * a.n_wfs + r.w) * 2 * a.n_valid;
    r.images_it = a.images ? a.images + it * npix : nullptr;
  }
  return r;
}

// Stage D for one item by one wavefront: photometry, Poisson + read noise, threshold and centre of
// gravity of the item's DET_N x DET_N detector values at det (global or LDS); each lane takes
// pixels l, l + 64, ...  q_pix [NPIX] and q_val [3][NPIX] are the wavefront's own queue arrays in
// LDS.  The per-pixel noise is keyed by pixel, sub-aperture and frame (reading O8), so every
// caller gives the same images; the centroid sums are FP32 (per lane, then a tree over the lanes)
// instead of FP64, which moves a slope by a few 1e-5 detector pixels at most.
template <int DET_N, int HEAD>
__device__ __forceinline__ void noise_image(const WfsLaunch& a, const ItemRef& ref, int64_t item,
                                            const float* __restrict__ det, int lane, int* __restrict__ q_pix,
                                            float* __restrict__ q_val) {
  constexpr int NPIX = DET_N * DET_N;
  constexpr float CD = 0.5f * (float)(DET_N - 1);
  const uint32_t gsub = (uint32_t)(ref.w * a.n_valid + ref.i);
  const bool need_rng = a.noise && a.ph_scale > 0.0f;
  constexpr int NJ = (NPIX + 63) / 64;
  // pair blocks serve pixels b and b + h; when h is a whole number of 64-pixel rounds
  // (n = 128 m), pixel lane + 64 j pairs with lane + 64 (j + NJ / 2) of the same lane, which
  // then draws one block for both
  constexpr int PH = (NPIX + 1) / 2;
  constexpr bool PAIRED = NJ % 2 == 0 && PH == 64 * (NJ / 2);
  float v[NJ], u[NJ], z[NJ];
  bool small[NJ];
  // all loads first, then branch-free tests (short-circuit tests would put a branch, and so a
  // wait for the load, between consecutive loads)
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int pix = lane + 64 * j;
    v[j] = pix < NPIX ? det[pix] : 0.0f;
  }
  const float scale = a.ph_scale > 0.0f ? a.ph_scale : 1.0f;  // to expected electrons
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    v[j] = scale * v[j];
    small[j] = need_rng & (lane + 64 * j < NPIX) & (v[j] > 0.0f) & (v[j] < kPoissonSplit);
  }
  if (need_rng) {
    if constexpr (PAIRED) {
#pragma unroll
      for (int j = 0; j < NJ / 2; ++j) {
        const uint4 w = pair_block((uint32_t)(lane + 64 * j), gsub, ref.frame, ref.key0, ref.key1);
        const float2 zz = read_noise_pair(w);
        u[j] = u01(w.x);
        z[j] = zz.x;
        u[j + NJ / 2] = u01(w.y);
        z[j + NJ / 2] = zz.y;
      }
    } else {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int pix = lane + 64 * j;
        const bool second = pix >= PH;
        const uint4 w = pair_block((uint32_t)(second ? pix - PH : pix), gsub, ref.frame, ref.key0, ref.key1);
        const float2 zz = read_noise_pair(w);
        u[j] = u01(second ? w.y : w.x);
        z[j] = second ? zz.y : zz.x;
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < NJ; ++j) u[j] = z[j] = 0.0f;
  }
  // Inversions: HEAD lockstep steps for the lane's pixels (most means are small and end there);
  // the ones still searching go to queue A and restart one per lane, so that the lane's long
  // searches do not hold its other pixels.  Means >= kPoissonSplit go to queue B (rejection sampler).  Both
  // queues share the LDS arrays: A from the front, B from the back.  HEAD changes which pixels reach
  // queue A, not their counts (the same steps either way).  Queue A restarts from exp(-mean),
  // recomputed (the same value the head started from).
  int k[NJ];
  bool more[NJ];
  float p0[NJ];
  poisson_inversion_head<NJ, HEAD>(v, u, small, k, more, p0);
  // centroid sums: FP32 over the lane's few pixels, then the 64-lane tree (wave_sum_tree); with
  // at most a dozen terms per lane the sums are exact to about 20 * 2^-24 of their magnitudes,
  // a few 1e-5 detector pixels at most in a slope
  float s0 = 0.0f, sx = 0.0f, sy = 0.0f;
  auto accumulate = [&](int pix, float img) {
    if (ref.images_it) ref.images_it[pix] = img;
    const int p = pix / DET_N;
    const int q = pix - p * DET_N;
    const float t = fmaxf(img - a.thr, 0.0f);
    s0 += t;
    sx = fmaf((float)q - CD, t, sx);
    sy = fmaf((float)p - CD, t, sy);
  };
  // set bits of a wavefront mask in the lanes below this one (the hardware's masked bit count)
  auto below = [](uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  };
  int na = 0, nq = 0;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int pix = lane + 64 * j;
    const bool in = pix < NPIX;
    const bool big = need_rng && in && v[j] >= kPoissonSplit;
    const uint64_t ma = __ballot(more[j]);
    const uint64_t mb = __ballot(big);
    if (more[j]) {
      const int e = na + below(ma);
      q_pix[e] = pix;
      q_val[e] = v[j];
      q_val[NPIX + e] = u[j];
      q_val[2 * NPIX + e] = z[j];
    } else if (big) {
      const int e = NPIX - 1 - (nq + below(mb));
      q_pix[e] = pix;
      q_val[e] = v[j];
      q_val[2 * NPIX + e] = z[j];
    } else if (in) {
      accumulate(pix, need_rng ? (float)k[j] + a.ron * z[j] : v[j]);
    }
    na += __popcll(ma);
    nq += __popcll(mb);
  }
  // the queues are written and read by this wavefront only: order its LDS accesses
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int e = lane; e < na; e += 64) {
    const float lam = q_val[e];
    const int kp = poisson_inversion_from(lam, q_val[NPIX + e], exp_neg(lam));
    accumulate(q_pix[e], (float)kp + a.ron * q_val[2 * NPIX + e]);
  }
  for (int t = lane; t < nq; t += 64) {
    const int e = NPIX - 1 - t;
    const int pix = q_pix[e];
    const int kp = poisson_ptrs(q_val[e], (uint32_t)pix, gsub, ref.frame, ref.key0, ref.key1);
    accumulate(pix, (float)kp + a.ron * q_val[2 * NPIX + e]);
  }
  // the queue arrays are reused by the wavefront's next item: its reads end before those writes
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // every lane of the wavefront is active here; the sums of non-negative terms are zero only
  // when every term is
  s0 = wave_sum_tree(s0);
  sx = wave_sum_tree(sx);
  sy = wave_sum_tree(sy);
  if (lane == 0) {
    const bool empty = !(s0 > 0.0f);
    const float r = __builtin_amdgcn_rcpf(s0);
    ref.slopes_fw[ref.i] = empty ? 0.0f : sx * r;
    ref.slopes_fw[a.n_valid + ref.i] = empty ? 0.0f : sy * r;
    if (a.flags && !a.list) a.flags[item] = empty ? 1 : 0;
  }
}

// LDS floats per item for the given shape.  Split row transforms keep N/2 spectrum rows (rows 0
// and N/2 packed), whole ones N/2 + 1; the detector-split variants keep no detector stage in LDS.
// Band-limited variants keep NPX spectrum rows and spread the rebinned detector rows over both planes.
template <int NPX, int FFT_N, int CONV_N, int DET_N, bool SPLIT, bool DSPLIT, bool BL = false>
struct FusedLayout {
  static constexpr int HN = CONV_N / 2;
  static constexpr int ST = CONV_N + 1;
  static constexpr int HROWS = BL ? NPX : (SPLIT ? HN : HN + 1);
  static constexpr int DROWS = BL ? (DET_N + 1) / 2 : DET_N;
  static constexpr int ROWS0 = NPX > HROWS ? NPX : HROWS;
  static constexpr int ROWS = ROWS0 > DROWS ? ROWS0 : DROWS;
  static constexpr int NPIX = DET_N * DET_N;
  static constexpr int DETA = NPIX + 1;                 // detector values, after the queue and its count
  static constexpr int RED = (DETA + NPIX + 1) & ~1;
  static constexpr int DNEED = (DSPLIT || BL) ? NPIX + 1 : RED + 6 * CONV_N;
  static constexpr int PLANE0 = ROWS * ST > DNEED ? ROWS * ST : DNEED;
  static constexpr int PLANE = (PLANE0 + 1) & ~1;
};

// One group of SPB work items (one block's worth).  Every lane of the block calls it.
template <int NPX, int FFT_N, int CONV_N, int DET_N, bool LGS, int SPB, bool SPLIT, bool SUB, bool DSPLIT,
          bool BL = false>
__device__ __forceinline__ void wfs_fused_group(const WfsLaunch& a, int64_t group, uint32_t frame_base,
                                                float* __restrict__ s_re, float* __restrict__ s_im, int tid,
                                                const float2* __restrict__ qtw) {
  constexpr int L = CONV_N;                  // lanes per item
  constexpr int R = FFT_N / NPX;             // column residues of the row pass
  constexpr int H = CONV_N / 2 + 1;          // stored half spectrum rows (kernel spectra)
  constexpr int HN = CONV_N / 2;             // half length; packed spectrum rows in LDS
  constexpr int ST = CONV_N + 1;             // odd LDS row stride (floats)
  using LY = FusedLayout<NPX, FFT_N, CONV_N, DET_N, SPLIT, DSPLIT, BL>;
  static_assert(!BL || (LGS && SPLIT && FFT_N == CONV_N && CONV_N == 4 * NPX),
                "band-limited path: LGS, split rows, FFT_N = CONV_N = 4 NPX");
  static_assert(!BL || DSPLIT || DET_N == 16, "band-limited path with noise in the kernel: 16 x 16 detector");
  constexpr int NPIX = LY::NPIX;
  // stage D reuses the imaginary plane: a queue of NPIX pixel indices, its count, then 3 L doubles
  constexpr int QCOUNT = NPIX;
  constexpr int DETA = LY::DETA;
  constexpr int RED = LY::RED;
  constexpr int PLANE = LY::PLANE;  // even: doubles stay 8-byte aligned
  constexpr int OFF = (CONV_N - FFT_N) / 2;  // spot offset in the convolution grid
  constexpr float INV_N2 = 1.0f / (float)(FFT_N * FFT_N);
  static_assert(FFT_N % NPX == 0 && CONV_N >= FFT_N && (CONV_N - FFT_N) % 2 == 0, "shape");

  const int s = tid / L;
  const int l = tid - s * L;
  const int64_t item = a.item0 + group * SPB + s;
  const bool active = item < a.total;
  const int64_t it = active ? item : a.item0;
  const ItemRef ref = resolve_item(a, it, frame_base, DET_N * DET_N);
  const int w = ref.w, i = ref.i;
  const int sidx = a.valid_idx[i];
  const int sa = (int)udiv_magic((uint32_t)sidx, a.dm_subap_m, a.dm_subap_s);
  const int sb = sidx - sa * a.n_subap;
  float* re = s_re + s * PLANE;
  float* im = s_im + s * PLANE;
  const float* opd_f = ref.opd_f;
  const int64_t row_pitch = ref.row_pitch, wfs_stride = ref.wfs_stride;
  float* slopes_fw = ref.slopes_fw;
  float* images_it = ref.images_it;
  const uint32_t key0 = ref.key0, key1 = ref.key1, frame = ref.frame;

  float col[CONV_N];
#pragma unroll
  for (int v = 0; v < CONV_N; ++v) col[v] = 0.0f;
  float2 ac[BL ? NPX : 1];  // BL: column spectrum rows 0 .. NPX-1 of this lane's column
#pragma unroll
  for (int k = 0; k < (BL ? NPX : 1); ++k) ac[k] = make_float2(0.0f, 0.0f);
  const int n_sub = SUB ? a.n_sub : 1;
#pragma unroll 1
  for (int sl = 0; sl < n_sub; ++sl) {
  if (SUB && sl > 0) __syncthreads();  // the previous sub-layer's column pass has read the plane
  // ---------------------------------------------------------------- A: row pass
  if (active && l < FFT_N) {
    // sub-layer kernels: the lane index passes through an opaque move in every sub-layer, so that
    // the FP64 ramp terms of the row (rb + x rx) are recomputed there, not kept live across the loop
    int lr = l;
    if constexpr (SUB) asm volatile("" : "+v"(lr));
    const int y = lr / R;
    const int k2 = lr - y * R;
    const int prow = sa * NPX + y;
    const float* src = opd_f + (int64_t)w * wfs_stride + (int64_t)prow * row_pitch + (int64_t)sb * NPX;
    // sub-layer kernels: the column offset passes through an opaque move in every sub-layer, so
    // that the per-pixel coordinates are recomputed there rather than kept live across the loop
    int x0 = sb * NPX;
    if constexpr (SUB) asm volatile("" : "+v"(x0));
    const float ay = (float)prow + 0.5f - a.half_n;
    const float ay2 = ay * ay;
    const double rb = (double)((FFT_N - 1) * y) * (1.0 / (2.0 * FFT_N));
    const double rx = (double)(FFT_N - 1 - 2 * k2) * (1.0 / (2.0 * FFT_N));
    double c_sub = 0.0, lx = 0.0, qy = 0.0;
    if constexpr (SUB) {
      src += (int64_t)sl * a.sub_stride;
      c_sub = 0.5 * a.sub_coef[2 * sl];
      lx = a.launch_px[2 * w];
      const double dy = (double)ay - a.launch_px[2 * w + 1];
      qy = c_sub * dy * dy;
    }
    // every OPD sample of the row is inside the pupil grid: load them all first, so that the
    // loads are in flight together, and mask unlit pixels by amplitude (no branch per pixel)
    // (the OPD is device memory: global loads, which wait on the vector memory counter only)
    using GlobalF = __attribute__((address_space(1))) const float;
    const GlobalF* gsrc = (const GlobalF*)src;
    float ov[NPX];
#pragma unroll
    for (int x = 0; x < NPX; ++x) ov[x] = gsrc[x];
    // pixel-centre x coordinates: ax0 + x is exact (half-integers far below 2^23)
    const float ax0 = (float)x0 + 0.5f - a.half_n;
    float2 z[NPX];
#pragma unroll
    for (int x = 0; x < NPX; ++x) {
      const float ax = ax0 + (float)x;
      const float r2 = ax * ax + ay2;
      const bool lit = (r2 <= a.r2_outer) && (r2 >= a.r2_inner);
      // band-limited single-layer path: the autocorrelation's 1/N enters as the amplitude
      // 1/sqrt(N) of the field (one factor per lane product instead of one per lag)
      constexpr float kAmp = BL && !SUB ? kBandAmp<FFT_N>() : 1.0f;
      const float amp = lit ? kAmp : 0.0f;
      // waves: OPD / lambda + centring ramp (FFT_N-1)(x+y)/(2 FFT_N) - x k2 / FFT_N = rb + x rx
      double wv = (double)ov[x] * a.inv_lambda + ((double)x * rx + rb);
      if constexpr (SUB) {
        const double dx = (double)ax - lx;
        wv += qy + c_sub * dx * dx;
      }
      wv = __builtin_amdgcn_fract(wv);  // wv - floor(wv), one instruction
      // hardware sine/cosine take the argument in revolutions: exp(2 pi i wv) after the FP64 reduction
      const float fw = (float)wv;
      z[x] = make_float2(amp * __builtin_amdgcn_cosf(fw), amp * __builtin_amdgcn_sinf(fw));
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
  if constexpr (BL) {
    // R[k] = sum_v I[v] w^(kv) = (1/N) sum_y G[y] conj(G[y + k]), k < NPX (zero for NPX <= k <= N/2)
    constexpr float INV_N = 1.0f / (float)FFT_N;
    const float wgt = SUB ? (float)a.sub_coef[2 * sl + 1] * INV_N : 1.0f;  // single layer: 1/N is in the field
    if (active) {
      float2 g[NPX];
#pragma unroll
      for (int y = 0; y < NPX; ++y) g[y] = make_float2(re[y * ST + l], im[y * ST + l]);
      // one FMA per real product: 4 per complex term
      float e0 = g[0].x * g[0].x;
      e0 = fmaf(g[0].y, g[0].y, e0);
#pragma unroll
      for (int y = 1; y < NPX; ++y) {
        e0 = fmaf(g[y].x, g[y].x, e0);
        e0 = fmaf(g[y].y, g[y].y, e0);
      }
      ac[0].x = SUB ? fmaf(e0, wgt, ac[0].x) : e0;
#pragma unroll
      for (int k = 1; k < NPX; ++k) {
        // G[y] conj(G[y + k])
        float tx = g[0].x * g[k].x, ty = g[0].y * g[k].x;
        tx = fmaf(g[0].y, g[k].y, tx);
        ty = fmaf(-g[0].x, g[k].y, ty);
#pragma unroll
        for (int y = 1; y + k < NPX; ++y) {
          tx = fmaf(g[y].x, g[y + k].x, tx);
          tx = fmaf(g[y].y, g[y + k].y, tx);
          ty = fmaf(g[y].y, g[y + k].x, ty);
          ty = fmaf(-g[y].x, g[y + k].y, ty);
        }
        ac[k].x = SUB ? fmaf(tx, wgt, ac[k].x) : tx;
        ac[k].y = SUB ? fmaf(ty, wgt, ac[k].y) : ty;
      }
    }
  } else {
    const float wgt = SUB ? (float)a.sub_coef[2 * sl + 1] * INV_N2 : INV_N2;
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
        for (int k1 = 0; k1 < NPX; ++k1) {
          const float p = (z[k1].x * z[k1].x + z[k1].y * z[k1].y) * wgt;
          if constexpr (SUB) {
            col[OFF + k2 + R * k1] += p;
          } else {
            col[OFF + k2 + R * k1] = p;
          }
        }
      }
    }
  }
  }  // sub-layers

  // ---------------------------------------------------------------- B: convolution with k
  // J = I (*) k through the half spectrum of the real image.  Columns: real transforms as
  // half-length complex transforms.  Rows 0 and N/2 of the column spectrum are real and are
  // packed into one complex row, leaving N/2 rows; each row is filtered by a lane pair that
  // splits its N-point transforms radix-2 (even/odd samples), exchanging halves through DPP.
  if constexpr (LGS) {
    static_assert(CONV_N % 4 == 0, "LGS convolution needs conv_n divisible by 4");
    __syncthreads();  // every lane has read the row-pass plane
    if constexpr (BL) {
      // rows 0 .. NPX-1 of the half spectrum; row 0 (real) packed with row N/2 (zero)
      re[l] = ac[0].x;
      im[l] = 0.0f;
#pragma unroll
      for (int k = 1; k < NPX; ++k) {
        re[k * ST + l] = ac[k].x;
        im[k * ST + l] = ac[k].y;
      }
    } else {
      // B1: R[k] = sum_v I[v] w^(kv), k = 0..N/2, from Z = FFT_{N/2}(I[2m] + i I[2m+1])
      float2 z[HN];
#pragma unroll
      for (int m = 0; m < HN; ++m) z[m] = make_float2(col[2 * m], col[2 * m + 1]);
      RegFFT<HN, -1>::run(z);
      float r0 = 0.0f, rh = 0.0f;
#pragma unroll
      for (int k = 0; k <= HN; ++k) {
        const float2 zk = z[k % HN];
        const float2 zc = cconj(z[(HN - k) % HN]);
        const float2 ev = cscale(cadd(zk, zc), 0.5f);
        // odd part: -i/2 (zk - zc), times w^k
        const float2 d = csub(zk, zc);
        const float2 od = twiddle_mul<CONV_N, -1>(make_float2(0.5f * d.y, -0.5f * d.x), k);
        const float2 r = cadd(ev, od);
        if (k == 0) {
          r0 = r.x;
        } else if (k == HN) {
          rh = r.x;
        } else {
          re[k * ST + l] = r.x;
          im[k * ST + l] = r.y;
        }
      }
      if constexpr (SPLIT) {
        re[l] = r0;  // rows 0 and N/2 are real: packed as one complex row
        im[l] = rh;
      } else {
        re[l] = r0;
        im[l] = 0.0f;
        re[HN * ST + l] = rh;
        im[HN * ST + l] = 0.0f;
      }
    }
    __syncthreads();
    if constexpr (!SPLIT) {
      // B2 (whole rows): lane k < N/2 + 1 transforms row k, multiplies by K^, transforms back
      if (active && l <= HN) {
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
    } else {
      // B2: lane pair (r, h): forward row transform, multiply by K^, inverse row transform.  The
      // packed row 0 mixes X[c] with conj X[-c] of the partner: its spectrum goes through LDS row
      // 0 and each lane of the item computes one of its 40 outputs.
      const int r = l >> 1, h = l & 1;
      float2 x[HN];
      const float* kh_item = a.khat + ((int64_t)(w * a.n_valid + i) * H) * CONV_N;
      if constexpr (BL) {
        // rows NPX .. N/2-1 are zero; row 0 holds the real row 0 only (row N/2 is zero), so its
        // filter is the plain product by K^ row 0.  Four lanes per row (q = l & 3, row l >> 2):
        // each transforms the samples 4t + q; spectral sample c + (N/4) m is then the sum over the
        // quad of W_4^(q m) W_N^(q c) X_q[c].  Only m = 0 and m = 3 (samples c and c - N/4) lie in
        // the spot's band, so the quad forms just those two sums (DPP adds, the same value in every
        // lane), filters them, and each lane takes back its share conj(W_N^(q c)) Z_0 +
        // conj(W_4^(3q) W_N^(q c)) Z_3 for the inverse transform.
        constexpr int M4 = CONV_N / 4;
        static_assert(M4 == NPX, "band-limited row filter: N = 4 NPX");
        const int r4 = l >> 2, q = l & 3;
        if (active) {
          float2 xq[M4];
#pragma unroll
          for (int t = 0; t < M4; ++t) xq[t] = make_float2(re[r4 * ST + 4 * t + q], im[r4 * ST + 4 * t + q]);
          RegFFT<M4, -1>::run(xq);
          // K^ row r4 at samples c and c + 3N/4 (sample 3N/4 is outside the band), from the
          // in-band copy: 2 NPX - 1 values per row, all read before the first is used
          constexpr int KB = 2 * NPX - 1;
          const float* kb = a.khat_band + ((int64_t)(w * a.n_valid + i) * NPX + r4) * KB;
          float k0[M4], k3[M4];
#pragma unroll
          for (int c = 0; c < M4; ++c) {
            k0[c] = kb[c];
            k3[c] = c > 0 ? kb[NPX - 1 + c] : 0.0f;
          }
          // sample c + 3N/4 is S3 = sum_q i^q v_q (v_q = W_N^(q c) X_q[c]); the lane's share of its
          // filtered value, conj(i^q) K3 S3, is K3 (d + i ps(d)) on even lanes and K3 (d - i ps(d))
          // on odd ones, d = v_q - v_(q^2), ps the partner lane q^1: one DPP difference and one
          // swap instead of a second product and quad sum
          const float sgn = (q & 1) ? 1.0f : -1.0f;
#pragma unroll
          for (int c = 0; c < M4; ++c) {
            const float2 w = qtw[q * M4 + c];  // W_N^(q c)
            const float2 v = cmul(xq[c], w);
            float2 y0 = make_float2(v.x + quad_swap2(v.x), v.y + quad_swap2(v.y));
            y0 = make_float2(y0.x + pair_swap(y0.x), y0.y + pair_swap(y0.y));
            float2 t = cscale(y0, k0[c]);
            if (c > 0) {
              const float2 d = make_float2(v.x - quad_swap2(v.x), v.y - quad_swap2(v.y));
              const float2 pd = pair_swap(d);
              const float2 g = make_float2(fmaf(sgn, pd.y, d.x), fmaf(-sgn, pd.x, d.y));
              t = make_float2(fmaf(k3[c], g.x, t.x), fmaf(k3[c], g.y, t.y));
            }
            xq[c] = cmul(t, cconj(w));
          }
          RegFFT<M4, 1>::run(xq);
#pragma unroll
          for (int t = 0; t < M4; ++t) {
            re[r4 * ST + 4 * t + q] = xq[t].x;
            im[r4 * ST + 4 * t + q] = xq[t].y;
          }
        }
      } else {
      if (active) {
#pragma unroll
        for (int u = 0; u < HN; ++u) x[u] = make_float2(re[r * ST + 2 * u + h], im[r * ST + 2 * u + h]);
        RegFFT<HN, -1>::run(x);
        if (h) {
#pragma unroll
          for (int c = 0; c < HN; ++c) x[c] = twiddle_mul<CONV_N, -1>(x[c], c);
        }
#pragma unroll
        for (int c = 0; c < HN; ++c) {
          const float2 o = pair_swap(x[c]);
          // h = 0: X[c] = E + W O (partner holds W O); h = 1: X[c + N/2] = E (partner) - W O
          x[c] = h ? csub(o, x[c]) : cadd(x[c], o);
        }
        if (r == 0) {
#pragma unroll
          for (int c = 0; c < HN; ++c) {
            re[c + h * HN] = x[c].x;
            im[c + h * HN] = x[c].y;
          }
        } else {
#pragma unroll
          for (int c = 0; c < HN; ++c) x[c] = cscale(x[c], kh_item[r * CONV_N + h * HN + c]);
        }
      }
      __syncthreads();
      // packed row: Y[j] = X[j] (K0 + KH)/2 + conj(X[-j]) (K0 - KH)/2, lane l takes j = l
      float2 yl = make_float2(0.0f, 0.0f);
      if (active) {
        const int m = l == 0 ? 0 : CONV_N - l;
        const float2 xj = make_float2(re[l], im[l]);
        const float2 xm = cconj(make_float2(re[m], im[m]));
        const float k0 = kh_item[l], kn = kh_item[HN * CONV_N + l];
        const float ka = 0.5f * (k0 + kn), kb = 0.5f * (k0 - kn);
        yl = cadd(cscale(xj, ka), cscale(xm, kb));
      }
      __syncthreads();
      if (active) {
        re[l] = yl.x;
        im[l] = yl.y;
      }
      __syncthreads();
      if (active) {
        if (r == 0) {
#pragma unroll
          for (int c = 0; c < HN; ++c) x[c] = make_float2(re[c + h * HN], im[c + h * HN]);
        }
        // inverse: h = 0 -> even outputs from Y[c] + Y[c+N/2]; h = 1 -> odd outputs from (Y[c] - Y[c+N/2]) W^-c
#pragma unroll
        for (int c = 0; c < HN; ++c) {
          const float2 o = pair_swap(x[c]);
          x[c] = h ? twiddle_mul<CONV_N, 1>(csub(o, x[c]), c) : cadd(x[c], o);
        }
        RegFFT<HN, 1>::run(x);
#pragma unroll
        for (int u = 0; u < HN; ++u) {
          re[r * ST + 2 * u + h] = x[u].x;
          im[r * ST + 2 * u + h] = x[u].y;
        }
      }
    
      }
    }
    __syncthreads();
    if constexpr (BL) {
      // B3 + column rebin as one linear map of the column's in-band spectrum rows (BandRebinPairs);
      // the detector rows are written after the barrier that frees the planes
      // the lane index through an opaque move: the compiler recomputes these LDS addresses here
      // instead of keeping the ones of the autocorrelation stores live across the row filter
      int lb = l;
      asm volatile("" : "+v"(lb));
      float zr[NPX], zi[NPX];
      zr[0] = re[lb];
      zi[0] = 0.0f;
#pragma unroll
      for (int k = 1; k < NPX; ++k) {
        zr[k] = re[k * ST + lb];
        zi[k] = im[k * ST + lb];
      }
      band_rebin_column<CONV_N, DET_N, NPX>(zr, zi, col);
    } else {
      // B3: real J from the half spectrum: y = IFFT_{N/2}(C), C[k] = (Z[k] + conj Z[N/2-k])
      //     + i W^-k (Z[k] - conj Z[N/2-k]); J[2m] = Re y[m], J[2m+1] = Im y[m]
      // computed in place pair by pair (k, N/2 - k): Z[k] and Z[N/2 - k] give C[k] and C[N/2 - k]
      float2 y[HN];
      const float z0 = re[l];
      const float zh = SPLIT ? im[l] : re[HN * ST + l];
#pragma unroll
      for (int k = 1; k < HN; ++k) y[k] = make_float2(re[k * ST + l], im[k * ST + l]);
      auto cfold = [](float2 zk, float2 zm, int k) {
        const float2 zc = cconj(zm);
        const float2 e = cadd(zk, zc);
        const float2 d = twiddle_mul<CONV_N, 1>(csub(zk, zc), k);
        return make_float2(e.x - d.y, e.y + d.x);
      };
      y[0] = cfold(make_float2(z0, 0.0f), make_float2(zh, 0.0f), 0);
#pragma unroll
      for (int k = 1; k <= HN / 2; ++k) {
        const int m = HN - k;
        const float2 a = y[k], b = y[m];
        y[k] = cfold(a, b, k);
        if (m != k) y[m] = cfold(b, a, m);
      }
      RegFFT<HN, 1>::run(y);
#pragma unroll
      for (int m = 0; m < HN; ++m) {
        col[2 * m] = y[m].x;
        col[2 * m + 1] = y[m].y;
      }
    }
  }

  // ---------------------------------------------------------------- C: rebin
  __syncthreads();  // the planes are free
  int* queue = reinterpret_cast<int*>(im);
  if (!DSPLIT && !BL && l == 0) queue[QCOUNT] = 0;
  // detector row p of the column-rebinned image: plane re, or (BL) rows from DROWS on in plane im
  auto det_row = [&](int p) -> float* {
    return (BL && p >= LY::DROWS) ? im + (p - LY::DROWS) * ST : re + p * ST;
  };
#pragma unroll
  for (int p = 0; p < DET_N; ++p) {
    float acc = 0.0f;
    if constexpr (BL) {
      acc = col[p];  // already rebinned along the column
    } else {
#pragma unroll
      for (int k = 0; k < CONV_N; ++k) {
        const float wgt = rebin_weight(CONV_N, DET_N, p, k);
        if (wgt != 0.0f) acc += wgt * col[k];
      }
    }
    det_row(p)[l] = acc;
  }
  __syncthreads();

  // ---------------------------------------------------------------- D: photometry, noise, centroid
  // Lane l takes detector row p = l / G and the QB consecutive pixels q0 .. q0 + QB - 1,
  // q0 = QB (l % G); b QB is an integer, so the row rebin of the block reads the KB = b QB
  // inputs from k0 = b q0 with weights known at compile time.
  // Pass 1 handles every pixel except noisy ones with mean >= kPoissonSplit, queued in LDS;
  // pass 2 runs the rejection sampler on the queue with the item's lanes side by side.
  constexpr int QB = det_block(CONV_N, DET_N, L);
  constexpr int G = DET_N / QB;
  constexpr int KB = CONV_N * QB / DET_N;
  constexpr float CD = 0.5f * (float)(DET_N - 1);
  static_assert(DET_N * G <= L && (CONV_N * QB) % DET_N == 0, "detector blocking");
  double s0 = 0.0, sx = 0.0, sy = 0.0;
  const uint32_t gsub = (uint32_t)(w * a.n_valid + i);
  auto accumulate = [&](int pix, float img) {
    const int p = pix / DET_N;
    const int q = pix - p * DET_N;
    if (images_it) images_it[pix] = img;
    const double t = (double)fmaxf(img - a.thr, 0.0f);
    s0 += t;
    sx += (double)((float)q - CD) * t;
    sy += (double)((float)p - CD) * t;
  };
  float* det_area = im + DETA;
  if constexpr (DSPLIT) {
    // it - item0 for the active lanes (the only ones that write), recomputed from the block's
    // group and the item slot rather than kept live from the start of the kernel
    int sd = s;
    asm volatile("" : "+v"(sd));
    det_area = a.det_ws + (group * SPB + sd) * NPIX;
  }
  if constexpr (BL && !DSPLIT) {
    // noise and centroid in this kernel: the detector values of the block's items go to one LDS
    // array once every lane has read the planes; then wavefronts 0 .. SPB/2 - 1 take two whole
    // images each (noise_image, as det_noise_kernel), and the last wavefront leaves (its
    // registers go to other blocks; nothing after this stage waits for it)
    float dv[QB];
    const int p = l / G;
    const int q0 = QB * (l - p * G);
    if (active && l < DET_N * G) {
      const float* row = det_row(p) + (q0 / QB) * KB;
      float in[KB];
#pragma unroll
      for (int t = 0; t < KB; ++t) in[t] = row[t];
#pragma unroll
      for (int j = 0; j < QB; ++j) {
        float det = 0.0f;
#pragma unroll
        for (int t = 0; t < KB; ++t) {
          const float wgt = rebin_weight(CONV_N, DET_N, j, t);
          if (wgt != 0.0f) det += wgt * in[t];
        }
        dv[j] = det;
      }
    }
    __syncthreads();  // every lane has read the planes
    constexpr int NW = SPB * L / 64;
    static_assert(SPB == 2 * (NW - 1), "two images for each wavefront but the last");
    // LDS: the detector values [SPB][NPIX] and one queue (NPIX + 3 NPIX words) per working
    // wavefront: three in the imaginary plane, the fourth after the detector values
    constexpr int QW = 4 * NPIX;
    static_assert(SPB * NPIX + QW <= SPB * PLANE && (NW - 2) * QW <= SPB * PLANE && NW - 1 == 4, "noise stage LDS");
    float* s_det = s_re;
    if (active && l < DET_N * G) {
#pragma unroll
      for (int j = 0; j < QB; ++j) s_det[s * NPIX + p * DET_N + q0 + j] = dv[j];
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: item arithmetic on the scalar unit
    if (wave == NW - 1) return;
    float* qbase = wave < NW - 2 ? s_im + wave * QW : s_re + SPB * NPIX;
    // unrolled: the rolled loop kept its uniform values live across both images and spilled
    // 25 scalar registers
#pragma unroll
    for (int si = 2 * wave; si < 2 * wave + 2; ++si) {
      const int64_t it2 = a.item0 + group * SPB + si;
      if (it2 >= a.total) break;  // uniform over the wavefront
      const ItemRef r2 = resolve_item(a, it2, frame_base, NPIX);
      noise_image<DET_N, 4>(a, r2, it2, s_det + si * NPIX, tid & 63, reinterpret_cast<int*>(qbase), qbase + NPIX);
    }
    return;
  } else {
  if (active && l < DET_N * G) {
    const int p = l / G;
    const int q0 = QB * (l - p * G);
    const float* row = det_row(p) + (q0 / QB) * KB;
    float in[KB];
#pragma unroll
    for (int t = 0; t < KB; ++t) in[t] = row[t];
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      float det = 0.0f;
#pragma unroll
      for (int t = 0; t < KB; ++t) {
        const float wgt = rebin_weight(CONV_N, DET_N, j, t);
        if (wgt != 0.0f) det += wgt * in[t];
      }
      det_area[p * DET_N + q0 + j] = det;
    }
  }
  if constexpr (DSPLIT) return;  // noise and centroid: det_noise_kernel
  __syncthreads();
  // every lane of the item takes pair blocks b = l, l + L, ... < h: pixels b and b + h share one
  // Philox block (their two uniforms and the two Box-Muller deviates)
  constexpr int PH = (NPIX + 1) / 2;
  auto finish = [&](int pix, float det, float u, float z) {
    float img = det;
    if (a.ph_scale > 0.0f) {
      const float lam = a.ph_scale * det;
      img = lam;
      if (a.noise) {
        if (lam >= kPoissonSplit) {
          queue[atomicAdd(&queue[QCOUNT], 1)] = pix;
          return;
        }
        const int k = lam > 0.0f ? poisson_inversion(lam, u) : 0;
        img = (float)k + a.ron * z;
      }
    }
    accumulate(pix, img);
  };
  if (active) {
    const bool need_rng = a.noise && a.ph_scale > 0.0f;
#pragma unroll 1
    for (int b = l; b < PH; b += L) {
      uint4 wd = make_uint4(0u, 0u, 0u, 0u);
      float2 z = make_float2(0.0f, 0.0f);
      if (need_rng) {
        wd = pair_block((uint32_t)b, gsub, frame, key0, key1);
        z = read_noise_pair(wd);
      }
      finish(b, det_area[b], u01(wd.x), z.x);
      if (b + PH < NPIX) finish(b + PH, det_area[b + PH], u01(wd.y), z.y);
    }
  }
  __syncthreads();
  if (active) {
    const int nq = queue[QCOUNT];
#pragma unroll 1
    for (int e = l; e < nq; e += L) {
      const int pix = queue[e];
      const float lam = a.ph_scale * det_area[pix];
      const bool second = pix >= PH;
      const float2 z = read_noise_pair(pair_block((uint32_t)(second ? pix - PH : pix), gsub, frame, key0, key1));
      const int k = poisson_ptrs(lam, (uint32_t)pix, gsub, frame, key0, key1);
      accumulate(pix, (float)k + a.ron * (second ? z.y : z.x));
    }
  }
  double* red = reinterpret_cast<double*>(im + RED);
  red[l] = s0;
  red[L + l] = sx;
  red[2 * L + l] = sy;
  __syncthreads();
  if (active && l == 0) {
    double t0 = 0.0, tx = 0.0, ty = 0.0;
#pragma unroll 4
    for (int j = 0; j < L; ++j) {
      t0 += red[j];
      tx += red[L + j];
      ty += red[2 * L + j];
    }
    const bool empty = !(t0 > 0.0);
    slopes_fw[i] = empty ? 0.0f : centroid_ratio(tx, t0);
    slopes_fw[a.n_valid + i] = empty ? 0.0f : centroid_ratio(ty, t0);
    if (a.flags && !a.list) a.flags[item] = empty ? 1 : 0;
  }
  }
}

// One-shot grid (one group per block) or persistent grid (blocks stride over the groups).
// The frame number of the first frame comes from a.frame0_dev (plus a.frame0) when set (graph replay).
template <int NPX, int FFT_N, int CONV_N, int DET_N, bool LGS, int SPB, int WPE, bool PERSIST, bool SPLIT, bool SUB,
          bool DSPLIT, bool BL>
__global__ __launch_bounds__(SPB * CONV_N) __attribute__((amdgpu_waves_per_eu(WPE))) void wfs_fused_kernel(
    const WfsLaunch a) {
  // with noise in the band-limited kernel a wavefront leaves before the others: one group only
  static_assert(!(BL && !DSPLIT && PERSIST), "band-limited noise stage: one-shot grid");
  using LY = FusedLayout<NPX, FFT_N, CONV_N, DET_N, SPLIT, DSPLIT, BL>;
  __shared__ __align__(16) float s_re[SPB * LY::PLANE];
  __shared__ __align__(16) float s_im[SPB * LY::PLANE];
  // band-limited kernels: W_N^(q c) = exp(-2 pi i q c / N), q < 4, c < N/4 (first read after a
  // barrier)
  constexpr int QTW = BL ? CONV_N : 1;
  __shared__ float2 s_qtw[QTW];
  if constexpr (BL) {
    constexpr TwiddleTable<CONV_N> tw{};
    if ((int)threadIdx.x < CONV_N) {
      const int q = threadIdx.x / (CONV_N / 4), c = threadIdx.x - q * (CONV_N / 4);
      const int j = (q * c) % CONV_N;
      s_qtw[threadIdx.x] = make_float2(tw.c[j], -tw.s[j]);
    }
  }
  // device frame counter (graph replay): *frame0_dev plus the launch's offset a.frame0
  const uint32_t frame_base = a.frame0_dev ? (uint32_t)*a.frame0_dev + a.frame0 : a.frame0;
  if constexpr (PERSIST) {
    const int64_t ngroups = (a.total - a.item0 + SPB - 1) / SPB;
    for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
      // band-limited kernels re-derive the lane index every iteration through an opaque move, so
      // that the compiler does not keep every per-lane address of the group live across the loop
      int zero = 0;
      if constexpr (BL) asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
      wfs_fused_group<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, SPLIT, SUB, DSPLIT, BL>(a, g, frame_base, s_re, s_im,
                                                                                (int)threadIdx.x + zero, s_qtw);
      __syncthreads();
    }
  } else {
    wfs_fused_group<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, SPLIT, SUB, DSPLIT, BL>(a, blockIdx.x, frame_base, s_re,
                                                                              s_im, (int)threadIdx.x, s_qtw);
  }
}

// Stage D of the detector-split variants: one wavefront per item over the detector values the
// fused kernel left in det_ws (noise_image).
template <int DET_N, int HEAD>
__global__ __launch_bounds__(256) void det_noise_kernel(const WfsLaunch a) {
  constexpr int NPIX = DET_N * DET_N;
  __shared__ int q_pix[4][NPIX];
  __shared__ float q_val[4][3 * NPIX];
  // device frame counter (graph replay): *frame0_dev plus the launch's offset a.frame0
  const uint32_t frame_base = a.frame0_dev ? (uint32_t)*a.frame0_dev + a.frame0 : a.frame0;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: item arithmetic on the scalar unit
  const int64_t item = a.item0 + (int64_t)blockIdx.x * 4 + wave;
  if (item >= a.total) return;  // whole wavefronts leave together; no block barrier below
  const ItemRef ref = resolve_item(a, item, frame_base, NPIX);
  noise_image<DET_N, HEAD>(a, ref, item, a.det_ws + (item - a.item0) * NPIX, lane, q_pix[wave], q_val[wave]);
}

// Items per block: the smallest count whose lanes fill whole 64-wide waves, at least 256 lanes.
constexpr int items_per_block(int lanes) {
  int spb = 1;
  while ((spb * lanes) % 64 != 0 || spb * lanes < 256) ++spb;
  return spb;
}

template <int NPX, int FFT_N, int CONV_N, int DET_N, bool LGS, int SPB, int WPE, bool PERSIST, bool SPLIT,
          bool SUB = false, bool DSPLIT = false, bool BL = false>
static hipError_t launch_variant(const WfsLaunch& a0, hipStream_t st) {
  auto kern = wfs_fused_kernel<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, WPE, PERSIST, SPLIT, SUB, DSPLIT, BL>;
  int64_t resident = 0;
  if constexpr (PERSIST) {
    static int per_dev = 0;  // blocks resident on the device for this kernel (per process, device 0 shape)
    if (per_dev == 0) {
      int dev = 0, cus = 0, per_cu = 0;
      hipError_t e = hipGetDevice(&dev);
      if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, SPB * CONV_N, 0);
      if (e != hipSuccess) return e;
      per_dev = (per_cu > 0 ? per_cu : 1) * cus;
    }
    resident = per_dev;
  }
  // detector-split variants run in chunks of the workspace; the others in one launch
  const int64_t step = DSPLIT ? a0.det_ws_items : a0.total - a0.item0;
  if (DSPLIT && (!a0.det_ws || step <= 0)) return hipErrorInvalidValue;
  for (int64_t i0 = a0.item0; i0 < a0.total; i0 += step) {
    WfsLaunch a = a0;
    a.item0 = i0;
    a.total = a0.total - i0 < step ? a0.total : i0 + step;
    const int64_t groups = (a.total - a.item0 + SPB - 1) / SPB;
    const int64_t blocks = PERSIST && groups > resident ? resident : groups;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(SPB * CONV_N), 0, st, a);
    if constexpr (DSPLIT) {
      const int64_t nb = (a.total - a.item0 + 3) / 4;
      switch (a.noise_head) {
        case 2: hipLaunchKernelGGL((det_noise_kernel<DET_N, 2>), dim3((unsigned)nb), dim3(256), 0, st, a); break;
        case 6: hipLaunchKernelGGL((det_noise_kernel<DET_N, 6>), dim3((unsigned)nb), dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((det_noise_kernel<DET_N, 4>), dim3((unsigned)nb), dim3(256), 0, st, a); break;
      }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Launch variants of the 40-point shapes: (row transforms whole or split over lane pairs,
// waves-per-EU target, persistent grid, noise in the fused kernel or after it).  Variants
// from kFirstDetSplit on end the fused kernel at the detector.
constexpr int kTunedVariants = 11;
// Band-limited variants (11: persistent, 5 waves per EU; 12: one-shot, 7 waves per EU; 13: as 12 with noise
// and centroid in the same kernel, inversion head 4), for LGS shapes with FFT_N = CONV_N.
constexpr int kBandLimitedVariants = 3;
template <int NPX, int FFT_N, int CONV_N, bool LGS>
constexpr bool band_limited_ok() {
  return LGS && FFT_N == CONV_N && CONV_N == 4 * NPX;
}
constexpr int kFirstDetSplit = 6;

// Sub-layer kernels: whole or split row transforms, waves-per-EU target 1; split rows with the
// detector split on a persistent grid; then (band-limited shapes) the band-limited path one-shot
// and persistent.
constexpr int kSubVariants = 3;

template <int NPX, int FFT_N, int CONV_N, int DET_N, bool LGS, bool SUB>
static hipError_t launch_one(int variant, const WfsLaunch& a, hipStream_t st) {
  constexpr int SPB = items_per_block(CONV_N);
  constexpr bool TUNED = (CONV_N == 40 && DET_N == 16);
  if constexpr (SUB) {
    switch (variant) {
      case 0: return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 1, false, false, true>(a, st);
      case 1: return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 1, false, true, true>(a, st);
      case 2: return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 4, true, true, true, true>(a, st);
      case 3:
      case 4:
        if constexpr (band_limited_ok<NPX, FFT_N, CONV_N, LGS>()) {
          if (variant == 3) return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 5, false, true, true, true, true>(a, st);
          return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 6, true, true, true, true, true>(a, st);
        }
        return hipErrorInvalidValue;
      default: return hipErrorInvalidValue;
    }
  } else if constexpr (TUNED) {
    switch (variant) {
      case 0: return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 1, false, false>(a, st);
      case 1: return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 4, false, false>(a, st);
      case 2: return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 1, false, true>(a, st);
      case 3: return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 4, false, true>(a, st);
      case 4: return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 1, true, false>(a, st);
      case 5: return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 4, true, false>(a, st);
      case 6: return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 1, false, false, false, true>(a, st);
      case 7: return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 4, true, false, false, true>(a, st);
      case 8: return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 1, false, true, false, true>(a, st);
      case 9: return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 4, true, true, false, true>(a, st);
      case 10: return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 1, true, true, false, true>(a, st);
      case 11:
      case 12:
      case 13:
        if constexpr (band_limited_ok<NPX, FFT_N, CONV_N, LGS>()) {
          if (variant == 11) return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 5, true, true, false, true, true>(a, st);
          if (variant == 12) return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 7, false, true, false, true, true>(a, st);
          return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 7, false, true, false, false, true>(a, st);
        }
        return hipErrorInvalidValue;
      default: return hipErrorInvalidValue;
    }
  } else {
    if (variant != 0) return hipErrorInvalidValue;
    return launch_variant<NPX, FFT_N, CONV_N, DET_N, LGS, SPB, 1, false, false>(a, st);
  }
}

#define SHW_WFS_SHAPES(X)       \
  X(8, 16, 16, 8, false, false) \
  X(8, 16, 16, 8, true, false)  \
  X(8, 16, 16, 16, false, false) \
  X(10, 40, 40, 16, true, false) \
  X(10, 40, 40, 16, false, false) \
  X(10, 20, 40, 16, true, false) \
  X(10, 20, 20, 10, false, false) \
  X(8, 16, 16, 8, true, true)   \
  X(10, 40, 40, 16, true, true)

#define SHW_SHAPE_MATCH(np, fn, cn, dn, lg, sb)                                                   \
  (s.npx == np && s.fft_n == fn && s.conv_n == cn && s.det_n == dn && (s.lgs != 0) == lg && \
   (s.sub != 0) == sb)

bool wfs_shape_supported(const WfsShape& s) {
#define X(np, fn, cn, dn, lg, sb) \
  if (SHW_SHAPE_MATCH(np, fn, cn, dn, lg, sb)) return true;
  SHW_WFS_SHAPES(X)
#undef X
  return false;
}

int wfs_variant_count(const WfsShape& s) {
  if (!wfs_shape_supported(s)) return 0;
  const bool bl = s.lgs && s.fft_n == s.conv_n && s.conv_n == 4 * s.npx;
  if (s.sub) return kSubVariants + (bl ? 2 : 0);
  if (!(s.conv_n == 40 && s.det_n == 16)) return 1;
  return kTunedVariants + (bl ? kBandLimitedVariants : 0);
}

bool wfs_variant_params(const WfsShape& s, int v, int32_t* out) {
  if (v < 0 || v >= wfs_variant_count(s)) return false;
  // {convolution form (0 whole rows, 1 split rows, 2 band-limited), waves-per-EU target, persistent
  // grid, noise in a second kernel, items per block, sodium sub-layers}
  struct Row {
    int8_t form, wpe, persist, dsplit;
  };
  static constexpr Row kTuned[] = {{0, 1, 0, 0}, {0, 4, 0, 0}, {1, 1, 0, 0}, {1, 4, 0, 0}, {0, 1, 1, 0},
                                   {0, 4, 1, 0}, {0, 1, 0, 1}, {0, 4, 1, 1}, {1, 1, 0, 1}, {1, 4, 1, 1},
                                   {1, 1, 1, 1}, {2, 5, 1, 1}, {2, 7, 0, 1}, {2, 7, 0, 0}};
  static constexpr Row kSub[] = {{0, 1, 0, 0}, {1, 1, 0, 0}, {1, 4, 1, 1}, {2, 5, 0, 1}, {2, 6, 1, 1}};
  Row r{0, 1, 0, 0};
  if (s.sub) r = kSub[v];
  else if (s.conv_n == 40 && s.det_n == 16) r = kTuned[v];
  out[0] = r.form;
  out[1] = r.wpe;
  out[2] = r.persist;
  out[3] = r.dsplit;
  out[4] = items_per_block(s.conv_n);
  out[5] = s.sub ? 1 : 0;
  return true;
}

int wfs_default_variant(const WfsShape& s) {
  // measured on the 6-LGS frame, with and without noise and sub-layers: the band-limited kernel
  // where the shape allows it (one-shot, noise in the same kernel: as fast as with the separate
  // noise kernel and 40 instead of 101 MB per frame; persistent with sub-layers), else split
  // rows + detector split + persistent grid
  const bool bl = s.lgs && s.fft_n == s.conv_n && s.conv_n == 4 * s.npx;
  if (s.sub) return bl ? 4 : 2;
  if (!(s.conv_n == 40 && s.det_n == 16)) return 0;
  return bl ? kTunedVariants + 2 : 9;
}

bool wfs_variant_needs_det_ws(const WfsShape& s, int variant) {
  if (s.sub) return variant >= 2;
  return s.conv_n == 40 && s.det_n == 16 && variant >= kFirstDetSplit && variant != kTunedVariants + 2;
}

// det_noise_kernel for 16 x 16 detectors over the items [a.item0, a.total) of a.det_ws (the MFMA
// precision form hands its detector values over this way).
hipError_t launch_det_noise16(const WfsLaunch& a, hipStream_t st) {
  const int64_t nb = (a.total - a.item0 + 3) / 4;
  if (nb <= 0) return hipSuccess;
  switch (a.noise_head) {
    case 2: hipLaunchKernelGGL((det_noise_kernel<16, 2>), dim3((unsigned)nb), dim3(256), 0, st, a); break;
    case 6: hipLaunchKernelGGL((det_noise_kernel<16, 6>), dim3((unsigned)nb), dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((det_noise_kernel<16, 4>), dim3((unsigned)nb), dim3(256), 0, st, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_wfs_fused(const WfsShape& s, int variant, const WfsLaunch& a, hipStream_t st) {
#define X(np, fn, cn, dn, lg, sb) \
  if (SHW_SHAPE_MATCH(np, fn, cn, dn, lg, sb)) return launch_one<np, fn, cn, dn, lg, sb>(variant, a, st);
  SHW_WFS_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

__global__ void counter_add_kernel(uint64_t* c, uint64_t inc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c[0] += inc;
}

hipError_t launch_counter_add(uint64_t* d_counter, uint64_t inc, hipStream_t st) {
  hipLaunchKernelGGL(counter_add_kernel, dim3(1), dim3(64), 0, st, d_counter, inc);
  return hipGetLastError();
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

// One thread per in-band value: band[item][k][j] = khat[item][k][j < npx ? j : conv_n - 2 npx + 1 + j].
__global__ __launch_bounds__(256) void khat_band_kernel(int conv_n, int npx, int64_t total, const float* __restrict__ khat,
                                                        float* __restrict__ band) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int kb = 2 * npx - 1;
  const int64_t item = e / ((int64_t)npx * kb);
  const int rem = (int)(e - item * npx * kb);
  const int k = rem / kb, j = rem - k * kb;
  const int col = j < npx ? j : conv_n - 2 * npx + 1 + j;
  band[e] = khat[(item * (conv_n / 2 + 1) + k) * conv_n + col];
}

hipError_t launch_khat_band(int conv_n, int npx, int64_t n, const float* d_khat, float* d_band, hipStream_t st) {
  if (conv_n != 4 * npx || !d_khat || !d_band) return hipErrorInvalidValue;
  const int64_t total = n * npx * (2 * npx - 1);
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(khat_band_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, conv_n, npx, total,
                     d_khat, d_band);
  return hipGetLastError();
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
