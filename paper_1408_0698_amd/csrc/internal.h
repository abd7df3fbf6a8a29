// internal.h - structures shared by the host library and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shw {

// One frame of a work list: its own buffers and noise key (device array of these).
struct FrameWork {
  const float* opd;
  int64_t row_pitch, wfs_stride;
  float* slopes;   // [n_wfs][2][n_valid]
  float* images;   // nullable [n_wfs][n_valid][det][det]
  uint64_t seed, frame;
};

// Arguments of one fused Shack-Hartmann launch (all work items share a plan geometry).
struct WfsLaunch {
  const float* opd;          // OPD metres
  int64_t row_pitch, wfs_stride, frame_stride;
  const int32_t* valid_idx;  // [n_valid] row-major sub-aperture index
  const float* khat;         // [n_wfs * n_valid][conv_n/2 + 1][conv_n] (LGS) or null
  // band-limited shapes (conv_n = fft_n = 4 npx): the in-band part of K^ that those variants read,
  // [n_wfs * n_valid][npx][2 npx - 1], row k < npx holding columns 0 .. npx-1 then
  // conv_n - npx + 1 .. conv_n - 1 (the frequencies 0 .. npx-1 and -(npx-1) .. -1); else null
  const float* khat_band;
  float* slopes;             // [items / n_valid][2][n_valid]
  float* images;             // nullable [items][det_n][det_n]
  uint8_t* flags;            // nullable [items]
  int64_t total;             // n_frames * n_wfs * n_valid
  int32_t n_valid, n_wfs, n_subap, pad0;
  // division by n_wfs * n_valid, n_valid and n_subap for dividends below 2^31 (host-filled by
  // div_magic): q = (umulhi(n, m) + n) >> s
  uint32_t dm_frame_m, dm_frame_s, dm_valid_m, dm_valid_s, dm_subap_m, dm_subap_s;
  double inv_lambda;         // 1 / wavelength (1/m)
  float r2_outer, r2_inner;  // pupil annulus in squared pixel units
  float half_n;              // pupil_n / 2
  float ph_scale;            // photons / npx^2, 0 = no photometry
  float ron, thr;
  int32_t noise;
  uint32_t key0, key1, frame0;
  const uint64_t* frame0_dev;  // nullable: frame number of the first frame (+ frame0), read on the device
  const FrameWork* list;       // nullable: frame f takes buffers, strides and key from list[f]
  // sodium sub-layers (kernels built with sub-layers only): sub-layer j adds c_j |r - L_w|^2 / 2
  // waves to the phase (r the pixel centre, L_w the launcher, both in pupil pixels from the axis)
  // and weighs its spot by weight_j
  int32_t n_sub;
  int32_t noise_head;          // lockstep inversion steps of det_noise_kernel (2, 4 or 6)
  int64_t sub_stride;          // OPD elements between the sub-layer wavefronts of a sensor (0: shared)
  const double* sub_coef;      // [n_sub][2] = (c_j waves / pixel^2, weight_j)
  const double* launch_px;     // [n_wfs][2] launcher (x, y) in pupil pixels from the axis
  // detector split: variants that end the fused kernel at the detector values write them to
  // det_ws[(item - item0) * det_n^2 + pixel] and run noise and centroid in a second kernel,
  // over chunks of at most det_ws_items items starting at item0
  float* det_ws;
  int64_t det_ws_items;
  int64_t item0;
};

// Multiplier m and shift s for unsigned division by an invariant d (1 <= d < 2^31) of dividends
// n < 2^31: with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1, floor(n / d) =
// (umulhi(n, m) + n) >> l (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, Theorem 4.2; the sum stays below 2^32 because n < 2^31).
inline void div_magic(uint32_t d, uint32_t* m, uint32_t* s) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  *m = (uint32_t)((((1ull << l) - d) << 32) / d + 1);
  *s = l;
}

// Shape of a compiled fused kernel.
struct WfsShape {
  int npx, fft_n, conv_n, det_n, lgs;
  int sub;  // 1: sodium sub-layer kernels (LGS shapes only)
};

// Returns true if a kernel for this shape is compiled in.
bool wfs_shape_supported(const WfsShape& s);

// Number of compiled launch variants of a shape (0 if unsupported).
int wfs_variant_count(const WfsShape& s);

// Variant a new plan starts with (the autotuner may pick another).
int wfs_default_variant(const WfsShape& s);
// Parameters of variant v: {convolution form (0 whole rows, 1 split rows, 2 band-limited),
// waves-per-EU target, persistent grid, noise in det_noise_kernel, items per block, sub-layers};
// false if v is not a variant of the shape.
bool wfs_variant_params(const WfsShape& s, int v, int32_t* out);

// True if the variant ends the fused kernel at the detector (needs a.det_ws).
bool wfs_variant_needs_det_ws(const WfsShape& s, int variant);

// Launch the fused kernel for a.total work items. Returns the HIP error.
hipError_t launch_wfs_fused(const WfsShape& s, int variant, const WfsLaunch& a, hipStream_t st);

// *d_counter += inc (one lane).
hipError_t launch_counter_add(uint64_t* d_counter, uint64_t inc, hipStream_t st);

// Kernel spectra: params [n][3] = (sigma_par, sigma_perp, psi) in conv-grid
// pixels / radians (device, FP64); out [n][conv_n/2+1][conv_n] FP32, scaled by 1/conv_n^2.
hipError_t launch_lgs_spectra(int conv_n, const double* d_params, int64_t n, float* d_out, hipStream_t st);

// In-band copy of the kernel spectra for the band-limited variants (layout of WfsLaunch::khat_band)
// from khat [n][conv_n/2+1][conv_n]; conv_n = 4 npx.
hipError_t launch_khat_band(int conv_n, int npx, int64_t n, const float* d_khat, float* d_band, hipStream_t st);

}  // namespace shw
