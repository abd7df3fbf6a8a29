/*
 * shwfs.h - C ABI of the MI355X Shack-Hartmann wavefront-sensor engine.
 *
 * Computes, for every valid sub-aperture of every sensor of every frame,
 * the measurement of the LGS Shack-Hartmann module described in Sec. 4 of
 * Arcidiacono et al., "End to end numerical simulations of the MAORY
 * multiconjugate adaptive optics system" (SPIE 2014, arXiv:1408.0698):
 * the wavefront is split into sub-apertures, each spot is computed by
 * Fourier transform, the spot is convolved with a Gaussian modelling the
 * extent of the laser projection on the sodium layer, noise is added and
 * the centroid of the final image gives the X and Y slopes that the closed
 * loop multiplies by the control matrix (Sec. 3, closed-loop block).  The
 * second user is the PSF block of Sec. 3: PSF at a chosen wavelength and
 * the Strehl ratio.
 *
 * Conventions shared by every entry point:
 *   - Return value: SHW_OK (0) or a negative SHW_E_* code.  On error
 *     shw_last_error() returns a message (thread-local, valid until the
 *     next call on the same thread).
 *   - Argument validation is done on the host before any HIP call, so a
 *     call that returns SHW_E_INVALID / SHW_E_ABI / SHW_E_UNSUPPORTED has
 *     launched nothing and touched no device memory.
 *   - Pointers named d_* are device pointers owned by the caller; they
 *     must stay valid until the work queued on the stream has completed.
 *     Plans own their internal tables and workspaces.
 *   - Compute calls are asynchronous on the given HIP stream (hipStream_t
 *     passed as void*; NULL = the default stream).  A plan must not be used
 *     from two streams at once.
 *   - Arrays are row-major (C order); strides are in elements.
 */
#ifndef SHWFS_H
#define SHWFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHW_ABI_VERSION 1

enum {
  SHW_OK = 0,
  SHW_E_INVALID = -1,     /* bad argument (null pointer, size, stride, geometry) */
  SHW_E_NOMEM = -2,       /* device allocation failed */
  SHW_E_DEVICE = -3,      /* a HIP call failed; message from shw_last_error() */
  SHW_E_UNSUPPORTED = -4, /* valid geometry for which no kernel is built */
  SHW_E_ABI = -5          /* abi_version does not match SHW_ABI_VERSION */
};

/* shw_wfs_config.flags */
#define SHW_FLAG_NOISE 1u          /* Poisson photon noise + Gaussian read noise */
#define SHW_PRECISION_SHIFT 4      /* bits 4..7 select the transform arithmetic */
#define SHW_PREC_FP32 0u           /* FP32 register/LDS FFTs */
#define SHW_PREC_BF16 1u           /* DFT-matrix GEMMs on MFMA, bf16 operands */
#define SHW_PREC_BF16X3 2u         /* bf16 hi+lo split, three products */
#define SHW_PREC_FP16X3 3u         /* scaled fp16 hi+lo split, three products */

/*
 * Sensor geometry (Sec. 4 LGS module inputs; Sec. 2 pupil sampling).
 *
 * Pupil: pupil_n x pupil_n pixels of pupil_dx_m metres; pixel (r, c) has its
 * centre at ((c + 1/2 - pupil_n/2), (r + 1/2 - pupil_n/2)) pixels from the
 * axis and is lit iff obstruction*pupil_n/2 <= radius <= pupil_n/2.
 * Sub-apertures: n_subap x n_subap squares of npx = pupil_n / n_subap pixels;
 * valid iff the lit fraction is >= min_illum; valid ones are numbered in
 * row-major order.
 * Spot: field A exp(2 pi i OPD / wavelength) of a sub-aperture zero padded
 * to fft_n x fft_n, transform centred half a pixel off the grid so that the
 * spot of a flat wavefront is symmetric about ((fft_n-1)/2, (fft_n-1)/2),
 * intensity |F|^2 / fft_n^2; embedded at the centre of a conv_n grid.
 * LGS (lgs != 0): circular convolution with a normalised elongated
 * Gaussian: long axis from the launcher to the sub-aperture, FWHM
 * sqrt(el^2 + spot_fwhm^2) with el = elong_max * distance / diameter
 * (or the geometric distance * na_fwhm / na_height^2 when elong_max <= 0),
 * short-axis FWHM spot_fwhm; periodised on the conv_n grid.
 * Detector: conv_n -> det_n pixels by area-overlap rebinning.
 * Photometry: photons_per_subap > 0 scales a sub-aperture image to
 * photons_per_subap * (lit fraction) electrons; with SHW_FLAG_NOISE the
 * image becomes Poisson counts + ron_e * N(0,1).  Centroid: image minus
 * threshold_e clipped at zero (threshold 0 when photons_per_subap == 0).
 */
typedef struct shw_wfs_config {
  int32_t abi_version;        /* must equal SHW_ABI_VERSION */
  int32_t pupil_n;            /* pixels across the pupil */
  double pupil_dx_m;          /* metres per pupil pixel, > 0 */
  double obstruction;         /* linear central obstruction, [0, 1) */
  int32_t n_subap;            /* sub-apertures across; divides pupil_n */
  int32_t fft_n;              /* spot transform size, in [npx, 4096] */
  int32_t conv_n;             /* convolution grid, >= fft_n, conv_n - fft_n even */
  int32_t det_n;              /* detector pixels across a sub-aperture, <= conv_n */
  int32_t lgs;                /* 0: NGS (no sodium kernel); 1: LGS */
  uint32_t flags;             /* SHW_FLAG_NOISE | (precision << SHW_PRECISION_SHIFT) */
  double min_illum;           /* valid if lit fraction >= min_illum, (0, 1] */
  double wavelength_m;        /* > 0 */
  double na_height_m;         /* sodium layer height (geometric law only) */
  double na_fwhm_m;           /* sodium layer thickness (geometric law only) */
  double elong_max_arcsec;    /* elongation across the full diameter; <= 0: geometric */
  double spot_fwhm_arcsec;    /* laser spot FWHM, > 0 when lgs */
  double photons_per_subap;   /* >= 0 */
  double ron_e;               /* read noise, electrons rms, >= 0 */
  double threshold_e;         /* centroid threshold, electrons */
} shw_wfs_config;

/* Launch-telescope position of one LGS sensor, pupil coordinates in metres. */
typedef struct shw_lgs_geom {
  double launch_x_m;
  double launch_y_m;
} shw_lgs_geom;

typedef struct shw_wfs_plan shw_wfs_plan;   /* opaque, owned by the library */
typedef struct shw_psf_plan shw_psf_plan;   /* opaque, owned by the library */

/* Message for the last non-OK return on this thread ("" if none). */
const char* shw_last_error(void);

/* Library version: SHW_ABI_VERSION. */
int32_t shw_abi_version(void);

/*
 * Host-only validation of a geometry (no HIP call).  Returns SHW_OK,
 * SHW_E_ABI, SHW_E_INVALID or SHW_E_UNSUPPORTED (no kernel instantiated for
 * this (npx, fft_n, conv_n, det_n, lgs) combination).  geom may be NULL
 * for NGS; for LGS it holds n_wfs entries.
 */
int shw_wfs_config_check(const shw_wfs_config* cfg, int32_t n_wfs, const shw_lgs_geom* geom);

/*
 * Host-only valid-sub-aperture table (Sec. 4: the wavefront is split into
 * sub-apertures).  *n_valid receives the count; valid_idx (nullable, room
 * for n_subap^2 entries) receives row-major indices a*n_subap + b; illum
 * (nullable, same room) the lit fractions.
 */
int shw_wfs_geometry(const shw_wfs_config* cfg, int32_t* n_valid, int32_t* valid_idx, double* illum);

/*
 * Create a plan for n_wfs sensors of one geometry (1 <= n_wfs <= 4096).
 * Allocates device tables on the current HIP device and, for LGS, computes
 * the kernel spectra of every valid sub-aperture on the GPU (FP64, stored
 * FP32, (conv_n/2 + 1) x conv_n reals per sub-aperture: the spectrum of a
 * point-symmetric kernel is real and point-symmetric).  Synchronous.
 * On success *out owns the plan; release it with shw_wfs_plan_destroy.
 */
int shw_wfs_plan_create(const shw_wfs_config* cfg, int32_t n_wfs, const shw_lgs_geom* geom,
                        shw_wfs_plan** out);

/*
 * Sodium sub-layer form of the LGS sensor (Sec. 4: the sodium layer is cut
 * into sub-layers; each gets its own tip-tilt and defocus, its spot is
 * weighted by the sodium profile, the laser extent is a Gaussian
 * convolution, the sub-layer images are piled up before noise and
 * centroid).  Sub-layer j lies at height na_height_m + dh_m[j] with profile
 * weight weight[j] (>= 0; normalised here to unit sum).  Seen from pupil
 * point r, the beam point of sensor w at height h is a point source at
 * (launch_w, h); against the focus at na_height_m = H it adds
 *     -|r - launch_w|^2 / 2 * (1/h - 1/H)   metres of OPD
 * (tip-tilt plus defocus over each sub-aperture, a constant otherwise).
 * The convolution kernel is then the round laser spot (FWHM
 * spot_fwhm_arcsec): the elongation comes from the sub-layers.
 * Requires lgs = 1, FP32 precision, 1 <= n_sub <= 16, a shape with a
 * sub-layer kernel (sub-apertures of 10 pixels, fft_n = conv_n = 40,
 * det_n = 16; or 8 / 16 / 16 / 8), else SHW_E_INVALID / SHW_E_UNSUPPORTED.
 * dh_m and weight are host arrays of n_sub entries, copied.
 */
int shw_wfs_plan_create_sodium(const shw_wfs_config* cfg, int32_t n_wfs, const shw_lgs_geom* geom, int32_t n_sub,
                               const double* dh_m, const double* weight, shw_wfs_plan** out);

/* Plan facts: valid sub-apertures per sensor, device bytes held.  Either pointer may be NULL. */
int shw_wfs_plan_info(const shw_wfs_plan* plan, int32_t* n_valid, size_t* device_bytes);

/*
 * Copy the stored kernel spectra of sensor wfs (LGS plans only) into d_out
 * (device, n_valid * (conv_n/2 + 1) * conv_n floats, layout
 * [subap][row k = 0..conv_n/2][column l], values K^(k,l) / conv_n^2).
 */
int shw_wfs_plan_kernel_spectra(const shw_wfs_plan* plan, int32_t wfs, float* d_out, void* hip_stream);

/*
 * sh_wfs_measure - slopes of n_frames x n_wfs sensors (Sec. 4 LGS SH module).
 *
 * d_opd_m     : OPD in metres, FP32, device.  Element (frame f, sensor w,
 *               row r, column c) at d_opd_m[f*frame_stride + w*wfs_stride +
 *               r*row_pitch + c]; row_pitch >= pupil_n, all strides >= 0.
 * n_frames    : >= 0 (0 is a no-op).
 * seed, frame0: noise key and the frame number of the first frame; the
 *               noise of sub-aperture i of sensor w in frame frame0 + f
 *               is drawn from Philox4x32-10 with key seed: pixels b and
 *               b + h of the det_n^2 pixels (h = ceil(det_n^2 / 2)) share
 *               the block of counter (0, b, w*n_valid + i, frame0 + f)
 *               (Poisson uniforms from words 0 and 1, both Box-Muller
 *               deviates from words 2 and 3); means >= 20 use the
 *               rejection sampler with counters (t >= 1, p, ...).  So a
 *               result does not depend on how frames are batched.
 *               frame0 + n_frames must be <= 2^32.
 * d_slopes    : [n_frames][n_wfs][2][n_valid] FP32, detector pixels from
 *               the sub-aperture centre, X (columns) block then Y block.
 * d_images    : nullable; [n_frames][n_wfs][n_valid][det_n][det_n] FP32
 *               detector images (electrons, before the threshold).
 * d_flags     : nullable; [n_frames][n_wfs][n_valid] uint8, 1 where nothing
 *               was left above the threshold (slopes set to 0).
 * Asynchronous on hip_stream.
 */
int sh_wfs_measure(shw_wfs_plan* plan, const float* d_opd_m, int64_t row_pitch, int64_t wfs_stride,
                   int64_t frame_stride, int32_t n_frames, uint64_t seed, uint64_t frame0,
                   float* d_slopes, float* d_images, uint8_t* d_flags, void* hip_stream);

/*
 * sh_wfs_measure_sodium - sh_wfs_measure for a plan made by
 * shw_wfs_plan_create_sodium, with one wavefront per sub-layer (Sec. 4: the
 * sensor takes the open-loop wavefront minus the DMs for each sodium
 * sub-layer): element (f, w, sub-layer j, r, c) at d_opd_m[f*frame_stride +
 * w*wfs_stride + j*sub_stride + r*row_pitch + c]; sub_stride = 0 gives every
 * sub-layer the same wavefront (what sh_wfs_measure does on such a plan).
 * SHW_E_INVALID for a plan without sub-layers or a negative stride.
 */
int sh_wfs_measure_sodium(shw_wfs_plan* plan, const float* d_opd_m, int64_t row_pitch, int64_t sub_stride,
                          int64_t wfs_stride, int64_t frame_stride, int32_t n_frames, uint64_t seed,
                          uint64_t frame0, float* d_slopes, float* d_images, uint8_t* d_flags, void* hip_stream);

/*
 * One item of a mixed batch: one frame of all sensors of a plan.
 * Fields as in sh_wfs_measure with n_frames = 1.
 */
typedef struct shw_work {
  shw_wfs_plan* plan;
  const float* d_opd_m;
  int64_t row_pitch;
  int64_t wfs_stride;
  uint64_t seed;
  uint64_t frame;
  float* d_slopes;     /* [n_wfs][2][n_valid] */
  float* d_images;     /* nullable, [n_wfs][n_valid][det_n][det_n] */
} shw_work;

/*
 * sh_wfs_measure_batch - n work items of possibly different plans in as few
 * launches as the plan geometries allow (one per distinct kernel shape).
 * Each item's result is identical to sh_wfs_measure on that item alone.
 * Items must not share output buffers.  Asynchronous on hip_stream: each
 * plan's work list is staged in a pinned host ring of 4 slots and uploaded
 * asynchronously, so the call returns without waiting for earlier work on
 * the stream (it waits only when a slot's upload from 4 calls earlier has
 * not run yet).  A plan's batches must all go to one stream.  The first call
 * with more than 256 frames of a plan (or more than any earlier call) grows
 * the plan's list: that call synchronises hip_stream and allocates.
 */
int sh_wfs_measure_batch(const shw_work* items, int32_t n, void* hip_stream);

int shw_wfs_plan_destroy(shw_wfs_plan* plan);

/*
 * Launch variants and autotuning (batching form: every sub-aperture of every
 * sensor of every frame in one launch).  A plan has 1..n compiled launch
 * variants of its fused kernel (register/occupancy target, one-shot or
 * persistent grid, row transforms whole or split over lane pairs, noise and
 * centroid in the fused kernel or in a second kernel over the detector
 * values kept in a plan-owned workspace).  Variants with the same row
 * transform give bitwise identical images, and bitwise identical slopes when
 * the centroid is taken in the same kernel (FP64 sums in the fused kernel,
 * FP32 sums in the second kernel: slopes within 1e-4 pixel of each other);
 * the row-transform families differ by FP32 rounding (about 1e-7 of an
 * image).  Band-limited variants
 * (LGS with fft_n = conv_n = 4 * sub-aperture pixels: 11, 12 and 13, sodium
 * plans 3 and 4) compute the column spectrum of the spot from
 * autocorrelations of the row transforms and filter only the rows inside
 * the spot's band; 13 (16 x 16 detector) takes noise and centroid in the
 * fused kernel with the second kernel's code (inversion head 4: the same
 * images and slopes as 12 at that head) and keeps no detector workspace.
 * New plans start on the fastest measured variant: 13 for band-limited
 * 40-point shapes, 9 for the other 40-point shapes, 4 for band-limited
 * sodium plans, 2 for the other sodium plans, 0 otherwise.
 * shw_wfs_plan_autotune times every variant on the given inputs
 * (reps launches each after two warm-up launches, HIP events on the stream;
 * synchronous), selects the fastest, except that the plan's starting variant
 * above is kept when it is within 2 % of the fastest (launch times vary by a
 * few per cent between runs; for band-limited shapes it is the form with the
 * least HBM traffic), and returns its index in *best and the per-variant
 * milliseconds per launch in ms (nullable, n entries).
 */
int shw_wfs_plan_variant_count(const shw_wfs_plan* plan, int32_t* n);
int shw_wfs_plan_set_variant(shw_wfs_plan* plan, int32_t variant);
int shw_wfs_plan_get_variant(const shw_wfs_plan* plan, int32_t* variant);
int shw_wfs_plan_autotune(shw_wfs_plan* plan, const float* d_opd_m, int64_t row_pitch, int64_t wfs_stride,
                          int64_t frame_stride, int32_t n_frames, float* d_slopes, int32_t reps, void* hip_stream,
                          int32_t* best, float* ms);

/*
 * shw_wfs_plan_variant_params - the parameters that variant `variant` fixes,
 * as 6 values in params: convolution form (0 whole-row transforms, 1 split
 * rows over lane pairs, 2 band-limited), waves-per-EU register target,
 * persistent grid (0/1), noise and centroid in a second kernel (0/1), work
 * items per block, sodium sub-layers (0/1).  SHW_E_UNSUPPORTED for plans
 * without launch variants (FFT 512, MFMA precision forms).
 */
int shw_wfs_plan_variant_params(const shw_wfs_plan* plan, int32_t variant, int32_t* params);

/*
 * Inversion head of the noise kernel (variants with noise in a second
 * kernel): the number of steps (2, 4 or 6; default 4) of the Poisson
 * sequential search that every lane runs in lockstep for its pixels before
 * the pixels still searching are queued and finished one per lane.  It
 * changes which pixels are queued, not their counts; the FP32 centroid sums
 * move by rounding (below 1e-4 detector px).
 * shw_wfs_plan_autotune_noise_head times the three values on the given
 * inputs for the current variant and keeps the fastest (ms: 3 entries,
 * nullable); it synchronises the stream.
 */
int shw_wfs_plan_set_noise_head(shw_wfs_plan* plan, int32_t head);
int shw_wfs_plan_get_noise_head(const shw_wfs_plan* plan, int32_t* head);
int shw_wfs_plan_autotune_noise_head(shw_wfs_plan* plan, const float* d_opd_m, int64_t row_pitch,
                                     int64_t wfs_stride, int64_t frame_stride, int32_t n_frames, float* d_slopes,
                                     int32_t reps, void* hip_stream, int32_t* best, float* ms);

/*
 * sh_wfs_measure with the frame number of the first frame read on the
 * device from *d_frame0 when the kernel runs (so a captured graph can be
 * replayed frame after frame; see shw_counter_add).  *d_frame0 + n_frames
 * must be <= 2^32 (not checked: the value is only known on the device).
 */
int sh_wfs_measure_devframe(shw_wfs_plan* plan, const float* d_opd_m, int64_t row_pitch, int64_t wfs_stride,
                            int64_t frame_stride, int32_t n_frames, uint64_t seed, const uint64_t* d_frame0,
                            float* d_slopes, float* d_images, uint8_t* d_flags, void* hip_stream);

/*
 * sh_wfs_measure_devframe with the first frame number *d_frame0 +
 * frame_offset (read on the device): several loop steps captured into one
 * graph take offsets 0, 1, ..., K-1 and one shw_counter_add(K) after them,
 * so that one replay measures K consecutive frames.  The sum must stay
 * below 2^32 (not checked).
 */
int sh_wfs_measure_devframe_at(shw_wfs_plan* plan, const float* d_opd_m, int64_t row_pitch, int64_t wfs_stride,
                               int64_t frame_stride, int32_t n_frames, uint64_t seed, const uint64_t* d_frame0,
                               uint32_t frame_offset, float* d_slopes, float* d_images, uint8_t* d_flags,
                               void* hip_stream);

/* *d_counter += inc on the device (a one-lane kernel, capturable). */
int shw_counter_add(uint64_t* d_counter, uint64_t inc, void* hip_stream);

/*
 * Loop-step graphs: every library call issued on hip_stream between
 * shw_graph_begin and shw_graph_end is recorded (nothing runs) into a HIP
 * graph, instantiated by shw_graph_end; shw_graph_launch replays it on a
 * stream.  Kernel arguments, including buffer addresses, are fixed at
 * capture.  hip_stream must not be the NULL stream.
 */
typedef struct shw_graph shw_graph;
int shw_graph_begin(void* hip_stream);
int shw_graph_end(void* hip_stream, shw_graph** out);
int shw_graph_launch(shw_graph* graph, void* hip_stream);
int shw_graph_destroy(shw_graph* graph);

/*
 * Science PSF (Sec. 3 PSF block, Sec. 5 integrated PSF and Strehl ratio).
 * P(v,u) = |sum_{y,x} A e^{2 pi i OPD/lambda} e^{-2 pi i ((u - M/2) x + (v - M/2) y)/M}|^2 / (sum A)^2
 * on an M x M grid (fft_m >= pupil_n); the on-axis direction is pixel
 * (M/2, M/2) and the diffraction-limited PSF has the value 1 there.
 */
int shw_psf_plan_create(int32_t abi_version, int32_t pupil_n, double pupil_dx_m, double obstruction,
                        int32_t fft_m, double wavelength_m, shw_psf_plan** out);

/*
 * psf_accumulate - d_psf_acc[v*M + u] += sum over the n_frames frames of P
 * (the caller zeroes the accumulator once), d_strehl[f] = P_f(M/2, M/2)
 * (nullable).  Frame f's OPD (metres, FP32) starts at
 * d_opd_m + f*frame_stride with rows row_pitch apart.  Asynchronous.
 */
int psf_accumulate(shw_psf_plan* plan, const float* d_opd_m, int64_t row_pitch, int64_t frame_stride,
                   int32_t n_frames, float* d_psf_acc, float* d_strehl, void* hip_stream);

/*
 * psf_accumulate over n_stars stars at once (the test-star grid of a science
 * field): star s frame f starts at d_opd_m + s*star_stride + f*frame_stride,
 * its accumulator at d_psf_acc + s*acc_stride (acc_stride >= fft_m^2), its
 * Strehl ratio at d_strehl[s*n_frames + f] (nullable).  The plan's workspace
 * grows (once, up to 4 GiB) to hold every frame of every star of the call;
 * growing synchronises the device.  Asynchronous otherwise.
 */
int psf_accumulate_stars(shw_psf_plan* plan, const float* d_opd_m, int64_t row_pitch, int64_t frame_stride,
                         int64_t star_stride, int32_t n_frames, int32_t n_stars, float* d_psf_acc,
                         int64_t acc_stride, float* d_strehl, void* hip_stream);

int shw_psf_plan_destroy(shw_psf_plan* plan);

/*
 * psf_encircled_energy - encircled energy of n_psf PSFs of the plan's size M
 * (Sec. 3 PSF block: encircled energy in the chosen radius).  PSF s is the
 * M x M FP32 array at d_psf + s*psf_stride (psf_stride >= M^2 when n_psf > 1),
 * e.g. an accumulator of psf_accumulate.  For each radius r_px[k] (pixels,
 * host array of 1 <= n_r <= 64 values >= 0):
 *   d_ee[s*n_r + k] = sum of P over pixels (v, u) with (u - M/2)^2 + (v - M/2)^2 <= r^2
 *                     divided by the sum of P over the whole array
 * (FP64 sums in a fixed order: the same inputs give the same result).  M <=
 * 4096 (SHW_E_UNSUPPORTED otherwise).  The plan keeps a workspace of n_psf *
 * 200 * (n_r + 1) doubles; growing it synchronises the device.  Asynchronous
 * otherwise; calls on one plan must not overlap.
 */
int psf_encircled_energy(shw_psf_plan* plan, const float* d_psf, int32_t n_psf, int64_t psf_stride, int32_t n_r,
                         const double* r_px, double* d_ee, void* hip_stream);

/*
 * psf_encircled_energy_noalloc - psf_encircled_energy for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, validation, result and
 * bits as psf_encircled_energy, but the workspace is a static device array of
 * 4 MiB (524,288 doubles) that the library holds on each GPU it runs on until
 * the process ends, instead of the plan's workspace.  The call allocates and
 * frees nothing and does not synchronise.  Limit: n_psf * 200 * (n_r + 1) <=
 * 524,288 (e.g. 39 PSFs at 64 radii, 124 PSFs at 20 radii); larger requests
 * return SHW_E_INVALID before any device work.  The first call on a device
 * looks up the array's address there (that device must be current, as for
 * every call on the plan).  All calls on one GPU share its array: calls that
 * overlap on one GPU (two streams, or two threads) race and give undefined
 * results; calls ordered on one stream do not.  Nothing carries over between
 * calls: each call writes every workspace entry it reads.
 */
int psf_encircled_energy_noalloc(const shw_psf_plan* plan, const float* d_psf, int32_t n_psf, int64_t psf_stride,
                                 int32_t n_r, const double* r_px, double* d_ee, void* hip_stream);

/*
 * psf_resample_accumulate - put a PSF computed at wavelength lambda_i on the
 * angular grid of a reference wavelength lambda_ref (both M x M, on-axis at
 * pixel (M/2, M/2)) and add it with a weight (Sec. 3 PSF block: PSFs at
 * several wavelengths combined by the colour of the object):
 *   d_dst[v*M + u] += weight * S(M/2 + (v - M/2) scale, M/2 + (u - M/2) scale),
 * scale = lambda_ref / lambda_i, S the bilinear interpolation of d_src
 * (sample (y, x) at row y, column x); points outside [0, M-1]^2 add nothing.
 * The PSF values are intensities relative to the diffraction-limited peak,
 * so the on-axis value of the sum is the weighted sum of the Strehl ratios.
 * d_src and d_dst must not overlap (SHW_E_INVALID).  Asynchronous.
 */
int psf_resample_accumulate(int32_t fft_m, const float* d_src, double scale, float weight, float* d_dst,
                            void* hip_stream);


/*
 * Open-loop wavefronts of finite-altitude sources (Sec. 4 open-loop
 * generation: shifted phase screens piled up per direction; an LGS sodium
 * sub-layer is a source at its own altitude, whose pupil projection on each
 * layer changes with the layer's altitude - the cone effect).
 *
 * Layers (1 <= n_layers <= 16): layer l is an FP32 OPD screen (metres) on the
 * device at d_screen[l], screen_rows[l] x screen_cols[l] samples (both >= 2),
 * rows screen_pitch[l] >= screen_cols[l] floats apart; layer_params[4l ..
 * 4l+3] = (sample spacing m > 0, altitude m >= 0, x0, y0): the point above the
 * telescope axis is at screen coordinates (x0, y0) in samples (sample (r, c)
 * at coordinates (x, y) = (c, r)).  Host arrays.
 *
 * shw_project_layers - for target t (host target_params[3t .. 3t+2] =
 * direction theta_x, theta_y in radians, source altitude H in metres, 0 for
 * a source at infinity) and pupil pixel (i, j) of a pupil_n x pupil_n grid of
 * spacing dx_m (centre r = ((j + 1/2 - pupil_n/2) dx, (i + 1/2 - pupil_n/2) dx)):
 *   d_out[t*out_stride + i*out_pitch + j] =
 *       sum_l S_l(x0_l + p_x / spacing_l, y0_l + p_y / spacing_l) + tilt_t . r,
 *   p = (1 - h_l/H) r + h_l theta   (p = r + h_l theta for H = 0),
 * S_l the bilinear interpolation of layer l, tilt_t = d_tilt[2t .. 2t+1]
 * (radians, device, nullable: no tilt) - e.g. the uplink tilts below.  Every
 * footprint must stay inside its screen and every finite-altitude target
 * above every layer (SHW_E_INVALID otherwise); out_pitch >= pupil_n, and
 * out_stride >= out_pitch * pupil_n when n_targets > 1.  FP64 positions and
 * sums, FP32 output.  Asynchronous.
 */
int shw_project_layers(int32_t n_layers, const float* const* d_screen, const int32_t* screen_rows,
                       const int32_t* screen_cols, const int64_t* screen_pitch, const double* layer_params,
                       int32_t pupil_n, double dx_m, int32_t n_targets, const double* target_params,
                       const double* d_tilt, float* d_out, int64_t out_pitch, int64_t out_stride, void* hip_stream);

/*
 * shw_uplink_tilt - tip-tilt picked up by each laser beam on its way up to
 * the sodium layer (Sec. 4: the projection of the beam on the sodium layer is
 * shifted by the tip-tilt integrated over the upward path).  LGS k (host
 * lgs_params[5k .. 5k+4] = launcher position x, y in the pupil plane (m),
 * direction theta_x, theta_y (rad), sodium altitude H > every layer's (m)):
 * the beam, of diameter llt_diameter_m, is centred at launcher (1 - h/H) +
 * h theta at altitude h.  It is sampled on an n_samples x n_samples grid
 * (2..256) over the square of side llt_diameter_m, keeping the points inside
 * the disc; the OPD at a sample is the sum over layers of the bilinear screen
 * values (as for shw_project_layers), and the tilt is its least-squares
 * slope over the samples (the sample set is symmetric, so it is
 * sum(s_x OPD) / sum(s_x^2) and likewise in y):
 *   d_tilt[2k], d_tilt[2k+1] = tilt in x and y, radians (device, FP64).
 * Every beam footprint must stay inside its screen (SHW_E_INVALID).
 * Asynchronous.  Adding the tilt to the sensor's wavefront (d_tilt of
 * shw_project_layers) moves the spots of every sub-aperture by that angle.
 */
int shw_uplink_tilt(int32_t n_layers, const float* const* d_screen, const int32_t* screen_rows,
                    const int32_t* screen_cols, const int64_t* screen_pitch, const double* layer_params,
                    int32_t n_lgs, const double* lgs_params, double llt_diameter_m, int32_t n_samples,
                    double* d_tilt, void* hip_stream);

/*
 * Deformable mirrors and residual OPD (Sec. 3 closed-loop block: the residual
 * phase is the open-loop wavefront minus the DM; Sec. 2: ~5000 / ~1400 /
 * ~1800 modes on the ground and two post-focal DMs with 1 m pitch; Sec. 3
 * influence-function block: analytic influence functions when none are
 * supplied).
 *
 * A DM conjugated at altitude alt_m has actuators on a square grid of pitch
 * pitch_px pupil pixels, centred on the axis, kept where the actuator lies
 * within the metapupil radius pupil_n/2 + alt_m * field_radius / dx (pixels).
 * Its surface is a size x size grid, size = 2 * ceil(metapupil radius), with
 * pixel centres at (j + 1/2 - size/2) pixels from the axis.  Influence
 * function: exp(-r^2 / (2 sigma^2)) with exp(-pitch^2 / (2 sigma^2)) =
 * coupling, on the patch x patch pixels nearest to the actuator.
 * Actuators are numbered row-major (y, then x).
 */
typedef struct shw_dm_plan shw_dm_plan;

int shw_dm_plan_create(int32_t abi_version, int32_t pupil_n, double pupil_dx_m, double alt_m, int32_t pitch_px,
                       double field_radius_arcsec, double coupling, int32_t patch, shw_dm_plan** out);

/* Actuator count, surface side, and (nullable) host copy of the actuator
 * positions [n_act][2] = (x, y) in pixels from the DM centre. */
int shw_dm_plan_info(const shw_dm_plan* plan, int32_t* n_act, int32_t* size, double* act_xy);

/* Host-only: the same facts without creating a plan (no HIP call).  act_xy
 * (nullable) needs room for the count returned by a first call with NULL. */
int shw_dm_geometry(int32_t pupil_n, double pupil_dx_m, double alt_m, int32_t pitch_px, double field_radius_arcsec,
                    int32_t* n_act, int32_t* size, double* act_xy);

/*
 * d_surface[size][size] (FP32, device, row pitch = size) = sum_k
 * d_coefs[k] * IF_k.  d_coefs: [n_act] FP32 OPD metres, device.  Asynchronous.
 */
int shw_dm_surface(shw_dm_plan* plan, const float* d_coefs, float* d_surface, void* hip_stream);

int shw_dm_plan_destroy(shw_dm_plan* plan);

/*
 * Push-pull calibration (Sec. 3 interaction-matrix block: the slopes the WFS
 * registers for each pushed mode; Sec. 5: a modal push-pull calibration of
 * one LGS sensor over 5000 modes).  The modes here are the influence
 * functions of the DM's actuators.
 *
 * shw_dm_influence_opd: d_out[k][y][x] (row pitch out_pitch, frame stride
 * out_stride) = d_amp[k] * IF of actuator d_act[k] at surface pixel
 * (row0 + y, col0 + x), for k < n, y, x < pupil_n; 0 outside the actuator's
 * patch.  d_act (int32) and d_amp (FP32) are device arrays of n entries
 * (n <= 65535); an index outside [0, n_act) yields a frame of NaN.  The
 * window must lie inside the size x size surface (SHW_E_INVALID otherwise).
 *
 * shw_push_pull: d_im[s * ld_im + m] = (d_slopes[2m][s] - d_slopes[2m+1][s]) * scale
 * for m < n_modes, s < n_slopes: frames 2m / 2m+1 are the push / pull of mode
 * m, scale = 1 / (2 amplitude); d_im is the interaction matrix, one row per slope
 * (ld_im >= n_modes, SHW_E_INVALID otherwise).  Both calls are asynchronous on
 * hip_stream; the caller owns every buffer.
 */
int shw_dm_influence_opd(const shw_dm_plan* plan, const int32_t* d_act, const float* d_amp, int32_t n, int32_t row0,
                         int32_t col0, int32_t pupil_n, float* d_out, int64_t out_pitch, int64_t out_stride,
                         void* hip_stream);
int shw_push_pull(const float* d_slopes, int32_t n_modes, int32_t n_slopes, float scale, float* d_im, int64_t ld_im,
                  void* hip_stream);

/*
 * Residual OPD of n_out pupils: out_k[y][x] = screen[sr_k + y][sc_k + x]
 * - sum_d surf_d[r_kd + y][c_kd + x] for y, x < pupil_n, where (sr_k, sc_k)
 * and (r_kd, c_kd) are window origins (rows, columns) given per output k
 * in the host arrays scr_origin[n_out][2] and dm_origin[n_out][n_dm][2].
 * The screen is screen_rows x screen_cols with row pitch screen_pitch;
 * surface d is surf_size[d] square with row pitch surf_size[d]; d_surf is a
 * host array of n_dm (<= 4) device pointers.  Output k starts at d_out +
 * k * out_stride with rows out_pitch apart.  Every window must lie inside
 * its array (checked on the host).  Asynchronous.
 */
int shw_residual_opd(const float* d_screen, int32_t screen_rows, int32_t screen_cols, int64_t screen_pitch,
                     int32_t n_dm, const float* const* d_surf, const int32_t* surf_size, int32_t pupil_n,
                     int32_t n_out, const int32_t* scr_origin, const int32_t* dm_origin, float* d_out,
                     int64_t out_pitch, int64_t out_stride, void* hip_stream);

/*
 * Closed-loop reconstructor and pure integrator (Sec. 3, closed-loop block:
 * the X and Y slope vectors of every sensor are multiplied by the control
 * matrix, which gives modal increments that a pure integrator accumulates
 * into the commands that shape the DMs).
 *
 * shw_recon_plan_create: a plan for an n_modes x n_slopes control matrix
 * (1 <= n_modes <= 2^22, n_slopes >= 1); owns a workspace of
 * ceil(n_slopes / 4096) * n_modes floats on the current device.
 *
 * shw_recon_step: delta[m] = sum_s d_cm[m * ld_cm + s] * d_slopes[s], then
 * d_coefs[m] += gain * delta[m], for m < n_modes; d_delta (nullable)
 * receives delta.  d_cm: FP32 device, 16-byte aligned, ld_cm >= n_slopes
 * and a multiple of 4 (SHW_E_INVALID otherwise).  FP32 products with FP32
 * sums over chunks of 4096 slopes, the chunk sums added in a fixed order:
 * the result does not depend on scheduling.  Asynchronous; the plan's
 * workspace makes concurrent steps of one plan race.
 */
typedef struct shw_recon_plan shw_recon_plan;
int shw_recon_plan_create(int32_t n_modes, int32_t n_slopes, shw_recon_plan** out);
int shw_recon_step(shw_recon_plan* plan, const float* d_cm, int64_t ld_cm, const float* d_slopes, float gain,
                   float* d_coefs, float* d_delta, void* hip_stream);
int shw_recon_plan_destroy(shw_recon_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* SHWFS_H */
