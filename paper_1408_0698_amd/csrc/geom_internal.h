// geom_internal.h - arguments of the LGS geometry kernels (layer projection, uplink tilt) and of
// the PSF extras (encircled energy, resampling), shared by the host library and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shw {

constexpr int kMaxLayers = 16;
constexpr int kProjectChunk = 32;  // targets per projection launch (their parameters travel in the arguments)
constexpr int kMaxRadii = 64;      // encircled-energy radii per call
constexpr int kEeGroups = 200;     // row groups of the encircled-energy pass

// One phase-screen layer: FP32 OPD metres, rows of cols samples pitch apart, sample spacing
// pitch_m metres, altitude alt_m; the point above the telescope axis sits at screen pixel
// coordinates (x0, y0) (pixel centres at integer coordinates).
struct LayerDesc {
  const float* screen;
  int32_t rows, cols;
  int64_t pitch;
  double pitch_m, alt_m, x0, y0;
};

struct LayerSet {
  LayerDesc layer[kMaxLayers];
  int32_t n_layers, pad0;
};

// OPD of target t at pupil pixel (i, j) (centre (j + 1/2 - N/2, i + 1/2 - N/2) dx from the axis):
// sum over layers of the bilinear screen sample at (1 - h/H) r + h theta, H the source altitude
// (0: infinity), plus tilt[t] . r when tilt is set.
struct ProjectLaunch {
  LayerSet L;
  int32_t pupil_n, n_t;
  double dx;
  double theta[kProjectChunk][2];
  double inv_h[kProjectChunk];   // 1 / source altitude, 0 for infinity
  const double* tilt;            // nullable [n_t][2] radians, already offset to the chunk
  float* out;                    // target t at out + t * out_stride
  int64_t out_pitch, out_stride;
};
hipError_t launch_project_layers(const ProjectLaunch& a, hipStream_t st);

// Uplink tilt of LGS k: least-squares tilt of the summed layer OPD over the launch telescope's
// beam, an n_s x n_s grid of samples inside the disc of diameter d, the beam centred at
// launcher (1 - h/H) + h theta at altitude h.
struct UplinkLaunch {
  LayerSet L;
  double lgs[kProjectChunk][5];  // launcher x, y (m), theta x, y (rad), sodium altitude (m)
  int32_t n, n_s;
  double d;
  double* tilt;                  // [n][2] radians, already offset to the chunk
};
hipError_t launch_uplink_tilt(const UplinkLaunch& a, hipStream_t st);

// Encircled energy of n_psf M x M PSFs: radii r_k (pixels, k < n_r) around (M/2, M/2).  Pass 1
// writes, per PSF and row group g, the sums over the group's rows of the energy inside each
// radius (ws [n_psf][kEeGroups][n_r + 1], the last entry the group's total); pass 2 adds the
// groups in order and divides by the total.
struct EeLaunch {
  const float* psf;
  int64_t psf_stride;
  int32_t m, n_psf, n_r, pad0;
  double r2[kMaxRadii];
  double* ws;
  double* ee;          // [n_psf][n_r]
};
hipError_t launch_encircled_energy(const EeLaunch& a, hipStream_t st);

// Allocation-free form: the workspace is a file-scope device array of kEeScratchDoubles doubles
// (4 MiB), one per GPU.  ee_scratch_device() returns its address on `device`, which must be the
// current device; the first call per device looks the address up (hipGetSymbolAddress) and keeps it.
constexpr size_t kEeScratchDoubles = (size_t)1 << 19;
constexpr int kMaxDevices = 64;
hipError_t ee_scratch_device(int device, double** out);

// dst[v][u] += w * bilinear(src at (M/2 + (v - M/2) s, M/2 + (u - M/2) s)), zero outside src.
hipError_t launch_psf_resample(const float* src, int32_t m, double s, float w, float* dst, hipStream_t st);

}  // namespace shw
