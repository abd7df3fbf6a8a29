// recon_internal.h - closed-loop reconstructor kernels (control-matrix product and integrator).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shw {

constexpr int kReconRows = 64;     // control-matrix rows per block (16 per wave)
constexpr int kReconCols = 4096;   // slope columns per block (staged in LDS)

// Number of column chunks of a product with n_slopes columns.
inline int recon_chunks(int64_t n_slopes) { return (int)((n_slopes + kReconCols - 1) / kReconCols); }

// partial[chunk][m] = sum over the chunk's columns s of cm[m * ld + s] * slopes[s].
hipError_t launch_recon_partial(const float* cm, int64_t ld, int32_t n_modes, int32_t n_slopes, const float* slopes,
                                float* partial, hipStream_t st);

// delta = sum_chunk partial[chunk][m] in chunk order; coefs[m] += gain * delta; delta_out[m] = delta if set.
hipError_t launch_recon_integrate(const float* partial, int32_t n_chunks, int32_t n_modes, float gain, float* coefs,
                                  float* delta_out, hipStream_t st);

}  // namespace shw
