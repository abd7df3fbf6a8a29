// valu_issue_probe.hip - calibration kernels for the VALU issue model of the roofline (measurement
// infrastructure, built into its own library; nothing on the measurement path uses it).
//
// Each kernel runs `iters` iterations of 16 instructions of one kind per lane (8 independent
// chains, unrolled twice), so a launch of B blocks of 256 lanes issues B * 4 * iters * 16 wave
// instructions of that kind; with B = 2048 every SIMD of a 256-CU GPU holds 8 wavefronts.  The host
// times the launch; SQ_ACTIVE_INST_VALU2 (rocprofv3) counts how many of them were dual-issued.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

enum Kind { kFmaF32 = 0, kAddF32 = 1, kMovDpp = 2, kSinF32 = 3, kFmaF64 = 4, kMad64 = 5, kKinds = 6 };

template <int K>
__global__ __launch_bounds__(256) void probe_kernel(float* __restrict__ out, int iters) {
  const int lane = threadIdx.x & 63;
  float r = 0.0f;
  if constexpr (K == kFmaF64) {
    double x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = lane * 1e-3 + c;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int c = 0; c < 8; ++c) x[c] = fma(x[c], 0.999, 1e-4);
#pragma unroll
    for (int c = 0; c < 8; ++c) r += (float)x[c];
  } else if constexpr (K == kMad64) {
    // the Philox round's 32 x 32 -> 64-bit product; the xor keeps each chain dependent
    uint32_t x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = (uint32_t)(lane + 977 * c + 1);
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const uint64_t p = (uint64_t)x[c] * 0xD2511F53u;
          x[c] = (uint32_t)(p >> 32) ^ (uint32_t)p;
        }
#pragma unroll
    for (int c = 0; c < 8; ++c) r += (float)x[c];
  } else {
    float x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = lane * 1e-3f + c;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          if constexpr (K == kFmaF32) x[c] = fmaf(x[c], 0.999f, 1e-4f);
          if constexpr (K == kAddF32) x[c] = x[c] + 1e-4f;
          if constexpr (K == kMovDpp)
            x[c] = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x[c]), 0xB1, 0xF, 0xF, true));
          if constexpr (K == kSinF32) x[c] = __builtin_amdgcn_sinf(x[c]);
        }
#pragma unroll
    for (int c = 0; c < 8; ++c) r += x[c];
  }
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = r;
}

}  // namespace

// Launches probe `kind` (0 FP32 FMA, 1 FP32 add, 2 DPP move, 3 sine, 4 FP64 FMA, 5 32 x 32 -> 64-bit
// integer multiply-add with an xor) over `blocks` blocks of 256 lanes; d_out holds blocks * 256
// floats.  Returns 0, or -1 for an unknown kind or a bad size, or the HIP error code of the launch.
extern "C" int shw_probe_valu(int kind, int blocks, int iters, float* d_out, void* stream) {
  if (blocks < 1 || iters < 1 || !d_out) return -1;
  hipStream_t st = (hipStream_t)stream;
  switch (kind) {
    case kFmaF32: hipLaunchKernelGGL(probe_kernel<kFmaF32>, dim3(blocks), dim3(256), 0, st, d_out, iters); break;
    case kAddF32: hipLaunchKernelGGL(probe_kernel<kAddF32>, dim3(blocks), dim3(256), 0, st, d_out, iters); break;
    case kMovDpp: hipLaunchKernelGGL(probe_kernel<kMovDpp>, dim3(blocks), dim3(256), 0, st, d_out, iters); break;
    case kSinF32: hipLaunchKernelGGL(probe_kernel<kSinF32>, dim3(blocks), dim3(256), 0, st, d_out, iters); break;
    case kFmaF64: hipLaunchKernelGGL(probe_kernel<kFmaF64>, dim3(blocks), dim3(256), 0, st, d_out, iters); break;
    case kMad64: hipLaunchKernelGGL(probe_kernel<kMad64>, dim3(blocks), dim3(256), 0, st, d_out, iters); break;
    default: return -1;
  }
  return (int)hipGetLastError();
}

extern "C" int shw_probe_valu_kinds(void) { return kKinds; }
