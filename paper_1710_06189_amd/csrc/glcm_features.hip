// Haralick statistics kernel: one workgroup per GLCM (Section I; the five
// statistics and their precision are described in glcm_features.h).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "glcm_features.h"
#include "glcm_internal.h"

namespace glcm {
namespace {

__global__ __launch_bounds__(256) void k_features(const uint32_t* glcm, int N, float* out) {
  __shared__ unsigned long long redu[256];
  __shared__ float redf[256];
  glcm_features_wg(glcm + (size_t)blockIdx.x * (uint32_t)N * (uint32_t)N, (uint32_t)N, out + (size_t)blockIdx.x * 5,
                   redu, redf);
}

// N <= kFeaturesWaveMaxN: one wavefront per GLCM, four per workgroup (the
// batch kernel takes its statistics the same way, so both agree bit for bit).
__global__ __launch_bounds__(256) void k_features_wave(const uint32_t* glcm, int K, int N, float* out) {
  const int k = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (k >= K) return;
  glcm_features_wave(glcm + (size_t)k * (uint32_t)N * (uint32_t)N, (uint32_t)N, out + (size_t)k * 5);
}

}  // namespace

hipError_t launch_features(const uint32_t* glcm, int K, int N, float* out, hipStream_t stream) {
  if (N <= kFeaturesWaveMaxN)
    hipLaunchKernelGGL(k_features_wave, dim3((K + 3) / 4), dim3(256), 0, stream, glcm, K, N, out);
  else
    hipLaunchKernelGGL(k_features, dim3(K), dim3(256), 0, stream, glcm, N, out);
  return hipGetLastError();
}

}  // namespace glcm
