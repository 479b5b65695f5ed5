// Interface between the host runtime and the post-processing kernels
// (symmetric / normalised / direction-averaged GLCMs, Haralick's statistics).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "glcm_internal.h"

namespace glcm {

// Arguments of the post-processing kernels over K matrices of N x N uint32
// counts (symmetric, normalised, direction-averaged GLCMs and the thirteen
// statistics).  floor(r / N) = (r + mulhi(r, nmagic)) >> nshift for r < 2^32.
struct StatsArgs {
  const uint32_t* in;  // [K][N][N]
  uint32_t* out_u;     // symmetric: [K][N][N] (may equal in)
  float* out_f;        // normalised [K][N][N], averaged [K/m][N][N], statistics [K][13]
  int K, N, m;         // m: matrices per averaged group
  uint32_t nmagic, nshift;
};
constexpr int kHaralickStats = 13;
constexpr int kHaralickMaxN = 1024;  // the marginal arrays (7 N doubles) fit the LDS
constexpr int kAverageMaxGroup = 64;

hipError_t launch_symmetrize(const StatsArgs& a, hipStream_t stream);
hipError_t launch_normalize(const StatsArgs& a, hipStream_t stream);
hipError_t launch_average(const StatsArgs& a, hipStream_t stream);
hipError_t launch_haralick(const StatsArgs& a, hipStream_t stream);
// out_f[k] = maximal correlation coefficient of matrix k (N <= kMccMaxLevels)
hipError_t launch_haralick_mcc(const StatsArgs& a, hipStream_t stream);
constexpr int kMccMaxLevels = 64;

}  // namespace glcm
