// Host entry points of the post-processing kernels (glcm_stats.hip): argument
// checks, then one asynchronous launch on the caller's stream.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "glcm.h"
#include "glcm_host.h"
#include "glcm_internal.h"
#include "glcm_stats.h"

namespace {

constexpr int kMaxMatrices = 1 << 20;

// Both buffers device memory on the current device.
int check_device_pair(const void* in, const void* out) {
  if (!in || !out) return GLCM_EINVAL;
  int din = -1, dout = -1, cur = 0;
  if (glcm::memory_kind(in, &din) != 2 || glcm::memory_kind(out, &dout) != 2) return GLCM_EINVAL;
  const hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return glcm::hip_error_status(e);
  return (din == cur && dout == cur) ? GLCM_OK : GLCM_EINVAL;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + nb && b0 < a0 + na;
}

glcm::StatsArgs stats_args(const uint32_t* in, int K, int N) {
  glcm::StatsArgs a{};
  a.in = in;
  a.K = K;
  a.N = N;
  a.m = 1;
  // floor(r / N) = (r + mulhi(r, magic)) >> shift with shift = ceil(log2 N),
  // magic = ceil(2^(32 + shift) / N) - 2^32 (exact for r < 2^32)
  uint32_t s = 0;
  while ((1ull << s) < (uint64_t)N) ++s;
  const uint64_t m = ((1ull << (32 + s)) + (uint64_t)N - 1u) / (uint64_t)N;
  a.nmagic = (uint32_t)(m - (1ull << 32));
  a.nshift = s;
  return a;
}

int launched(hipError_t e) { return e == hipSuccess ? GLCM_OK : glcm::hip_error_status(e); }

}  // namespace

extern "C" {

GLCM_API int glcm_symmetrize(const uint32_t* glcm_u32, int K, int N, uint32_t* out, void* stream) {
  if (K < 1 || K > kMaxMatrices || N < 1 || N > GLCM_MAX_LEVELS) return GLCM_EINVAL;
  const int rc = check_device_pair(glcm_u32, out);
  if (rc != GLCM_OK) return rc;
  const size_t bytes = (size_t)K * N * N * 4u;
  if (out != glcm_u32 && overlap(glcm_u32, bytes, out, bytes)) return GLCM_EINVAL;
  glcm::StatsArgs a = stats_args(glcm_u32, K, N);
  a.out_u = out;
  return launched(glcm::launch_symmetrize(a, (hipStream_t)stream));
}

GLCM_API int glcm_normalize(const uint32_t* glcm_u32, int K, int N, float* out, void* stream) {
  if (K < 1 || K > kMaxMatrices || N < 1 || N > GLCM_MAX_LEVELS) return GLCM_EINVAL;
  const int rc = check_device_pair(glcm_u32, out);
  if (rc != GLCM_OK) return rc;
  const size_t bytes = (size_t)K * N * N * 4u;
  if (overlap(glcm_u32, bytes, out, bytes)) return GLCM_EINVAL;
  glcm::StatsArgs a = stats_args(glcm_u32, K, N);
  a.out_f = out;
  return launched(glcm::launch_normalize(a, (hipStream_t)stream));
}

GLCM_API int glcm_average(const uint32_t* glcm_u32, int K, int N, int m, float* out, void* stream) {
  if (K < 1 || K > kMaxMatrices || N < 1 || N > GLCM_MAX_LEVELS) return GLCM_EINVAL;
  if (m < 1 || m > glcm::kAverageMaxGroup || K % m) return GLCM_EINVAL;
  const int rc = check_device_pair(glcm_u32, out);
  if (rc != GLCM_OK) return rc;
  if (overlap(glcm_u32, (size_t)K * N * N * 4u, out, (size_t)(K / m) * N * N * 4u)) return GLCM_EINVAL;
  glcm::StatsArgs a = stats_args(glcm_u32, K, N);
  a.out_f = out;
  a.m = m;
  return launched(glcm::launch_average(a, (hipStream_t)stream));
}

GLCM_API int glcm_haralick(const uint32_t* glcm_u32, int K, int N, float* out, void* stream) {
  if (K < 1 || K > kMaxMatrices || N < 1 || N > GLCM_MAX_LEVELS) return GLCM_EINVAL;
  const int rc = check_device_pair(glcm_u32, out);
  if (rc != GLCM_OK) return rc;
  if (overlap(glcm_u32, (size_t)K * N * N * 4u, out, (size_t)K * glcm::kHaralickStats * 4u)) return GLCM_EINVAL;
  if (N > glcm::kHaralickMaxN) return GLCM_EUNSUPPORTED;
  glcm::StatsArgs a = stats_args(glcm_u32, K, N);
  a.out_f = out;
  return launched(glcm::launch_haralick(a, (hipStream_t)stream));
}

GLCM_API int glcm_haralick_mcc(const uint32_t* glcm_u32, int K, int N, float* out, void* stream) {
  if (K < 1 || K > kMaxMatrices || N < 1 || N > GLCM_MAX_LEVELS) return GLCM_EINVAL;
  const int rc = check_device_pair(glcm_u32, out);
  if (rc != GLCM_OK) return rc;
  if (overlap(glcm_u32, (size_t)K * N * N * 4u, out, (size_t)K * 4u)) return GLCM_EINVAL;
  if (N > glcm::kMccMaxLevels) return GLCM_EUNSUPPORTED;
  glcm::StatsArgs a = stats_args(glcm_u32, K, N);
  a.out_f = out;
  return launched(glcm::launch_haralick_mcc(a, (hipStream_t)stream));
}

}  // extern "C"
