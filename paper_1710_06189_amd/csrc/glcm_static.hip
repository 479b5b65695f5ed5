// glcm_compute_static: glcm_compute for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc).  Its only device memory beyond the caller's input and output is
// the per-XCD accumulation slices of the merge, which live in `scratch`, a
// file-scope device array of fixed size that every GPU the library runs on
// holds until the process ends.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "glcm.h"
#include "glcm_host.h"
#include "glcm_internal.h"

namespace {

// kXcdSlots slices of up to GLCM_STATIC_MAX_WORDS counts each (16 MiB).
constexpr size_t kScratchWords = (size_t)glcm::kXcdSlots * GLCM_STATIC_MAX_WORDS;
static_assert(kScratchWords * 4u == (16u << 20), "16 MiB of slices");

__device__ __align__(256) uint32_t scratch[kScratchWords];

// In host code `scratch` names a host-side stand-in, not the device array:
// each device's own copy is found once, with that device current, and only
// that address is handed to kernels.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint32_t* g_ptr[kMaxDevices] = {};

int scratch_on(int device, uint32_t** ptr) {
  if (device < 0 || device >= kMaxDevices) return GLCM_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return e != hipSuccess ? glcm::hip_error_status(e) : GLCM_EHIP;
    g_ptr[device] = (uint32_t*)p;
  }
  *ptr = g_ptr[device];
  return GLCM_OK;
}

}  // namespace

GLCM_API int glcm_compute_static(const void* img, int W, int H, int64_t stride, int dtype, int N, uint32_t lo,
                                 uint32_t hi, const glcm_offset_t* offsets, int K, uint32_t* out, void* stream) {
  if (N >= 1 && K >= 1 && (uint64_t)K * (uint64_t)N * (uint64_t)N > GLCM_STATIC_MAX_WORDS) return GLCM_EINVAL;
  int device = 0;
  const hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return glcm::hip_error_status(e);
  uint32_t* slices = nullptr;
  const int rc = scratch_on(device, &slices);
  if (rc != GLCM_OK) return rc;
  return glcm::compute_in_workspace(slices, kScratchWords, img, W, H, stride, dtype, N, lo, hi, offsets, K, out,
                                    (hipStream_t)stream);
}
