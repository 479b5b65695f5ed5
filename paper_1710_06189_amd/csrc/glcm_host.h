// Host-side helpers of glcm_api.cpp that the request server shares (not
// exported from the library).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "glcm.h"

namespace glcm {

// Records a failed HIP call for glcm_last_hip_error() and maps it to
// GLCM_ENOMEM / GLCM_EHIP (GLCM_OK for hipSuccess).
int hip_error_status(hipError_t e);

// The argument checks of glcm_compute that need no HIP call (out may be NULL
// here: the server allocates it later).
int check_request_args(const void* img, int W, int H, int64_t stride, int dtype, int N, uint32_t lo, uint32_t hi,
                       const glcm_offset_t* offsets, int K);

// 0 = pageable host, 1 = pinned host, 2 = device memory; *device = its device.
int memory_kind(const void* p, int* device);

// glcm_compute on a device image without a plan and without allocating:
// a plan lives on the stack for the call, its per-XCD accumulation slices are
// `slices` (device memory of slice_words 32-bit words, any content on entry,
// zero on return), misaligned images take the per-pixel kernels instead of a
// staging copy.  GLCM_EINVAL when kXcdSlots * K * N * N > slice_words or
// either pointer is not device memory of the current device.
int compute_in_workspace(uint32_t* slices, size_t slice_words, const void* img, int W, int H, int64_t stride,
                         int dtype, int N, uint32_t lo, uint32_t hi, const glcm_offset_t* offsets, int K,
                         uint32_t* out, hipStream_t stream);

// glcm_batch_compute with a destination per image: image t's counts go to
// outs[t] (device, K*N*N words) and its statistics to feats[t] (K*5 floats;
// feats or feats[t] NULL: none).  Same checks and errors otherwise, except
// that the destinations are not checked against the tiles.
int batch_compute_to(glcm_plan_t plan, const glcm_tile_t* tiles, int T, uint32_t lo, uint32_t hi,
                     uint32_t* const* outs, float* const* feats, hipStream_t stream);

}  // namespace glcm
