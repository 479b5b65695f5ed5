// Interface between the host runtime and the 1-D histogram kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "glcm_internal.h"

namespace glcm {

// Arguments of the 1-D histogram kernel.  The quantizer fields match VoteArgs
// so the packed quantizers take either.
struct HistArgs {
  const void* img;     // row y at img + y * stride elements
  int64_t stride;      // elements
  int W, H;
  Quant q;             // q.nlev = N levels
  int qfast;
  uint32_t qfast_shift, qfast_mask;
  int vec;             // 1: base and row pitch 16-byte aligned (16-byte chunk loads)
  uint32_t D;          // LDS copies per level, a power of two <= 32
  uint32_t cpr;        // 16-pixel chunks per row
  uint64_t per_block;  // chunks per workgroup
  uint32_t* partials;  // [gridDim][N] per-workgroup histograms
};
constexpr int kHistThreads = 1024;

// 1-D histogram: `groups` workgroups write a.partials; lds_bytes = 4 N D.
hipError_t launch_histogram(const HistArgs& a, int dtype_bytes, int groups, size_t lds_bytes, hipStream_t stream,
                            const LaunchTiming& tm = {});

}  // namespace glcm
