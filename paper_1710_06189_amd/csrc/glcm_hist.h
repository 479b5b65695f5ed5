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

// Launch geometry of the histogram over H rows of cpr chunks: at least two
// chunks per thread, at most one workgroup per CU; workgroup b owns chunks
// [b per_block, (b + 1) per_block).  Returns the workgroup count.
inline int hist_geometry(uint64_t chunks, int num_cus, uint64_t* per_block) {
  const uint64_t want = (chunks + 2u * kHistThreads - 1u) / (2u * kHistThreads);
  const uint64_t cap = num_cus > 0 ? (uint64_t)num_cus : 1u;
  const uint64_t groups = want < 1 ? 1 : (want < cap ? want : cap);
  *per_block = (chunks + groups - 1) / groups;
  return (int)((chunks + *per_block - 1) / *per_block);
}

// 1-D histogram: `groups` workgroups write a.partials; lds_bytes = 4 N D.
hipError_t launch_histogram(const HistArgs& a, int dtype_bytes, int groups, size_t lds_bytes, hipStream_t stream,
                            const LaunchTiming& tm = {});

}  // namespace glcm
