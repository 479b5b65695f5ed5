// 1-D gray-level histogram of a device image, h[i] = number of pixels whose
// quantized level is i.  The paper observes (Contributions) that its analysis
// of colliding increments applies to statistical histograms as well; this is
// that histogram, counted with the same replicated-LDS votes as the GLCM:
// D copies of every level, lane g of a 32-lane LDS pass voting into copy
// g mod D, so with D = 32 no two lanes of a pass ever share a bank and equal
// levels never collide.
//
// Workgroup b owns chunks [b * per_block, (b + 1) * per_block) of the image
// taken as rows of 16-pixel chunks; it writes its D-copy sum to partials[b]
// and the band-partial reduction adds the workgroups up.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "glcm_device.h"
#include "glcm_hist.h"

namespace glcm {
namespace {

typedef __attribute__((address_space(3))) uint32_t lds_u32_t;

__device__ __forceinline__ void vote_level(uint32_t base_g, uint32_t lv, uint32_t stride_d) {
  __hip_atomic_fetch_add((lds_u32_t*)(size_t)(base_g + lv * stride_d), 1u, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The 16 pixels of a chunk as loaded: 16-byte blocks that hold at least one
// pixel of the row (the row base and pitch are 16-byte aligned, so such a
// block never leaves the allocation); a u16 chunk's second block only when it
// starts inside the row.
struct ChunkRaw {
  uint4 v0, v1;
};

template <typename Pix>
__device__ __forceinline__ ChunkRaw load_chunk(const HistArgs& a, const char* row, int x0) {
  ChunkRaw r;
  r.v0 = *(const uint4*)(row + (size_t)x0 * sizeof(Pix));
  r.v1 = r.v0;
  if (sizeof(Pix) == 2 && chunk_second_block(x0, a.W)) r.v1 = *(const uint4*)(row + (size_t)(x0 + 8) * 2u);
  return r;
}

// Votes the first n (<= 16) pixels of a loaded chunk.
template <typename Pix>
__device__ __forceinline__ void vote_chunk(const HistArgs& a, const ChunkRaw& r, int n, uint32_t base_g,
                                           uint32_t stride_d) {
  if (a.q.nlev <= 256u) {
    uint32_t c[4];
    if (sizeof(Pix) == 1) {
      c[0] = quant4_u8(r.v0.x, a); c[1] = quant4_u8(r.v0.y, a); c[2] = quant4_u8(r.v0.z, a); c[3] = quant4_u8(r.v0.w, a);
    } else {
      c[0] = quant4_u16(r.v0.x, r.v0.y, a); c[1] = quant4_u16(r.v0.z, r.v0.w, a);
      c[2] = quant4_u16(r.v1.x, r.v1.y, a); c[3] = quant4_u16(r.v1.z, r.v1.w, a);
    }
    if (n == 16) {
#pragma unroll
      for (int t = 0; t < 16; ++t) vote_level(base_g, (c[t >> 2] >> ((t & 3) * 8)) & 0xffu, stride_d);
    } else {
      for (int t = 0; t < n; ++t) vote_level(base_g, (c[t >> 2] >> ((t & 3) * 8)) & 0xffu, stride_d);
    }
  } else {
    const uint32_t w[8] = {r.v0.x, r.v0.y, r.v0.z, r.v0.w, r.v1.x, r.v1.y, r.v1.z, r.v1.w};
    for (int t = 0; t < n; ++t) {
      const uint32_t px = sizeof(Pix) == 1 ? (w[t >> 2] >> ((t & 3) * 8)) & 0xffu
                                           : (w[t >> 1] >> ((t & 1) * 16)) & 0xffffu;
      vote_level(base_g, quantize(px, a.q), stride_d);
    }
  }
}

constexpr int kHistUnroll = 4;  // chunk loads a thread keeps in flight

template <typename Pix>
__global__ __launch_bounds__(kHistThreads) void k_histogram(HistArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  const uint32_t N = a.q.nlev, D = a.D;
  zero_lds(lds, N * D);
  const uint32_t g = threadIdx.x & (D - 1u);
  const uint32_t base_g = (uint32_t)(size_t)(const lds_u32_t*)lds + 4u * g, stride_d = 4u * D;
  const uint64_t c0 = (uint64_t)blockIdx.x * a.per_block;
  const uint64_t c1 = min(c0 + a.per_block, (uint64_t)a.H * a.cpr);
  const uint64_t first = c0 + threadIdx.x;
  ChunkPos pos{first, (int)(first / a.cpr), (uint32_t)(first % a.cpr)};
  const uint32_t sy = blockDim.x / a.cpr, sc = blockDim.x % a.cpr;
  __syncthreads();
  const size_t pitch = (size_t)a.stride * sizeof(Pix);
  if (a.vec) {
    while (pos.i < c1) {
      ChunkRaw raw[kHistUnroll];
      int n[kHistUnroll];
#pragma unroll
      for (int u = 0; u < kHistUnroll; ++u) {
        n[u] = 0;
        if (pos.i < c1) {
          const int x0 = (int)(pos.c << 4);
          raw[u] = load_chunk<Pix>(a, (const char*)a.img + (size_t)pos.y * pitch, x0);
          n[u] = min(16, a.W - x0);
        }
        pos.step(blockDim.x, sy, sc, a.cpr);
      }
#pragma unroll
      for (int u = 0; u < kHistUnroll; ++u)
        if (n[u]) vote_chunk<Pix>(a, raw[u], n[u], base_g, stride_d);
    }
  } else {
    for (; pos.i < c1; pos.step(blockDim.x, sy, sc, a.cpr)) {
      const int x0 = (int)(pos.c << 4), n = min(16, a.W - x0);
      const Pix* p = (const Pix*)((const char*)a.img + (size_t)pos.y * pitch) + x0;
      for (int t = 0; t < n; ++t) vote_level(base_g, quantize((uint32_t)p[t], a.q), stride_d);
    }
  }
  __syncthreads();
  // sum the D copies of each level, reading them in an order rotated by the
  // level so the lanes of a pass hit different banks
  uint32_t* dst = a.partials + (size_t)blockIdx.x * N;
  for (uint32_t v = threadIdx.x; v < N; v += blockDim.x) {
    uint32_t s = 0;
    for (uint32_t k = 0; k < D; ++k) s += lds[v * D + ((k + v) & (D - 1u))];
    dst[v] = s;
  }
}

}  // namespace

hipError_t launch_histogram(const HistArgs& a, int dtype_bytes, int groups, size_t lds_bytes, hipStream_t stream,
                            const LaunchTiming& tm) {
  const dim3 grid((unsigned)groups), block(kHistThreads);
  if (dtype_bytes == 1)
    hipExtLaunchKernelGGL(k_histogram<uint8_t>, grid, block, (uint32_t)lds_bytes, stream, tm.start, tm.stop, 0u, a);
  else
    hipExtLaunchKernelGGL(k_histogram<uint16_t>, grid, block, (uint32_t)lds_bytes, stream, tm.start, tm.stop, 0u, a);
  return hipGetLastError();
}

}  // namespace glcm
