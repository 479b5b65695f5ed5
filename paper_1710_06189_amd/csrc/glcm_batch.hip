// Batch kernel: many images in one launch, quantize -> vote -> merge ->
// statistics fused per image.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "glcm_device.h"
#include "glcm_features.h"
#include "glcm_internal.h"

namespace glcm {
namespace {

// ---------------------------------------------------------------------------
// Batch kernel: one workgroup per image of a batch, fusing quantize, vote,
// merge and the Haralick statistics; results are stored directly (the
// workgroup owns the whole image, so no atomics and no second kernel).
// Images arrive largest first, so the hardware dispatcher balances the
// workgroups over the CUs.
//
// Images (16-byte aligned: misaligned ones are first copied by
// k_batch_realign) use the strip machinery with the wavefront split into row
// segments when the image is narrower than 1024 columns: lane l handles chunk
// l mod cw of segment l / cw (cw = chunks per row), each segment walking its
// own run of rows; halo pixels outside [0, W) take the sentinel.  Votes go to
// the strip LDS layout (kp = K GLCMs, D dwords per bin).
// ---------------------------------------------------------------------------
template <int MAXDY, int D, int KI, int CUR>
__device__ __forceinline__ void batch_vote(const uint32_t (&fa)[16], const TermRow<MAXDY> (&ring)[MAXDY + 1],
                                           const int (&code)[4], int K, uint32_t inc) {
  vote_glcm<MAXDY, D, KI, CUR>(fa, ring, code[KI], inc);  // 32-bit counters
  if constexpr (KI + 1 < kStripMaxKp) {
    if (K > KI + 1) batch_vote<MAXDY, D, KI + 1, CUR>(fa, ring, code, K, inc);
  }
}

template <typename Pix, int MAXDY, int D, int CUR>
__device__ __forceinline__ void batch_step(const BatchArgs& a, const Geom& geo, TermRow<MAXDY> (&ring)[MAXDY + 1],
                                           RawChunk<Pix> (&raw)[MAXDY + 1], int y, int x0, const LaneCols& cols,
                                           uint32_t C, uint32_t n1,
                                           uint32_t mb, uint32_t sent4, const int (&code)[4]) {
  constexpr int NR = MAXDY + 1;
  uint32_t fa[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) fa[t] = mad_u24(ring[CUR].s[MAXDY + t], n1, C);
  batch_vote<MAXDY, D, 0, CUR>(fa, ring, code, a.K, 1u);
  to_terms<Pix, MAXDY, true>(ring[CUR], raw[CUR], a, geo, y + NR, x0, sent4, mb, true);
  load_row<Pix>(raw[CUR], geo, y + 2 * NR, cols);
}

template <typename Pix, int MAXDY, int D>
__global__ __launch_bounds__(kBatchThreads) void k_batch(BatchArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  constexpr int NR = MAXDY + 1;
  const BatchTile t = a.tiles[blockIdx.x];
  const Geom geo{t.img, t.stride, t.W, t.H};
  const int K = a.K;
  const uint32_t N = a.q.nlev, n1 = a.pitch, NN = N * N;
  const uint32_t mb = 4u * D * (uint32_t)K;
  const uint32_t vote_words = n1 * n1 * (uint32_t)K * D;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const uint32_t g = threadIdx.x & (D - 1u);
  const uint32_t C = lds_address(lds) + 4u * g;
  const uint32_t sent4 = N * 0x01010101u;
  zero_lds(lds, vote_words);
  __syncthreads();

  {
    int code[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) code[q] = q < K ? a.vcode[q] : -1;
    // lane -> (segment, chunk)
    const int chunks = (t.W + 15) >> 4;
    const int cw = min(chunks, 64), segs = 64 / cw, spans = (chunks + 63) >> 6;
    const int seg = lane / cw, c = lane - seg * cw;
    const bool live = seg < segs;
    const int slots = nwaves * segs;  // row segments walked at once by the workgroup
    const int h = max(a.min_rows, (t.H * spans + slots - 1) / slots);
    const int blocks = (t.H + segs * h - 1) / (segs * h);
    for (int u = wave; u < spans * blocks; u += nwaves) {
      const int span = u % spans, blk = u / spans;
      const int x0 = live ? ((span << 6) + c) << 4 : spans << 10;  // idle lanes: past the right edge
      const int ya = (blk * segs + (live ? seg : 0)) * h;
      TermRow<MAXDY> ring[NR];
      RawChunk<Pix> raw[NR];
      const LaneCols cols = lane_cols<Pix>(geo, x0);
#pragma unroll
      for (int r = 0; r < NR; ++r) load_row<Pix>(raw[r], geo, ya + r, cols);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        to_terms<Pix, MAXDY, true>(ring[r], raw[r], a, geo, ya + r, x0, sent4, mb, true);
        load_row<Pix>(raw[r], geo, ya + NR + r, cols);
      }
      // every lane takes h steps; rows past the image or the lane's segment
      // end carry the sentinel or belong to this segment's own run
      for (int j = 0; j < h; j += NR) {
        batch_step<Pix, MAXDY, D, 0>(a, geo, ring, raw, ya + j, x0, cols, C, n1, mb, sent4, code);
        if (j + 1 >= h) break;
        batch_step<Pix, MAXDY, D, 1>(a, geo, ring, raw, ya + j + 1, x0, cols, C, n1, mb, sent4, code);
        if constexpr (NR > 2) {
          if (j + 2 >= h) break;
          batch_step<Pix, MAXDY, D, 2>(a, geo, ring, raw, ya + j + 2, x0, cols, C, n1, mb, sent4, code);
        }
      }
    }
  }

  // merge: consecutive 16-byte units, D / 4 lanes per bin, into out and into
  // an LDS copy for the statistics
  __syncthreads();
  constexpr uint32_t QPB = D / 4;
  uint32_t* merged = lds + vote_words;
  uint32_t* dst = a.out + (size_t)t.index * K * NN;
  // unit u = ((i * n1 + j) * K + k) * QPB + r: (i, j, k) step by the
  // mixed-radix digits of blockDim / QPB each pass, so nothing is divided
  const uint32_t S = blockDim.x / QPB, uK = (uint32_t)K;
  const uint32_t sk = S % uK, sj = S / uK % n1, si = S / uK / n1;
  const uint32_t blk0 = threadIdx.x / QPB;
  uint32_t mk = blk0 % uK, mj = blk0 / uK % n1, mi = blk0 / uK / n1;
  const bool lead = threadIdx.x % QPB == 0;
  for (uint32_t u = threadIdx.x; u < vote_words / 4u; u += blockDim.x) {
    const uint4 v = ((const uint4*)lds)[u];
    uint32_t sum = (v.x + v.y) + (v.z + v.w);
    if (QPB >= 2) sum += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)sum, 0xb1, 0xf, 0xf, false);
    if (QPB >= 4) sum += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)sum, 0x4e, 0xf, 0xf, false);
    if (lead && mi < N && mj < N) {
      const bool tr = (a.tmask >> mk) & 1ull;
      const uint32_t w = mk * NN + (tr ? mj * N + mi : mi * N + mj);
      dst[w] = sum;
      merged[w] = sum;
    }
    mk += sk;
    const uint32_t ck = mk >= uK;
    mk -= ck ? uK : 0u;
    mj += sj + ck;  // < 2 n1
    const uint32_t cj = mj >= n1;
    mj -= cj ? n1 : 0u;
    mi += si + cj;
  }
  if (!a.feat) return;
  __syncthreads();
  unsigned long long* redu = (unsigned long long*)(merged + K * NN + ((K * NN) & 1u));
  float* redf = (float*)(redu + blockDim.x);
  for (int k = 0; k < K; ++k)
    glcm_features_wg(merged + k * NN, N, a.feat + ((size_t)t.index * K + k) * 5, redu, redf);
}

// Copies each misaligned image of a batch into the staging buffer with a
// 16-byte row pitch, so the batch kernel reads every image with 16-byte
// loads.  One workgroup per image; a thread makes one 16-byte group of a
// destination row from the (up to) five aligned source dwords that span it
// (v_alignbyte), reading only dwords that hold a byte of the row, zeroes the
// bytes past W and stores the group whole.  (row, group) advance by the
// mixed-radix digits of blockDim: no division.
template <typename Pix>
__global__ __launch_bounds__(256) void k_batch_realign(const RealignDesc* d, char* stage) {
  const RealignDesc e = d[blockIdx.x];
  uint4* dst = (uint4*)(stage + e.dst_off);
  const uint32_t rowbytes = (uint32_t)e.W * (uint32_t)sizeof(Pix);
  const uint32_t gw = (rowbytes + 15u) / 16u;                           // groups of a row that hold pixels
  const uint32_t gpitch = (uint32_t)e.dpitch * (uint32_t)sizeof(Pix) / 16u;  // groups per copy row
  const uint32_t sy = blockDim.x / gw, sg = blockDim.x % gw;
  uint32_t y = threadIdx.x / gw, g = threadIdx.x % gw;
  while (y < (uint32_t)e.H) {
    const uintptr_t r0 = (uintptr_t)((const char*)e.src + (int64_t)y * e.sstride * (int64_t)sizeof(Pix));
    const uint32_t* a0 = (const uint32_t*)(r0 & ~(uintptr_t)3);
    const uint32_t sh = (uint32_t)(r0 & 3u);  // bytes the row starts past a dword boundary
    // source dword 4g + i spans row bytes [16g + 4i - sh, 16g + 4i + 4 - sh)
    uint32_t a[5];
#pragma unroll
    for (uint32_t i = 0; i < 5; ++i) a[i] = 16u * g + 4u * i < rowbytes + sh ? a0[4u * g + i] : 0u;
    uint32_t v[4];
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
      v[i] = sh ? __builtin_amdgcn_alignbyte(a[i + 1], a[i], sh) : a[i];
      const int32_t left = (int32_t)rowbytes - (int32_t)(16u * g + 4u * i);  // row bytes from this dword on
      if (left <= 0) v[i] = 0u;
      else if (left < 4) v[i] &= (1u << (8u * (uint32_t)left)) - 1u;
    }
    dst[(size_t)y * gpitch + g] = make_uint4(v[0], v[1], v[2], v[3]);
    g += sg;
    y += sy;
    if (g >= gw) {
      g -= gw;
      ++y;
    }
  }
}

}  // namespace

hipError_t launch_batch_realign(const RealignDesc* d, int n, char* stage, int dtype_bytes, hipStream_t stream) {
  if (dtype_bytes == 1)
    hipLaunchKernelGGL(k_batch_realign<uint8_t>, dim3(n), dim3(256), 0, stream, d, stage);
  else
    hipLaunchKernelGGL(k_batch_realign<uint16_t>, dim3(n), dim3(256), 0, stream, d, stage);
  return hipGetLastError();
}

template <typename Pix, int MAXDY>
static hipError_t launch_batch_t(const BatchArgs& a, int T, int D, size_t lds_bytes, hipStream_t stream) {
  const dim3 grid(T), block(kBatchThreads);
  switch (D) {
    case 4: hipLaunchKernelGGL((k_batch<Pix, MAXDY, 4>), grid, block, lds_bytes, stream, a); break;
    case 8: hipLaunchKernelGGL((k_batch<Pix, MAXDY, 8>), grid, block, lds_bytes, stream, a); break;
    case 16: hipLaunchKernelGGL((k_batch<Pix, MAXDY, 16>), grid, block, lds_bytes, stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& a, int T, int dtype_bytes, int maxdy, int D, size_t lds_bytes,
                        hipStream_t stream) {
  if (maxdy == 1)
    return dtype_bytes == 1 ? launch_batch_t<uint8_t, 1>(a, T, D, lds_bytes, stream)
                            : launch_batch_t<uint16_t, 1>(a, T, D, lds_bytes, stream);
  if (maxdy == 2)
    return dtype_bytes == 1 ? launch_batch_t<uint8_t, 2>(a, T, D, lds_bytes, stream)
                            : launch_batch_t<uint16_t, 2>(a, T, D, lds_bytes, stream);
  return hipErrorInvalidValue;
}

}  // namespace glcm
