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
// Every image uses the strip machinery with the wavefront split into row
// segments when the image is narrower than 1024 columns: lane l handles chunk
// l mod cw of segment l / cw (cw = chunks per row), each segment walking its
// own run of rows; halo pixels outside [0, W) take the sentinel.  Votes go to
// the strip LDS layout (kp = K GLCMs, D dwords per bin).  Rows of an image
// whose base or pitch is not 16-byte aligned are assembled from dword loads
// (load_row_unaligned) instead of 16-byte loads.
// ---------------------------------------------------------------------------
template <int MAXDY, int D, int KI, int CUR>
__device__ __forceinline__ void batch_vote(const uint32_t (&fa)[16], const TermRow<MAXDY> (&ring)[MAXDY + 1],
                                           const int (&code)[4], int K, uint32_t inc) {
  vote_glcm<MAXDY, D, KI, CUR>(fa, ring, code[KI], inc);  // 32-bit counters
  if constexpr (KI + 1 < kStripMaxKp) {
    if (K > KI + 1) batch_vote<MAXDY, D, KI + 1, CUR>(fa, ring, code, K, inc);
  }
}

// Row loads of an image whose base or row pitch is not 16-byte aligned: the
// lane's 16-pixel chunk and its 4-pixel halos are assembled from the aligned
// dwords that span them (v_alignbyte_b32).  Only dwords that hold a byte of
// the row are read; the others count as zero, and to_terms replaces every
// pixel outside [0, W) by the sentinel anyway.
template <typename Pix>
__device__ __forceinline__ void load_row_unaligned(RawChunk<Pix>& rc, const Geom& g, int y, int x0) {
  constexpr int B = (int)sizeof(Pix);
  constexpr int NC = 4 * B;  // chunk dwords (16 pixels)
  constexpr int NH = B;      // halo dwords (4 pixels) on each side
  const UnalignedRow u = unaligned_row<Pix>(g, y, x0);
  const uint32_t* a0 = (const uint32_t*)u.a0;
  const uint32_t sh = u.sh;
  static_assert(NC + 2 * NH + 1 == unaligned_row_dwords<Pix>(), "dwords per unaligned row");
  uint32_t d[NC + 2 * NH + 1];
#pragma unroll
  for (int k = 0; k < NC + 2 * NH + 1; ++k) {
    const int j = u.j0 + k;
    d[k] = unaligned_dword_in_row(j, u.lim) ? a0[j] : 0u;
  }
  // dword m of the halo-chunk-halo run covers row bytes [4 (j0 + m), +4)
  uint32_t o[NC + 2 * NH];
#pragma unroll
  for (int m = 0; m < NC + 2 * NH; ++m) o[m] = __builtin_amdgcn_alignbyte(d[m + 1], d[m], sh);
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    rc.lh[h] = o[h];
    rc.rh[h] = o[NH + NC + h];
  }
#pragma unroll
  for (int v = 0; v < B; ++v) rc.v[v] = make_uint4(o[NH + 4 * v], o[NH + 4 * v + 1], o[NH + 4 * v + 2], o[NH + 4 * v + 3]);
}

// UNAL: the image is read by load_row_unaligned (cols unused), else by the
// 16-byte loads of the strip machinery.
template <typename Pix, bool UNAL>
__device__ __forceinline__ void batch_load(RawChunk<Pix>& rc, const Geom& g, int y, int x0, const LaneCols& cols) {
  if constexpr (UNAL)
    load_row_unaligned<Pix>(rc, g, y, x0);
  else
    load_row<Pix>(rc, g, y, cols);
}

template <typename Pix, int MAXDY, int D, int CUR, bool UNAL>
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
  batch_load<Pix, UNAL>(raw[CUR], geo, y + 2 * NR, x0, cols);
}

// The votes of one image: lane -> (segment, chunk), every wavefront walking
// runs of rows of its segments.
template <typename Pix, int MAXDY, int D, bool UNAL>
__device__ __forceinline__ void batch_votes(const BatchArgs& a, const BatchTile& t, const Geom& geo, uint32_t C,
                                            uint32_t n1, uint32_t mb, uint32_t sent4) {
  constexpr int NR = MAXDY + 1;
  const int K = a.K;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  int code[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) code[q] = q < K ? a.vcode[q] : -1;
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
    LaneCols cols{};
    if constexpr (!UNAL) cols = lane_cols<Pix>(geo, x0);
#pragma unroll
    for (int r = 0; r < NR; ++r) batch_load<Pix, UNAL>(raw[r], geo, ya + r, x0, cols);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      to_terms<Pix, MAXDY, true>(ring[r], raw[r], a, geo, ya + r, x0, sent4, mb, true);
      batch_load<Pix, UNAL>(raw[r], geo, ya + NR + r, x0, cols);
    }
    // every lane takes h steps; rows past the image or the lane's segment
    // end carry the sentinel or belong to this segment's own run
    for (int j = 0; j < h; j += NR) {
      batch_step<Pix, MAXDY, D, 0, UNAL>(a, geo, ring, raw, ya + j, x0, cols, C, n1, mb, sent4, code);
      if (j + 1 >= h) break;
      batch_step<Pix, MAXDY, D, 1, UNAL>(a, geo, ring, raw, ya + j + 1, x0, cols, C, n1, mb, sent4, code);
      if constexpr (NR > 2) {
        if (j + 2 >= h) break;
        batch_step<Pix, MAXDY, D, 2, UNAL>(a, geo, ring, raw, ya + j + 2, x0, cols, C, n1, mb, sent4, code);
      }
    }
  }
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
  if (t.unaligned)
    batch_votes<Pix, MAXDY, D, true>(a, t, geo, C, n1, mb, sent4);
  else
    batch_votes<Pix, MAXDY, D, false>(a, t, geo, C, n1, mb, sent4);

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

}  // namespace

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
