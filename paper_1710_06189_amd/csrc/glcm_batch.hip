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

// BAND: the item is a band of an image's first-pixel rows; rows at or past
// y_end (still read as second pixels) vote as the sentinel level (fsent).
template <typename Pix, int MAXDY, int D, int CUR, bool UNAL, bool BAND>
__device__ __forceinline__ void batch_step(const BatchArgs& a, const Geom& geo, TermRow<MAXDY> (&ring)[MAXDY + 1],
                                           RawChunk<Pix> (&raw)[MAXDY + 1], int y, int x0, const LaneCols& cols,
                                           uint32_t C, uint32_t n1,
                                           uint32_t mb, uint32_t sent4, const int (&code)[4], int y_end,
                                           uint32_t fsent) {
  constexpr int NR = MAXDY + 1;
  uint32_t fa[16];
  const bool first = !BAND || y < y_end;
#pragma unroll
  for (int t = 0; t < 16; ++t) fa[t] = first ? mad_u24(ring[CUR].s[MAXDY + t], n1, C) : fsent;
  batch_vote<MAXDY, D, 0, CUR>(fa, ring, code, a.K, 1u);
  to_terms<Pix, MAXDY, true>(ring[CUR], raw[CUR], a, geo, y + NR, x0, sent4, mb, true);
  row_load<Pix, UNAL>(raw[CUR], geo, y + 2 * NR, x0, cols);
}

// The votes of one item (first-pixel rows [t.y0, t.y1) of an image): lane ->
// (segment, chunk), every wavefront walking runs of rows of its segments.
template <typename Pix, int MAXDY, int D, bool UNAL, bool BAND>
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
  const int rows = t.y1 - t.y0;
  const int h = max(a.min_rows, (rows * spans + slots - 1) / slots);
  const int blocks = (rows + segs * h - 1) / (segs * h);
  const uint32_t fsent = mad_u24(a.q.nlev * mb, n1, C);
  for (int u = wave; u < spans * blocks; u += nwaves) {
    const int span = u % spans, blk = u / spans;
    const int x0 = live ? ((span << 6) + c) << 4 : spans << 10;  // idle lanes: past the right edge
    const int ya = t.y0 + (blk * segs + (live ? seg : 0)) * h;
    TermRow<MAXDY> ring[NR];
    RawChunk<Pix> raw[NR];
    LaneCols cols{};
    if constexpr (!UNAL) cols = lane_cols<Pix>(geo, x0);
#pragma unroll
    for (int r = 0; r < NR; ++r) row_load<Pix, UNAL>(raw[r], geo, ya + r, x0, cols);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      to_terms<Pix, MAXDY, true>(ring[r], raw[r], a, geo, ya + r, x0, sent4, mb, true);
      row_load<Pix, UNAL>(raw[r], geo, ya + NR + r, x0, cols);
    }
    // every lane takes h steps; rows past the image or the lane's segment
    // end carry the sentinel or belong to this segment's own run
    for (int j = 0; j < h; j += NR) {
      batch_step<Pix, MAXDY, D, 0, UNAL, BAND>(a, geo, ring, raw, ya + j, x0, cols, C, n1, mb, sent4, code, t.y1,
                                               fsent);
      if (j + 1 >= h) break;
      batch_step<Pix, MAXDY, D, 1, UNAL, BAND>(a, geo, ring, raw, ya + j + 1, x0, cols, C, n1, mb, sent4, code,
                                               t.y1, fsent);
      if constexpr (NR > 2) {
        if (j + 2 >= h) break;
        batch_step<Pix, MAXDY, D, 2, UNAL, BAND>(a, geo, ring, raw, ya + j + 2, x0, cols, C, n1, mb, sent4, code,
                                                 t.y1, fsent);
      }
    }
  }
}

// One item (an image or a band of one) into the workgroup's LDS copies,
// which are zero on entry and zero again on return (the merge clears what it
// reads, so the next item needs no clearing pass).
template <typename Pix, int MAXDY, int D>
__device__ __forceinline__ void batch_item(const BatchArgs& a, const BatchTile& t, uint32_t* lds) {
  const Geom geo{t.img, t.stride, t.W, t.H};
  const int K = a.K;
  const uint32_t N = a.q.nlev, n1 = a.pitch, NN = N * N;
  const uint32_t mb = 4u * D * (uint32_t)K;
  const uint32_t vote_words = n1 * n1 * (uint32_t)K * D;
  const int wave = threadIdx.x >> 6;
  const uint32_t g = threadIdx.x & (D - 1u);
  const uint32_t C = lds_address(lds) + 4u * g;
  const uint32_t sent4 = N * 0x01010101u;
  const bool band = t.slot >= 0;
  if (t.unaligned) {
    if (band) batch_votes<Pix, MAXDY, D, true, true>(a, t, geo, C, n1, mb, sent4);
    else batch_votes<Pix, MAXDY, D, true, false>(a, t, geo, C, n1, mb, sent4);
  } else {
    if (band) batch_votes<Pix, MAXDY, D, false, true>(a, t, geo, C, n1, mb, sent4);
    else batch_votes<Pix, MAXDY, D, false, false>(a, t, geo, C, n1, mb, sent4);
  }

  // merge: consecutive 16-byte units, D / 4 lanes per bin, into out and into
  // an LDS copy for the statistics; each unit is cleared once read
  __syncthreads();
  constexpr uint32_t QPB = D / 4;
  uint32_t* merged = lds + vote_words;
  // a whole image: its counts; a band: its partial counts, summed (and the
  // statistics taken) by k_batch_fin
  uint32_t* dst = band ? a.partials + (size_t)t.slot * K * NN
                       : (a.outs ? a.outs[t.index] : a.out + (size_t)t.index * K * NN);
  // unit u = ((i * n1 + j) * K + k) * QPB + r: (i, j, k) step by the
  // mixed-radix digits of blockDim / QPB each pass, so nothing is divided
  const uint32_t S = blockDim.x / QPB, uK = (uint32_t)K;
  const uint32_t sk = S % uK, sj = S / uK % n1, si = S / uK / n1;
  const uint32_t blk0 = threadIdx.x / QPB;
  uint32_t mk = blk0 % uK, mj = blk0 / uK % n1, mi = blk0 / uK / n1;
  const bool lead = threadIdx.x % QPB == 0;
  for (uint32_t u = threadIdx.x; u < vote_words / 4u; u += blockDim.x) {
    const uint4 v = ((const uint4*)lds)[u];
    ((uint4*)lds)[u] = make_uint4(0u, 0u, 0u, 0u);
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
  if (band) return;
  float* const fdst = a.outs ? (a.feats ? a.feats[t.index] : nullptr)
                             : (a.feat ? a.feat + (size_t)t.index * K * 5 : nullptr);
  if (!fdst) return;  // (the same on every thread of the workgroup)
  __syncthreads();
  // one wavefront per GLCM (a wavefront takes several when the workgroup has
  // fewer wavefronts than K)
  for (int k = wave; k < K; k += (int)(blockDim.x >> 6)) glcm_features_wave(merged + k * NN, N, fdst + k * 5);
}

// Persistent workgroups: each takes the next item from a counter (items are
// ordered largest first) until none is left.  The counter is zero at launch.
// Every workgroup takes one number past the last item before it stops, so
// the counter ends at nitems + gridDim.x, and the workgroup that drew the
// last number sets it back to zero: no other workgroup touches it after.
template <typename Pix, int MAXDY, int D, int WG>
__global__ __launch_bounds__(WG) void k_batch(BatchArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  __shared__ uint32_t s_item;
  const uint32_t vote_words = a.pitch * a.pitch * (uint32_t)a.K * D;
  zero_lds(lds, vote_words);
  if (threadIdx.x == 0) s_item = __hip_atomic_fetch_add(a.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  for (;;) {
    const uint32_t item = s_item;
    if (item >= (uint32_t)a.nitems) {
      if (threadIdx.x == 0 && item == (uint32_t)a.nitems + gridDim.x - 1u)
        __hip_atomic_store(a.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    // the next item's number is fetched while this one is counted
    uint32_t next = 0;
    if (threadIdx.x == 0) next = __hip_atomic_fetch_add(a.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    batch_item<Pix, MAXDY, D>(a, a.tiles[item], lds);
    __syncthreads();  // the item's LDS use and its read of s_item are over
    if (threadIdx.x == 0) s_item = next;
    __syncthreads();
  }
}

// The images split into bands: one workgroup per image sums its bands'
// partial counts (in band order) into out and takes the statistics.
__global__ __launch_bounds__(kBatchThreads) void k_batch_fin(BatchArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  const BatchFin f = a.fins[blockIdx.x];
  const uint32_t N = a.q.nlev, NN = N * N, KNN = (uint32_t)a.K * NN;
  uint32_t* dst = a.outs ? a.outs[f.index] : a.out + (size_t)f.index * KNN;
  const uint32_t* src = a.partials + (size_t)f.slot0 * KNN;
  for (uint32_t w = threadIdx.x; w < KNN; w += blockDim.x) {
    uint32_t s = 0;
    for (int p = 0; p < f.parts; ++p) s += src[(size_t)p * KNN + w];
    dst[w] = s;
    lds[w] = s;
  }
  float* const fdst = a.outs ? (a.feats ? a.feats[f.index] : nullptr)
                             : (a.feat ? a.feat + (size_t)f.index * a.K * 5 : nullptr);
  if (!fdst) return;
  __syncthreads();
  const int wave = (int)(threadIdx.x >> 6);
  for (int k = wave; k < a.K; k += (int)(blockDim.x >> 6)) glcm_features_wave(lds + k * NN, N, fdst + k * 5);
}

}  // namespace

template <typename Pix, int MAXDY, int WG>
static hipError_t launch_batch_w(const BatchArgs& a, int T, int D, size_t lds_bytes, hipStream_t stream) {
  const dim3 grid(T), block(WG);  // T persistent workgroups
  switch (D) {
    case 4: hipLaunchKernelGGL((k_batch<Pix, MAXDY, 4, WG>), grid, block, lds_bytes, stream, a); break;
    case 8: hipLaunchKernelGGL((k_batch<Pix, MAXDY, 8, WG>), grid, block, lds_bytes, stream, a); break;
    case 16: hipLaunchKernelGGL((k_batch<Pix, MAXDY, 16, WG>), grid, block, lds_bytes, stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Pix, int MAXDY>
static hipError_t launch_batch_t(const BatchArgs& a, int T, int D, int wg, size_t lds_bytes, hipStream_t stream) {
  if (wg == 256) return launch_batch_w<Pix, MAXDY, 256>(a, T, D, lds_bytes, stream);
  if (wg == 512) return launch_batch_w<Pix, MAXDY, 512>(a, T, D, lds_bytes, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_batch_fin(const BatchArgs& a, int F, hipStream_t stream) {
  if (F <= 0) return hipSuccess;
  const size_t lds = batch_fin_lds_bytes((int)a.q.nlev, a.K);
  hipLaunchKernelGGL(k_batch_fin, dim3(F), dim3(kBatchThreads), lds, stream, a);
  return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& a, int T, int dtype_bytes, int maxdy, int D, int wg, size_t lds_bytes,
                        hipStream_t stream) {
  if (maxdy == 1)
    return dtype_bytes == 1 ? launch_batch_t<uint8_t, 1>(a, T, D, wg, lds_bytes, stream)
                            : launch_batch_t<uint16_t, 1>(a, T, D, wg, lds_bytes, stream);
  if (maxdy == 2)
    return dtype_bytes == 1 ? launch_batch_t<uint8_t, 2>(a, T, D, wg, lds_bytes, stream)
                            : launch_batch_t<uint16_t, 2>(a, T, D, wg, lds_bytes, stream);
  return hipErrorInvalidValue;
}

}  // namespace glcm
