// Internal interface between the C-ABI host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace glcm {

constexpr int kMaxK = 64;
// Accumulation slices for the per-XCD merge (an MI355X has 8 XCDs; the slice
// is XCC_ID mod kXcdSlots, which stays one slice per XCD up to 16 XCDs).
constexpr uint32_t kXcdSlots = 16;
// GLCMs per partition of the strip kernel (its vote loop is unrolled over them).
constexpr int kStripMaxKp = 4;
// Threads per workgroup the strip kernel accepts for a pixel size and template
// reach (1, 2 or 4): a ring of five term rows (reach 4), or uint16 raw rows at
// reach 2, need more than the 128 registers a 1024-thread workgroup leaves a
// lane.
constexpr int strip_max_threads(int pixel_bytes, int maxdy) {
  return maxdy > 2 || (pixel_bytes == 2 && maxdy == 2) ? 512 : 1024;
}
// Threads per workgroup the slab kernel accepts: uint16 rows of reach 4 read in
// place (eight rows of 13 dwords in flight) need more than a 1024-thread
// workgroup's 128 registers per lane.
constexpr int rows_max_threads(int pixel_bytes, int maxdy, bool unaligned) {
  return unaligned && pixel_bytes == 2 && maxdy > 2 ? 512 : 1024;
}

// Gray-level reduction q(v): 0 below lo, N-1 above hi, otherwise
// floor(x / D) with x = (v - lo) * N and D = hi - lo + 1, evaluated as
// (x + mulhi(x, magic)) >> shift.  With shift = ceil(log2 D) and
// magic = ceil(2^(32+shift) / D) - 2^32 this is exact for every x < 2^32
// (Granlund-Montgomery division by an invariant integer).
struct Quant {
  uint32_t lo, hi, nlev, magic, shift;
};

// Arguments shared by every counting kernel.  Passed by value.
struct VoteArgs {
  const void* img;            // first row of the (tile) image
  int64_t stride;             // row pitch in elements
  int W, H;                   // image (tile) size; second pixels must lie inside
  int y_begin, y_end;         // rows whose pixels act as FIRST pixel of a pair
  Quant q;
  int qfast;                  // 1: lo = 0, hi = dtype max, N = 2^n: level = pixel >> qfast_shift
  uint32_t qfast_shift, qfast_mask;  // shift and per-byte (u8) / per-halfword (u16) mask
  int unaligned;              // strip and slab kernels: 1 = base or row pitch not 16-byte aligned
                              // (rows assembled from the dwords that hold them), 0 = 16-byte loads
  int K;
  int32_t dx[kMaxK], dy[kMaxK];
  unsigned long long tmask;   // row kernel: bit k set = offset k was negated, vote (j, i)
  int log2R;                  // LDS replicas per workgroup = 1 << log2R
  uint32_t words_total;       // K * N * N
  uint32_t part_words;        // GLCM words held in LDS per partition
  int P;                      // bin partitions
  int nregions;               // row bands; workgroup g counts band g / P, partition g % P
  int region_rows;            // first-pixel rows per band
  int rows_per_wave;          // row kernel: first-pixel rows per wavefront slab (4)
  uint32_t pitch;             // row kernel: LDS row pitch of a GLCM, >= N + 1 (row/column N: sentinel)
  Quant div_n, div_nn;        // magic/shift for dividing by N and by N*N (only those fields used)
  int c16;                    // slab kernel: 16-bit counters, two copies per dword; strip kernel:
                              // 16-bit counters, two GLCMs per dword; generic kernel: 16-bit
                              // counters, two consecutive words per dword (one copy)
  int kp;                     // strip kernel: GLCMs per partition (<= 4)
  int kg;                     // strip kernel: dword groups per bin (kp, or kp / 2 rounded up with c16)
  int strip_rows;             // strip kernel: first-pixel rows per wavefront strip
  int merge_pack;             // strip kernel, 16-bit pairs: copies the merge may add before splitting
                              // the halves (merge_pack times the largest count stays below 2^16)
  int32_t vcode[kMaxK];       // strip kernel: dy * (2 MAXDY + 1) + dx + MAXDY of each canonical offset
                              // (dwords: the kernel reads them with scalar loads)
  uint32_t* partials;         // [nregions][words_total] per-band counts (band-partial merge)
  uint32_t* xbuf;             // [kXcdSlots][words_total] per-XCD accumulators, or null
  uint32_t* out;              // global-atomic kernel: [words_total] counts, zeroed beforehand
};

// Block-code kernel (the four d = 1 directions).  Each first pixel (x, y) and
// its 2x2 block [a b; d e] (a = (x, y), b = (x+1, y), d = (x, y+1), e =
// (x+1, y+1)) hold exactly one pair of each d = 1 GLCM: (1,0) -> (a, b),
// (-1,1) -> (b, d), (0,1) -> (a, d), (1,1) -> (a, e).  The kernel votes two
// codes per block instead of four pairs:
//   code 1 = 16 a + 4 (b - a + 1) + (d - a + 1) = 11 a + 4 b + d + 5
//            (the block's (1,0), (-1,1) and (0,1) pairs),
//   code 2 = 16 a + 4 (b - a + 1) + (e - a + 1) = 11 a + 4 b + e + 5
//            (its (1,1) pair),
// exact whenever the three differences lie in [-1, 2]; blocks outside that
// window are corrected one pair at a time.  Block GLCM g of the four above.
constexpr int kBlockGlcms = 4;
struct BlockArgs {
  const void* img;            // 16-byte aligned base and row pitch
  int64_t stride;             // elements
  int W, H;
  int y_begin, y_end;         // first-pixel rows
  Quant q;
  int qfast;
  uint32_t qfast_shift, qfast_mask;
  unsigned long long kmask[kBlockGlcms];  // bit k of kmask[g]: offset k is block direction g or its opposite
  unsigned long long tmask;   // bit k: offset k is the opposite of its block direction (stored transposed)
  int nregions, region_rows, strip_rows;
  uint32_t nbins;             // code bins: 16 N + 6 (every level combination, sentinel included, lands inside)
  int fb_copies;              // copies of the block GLCMs (1, 2 or 4; lane mod fb_copies)
  Quant div_n;                // magic/shift for dividing by N
  uint32_t words_total;       // K N N
  uint32_t* xbuf;             // per-XCD accumulation slices [kXcdSlots][words_total]
};
// LDS bytes of the block kernel: code bins (32 dwords each), the four block
// GLCMs in fbc copies (N^2 words each), one trash word per lane, queues of
// 512 dwords with blocks outside the code window (32 bytes each, 32 per
// wavefront) and their 16 counts.
inline size_t block_lds_bytes(int N, int fbc) {
  return (16u * (size_t)N + 6u) * 128u + (size_t)kBlockGlcms * (size_t)N * (size_t)N * (size_t)fbc * 4u + 64u * 4u +
         512u * 32u + 64u;
}

// One work item of a batch as the batch kernel reads it (device memory, 48
// bytes): an image, or a band of first-pixel rows of an image too large for
// one workgroup to finish with the others.
struct BatchTile {
  const void* img;  // device pixels, row y at img + y * stride elements
  int64_t stride;   // elements
  int32_t W, H;
  int32_t index;    // slot of this image in the caller's order (output position)
  int32_t unaligned; // 1: base or row pitch not 16-byte aligned (rows read as dwords), else 0
  int32_t y0, y1;   // first-pixel rows of the item (0, H for a whole image)
  int32_t slot;     // -1: a whole image; else the band's row of partial counts
  int32_t pad;
};
// An image split into bands: its bands' partial rows are slot0 .. slot0 + parts - 1.
struct BatchFin {
  int32_t index, slot0, parts, pad;
};

// Arguments of the fused batch kernel (quantize, vote, merge, features per
// image).  The quantizer fields match VoteArgs so the row helpers take either.
struct BatchArgs {
  Quant q;
  int qfast;
  uint32_t qfast_shift, qfast_mask;
  int K;                               // offsets, <= kStripMaxKp
  int32_t dx[kStripMaxKp], dy[kStripMaxKp];  // offsets as given (per-pixel path)
  int32_t vcode[kStripMaxKp];          // canonical codes (strip path), as in VoteArgs
  unsigned long long tmask;            // bit k: offset k counted as its opposite, stored transposed
  uint32_t pitch;                      // N + 1
  int min_rows;                        // shortest row segment a lane walks
  const BatchTile* tiles;              // [nitems], largest first
  const BatchFin* fins;                // [nfins] images split into bands
  uint32_t* partials;                  // [band slots][K][N][N] partial counts of the bands
  uint32_t* counter;                   // next item (zero at launch and again at the end)
  int nitems, nfins;
  uint32_t* out;                       // [T][K][N][N]
  float* feat;                         // [T][K][5] or null
  // or, when outs is set, image t's counts go to outs[t] ([K][N][N]) and its
  // statistics to feats[t] ([K][5]; feats or feats[t] null: none); device tables
  uint32_t* const* outs;
  float* const* feats;
};

// Optional events the counting kernel's dispatch stamps with its own start
// and end time (both null: plain launch).
struct LaunchTiming {
  hipEvent_t start = nullptr, stop = nullptr;
};

// Launchers (all asynchronous on `stream`; return the launch error).
hipError_t launch_vote_generic(const VoteArgs& a, int dtype_bytes, int wg, size_t lds_bytes, hipStream_t stream,
                               const LaunchTiming& tm = {});
hipError_t launch_vote_rows(const VoteArgs& a, int dtype_bytes, int maxdy, int rpw, int wg, size_t lds_bytes,
                            hipStream_t stream, const LaunchTiming& tm = {});
// D = dwords per bin (4, 8, 16 or 32), maxdy = 1, 2 or 4 (the ring holds maxdy + 1 rows).
hipError_t launch_vote_strips(const VoteArgs& a, int dtype_bytes, int maxdy, int D, int wg, size_t lds_bytes,
                              hipStream_t stream, const LaunchTiming& tm = {});
// out[w] = (accumulate ? out[w] : 0) + sum_b partials[b * M + w] for w < M.
hipError_t launch_reduce(const uint32_t* partials, uint32_t* out, uint32_t M, int nbands, bool accumulate,
                         hipStream_t stream);
// out[w] = (accumulate ? out[w] : 0) + sum_{x < nslots} xbuf[x * M + w]; zeroes those slices.
hipError_t launch_finish(uint32_t* xbuf, uint32_t* out, uint32_t M, uint32_t nslots, bool accumulate,
                         hipStream_t stream);
// p[w] = 0 for w < words (a kernel, not a memset node: capturable in a graph).
hipError_t launch_zero(uint32_t* p, uint64_t words, hipStream_t stream);
// ids[b] = XCC_ID of the XCD that ran workgroup b (b < blocks).
hipError_t launch_xcc_probe(uint32_t* ids, int blocks, hipStream_t stream);
hipError_t launch_vote_global(const VoteArgs& a, int dtype_bytes, hipStream_t stream);
// Large-N path: pairs added straight into the per-XCD slices (a.xbuf), rows
// in runs of a.region_rows; `groups` workgroups of 256 threads.
hipError_t launch_vote_l2(const VoteArgs& a, int dtype_bytes, int groups, hipStream_t stream,
                          const LaunchTiming& tm = {});
// Statistics of K GLCMs: one wavefront per GLCM up to this N, one workgroup above.
constexpr int kFeaturesWaveMaxN = 128;
hipError_t launch_features(const uint32_t* glcm, int K, int N, float* out, hipStream_t stream);
// Block-code kernel: a.nregions workgroups of `wg` threads, block_lds_bytes(N, a.fb_copies) of LDS.
hipError_t launch_vote_blocks(const BlockArgs& a, int dtype_bytes, int wg, hipStream_t stream,
                              const LaunchTiming& tm = {});
// T persistent workgroups of wg threads (256 or 512) over the a.nitems items
// of a batch; D = dwords per bin (4, 8 or 16), maxdy = 1 or 2.  lds_bytes
// from batch_lds_bytes().
hipError_t launch_batch(const BatchArgs& a, int T, int dtype_bytes, int maxdy, int D, int wg, size_t lds_bytes,
                        hipStream_t stream);
constexpr int kBatchThreads = 256;
// Sums the bands of the F split images into out (and their statistics);
// nothing is launched when F = 0.
hipError_t launch_batch_fin(const BatchArgs& a, int F, hipStream_t stream);
inline size_t batch_fin_lds_bytes(int N, int K) { return (size_t)K * N * N * 4u; }
inline size_t batch_lds_bytes(int N, int K, int D) {
  const size_t n1 = (size_t)N + 1u;
  // vote copies, then the merged counts the statistics read
  return (n1 * n1 * (size_t)K * (size_t)D + (size_t)K * N * N) * 4u;
}

}  // namespace glcm
