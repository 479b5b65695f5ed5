// Block-code counting kernel for the four d = 1 directions of Eq. (2).
//
// Each first pixel (x, y) and its 2x2 block [a b; d e] hold exactly one pair
// of each of the four d = 1 GLCMs (Eq. (1) at theta = 0, 45, 90, 135 degrees
// with the direction table of Eq. (2)): (a, b), (b, d), (a, d), (a, e).  On
// images whose gray levels vary slowly (the same-address case the copies of
// Section II.A are for) the levels of a block differ by at most one or two,
// so a block is summarised by two codes that carry its four pairs:
//
//   code 1 = 16 a + 4 (d - a + 1) + (b - a + 1) = 11 a + b + 4 d + 5
//   code 2 = 16 a + 4 (e - a + 1) + (b - a + 1) = 11 a + b + 4 e + 5
//
// Both are exact (decodable back to the pairs) when b - a, d - a and e - a lie
// in [-1, 2]; code 1 carries the pairs (a, b), (b, d), (a, d), code 2 the pair
// (a, e), and the two share their first-row part 11 a + b.  Every block votes both codes unconditionally (two LDS atomics
// per first pixel instead of four); a cheap byte-wise test then finds the
// blocks outside the window, whose two votes are taken back and whose four
// pairs are counted one by one.  The codes are linear in the four levels, so
// every level combination (sentinel included) lands inside the code table and
// a vote that is taken back never touches memory outside it.
//
// LDS: code bins [0, 16 N + 6), 32 dwords each (copy = lane mod 32, so the 32
// lanes of an LDS pass always write 32 different banks); the low half of a
// dword counts code 1, the high half code 2.  Then the four block GLCMs with a
// sentinel row and column ((N + 1)^2 words each), which receive the corrected
// pairs and, at the end, the decoded code counts.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "glcm_device.h"
#include "glcm_internal.h"

namespace glcm {
namespace {

constexpr uint32_t kOnes = 0x01010101u;
constexpr uint32_t kWindow = 0xfcfcfcfcu;  // digit bytes outside [0, 3]
constexpr uint32_t kBin = 128u;            // bytes per code bin (32 copies)

// A row as the lower row of the blocks of the row above it.
struct Lower {
  uint32_t s[17];  // kBin * level of chunk pixels 0..15 and of the pixel right of the chunk
  uint32_t l1[4];  // levels + 1 of pixels 0..15, packed bytes
  uint32_t r1[4];  // levels + 1 of pixels 1..16, packed bytes
};

// A row as the upper row (its pixels are the first pixels a).
struct Upper {
  uint32_t w[16];  // kBin * (11 a + b) + lane offset
  uint32_t l[4];   // levels a, packed
  uint32_t r1[4];  // levels + 1 of the right neighbours b, packed
};

// One row as a lane loads it: its 16-pixel chunk and the 4 pixels right of
// the wavefront's last chunk (the same address on every lane; only the last
// lane uses them, the others take their right neighbour's first pixel).
template <typename Pix>
struct BlockRaw {
  uint4 v[sizeof(Pix)];
  uint32_t rh[sizeof(Pix)];
};

// Row y (rows below the last read as the last; the caller replaces them by
// the sentinel).  xc / xc2: the lane's chunk offsets (lane_cols); xn: byte
// offset of the pixel right of the wavefront's chunks, or 0 where that lies
// outside the row (then clipped to the sentinel).
template <typename Pix>
__device__ __forceinline__ void load_block_row(BlockRaw<Pix>& rc, const Geom& g, int y, const LaneCols& o,
                                               uint32_t xn) {
  const char* row = (const char*)g.img + row_offset<Pix>(g, y);
  rc.v[0] = *(const uint4*)(row + o.c);
  if (sizeof(Pix) == 2) rc.v[sizeof(Pix) - 1] = *(const uint4*)(row + o.c2);
  // (xn arrives in a VGPR, so the halo is a vector load: a scalar load would
  // share its wait counter with the LDS atomics)
  if (sizeof(Pix) == 1) {
    rc.rh[0] = *(const uint32_t*)(row + xn);
  } else {
    const uint2 h = *(const uint2*)(row + xn);
    rc.rh[0] = h.x;
    rc.rh[sizeof(Pix) - 1] = h.y;
  }
}

// Levels of a lane's 16 chunk pixels (c) and of the 4 pixels right of the
// chunk (rh), quantized four per dword.  QF: the shift form of q().
template <typename Pix, bool QF>
__device__ __forceinline__ void quant_chunk(uint32_t (&c)[4], uint32_t& rh, const BlockRaw<Pix>& rc,
                                            const BlockArgs& a) {
  if (sizeof(Pix) == 1) {
    if (QF) {
      c[0] = (rc.v[0].x >> a.qfast_shift) & a.qfast_mask; c[1] = (rc.v[0].y >> a.qfast_shift) & a.qfast_mask;
      c[2] = (rc.v[0].z >> a.qfast_shift) & a.qfast_mask; c[3] = (rc.v[0].w >> a.qfast_shift) & a.qfast_mask;
      rh = (rc.rh[0] >> a.qfast_shift) & a.qfast_mask;
    } else {
      c[0] = quant4_u8(rc.v[0].x, a); c[1] = quant4_u8(rc.v[0].y, a);
      c[2] = quant4_u8(rc.v[0].z, a); c[3] = quant4_u8(rc.v[0].w, a);
      rh = quant4_u8(rc.rh[0], a);
    }
  } else {
    c[0] = quant4_u16(rc.v[0].x, rc.v[0].y, a); c[1] = quant4_u16(rc.v[0].z, rc.v[0].w, a);
    c[2] = quant4_u16(rc.v[sizeof(Pix) - 1].x, rc.v[sizeof(Pix) - 1].y, a);
    c[3] = quant4_u16(rc.v[sizeof(Pix) - 1].z, rc.v[sizeof(Pix) - 1].w, a);
    rh = quant4_u16(rc.rh[0], rc.rh[sizeof(Pix) - 1], a);
  }
}

// Raw row -> lower form.  Pixels at or past W (edge strips only) and rows at
// or below H take the sentinel level N; the pixel right of the chunk comes
// from the next lane (the last lane of the wavefront uses the halo it loaded).
template <typename Pix, bool QF>
__device__ __forceinline__ void to_lower(Lower& o, const BlockRaw<Pix>& rc, const BlockArgs& a, int y, int x0,
                                         uint32_t sent4, bool edge) {
  uint32_t c[4], rh;
  quant_chunk<Pix, QF>(c, rh, rc, a);
  if (y >= a.H) {
    c[0] = c[1] = c[2] = c[3] = rh = sent4;
  } else if (edge) {
#pragma unroll
    for (int m = 0; m < 4; ++m) c[m] = clip_dword(c[m], x0 + 4 * m, a.W, sent4);
    rh = clip_dword(rh, x0 + 16, a.W, sent4);
  }
  const uint32_t nx = (uint32_t)__builtin_amdgcn_update_dpp((int)rh, (int)c[0], kDppWaveShl1, 0xf, 0xf, false);
  const uint32_t r[4] = {__builtin_amdgcn_alignbyte(c[1], c[0], 1u), __builtin_amdgcn_alignbyte(c[2], c[1], 1u),
                         __builtin_amdgcn_alignbyte(c[3], c[2], 1u), __builtin_amdgcn_alignbyte(nx, c[3], 1u)};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    o.l1[m] = c[m] + kOnes;
    o.r1[m] = r[m] + kOnes;
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) o.s[t] = __umul24((c[t >> 2] >> ((t & 3) * 8)) & 0xffu, kBin);
  o.s[16] = __umul24(nx & 0xffu, kBin);
}

__device__ __forceinline__ void to_upper(Upper& t, const Lower& lo, uint32_t lane_off) {
#pragma unroll
  for (int x = 0; x < 16; ++x) t.w[x] = __umul24(lo.s[x], 11u) + lo.s[x + 1] + lane_off;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    t.l[m] = lo.l1[m] - kOnes;
    t.r1[m] = lo.r1[m];
  }
}

__device__ __forceinline__ void lds_add(uint32_t addr, uint32_t v) {
  __hip_atomic_fetch_add((lds_word_t*)(size_t)addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_sub(uint32_t addr, uint32_t v) {
  __hip_atomic_fetch_sub((lds_word_t*)(size_t)addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The block GLCMs: FB[g][i][j] in fbc copies (lane mod fbc), without the
// sentinel row and column: a pair with a pixel outside the image goes to the
// lane's own trash word instead.
struct Fb {
  uint32_t base;     // LDS byte address of FB[0][0][0] copy 0
  uint32_t trash;    // LDS byte address of this lane's trash word
  uint32_t lane_c;   // 4 * (lane mod fbc)
  uint32_t stride;   // bytes per bin: 4 * fbc
  uint32_t N;
};

__device__ __forceinline__ void fb_add(const Fb& f, uint32_t g, uint32_t i, uint32_t j) {
  const uint32_t at = f.base + ((g * f.N + i) * f.N + j) * f.stride + f.lane_c;
  lds_add((i < f.N && j < f.N) ? at : f.trash, 1u);
}

// Blocks outside the window.  A lane's dword m of a row (four blocks) with
// any block outside the window is queued for the whole workgroup: the four
// level dwords it needs (a, b + 1, d + 1, e + 1 of its four pixels), the
// mask of its blocks outside the window and the code copy its votes went to.
// After the rows, every thread of the workgroup takes queued dwords and
// corrects their blocks: both code votes taken back, the four pairs counted
// one by one.  A dword that finds the queue full is corrected at once by its
// own lane.
constexpr uint32_t kQueue = 512;  // queued dwords per workgroup

struct Pending {
  uint32_t a, b1, d1, e1;  // packed levels of four blocks: a, b + 1, d + 1, e + 1
  uint32_t out;            // bytes of the blocks outside the window (bits of kWindow)
  uint32_t copy;           // code copy of the votes (lane mod 32)
};

// Corrects the blocks of p marked in p.out.
__device__ __forceinline__ void correct_blocks(const Pending& p, uint32_t code_base, const Fb& f) {
  uint32_t pend = p.out;
  const uint32_t lane_off = code_base + 4u * p.copy;
  while (pend) {
    const uint32_t sh = (uint32_t)__builtin_ctz(pend) & ~7u;
    pend &= ~(0xffu << sh);
    const uint32_t av = (p.a >> sh) & 0xffu, bv = ((p.b1 >> sh) & 0xffu) - 1u, dv = ((p.d1 >> sh) & 0xffu) - 1u,
                   ev = ((p.e1 >> sh) & 0xffu) - 1u;
    lds_sub(kBin * (11u * av + bv + 4u * dv + 5u) + lane_off, 1u);
    lds_sub(kBin * (11u * av + bv + 4u * ev + 5u) + lane_off, 1u << 16);
    fb_add(f, 0u, av, bv);
    fb_add(f, 1u, bv, dv);
    fb_add(f, 2u, av, dv);
    fb_add(f, 3u, av, ev);
  }
}

// One first-pixel row: both codes of all 16 blocks of the lane; the dwords
// with blocks outside the window go to the workgroup's queue.  A row whose
// lower row lies below the image (the last image row) holds only (1,0)
// pairs, counted directly.
__device__ __forceinline__ void block_row(const Upper& t, const Lower& lo, uint32_t copy, uint32_t code_base,
                                          const Fb& f, uint4* queue, uint32_t* qcount, bool last) {
  if (last) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (uint32_t sh = 0; sh < 32; sh += 8)
        fb_add(f, 0u, (t.l[m] >> sh) & 0xffu, ((t.r1[m] >> sh) & 0xffu) - 1u);
    return;
  }
#pragma unroll
  for (int x = 0; x < 16; ++x) {
    lds_add((lo.s[x] << 2) + t.w[x] + 5u * kBin, 1u);            // code 1
    lds_add((lo.s[x + 1] << 2) + t.w[x] + 5u * kBin, 1u << 16);  // code 2
  }
  // Digits b - a + 1, d - a + 1, e - a + 1, four per dword, each biased by
  // 0x40 (X - (a - 0x40404040) = X - a + 0x40 per byte, every byte in
  // [0, 0x80) for N <= 62, no borrow): a block lies in the window iff its
  // three digit bytes are in [0x40, 0x43], i.e. have bit 6 set and bits 2..5
  // clear.
  constexpr uint32_t kBias = 0x40404040u;
  uint32_t bad[4], any = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const uint32_t lb = t.l[m] - kBias;
    const uint32_t db = t.r1[m] - lb, dd = lo.l1[m] - lb, de = lo.r1[m] - lb;
    bad[m] = (~(db & dd & de) & kBias) | ((db | dd | de) & 0x3c3c3c3cu);  // nonzero bytes: outside the window
    any |= bad[m];
  }
  if (__ballot(any != 0u) == 0ull) return;
  // one queue reservation for the row: the dwords m = 0..3 of every lane, in
  // that order
  unsigned long long bal[4];
  uint32_t total = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    bal[m] = __ballot(bad[m] != 0u);
    total += (uint32_t)__popcll(bal[m]);
  }
  uint32_t first = 0;
  if (__lane_id() == 0u)
    first = __hip_atomic_fetch_add(qcount, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  uint32_t slot = (uint32_t)__builtin_amdgcn_readfirstlane((int)first);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    if (bad[m]) {
      const uint32_t s = slot + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal[m] >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)bal[m], 0u));
      const Pending p{t.l[m], t.r1[m], lo.l1[m], lo.r1[m], bad[m], copy};
      if (s < kQueue) {
        queue[2u * s] = make_uint4(p.a, p.b1, p.d1, p.e1);
        queue[2u * s + 1u] = make_uint4(p.out, p.copy, 0u, 0u);
      } else {
        correct_blocks(p, code_base, f);
      }
    }
    slot += (uint32_t)__popcll(bal[m]);
  }
}

// Workgroup -> band: workgroups go to the XCDs round-robin, so workgroup
// 8 s + x takes band x * (nregions / 8) + s, and consecutive bands (which share
// their boundary row) are counted on one XCD.
__device__ __forceinline__ int block_band(int b, int nregions) {
  const int full = nregions / 8 * 8;
  if (b >= full) return b;
  return (b % 8) * (full / 8) + b / 8;
}

// Byte offset of the first pixel right of span `span` (1024 pixels per span),
// or 0 when it lies outside the row.
template <typename Pix>
__device__ __forceinline__ uint32_t next_span_offset(int span, int W) {
  const int x = (span + 1) << 10;
  return x < W ? (uint32_t)x * (uint32_t)sizeof(Pix) : 0u;
}

// A uniform value the compiler must keep (it cannot load it again from the
// kernel arguments later: a late scalar load would wait for the LDS atomics
// in flight, which share its wait counter).
__device__ __forceinline__ uint32_t keep(uint32_t v) {
  uint32_t r;
  asm volatile("s_mov_b32 %0, %1" : "=s"(r) : "s"(v));
  return r;
}
__device__ __forceinline__ unsigned long long keep64(unsigned long long v) {
  unsigned long long r;
  asm volatile("s_mov_b64 %0, %1" : "=s"(r) : "s"(v));
  return r;
}

// A uniform value moved into a vector register (so that loads addressed by it
// stay vector loads).
__device__ __forceinline__ uint32_t vgpr(uint32_t v) {
  uint32_t r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(v));
  return r;
}

template <typename Pix, bool QF>
__global__ __launch_bounds__(1024) void k_vote_blocks(BlockArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  const int region = block_band(blockIdx.x, a.nregions);
  const uint32_t N = a.q.nlev;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nwaves = blockDim.x >> 6;
  const uint32_t base = lds_address(lds);
  const uint32_t lane_off = base + 4u * (uint32_t)(lane & 31);
  const uint32_t fbc = keep((uint32_t)a.fb_copies), nbins = keep(a.nbins);
  const uint32_t fbw0 = nbins * (kBin / 4u);                      // word index of FB
  const uint32_t fbwords = (uint32_t)kBlockGlcms * N * N * fbc;
  const Fb f{base + fbw0 * 4u, base + (fbw0 + fbwords) * 4u + 4u * (uint32_t)lane, 4u * ((uint32_t)lane & (fbc - 1u)),
             4u * fbc, N};
  // the workgroup's queue of dwords with blocks outside the window, and its count
  uint4* queue = (uint4*)(lds + fbw0 + fbwords + 64u);
  uint32_t* qcount = lds + fbw0 + fbwords + 64u + kQueue * 8u;
  const uint32_t copy = (uint32_t)lane & 31u;
  const uint32_t sent4 = N * kOnes;
  const int y0 = a.y_begin + region * a.region_rows;
  const int y1 = min(a.y_end, y0 + a.region_rows);
  const int chunks = (a.W + 15) >> 4;
  const int spans = (chunks + 63) >> 6;
  const int rows = max(0, y1 - y0);
  const int per_span = (rows + a.strip_rows - 1) / a.strip_rows;
  const int nstrips = spans * per_span;
  const Geom geo{a.img, a.stride, a.W, a.H};

  // raw rows in flight: a ring of RING rows, loaded RING - 1 rows ahead
  constexpr int RING = sizeof(Pix) == 1 ? 4 : 2;
  BlockRaw<Pix> raw[RING];
  int strip = wave;
  if (strip < nstrips) {
    const int x0 = (((strip % spans) << 6) + lane) << 4, ya = y0 + (strip / spans) * a.strip_rows;
    const LaneCols cols = lane_cols<Pix>(geo, x0);
    const uint32_t xn = vgpr(next_span_offset<Pix>(strip % spans, a.W));
#pragma unroll
    for (int r = 0; r < RING; ++r) load_block_row<Pix>(raw[r], geo, ya + r, cols, xn);
  }
  zero_lds(lds, fbw0 + fbwords);
  if (threadIdx.x == 0) *qcount = 0u;
  // the kernel arguments read after the rows, held from here on (a first
  // read there would wait for the LDS atomics in flight as well)
  const unsigned long long km[kBlockGlcms] = {keep64(a.kmask[0]), keep64(a.kmask[1]), keep64(a.kmask[2]),
                                              keep64(a.kmask[3])};
  const unsigned long long tmask = keep64(a.tmask);
  uint32_t* const xbuf = (uint32_t*)keep64((unsigned long long)a.xbuf);
  const uint32_t xslots = keep(a.xslots), spread = keep(a.spread);
  const uint32_t words_total = keep(a.words_total), dmagic = keep(a.div_n.magic), dshift = keep(a.div_n.shift);
  asm volatile("" ::"s"(a.qfast), "s"(a.qfast_shift), "s"(a.qfast_mask), "s"(a.q.lo), "s"(a.q.hi), "s"(a.q.nlev),
               "s"(a.q.magic), "s"(a.q.shift), "s"(a.H), "s"(a.W));
  __syncthreads();

  for (; strip < nstrips; strip += nwaves) {
    const int span = strip % spans;
    const int x0 = ((span << 6) + lane) << 4;
    const int ya = y0 + (strip / spans) * a.strip_rows;
    const int yb = min(y1, ya + a.strip_rows);
    const LaneCols cols = lane_cols<Pix>(geo, x0);
    const uint32_t xn = vgpr(next_span_offset<Pix>(span, a.W));
    const bool edge = ((span + 1) << 10) + 4 > a.W;  // chunks or right halos reach column W
    if (strip != wave) {
#pragma unroll
      for (int r = 0; r < RING; ++r) load_block_row<Pix>(raw[r], geo, ya + r, cols, xn);
    }
    Upper up;
    Lower lo;
    to_lower<Pix, QF>(lo, raw[0], a, ya, x0, sent4, edge);
    load_block_row<Pix>(raw[0], geo, ya + RING, cols, xn);
    to_upper(up, lo, lane_off);
    // block row y pairs the upper row y with the lower row y + 1, which sits
    // in ring slot (y + 1 - ya) mod RING; the slot then takes row y + 1 + RING
    for (int y = ya;; y += RING) {
      bool done = false;
#pragma unroll
      for (int r = 1; r <= RING; ++r) {
        if (!done) {
          to_lower<Pix, QF>(lo, raw[r % RING], a, y + r, x0, sent4, edge);
          load_block_row<Pix>(raw[r % RING], geo, y + r + RING, cols, xn);
          block_row(up, lo, copy, base, f, queue, qcount, y + r >= a.H);
          if (y + r >= yb) done = true;
          else to_upper(up, lo, lane_off);
        }
      }
      if (done) break;
    }
  }
  __syncthreads();
  // the queued dwords, one per thread at a time
  const uint32_t queued = min(*qcount, kQueue);
  for (uint32_t e = threadIdx.x; e < queued; e += blockDim.x) {
    const uint4 v = queue[2u * e], w = queue[2u * e + 1u];
    correct_blocks(Pending{v.x, v.y, v.z, v.w, w.x, w.y}, base, f);
  }
  __syncthreads();

  // Merge, step 1: the 32 copies of every code bin, summed in two groups of
  // 16 by two threads (packed: a group holds the votes of half the lanes and
  // the host keeps a band below 2^17 first pixels, so a group's halves stay
  // below 2^16), decoded and added into the block GLCMs (copy job mod fbc).
  for (uint32_t job = threadIdx.x; job < 2u * nbins; job += blockDim.x) {
    const uint32_t bin = job >> 1, half = job & 1u;
    const uint4* units = (const uint4*)(lds + bin * (kBin / 4u)) + 4u * half;
    uint32_t s = 0;
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) {
      const uint4 v = units[(u + bin) & 3u];  // rotated so neighbouring threads read different banks
      s += (v.x + v.y) + (v.z + v.w);
    }
    const uint32_t c1 = s & 0xffffu, c2 = s >> 16;
    const uint32_t at = f.base + 4u * (job & (fbc - 1u));
    if (c1 && bin < 16u * N) {
      const uint32_t av = bin >> 4;
      const uint32_t bv = av + (bin & 3u) - 1u, dv = av + ((bin >> 2) & 3u) - 1u;  // may wrap below 0
      const bool bok = bv < N, dok = dv < N;
      if (bok) lds_add(at + (av * N + bv) * f.stride, c1);
      if (bok && dok) lds_add(at + ((N + bv) * N + dv) * f.stride, c1);
      if (dok) lds_add(at + ((2u * N + av) * N + dv) * f.stride, c1);
    }
    if (c2 && bin < 16u * N) {
      const uint32_t av = bin >> 4, ev = av + ((bin >> 2) & 3u) - 1u;
      if (ev < N) lds_add(at + ((3u * N + av) * N + ev) * f.stride, c2);
    }
  }
  __syncthreads();

  // Merge, step 2: the block GLCMs (all copies) into the per-XCD slice, once
  // per requested offset (transposed for the opposite directions).
  uint32_t xcc;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(xcc));
  // the slice of this XCD (the hardware's XCC_ID, so no two XCDs ever share
  // one) and of this workgroup's group: fewer workgroups adding to one
  // address in L2 at the end of the kernel
  const uint32_t slice = (xcc & (kXcdSlots - 1u)) + xslots * (((uint32_t)blockIdx.x >> 3) & (spread - 1u));
  uint32_t* xs = xbuf + (size_t)slice * words_total;
  const uint32_t NN = N * N;
  const uint32_t* fbw = lds + fbw0;
  for (uint32_t w = threadIdx.x; w < NN; w += blockDim.x) {
    const uint32_t i = divide(w, dmagic, dshift), j = w - i * N;
#pragma unroll
    for (int g = 0; g < kBlockGlcms; ++g) {
      uint32_t v = 0;
      for (uint32_t c = 0; c < fbc; ++c) v += fbw[((uint32_t)g * NN + w) * fbc + ((c + w) & (fbc - 1u))];
      if (v == 0u) continue;
      for (unsigned long long m = km[g]; m; m &= m - 1ull) {
        const uint32_t k = (uint32_t)__builtin_ctzll(m);
        __hip_atomic_fetch_add(xs + (size_t)k * NN + (((tmask >> k) & 1ull) ? j * N + i : w), v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
}

}  // namespace

hipError_t launch_vote_blocks(const BlockArgs& a, int dtype_bytes, int wg, hipStream_t stream,
                              const LaunchTiming& tm) {
  const dim3 grid(a.nregions), block(wg);
  const uint32_t lds = (uint32_t)block_lds_bytes((int)a.q.nlev, a.fb_copies);
  if (dtype_bytes == 1) {
    if (a.qfast)
      hipExtLaunchKernelGGL((k_vote_blocks<uint8_t, true>), grid, block, lds, stream, tm.start, tm.stop, 0u, a);
    else
      hipExtLaunchKernelGGL((k_vote_blocks<uint8_t, false>), grid, block, lds, stream, tm.start, tm.stop, 0u, a);
  } else {
    hipExtLaunchKernelGGL((k_vote_blocks<uint16_t, false>), grid, block, lds, stream, tm.start, tm.stop, 0u, a);
  }
  return hipGetLastError();
}

}  // namespace glcm
