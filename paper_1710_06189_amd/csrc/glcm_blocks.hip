// Block-code counting kernel for the four d = 1 directions of Eq. (2).
//
// Each first pixel (x, y) and its 2x2 block [a b; d e] hold exactly one pair
// of each of the four d = 1 GLCMs (Eq. (1) at theta = 0, 45, 90, 135 degrees
// with the direction table of Eq. (2)): (a, b), (b, d), (a, d), (a, e).  On
// images whose gray levels vary slowly (the same-address case the copies of
// Section II.A are for) the levels of a block differ by at most one or two,
// so a block is summarised by two codes that carry its four pairs:
//
//   code 1 = 16 a + 4 (b - a + 1) + (d - a + 1) = 11 a + 4 b + d + 5
//   code 2 = 16 a + 4 (b - a + 1) + (e - a + 1) = 11 a + 4 b + e + 5
//
// Both are exact (decodable back to the pairs) when b - a, d - a and e - a lie
// in [-1, 2]; code 1 carries the pairs (a, b), (b, d), (a, d), code 2 the pair
// (a, e).  The two share their upper-row part 11 a + 4 b + 5, and the lower
// row enters with weight one, so each vote address is one addition of two
// per-pixel terms.  Every block votes both codes unconditionally (two LDS
// atomics per first pixel instead of four); a cheap byte-wise test then finds
// the blocks outside the window, whose two votes are taken back and whose four
// pairs are counted one by one.  The codes are linear in the four levels, so
// every level combination (sentinel included) lands inside the code table and
// a vote that is taken back never touches memory outside it.
//
// LDS: code bins [0, 16 N + 6), 32 dwords each (copy = lane mod 32, so the 32
// lanes of an LDS pass always write 32 different banks); the low half of a
// dword counts code 1, the high half code 2.  Then the four block GLCMs (N^2
// words each, in 1, 2 or 4 copies), which receive the corrections and, at the
// end, the decoded code counts; a trash word per lane takes the pairs with a
// level outside [0, N).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "glcm_device.h"
#include "glcm_internal.h"

namespace glcm {
namespace {

constexpr uint32_t kOnes = 0x01010101u;
constexpr uint32_t kBin = 128u;            // bytes per code bin (32 copies)
constexpr int kDppQuadSwap1 = 0xb1;       // DPP quad_perm [1, 0, 3, 2]: lane l receives lane l ^ 1
// Window test bias: a digit X - a + 1 (X = b, d or e) is formed per byte as
// X - (a - kDigitBias) = X - a + 1 + 0x40, so that no byte borrows from the
// next (every byte stays in [0, 0x80) for N <= 62) and a digit in [0, 3]
// reads 0x40..0x43: bit 6 set, bits 2..5 clear.
constexpr uint32_t kDigitBias = 0x41414141u;

// A row as the lower row of the blocks of the row above it.
struct Lower {
  uint32_t s[17];  // kBin * level of chunk pixels 0..15 and of the pixel right of the chunk
  uint32_t l[4];   // levels of pixels 0..15, packed bytes
  uint32_t r[4];   // levels of pixels 1..16, packed bytes
};

// A row as the upper row (its pixels are the first pixels a).
struct Upper {
  uint32_t w[16];  // kBin * (11 a + 4 b + 5) + lane offset
  uint32_t lb[4];  // a - kDigitBias (32-bit difference of the packed levels)
  uint32_t db[4];  // b - lb: the biased digits b - a + 1 + 0x40, one per byte
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

// kBin * byte j of v, in one instruction (the byte selected by SDWA).
template <int J>
__device__ __forceinline__ uint32_t byte_bin(uint32_t v, uint32_t seven) {
  uint32_t r;
  if (J == 0)
    asm("v_lshlrev_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
        : "=v"(r) : "v"(seven), "v"(v));
  else if (J == 1)
    asm("v_lshlrev_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1"
        : "=v"(r) : "v"(seven), "v"(v));
  else if (J == 2)
    asm("v_lshlrev_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2"
        : "=v"(r) : "v"(seven), "v"(v));
  else
    asm("v_lshlrev_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3"
        : "=v"(r) : "v"(seven), "v"(v));
  return r;
}

// Raw row (inside the image) -> lower form.  Pixels at or past W (edge strips
// only) take the sentinel level N; the pixel right of the chunk comes from the
// next lane (the last lane of the wavefront uses the halo it loaded).  seven:
// a register holding 7 (log2 kBin).
template <typename Pix, bool QF>
__device__ __forceinline__ void to_lower(Lower& o, const BlockRaw<Pix>& rc, const BlockArgs& a, int x0,
                                         uint32_t sent4, bool edge, uint32_t seven) {
  static_assert(kBin == 128u, "byte_bin shifts by 7");
  uint32_t c[4], rh;
  quant_chunk<Pix, QF>(c, rh, rc, a);
  if (edge) {
#pragma unroll
    for (int m = 0; m < 4; ++m) c[m] = clip_dword(c[m], x0 + 4 * m, a.W, sent4);
    rh = clip_dword(rh, x0 + 16, a.W, sent4);
  }
  const uint32_t nx = (uint32_t)__builtin_amdgcn_update_dpp((int)rh, (int)c[0], kDppWaveShl1, 0xf, 0xf, false);
  const uint32_t r[4] = {__builtin_amdgcn_alignbyte(c[1], c[0], 1u), __builtin_amdgcn_alignbyte(c[2], c[1], 1u),
                         __builtin_amdgcn_alignbyte(c[3], c[2], 1u), __builtin_amdgcn_alignbyte(nx, c[3], 1u)};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    o.l[m] = c[m];
    o.r[m] = r[m];
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    o.s[4 * m] = byte_bin<0>(c[m], seven);
    o.s[4 * m + 1] = byte_bin<1>(c[m], seven);
    o.s[4 * m + 2] = byte_bin<2>(c[m], seven);
    o.s[4 * m + 3] = byte_bin<3>(c[m], seven);
  }
  o.s[16] = byte_bin<0>(nx, seven);
}

// 11 s + t in one instruction (the compiler would split it into three).
__device__ __forceinline__ uint32_t mad11(uint32_t s, uint32_t t) {
  uint32_t r;
  asm("v_mad_u32_u24 %0, %1, 11, %2" : "=v"(r) : "v"(s), "v"(t));
  return r;
}

// c5 = lane offset + 5 kBin.
__device__ __forceinline__ void to_upper(Upper& t, const Lower& lo, uint32_t c5) {
#pragma unroll
  for (int x = 0; x < 16; ++x) t.w[x] = mad11(lo.s[x], (lo.s[x + 1] << 2) + c5);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    t.lb[m] = lo.l[m] - kDigitBias;
    t.db[m] = lo.r[m] - t.lb[m];
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
  uint32_t sshift;   // log2 of the bytes per bin (4 * fbc)
  uint32_t N;
  // byte offset of FB[g][i][j] copy 0 from base (24-bit products: the
  // indices of a pair that is counted are below N <= 62; others only form a
  // discarded address)
  __device__ __forceinline__ uint32_t at(uint32_t g, uint32_t i, uint32_t j) const {
    return (__umul24(__umul24(g, N) + i, N) + j) << sshift;
  }
};

__device__ __forceinline__ void fb_add(const Fb& f, uint32_t g, uint32_t i, uint32_t j) {
  const uint32_t at = f.base + f.at(g, i, j) + f.lane_c;
  lds_add((i < f.N && j < f.N) ? at : f.trash, 1u);
}


// Blocks outside the window.  A lane's dword m of a row (four blocks) with
// any block outside the window is queued: the four level dwords it needs (a,
// b, d, e of its four blocks), the mask of its blocks outside the window and
// the code copy its votes went to.
// Each wavefront has a queue of its own, so that a reservation is a scalar
// addition (a returning LDS atomic would wait for every vote the wavefront has
// in flight).  After the rows, every thread of the workgroup takes queued
// dwords and corrects their blocks.  A dword that finds its queue full is
// corrected at once by its own lane.
constexpr uint32_t kQueue = 512;                  // queued dwords per workgroup
constexpr uint32_t kQueueWave = kQueue / 16u;     // per wavefront (up to 16 per workgroup)

struct Pending {
  uint32_t a, b, d, e;  // packed levels of four blocks
  uint32_t out;         // nonzero bytes: the blocks outside the window
  uint32_t copy;        // code copy of the votes (lane mod 32)
};

// Corrects the blocks of p marked in p.out: both code votes taken back from
// the lane's code copy, the four pairs counted one by one.
__device__ __forceinline__ void correct_blocks(const Pending& p, uint32_t code_base, const Fb& f) {
  uint32_t pend = p.out;
  const uint32_t lane_off = code_base + 4u * p.copy;
  while (pend) {
    const uint32_t sh = (uint32_t)__builtin_ctz(pend) & ~7u;
    pend &= ~(0xffu << sh);
    const uint32_t av = (p.a >> sh) & 0xffu, bv = (p.b >> sh) & 0xffu, dv = (p.d >> sh) & 0xffu,
                   ev = (p.e >> sh) & 0xffu;
    const uint32_t u = __umul24(av, 11u) + 4u * bv + 5u;
    lds_sub(kBin * (u + dv) + lane_off, 1u);
    lds_sub(kBin * (u + ev) + lane_off, 1u << 16);
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
                                          const Fb& f, uint4* wq, uint32_t& qn, bool last) {
  if (last) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const uint32_t av = t.lb[m] + kDigitBias, bv = t.db[m] + t.lb[m];
#pragma unroll
      for (uint32_t sh = 0; sh < 32; sh += 8) fb_add(f, 0u, (av >> sh) & 0xffu, (bv >> sh) & 0xffu);
    }
    return;
  }
#pragma unroll
  for (int x = 0; x < 16; ++x) {
    lds_add(t.w[x] + lo.s[x], 1u);             // code 1
    lds_add(t.w[x] + lo.s[x + 1], 1u << 16);   // code 2
  }
  // The biased digits of b, d and e (kDigitBias): a block lies in the window
  // iff its three digit bytes have bit 6 set and bits 2..5 clear.
  uint32_t bad[4], any = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const uint32_t db = t.db[m], dd = lo.l[m] - t.lb[m], de = lo.r[m] - t.lb[m];
    bad[m] = (~(db & dd & de) & 0x40404040u) | ((db | dd | de) & 0x3c3c3c3cu);  // nonzero bytes: outside
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
  uint32_t slot = qn;
  qn += total;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    if (bad[m]) {
      const uint32_t s = slot + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal[m] >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)bal[m], 0u));
      const Pending p{t.lb[m] + kDigitBias, t.db[m] + t.lb[m], lo.l[m], lo.r[m], bad[m], copy};
      if (s < kQueueWave) {
        wq[2u * s] = make_uint4(p.a, p.b, p.d, p.e);
        wq[2u * s + 1u] = make_uint4(p.out, p.copy, 0u, 0u);
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

// v, hidden from the compiler's arithmetic simplification.
__device__ __forceinline__ uint32_t opaque(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
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
  const uint32_t fbc = keep((uint32_t)a.fb_copies), nbins = keep(a.nbins);
  const uint32_t fbw0 = nbins * (kBin / 4u);                      // word index of FB
  const uint32_t fbwords = (uint32_t)kBlockGlcms * N * N * fbc;
  const Fb f{base + fbw0 * 4u, base + (fbw0 + fbwords) * 4u + 4u * (uint32_t)lane, 4u * ((uint32_t)lane & (fbc - 1u)),
             2u + (uint32_t)__builtin_ctz(fbc), N};
  // the wavefronts' queues of dwords with blocks outside the window, and their counts
  uint4* queue = (uint4*)(lds + fbw0 + fbwords + 64u);
  uint32_t* qcount = lds + fbw0 + fbwords + 64u + kQueue * 8u;
  uint4* const wq = queue + 2u * kQueueWave * (uint32_t)wave;
  uint32_t qn = 0;
  const uint32_t sent4 = N * kOnes;
  const uint32_t seven = vgpr(7u);
  const uint32_t copy = (uint32_t)lane & 31u;
  // the lane's code copy plus the codes' + 5 (opaque, so that the compiler
  // keeps 4 s + c5 one instruction instead of distributing the shift)
  const uint32_t c5 = opaque(base + 4u * (uint32_t)(lane & 31) + 5u * kBin);
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
  // The first strip's first two rows (its first block row) are requested
  // before the LDS is cleared, the rest of its ring after the barrier: every
  // wavefront's first block row is then among the first bytes the workgroup
  // asks for.
  constexpr int kEarly = 2;
  int strip = wave;
  if (strip < nstrips) {
    const int x0 = (((strip % spans) << 6) + lane) << 4, ya = y0 + (strip / spans) * a.strip_rows;
    const LaneCols cols = lane_cols<Pix>(geo, x0);
    const uint32_t xn = vgpr(next_span_offset<Pix>(strip % spans, a.W));
#pragma unroll
    for (int r = 0; r < kEarly; ++r) load_block_row<Pix>(raw[r], geo, ya + r, cols, xn);
  }
  zero_lds(lds, fbw0 + fbwords);
  // the kernel arguments read after the rows, held from here on (a first
  // read there would wait for the LDS atomics in flight as well)
  const unsigned long long km[kBlockGlcms] = {keep64(a.kmask[0]), keep64(a.kmask[1]), keep64(a.kmask[2]),
                                              keep64(a.kmask[3])};
  const unsigned long long tmask = keep64(a.tmask);
  uint32_t* const xbuf = (uint32_t*)keep64((unsigned long long)a.xbuf);
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
    } else {
#pragma unroll
      for (int r = kEarly; r < RING; ++r) load_block_row<Pix>(raw[r], geo, ya + r, cols, xn);
    }
    // Wavefront priority falls as a strip advances (3 before its first block
    // row, 0 from its third on): the arbiter otherwise favours the oldest
    // wavefronts, and the youngest ones finish their strips long after the
    // rest while the CU is half idle.
    __builtin_amdgcn_s_setprio(3);
    Upper up;
    Lower lo;
    to_lower<Pix, QF>(lo, raw[0], a, x0, sent4, edge, seven);
    if (ya + RING <= yb) load_block_row<Pix>(raw[0], geo, ya + RING, cols, xn);
    to_upper(up, lo, c5);
    // block row y pairs the upper row y with the lower row y + 1, which sits
    // in ring slot (y + 1 - ya) mod RING; the slot then takes row y + 1 + RING
    for (int y = ya;; y += RING) {
      bool done = false;
#pragma unroll
      for (int r = 1; r <= RING; ++r) {
        if (!done) {
          // (the row below the image is no lower row: the last image row
          // holds only (1,0) pairs, counted from its upper form)
          if (y + r < a.H) to_lower<Pix, QF>(lo, raw[r % RING], a, x0, sent4, edge, seven);
          if (y + r + RING <= yb) load_block_row<Pix>(raw[r % RING], geo, y + r + RING, cols, xn);
          block_row(up, lo, copy, base, f, wq, qn, y + r >= a.H);
          if (r == 1) __builtin_amdgcn_s_setprio(2);
          else if (r == 2) __builtin_amdgcn_s_setprio(1);
          else __builtin_amdgcn_s_setprio(0);
          if (y + r >= yb) done = true;
          else to_upper(up, lo, c5);
        }
      }
      if (done) break;
    }
  }
  __builtin_amdgcn_s_setprio(0);
  if (lane == 0) qcount[wave] = min(qn, kQueueWave);
  __syncthreads();
  // the queued dwords, one per thread at a time
  for (uint32_t e = threadIdx.x; e < (uint32_t)nwaves * kQueueWave; e += blockDim.x) {
    if (e % kQueueWave >= qcount[e / kQueueWave]) continue;
    const uint4 v = queue[2u * e], w = queue[2u * e + 1u];
    correct_blocks(Pending{v.x, v.y, v.z, v.w, w.x, w.y}, base, f);
  }
  __syncthreads();

  // Merge, step 1: the 32 copies of every code bin with a level a < N
  // (the codes of a sentinel first pixel are dropped), summed in two groups of
  // 16 by two neighbouring threads (packed: a group holds the votes of half
  // the lanes and the host keeps a band below 2^17 first pixels, so a group's
  // halves stay below 2^16), exchanged between the two, decoded and added into
  // the block GLCMs: the even thread adds the (1,0) and (-1,1) pairs of code 1,
  // the odd one its (0,1) pair and the (1,1) pair of code 2.
  for (uint32_t job = threadIdx.x; job < 32u * N; job += blockDim.x) {
    const uint32_t bin = job >> 1, half = job & 1u;
    const uint4* units = (const uint4*)(lds + bin * (kBin / 4u)) + 4u * half;
    uint32_t s = 0;
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) {
      // rotated by bin / 2: the 16 lanes of a 128-bit LDS pass (8 bins, both
      // halves) then cover all 64 banks
      const uint4 v = units[(u + (bin >> 1)) & 3u];
      s += (v.x + v.y) + (v.z + v.w);
    }
    const uint32_t o = (uint32_t)__builtin_amdgcn_mov_dpp((int)s, kDppQuadSwap1, 0xf, 0xf, true);
    const uint32_t c1 = (s & 0xffffu) + (o & 0xffffu), c2 = (s >> 16) + (o >> 16);
    const uint32_t at = f.base + 4u * (bin & (fbc - 1u));
    const uint32_t av = bin >> 4;
    const uint32_t bv = av + ((bin >> 2) & 3u) - 1u, dv = av + (bin & 3u) - 1u;  // may wrap below 0; dv = ev
    const bool bok = bv < N, dok = dv < N;
    if (half == 0u) {
      if (c1 && bok) lds_add(at + f.at(0u, av, bv), c1);
      if (c1 && bok && dok) lds_add(at + f.at(1u, bv, dv), c1);
    } else {
      if (c1 && dok) lds_add(at + f.at(2u, av, dv), c1);
      if (c2 && dok) lds_add(at + f.at(3u, av, dv), c2);
    }
  }
  __syncthreads();

  // Merge, step 2: the block GLCMs (all copies) into the per-XCD slice, once
  // per requested offset (transposed for the opposite directions).
  uint32_t xcc;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(xcc));
  // the slice of this XCD (the hardware's XCC_ID, so no two XCDs ever share
  // one: every global atomic is performed in the issuing XCD's L2)
  const uint32_t slice = xcc & (kXcdSlots - 1u);
  uint32_t* xs = xbuf + (size_t)slice * words_total;
  const uint32_t NN = N * N;
  const uint32_t* fbw = lds + fbw0;
  for (uint32_t w = threadIdx.x; w < NN; w += blockDim.x) {
    uint32_t v[kBlockGlcms];
    if (fbc == 4u) {
#pragma unroll
      for (int g = 0; g < kBlockGlcms; ++g) {
        const uint4 q = ((const uint4*)fbw)[(uint32_t)g * NN + w];
        v[g] = (q.x + q.y) + (q.z + q.w);
      }
    } else {
#pragma unroll
      for (int g = 0; g < kBlockGlcms; ++g) {
        v[g] = 0;
        for (uint32_t c = 0; c < fbc; ++c) v[g] += fbw[((uint32_t)g * NN + w) * fbc + ((c + w) & (fbc - 1u))];
      }
    }
    uint32_t wt = w;  // (j, i) for the offsets stored transposed
    if (tmask) {
      const uint32_t i = divide(w, dmagic, dshift);
      wt = (w - i * N) * N + i;
    }
#pragma unroll
    for (int g = 0; g < kBlockGlcms; ++g) {
      if (v[g] == 0u) continue;
      for (unsigned long long m = km[g]; m; m &= m - 1ull) {
        const uint32_t k = (uint32_t)__builtin_ctzll(m);
        __hip_atomic_fetch_add(xs + (size_t)k * NN + (((tmask >> k) & 1ull) ? wt : w), v[g], __ATOMIC_RELAXED,
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
