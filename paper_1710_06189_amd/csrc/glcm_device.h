// Device helpers shared by the counting kernels (vote) and the batch kernel:
// the quantizer, row loads of the strip machinery, the address terms and the
// LDS votes.  Included by the .hip files only; everything sits in an
// anonymous namespace, so each file gets its own copy.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "glcm_internal.h"

namespace glcm {
namespace {

// floor(x / d) for x < 2^32 with (magic, shift) from the host (see Quant).
__device__ __forceinline__ uint32_t divide(uint32_t x, uint32_t magic, uint32_t shift) {
  return (uint32_t)(((uint64_t)x + __umulhi(x, magic)) >> shift);
}

// Zeroes n dwords of LDS starting at a 16-byte aligned address.
__device__ __forceinline__ void zero_lds(uint32_t* lds, uint32_t n) {
  uint4* v = (uint4*)lds;
  const uint32_t n4 = n / 4u;
  for (uint32_t i = threadIdx.x; i < n4; i += blockDim.x) v[i] = make_uint4(0u, 0u, 0u, 0u);
  for (uint32_t i = n4 * 4u + threadIdx.x; i < n; i += blockDim.x) lds[i] = 0u;
}

__device__ __forceinline__ uint32_t quantize(uint32_t v, const Quant& q) {
  const uint32_t x = (v - q.lo) * q.nlev;
  const uint32_t lv = (x + __umulhi(x, q.magic)) >> q.shift;
  return v < q.lo ? 0u : (v > q.hi ? q.nlev - 1u : lv);
}

constexpr uint32_t kDppWaveShr1 = 0x138;  // lane l receives lane l-1
constexpr uint32_t kDppWaveShl1 = 0x130;  // lane l receives lane l+1

__device__ __forceinline__ uint32_t pack4(uint32_t l0, uint32_t l1, uint32_t l2, uint32_t l3) {
  return l0 | (l1 << 8) | (l2 << 16) | (l3 << 24);
}

// Four packed 8-bit pixels -> four packed levels (QA: any argument struct with
// the quantizer fields q, qfast, qfast_shift, qfast_mask).
template <class QA>
__device__ __forceinline__ uint32_t quant4_u8(uint32_t raw, const QA& a) {
  if (a.qfast) return (raw >> a.qfast_shift) & a.qfast_mask;
  return pack4(quantize(raw & 0xffu, a.q), quantize((raw >> 8) & 0xffu, a.q), quantize((raw >> 16) & 0xffu, a.q),
               quantize(raw >> 24, a.q));
}

// Four 16-bit pixels (two dwords) -> four packed levels.
template <class QA>
__device__ __forceinline__ uint32_t quant4_u16(uint32_t lo2, uint32_t hi2, const QA& a) {
  if (a.qfast) {
    const uint32_t l = (lo2 >> a.qfast_shift) & a.qfast_mask;  // levels in bits 0..7 and 16..23
    const uint32_t h = (hi2 >> a.qfast_shift) & a.qfast_mask;
    return __builtin_amdgcn_perm(h, l, 0x06040200u);            // bytes l0, l2, h0, h2
  }
  return pack4(quantize(lo2 & 0xffffu, a.q), quantize(lo2 >> 16, a.q), quantize(hi2 & 0xffffu, a.q),
               quantize(hi2 >> 16, a.q));
}

// Byte mask keeping the first n (0..4) bytes of a dword.
__device__ __forceinline__ uint32_t keep_bytes(int n) {
  return n <= 0 ? 0u : (n >= 4 ? 0xffffffffu : ((1u << (8 * n)) - 1u));
}

// Replaces the levels of pixels at or beyond W by the sentinel.
__device__ __forceinline__ uint32_t clip_dword(uint32_t lv, int x, int W, uint32_t sent4) {
  const uint32_t m = keep_bytes(W - x);
  return (lv & m) | (sent4 & ~m);
}

template <typename Pix>
struct RawChunk {
  uint4 v[sizeof(Pix)];  // 16 pixels
  uint32_t lh[sizeof(Pix)], rh[sizeof(Pix)];  // 4-pixel halos of the wave-boundary lanes
};

// ---------------------------------------------------------------------------
// Strip kernel: the fast path for aligned images, N <= 255 and offsets with
// 0 <= dy <= MAXDY and |dx| <= MAXDY (MAXDY <= 2) after canonicalisation.
//
// A wavefront owns a strip: 64 lanes x 16-pixel chunks (1024 columns) and a
// run of consecutive first-pixel rows.  It walks down the strip keeping the
// MAXDY + 1 rows that pairs starting on the current row can reach, each pixel
// already turned into its share of an LDS address, and prefetches the rows
// below while it votes, so each pixel is read from memory once per strip.
//
// LDS layout of a partition (kp GLCMs in kg dword groups): dword
// ((bin * kg + q) * D + g) holds copy g (lane mod D) of bin = a * n1 + b,
// n1 = N + 1 (row and column N catch pixels outside the image), for GLCM q of
// the partition (kg = kp, 32-bit counters) or for GLCMs 2q and 2q+1 in its
// low and high halves (PAIR: kg = kp / 2 rounded up, 16-bit counters, used
// when the host has bounded every count below 2^16).  The byte address splits
// as
//     base(a) + term(b) + 4 D q,   term(v) = v * 4 D kg,   base(a) = 4 g + term(a) * n1,
// so a vote costs one VALU add of a first-pixel base and a second-pixel term;
// 4 D q rides in the offset field of the LDS atomic and the half in the
// added value.  gfx950's LDS serves 32 lanes per pass over 32 banks: with
// D = 32 every lane of a pass writes its own bank whatever the bins; with
// D = 16 lanes l and l + 16 share one (a two-way conflict on every vote).
// ---------------------------------------------------------------------------
template <int NX>
struct TermRow {
  uint32_t s[16 + 2 * NX];  // [NX left halo | 16 chunk pixels | NX right halo]
};

// Loads of one row of a strip lane: its 16-pixel chunk and 4-pixel halo
// blocks on both sides.  Every lane issues the same loads with addresses
// clamped into the image (the row below the last, a chunk past the right
// edge or a halo outside [0, W) read some other pixels of the image, which
// to_terms replaces by the sentinel), so the number of loads in flight is the
// same on every path and the prefetch needs no full wait.  Every access lies
// in a 16-byte block that holds a pixel of the row it addresses.
struct Geom {
  const void* img;  // 16-byte aligned, row pitch a multiple of 16 bytes
  int64_t stride;   // elements
  int W, H;
};

// Byte offsets, within a row, of what a lane loads: its chunk (a chunk that
// starts inside the row), the chunk's second half for 16-bit pixels (only
// when it starts inside the row: the pitch is a multiple of 8 pixels, not
// necessarily of 16) and the halo blocks (only where they start inside the
// row: a lane past the right edge must not read x0 - 4, which on the last
// row is past the image).  Fixed for a lane's whole strip.
struct LaneCols {
  uint32_t c, c2, l, r;
};

// (The address helpers below are also compiled for the host, where a CPU
// test replays every lane's loads against the image bounds.)
template <typename Pix>
__host__ __device__ inline LaneCols lane_cols(const Geom& a, int x0) {
  const int last = (a.W - 1) & ~15;
  const int xc = x0 < last ? x0 : last;
  const int xl = (x0 >= 16 && x0 - 4 < a.W) ? x0 - 4 : xc;
  const int xr = x0 + 16 < a.W ? x0 + 16 : xc;
  const int xc2 = xc + 8 < a.W ? xc + 8 : xc;
  constexpr uint32_t b = sizeof(Pix);
  return {(uint32_t)xc * b, (uint32_t)xc2 * b, (uint32_t)xl * b, (uint32_t)xr * b};
}

// Block-code kernel: byte offset of the first pixel right of span `span`
// (64 lanes of 16 pixels), where the span's last lane reads its right halo,
// or 0 when that pixel lies outside the row.
template <typename Pix>
__host__ __device__ inline uint32_t next_span_offset(int span, int W) {
  const int x = (span + 1) << 10;
  return x < W ? (uint32_t)x * (uint32_t)sizeof(Pix) : 0u;
}

// Byte offset of row y of the image, rows below the last read as the last.
template <typename Pix>
__host__ __device__ inline int64_t row_offset(const Geom& a, int y) {
  return (int64_t)(y < a.H - 1 ? y : a.H - 1) * a.stride * (int64_t)sizeof(Pix);
}

// Rows of an image whose base or pitch is not 16-byte aligned are read as the
// aligned dwords that span a lane's chunk and halos: dword j (from a0) for
// j = j0 .. j0 + 6 B, and only those that hold a byte of the row.
struct UnalignedRow {
  uintptr_t a0;  // the dword boundary at or before the row's first byte
  uint32_t sh;   // bytes the row starts past a0
  int lim;       // dword j holds a byte of the row iff 0 <= j and 4 j < lim
  int j0;        // dword of the left halo's first byte
};

template <typename Pix>
__host__ __device__ inline UnalignedRow unaligned_row(const Geom& g, int y, int x0) {
  constexpr int B = (int)sizeof(Pix);
  const uintptr_t r0 = (uintptr_t)g.img + (uintptr_t)row_offset<Pix>(g, y);
  const uint32_t sh = (uint32_t)(r0 & 3u);
  return {r0 & ~(uintptr_t)3, sh, g.W * B + (int)sh, x0 * B / 4 - B};
}

__host__ __device__ inline bool unaligned_dword_in_row(int j, int lim) { return j >= 0 && 4 * j < lim; }
// Dword j clamped into the row: the nearest dword that holds a byte of it (the
// bytes it brings in for positions outside the row are replaced by the
// sentinel level afterwards, as every pixel outside [0, W) is).
__host__ __device__ inline int unaligned_dword_clamped(int j, int lim) {
  const int last = (lim - 1) >> 2;
  return j < 0 ? 0 : (j > last ? last : j);
}

// Dwords load_row_unaligned reads per row: chunk (4 B), halos (B each side),
// and one more for the byte shift.
template <typename Pix>
constexpr int unaligned_row_dwords() { return 6 * (int)sizeof(Pix) + 1; }

// The histogram's chunk loads (16-byte aligned rows): the block at x0 and, for
// 16-bit pixels, the block at x0 + 8 when it starts inside the row.
__host__ __device__ inline bool chunk_second_block(int x0, int W) { return x0 + 8 < W; }

// Position of a histogram thread in its workgroup's run of chunks: chunk index
// i, row y, column chunk c (x0 = 16 c); step() advances by n chunks (sy rows
// and sc chunks, sc < cpr) with a mixed-radix carry.
struct ChunkPos {
  uint64_t i;
  int y;
  uint32_t c;
  __host__ __device__ inline void step(uint32_t n, uint32_t sy, uint32_t sc, uint32_t cpr) {
    i += n;
    c += sc;
    y += (int)sy;
    if (c >= cpr) {
      c -= cpr;
      ++y;
    }
  }
};

// (In the strip kernel y is the same on every lane, so the row address stays
// in scalar registers and each load is a scalar base plus the lane's offset.)
template <typename Pix>
__device__ __forceinline__ void load_row(RawChunk<Pix>& rc, const Geom& a, int y, const LaneCols& o) {
  const char* row = (const char*)a.img + row_offset<Pix>(a, y);
  rc.v[0] = *(const uint4*)(row + o.c);
  if (sizeof(Pix) == 1) {
    rc.lh[0] = *(const uint32_t*)(row + o.l);
    rc.rh[0] = *(const uint32_t*)(row + o.r);
  } else {
    rc.v[sizeof(Pix) - 1] = *(const uint4*)(row + o.c2);
    const uint2 l = *(const uint2*)(row + o.l), r = *(const uint2*)(row + o.r);
    rc.lh[0] = l.x; rc.lh[sizeof(Pix) - 1] = l.y;
    rc.rh[0] = r.x; rc.rh[sizeof(Pix) - 1] = r.y;
  }
}

// Row loads of an image whose base or row pitch is not 16-byte aligned: the
// lane's 16-pixel chunk and its 4-pixel halos are assembled from the aligned
// dwords that span them (v_alignbyte_b32).  Only dwords that hold a byte of
// the row are read (an index outside the row reads the nearest one), and
// every pixel outside [0, W) is replaced by the sentinel afterwards.
// ALLHALO false: only the wave-boundary lanes read their halo dwords (the
// others take their halo pixels from the neighbouring lanes; theirs read as
// zero).
template <typename Pix, bool ALLHALO = true>
__device__ __forceinline__ void load_row_unaligned(RawChunk<Pix>& rc, const Geom& g, int y, int x0) {
  constexpr int B = (int)sizeof(Pix);
  constexpr int NC = 4 * B;  // chunk dwords (16 pixels)
  constexpr int NH = B;      // halo dwords (4 pixels) on each side
  const UnalignedRow u = unaligned_row<Pix>(g, y, x0);
  const uint32_t* a0 = (const uint32_t*)u.a0;
  const uint32_t sh = u.sh;
  static_assert(NC + 2 * NH + 1 == unaligned_row_dwords<Pix>(), "dwords per unaligned row");
  uint32_t d[NC + 2 * NH + 1];
  const int lane = (int)(threadIdx.x & 63u);
  const bool lneed = ALLHALO || lane == 0, rneed = ALLHALO || lane == 63;
#pragma unroll
  for (int k = 0; k < NC + 2 * NH + 1; ++k) {
    const int j = u.j0 + k;
    d[k] = 0u;
    if (k < NH ? lneed : (k > NH + NC ? rneed : true)) d[k] = a0[unaligned_dword_clamped(j, u.lim)];
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
// 16-byte loads of load_row.
template <typename Pix, bool UNAL>
__device__ __forceinline__ void row_load(RawChunk<Pix>& rc, const Geom& g, int y, int x0, const LaneCols& cols) {
  if constexpr (UNAL)
    load_row_unaligned<Pix, false>(rc, g, y, x0);
  else
    load_row<Pix>(rc, g, y, cols);
}

// Raw row -> per-pixel address terms (level * mb), sentinel level N outside
// the image.  Halo pixels come from the neighbouring lanes; the wave-boundary
// lanes use the halo dwords they loaded themselves.  SEG: a wavefront holds
// several row segments side by side, so a halo pixel outside [0, W) takes the
// sentinel whatever the neighbouring lane holds.  edge (the same on every
// lane): some pixel of the wavefront's chunks or halos lies at or past W;
// otherwise the per-byte clipping is skipped.
template <typename Pix, int NX, bool SEG = false, class QA>
__device__ __forceinline__ void to_terms(TermRow<NX>& r, const RawChunk<Pix>& rc, const QA& a, const Geom& g, int y,
                                         int x0, uint32_t sent4, uint32_t mb, bool edge) {
  uint32_t c[4], lh, rh;
  if (sizeof(Pix) == 1) {
    c[0] = quant4_u8(rc.v[0].x, a); c[1] = quant4_u8(rc.v[0].y, a);
    c[2] = quant4_u8(rc.v[0].z, a); c[3] = quant4_u8(rc.v[0].w, a);
    lh = quant4_u8(rc.lh[0], a);
    rh = quant4_u8(rc.rh[0], a);
  } else {
    c[0] = quant4_u16(rc.v[0].x, rc.v[0].y, a); c[1] = quant4_u16(rc.v[0].z, rc.v[0].w, a);
    c[2] = quant4_u16(rc.v[sizeof(Pix) - 1].x, rc.v[sizeof(Pix) - 1].y, a);
    c[3] = quant4_u16(rc.v[sizeof(Pix) - 1].z, rc.v[sizeof(Pix) - 1].w, a);
    lh = quant4_u16(rc.lh[0], rc.lh[sizeof(Pix) - 1], a);
    rh = quant4_u16(rc.rh[0], rc.rh[sizeof(Pix) - 1], a);
  }
  if (y >= g.H) {
    c[0] = c[1] = c[2] = c[3] = lh = rh = sent4;
  } else if (edge) {
#pragma unroll
    for (int m = 0; m < 4; ++m) c[m] = clip_dword(c[m], x0 + 4 * m, g.W, sent4);
    lh = x0 >= 16 ? clip_dword(lh, x0 - 4, g.W, sent4) : sent4;
    rh = clip_dword(rh, x0 + 16, g.W, sent4);
  } else {
    lh = x0 >= 16 ? lh : sent4;
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) r.s[NX + t] = __umul24((c[t >> 2] >> ((t & 3) * 8)) & 0xffu, mb);
#pragma unroll
  for (int e = 0; e < NX; ++e) {
    // pixel x0 - 1 - e is pixel 15 - e of the lane on the left; x0 + 16 + e is
    // pixel e of the lane on the right (lanes 0 and 63 keep their own value)
    const uint32_t own_l = __umul24((lh >> ((3 - e) * 8)) & 0xffu, mb);
    const uint32_t own_r = __umul24((rh >> (e * 8)) & 0xffu, mb);
    uint32_t left = (uint32_t)__builtin_amdgcn_update_dpp((int)own_l, (int)r.s[NX + 15 - e], kDppWaveShr1, 0xf, 0xf, false);
    uint32_t right = (uint32_t)__builtin_amdgcn_update_dpp((int)own_r, (int)r.s[NX + e], kDppWaveShl1, 0xf, 0xf, false);
    if (SEG) {
      const uint32_t sent = __umul24(sent4 & 0xffu, mb);
      if (x0 - 1 - e < 0) left = sent;
      if (x0 + 16 + e >= g.W) right = sent;
    }
    r.s[NX - 1 - e] = left;
    r.s[NX + 16 + e] = right;
  }
}

// The 16 votes of one first-pixel row for offset (DX, dy): second pixel of
// chunk pixel t is ring pixel NX + t + DX.
// (fa[t] holds the LDS byte address of the first pixel's bin row, LDS base
// included, so the vote is one add; KOFF lands in the instruction's offset.)
typedef __attribute__((address_space(3))) uint32_t lds_word_t;

__device__ __forceinline__ uint32_t lds_address(const uint32_t* p) {
  return (uint32_t)(size_t)(const lds_word_t*)p;
}

// a * b + c on the 24-bit multiplier.  Callers pass a and b below 2^24 (a term
// level * mb and the row pitch); written out because the compiler cannot
// always see that bound and would mask a first.
__device__ __forceinline__ uint32_t mad_u24(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
  return r;
}

template <int NX, int DX, uint32_t KOFF>
__device__ __forceinline__ void vote_row(const uint32_t (&fa)[16], const TermRow<NX>& second, uint32_t inc) {
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const uint32_t addr = fa[t] + second.s[NX + t + DX];
    __hip_atomic_fetch_add((lds_word_t*)(size_t)(addr + KOFF), inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Votes of the partition's GLCM number KI (compile time, so its LDS offset is
// an immediate) for first-pixel row `cur` of the ring.
template <int MAXDY, int D, int KI, int CUR, bool PAIR = false>
__device__ __forceinline__ void vote_glcm(const uint32_t (&fa)[16],
                                          const TermRow<MAXDY> (&ring)[MAXDY + 1], int code, uint32_t one) {
  constexpr int NR = MAXDY + 1, NXS = 2 * MAXDY + 1;
  constexpr uint32_t KOFF = 4u * D * (PAIR ? KI / 2 : KI);
  const uint32_t inc = PAIR && (KI & 1) ? one << 16 : one;
  // code = dy * (2 MAXDY + 1) + dx + MAXDY
  // (the asm marker keeps the compiler from merging the cases into one body
  // that would index the ring through memory)
#define GLCM_STRIP_CASE(DY, DX)                                                                   \
  case (DY) * NXS + (DX) + MAXDY:                                                                 \
    vote_row<MAXDY, (DX), KOFF>(fa, ring[(CUR + (DY)) % NR], inc);                               \
    asm volatile("; strip offset dy=" #DY " dx=" #DX);                                            \
    break;
  switch (code) {
    GLCM_STRIP_CASE(0, 0) GLCM_STRIP_CASE(0, 1) GLCM_STRIP_CASE(1, -1) GLCM_STRIP_CASE(1, 0) GLCM_STRIP_CASE(1, 1)
    default:
      if constexpr (MAXDY >= 2) {
        switch (code) {
          GLCM_STRIP_CASE(0, 2) GLCM_STRIP_CASE(1, -2) GLCM_STRIP_CASE(1, 2)
          GLCM_STRIP_CASE(2, -2) GLCM_STRIP_CASE(2, -1) GLCM_STRIP_CASE(2, 0) GLCM_STRIP_CASE(2, 1) GLCM_STRIP_CASE(2, 2)
          default:
            // reach 3 and 4: the four directions of Eq.(2) only (0, 45, 90
            // and 135 degrees); the host sends other offsets to the slabs
            if constexpr (MAXDY >= 4) {
              switch (code) {
                GLCM_STRIP_CASE(0, 3) GLCM_STRIP_CASE(3, -3) GLCM_STRIP_CASE(3, 0) GLCM_STRIP_CASE(3, 3)
                GLCM_STRIP_CASE(0, 4) GLCM_STRIP_CASE(4, -4) GLCM_STRIP_CASE(4, 0) GLCM_STRIP_CASE(4, 4)
                default: break;
              }
            }
            break;  // the host launches only canonical offsets within reach
        }
      }
      break;
  }
#undef GLCM_STRIP_CASE
}

}  // namespace
}  // namespace glcm
