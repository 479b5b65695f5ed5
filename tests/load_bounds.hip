// CPU replay of the kernels' global loads against the image bounds.
//
// Built by tests/test_load_bounds_cpu.py with hipcc and run on the host (no
// GPU): it calls the same __host__ __device__ address helpers the kernels use
// (lane_cols, row_offset, next_span_offset, unaligned_row,
// unaligned_dword_clamped, chunk_second_block, ChunkPos, hist_geometry) for every lane position a
// kernel can take, and checks each access:
//  * 16-byte aligned rows (strip, slab-halo, block-code and batch loads,
//    histogram chunks):
//    the access stays inside one 16-byte block of the row, and that block
//    holds at least one pixel of the row;
//  * rows read as dwords (batch images that are not 16-byte aligned): every
//    dword read holds at least one byte of the row.
// Prints one line per failure (at most 20) and the totals; exits 1 on any.
#include "glcm_device.h"
#include "glcm_hist.h"

#include <cstdio>
#include <cstdlib>

using namespace glcm;

static long g_checked = 0, g_bad = 0;

static void fail(const char* what, int B, int W, int H, long x0, int y, long off, long len) {
  if (g_bad++ < 20)
    std::printf("FAIL %s B=%d W=%d H=%d x0=%ld y=%d off=%ld len=%ld\n", what, B, W, H, x0, y, off, len);
}

// An access of len bytes at byte offset off of an image whose rows start at
// multiples of pitch (bytes, a multiple of 16) and hold W*B bytes of pixels.
static void check_block(const char* what, int B, int W, int H, long pitch, long x0, int y, long off, long len) {
  ++g_checked;
  const int yy = y < H - 1 ? y : H - 1;
  const long row = (long)yy * pitch, blk = off & ~15L;
  const bool ok = off >= row && (off + len - 1) / 16 == off / 16 && blk < row + (long)W * B;
  if (!ok) fail(what, B, W, H, x0, y, off, len);
}

// Strip and batch loads of aligned rows: every lane x0 the kernels can give
// (multiples of 16 up to and including spans * 1024, the x0 of idle batch
// lanes), rows past the image included (they read the last row).
template <typename Pix>
static void aligned_rows(int W, int H, int extra_blocks) {
  constexpr int B = (int)sizeof(Pix);
  const long pitch = ((long)W * B + 15) / 16 * 16 + 16L * extra_blocks;
  const Geom g{nullptr, pitch / B, W, H};
  const int chunks = (W + 15) / 16, spans = (chunks + 63) / 64;
  for (int x0 = 0; x0 <= spans * 1024; x0 += 16) {
    const LaneCols o = lane_cols<Pix>(g, x0);
    for (int y = 0; y < H + 7; ++y) {
      const long row = (long)row_offset<Pix>(g, y);
      check_block("chunk", B, W, H, pitch, x0, y, row + o.c, 16);
      if (B == 2) check_block("chunk2", B, W, H, pitch, x0, y, row + o.c2, 16);
      check_block("left halo", B, W, H, pitch, x0, y, row + o.l, 4 * B);
      check_block("right halo", B, W, H, pitch, x0, y, row + o.r, 4 * B);
    }
  }
}

// Block-code kernel loads (16-byte aligned rows): each lane's chunk (and its
// second half for 16-bit pixels) at lane_cols, and the 4-pixel right halo at
// next_span_offset that the last lane of a 64-lane span reads (the other lanes
// load it too, at the same address), for every span and lane, rows past the
// image included.
template <typename Pix>
static void block_rows(int W, int H, int extra_blocks) {
  constexpr int B = (int)sizeof(Pix);
  const long pitch = ((long)W * B + 15) / 16 * 16 + 16L * extra_blocks;
  const Geom g{nullptr, pitch / B, W, H};
  const int chunks = (W + 15) / 16, spans = (chunks + 63) / 64;
  for (int span = 0; span < spans; ++span) {
    const uint32_t xn = next_span_offset<Pix>(span, W);
    for (int lane = 0; lane < 64; ++lane) {
      const int x0 = ((span << 6) + lane) << 4;
      const LaneCols o = lane_cols<Pix>(g, x0);
      for (int y = 0; y < H + 7; ++y) {
        const long row = (long)row_offset<Pix>(g, y);
        check_block("block chunk", B, W, H, pitch, x0, y, row + o.c, 16);
        if (B == 2) check_block("block chunk2", B, W, H, pitch, x0, y, row + o.c2, 16);
        check_block("block halo", B, W, H, pitch, x0, y, row + xn, 4 * B);
      }
    }
  }
}

// Loads of rows that are not 16-byte aligned (batch, strip and slab kernels):
// base at byte `base`, row pitch W + extra pixels.
template <typename Pix>
static void unaligned_rows(int W, int H, int base, int extra) {
  constexpr int B = (int)sizeof(Pix);
  const long pitch = (long)(W + extra) * B;
  const Geom g{(const void*)(uintptr_t)base, W + extra, W, H};
  const int chunks = (W + 15) / 16, spans = (chunks + 63) / 64;
  for (int x0 = 0; x0 <= spans * 1024; x0 += 16) {
    for (int y = 0; y < H + 7; ++y) {
      const int yy = y < H - 1 ? y : H - 1;
      const long r0 = base + (long)yy * pitch, r1 = r0 + (long)W * B;
      const UnalignedRow u = unaligned_row<Pix>(g, y, x0);
      for (int k = 0; k < unaligned_row_dwords<Pix>(); ++k) {
        const int j = unaligned_dword_clamped(u.j0 + k, u.lim);
        ++g_checked;
        const long a = (long)u.a0 + 4L * j;
        if (!(a < r1 && a + 4 > r0)) fail("unaligned dword", B, W, H, x0, y, a, 4);
        if (unaligned_dword_in_row(u.j0 + k, u.lim) && j != u.j0 + k) fail("clamped in-row dword", B, W, H, x0, y, a, 4);
      }
    }
  }
}

// Histogram: every thread's walk over its workgroup's chunks.
template <typename Pix>
static void histogram(int W, int H, int num_cus) {
  constexpr int B = (int)sizeof(Pix);
  const long pitch = ((long)W * B + 15) / 16 * 16;
  const uint32_t cpr = (uint32_t)((W + 15) / 16);
  const uint64_t chunks = (uint64_t)H * cpr;
  uint64_t per_block = 0;
  const int groups = hist_geometry(chunks, num_cus, &per_block);
  if ((uint64_t)groups * per_block < chunks) fail("hist cover", B, W, H, 0, 0, groups, (long)per_block);
  const uint32_t sy = kHistThreads / cpr, sc = kHistThreads % cpr;
  for (int b = 0; b < groups; ++b) {
    const uint64_t c0 = (uint64_t)b * per_block;
    const uint64_t c1 = c0 + per_block < chunks ? c0 + per_block : chunks;
    for (int t = 0; t < kHistThreads; ++t) {
      const uint64_t first = c0 + (uint64_t)t;
      ChunkPos pos{first, (int)(first / cpr), (uint32_t)(first % cpr)};
      for (; pos.i < c1; pos.step(kHistThreads, sy, sc, cpr)) {
        if (pos.y != (int)(pos.i / cpr) || pos.c != (uint32_t)(pos.i % cpr)) {
          fail("hist position", B, W, H, (long)pos.c * 16, pos.y, (long)pos.i, 0);
          break;
        }
        const int x0 = (int)(pos.c << 4);
        const long row = (long)pos.y * pitch;
        if (pos.y >= H) fail("hist row", B, W, H, x0, pos.y, row, 0);
        check_block("hist chunk", B, W, H, pitch, x0, pos.y, row + (long)x0 * B, 16);
        if (B == 2 && chunk_second_block(x0, W)) check_block("hist chunk2", B, W, H, pitch, x0, pos.y,
                                                            row + (long)(x0 + 8) * 2, 16);
      }
    }
  }
}

int main() {
  for (int W = 1; W <= 2100; ++W) {
    for (int H : {1, 2, 3}) {
      aligned_rows<uint8_t>(W, H, 0);
      aligned_rows<uint16_t>(W, H, 0);
      block_rows<uint8_t>(W, H, 0);
      block_rows<uint16_t>(W, H, 0);
      for (int base : {0, 1, 2, 3, 5, 7, 13}) {
        for (int extra : {0, 1, 3}) {
          unaligned_rows<uint8_t>(W, H, base, extra);
          if (base % 2 == 0) unaligned_rows<uint16_t>(W, H, base, extra);
        }
      }
    }
    if (W % 3 == 0) {
      aligned_rows<uint8_t>(W, 2, 1);
      aligned_rows<uint16_t>(W, 2, 1);
      block_rows<uint8_t>(W, 2, 1);
      block_rows<uint16_t>(W, 2, 1);
    }
    histogram<uint8_t>(W, 1, 256);
    histogram<uint16_t>(W, 2, 256);
  }
  for (int W : {1, 2, 7, 15, 16, 17, 31, 33, 63, 64, 65, 100, 1000, 1025}) {
    for (int H : {700, 4097}) {
      for (int cus : {1, 7, 256}) {
        histogram<uint8_t>(W, H, cus);
        histogram<uint16_t>(W, H, cus);
      }
    }
  }
  std::printf("checked %ld accesses, %ld outside their row\n", g_checked, g_bad);
  return g_bad ? 1 : 0;
}
