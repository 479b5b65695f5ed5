// gfx950 kernels for gray-level co-occurrence matrices (Eq. (1)) and Haralick
// statistics.
//
// Counting follows the replica idea of Scheme 2 (Section II.A): every
// workgroup keeps R copies of its GLCM words in LDS and each thread votes into
// copy (thread index mod R), which divides same-address atomic collisions on
// smooth images by R.  The copies are interleaved word by word (counter of
// word w, copy r at LDS index w*R + r) so lanes voting the same bin hit
// different banks.  The merge of all copies into one result (the final sum in
// Section II.A) takes two steps: every workgroup writes its band's counts to
// a partial buffer, and a second kernel sums the partials into `out`.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "glcm_device.h"
#include "glcm_internal.h"

namespace glcm {
namespace {

// ---------------------------------------------------------------------------
// Merge of the LDS copies (the final sum of Section II.A), in two steps that
// need no synchronisation between workgroups inside a kernel:
//
//  * merge = per-XCD accumulation: every workgroup adds its non-zero counts to
//    the accumulation slice of the XCD it runs on (hardware register XCC_ID),
//    with workgroup-scope atomics, which execute in that XCD's L2 (all CUs of
//    an XCD share it, and no other XCD touches the slice).  The kernel
//    boundary writes the L2s back; k_finish sums the slices into `out` and
//    clears them for the next launch.
//  * merge = band partials: every workgroup stores its counts to its own row
//    of a partial buffer and k_reduce sums the rows.
//
// The LDS matrices may be padded: word (k, i, j) of the partition (k counted
// from the partition's first GLCM) sits at copy-block k * nn1 + i * n1 + j,
// each block holding R copies (R / 2 dwords with 16-bit counters).
// ---------------------------------------------------------------------------
__device__ void store_partial(const VoteArgs& a, const uint32_t* lds, uint32_t pbase, uint32_t pwords, int region,
                              uint32_t n1, uint32_t nn1, bool c16) {
  __syncthreads();
  const uint32_t R = 1u << a.log2R;
  const uint32_t D = c16 ? R / 2u : R;  // dwords per bin (a multiple of 4 when D >= 4)
  const uint32_t N = a.q.nlev, NN = N * N;
  uint32_t* dst = a.partials + (size_t)region * a.words_total + pbase;
  for (uint32_t w = threadIdx.x; w < pwords; w += blockDim.x) {
    uint32_t src = w;
    if (n1 != N) {
      const uint32_t k = divide(w, a.div_nn.magic, a.div_nn.shift), rem = w - k * NN;
      const uint32_t i = divide(rem, a.div_n.magic, a.div_n.shift), j = rem - i * N;
      src = k * nn1 + i * n1 + j;
    }
    const uint32_t* c = lds + src * D;
    uint32_t s = 0;
    if (D >= 4) {
      for (uint32_t d = 0; d < D; d += 4) {
        const uint4 v = *(const uint4*)(c + d);
        s += c16 ? (v.x & 0xffffu) + (v.x >> 16) + (v.y & 0xffffu) + (v.y >> 16) + (v.z & 0xffffu) + (v.z >> 16) +
                       (v.w & 0xffffu) + (v.w >> 16)
                 : (v.x + v.y) + (v.z + v.w);
      }
    } else if (c16) {
      for (uint32_t d = 0; d < D; ++d) s += (c[d] & 0xffffu) + (c[d] >> 16);
    } else {
      for (uint32_t d = 0; d < D; ++d) s += c[d];
    }
    if (a.xbuf) {
      if (s) {
        uint32_t xcc;
        asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(xcc));
        __hip_atomic_fetch_add(a.xbuf + (size_t)(xcc & (kXcdSlots - 1u)) * a.words_total + pbase + w, s,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    } else {
      dst[w] = s;
    }
  }
}

// Merge of the generic kernel's 16-bit layout (word w in half w & 1 of dword
// w >> 1, one copy): into the XCD slice or the band partial.
__device__ void store_partial_bin_pairs(const VoteArgs& a, const uint32_t* lds, uint32_t pbase, uint32_t pwords,
                                        int region) {
  __syncthreads();
  uint32_t* dst = a.partials + (size_t)region * a.words_total + pbase;
  uint32_t xcc = 0;
  if (a.xbuf) asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(xcc));
  uint32_t* xs = a.xbuf + (size_t)(xcc & (kXcdSlots - 1u)) * a.words_total + pbase;
  for (uint32_t m = threadIdx.x; 2u * m < pwords; m += blockDim.x) {
    const uint32_t d = lds[m];
#pragma unroll
    for (uint32_t h = 0; h < 2; ++h) {
      const uint32_t w = 2u * m + h;
      if (w >= pwords) break;
      const uint32_t s = (d >> (16u * h)) & 0xffffu;
      if (a.xbuf) {
        if (s) __hip_atomic_fetch_add(xs + w, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      } else {
        dst[w] = s;
      }
    }
  }
}

// out[w] = (accumulate ? out[w] : 0) + sum of the first nslots accumulation
// slices (the others stay zero); clears them.
__global__ __launch_bounds__(256) void k_finish(uint32_t* xbuf, uint32_t* out, uint32_t M, uint32_t nslots,
                                                int accumulate) {
  const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= M) return;
  uint32_t s = accumulate ? out[w] : 0u;
  for (uint32_t x0 = 0; x0 < nslots; x0 += kXcdSlots) {
    uint32_t v[kXcdSlots];
#pragma unroll
    for (uint32_t x = 0; x < kXcdSlots; ++x) v[x] = x0 + x < nslots ? xbuf[(size_t)(x0 + x) * M + w] : 0u;
#pragma unroll
    for (uint32_t x = 0; x < kXcdSlots; ++x) {
      s += v[x];
      if (x0 + x < nslots) xbuf[(size_t)(x0 + x) * M + w] = 0u;
    }
  }
  out[w] = s;
}

// p[w] = 0 for w < n (a kernel rather than a memset node, so that a caller
// may capture it into a HIP graph).
__global__ __launch_bounds__(256) void k_zero(uint32_t* p, uint64_t n) {
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < n; w += (uint64_t)gridDim.x * blockDim.x)
    p[w] = 0u;
}

// Each workgroup records the XCC_ID of the XCD it runs on.
__global__ __launch_bounds__(64) void k_xcc_probe(uint32_t* ids) {
  uint32_t xcc;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(xcc));
  if (threadIdx.x == 0) ids[blockIdx.x] = xcc;
}

// out[w] (+)= sum over bands of partials[band][w].  Each workgroup owns
// kReduceQuads quads of words; its threads are kReduceQuads x kReduceGroups,
// group g loading bands g, g + kReduceGroups, ... 16 bytes at a time (all
// loads of a thread in flight together), and the groups meet in an LDS tree.
constexpr int kReduceQuads = 4, kReduceGroups = 256;

__global__ __launch_bounds__(kReduceQuads * kReduceGroups) void k_reduce(const uint32_t* partials, uint32_t* out,
                                                                       uint32_t M, int nbands, int accumulate) {
  __shared__ uint4 part[kReduceGroups][kReduceQuads];
  const int q = threadIdx.x % kReduceQuads, g = threadIdx.x / kReduceQuads;
  const uint32_t w = (blockIdx.x * kReduceQuads + q) * 4u;  // first word of this thread's quad
  uint4 acc = make_uint4(0u, 0u, 0u, 0u);
  if (w < M) {
    const bool whole = w + 4 <= M && (M % 4u) == 0;
    for (int b0 = g; b0 < nbands; b0 += 4 * kReduceGroups) {
      uint4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {  // independent loads in flight
        const int b = b0 + u * kReduceGroups;
        v[u] = make_uint4(0u, 0u, 0u, 0u);
        if (b < nbands) {
          const uint32_t* p = partials + (size_t)b * M + w;
          if (whole) {
            v[u] = *(const uint4*)p;
          } else {
            v[u].x = p[0];
            if (w + 1 < M) v[u].y = p[1];
            if (w + 2 < M) v[u].z = p[2];
            if (w + 3 < M) v[u].w = p[3];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc.x += v[u].x; acc.y += v[u].y; acc.z += v[u].z; acc.w += v[u].w;
      }
    }
  }
  part[g][q] = acc;
  __syncthreads();
  for (int half = kReduceGroups / 2; half > 0; half >>= 1) {
    if (g < half) {
      const uint4 o = part[g + half][q];
      uint4 t = part[g][q];
      t.x += o.x; t.y += o.y; t.z += o.z; t.w += o.w;
      part[g][q] = t;
    }
    __syncthreads();
  }
  if (g == 0 && w < M) {
    const uint4 t = part[0][q];
    const uint32_t r[4] = {t.x, t.y, t.z, t.w};
    for (int e = 0; e < 4 && w + e < M; ++e) out[w + e] = (accumulate ? out[w + e] : 0u) + r[e];
  }
}

// Workgroup -> (band, partition).  Workgroups go to the XCDs round-robin
// (workgroup b runs on XCD b mod 8), and every partition of a band reads the
// band's rows: keeping the partitions of one band on one XCD lets its L2
// serve the second read instead of HBM.  Workgroup b = 8 s + x takes
// partition s mod P of band 8 (s / P) + x for the first 8 floor(nregions / 8)
// bands; the remaining bands take the plain order (a bijection either way).
constexpr int kXcds = 8;
__device__ __forceinline__ int2 band_of_block(int b, int P, int nregions) {
  const int full = nregions / kXcds * kXcds;
  if (P > 1 && b < full * P) {
    const int x = b % kXcds, s = b / kXcds;
    return make_int2(s / P * kXcds + x, s % P);
  }
  const int r = b - full * P;
  return make_int2(full + r / P, r % P);
}

// ---------------------------------------------------------------------------
// Generic counting kernel: any alignment, stride and offsets.  One thread per
// first pixel, loads through the cache, votes into the LDS copies of the
// partition this workgroup owns.
// ---------------------------------------------------------------------------
// A uniform value the compiler must keep in a register: reading it again from
// the kernel arguments inside the loop would be a scalar load, whose wait
// also waits for every LDS vote in flight (they share one counter).
__device__ __forceinline__ int keep_s(int v) {
  int r;
  asm volatile("s_mov_b32 %0, %1" : "=s"(r) : "s"(v));
  return r;
}

// The loop of a partition whose bins belong to NK consecutive offsets k0 ..
// k0 + NK - 1 (NK <= 4, the usual case: a partition holds about one GLCM of
// the large N that need partitions).  Each thread takes 4 pixels of a row (2
// for NK > 2) at once and issues all their first- and second-pixel loads
// before any vote,
// with the offsets held in registers; a pair whose bin lies outside the
// partition (or whose second pixel lies outside the image) votes nowhere.
template <typename Pix, int NK>
__device__ __forceinline__ void generic_votes(const VoteArgs& a, uint32_t* lds, int k0, uint32_t pbase,
                                              uint32_t pwords, uint32_t r, int y0, int y1, int tw, int tr, int tx,
                                              int ty) {
  constexpr int U = NK <= 2 ? 4 : 2;  // (more would spill at 1024 threads)
  const Pix* img = (const Pix*)a.img;
  const uint32_t N = a.q.nlev, NN = N * N;
  int dx[NK], dy[NK];
  int64_t off[NK];
  uint32_t wbase[NK];  // k N^2 - pbase (wraps: a bin below the partition reads as >= pwords)
#pragma unroll
  for (int j = 0; j < NK; ++j) {
    dx[j] = keep_s(a.dx[k0 + j]);
    dy[j] = keep_s(a.dy[k0 + j]);
    off[j] = (int64_t)dy[j] * a.stride + dx[j];
    wbase[j] = (uint32_t)(k0 + j) * NN - pbase;
  }
  const int W = keep_s(a.W), H = keep_s(a.H);
  const bool qf = a.qfast != 0;
  const uint32_t qs = (uint32_t)keep_s((int)a.qfast_shift);
  const Quant q{(uint32_t)keep_s((int)a.q.lo), (uint32_t)keep_s((int)a.q.hi), N, (uint32_t)keep_s((int)a.q.magic),
                (uint32_t)keep_s((int)a.q.shift)};
  const bool c16 = a.c16 != 0;
  const int log2R = keep_s(a.log2R);
  for (int y = y0 + ty; y < y1; y += tr) {
    const Pix* row = img + (int64_t)y * a.stride;
    for (int x = tx; x < W; x += U * tw) {
      uint32_t v1[U], v2[U][NK];
      bool ok[U][NK];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int xu = x + u * tw;
        const bool in = xu < W;
        v1[u] = in ? (uint32_t)row[xu] : 0u;
#pragma unroll
        for (int j = 0; j < NK; ++j) {
          ok[u][j] = in && (unsigned)(xu + dx[j]) < (unsigned)W && (unsigned)(y + dy[j]) < (unsigned)H;
          v2[u][j] = ok[u][j] ? (uint32_t)row[xu + off[j]] : 0u;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t av = qf ? v1[u] >> qs : quantize(v1[u], q);
#pragma unroll
        for (int j = 0; j < NK; ++j) {
          const uint32_t w = wbase[j] + av * N + (qf ? v2[u][j] >> qs : quantize(v2[u][j], q));
          if (ok[u][j] && w < pwords) {
            if (c16)
              __hip_atomic_fetch_add(&lds[w >> 1], 1u << ((w & 1u) << 4), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
            else
              __hip_atomic_fetch_add(&lds[(w << log2R) + r], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
      }
    }
  }
}

template <typename Pix>
__global__ __launch_bounds__(1024) void k_vote_generic(VoteArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  const int2 rp = band_of_block(blockIdx.x, a.P, a.nregions);
  const int region = rp.x, part = rp.y;
  const uint32_t pbase = (uint32_t)part * a.part_words;
  const uint32_t pwords = min(a.part_words, a.words_total - pbase);
  // c16: 16-bit counters, words 2m and 2m + 1 in the low and high halves of
  // dword m (one copy); the host keeps every band below 2^16 first pixels
  zero_lds(lds, a.c16 ? (pwords + 1u) >> 1 : pwords << a.log2R);
  __syncthreads();

  const Pix* img = (const Pix*)a.img;
  const uint32_t r = threadIdx.x & ((1u << a.log2R) - 1u);
  const uint32_t N = a.q.nlev, NN = N * N;
  const int y0 = a.y_begin + region * a.region_rows;
  const int y1 = min(a.y_end, y0 + a.region_rows);
  // GLCMs [k0, k1) overlap this partition's words [pbase, pbase + pwords);
  // within them, a first pixel of level i can only vote if its row of bins
  // (k, i, *) overlaps the range too, checked before the second pixel is read
  const int k0 = (int)(pbase / NN), k1 = min(a.K, (int)((pbase + pwords + NN - 1) / NN));
  // threads as (rows at once) x (columns at once): tw columns, a power of
  // two from 64 up to blockDim (also a power of two, so tw divides it), and
  // blockDim / tw rows; no division inside the loops
  int tw = 64;
  while (tw < a.W && tw < (int)blockDim.x) tw *= 2;
  const int tr = (int)blockDim.x / tw, tx = (int)threadIdx.x & (tw - 1), ty = (int)threadIdx.x / tw;
  const int nk = k1 - k0;
  if (nk == 1) generic_votes<Pix, 1>(a, lds, k0, pbase, pwords, r, y0, y1, tw, tr, tx, ty);
  else if (nk == 2) generic_votes<Pix, 2>(a, lds, k0, pbase, pwords, r, y0, y1, tw, tr, tx, ty);
  else if (nk == 3) generic_votes<Pix, 3>(a, lds, k0, pbase, pwords, r, y0, y1, tw, tr, tx, ty);
  else if (nk == 4) generic_votes<Pix, 4>(a, lds, k0, pbase, pwords, r, y0, y1, tw, tr, tx, ty);
  else
  for (int y = y0 + ty; y < y1; y += tr) {
    for (int x = tx; x < a.W; x += tw) {
      const uint32_t v = img[(int64_t)y * a.stride + x];
      const uint32_t av = a.qfast ? v >> a.qfast_shift : quantize(v, a.q);
      for (int k = k0; k < k1; ++k) {
        const uint32_t row = (uint32_t)k * NN + av * N;  // first word of bins (k, av, *)
        if (a.P > 1 && (row + N <= pbase || row >= pbase + pwords)) continue;
        const int x2 = x + a.dx[k], y2 = y + a.dy[k];
        if ((unsigned)x2 >= (unsigned)a.W || (unsigned)y2 >= (unsigned)a.H) continue;
        const uint32_t v2 = img[(int64_t)y2 * a.stride + x2];
        const uint32_t w = row + (a.qfast ? v2 >> a.qfast_shift : quantize(v2, a.q)) - pbase;
        if (w < pwords) {
          if (a.c16)
            __hip_atomic_fetch_add(&lds[w >> 1], 1u << ((w & 1u) << 4), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
          else
            __hip_atomic_fetch_add(&lds[(w << a.log2R) + r], 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }
  }
  if (a.c16)
    store_partial_bin_pairs(a, lds, pbase, pwords, region);
  else
    store_partial(a, lds, pbase, pwords, region, a.q.nlev, a.q.nlev * a.q.nlev, false);
}

// ---------------------------------------------------------------------------
// Global-atomic counting (the one-thread-per-pixel, global-memory-atomics
// scheme of Section I.B): no LDS, `out` must be zeroed beforehand.  Used as an
// ablation and for N too large for LDS partitions to pay off.
// ---------------------------------------------------------------------------
template <typename Pix>
__global__ __launch_bounds__(256) void k_vote_global(VoteArgs a) {
  const Pix* img = (const Pix*)a.img;
  const uint32_t N = a.q.nlev, NN = N * N;
  const uint64_t n = (uint64_t)(a.y_end - a.y_begin) * (uint64_t)a.W;
  for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (uint64_t)gridDim.x * blockDim.x) {
    const int y = a.y_begin + (int)(idx / (uint64_t)a.W);
    const int x = (int)(idx % (uint64_t)a.W);
    const uint32_t av = quantize(img[(int64_t)y * a.stride + x], a.q);
    for (int k = 0; k < a.K; ++k) {
      const int x2 = x + a.dx[k], y2 = y + a.dy[k];
      if ((unsigned)x2 >= (unsigned)a.W || (unsigned)y2 >= (unsigned)a.H) continue;
      const uint32_t bv = quantize(img[(int64_t)y2 * a.stride + x2], a.q);
      __hip_atomic_fetch_add(&a.out[(size_t)k * NN + av * N + bv], 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// L2-slice counting for large N, where LDS bin partitions would re-read the
// image many times: no LDS copies.  Each pair is added, with a
// workgroup-scope atomic, to the accumulation slice of the XCD the workgroup
// runs on (the atomic executes in that XCD's L2, and no other XCD touches the
// slice); k_finish then sums the slices into `out`.  A wavefront walks 64
// consecutive columns down a run of region_rows rows, so first-pixel loads
// are coalesced and second pixels mostly hit the caches.  Any alignment.
// ---------------------------------------------------------------------------
template <typename Pix>
__global__ __launch_bounds__(256) void k_vote_l2(VoteArgs a) {
  uint32_t xcc;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(xcc));
  uint32_t* xs = a.xbuf + (size_t)(xcc & (kXcdSlots - 1u)) * a.words_total;
  const Pix* img = (const Pix*)a.img;
  const uint32_t N = a.q.nlev, NN = N * N;
  const int cols = (a.W + 63) >> 6;
  const int runs = (a.y_end - a.y_begin + a.region_rows - 1) / a.region_rows;
  const int lane = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  const int tasks = cols * runs;
  for (int task = __builtin_amdgcn_readfirstlane((int)blockIdx.x * nw + (int)(threadIdx.x >> 6)); task < tasks;
       task += (int)gridDim.x * nw) {
    const int x = (task % cols) * 64 + lane;
    const int ya = a.y_begin + (task / cols) * a.region_rows;
    const int yb = min(a.y_end, ya + a.region_rows);
    if (x >= a.W) continue;
    for (int y = ya; y < yb; ++y) {
      const uint32_t v = img[(int64_t)y * a.stride + x];
      const uint32_t base = (a.qfast ? v >> a.qfast_shift : quantize(v, a.q)) * N;
      for (int k = 0; k < a.K; ++k) {
        const int x2 = x + a.dx[k], y2 = y + a.dy[k];
        if ((unsigned)x2 >= (unsigned)a.W || (unsigned)y2 >= (unsigned)a.H) continue;
        const uint32_t v2 = img[(int64_t)y2 * a.stride + x2];
        const uint32_t bv = a.qfast ? v2 >> a.qfast_shift : quantize(v2, a.q);
        __hip_atomic_fetch_add(xs + (size_t)k * NN + base + bv, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Row kernel: the fast path for aligned images (base and row pitch multiples
// of 16 bytes), N <= 255, offsets with |dx| <= 4 and 0 <= dy <= MAXDY <= 4 after
// canonicalisation (an offset with dy < 0 is counted as its opposite and voted
// transposed).  Each lane owns a 16-pixel column chunk; a wavefront covers 64
// chunks (1024 pixels) of RPW consecutive rows (a slab).  All RPW + MAXDY rows
// of the slab are loaded at once, quantized into bytes, and the horizontal
// neighbours come from the adjacent lanes through DPP wave shifts, so each
// pixel is read from memory once per slab.
//
// Pixels outside the image (x < 0, x >= W, or rows >= H) get the sentinel
// level N.  The LDS copy of each GLCM is (N+1) x (N+1); votes touching a
// sentinel land in row or column N and are dropped by the merge, so the vote
// loop carries no bounds checks at all.
// ---------------------------------------------------------------------------
struct Ring {
  uint32_t w[6];  // [left halo (4 px) | 16 px chunk | right halo (4 px)], one level per byte
};

// UNAL: a row of an image whose base or pitch is not 16-byte aligned, read in
// place as the dwords that hold it (load_row_unaligned; only the wave-boundary
// lanes read halo dwords, the only ones finish_row uses).
template <typename Pix, bool UNAL>
__device__ __forceinline__ void issue_row(RawChunk<Pix>& rc, const VoteArgs& a, int y, int x0, int lane) {
#pragma unroll
  for (int h = 0; h < (int)sizeof(Pix); ++h) {
    rc.v[h] = make_uint4(0u, 0u, 0u, 0u);
    rc.lh[h] = 0u;
    rc.rh[h] = 0u;
  }
  if (y >= a.H) return;
  if constexpr (UNAL) {
    load_row_unaligned<Pix, false>(rc, Geom{a.img, a.stride, a.W, a.H}, y, x0);
    return;
  }
  const Pix* row = (const Pix*)a.img + (int64_t)y * a.stride;
  if (x0 < a.W) rc.v[0] = *(const uint4*)(row + x0);
  if (sizeof(Pix) == 2 && x0 + 8 < a.W) rc.v[sizeof(Pix) - 1] = *(const uint4*)(row + x0 + 8);
  if (lane == 0 && x0 >= 16 && x0 - 4 < a.W) {
    if (sizeof(Pix) == 1) rc.lh[0] = *(const uint32_t*)(row + x0 - 4);
    else { const uint2 t = *(const uint2*)(row + x0 - 4); rc.lh[0] = t.x; rc.lh[sizeof(Pix) - 1] = t.y; }
  }
  if (lane == 63 && x0 + 16 < a.W) {
    if (sizeof(Pix) == 1) rc.rh[0] = *(const uint32_t*)(row + x0 + 16);
    else { const uint2 t = *(const uint2*)(row + x0 + 16); rc.rh[0] = t.x; rc.rh[sizeof(Pix) - 1] = t.y; }
  }
}

template <typename Pix>
__device__ __forceinline__ void finish_row(Ring& rg, const RawChunk<Pix>& rc, const VoteArgs& a, int y, int x0,
                                           int lane, uint32_t sent4) {
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
  if (y >= a.H) {
    c[0] = c[1] = c[2] = c[3] = sent4;
  } else {
#pragma unroll
    for (int m = 0; m < 4; ++m) c[m] = clip_dword(c[m], x0 + 4 * m, a.W, sent4);
  }
  const uint32_t from_left = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c[3], kDppWaveShr1, 0xf, 0xf, false);
  const uint32_t from_right = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c[0], kDppWaveShl1, 0xf, 0xf, false);
  // wave-boundary lanes take the halo they loaded themselves (sentinel outside the image)
  lh = (y < a.H && x0 >= 16) ? clip_dword(lh, x0 - 4, a.W, sent4) : sent4;
  rh = (y < a.H) ? clip_dword(rh, x0 + 16, a.W, sent4) : sent4;
  rg.w[0] = lane == 0 ? lh : from_left;
  rg.w[1] = c[0]; rg.w[2] = c[1]; rg.w[3] = c[2]; rg.w[4] = c[3];
  rg.w[5] = lane == 63 ? rh : from_right;
}

// Second-pixel levels of the 16 chunk pixels for horizontal shift dx in [-4, 4]:
// bytes 4+dx .. 19+dx of the 24-byte ring row, as a funnel shift of 64-bit
// values (no indexed register access, which the compiler would spill).
__device__ __forceinline__ void window(const Ring& rg, int dx, uint32_t out[4]) {
  const uint64_t r0 = (uint64_t)rg.w[0] | ((uint64_t)rg.w[1] << 32);
  const uint64_t r1 = (uint64_t)rg.w[2] | ((uint64_t)rg.w[3] << 32);
  const uint64_t r2 = (uint64_t)rg.w[4] | ((uint64_t)rg.w[5] << 32);
  const uint32_t sh = (uint32_t)(4 + dx) * 8u;  // 0 .. 64
  uint64_t lo, hi;
  if (sh == 0) {
    lo = r0; hi = r1;
  } else if (sh == 64) {
    lo = r1; hi = r2;
  } else {
    lo = (r0 >> sh) | (r1 << (64u - sh));
    hi = (r1 >> sh) | (r2 << (64u - sh));
  }
  out[0] = (uint32_t)lo; out[1] = (uint32_t)(lo >> 32);
  out[2] = (uint32_t)hi; out[3] = (uint32_t)(hi >> 32);
}

// Votes of one offset whose canonical dy is S, for the RPW first-pixel rows of
// the slab: LDS byte address = C + a * MA + b * MB.
template <int S, int RPW, int NROWS>
__device__ __forceinline__ void vote_offset(uint32_t* lds, const Ring (&rows)[NROWS], int nrows_first, int dx,
                                            uint32_t C, uint32_t MA, uint32_t MB, uint32_t inc) {
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    if (i < nrows_first) {
      uint32_t b[4];
      window(rows[i + S], dx, b);
      const uint32_t f[4] = {rows[i].w[1], rows[i].w[2], rows[i].w[3], rows[i].w[4]};
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const uint32_t av = (f[t >> 2] >> ((t & 3) * 8)) & 0xffu;
        const uint32_t bv = (b[t >> 2] >> ((t & 3) * 8)) & 0xffu;
        const uint32_t addr = C + __umul24(av, MA) + __umul24(bv, MB);  // full-rate 24-bit multiplies
        __hip_atomic_fetch_add((uint32_t*)((char*)lds + addr), inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
}

template <typename Pix, int MAXDY, int RPW, bool UNAL>
__global__ __launch_bounds__(rows_max_threads(sizeof(Pix), MAXDY, UNAL)) void k_vote_rows(VoteArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  const int2 rp = band_of_block(blockIdx.x, a.P, a.nregions);
  const int region = rp.x, part = rp.y;
  const uint32_t N = a.q.nlev, N1 = a.pitch, NN = N * N, NN1 = N1 * N1;
  // Partitions of the row kernel are groups of whole GLCMs (offsets).
  const uint32_t pbase = (uint32_t)part * a.part_words;
  const uint32_t pwords = min(a.part_words, a.words_total - pbase);
  const int kp0 = (int)(pbase / NN), kp1 = (int)((pbase + pwords) / NN);
  // Counters: R copies per bin, 32 bits each, or 16 bits each (copies 2m and
  // 2m+1 share a dword) when the host has bounded every count below 2^16.
  const uint32_t R = 1u << a.log2R;
  const uint32_t dwords_per_bin = a.c16 ? R / 2u : R;
  zero_lds(lds, (uint32_t)(kp1 - kp0) * NN1 * dwords_per_bin);
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  // This thread's dword of a bin is lane mod D (D = dwords per bin): lanes
  // sharing a dword are D chunks (16 D pixels) apart, so on smooth images they
  // rarely vote the same bin; with 16-bit counters the half is bit log2(D).
  const uint32_t D = dwords_per_bin;
  const uint32_t g = threadIdx.x & (D - 1u);
  const uint32_t h = (threadIdx.x / D) & 1u;
  const uint32_t B = D * 4u;  // bytes per bin (all copies)
  const uint32_t Cr = g * 4u;
  const uint32_t inc = a.c16 ? (1u << (h * 16u)) : 1u;
  const uint32_t sent4 = N * 0x01010101u;
  const int y0 = a.y_begin + region * a.region_rows;
  const int y1 = min(a.y_end, y0 + a.region_rows);
  const int chunks = (a.W + 15) >> 4;
  const int spans = (chunks + 63) >> 6;
  const int bands = y1 > y0 ? (y1 - y0 + RPW - 1) / RPW : 0;
  constexpr int NROWS = RPW + MAXDY;

  for (int slab = wave; slab < spans * bands; slab += nwaves) {
    const int span = slab % spans, band = slab / spans;
    const int x0 = ((span << 6) + lane) << 4;
    const int ys = y0 + band * RPW;
    const int nfirst = min(RPW, y1 - ys);
    Ring rows[NROWS];
    {
      RawChunk<Pix> raw[NROWS];
#pragma unroll
      for (int i = 0; i < NROWS; ++i) issue_row<Pix, UNAL>(raw[i], a, ys + i, x0, lane);
#pragma unroll
      for (int i = 0; i < NROWS; ++i) finish_row<Pix>(rows[i], raw[i], a, ys + i, x0, lane, sent4);
    }
    for (int k = kp0; k < kp1; ++k) {
      const int dy = a.dy[k], dx = a.dx[k];
      const bool tr = (a.tmask >> k) & 1ull;
      const uint32_t C = (uint32_t)(k - kp0) * NN1 * B + Cr;
      const uint32_t MA = tr ? B : N1 * B, MB = tr ? N1 * B : B;
      switch (dy) {
        case 0: vote_offset<0, RPW>(lds, rows, nfirst, dx, C, MA, MB, inc); break;
        case 1: if (MAXDY >= 1) vote_offset<(MAXDY >= 1 ? 1 : 0), RPW>(lds, rows, nfirst, dx, C, MA, MB, inc); break;
        case 2: if (MAXDY >= 2) vote_offset<(MAXDY >= 2 ? 2 : 0), RPW>(lds, rows, nfirst, dx, C, MA, MB, inc); break;
        case 3: if (MAXDY >= 3) vote_offset<(MAXDY >= 3 ? 3 : 0), RPW>(lds, rows, nfirst, dx, C, MA, MB, inc); break;
        case 4: if (MAXDY >= 4) vote_offset<(MAXDY >= 4 ? 4 : 0), RPW>(lds, rows, nfirst, dx, C, MA, MB, inc); break;
        default: break;  // the host never launches an offset with dy > MAXDY
      }
    }
  }
  store_partial(a, lds, pbase, pwords, region, N1, NN1, a.c16 != 0);
}

// One first-pixel row of a strip: bases, votes of every GLCM of the
// partition, then the ring slot of this row takes the row NR below (from the
// prefetched raw row) and the raw slot starts loading the row 2 NR below.
template <typename Pix, int MAXDY, int D, bool PAIR, int CUR, bool UNAL>
__device__ __forceinline__ void strip_step(const VoteArgs& a, const Geom& geo, TermRow<MAXDY> (&ring)[MAXDY + 1],
                                           RawChunk<Pix> (&raw)[MAXDY + 1], int y, int x0, const LaneCols& cols,
                                           bool edge, uint32_t C,
                                           uint32_t n1, uint32_t mb, uint32_t sent4,
                                           const int (&code)[4], int kp) {
  constexpr int NR = MAXDY + 1;
  uint32_t fa[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) fa[t] = mad_u24(ring[CUR].s[MAXDY + t], n1, C);
  // (the code of a GLCM slot beyond kp is -1, which no case matches)
  vote_glcm<MAXDY, D, 0, CUR, PAIR>(fa, ring, code[0], 1u);
  vote_glcm<MAXDY, D, 1, CUR, PAIR>(fa, ring, code[1], 1u);
  vote_glcm<MAXDY, D, 2, CUR, PAIR>(fa, ring, code[2], 1u);
  vote_glcm<MAXDY, D, 3, CUR, PAIR>(fa, ring, code[3], 1u);
  to_terms<Pix, MAXDY>(ring[CUR], raw[CUR], a, geo, y + NR, x0, sent4, mb, edge);
  row_load<Pix, UNAL>(raw[CUR], geo, y + 2 * NR, x0, cols);
}

// Merge of the strip layout: one lane per (bin, dword group).  The lane reads
// the group's D dwords as D/4 16-byte units, all at once, in an order rotated
// by the group index so that the lanes of an LDS pass cover different banks,
// sums them and adds the sum to the per-XCD accumulator (or stores it to the
// band partial), transposed for offsets that were negated.  PAIR: the low and
// high halves belong to GLCMs 2q and 2q + 1; while at most a.merge_pack
// copies are added a half cannot carry into the other (the host bounds
// merge_pack times the largest count below 2^16), so the dwords are added
// packed first and split into halves afterwards.
template <int D, bool PAIR>
__device__ void store_partial_strips(const VoteArgs& a, const uint32_t* lds, int region, int kp0, int kp,
                                     uint32_t n1) {
  constexpr uint32_t U = D / 4;                                   // 16-byte units per group
  constexpr uint32_t ROT = D == 32 ? 0 : (D == 16 ? 1 : (D == 8 ? 2 : 3));  // log2(32 / D)
  __syncthreads();
  const uint32_t N = a.q.nlev, NN = N * N, kg = (uint32_t)a.kg;
  const uint32_t groups = n1 * n1 * kg;
  uint32_t* dst = a.partials + (size_t)region * a.words_total;
  uint32_t xcc = 0;
  if (a.xbuf) asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(xcc));
  uint32_t* xs = a.xbuf + (size_t)(xcc & (kXcdSlots - 1u)) * a.words_total;
  // group b = (i * n1 + j) * kg + q; (i, j, q) advance by the mixed-radix
  // digits of blockDim each pass, so the loop divides nothing
  const uint32_t S = blockDim.x;
  const uint32_t sq = S % kg, sj = S / kg % n1, si = S / kg / n1;
  uint32_t q = threadIdx.x % kg, j = threadIdx.x / kg % n1, i = threadIdx.x / kg / n1;
  const uint4* units = (const uint4*)lds;
  for (uint32_t b = threadIdx.x; b < groups; b += S) {
    uint4 v[U];
    const uint32_t rot = b >> ROT;
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) v[u] = units[b * U + ((u + rot) & (U - 1u))];
    uint32_t lo = 0, hi = 0;
    if (!PAIR) {
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) lo += (v[u].x + v[u].y) + (v[u].z + v[u].w);
    } else if (U >= 2 && a.merge_pack >= 8) {
#pragma unroll
      for (uint32_t u = 0; u + 1 < U; u += 2) {
        const uint32_t s8 = ((v[u].x + v[u].y) + (v[u].z + v[u].w)) + ((v[u + 1].x + v[u + 1].y) + (v[u + 1].z + v[u + 1].w));
        lo += s8 & 0xffffu;
        hi += s8 >> 16;
      }
    } else if (a.merge_pack >= 4) {
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        const uint32_t s4 = (v[u].x + v[u].y) + (v[u].z + v[u].w);
        lo += s4 & 0xffffu;
        hi += s4 >> 16;
      }
    } else {
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        lo += (v[u].x & 0xffffu) + (v[u].y & 0xffffu) + (v[u].z & 0xffffu) + (v[u].w & 0xffffu);
        hi += (v[u].x >> 16) + (v[u].y >> 16) + (v[u].z >> 16) + (v[u].w >> 16);
      }
    }
    if (i < N && j < N) {
#pragma unroll
      for (uint32_t h = 0; h < (PAIR ? 2u : 1u); ++h) {
        const uint32_t k = PAIR ? 2u * q + h : q;
        if ((int)k >= kp) break;
        const uint32_t s = h ? hi : lo;
        const uint32_t kgl = (uint32_t)kp0 + k;
        const bool tr = (a.tmask >> kgl) & 1ull;
        const uint32_t w = kgl * NN + (tr ? j * N + i : i * N + j);
        if (a.xbuf) {
          if (s) __hip_atomic_fetch_add(xs + w, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
          dst[w] = s;
        }
      }
    }
    q += sq;
    const uint32_t cq = q >= kg;
    q -= cq ? kg : 0u;
    j += sj + cq;  // < 2 n1
    const uint32_t cj = j >= n1;
    j -= cj ? n1 : 0u;
    i += si + cj;
  }
}

// (reach 4, and uint16 pixels with a reach of 2, need more than the 128
// registers a 1024-thread workgroup leaves a lane: those variants take at most
// 512 threads, as strip_max_threads tells the host)
// UNAL: rows of an image whose base or pitch is not 16-byte aligned, read in
// place as the dwords that hold them (row_load).
template <typename Pix, int MAXDY, int D, bool PAIR, bool UNAL>
__global__ __launch_bounds__(strip_max_threads(sizeof(Pix), MAXDY)) void k_vote_strips(VoteArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  constexpr int NR = MAXDY + 1;
  const int2 rp = band_of_block(blockIdx.x, a.P, a.nregions);
  const int region = rp.x, part = rp.y;
  const int kp0 = part * a.kp, kp = min(a.kp, a.K - kp0);
  const uint32_t N = a.q.nlev, n1 = a.pitch;
  const uint32_t mb = 4u * D * (uint32_t)a.kg;
  // (readfirstlane tells the compiler the wavefront index is uniform, so
  // strip and row indices, and the row addresses, live in scalar registers)
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nwaves = blockDim.x >> 6;
  const uint32_t g = threadIdx.x & (D - 1u);
  const uint32_t C = lds_address(lds) + 4u * g;
  const uint32_t sent4 = N * 0x01010101u;
  const int y0 = a.y_begin + region * a.region_rows;
  const int y1 = min(a.y_end, y0 + a.region_rows);
  const int chunks = (a.W + 15) >> 4;
  const int spans = (chunks + 63) >> 6;
  const int rows = max(0, y1 - y0);
  const int per_span = (rows + a.strip_rows - 1) / a.strip_rows;
  const int nstrips = spans * per_span;
  // offset codes of this partition, read once (scalar loads)
  int code[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) code[q] = q < kp ? __builtin_amdgcn_readfirstlane(a.vcode[kp0 + q]) : -1;
  const Geom geo{a.img, a.stride, a.W, a.H};

  TermRow<MAXDY> ring[NR];
  RawChunk<Pix> raw[NR];
  // the first strip's loads go out before the LDS is cleared
  int strip = wave;
  if (strip < nstrips) {
    const int x0 = (((strip % spans) << 6) + lane) << 4, ya = y0 + (strip / spans) * a.strip_rows;
    const LaneCols cols = lane_cols<Pix>(geo, x0);
#pragma unroll
    for (int r = 0; r < NR; ++r) row_load<Pix, UNAL>(raw[r], geo, ya + r, x0, cols);
  }
  zero_lds(lds, n1 * n1 * (uint32_t)a.kg * D);
  // the quantizer's scalars are waited for here, once: a first use inside
  // the loop would wait on the counter the LDS votes share, every row
  asm volatile("" ::"s"(a.qfast), "s"(a.qfast_shift), "s"(a.qfast_mask), "s"(a.q.lo), "s"(a.q.hi), "s"(a.q.nlev),
               "s"(a.q.magic), "s"(a.q.shift));
  __syncthreads();

  for (; strip < nstrips; strip += nwaves) {
    const int span = strip % spans;
    const int x0 = ((span << 6) + lane) << 4;
    const int ya = y0 + (strip / spans) * a.strip_rows;
    const int yb = min(y1, ya + a.strip_rows);
    const LaneCols cols = lane_cols<Pix>(geo, x0);
    const bool edge = ((span + 1) << 10) + 4 > a.W;  // chunks or right halos reach column W
    if (strip != wave) {
#pragma unroll
      for (int r = 0; r < NR; ++r) row_load<Pix, UNAL>(raw[r], geo, ya + r, x0, cols);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      to_terms<Pix, MAXDY>(ring[r], raw[r], a, geo, ya + r, x0, sent4, mb, edge);
      row_load<Pix, UNAL>(raw[r], geo, ya + NR + r, x0, cols);
    }
    for (int y = ya; y < yb; y += NR) {
      strip_step<Pix, MAXDY, D, PAIR, 0, UNAL>(a, geo, ring, raw, y, x0, cols, edge, C, n1, mb, sent4, code, kp);
      if (y + 1 >= yb) break;
      strip_step<Pix, MAXDY, D, PAIR, 1, UNAL>(a, geo, ring, raw, y + 1, x0, cols, edge, C, n1, mb, sent4, code, kp);
      if constexpr (NR > 2) {
        if (y + 2 >= yb) break;
        strip_step<Pix, MAXDY, D, PAIR, 2, UNAL>(a, geo, ring, raw, y + 2, x0, cols, edge, C, n1, mb, sent4, code,
                                                 kp);
      }
      if constexpr (NR > 4) {
        if (y + 3 >= yb) break;
        strip_step<Pix, MAXDY, D, PAIR, 3, UNAL>(a, geo, ring, raw, y + 3, x0, cols, edge, C, n1, mb, sent4, code,
                                                 kp);
        if (y + 4 >= yb) break;
        strip_step<Pix, MAXDY, D, PAIR, 4, UNAL>(a, geo, ring, raw, y + 4, x0, cols, edge, C, n1, mb, sent4, code,
                                                 kp);
      }
    }
  }
  store_partial_strips<D, PAIR>(a, lds, region, kp0, kp, n1);
}

}  // namespace

template <typename K>
static hipError_t launch(K kernel, const VoteArgs& a, dim3 grid, dim3 block, size_t lds_bytes, hipStream_t stream,
                         const LaunchTiming& tm) {
  // with events, the dispatch itself stamps the kernel's start and end
  hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds_bytes, stream, tm.start, tm.stop, 0u, a);
  return hipGetLastError();
}

hipError_t launch_vote_generic(const VoteArgs& a, int dtype_bytes, int wg, size_t lds_bytes, hipStream_t stream,
                               const LaunchTiming& tm) {
  const dim3 grid(a.nregions * a.P), block(wg);
  if (dtype_bytes == 1) return launch(k_vote_generic<uint8_t>, a, grid, block, lds_bytes, stream, tm);
  return launch(k_vote_generic<uint16_t>, a, grid, block, lds_bytes, stream, tm);
}

template <typename Pix, bool UNAL>
static hipError_t launch_rows_u(const VoteArgs& a, int maxdy, int wg, size_t lds_bytes, hipStream_t stream,
                                const LaunchTiming& tm) {
  const dim3 grid(a.nregions * a.P), block(wg);
  switch (maxdy) {
    case 1: return launch(k_vote_rows<Pix, 1, 4, UNAL>, a, grid, block, lds_bytes, stream, tm);
    case 2: return launch(k_vote_rows<Pix, 2, 4, UNAL>, a, grid, block, lds_bytes, stream, tm);
    case 4: return launch(k_vote_rows<Pix, 4, 4, UNAL>, a, grid, block, lds_bytes, stream, tm);
    default: return hipErrorInvalidValue;
  }
}

template <typename Pix>
static hipError_t launch_rows_t(const VoteArgs& a, int maxdy, int wg, size_t lds_bytes, hipStream_t stream,
                               const LaunchTiming& tm) {
  return a.unaligned ? launch_rows_u<Pix, true>(a, maxdy, wg, lds_bytes, stream, tm)
                     : launch_rows_u<Pix, false>(a, maxdy, wg, lds_bytes, stream, tm);
}

hipError_t launch_vote_rows(const VoteArgs& a, int dtype_bytes, int maxdy, int rpw, int wg, size_t lds_bytes,
                            hipStream_t stream, const LaunchTiming& tm) {
  if (rpw != 4) return hipErrorInvalidValue;
  return dtype_bytes == 1 ? launch_rows_t<uint8_t>(a, maxdy, wg, lds_bytes, stream, tm)
                          : launch_rows_t<uint16_t>(a, maxdy, wg, lds_bytes, stream, tm);
}

template <typename Pix, int MAXDY, bool PAIR, bool UNAL>
static hipError_t launch_strips_u(const VoteArgs& a, int D, int wg, size_t lds_bytes, hipStream_t stream,
                                  const LaunchTiming& tm) {
  const dim3 grid(a.nregions * a.P), block(wg);
  switch (D) {
    case 4: return launch(k_vote_strips<Pix, MAXDY, 4, PAIR, UNAL>, a, grid, block, lds_bytes, stream, tm);
    case 8: return launch(k_vote_strips<Pix, MAXDY, 8, PAIR, UNAL>, a, grid, block, lds_bytes, stream, tm);
    case 16: return launch(k_vote_strips<Pix, MAXDY, 16, PAIR, UNAL>, a, grid, block, lds_bytes, stream, tm);
    case 32: return launch(k_vote_strips<Pix, MAXDY, 32, PAIR, UNAL>, a, grid, block, lds_bytes, stream, tm);
    default: return hipErrorInvalidValue;
  }
}

template <typename Pix, int MAXDY, bool PAIR>
static hipError_t launch_strips_p(const VoteArgs& a, int D, int wg, size_t lds_bytes, hipStream_t stream,
                                 const LaunchTiming& tm) {
  return a.unaligned ? launch_strips_u<Pix, MAXDY, PAIR, true>(a, D, wg, lds_bytes, stream, tm)
                     : launch_strips_u<Pix, MAXDY, PAIR, false>(a, D, wg, lds_bytes, stream, tm);
}

template <typename Pix, int MAXDY>
static hipError_t launch_strips_t(const VoteArgs& a, int D, int wg, size_t lds_bytes, hipStream_t stream,
                                 const LaunchTiming& tm) {
  return a.c16 ? launch_strips_p<Pix, MAXDY, true>(a, D, wg, lds_bytes, stream, tm)
               : launch_strips_p<Pix, MAXDY, false>(a, D, wg, lds_bytes, stream, tm);
}

hipError_t launch_vote_strips(const VoteArgs& a, int dtype_bytes, int maxdy, int D, int wg, size_t lds_bytes,
                              hipStream_t stream, const LaunchTiming& tm) {
  if (maxdy == 1)
    return dtype_bytes == 1 ? launch_strips_t<uint8_t, 1>(a, D, wg, lds_bytes, stream, tm)
                            : launch_strips_t<uint16_t, 1>(a, D, wg, lds_bytes, stream, tm);
  if (maxdy == 2)
    return dtype_bytes == 1 ? launch_strips_t<uint8_t, 2>(a, D, wg, lds_bytes, stream, tm)
                            : launch_strips_t<uint16_t, 2>(a, D, wg, lds_bytes, stream, tm);
  if (maxdy == 4)
    return dtype_bytes == 1 ? launch_strips_t<uint8_t, 4>(a, D, wg, lds_bytes, stream, tm)
                            : launch_strips_t<uint16_t, 4>(a, D, wg, lds_bytes, stream, tm);
  return hipErrorInvalidValue;
}

hipError_t launch_zero(uint32_t* p, uint64_t words, hipStream_t stream) {
  if (words == 0) return hipSuccess;
  const uint64_t blocks = std::min<uint64_t>((words + 255) / 256, 2048);
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, stream, p, words);
  return hipGetLastError();
}

hipError_t launch_xcc_probe(uint32_t* ids, int blocks, hipStream_t stream) {
  hipLaunchKernelGGL(k_xcc_probe, dim3(blocks), dim3(64), 0, stream, ids);
  return hipGetLastError();
}

hipError_t launch_finish(uint32_t* xbuf, uint32_t* out, uint32_t M, uint32_t nslots, bool accumulate,
                         hipStream_t stream) {
  hipLaunchKernelGGL(k_finish, dim3((M + 255) / 256), dim3(256), 0, stream, xbuf, out, M, nslots, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_reduce(const uint32_t* partials, uint32_t* out, uint32_t M, int nbands, bool accumulate,
                         hipStream_t stream) {
  const uint32_t per = 4u * kReduceQuads;
  hipLaunchKernelGGL(k_reduce, dim3((M + per - 1) / per), dim3(kReduceQuads * kReduceGroups), 0, stream, partials,
                     out, M, nbands, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_vote_l2(const VoteArgs& a, int dtype_bytes, int groups, hipStream_t stream, const LaunchTiming& tm) {
  const dim3 grid(groups), block(256);
  if (dtype_bytes == 1) return launch(k_vote_l2<uint8_t>, a, grid, block, 0, stream, tm);
  return launch(k_vote_l2<uint16_t>, a, grid, block, 0, stream, tm);
}

hipError_t launch_vote_global(const VoteArgs& a, int dtype_bytes, hipStream_t stream) {
  const uint64_t n = (uint64_t)(a.y_end - a.y_begin) * (uint64_t)a.W;
  const uint64_t want = (n + 255) / 256;
  const dim3 grid((unsigned)(want < 65536 ? (want ? want : 1) : 65536)), block(256);
  if (dtype_bytes == 1)
    hipLaunchKernelGGL(k_vote_global<uint8_t>, grid, block, 0, stream, a);
  else
    hipLaunchKernelGGL(k_vote_global<uint16_t>, grid, block, 0, stream, a);
  return hipGetLastError();
}

}  // namespace glcm
