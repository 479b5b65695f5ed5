// C-ABI host runtime of the GLCM library: argument checks, plans, path choice,
// workspace management and the streamed upload of host-resident images.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "glcm.h"
#include "glcm_host.h"
#include "glcm_internal.h"
#include "glcm_hist.h"

using glcm::VoteArgs;

namespace {

thread_local int g_last_hip = 0;

int hip_status(hipError_t e) {
  if (e == hipSuccess) return GLCM_OK;
  g_last_hip = (int)e;
  return e == hipErrorOutOfMemory ? GLCM_ENOMEM : GLCM_EHIP;
}

#define GLCM_TRY(expr)                      \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return hip_status(e_); \
  } while (0)

#define GLCM_TRY_RC(expr)          \
  do {                             \
    const int rc_ = (expr);        \
    if (rc_ != GLCM_OK) return rc_; \
  } while (0)

constexpr uint32_t kKnownFlags = GLCM_FLAG_FORCE_GENERIC | GLCM_FLAG_FORCE_PARTITIONED |
                                 GLCM_FLAG_FORCE_GLOBAL | GLCM_FLAG_SERIAL_UPLOAD | GLCM_FLAG_TIMING |
                                 GLCM_FLAG_FORCE_SLABS | GLCM_FLAG_FORCE_L2 | GLCM_FLAG_FORCE_BLOCKS;

enum Path {
  kPathGeneric = 0, kPathRows = 1, kPathPartitioned = 2, kPathGlobal = 3, kPathStrips = 4, kPathL2 = 5,
  kPathBlocks = 6
};

// Misaligned device images (base or pitch not 16-byte aligned) of at least
// this many pixels: the strip and slab kernels read them in place (rows
// assembled from the dwords that hold them); for the block-code kernel, which
// needs 16-byte rows, they are copied into an aligned staging buffer.
// Smaller ones take the per-pixel kernel, faster there.  Measured on MI355X:
// 4096 uint8 images of 32-512 px, one call each, 138 ms per-pixel against
// 175 ms in place; 4096^2 uint16 images 62-105 us per call in place against
// 93-133 us copied first (the pitched copy alone costs 40-60 us).
constexpr uint64_t kStageMinPixels = 1u << 16;



int dtype_bytes(int dtype) { return dtype == GLCM_U8 ? 1 : (dtype == GLCM_U16 ? 2 : 0); }

// ---------------------------------------------------------------------------
// Validation shared by the entry points (no HIP calls).
// ---------------------------------------------------------------------------
int check_offsets(const glcm_offset_t* offsets, int K) {
  if (!offsets || K < 1 || K > GLCM_MAX_OFFSETS) return GLCM_EINVAL;
  for (int k = 0; k < K; ++k) {
    if (offsets[k].dx < -GLCM_MAX_DISPLACEMENT || offsets[k].dx > GLCM_MAX_DISPLACEMENT ||
        offsets[k].dy < -GLCM_MAX_DISPLACEMENT || offsets[k].dy > GLCM_MAX_DISPLACEMENT)
      return GLCM_EINVAL;
  }
  return GLCM_OK;
}

int check_image_args(const void* img, int W, int H, int64_t stride, int dtype, int N, uint32_t lo, uint32_t hi,
                     const glcm_offset_t* offsets, int K) {
  const int b = dtype_bytes(dtype);
  if (!img || b == 0) return GLCM_EINVAL;
  if (W < 1 || H < 1 || stride < W) return GLCM_EINVAL;
  if ((uint64_t)W * (uint64_t)H > 0xffffffffull) return GLCM_EINVAL;
  if (N < 1 || N > GLCM_MAX_LEVELS) return GLCM_EINVAL;
  if (lo > hi || hi > (b == 1 ? 255u : 65535u)) return GLCM_EINVAL;
  if (((uintptr_t)img) % (uintptr_t)b) return GLCM_EINVAL;
  if (check_offsets(offsets, K) != GLCM_OK) return GLCM_EINVAL;
  return GLCM_OK;
}

int check_compute_args(const void* img, int W, int H, int64_t stride, int dtype, int N, uint32_t lo,
                       uint32_t hi, const glcm_offset_t* offsets, int K, const uint32_t* out) {
  const int rc = check_image_args(img, W, H, stride, dtype, N, lo, hi, offsets, K);
  if (rc != GLCM_OK) return rc;
  if (!out) return GLCM_EINVAL;
  const int b = dtype_bytes(dtype);
  // out must not overlap the image bytes
  const uintptr_t i0 = (uintptr_t)img;
  const uintptr_t i1 = i0 + (uintptr_t)(((uint64_t)(H - 1) * (uint64_t)stride + (uint64_t)W) * (uint64_t)b);
  const uintptr_t o0 = (uintptr_t)out;
  const uintptr_t o1 = o0 + (uintptr_t)((uint64_t)K * N * N * 4u);
  if (o0 < i1 && i0 < o1) return GLCM_EINVAL;
  return GLCM_OK;
}

glcm::Quant make_quant(int N, uint32_t lo, uint32_t hi) {
  glcm::Quant q{};
  q.lo = lo;
  q.hi = hi;
  q.nlev = (uint32_t)N;
  const uint64_t D = (uint64_t)hi - lo + 1u;  // 1 .. 65536
  uint32_t s = 0;
  while ((1ull << s) < D) ++s;               // ceil(log2 D)
  const uint64_t m = ((1ull << (32 + s)) + D - 1) / D;  // ceil(2^(32+s) / D), in (2^32, 2^33]
  q.magic = (uint32_t)(m - (1ull << 32));
  q.shift = s;
  return q;
}

// The shift form of q(): lo = 0, hi = dtype max and N a power of two give
// level = pixel >> (bits - log2 N), applied to 4 packed u8 / 2 packed u16.
void fast_quant(int b, int N, uint32_t lo, uint32_t hi, int* on, uint32_t* shift, uint32_t* mask) {
  const uint32_t top = b == 1 ? 255u : 65535u, bits = b == 1 ? 8u : 16u;
  uint32_t n = 0;
  while ((1u << n) < (uint32_t)N) ++n;
  *on = 0;
  *shift = 0;
  *mask = 0;
  if (lo == 0 && hi == top && (1u << n) == (uint32_t)N && n <= bits) {
    *on = 1;
    *shift = bits - n;
    *mask = b == 1 ? (0xffu >> *shift) * 0x01010101u : (0xffffu >> *shift) * 0x00010001u;
  }
}

// Offsets as the row kernel wants them: dy >= 0 (and dx >= 0 when dy == 0);
// a negated offset is counted as its opposite and voted transposed.
struct Canon {
  int32_t dx[glcm::kMaxK], dy[glcm::kMaxK];
  unsigned long long tmask = 0;
  int maxdy = 0, maxadx = 0;
  int up = 0, down = 0;  // rows of halo above / below a row band (original offsets)
};

Canon canonicalize(const glcm_offset_t* o, int K) {
  Canon c;
  for (int k = 0; k < K; ++k) {
    int dx = o[k].dx, dy = o[k].dy;
    c.up = std::max(c.up, -dy);
    c.down = std::max(c.down, dy);
    if (dy < 0 || (dy == 0 && dx < 0)) {
      dx = -dx;
      dy = -dy;
      c.tmask |= 1ull << k;
    }
    c.dx[k] = dx;
    c.dy[k] = dy;
    c.maxdy = std::max(c.maxdy, dy);
    c.maxadx = std::max(c.maxadx, std::abs(dx));
  }
  return c;
}

int pointer_kind(const void* p, int* device) {
  // 0 = pageable host, 1 = pinned host, 2 = device
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  if (device) *device = attr.device;
  if (attr.type == hipMemoryTypeDevice) return 2;
  if (attr.type == hipMemoryTypeHost) return 1;
  if (attr.type == hipMemoryTypeManaged) return 2;
  return 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// Plans
// ---------------------------------------------------------------------------
struct glcm_plan_s {
  int device = 0;
  int dtype = 0;
  int N = 0, K = 0;
  int k_cap = 0;  // the K the workspace was sized for (glcm_plan_rebind may lower K)
  glcm_offset_t offsets[GLCM_MAX_OFFSETS];
  int max_W = 0, max_H = 0;
  uint32_t flags = 0;
  glcm_tuning_t tuning{};
  bool user_tuned = false;
  int lds_budget_words = 0;
  int num_cus = 0;

  // device workspace
  uint32_t* partials = nullptr;
  size_t partials_bytes = 0;
  void* stage = nullptr;  // aligned copy of a misaligned device image (row pitch a multiple of 16 bytes)
  size_t stage_bytes = 0;
  uint32_t* xbuf = nullptr;  // [kXcdSlots][K*N*N] accumulation slices, kept zero between calls
  uint32_t xslots = glcm::kXcdSlots;  // slices the device's XCC_IDs reach (the rest stay zero)
  bool no_alloc = false;  // a transient plan of compute_in_workspace: never allocate (no staging copy)


  // ordering across streams
  hipEvent_t done = nullptr;
  hipStream_t last_stream = nullptr;
  bool has_done = false;

  // host-image upload resources
  hipStream_t copy_stream = nullptr;
  static constexpr int kSlots = 2;
  void* dev_tile[kSlots] = {nullptr, nullptr};
  void* pin_tile[kSlots] = {nullptr, nullptr};
  size_t tile_bytes = 0;
  hipEvent_t uploaded[kSlots] = {nullptr, nullptr};
  bool pin_pending[kSlots] = {false, false};  // a staging slot's upload may still be running
  hipEvent_t consumed[kSlots] = {nullptr, nullptr};

  // batch descriptors: pinned staging and its device copy
  void* batch_pin = nullptr;
  void* batch_dev = nullptr;
  size_t batch_cap = 0;
  hipEvent_t batch_uploaded = nullptr;
  bool batch_pending = false;

  // batch kernel layout: LDS copies per bin (0: the default rule) and the
  // shortest run of rows a wavefront segment walks (0: kBatchDefaultMinRows, 4); glcm_batch_tuning
  int batch_D = 0, batch_min_rows = 0;
  int batch_wg = 0;  // threads per batch workgroup (0: glcm::kBatchThreads)

  // GLCM_FLAG_TIMING: events around every counting-kernel launch
  std::vector<std::pair<hipEvent_t, hipEvent_t>> timing;

  std::mutex mu;
};

namespace {

// Accumulation slices the per-XCD merge uses on a device: one more than the
// largest XCC_ID (mod kXcdSlots) its workgroups report.  Workgroups go to the
// XCDs round-robin, so 1024 probe workgroups visit every XCD.  Probed once
// per device; on any failure all kXcdSlots slices are kept.
uint32_t xcc_slots(int device) {
  static std::mutex m;
  static std::map<int, uint32_t> cache;
  std::lock_guard<std::mutex> g(m);
  auto it = cache.find(device);
  if (it != cache.end()) return it->second;
  constexpr int kBlocks = 1024;
  uint32_t slots = glcm::kXcdSlots;
  uint32_t* d = nullptr;
  if (hipMalloc((void**)&d, kBlocks * sizeof(uint32_t)) == hipSuccess) {
    std::vector<uint32_t> h(kBlocks, glcm::kXcdSlots - 1u);
    if (glcm::launch_xcc_probe(d, kBlocks, nullptr) == hipSuccess &&
        hipMemcpy(h.data(), d, kBlocks * sizeof(uint32_t), hipMemcpyDeviceToHost) == hipSuccess) {
      uint32_t mx = 0;
      for (uint32_t v : h) mx = std::max(mx, v & (glcm::kXcdSlots - 1u));
      slots = mx + 1u;
    }
    (void)hipFree(d);
  }
  cache[device] = slots;
  return slots;
}

// Row pitch of the LDS copy of a GLCM in the row kernel: at least N + 1 (row
// and column N take the votes of pixels outside the image) and 2 mod 4, so
// that the bins of the diagonal, where smooth images put most of their pairs,
// spread over all banks of a copy group (bank = bin index mod 4 there).
uint32_t row_pitch(int N) {
  uint32_t n1 = (uint32_t)N + 1u;
  while (n1 % 4u != 2u) ++n1;
  return n1;
}

// LDS dwords of one GLCM in the row kernel for R copies of `bits`-bit counters.
uint64_t row_glcm_dwords(int N, int R, int bits) {
  const uint64_t p = row_pitch(N);
  return p * p * (uint64_t)(bits == 16 ? R / 2 : R);
}

// Partitions (groups of whole GLCMs) the row kernel needs; 0 if one GLCM
// does not fit.
int row_partitions(const glcm_plan_s* p, int R, int bits) {
  const uint64_t per = (uint64_t)p->lds_budget_words / row_glcm_dwords(p->N, R, bits);
  if (per == 0) return 0;
  return (int)(((uint64_t)p->K + per - 1) / per);
}

// Strip kernel: dwords per bin for R copies (4, 8, 16 or 32), or 0 when the
// kernel has no such variant.  With 16-bit counters the copies stay R and each
// dword holds two GLCMs.
int strip_dwords(int R) { return (R == 4 || R == 8 || R == 16 || R == 32) ? R : 0; }

// Strip kernel: GLCMs per partition for D dwords per bin ((N+1)^2 bins each),
// two per dword group with 16-bit pairs, at most kStripMaxKp; 0 if none fits.
int strip_kp(const glcm_plan_s* p, int D, bool pair) {
  const uint64_t n1 = (uint64_t)p->N + 1u;
  const uint64_t groups = (uint64_t)p->lds_budget_words / (n1 * n1 * (uint64_t)D);
  return (int)std::min<uint64_t>(groups * (pair ? 2u : 1u), (uint64_t)glcm::kStripMaxKp);
}

int strip_partitions(const glcm_plan_s* p, int R, int bits) {
  const int D = strip_dwords(R);
  if (D == 0) return 0;
  const int kp = strip_kp(p, D, bits == 16);
  if (kp == 0) return 0;
  return (p->K + kp - 1) / kp;
}

// Strip kernel layout for `rows` first-pixel rows of width W: D dwords per
// bin, kp GLCMs per partition in kg dword groups, row bands and strips.  The
// 16-bit pair layout only when no counter can reach 2^16: a counter (bin,
// copy, GLCM) is shared by wg / D lanes, each voting at most 16 pixels per row
// it walks; otherwise 32-bit counters (fewer GLCMs per partition).
struct StripLayout {
  int D = 0, kp = 0, kg = 0, P = 0, pair = 0, nregions = 0, region_rows = 0, strip_rows = 0;
  int pack = 1;  // 16-bit pairs: copies the merge may add packed (pack * largest count < 2^16)
  size_t lds = 0;
};

bool strip_layout(const glcm_plan_s* p, int W, int rows, int R, bool want_pair, int wg, StripLayout* L) {
  const int spans = (((W + 15) / 16) + 63) / 64, nwaves = wg / 64;
  const uint64_t n1 = (uint64_t)p->N + 1u, words = (uint64_t)p->K * p->N * p->N;
  const int D = strip_dwords(R);
  if (D == 0 || rows < 1) return false;
  for (int pair = want_pair ? 1 : 0; pair >= 0; --pair) {
    const int kp = strip_kp(p, D, pair != 0);
    if (kp == 0) continue;
    const int kg = pair ? (kp + 1) / 2 : kp;
    const int P = (p->K + kp - 1) / kp;
    const size_t lds = (size_t)(n1 * n1) * (size_t)kg * (size_t)D * 4u;
    // as many bands per partition as the CUs hold at once, each tall enough
    // for strips of >= 4 rows on every wavefront
    const int per_cu =
        std::max(1, std::min((int)(((size_t)p->lds_budget_words * 4u + 1024u) / std::max(lds, (size_t)wg * 4u)),
                             32 / nwaves));
    int nregions = std::min(rows, std::max(1, p->num_cus * per_cu / P));
    nregions = std::max(1, std::min(nregions, rows * spans / (4 * nwaves)));
    while (nregions > 1 && (uint64_t)nregions * words * 4ull > (256ull << 20)) nregions = (nregions + 1) / 2;
    const int region_rows = (rows + nregions - 1) / nregions;
    nregions = (rows + region_rows - 1) / region_rows;
    const int strips_per_span = std::max(1, nwaves / spans);
    const int strip_rows = std::max(1, (region_rows + strips_per_span - 1) / strips_per_span);
    if (pair) {
      const int nstrips = spans * ((region_rows + strip_rows - 1) / strip_rows);
      const uint64_t rows_per_lane = (uint64_t)((nstrips + nwaves - 1) / nwaves) * (uint64_t)strip_rows;
      const uint64_t most = (uint64_t)wg / (uint64_t)D * 16u * rows_per_lane;  // largest count of a copy
      if (most > 65535u) continue;
      L->pack = 1;
      while (L->pack < D && (uint64_t)(2 * L->pack) * most <= 65535u) L->pack *= 2;
    }
    L->D = D; L->kp = kp; L->kg = kg; L->P = P; L->pair = pair; L->lds = lds;
    L->nregions = nregions; L->region_rows = region_rows; L->strip_rows = strip_rows;
    return true;
  }
  return false;
}

// The per-XCD accumulation slices of all K GLCMs stay within 256 MiB (then
// the plan keeps them and the L2-slice path is possible).
bool l2_slices_fit(const glcm_plan_s* p) {
  return (uint64_t)glcm::kXcdSlots * (uint64_t)p->k_cap * (uint64_t)p->N * (uint64_t)p->N * 4ull <= (256ull << 20);
}

// Block-code kernel: every offset is one of the four d = 1 directions or its
// opposite, the code bins and block GLCMs fit one workgroup's LDS, and the
// plan keeps the per-XCD slices (its merge adds into them).
int block_glcm(const glcm_offset_t& o) {
  int dx = o.dx, dy = o.dy;
  if (dy < 0 || (dy == 0 && dx < 0)) {
    dx = -dx;
    dy = -dy;
  }
  if (dy == 0 && dx == 1) return 0;
  if (dy == 1 && dx == -1) return 1;
  if (dy == 1 && dx == 0) return 2;
  if (dy == 1 && dx == 1) return 3;
  return -1;
}

// Copies of the block kernel's block GLCMs: the most of 4, 2, 1 whose LDS
// fits (0: none).
int block_fb_copies(const glcm_plan_s* p) {
  for (int c = 4; c >= 1; c /= 2)
    if (glcm::block_lds_bytes(p->N, c) <= (size_t)p->lds_budget_words * 4u) return c;
  return 0;
}

bool blocks_fit(const glcm_plan_s* p) {
  // N <= 62: the window test's biased digit bytes X - a + 0x40 (X up to N + 1,
  // a up to the sentinel N) stay in [0, 0x80) without a borrow
  if (p->N > 62 || p->max_W > 65536 || block_fb_copies(p) == 0) return false;
  for (int k = 0; k < p->K; ++k)
    if (block_glcm(p->offsets[k]) < 0) return false;
  return true;
}

// Image passes of the partitioned kernel worth one GLCM's pairs added into
// the per-XCD L2 slices: measured on MI355X, 4096^2 u8 images, a pass costs
// 0.04-0.05 ms and a GLCM in the slices 0.63 ms on noise (more on smooth
// images, where the slice atomics collide: 0.5-1.5 ms).  The slices take
// over beyond this many passes per GLCM.
constexpr int kPassesPerSliceGlcm = 13;

// Shortest run of rows a wavefront segment of the batch kernel walks, unless
// tuned: on 4096 tiles of 32-512 px (N = 16, K = 4) the autotuner picks 4
// over 8 in every run measured on MI355X (0.291 against 0.309 ms per batch).
constexpr int kBatchDefaultMinRows = 4;

// Row kernels (strips, slabs, blocks) store a level and the sentinel N in one
// byte; the strip kernel reaches |dx|, dy <= 2 for any offset and 4 along the
// four directions of Eq.(2) (dx = 0, dy = 0 or |dx| = dy), the slab kernel 4
// for any offset.
bool row_kernels_ok(const glcm_plan_s* p) {
  return !(p->flags & (GLCM_FLAG_FORCE_GENERIC | GLCM_FLAG_FORCE_PARTITIONED)) && p->N <= 255;
}
bool strip_offsets_ok(const glcm_plan_s* p, const Canon& c) {
  for (int k = 0; k < p->K; ++k) {
    const int ax = std::abs(c.dx[k]), dy = c.dy[k], r = std::max(ax, dy);
    if (r > 4 || (r > 2 && ax != 0 && dy != 0 && ax != dy)) return false;
  }
  return true;
}
// The strip kernel's template reach (ring of reach + 1 rows): 1, 2 or 4.
int strip_reach(const Canon& c) {
  const int r = std::max(c.maxdy, c.maxadx);
  return r <= 1 ? 1 : (r <= 2 ? 2 : 4);
}
bool strips_eligible(const glcm_plan_s* p, const Canon& c) {
  return row_kernels_ok(p) && !(p->flags & GLCM_FLAG_FORCE_SLABS) && strip_offsets_ok(p, c) &&
         strip_partitions(p, 4, 16) > 0;
}
bool slabs_eligible(const glcm_plan_s* p, const Canon& c) {
  return row_kernels_ok(p) && c.maxadx <= 4 && c.maxdy <= 4 && row_partitions(p, 1, 32) > 0;
}

// Whether the strip layout with R dwords per bin beats the slab kernel by
// default.  Measured on MI355X (4096^2 smooth and noise images and an 8192^2
// band, u8 and u16, N = 8 to 64, d = 1, 2 and both): with 16 or 32 dwords per
// bin, and with 8 at a reach of 1, strips are 1.0-1.5x faster; with 8 at a
// reach of 2, or 4, they tie on smooth images and are up to 1.5x slower on
// noise and on 8192-pixel rows (the few copies concentrate same-bank votes).
// At a reach of 3 or 4 (five-row ring, half the waves) strips were 0.63-1.02x
// the slab speed except on smooth images at N = 32 with 12 offsets (1.2x), so
// they are left to the autotuner there.
bool strips_beat_slabs(int R, int reach) { return reach <= 2 && (R >= 16 || (R == 8 && reach <= 1)); }

int choose_tuning(glcm_plan_t p, glcm_tuning_t* t) {
  // Path and LDS layout for this plan's (dtype, N, K, offsets, flags).
  const uint32_t NN = (uint32_t)p->N * (uint32_t)p->N;
  const uint64_t words = (uint64_t)p->K * NN;
  const Canon c = canonicalize(p->offsets, p->K);
  const uint64_t budget = (uint64_t)p->lds_budget_words;
  glcm_tuning_t d{};
  d.wg_size = 1024;
  d.rows_per_wave = 0;
  d.tile_rows = 1024;
  d.counter_bits = 32;
  d.merge = 0;
  if (p->flags & GLCM_FLAG_FORCE_GLOBAL) {
    d.path = kPathGlobal;
    d.replicas = 1;
    d.partitions = 1;
  } else if ((p->flags & GLCM_FLAG_FORCE_L2) && l2_slices_fit(p)) {
    d.path = kPathL2;
    d.replicas = 1;
    d.partitions = 1;
  } else {
    const bool blocks_ok = row_kernels_ok(p) && (p->flags & GLCM_FLAG_FORCE_BLOCKS) && blocks_fit(p);
    const bool rows_ok = slabs_eligible(p, c);
    bool strips_ok = strips_eligible(p, c);
    glcm_tuning_t st = d;
    if (strips_ok) {
      st.path = kPathStrips;
      // The most dwords per bin (32 put every lane of a 32-lane LDS pass on
      // its own bank) that costs at most max(2, minimum) image passes, with
      // two GLCMs per dword (16-bit counters) unless 32-bit counters fit in as
      // few passes (measured on MI355X, 4096^2 at N = 32: 32 copies in pairs
      // over two passes is the fastest layout on smooth and constant images)
      const int Pmin = strip_partitions(p, 4, 16);
      for (int R = 32; R >= 4; R /= 2) {
        const int P32 = strip_partitions(p, R, 32), P16 = strip_partitions(p, R, 16);
        const int bits = (P16 > 0 && (P32 == 0 || P16 < P32)) ? 16 : 32;
        const int P = bits == 16 ? P16 : P32;
        if (P > 0 && P <= std::max(2, Pmin)) {
          st.replicas = R;
          st.counter_bits = bits;
          st.partitions = P;
          break;
        }
      }
      if (rows_ok && !strips_beat_slabs(st.replicas, std::max(c.maxdy, c.maxadx))) strips_ok = false;
    }
    if (blocks_ok) {
      d.path = kPathBlocks;
      d.replicas = 32;
      d.counter_bits = 16;
      d.partitions = 1;
    } else if (strips_ok) {
      d = st;
    } else if (rows_ok) {
      d.path = kPathRows;
      d.rows_per_wave = 4;
      // The most dwords per bin (copies spread same-bin votes over more
      // addresses and banks) that costs at most max(2, minimum) partitions:
      // measured on MI355X, fewer LDS conflicts are worth reading the image
      // twice, not more.
      const int Pmin = row_partitions(p, 1, 32);
      for (int R = 16; R >= 1; R /= 2) {
        const int P = row_partitions(p, R, 32);
        if (P > 0 && P <= std::max(2, Pmin)) {
          d.replicas = R;
          d.counter_bits = 32;
          d.partitions = P;
          break;
        }
      }
    } else {
      uint64_t P1 = (words + budget - 1) / budget;
      if (p->flags & GLCM_FLAG_FORCE_PARTITIONED) P1 = std::max<uint64_t>(P1, std::min<uint64_t>(words, 3));
      // the passes the partitioned kernel runs: half as many with 16-bit
      // counters, which need the XCD slices and rows below 2^16 pixels
      const bool c16 = P1 > 1 && l2_slices_fit(p) && p->max_W <= 65535;
      const uint64_t passes = c16 ? (words + 2 * budget - 1) / (2 * budget) : P1;
      if (passes > (uint64_t)kPassesPerSliceGlcm * (uint64_t)p->K) {
        // more LDS passes than pay off: pairs straight into the per-XCD
        // slices when they fit (never slower than device-wide atomics on
        // MI355X, faster on smooth images), else device-wide atomics
        d.path = l2_slices_fit(p) ? kPathL2 : kPathGlobal;
        d.replicas = 1;
        d.partitions = 1;
      } else {
        int R = 1;
        while (R < 16 && (words * 2 * R + budget - 1) / budget <= P1) R *= 2;
        d.path = P1 > 1 ? kPathPartitioned : kPathGeneric;
        d.replicas = R;
        d.partitions = (int)P1;
        // several bin partitions with one copy: 16-bit counters, two bins per
        // dword, half the passes (faster on smooth images; on noise the
        // shorter bands' merge can cost more, which the autotuner weighs)
        if (P1 > 1 && R == 1) d.counter_bits = 16;
      }
    }
  }
  *t = d;
  return GLCM_OK;
}

int plan_init(glcm_plan_t p) {
  GLCM_TRY(hipGetDevice(&p->device));
  int lds = 0;
  GLCM_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device));
  GLCM_TRY(hipDeviceGetAttribute(&p->num_cus, hipDeviceAttributeMultiprocessorCount, p->device));
  // keep 1 KiB for static LDS (reduction scratch) and the 64 trash words
  p->lds_budget_words = (lds - 1024) / 4;
  choose_tuning(p, &p->tuning);
  if (p->tuning.path != kPathGlobal) {
    const size_t glcm_bytes = (size_t)p->K * p->N * p->N * 4u;
    if ((size_t)glcm::kXcdSlots * glcm_bytes <= (256u << 20)) {
      p->xslots = xcc_slots(p->device);
      const size_t bytes = (size_t)glcm::kXcdSlots * glcm_bytes;
      GLCM_TRY(hipMalloc((void**)&p->xbuf, bytes));
      // zeroed before the plan is returned: its first call may come on a
      // non-blocking stream, which is not ordered after the null stream
      GLCM_TRY(hipMemsetAsync(p->xbuf, 0, bytes, nullptr));
      GLCM_TRY(hipStreamSynchronize(nullptr));
    } else {
      p->tuning.merge = 1;  // band partials only
    }
  }

  GLCM_TRY(hipEventCreateWithFlags(&p->done, hipEventDisableTiming));
  return GLCM_OK;
}

void plan_release(glcm_plan_t p) {
  if (p->has_done) (void)hipEventSynchronize(p->done);
  if (p->copy_stream) (void)hipStreamSynchronize(p->copy_stream);
  for (int s = 0; s < glcm_plan_s::kSlots; ++s) {
    if (p->dev_tile[s]) (void)hipFree(p->dev_tile[s]);
    if (p->pin_tile[s]) (void)hipHostFree(p->pin_tile[s]);
    if (p->uploaded[s]) (void)hipEventDestroy(p->uploaded[s]);
    if (p->consumed[s]) (void)hipEventDestroy(p->consumed[s]);
  }
  if (p->copy_stream) (void)hipStreamDestroy(p->copy_stream);
  if (p->partials) (void)hipFree(p->partials);
  if (p->stage) (void)hipFree(p->stage);
  if (p->xbuf) (void)hipFree(p->xbuf);
  if (p->batch_pending) (void)hipEventSynchronize(p->batch_uploaded);
  if (p->batch_pin) (void)hipHostFree(p->batch_pin);
  if (p->batch_dev) (void)hipFree(p->batch_dev);
  if (p->batch_uploaded) (void)hipEventDestroy(p->batch_uploaded);

  if (p->done) (void)hipEventDestroy(p->done);
  for (auto& ev : p->timing) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
}

// Makes sure the plan's workspace can hold `bytes` of partials.  Waits for the
// plan's queued work before replacing a buffer.
int ensure_partials(glcm_plan_t p, size_t bytes) {
  if (bytes <= p->partials_bytes) return GLCM_OK;
  if (p->has_done) GLCM_TRY(hipEventSynchronize(p->done));
  if (p->partials) GLCM_TRY(hipFree(p->partials));
  p->partials = nullptr;
  p->partials_bytes = 0;
  GLCM_TRY(hipMalloc((void**)&p->partials, bytes));
  p->partials_bytes = bytes;
  return GLCM_OK;
}

// Makes sure the plan's staging buffer holds `bytes`; waits for the plan's
// queued work before replacing it.
int ensure_stage(glcm_plan_t p, size_t bytes) {
  if (bytes <= p->stage_bytes) return GLCM_OK;
  if (p->has_done) GLCM_TRY(hipEventSynchronize(p->done));
  if (p->stage) GLCM_TRY(hipFree(p->stage));
  p->stage = nullptr;
  p->stage_bytes = 0;
  GLCM_TRY(hipMalloc(&p->stage, bytes));
  p->stage_bytes = bytes;
  return GLCM_OK;
}

// Orders this call after the plan's previous call when it ran on another stream.
int order_after_previous(glcm_plan_t p, hipStream_t s) {
  if (p->has_done && p->last_stream != s) GLCM_TRY(hipStreamWaitEvent(s, p->done, 0));
  return GLCM_OK;
}

int record_done(glcm_plan_t p, hipStream_t s) {
  GLCM_TRY(hipEventRecord(p->done, s));
  p->has_done = true;
  p->last_stream = s;
  return GLCM_OK;
}

// Queues the counting of first-pixel rows [y_begin, y_end) of a device image
// whose rows [0, H) are all resident, writing (or adding into) out.
// finish = false leaves the counts in the per-XCD accumulators (host tiles);
// the last call then finishes with accumulate = false.
int count_device(glcm_plan_t p, const void* img, int W, int H, int64_t stride, int y_begin, int y_end,
                 uint32_t lo, uint32_t hi, uint32_t* out, bool accumulate, bool finish, hipStream_t stream) {
  const glcm_tuning_t& t = p->tuning;
  const int b = dtype_bytes(p->dtype);
  const uint32_t NN = (uint32_t)p->N * (uint32_t)p->N;
  const uint32_t words = (uint32_t)p->K * NN;

  VoteArgs a;
  std::memset(&a, 0, sizeof(a));
  a.img = img;
  a.stride = stride;
  a.W = W;
  a.H = H;
  a.y_begin = y_begin;
  a.y_end = y_end;
  a.q = make_quant(p->N, lo, hi);
  // x / N and x / N^2 as multiply-high + shift: make_quant(1, 0, d - 1) has
  // D = d and the same division constants
  a.div_n = make_quant(1, 0, (uint32_t)p->N - 1);
  a.div_nn = make_quant(1, 0, NN - 1);
  fast_quant(b, p->N, lo, hi, &a.qfast, &a.qfast_shift, &a.qfast_mask);
  a.K = p->K;
  a.words_total = words;
  a.out = out;

  int path = t.path;
  const Canon c = canonicalize(p->offsets, p->K);
  // the block kernel merges into the per-XCD slices only
  if (path == kPathBlocks && (t.merge != 0 || !p->xbuf)) path = kPathStrips;
  if (path == kPathRows || path == kPathStrips || path == kPathBlocks) {
    const bool aligned = ((uintptr_t)img % 16 == 0) && (((uint64_t)stride * b) % 16 == 0);
    const bool large = (uint64_t)W * (uint64_t)H >= kStageMinPixels;
    const bool can_stage = !p->no_alloc && y_begin == 0 && y_end == H;
    if (!aligned && path != kPathBlocks && large) {
      a.unaligned = 1;  // read in place
    } else if (!aligned && large && can_stage) {
      // one pitched copy into the plan's aligned buffer, then the fast kernels
      const size_t pitch = ((size_t)W * b + 15) & ~(size_t)15;
      GLCM_TRY_RC(ensure_stage(p, pitch * (size_t)H));
      GLCM_TRY(hipMemcpy2DAsync(p->stage, pitch, img, (size_t)stride * b, (size_t)W * b, (size_t)H,
                                hipMemcpyDeviceToDevice, stream));
      img = p->stage;
      stride = (int64_t)(pitch / b);
      a.img = img;
      a.stride = stride;
    } else if (!aligned) {
      path = (words <= (uint32_t)p->lds_budget_words) ? kPathGeneric : kPathPartitioned;
    }
  }
  const bool xcd = t.merge == 0 && p->xbuf != nullptr && path != kPathGlobal;
  if (y_end <= y_begin) {
    // nothing to count: clear (or keep) the output
    if (xcd && finish) GLCM_TRY(glcm::launch_finish(p->xbuf, out, words, p->xslots, accumulate, stream));
    else if (!accumulate && !xcd) GLCM_TRY(glcm::launch_zero(out, words, stream));
    return GLCM_OK;
  }

  if (path == kPathGlobal || (path == kPathL2 && !xcd)) {
    for (int k = 0; k < p->K; ++k) {
      a.dx[k] = p->offsets[k].dx;
      a.dy[k] = p->offsets[k].dy;
    }
    if (!accumulate) GLCM_TRY(glcm::launch_zero(out, words, stream));
    GLCM_TRY(glcm::launch_vote_global(a, b, stream));
    return GLCM_OK;
  }
  if (path == kPathL2) {
    for (int k = 0; k < p->K; ++k) {
      a.dx[k] = p->offsets[k].dx;
      a.dy[k] = p->offsets[k].dy;
    }
    a.xbuf = p->xbuf;
    a.region_rows = 16;
    glcm::LaunchTiming tm;
    if (p->flags & GLCM_FLAG_TIMING) {
      GLCM_TRY(hipEventCreate(&tm.start));
      GLCM_TRY(hipEventCreate(&tm.stop));
      p->timing.emplace_back(tm.start, tm.stop);
    }
    const int cols = (W + 63) / 64, runs = (y_end - y_begin + 15) / 16;
    const int groups = std::max(1, std::min((cols * runs + 3) / 4, p->num_cus * 8));
    hipError_t e = glcm::launch_vote_l2(a, b, groups, stream, tm);
    if (e == hipSuccess && finish) e = glcm::launch_finish(p->xbuf, out, words, p->xslots, accumulate, stream);
    if (e != hipSuccess) {
      (void)glcm::launch_zero(p->xbuf, (uint64_t)p->xslots * words, stream);
      return hip_status(e);
    }
    return GLCM_OK;
  }

  if (path == kPathBlocks) {
    glcm::BlockArgs ba;
    std::memset(&ba, 0, sizeof(ba));
    ba.img = img;
    ba.stride = stride;
    ba.W = W;
    ba.H = H;
    ba.y_begin = y_begin;
    ba.y_end = y_end;
    ba.q = a.q;
    ba.qfast = a.qfast;
    ba.qfast_shift = a.qfast_shift;
    ba.qfast_mask = a.qfast_mask;
    for (int k = 0; k < p->K; ++k) ba.kmask[block_glcm(p->offsets[k])] |= 1ull << k;
    ba.tmask = c.tmask;
    ba.nbins = 16u * (uint32_t)p->N + 6u;
    ba.fb_copies = block_fb_copies(p);
    ba.div_n = a.div_n;
    ba.words_total = words;
    ba.xbuf = p->xbuf;
    // bands: one workgroup of 16 wavefronts per band, as many bands as the
    // CUs hold at once, each tall enough for strips of >= 4 rows on every
    // wavefront; a band holds fewer than 2^17 chunk pixels (the merge adds
    // the copies of half the lanes packed, 16 bits per code)
    constexpr int kWg = 1024, kWaves = kWg / 64;
    const int rows = y_end - y_begin;
    const int spans = (((W + 15) / 16) + 63) / 64;
    const size_t lds = glcm::block_lds_bytes(p->N, ba.fb_copies);
    const int per_cu =
        std::max(1, std::min((int)(((size_t)p->lds_budget_words * 4u + 1024u) / lds), 32 / kWaves));
    int nregions = std::min(rows, std::max(1, p->num_cus * per_cu));
    nregions = std::max(1, std::min(nregions, rows * spans / (4 * kWaves)));
    int region_rows = (rows + nregions - 1) / nregions;
    region_rows = std::min(region_rows, std::max(1, 131070 / (spans * 1024)));
    nregions = (rows + region_rows - 1) / region_rows;
    const int strips_per_span = std::max(1, kWaves / spans);
    ba.nregions = nregions;
    ba.region_rows = region_rows;
    ba.strip_rows = std::max(1, (region_rows + strips_per_span - 1) / strips_per_span);
    glcm::LaunchTiming tm;
    if (p->flags & GLCM_FLAG_TIMING) {
      GLCM_TRY(hipEventCreate(&tm.start));
      GLCM_TRY(hipEventCreate(&tm.stop));
      p->timing.emplace_back(tm.start, tm.stop);
    }
    const uint32_t nslots = p->xslots;
    hipError_t e = glcm::launch_vote_blocks(ba, b, kWg, stream, tm);
    if (e == hipSuccess && finish) e = glcm::launch_finish(p->xbuf, out, words, nslots, accumulate, stream);
    if (e != hipSuccess) {
      (void)glcm::launch_zero(p->xbuf, (uint64_t)nslots * words, stream);
      return hip_status(e);
    }
    return GLCM_OK;
  }

  int R = t.replicas, P = t.partitions;  // R may drop below if 16-bit counters cannot be used
  if (path != t.path && (path == kPathGeneric || path == kPathPartitioned)) {
    // fell back from the row kernel: size the generic partitions
    const uint64_t budget = (uint64_t)p->lds_budget_words;
    P = (int)((words + budget - 1) / budget);
    R = 1;
    while (R < 16 && ((uint64_t)words * 2 * R + budget - 1) / budget <= (uint64_t)P) R *= 2;
  }
  // generic kernel over two or more bin partitions with one copy: 16-bit
  // counters, two words per dword, halve the partitions (each band is then
  // kept below 2^16 first pixels, the most one counter can receive, which
  // needs rows of at most 65535 pixels)
  bool g16 = false;
  if ((path == kPathGeneric || path == kPathPartitioned) && t.counter_bits == 16 && P >= 2 && R == 1 && xcd &&
      W <= 65535) {
    const uint64_t budget = (uint64_t)p->lds_budget_words;
    const int P16 = (int)(((uint64_t)words + 2 * budget - 1) / (2 * budget));
    P = (p->flags & GLCM_FLAG_FORCE_PARTITIONED) ? std::max(P16, P) : P16;  // forced: keep the passes
    g16 = true;
  }
  int log2R = 0;
  while ((1 << log2R) < R) ++log2R;
  a.log2R = log2R;
  const int rpw = 4;
  // strip kernel: layout, template reach (1, 2 or 4) and workgroup size
  StripLayout sl;
  const int smd = strip_reach(c);
  if (path == kPathStrips) {
    const int swg = std::min(t.wg_size, glcm::strip_max_threads(b, smd));
    if (!strip_layout(p, W, y_end - y_begin, R, t.counter_bits == 16, swg, &sl))
      return GLCM_EINVAL;  // tunings are validated when set
    a.kp = sl.kp;
    a.kg = sl.kg;
    a.c16 = sl.pair;
    a.merge_pack = sl.pack;
    a.part_words = (uint32_t)sl.kp * NN;
    a.P = sl.P;
    a.pitch = (uint32_t)p->N + 1u;
    for (int k = 0; k < p->K; ++k) {
      a.dx[k] = c.dx[k];
      a.dy[k] = c.dy[k];
      a.vcode[k] = c.dy[k] * (2 * smd + 1) + c.dx[k] + smd;
    }
    a.tmask = c.tmask;
  } else if (path == kPathRows) {
    const uint32_t per = (uint32_t)p->K / (uint32_t)P + ((uint32_t)p->K % (uint32_t)P ? 1u : 0u);
    a.part_words = per * NN;
    a.P = (int)((p->K + per - 1) / per);
    for (int k = 0; k < p->K; ++k) {
      a.dx[k] = c.dx[k];
      a.dy[k] = c.dy[k];
    }
    a.tmask = c.tmask;
  } else {
    a.part_words = (words + (uint32_t)P - 1) / (uint32_t)P;
    a.P = P;
    for (int k = 0; k < p->K; ++k) {
      a.dx[k] = p->offsets[k].dx;
      a.dy[k] = p->offsets[k].dy;
    }
  }

  // Row bands: as many workgroups per partition as the CUs hold at once
  // (limited by LDS and by 32 wavefronts per CU).
  const int rows = y_end - y_begin;
  const int wg = path == kPathStrips ? std::min(t.wg_size, glcm::strip_max_threads(b, smd))
                 : path == kPathRows ? std::min(t.wg_size, glcm::rows_max_threads(b, c.maxdy, a.unaligned != 0))
                                     : t.wg_size;
  const int nwaves = wg / 64;
  if (g16) a.c16 = 1;
  size_t lds_need = g16 ? (size_t)((a.part_words + 1u) / 2u) * 4u : ((size_t)a.part_words << log2R) * 4u;
  if (path == kPathRows)
    lds_need = (size_t)(a.part_words / NN) * row_glcm_dwords(p->N, R, t.counter_bits == 16 ? 16 : 32) * 4u;
  lds_need = std::max(lds_need, (size_t)wg * 4u);
  const int per_cu = std::max(1, std::min((int)(((size_t)p->lds_budget_words * 4u + 1024u) / lds_need), 32 / nwaves));
  int target_groups = std::max(1, p->num_cus * per_cu / a.P);
  int nregions = std::min(rows, target_groups);
  // keep partials within 256 MiB
  while (nregions > 1 && (uint64_t)nregions * words * 4ull > (256ull << 20)) nregions = (nregions + 1) / 2;
  int region_rows = (rows + nregions - 1) / nregions;
  nregions = (rows + region_rows - 1) / region_rows;
  if (path == kPathStrips) {
    nregions = sl.nregions;
    region_rows = sl.region_rows;
    a.strip_rows = sl.strip_rows;
  }
  if (g16 && (uint64_t)region_rows * (uint64_t)W > 65535u) {
    region_rows = std::max(1, 65535 / W);
    nregions = (rows + region_rows - 1) / region_rows;
  }
  a.nregions = nregions;
  a.region_rows = region_rows;
  a.rows_per_wave = rpw;

  if (xcd) {
    a.xbuf = p->xbuf;
  } else {
    int rc = ensure_partials(p, (size_t)a.nregions * words * 4u);
    if (rc != GLCM_OK) return rc;
    a.partials = p->partials;
  }

  // LDS: the copies (at least one word per thread)
  size_t lds_bytes = g16 ? (size_t)((a.part_words + 1u) / 2u) * 4u : ((size_t)a.part_words << log2R) * 4u;
  if (path == kPathRows) {
    // 16-bit counters only when no count can reach 2^16: each slab gives a
    // copy at most 64 lanes / R x 16 pixels x 4 rows votes into one bin.
    int bits = t.counter_bits == 16 && R >= 2 ? 16 : 32;
    const uint64_t chunks = ((uint64_t)W + 15) / 16, spans = (chunks + 63) / 64;
    const uint64_t slabs = spans * (((uint64_t)a.region_rows + rpw - 1) / rpw);
    if (bits == 16 && slabs * 4096u / (uint64_t)R > 65535u) {
      bits = 32;  // same LDS footprint with half the copies
      R /= 2;
      a.log2R -= 1;
    }
    a.c16 = bits == 16 ? 1 : 0;
    a.pitch = row_pitch(p->N);
    lds_bytes = (size_t)(a.part_words / NN) * row_glcm_dwords(p->N, R, bits) * 4u;
  }
  if (path == kPathStrips) lds_bytes = sl.lds;
  lds_bytes = std::max(lds_bytes, (size_t)wg * 4u);

  const int maxdy = c.maxdy <= 1 ? 1 : (c.maxdy <= 2 ? 2 : 4);
  glcm::LaunchTiming tm;
  if (p->flags & GLCM_FLAG_TIMING) {
    // the dispatch stamps the events with the kernel's own start and end
    GLCM_TRY(hipEventCreate(&tm.start));
    GLCM_TRY(hipEventCreate(&tm.stop));
    p->timing.emplace_back(tm.start, tm.stop);
  }
  hipError_t e;
  if (path == kPathStrips) {
    e = glcm::launch_vote_strips(a, b, smd, sl.D, wg, lds_bytes, stream, tm);
  } else if (path == kPathRows) {
    e = glcm::launch_vote_rows(a, b, maxdy, rpw, wg, lds_bytes, stream, tm);
  } else {
    e = glcm::launch_vote_generic(a, b, wg, lds_bytes, stream, tm);
  }
  if (e == hipSuccess) {
    if (!xcd)
      e = glcm::launch_reduce(a.partials, out, words, a.nregions, accumulate, stream);
    else if (finish)
      e = glcm::launch_finish(p->xbuf, out, words, p->xslots, accumulate, stream);
  }
  if (e != hipSuccess) {
    // leave the accumulators clean for the next call
    if (xcd) (void)glcm::launch_zero(p->xbuf, (uint64_t)p->xslots * words, stream);
    return hip_status(e);
  }
  return GLCM_OK;
}

// Host-resident image: uploads it in tiles of `tile_rows` first-pixel rows,
// each with the halo rows its offsets reach (the 2-D form of the chunk bounds
// of Eq. (7)-(9): a tile owns the pairs whose first pixel lies in its rows,
// or, on the kernels that count an upward offset as its opposite, whose upper
// pixel does),
// through two pinned staging slots and two device tile buffers.  Copies run on
// the plan's upload stream and counting on `stream`, so the upload of tile
// t+1 overlaps the counting of tile t (Section III); tile results are summed
// into `out` by the reduce step.  With GLCM_FLAG_SERIAL_UPLOAD everything runs
// on `stream` (no overlap).  Returns once the last upload is queued.
int count_host(glcm_plan_t p, const void* img, bool pinned, int W, int H, int64_t stride, uint32_t lo, uint32_t hi,
               uint32_t* out, hipStream_t stream) {
  const int b = dtype_bytes(p->dtype);
  const Canon c = canonicalize(p->offsets, p->K);
  // Halo rows: the generic, partitioned, L2 and global kernels pair a first
  // pixel in the tile with the pixel dy rows away, so they need max(-dy)
  // rows above and max(dy) below; the strip and slab kernels count an offset
  // with dy < 0 as its opposite from the upper pixel, so they need max|dy|
  // rows below.  The tile carries both (extra rows are never first pixels).
  const int up = std::min(c.up, H), down = std::min(std::max(c.down, c.maxdy), H);
  const int T = std::max(1, p->tuning.tile_rows);
  const bool serial = (p->flags & GLCM_FLAG_SERIAL_UPLOAD) != 0;
  // device rows padded to 256 bytes so the row kernel's alignment holds
  const size_t pitch_bytes = (((size_t)W * b) + 255) / 256 * 256;
  const int max_rows = std::min(H, T + up + down);
  const size_t slot_bytes = pitch_bytes * (size_t)max_rows;
  if (slot_bytes > p->tile_bytes) {
    if (p->has_done) GLCM_TRY(hipEventSynchronize(p->done));
    if (p->copy_stream) GLCM_TRY(hipStreamSynchronize(p->copy_stream));
    for (int s = 0; s < glcm_plan_s::kSlots; ++s) {
      if (p->dev_tile[s]) GLCM_TRY(hipFree(p->dev_tile[s]));
      if (p->pin_tile[s]) GLCM_TRY(hipHostFree(p->pin_tile[s]));
      p->dev_tile[s] = p->pin_tile[s] = nullptr;
      p->pin_pending[s] = false;
    }
    p->tile_bytes = 0;
    for (int s = 0; s < glcm_plan_s::kSlots; ++s) {
      GLCM_TRY(hipMalloc(&p->dev_tile[s], slot_bytes));
      GLCM_TRY(hipHostMalloc(&p->pin_tile[s], slot_bytes, hipHostMallocDefault));
      if (!p->uploaded[s]) GLCM_TRY(hipEventCreateWithFlags(&p->uploaded[s], hipEventDisableTiming));
      if (!p->consumed[s]) GLCM_TRY(hipEventCreateWithFlags(&p->consumed[s], hipEventDisableTiming));
    }
    p->tile_bytes = slot_bytes;
  }
  if (!p->copy_stream) GLCM_TRY(hipStreamCreateWithFlags(&p->copy_stream, hipStreamNonBlocking));
  hipStream_t cs = serial ? stream : p->copy_stream;
  // the previous call on this plan may still read the device tile buffers
  if (p->has_done && !serial) GLCM_TRY(hipStreamWaitEvent(cs, p->done, 0));
  const char* src = (const char*)img;
  const size_t row_bytes = (size_t)W * b, src_pitch = (size_t)stride * b;
  bool slot_used[glcm_plan_s::kSlots] = {false, false};
  int tile = 0;
  for (int r0 = 0; r0 < H; r0 += T, ++tile) {
    const int r1 = std::min(H, r0 + T);
    const int ra = std::max(0, r0 - up), rb = std::min(H, r1 + down);
    const int rows = rb - ra;
    const int s = tile % glcm_plan_s::kSlots;
    char* dev = (char*)p->dev_tile[s];
    // the device slot is free once the count that read it has run
    if (slot_used[s] && !serial) GLCM_TRY(hipStreamWaitEvent(cs, p->consumed[s], 0));
    if (pinned) {
      GLCM_TRY(hipMemcpy2DAsync(dev, pitch_bytes, src + (size_t)ra * src_pitch, src_pitch, row_bytes, rows,
                                hipMemcpyHostToDevice, cs));
    } else {
      // the staging slot is free once its previous upload (of this call or of
      // an earlier one) has completed
      if (p->pin_pending[s]) GLCM_TRY(hipEventSynchronize(p->uploaded[s]));
      char* pin = (char*)p->pin_tile[s];
      for (int y = 0; y < rows; ++y)
        std::memcpy(pin + (size_t)y * pitch_bytes, src + (size_t)(ra + y) * src_pitch, row_bytes);
      GLCM_TRY(hipMemcpyAsync(dev, pin, pitch_bytes * rows, hipMemcpyHostToDevice, cs));
    }
    GLCM_TRY(hipEventRecord(p->uploaded[s], cs));
    p->pin_pending[s] = !pinned;
    if (!serial) GLCM_TRY(hipStreamWaitEvent(stream, p->uploaded[s], 0));
    const bool last = r1 >= H;
    const bool xcd = p->tuning.merge == 0 && p->xbuf != nullptr;
    int rc = count_device(p, dev, W, rows, (int64_t)(pitch_bytes / b), r0 - ra, r1 - ra, lo, hi, out,
                          xcd ? false : tile > 0, xcd ? last : true, stream);
    if (rc != GLCM_OK) return rc;
    GLCM_TRY(hipEventRecord(p->consumed[s], stream));
    slot_used[s] = true;
  }
  return GLCM_OK;
}

size_t plan_device_bytes(const glcm_plan_s* p) {
  size_t b = p->partials_bytes + p->batch_cap + p->stage_bytes;
  if (p->xbuf) b += (size_t)glcm::kXcdSlots * (size_t)p->k_cap * p->N * p->N * 4u;
  for (int s = 0; s < glcm_plan_s::kSlots; ++s)
    if (p->dev_tile[s]) b += p->tile_bytes;
  return b;
}

// Plans made for calls with plan = NULL, one per (device, dtype, N, K,
// offsets), kept for reuse but bounded: at most kCachePlans plans and
// kCacheBytes of device workspace.  When a call ends over a bound, idle plans
// (no call using them) go, least recently used first; a plan in use is never
// destroyed, so the bounds can be exceeded while many calls run at once.
class PlanCache {
 public:
  using Key = std::tuple<int, int, int, int, std::vector<int32_t>>;
  static constexpr size_t kCachePlans = 32;
  static constexpr size_t kCacheBytes = 512ull << 20;

  // The cached plan for `key` (made by `make` if absent), marked in use until
  // release(); GLCM_OK or make's error.
  template <class Make>
  int acquire(const Key& key, Make make, glcm_plan_t* out) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = map_.find(key);
    if (it == map_.end()) {
      glcm_plan_t np = nullptr;
      const int rc = make(&np);
      if (rc != GLCM_OK) return rc;
      it = map_.emplace(key, Entry{np, 0, 0, plan_device_bytes(np)}).first;
    }
    it->second.users += 1;
    it->second.last_use = ++tick_;
    *out = it->second.plan;
    return GLCM_OK;
  }

  // Ends a use of `p`, then trims the cache to its bounds.
  void release(glcm_plan_t p) {
    std::vector<glcm_plan_t> gone;
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (auto& kv : map_)
        if (kv.second.plan == p) {
          kv.second.users -= 1;
          if (kv.second.users == 0) kv.second.bytes = plan_device_bytes(p);
          break;
        }
      trim_locked(kCachePlans, kCacheBytes, &gone);
    }
    destroy(gone);
  }

  // Destroys every idle plan.
  void clear() {
    std::vector<glcm_plan_t> gone;
    {
      std::lock_guard<std::mutex> lk(mu_);
      trim_locked(0, 0, &gone);
    }
    destroy(gone);
  }

  void stats(int* plans, uint64_t* bytes) {
    std::lock_guard<std::mutex> lk(mu_);
    uint64_t b = 0;
    for (const auto& kv : map_) b += kv.second.bytes;
    if (plans) *plans = (int)map_.size();
    if (bytes) *bytes = b;
  }

 private:
  struct Entry {
    glcm_plan_t plan;
    int users;
    uint64_t last_use;
    size_t bytes;  // device workspace when last idle
  };

  void trim_locked(size_t max_plans, size_t max_bytes, std::vector<glcm_plan_t>* gone) {
    for (;;) {
      size_t bytes = 0;
      for (const auto& kv : map_) bytes += kv.second.bytes;
      if (map_.size() <= max_plans && bytes <= max_bytes) return;
      auto victim = map_.end();
      for (auto it = map_.begin(); it != map_.end(); ++it)
        if (it->second.users == 0 && (victim == map_.end() || it->second.last_use < victim->second.last_use))
          victim = it;
      if (victim == map_.end()) return;  // everything left is in use
      gone->push_back(victim->second.plan);
      map_.erase(victim);
    }
  }

  // (outside the lock: destroying a plan waits for its queued work)
  static void destroy(const std::vector<glcm_plan_t>& gone) {
    for (glcm_plan_t p : gone) {
      plan_release(p);
      delete p;
    }
  }

  std::mutex mu_;
  std::map<Key, Entry> map_;
  uint64_t tick_ = 0;
};

PlanCache& plan_cache() {
  static PlanCache* c = new PlanCache();  // never destroyed: plans may outlive static destruction order
  return *c;
}

// Holds a cached plan for the duration of one call.
struct CachedPlanUse {
  glcm_plan_t plan = nullptr;
  ~CachedPlanUse() {
    if (plan) plan_cache().release(plan);
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

GLCM_API int glcm_abi_version(void) { return GLCM_ABI_VERSION; }

GLCM_API const char* glcm_strerror(int s) {
  switch (s) {
    case GLCM_OK: return "success";
    case GLCM_EINVAL: return "invalid argument";
    case GLCM_ENOMEM: return "out of memory";
    case GLCM_EUNSUPPORTED: return "unsupported request";
    case GLCM_EHIP: return "HIP runtime error";
    case GLCM_EBUSY: return "busy";
    default: return "unknown status";
  }
}

GLCM_API int glcm_last_hip_error(void) { return g_last_hip; }

GLCM_API int glcm_offset_polar(int d, int theta_deg, glcm_offset_t* out) {
  if (!out || d < 1 || d > GLCM_MAX_DISPLACEMENT || theta_deg < 0 || theta_deg >= 360 || theta_deg % 45)
    return GLCM_EINVAL;
  // Eq. (2): 0, 45, 90, 135 degrees move the second pixel by +d, +d(W-1),
  // +dW, +d(W+1) elements in row-major order.
  static const int ux[8] = {1, -1, 0, 1, -1, 1, 0, -1};
  static const int uy[8] = {0, 1, 1, 1, 0, -1, -1, -1};
  const int i = theta_deg / 45;
  out->dx = ux[i] * d;
  out->dy = uy[i] * d;
  return GLCM_OK;
}

GLCM_API int glcm_plan_create(glcm_plan_t* plan, int dtype, int N, int K, const glcm_offset_t* offsets, int max_W,
                     int max_H, uint32_t flags) {
  if (!plan) return GLCM_EINVAL;
  *plan = nullptr;
  if (dtype_bytes(dtype) == 0 || N < 1 || N > GLCM_MAX_LEVELS) return GLCM_EINVAL;
  if (check_offsets(offsets, K) != GLCM_OK) return GLCM_EINVAL;
  if (max_W < 1 || max_H < 1 || (uint64_t)max_W * (uint64_t)max_H > 0xffffffffull) return GLCM_EINVAL;
  if (flags & ~kKnownFlags) return GLCM_EINVAL;
  std::unique_ptr<glcm_plan_s> p(new (std::nothrow) glcm_plan_s());
  if (!p) return GLCM_ENOMEM;
  p->dtype = dtype;
  p->N = N;
  p->K = K;
  p->k_cap = K;
  std::memcpy(p->offsets, offsets, sizeof(glcm_offset_t) * K);
  p->max_W = max_W;
  p->max_H = max_H;
  p->flags = flags;
  int rc = plan_init(p.get());
  if (rc != GLCM_OK) {
    plan_release(p.get());
    return rc;
  }
  *plan = p.release();
  return GLCM_OK;
}

GLCM_API int glcm_plan_tuning(glcm_plan_t plan, glcm_tuning_t* tuning, int set) {
  if (!plan || !tuning) return GLCM_EINVAL;
  std::lock_guard<std::mutex> lk(plan->mu);
  if (set) {
    const glcm_tuning_t& n = *tuning;
    if (n.replicas < 1 || n.replicas > 64 || (n.replicas & (n.replicas - 1))) return GLCM_EINVAL;
    if (n.wg_size != 256 && n.wg_size != 512 && n.wg_size != 1024) return GLCM_EINVAL;
    if (n.rows_per_wave < 0 || n.rows_per_wave > 65536) return GLCM_EINVAL;
    if (n.tile_rows < 1 || n.tile_rows > 65536) return GLCM_EINVAL;
    const uint32_t NN = (uint32_t)plan->N * (uint32_t)plan->N;
    glcm_tuning_t& t = plan->tuning;
    if (n.counter_bits != 0 && n.counter_bits != 16 && n.counter_bits != 32) return GLCM_EINVAL;
    int bits = n.counter_bits == 0 ? t.counter_bits : n.counter_bits;
    // the two row-kernel families may be swapped where the offsets allow both
    // (the slab height then takes its default, 4)
    int path = t.path;
    const bool row_family = t.path == kPathStrips || t.path == kPathRows;
    if (row_family && n.path != t.path && (n.path == kPathStrips || n.path == kPathRows)) {
      const Canon c = canonicalize(plan->offsets, plan->K);
      if (!(n.path == kPathStrips ? strips_eligible(plan, c) : slabs_eligible(plan, c))) return GLCM_EINVAL;
      path = n.path;
    }
    int parts = t.partitions, new_path = path;
    const int rpw = path == t.path ? n.rows_per_wave : (path == kPathRows ? 4 : 0);
    if (path == kPathBlocks) {
      // the block kernel's layout is fixed (32 copies, 16-bit halves, 1024
      // threads); only the upload tile height and the merge are tunable
      if (n.wg_size != 1024 || n.rows_per_wave != 0) return GLCM_EINVAL;
      if (n.replicas != 32 || bits != 16) return GLCM_EINVAL;
    } else if (path == kPathStrips) {
      if (rpw != 0) return GLCM_EINVAL;  // strips have no slab height
      const int P = strip_partitions(plan, n.replicas, bits);
      if (P == 0) return GLCM_EINVAL;
      parts = P;
    } else if (path == kPathRows) {
      // partitions are groups of whole GLCMs; the copies must fit one
      if (bits == 16 && n.replicas < 2) return GLCM_EINVAL;
      if (rpw != 0 && rpw != 4) return GLCM_EINVAL;
      const int P = row_partitions(plan, n.replicas, bits);
      if (P == 0) return GLCM_EINVAL;
      parts = P;
    } else if (t.path != kPathGlobal && t.path != kPathL2) {
      if (bits == 16 && n.replicas != 1) return GLCM_EINVAL;  // 16-bit bins: one copy
      const uint64_t words = (uint64_t)plan->K * NN;
      if ((uint64_t)n.replicas > (uint64_t)plan->lds_budget_words) return GLCM_EINVAL;
      const uint64_t cap = (uint64_t)plan->lds_budget_words / n.replicas;
      parts = (int)((words + cap - 1) / cap);
      if (parts > 1) new_path = kPathPartitioned;
    }
    if (n.merge != 0 && n.merge != 1) return GLCM_EINVAL;
    if (n.merge == 0 && !plan->xbuf && t.path != kPathGlobal) return GLCM_EINVAL;
    t.counter_bits = bits;
    t.merge = n.merge;
    t.replicas = n.replicas;
    t.wg_size = n.wg_size;
    t.partitions = parts;
    if (path != t.path) {
      t.rows_per_wave = rpw;
    } else if (t.path == kPathRows && n.rows_per_wave != 0) {
      t.rows_per_wave = n.rows_per_wave;
    }
    t.path = new_path;
    t.tile_rows = n.tile_rows;
    plan->user_tuned = true;
  }
  *tuning = plan->tuning;
  return GLCM_OK;
}

GLCM_API int glcm_plan_autotune(glcm_plan_t plan, const void* img, int W, int H, int64_t stride, uint32_t lo,
                                uint32_t hi, int repeats, void* stream_, glcm_tuning_t* chosen) {
  if (!plan || !img || W < 1 || H < 1 || stride < W || W > plan->max_W || H > plan->max_H) return GLCM_EINVAL;
  if (repeats < 1 || repeats > 1000) return GLCM_EINVAL;
  if (lo > hi || hi > (plan->dtype == GLCM_U8 ? 255u : 65535u)) return GLCM_EINVAL;
  if (((uintptr_t)img) % (uintptr_t)dtype_bytes(plan->dtype)) return GLCM_EINVAL;
  int dev = -1;
  if (pointer_kind(img, &dev) != 2) return GLCM_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  std::lock_guard<std::mutex> lk(plan->mu);
  const glcm_tuning_t start = plan->tuning;
  if (start.path == kPathGlobal) {
    if (chosen) *chosen = start;
    return GLCM_OK;
  }
  // candidates: copies x counter width x workgroup size, within 4x the
  // minimal number of partitions
  // (the plan's own tuning first: a later candidate must beat it by 3%)
  std::vector<glcm_tuning_t> cand{start};
  auto add = [&](const glcm_tuning_t& t) {
    for (const glcm_tuning_t& u : cand)
      if (u.path == t.path && u.replicas == t.replicas && u.counter_bits == t.counter_bits &&
          u.partitions == t.partitions && u.wg_size == t.wg_size && u.rows_per_wave == t.rows_per_wave &&
          u.merge == t.merge)
        return;
    cand.push_back(t);
  };
  const Canon cn = canonicalize(plan->offsets, plan->K);
  if (start.path == kPathBlocks) {
    // forced by GLCM_FLAG_FORCE_BLOCKS: its layout is fixed
  } else if (start.path == kPathStrips || start.path == kPathRows) {
    // both row-kernel families wherever the offsets allow them
    if (strips_eligible(plan, cn)) {
      const int Pmin = strip_partitions(plan, 4, 16);
      for (int bits : {32, 16})
        for (int R = 4; R <= 32; R *= 2) {
          const int P = strip_partitions(plan, R, bits);
          if (P == 0 || P > 4 * Pmin) continue;
          for (int wg : {512, 1024}) {
            glcm_tuning_t t = start;
            t.path = kPathStrips;
            t.rows_per_wave = 0;
            t.replicas = R;
            t.counter_bits = bits;
            t.partitions = P;
            t.wg_size = wg;
            add(t);
          }
        }
    }
    if (slabs_eligible(plan, cn)) {
      const int Pmin = row_partitions(plan, 1, 32);
      for (int bits : {32, 16})
        for (int R = bits == 16 ? 2 : 1; R <= 64; R *= 2) {
          const int P = row_partitions(plan, R, bits);
          if (P == 0 || P > 4 * Pmin) continue;
          for (int wg : {512, 1024}) {
            glcm_tuning_t t = start;
            t.path = kPathRows;
            t.rows_per_wave = 4;
            t.replicas = R;
            t.counter_bits = bits;
            t.partitions = P;
            t.wg_size = wg;
            add(t);
          }
        }
    }
    // the block-code kernel, where every offset is a d = 1 direction: faster
    // on smooth images, slower where most 2x2 blocks leave its code window
    // (noise), which is what the timing decides
    if (plan->xbuf && blocks_fit(plan) && row_kernels_ok(plan) && !(plan->flags & GLCM_FLAG_FORCE_SLABS)) {
      glcm_tuning_t t = start;
      t.path = kPathBlocks;
      t.rows_per_wave = 0;
      t.replicas = 32;
      t.counter_bits = 16;
      t.partitions = 1;
      t.wg_size = 1024;
      t.merge = 0;
      add(t);
    }
  } else {
    const uint64_t words = (uint64_t)plan->K * plan->N * plan->N, budget = (uint64_t)plan->lds_budget_words;
    for (int R = 1; R <= 16; R *= 2) {
      const uint64_t P = (words * R + budget - 1) / budget;
      for (int bits : {32, 16}) {
        if (bits == 16 && (R != 1 || P < 2)) continue;  // 16-bit bins: one copy, several passes
        if ((bits == 16 ? (P + 1) / 2 : P) > (uint64_t)kPassesPerSliceGlcm * (uint64_t)plan->K) continue;
        for (int wg : {256, 512, 1024}) {
          glcm_tuning_t t = start;
          t.replicas = R;
          t.partitions = (int)P;
          t.path = P > 1 ? kPathPartitioned : kPathGeneric;
          t.counter_bits = bits;
          t.wg_size = wg;
          add(t);
        }
      }
    }
    if (plan->xbuf && l2_slices_fit(plan)) {  // no LDS copies: pairs straight into the XCD slices
      glcm_tuning_t t = start;
      t.path = kPathL2;
      t.replicas = 1;
      t.partitions = 1;
      t.merge = 0;
      add(t);
    }
  }
  const size_t words = (size_t)plan->K * plan->N * plan->N;
  uint32_t* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  GLCM_TRY(hipMalloc((void**)&out, words * 4u));
  int rc = GLCM_OK;
  float best = 0.f;
  glcm_tuning_t best_t = start;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) rc = hip_status(he);
  if (rc == GLCM_OK) rc = order_after_previous(plan, stream);
  for (size_t c = 0; c < cand.size() && rc == GLCM_OK; ++c) {
    plan->tuning = cand[c];
    for (int i = 0; i < 2 && rc == GLCM_OK; ++i)
      rc = count_device(plan, img, W, H, stride, 0, H, lo, hi, out, false, true, stream);
    if (rc != GLCM_OK) break;
    if ((he = hipEventRecord(e0, stream)) != hipSuccess) { rc = hip_status(he); break; }
    for (int i = 0; i < repeats && rc == GLCM_OK; ++i)
      rc = count_device(plan, img, W, H, stride, 0, H, lo, hi, out, false, true, stream);
    if (rc != GLCM_OK) break;
    if ((he = hipEventRecord(e1, stream)) != hipSuccess || (he = hipEventSynchronize(e1)) != hipSuccess) {
      rc = hip_status(he);
      break;
    }
    float ms = 0.f;
    if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { rc = hip_status(he); break; }
    // a later candidate must win by 3% to replace the kept one, so near ties
    // resolve the same way from run to run
    if (c == 0 || ms < 0.97f * best) {
      best = ms;
      best_t = cand[c];
    }
  }
  if (rc == GLCM_OK) rc = record_done(plan, stream);
  (void)hipStreamSynchronize(stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  plan->tuning = rc == GLCM_OK ? best_t : start;
  if (rc == GLCM_OK) plan->user_tuned = true;
  if (chosen) *chosen = plan->tuning;
  return rc;
}

GLCM_API int glcm_plan_kernel_time(glcm_plan_t plan, double* ms_total, int* launches) {
  if (!plan || !ms_total || !launches) return GLCM_EINVAL;
  std::lock_guard<std::mutex> lk(plan->mu);
  double sum = 0.0;
  int n = 0, rc = GLCM_OK;
  for (auto& ev : plan->timing) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(ev.second);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.first, ev.second);
    if (e != hipSuccess && rc == GLCM_OK) rc = hip_status(e);
    sum += ms;
    ++n;
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  plan->timing.clear();
  *ms_total = sum;
  *launches = n;
  return rc;
}

GLCM_API int glcm_plan_rebind(glcm_plan_t plan, const glcm_offset_t* offsets, int K) {
  if (!plan || check_offsets(offsets, K) != GLCM_OK || K > plan->k_cap) return GLCM_EINVAL;
  std::lock_guard<std::mutex> lk(plan->mu);
  // queued launches took their offsets by value; the XCD slices are zero
  // between calls whatever K, so only the host-side layout changes
  plan->K = K;
  std::memcpy(plan->offsets, offsets, sizeof(glcm_offset_t) * K);
  plan->user_tuned = false;
  glcm_tuning_t t{};
  const int rc = choose_tuning(plan, &t);
  if (rc != GLCM_OK) return rc;
  if (t.path != kPathGlobal && !plan->xbuf) t.merge = 1;
  plan->tuning = t;
  return GLCM_OK;
}

GLCM_API int glcm_plan_workspace(glcm_plan_t plan, size_t* device_bytes) {
  if (!plan || !device_bytes) return GLCM_EINVAL;
  std::lock_guard<std::mutex> lk(plan->mu);
  *device_bytes = plan_device_bytes(plan);
  return GLCM_OK;
}

GLCM_API int glcm_plan_cache_stats(int* plans, uint64_t* device_bytes) {
  plan_cache().stats(plans, device_bytes);
  return GLCM_OK;
}

GLCM_API int glcm_plan_cache_clear(void) {
  plan_cache().clear();
  return GLCM_OK;
}

GLCM_API int glcm_plan_destroy(glcm_plan_t plan) {
  if (!plan) return GLCM_OK;
  plan_release(plan);
  delete plan;
  return GLCM_OK;
}

extern "C++" {
namespace glcm {

int compute_in_workspace(uint32_t* slices, size_t slice_words, const void* img, int W, int H, int64_t stride,
                         int dtype, int N, uint32_t lo, uint32_t hi, const glcm_offset_t* offsets, int K,
                         uint32_t* out, hipStream_t stream) {
  int rc = check_compute_args(img, W, H, stride, dtype, N, lo, hi, offsets, K, out);
  if (rc != GLCM_OK) return rc;
  const uint64_t words = (uint64_t)K * (uint64_t)N * (uint64_t)N;
  if (!slices || (uint64_t)kXcdSlots * words > (uint64_t)slice_words) return GLCM_EINVAL;
  int out_dev = -1, img_dev = -1, cur = 0;
  if (pointer_kind(out, &out_dev) != 2 || pointer_kind(img, &img_dev) != 2) return GLCM_EINVAL;
  GLCM_TRY(hipGetDevice(&cur));
  if (out_dev != cur || img_dev != cur) return GLCM_EINVAL;
  // a plan for this one call: no events, no workspace of its own
  glcm_plan_s p;
  p.device = cur;
  p.dtype = dtype;
  p.N = N;
  p.K = K;
  p.k_cap = K;
  std::memcpy(p.offsets, offsets, sizeof(glcm_offset_t) * (size_t)K);
  p.max_W = W;
  p.max_H = H;
  int lds = 0;
  GLCM_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, cur));
  GLCM_TRY(hipDeviceGetAttribute(&p.num_cus, hipDeviceAttributeMultiprocessorCount, cur));
  p.lds_budget_words = (lds - 1024) / 4;
  choose_tuning(&p, &p.tuning);
  p.tuning.merge = 0;  // the slices, never band partials
  p.xbuf = slices;
  p.xslots = kXcdSlots;
  p.no_alloc = true;
  // the slices start at zero whatever an earlier call left (a fill kernel:
  // the call stays capturable in a graph)
  GLCM_TRY(launch_zero(slices, (uint64_t)kXcdSlots * words, stream));
  return count_device(&p, img, W, H, stride, 0, H, lo, hi, out, false, true, stream);
}

}  // namespace glcm
}  // extern "C++"

GLCM_API int glcm_compute(glcm_plan_t plan, const void* img, int W, int H, int64_t stride, int dtype, int N, uint32_t lo,
                 uint32_t hi, const glcm_offset_t* offsets, int K, uint32_t* out, void* stream_) {
  int rc = check_compute_args(img, W, H, stride, dtype, N, lo, hi, offsets, K, out);
  if (rc != GLCM_OK) return rc;
  hipStream_t stream = (hipStream_t)stream_;
  if (plan) {
    if (plan->dtype != dtype || plan->N != N || plan->K != K ||
        std::memcmp(plan->offsets, offsets, sizeof(glcm_offset_t) * K) != 0 || W > plan->max_W ||
        H > plan->max_H)
      return GLCM_EINVAL;
  }
  int out_dev = -1;
  if (pointer_kind(out, &out_dev) != 2) return GLCM_EINVAL;
  int img_dev = -1;
  const int kind = pointer_kind(img, &img_dev);
  int cur = 0;
  GLCM_TRY(hipGetDevice(&cur));
  if (out_dev != cur || (kind == 2 && img_dev != cur)) return GLCM_EINVAL;

  CachedPlanUse cached;
  if (!plan) {
    std::vector<int32_t> key;
    for (int k = 0; k < K; ++k) {
      key.push_back(offsets[k].dx);
      key.push_back(offsets[k].dy);
    }
    rc = plan_cache().acquire(
        std::make_tuple(cur, dtype, N, K, key),
        [&](glcm_plan_t* np) { return glcm_plan_create(np, dtype, N, K, offsets, 65535, 65535, 0); }, &plan);
    if (rc != GLCM_OK) return rc;
    cached.plan = plan;
  }

  std::lock_guard<std::mutex> lk(plan->mu);
  rc = order_after_previous(plan, stream);
  if (rc != GLCM_OK) return rc;
  if (kind == 2) {
    rc = count_device(plan, img, W, H, stride, 0, H, lo, hi, out, false, true, stream);
  } else {
    rc = count_host(plan, img, kind == 1, W, H, stride, lo, hi, out, stream);
  }
  if (rc != GLCM_OK) return rc;
  return record_done(plan, stream);
}

namespace {

// What a batch launch needs besides lo, hi and the output pointers.
struct BatchLayout {
  int D = 0, smd = 1, b = 1, wg = glcm::kBatchThreads;
  size_t lds_bytes = 0;
  int groups = 0;  // persistent workgroups: as many as the CUs hold at once
  glcm::BatchArgs args{};  // offsets, codes and layout; quantizer and outputs filled per launch
};

// Checks a batch request against the plan and picks its LDS layout.
// The default LDS layout of the batch kernel: the most dwords per bin (16, 8
// or 4) that leave room for two workgroups per CU (measured on MI355X with
// the persistent kernel, 4096 images of 32-512 px, N = 16, K = 4: 16 copies
// and two workgroups per CU 245 us, 8 copies and three 287 us).
int batch_default_copies(const glcm_plan_s* plan) {
  const size_t lds_cu = (size_t)plan->lds_budget_words * 4u + 1024u;
  int D = 16;
  while (D > 4 && glcm::batch_lds_bytes(plan->N, plan->K, D) * 2u > lds_cu) D /= 2;
  return D;
}

int batch_layout(glcm_plan_t plan, const glcm_tile_t* tiles, int T, BatchLayout* L) {
  if (!plan || !tiles || T < 1 || T > (1 << 20)) return GLCM_EINVAL;
  const int b = dtype_bytes(plan->dtype);
  for (int t = 0; t < T; ++t) {
    const glcm_tile_t& e = tiles[t];
    if (!e.img || e.W < 1 || e.H < 1 || e.W > plan->max_W || e.H > plan->max_H || e.stride < e.W) return GLCM_EINVAL;
    if ((uint64_t)e.W * (uint64_t)e.H > 0xffffffffull || ((uintptr_t)e.img % (uintptr_t)b)) return GLCM_EINVAL;
  }
  const Canon c = canonicalize(plan->offsets, plan->K);
  if (plan->N > 255 || plan->K > glcm::kStripMaxKp || c.maxdy > 2 || c.maxadx > 2) return GLCM_EUNSUPPORTED;
  const size_t lds_cu = (size_t)plan->lds_budget_words * 4u + 1024u;
  const int D = plan->batch_D ? plan->batch_D : batch_default_copies(plan);
  const size_t lds_bytes = glcm::batch_lds_bytes(plan->N, plan->K, D);
  if (lds_bytes > lds_cu - 1024u) return GLCM_EUNSUPPORTED;
  L->D = D;
  L->b = b;
  L->lds_bytes = lds_bytes;
  L->wg = plan->batch_wg ? plan->batch_wg : glcm::kBatchThreads;
  const int per_cu = std::max(1, std::min((int)(lds_cu / lds_bytes), 32 / (L->wg / 64)));
  L->groups = per_cu * std::max(1, plan->num_cus);
  L->smd = std::max(c.maxdy, c.maxadx) <= 1 ? 1 : 2;
  glcm::BatchArgs& a = L->args;
  std::memset(&a, 0, sizeof(a));
  a.K = plan->K;
  for (int k = 0; k < plan->K; ++k) {
    a.dx[k] = plan->offsets[k].dx;
    a.dy[k] = plan->offsets[k].dy;
    a.vcode[k] = c.dy[k] * (2 * L->smd + 1) + c.dx[k] + L->smd;
  }
  a.tmask = c.tmask;
  a.pitch = (uint32_t)plan->N + 1u;
  a.min_rows = plan->batch_min_rows ? plan->batch_min_rows : kBatchDefaultMinRows;
  return GLCM_OK;
}

bool tile_aligned(const glcm_tile_t& e, int b) {
  return (uintptr_t)e.img % 16u == 0 && ((uint64_t)e.stride * (uint64_t)b) % 16u == 0;
}

// Byte range [first, end) of a tile's pixels.
std::pair<uintptr_t, uintptr_t> tile_extent(const glcm_tile_t& e, int b) {
  const uintptr_t i0 = (uintptr_t)e.img;
  return {i0, i0 + (uintptr_t)(((uint64_t)(e.H - 1) * (uint64_t)e.stride + (uint64_t)e.W) * (uint64_t)b)};
}

// Every tile must lie inside one device allocation of the current device (the
// kernel reads it with plain loads; a host pointer would fault the GPU).
// Allocations are looked up once each (hipMemGetAddressRange), then tiles
// inside a known allocation cost one map lookup.
int check_tile_memory(const glcm_tile_t* tiles, int T, int b) {
  int cur = 0;
  GLCM_TRY(hipGetDevice(&cur));
  std::map<uintptr_t, uintptr_t> known;  // allocation base -> end
  for (int t = 0; t < T; ++t) {
    const auto x = tile_extent(tiles[t], b);
    auto it = known.upper_bound(x.first);
    if (it != known.begin() && x.first >= std::prev(it)->first && x.second <= std::prev(it)->second) continue;
    int dev = -1;
    if (pointer_kind(tiles[t].img, &dev) != 2 || dev != cur) return GLCM_EINVAL;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)tiles[t].img) != hipSuccess) {
      (void)hipGetLastError();
      return GLCM_EINVAL;
    }
    const uintptr_t a0 = (uintptr_t)base, a1 = a0 + size;
    if (x.first < a0 || x.second > a1) return GLCM_EINVAL;
    known[a0] = a1;
  }
  return GLCM_OK;
}

// No tile may overlap [o0, o1) (an output the kernel writes while it reads
// the tiles).
bool tiles_clear_of(const std::vector<std::pair<uintptr_t, uintptr_t>>& ext, uintptr_t o0, uintptr_t o1) {
  for (const auto& x : ext)
    if (x.first < o1 && o0 < x.second) return false;
  return true;
}

// Output pointers of a batch launch: device memory of the current device,
// clear of every tile.
int check_batch_outputs(const std::vector<std::pair<uintptr_t, uintptr_t>>& ext, int T, int K, int N,
                        const uint32_t* out, const float* features) {
  int cur = 0, dev = -1;
  GLCM_TRY(hipGetDevice(&cur));
  if (pointer_kind(out, &dev) != 2 || dev != cur) return GLCM_EINVAL;
  if (features && (pointer_kind(features, &dev) != 2 || dev != cur)) return GLCM_EINVAL;
  const uintptr_t o0 = (uintptr_t)out, o1 = o0 + (uintptr_t)T * (uintptr_t)K * (uintptr_t)N * (uintptr_t)N * 4u;
  if (!tiles_clear_of(ext, o0, o1)) return GLCM_EINVAL;
  if (features) {
    const uintptr_t f0 = (uintptr_t)features, f1 = f0 + (uintptr_t)T * (uintptr_t)K * 5u * 4u;
    if (!tiles_clear_of(ext, f0, f1) || (f0 < o1 && o0 < f1)) return GLCM_EINVAL;
  }
  return GLCM_OK;
}

std::vector<std::pair<uintptr_t, uintptr_t>> tile_extents(const glcm_tile_t* tiles, int T, int b) {
  std::vector<std::pair<uintptr_t, uintptr_t>> ext((size_t)T);
  for (int t = 0; t < T; ++t) ext[(size_t)t] = tile_extent(tiles[t], b);
  return ext;
}

// Work items of a batch: an image of more than kBatchSplitPixels pixels is
// split into bands of about kBatchItemPixels first pixels (whole rows, at
// least kBatchMinBandRows), each counted by its own workgroup into a row of
// partial counts that k_batch_fin sums; the others are one item each.  Items
// go largest first to the persistent workgroups.  Every item costs a fixed
// set-up (its descriptor, its first rows, the merge), so splitting only pays
// for images far larger than the rest: measured on MI355X, 4096 images of
// 32-512 px, splitting those above 64 Ki pixels into bands of 32 Ki made the
// batch 291 us against 245 us whole, though the largest image alone fell
// from 114 to 44 us.
constexpr uint64_t kBatchItemPixels = 1u << 18, kBatchSplitPixels = 1u << 20;
constexpr int kBatchMinBandRows = 8;

constexpr size_t kBatchDescOff = 256;

struct BatchItems {
  std::vector<glcm::BatchTile> items;
  std::vector<glcm::BatchFin> fins;
  int slots = 0;   // band rows of partial counts
  int tables = 0;  // entries of the per-image destination tables (0: one contiguous output)
  // device layout: the item counter (at offset 0 whatever the batch, so a
  // buffer reused for another batch keeps it zero), the items from offset
  // kBatchDescOff, the fins, the destination tables (counts, then
  // statistics), then the partial rows (256-byte aligned)
  size_t fins_off() const { return kBatchDescOff + items.size() * sizeof(glcm::BatchTile); }
  size_t tables_off() const { return (fins_off() + fins.size() * sizeof(glcm::BatchFin) + 7u) & ~(size_t)7u; }
  size_t tables_end() const { return tables_off() + 2u * (size_t)tables * sizeof(void*); }
  size_t partials_off() const { return (tables_end() + 255u) & ~(size_t)255u; }
  size_t desc_bytes() const { return tables_end() - kBatchDescOff; }
  size_t dev_bytes(int K, int N) const { return partials_off() + (size_t)slots * K * N * N * 4u; }
};

void batch_items(const glcm_tile_t* tiles, int T, int b, BatchItems* it) {
  it->items.clear();
  it->fins.clear();
  it->slots = 0;
  it->tables = 0;
  for (int t = 0; t < T; ++t) {
    const glcm_tile_t& e = tiles[t];
    glcm::BatchTile d{};
    d.img = e.img;
    d.stride = e.stride;
    d.W = e.W;
    d.H = e.H;
    d.index = t;
    d.unaligned = tile_aligned(e, b) ? 0 : 1;
    const uint64_t area = (uint64_t)e.W * (uint64_t)e.H;
    int parts = 1;
    if (area > kBatchSplitPixels)
      parts = (int)std::min<uint64_t>((area + kBatchItemPixels - 1) / kBatchItemPixels,
                                      (uint64_t)std::max(1, e.H / kBatchMinBandRows));
    if (parts <= 1) {
      d.y0 = 0;
      d.y1 = e.H;
      d.slot = -1;
      it->items.push_back(d);
      continue;
    }
    const int rp = (e.H + parts - 1) / parts;
    parts = (e.H + rp - 1) / rp;
    it->fins.push_back(glcm::BatchFin{t, it->slots, parts, 0});
    for (int p = 0; p < parts; ++p) {
      d.y0 = p * rp;
      d.y1 = std::min(e.H, (p + 1) * rp);
      d.slot = it->slots + p;
      it->items.push_back(d);
    }
    it->slots += parts;
  }
  std::stable_sort(it->items.begin(), it->items.end(), [](const glcm::BatchTile& x, const glcm::BatchTile& y) {
    return (uint64_t)x.W * (uint64_t)(x.y1 - x.y0) > (uint64_t)y.W * (uint64_t)(y.y1 - y.y0);
  });
}

// Copies the descriptors (items, then fins: desc_bytes() bytes, uploaded to
// offset kBatchDescOff) to `host`.
void batch_descriptors(const BatchItems& it, void* host) {
  const size_t ib = it.items.size() * sizeof(glcm::BatchTile);
  std::memcpy(host, it.items.data(), ib);
  if (!it.fins.empty()) std::memcpy((char*)host + ib, it.fins.data(), it.fins.size() * sizeof(glcm::BatchFin));
}

// Queues the fused batch kernel (and the sum of the split images' bands).
// The item counter (the buffer's first word) must be zero.
int batch_launch(const BatchLayout& L, int nitems, int nfins, size_t fins_off, size_t partials_off,
                 const void* desc_dev, uint32_t N, uint32_t lo, uint32_t hi, uint32_t* out, float* features,
                 hipStream_t stream, uint32_t* const* outs = nullptr, float* const* feats = nullptr) {
  glcm::BatchArgs a = L.args;
  a.q = make_quant((int)N, lo, hi);
  fast_quant(L.b, (int)N, lo, hi, &a.qfast, &a.qfast_shift, &a.qfast_mask);
  a.tiles = (const glcm::BatchTile*)((const char*)desc_dev + kBatchDescOff);
  a.fins = (const glcm::BatchFin*)((const char*)desc_dev + fins_off);
  a.partials = (uint32_t*)((char*)const_cast<void*>(desc_dev) + partials_off);
  a.counter = (uint32_t*)const_cast<void*>(desc_dev);
  a.nitems = nitems;
  a.nfins = nfins;
  a.out = out;
  a.feat = features;
  a.outs = outs;
  a.feats = feats;
  GLCM_TRY(glcm::launch_batch(a, std::min(nitems, L.groups), L.b, L.smd, L.D, L.wg, L.lds_bytes, stream));
  GLCM_TRY(glcm::launch_batch_fin(a, nfins, stream));
  return GLCM_OK;
}

// glcm_batch_compute's work, into one contiguous output (out, features) or,
// with outs set, image t's counts into outs[t] and its statistics into
// feats[t] (feats or feats[t] null: none).
int batch_compute_common(glcm_plan_t plan, const glcm_tile_t* tiles, int T, uint32_t lo, uint32_t hi,
                         uint32_t* out, float* features, uint32_t* const* outs, float* const* feats,
                         hipStream_t stream) {
  if (!plan || !tiles || (!out && !outs) || T < 1 || T > (1 << 20)) return GLCM_EINVAL;  // before touching the plan
  if (lo > hi || hi > (plan->dtype == GLCM_U8 ? 255u : 65535u)) return GLCM_EINVAL;
  if (outs)
    for (int t = 0; t < T; ++t)
      if (!outs[t]) return GLCM_EINVAL;
  std::lock_guard<std::mutex> lk(plan->mu);
  BatchLayout L;
  int rc = batch_layout(plan, tiles, T, &L);
  if (rc != GLCM_OK) return rc;
  GLCM_TRY_RC(check_tile_memory(tiles, T, L.b));
  if (!outs) GLCM_TRY_RC(check_batch_outputs(tile_extents(tiles, T, L.b), T, plan->K, plan->N, out, features));
  GLCM_TRY_RC(order_after_previous(plan, stream));
  BatchItems it;
  batch_items(tiles, T, L.b, &it);
  if (outs) it.tables = T;
  const size_t need = it.dev_bytes(plan->K, plan->N);
  if (plan->batch_pending) GLCM_TRY(hipEventSynchronize(plan->batch_uploaded));
  plan->batch_pending = false;
  if (need > plan->batch_cap) {
    if (plan->batch_pin) GLCM_TRY(hipHostFree(plan->batch_pin));
    if (plan->batch_dev) {
      if (plan->has_done) GLCM_TRY(hipEventSynchronize(plan->done));  // the last batch may still read it
      GLCM_TRY(hipFree(plan->batch_dev));
    }
    plan->batch_pin = plan->batch_dev = nullptr;
    plan->batch_cap = 0;
    GLCM_TRY(hipHostMalloc(&plan->batch_pin, need, hipHostMallocDefault));
    GLCM_TRY(hipMalloc(&plan->batch_dev, need));
    plan->batch_cap = need;
    // the item counter starts at zero (each batch launch leaves it zero again)
    GLCM_TRY(glcm::launch_zero((uint32_t*)plan->batch_dev, need / 4u, stream));
  }
  if (!plan->batch_uploaded) GLCM_TRY(hipEventCreateWithFlags(&plan->batch_uploaded, hipEventDisableTiming));
  batch_descriptors(it, plan->batch_pin);
  uint32_t* const* outs_dev = nullptr;
  float* const* feats_dev = nullptr;
  if (outs) {
    char* tab = (char*)plan->batch_pin + (it.tables_off() - kBatchDescOff);
    std::memcpy(tab, outs, (size_t)T * sizeof(void*));
    if (feats) std::memcpy(tab + (size_t)T * sizeof(void*), feats, (size_t)T * sizeof(void*));
    else std::memset(tab + (size_t)T * sizeof(void*), 0, (size_t)T * sizeof(void*));
    outs_dev = (uint32_t* const*)((char*)plan->batch_dev + it.tables_off());
    if (feats) feats_dev = (float* const*)((char*)plan->batch_dev + it.tables_off() + (size_t)T * sizeof(void*));
  }
  GLCM_TRY(hipMemcpyAsync((char*)plan->batch_dev + kBatchDescOff, plan->batch_pin, it.desc_bytes(),
                           hipMemcpyHostToDevice, stream));
  GLCM_TRY(hipEventRecord(plan->batch_uploaded, stream));
  plan->batch_pending = true;
  GLCM_TRY_RC(batch_launch(L, (int)it.items.size(), (int)it.fins.size(), it.fins_off(), it.partials_off(),
                           plan->batch_dev, (uint32_t)plan->N, lo, hi, out, features, stream, outs_dev, feats_dev));
  return record_done(plan, stream);
}

}  // namespace

extern "C++" {
namespace glcm {

int batch_compute_to(glcm_plan_t plan, const glcm_tile_t* tiles, int T, uint32_t lo, uint32_t hi,
                     uint32_t* const* outs, float* const* feats, hipStream_t stream) {
  if (!outs) return GLCM_EINVAL;
  return batch_compute_common(plan, tiles, T, lo, hi, nullptr, nullptr, outs, feats, stream);
}

}  // namespace glcm
}  // extern "C++"

GLCM_API int glcm_batch_compute(glcm_plan_t plan, const glcm_tile_t* tiles, int T, uint32_t lo, uint32_t hi,
                                uint32_t* out, float* features, void* stream_) {
  if (!out) return GLCM_EINVAL;
  return batch_compute_common(plan, tiles, T, lo, hi, out, features, nullptr, nullptr, (hipStream_t)stream_);
}

struct glcm_batch_s {
  BatchLayout layout;
  int T = 0;
  int nitems = 0, nfins = 0;
  size_t fins_off = 0, partials_off = 0;
  int dtype = 0;
  uint32_t N = 0;
  int K = 0;
  void* desc = nullptr;  // device: descriptors
  std::vector<std::pair<uintptr_t, uintptr_t>> extents;  // the tiles' byte ranges (output checks)
  std::mutex mu;
  hipEvent_t ran = nullptr;  // recorded after each launch queued outside a graph capture
  bool has_ran = false;
};

GLCM_API int glcm_batch_prepare(glcm_plan_t plan, const glcm_tile_t* tiles, int T, glcm_batch_t* batch) {
  if (!batch || !plan || !tiles || T < 1 || T > (1 << 20)) return GLCM_EINVAL;
  *batch = nullptr;
  std::unique_ptr<glcm_batch_s> h(new (std::nothrow) glcm_batch_s());
  if (!h) return GLCM_ENOMEM;
  std::lock_guard<std::mutex> lk(plan->mu);
  int rc = batch_layout(plan, tiles, T, &h->layout);
  if (rc != GLCM_OK) return rc;
  GLCM_TRY_RC(check_tile_memory(tiles, T, h->layout.b));
  h->T = T;
  h->dtype = plan->dtype;
  h->N = (uint32_t)plan->N;
  h->K = plan->K;
  h->extents = tile_extents(tiles, T, h->layout.b);
  BatchItems it;
  batch_items(tiles, T, h->layout.b, &it);
  h->nitems = (int)it.items.size();
  h->nfins = (int)it.fins.size();
  h->fins_off = it.fins_off();
  h->partials_off = it.partials_off();
  const size_t need = it.dev_bytes(plan->K, plan->N);
  std::vector<char> host(it.desc_bytes());
  hipError_t e = hipEventCreateWithFlags(&h->ran, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc(&h->desc, need);
  if (e == hipSuccess) e = hipMemset(h->desc, 0, need);  // the item counter starts at zero
  if (e == hipSuccess) {
    batch_descriptors(it, host.data());
    e = hipMemcpy((char*)h->desc + kBatchDescOff, host.data(), host.size(), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    if (h->desc) (void)hipFree(h->desc);
    if (h->ran) (void)hipEventDestroy(h->ran);
    return hip_status(e);
  }
  *batch = h.release();
  return GLCM_OK;
}

GLCM_API int glcm_batch_run(glcm_batch_t batch, uint32_t lo, uint32_t hi, uint32_t* out, float* features,
                            void* stream_) {
  if (!batch || !out) return GLCM_EINVAL;
  if (lo > hi || hi > (batch->dtype == GLCM_U8 ? 255u : 65535u)) return GLCM_EINVAL;
  GLCM_TRY_RC(check_batch_outputs(batch->extents, batch->T, batch->K, (int)batch->N, out, features));
  hipStream_t stream = (hipStream_t)stream_;
  GLCM_TRY_RC(batch_launch(batch->layout, batch->nitems, batch->nfins, batch->fins_off, batch->partials_off,
                           batch->desc, batch->N, lo, hi, out, features, stream));
  // remember the launch for glcm_batch_destroy (a launch captured into a
  // graph is the caller's to wait for)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess) {
    (void)hipGetLastError();
    cs = hipStreamCaptureStatusActive;  // unknown: record nothing
  }
  if (cs == hipStreamCaptureStatusNone) {
    std::lock_guard<std::mutex> lk(batch->mu);
    GLCM_TRY(hipEventRecord(batch->ran, stream));
    batch->has_ran = true;
  }
  return GLCM_OK;
}

GLCM_API int glcm_batch_destroy(glcm_batch_t batch) {
  if (!batch) return GLCM_OK;
  {
    // the last launch queued through glcm_batch_run may still read the
    // descriptors (on one stream per run, launches complete in order; runs on
    // several streams at once are the caller's to wait for, as are graphs)
    std::lock_guard<std::mutex> lk(batch->mu);
    if (batch->has_ran) (void)hipEventSynchronize(batch->ran);
  }
  if (batch->desc) (void)hipFree(batch->desc);
  if (batch->ran) (void)hipEventDestroy(batch->ran);
  delete batch;
  return GLCM_OK;
}

GLCM_API int glcm_histogram(glcm_plan_t plan, const void* img, int W, int H, int64_t stride, int dtype, int N,
                            uint32_t lo, uint32_t hi, uint32_t* out, void* stream_) {
  static const glcm_offset_t kZero{0, 0};
  int rc = check_image_args(img, W, H, stride, dtype, N, lo, hi, &kZero, 1);
  if (rc != GLCM_OK) return rc;
  if (!out || (plan && (plan->dtype != dtype || plan->N != N))) return GLCM_EINVAL;
  const int b = dtype_bytes(dtype);
  const uintptr_t i0 = (uintptr_t)img;
  const uintptr_t i1 = i0 + (uintptr_t)(((uint64_t)(H - 1) * (uint64_t)stride + (uint64_t)W) * (uint64_t)b);
  const uintptr_t o0 = (uintptr_t)out, o1 = o0 + (uintptr_t)N * 4u;
  if (o0 < i1 && i0 < o1) return GLCM_EINVAL;
  int out_dev = -1, img_dev = -1, cur = 0;
  if (pointer_kind(out, &out_dev) != 2) return GLCM_EINVAL;
  if (pointer_kind(img, &img_dev) != 2) return GLCM_EUNSUPPORTED;
  GLCM_TRY(hipGetDevice(&cur));
  if (out_dev != cur || img_dev != cur) return GLCM_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  CachedPlanUse cached;
  if (!plan) {
    // a plan of its own (K = 0 in the key, which no glcm_compute call uses),
    // made on the global-atomic path so that it allocates no per-XCD slices:
    // the histogram needs only the partials
    rc = plan_cache().acquire(
        std::make_tuple(cur, dtype, N, 0, std::vector<int32_t>{}),
        [&](glcm_plan_t* np) {
          return glcm_plan_create(np, dtype, N, 1, &kZero, 65535, 65535, GLCM_FLAG_FORCE_GLOBAL);
        },
        &plan);
    if (rc != GLCM_OK) return rc;
    cached.plan = plan;
  }
  std::lock_guard<std::mutex> lk(plan->mu);
  GLCM_TRY_RC(order_after_previous(plan, stream));
  glcm::HistArgs a{};
  a.img = img;
  a.stride = stride;
  a.W = W;
  a.H = H;
  a.q = make_quant(N, lo, hi);
  fast_quant(b, N, lo, hi, &a.qfast, &a.qfast_shift, &a.qfast_mask);
  a.vec = (i0 % 16u == 0) && ((uint64_t)stride * (uint64_t)b) % 16u == 0;
  // 32 copies (every lane of an LDS pass its own bank) while 4 N D bytes stay
  // within 64 KiB, so several workgroups share a CU
  a.D = 32;
  while (a.D > 1 && (uint64_t)N * a.D * 4u > 65536u) a.D >>= 1;
  a.cpr = (uint32_t)((W + 15) / 16);
  const int groups = glcm::hist_geometry((uint64_t)H * a.cpr, plan->num_cus, &a.per_block);
  GLCM_TRY_RC(ensure_partials(plan, (size_t)groups * N * 4u));
  a.partials = plan->partials;
  glcm::LaunchTiming tm;
  if (plan->flags & GLCM_FLAG_TIMING) {
    GLCM_TRY(hipEventCreate(&tm.start));
    GLCM_TRY(hipEventCreate(&tm.stop));
    plan->timing.emplace_back(tm.start, tm.stop);
  }
  GLCM_TRY(glcm::launch_histogram(a, b, groups, (size_t)N * a.D * 4u, stream, tm));
  GLCM_TRY(glcm::launch_reduce(a.partials, out, (uint32_t)N, groups, false, stream));
  return record_done(plan, stream);
}

GLCM_API int glcm_batch_tuning(glcm_plan_t plan, glcm_batch_tuning_t* t, int set) {
  if (!plan || !t) return GLCM_EINVAL;
  std::lock_guard<std::mutex> lk(plan->mu);
  if (set) {
    if (t->replicas != 0 && t->replicas != 4 && t->replicas != 8 && t->replicas != 16) return GLCM_EINVAL;
    if (t->min_rows < 0 || t->min_rows > 256) return GLCM_EINVAL;
    if (t->wg_size != 0 && t->wg_size != 256 && t->wg_size != 512) return GLCM_EINVAL;
    if (t->replicas) {
      const size_t lds_cu = (size_t)plan->lds_budget_words * 4u + 1024u;
      if (glcm::batch_lds_bytes(plan->N, plan->K, t->replicas) > lds_cu - 1024u) return GLCM_EUNSUPPORTED;
    }
    plan->batch_D = t->replicas;
    plan->batch_min_rows = t->min_rows;
    plan->batch_wg = t->wg_size;
  }
  t->replicas = plan->batch_D ? plan->batch_D : batch_default_copies(plan);
  t->min_rows = plan->batch_min_rows ? plan->batch_min_rows : kBatchDefaultMinRows;
  t->wg_size = plan->batch_wg ? plan->batch_wg : glcm::kBatchThreads;
  return GLCM_OK;
}

GLCM_API int glcm_batch_autotune(glcm_plan_t plan, const glcm_tile_t* tiles, int T, uint32_t lo, uint32_t hi,
                                 int repeats, glcm_batch_tuning_t* chosen) {
  if (!plan || !tiles || T < 1 || T > (1 << 20) || repeats < 1 || repeats > 1000) return GLCM_EINVAL;
  if (lo > hi || hi > (plan->dtype == GLCM_U8 ? 255u : 65535u)) return GLCM_EINVAL;
  int old_D = 0, old_rows = 0, old_wg = 0;
  {
    std::lock_guard<std::mutex> lk(plan->mu);
    BatchLayout L;
    const int rc = batch_layout(plan, tiles, T, &L);  // validates the tiles and the plan
    if (rc != GLCM_OK) return rc;
    old_D = plan->batch_D;
    old_rows = plan->batch_min_rows;
    old_wg = plan->batch_wg;
  }
  const size_t words = (size_t)T * plan->K * plan->N * plan->N;
  uint32_t* out = nullptr;
  float* feat = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int best_D = 0, best_rows = 0, best_wg = 0, rc = GLCM_OK;
  float best = 0.0f;
  hipError_t e = hipMalloc((void**)&out, words * 4u);
  if (e == hipSuccess) e = hipMalloc((void**)&feat, (size_t)T * plan->K * 5u * sizeof(float));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) rc = hip_status(e);
  const int rows_grid[] = {4, 8, 16, 32};
  for (int wg = 256; rc == GLCM_OK && wg <= 512; wg *= 2)
  for (int D = 4; rc == GLCM_OK && D <= 16; D *= 2) {
    const size_t lds_cu = (size_t)plan->lds_budget_words * 4u + 1024u;
    if (glcm::batch_lds_bytes(plan->N, plan->K, D) > lds_cu - 1024u) continue;
    for (int rows : rows_grid) {
      {
        std::lock_guard<std::mutex> lk(plan->mu);
        plan->batch_D = D;
        plan->batch_min_rows = rows;
        plan->batch_wg = wg;
      }
      // a prepared batch: the timed runs queue kernels only (no host staging)
      glcm_batch_t pb = nullptr;
      rc = glcm_batch_prepare(plan, tiles, T, &pb);
      if (rc == GLCM_OK) rc = glcm_batch_run(pb, lo, hi, out, feat, s);  // warm-up
      if (rc == GLCM_OK && (e = hipEventRecord(e0, s)) != hipSuccess) rc = hip_status(e);
      for (int r = 0; rc == GLCM_OK && r < repeats; ++r) rc = glcm_batch_run(pb, lo, hi, out, feat, s);
      float ms = 0.0f;
      if (rc == GLCM_OK && (e = hipEventRecord(e1, s)) != hipSuccess) rc = hip_status(e);
      if (rc == GLCM_OK && (e = hipEventSynchronize(e1)) != hipSuccess) rc = hip_status(e);
      if (rc == GLCM_OK && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) rc = hip_status(e);
      if (pb) {
        if (s) (void)hipStreamSynchronize(s);
        (void)glcm_batch_destroy(pb);
      }
      if (rc != GLCM_OK) break;
      if (best_D == 0 || ms < best) {
        best = ms;
        best_D = D;
        best_rows = rows;
        best_wg = wg;
      }
    }
  }
  if (s) (void)hipStreamSynchronize(s);
  {
    std::lock_guard<std::mutex> lk(plan->mu);
    plan->batch_D = rc == GLCM_OK ? best_D : old_D;
    plan->batch_min_rows = rc == GLCM_OK ? best_rows : old_rows;
    plan->batch_wg = rc == GLCM_OK ? best_wg : old_wg;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (out) (void)hipFree(out);
  if (feat) (void)hipFree(feat);
  if (rc != GLCM_OK) return rc;
  if (chosen) {
    chosen->replicas = best_D;
    chosen->min_rows = best_rows;
    chosen->wg_size = best_wg;
  }
  return GLCM_OK;
}

GLCM_API int glcm_features(const uint32_t* glcm_u32, int K, int N, float* out, void* stream) {
  if (!glcm_u32 || !out || K < 1 || K > (1 << 20) || N < 1 || N > GLCM_MAX_LEVELS) return GLCM_EINVAL;
  int d1 = -1, d2 = -1;
  if (pointer_kind(glcm_u32, &d1) != 2 || pointer_kind(out, &d2) != 2) return GLCM_EINVAL;
  GLCM_TRY(glcm::launch_features(glcm_u32, K, N, out, (hipStream_t)stream));
  return GLCM_OK;
}

}  // extern "C"

namespace glcm {

int hip_error_status(hipError_t e) { return hip_status(e); }

int check_request_args(const void* img, int W, int H, int64_t stride, int dtype, int N, uint32_t lo, uint32_t hi,
                       const glcm_offset_t* offsets, int K) {
  return check_image_args(img, W, H, stride, dtype, N, lo, hi, offsets, K);
}

int memory_kind(const void* p, int* device) { return pointer_kind(p, device); }

}  // namespace glcm
