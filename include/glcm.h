/*
 * glcm.h - C ABI of the MI355X (gfx950) gray-level co-occurrence matrix library.
 *
 * The library computes the gray-level co-occurrence matrix of Eq. (1) of
 * Hong, Zheng and Pan, "Computation of gray-level co-occurrence matrix based on
 * CUDA and its optimization" (Section I.A): for an offset (dx, dy),
 *
 *     P[i][j] = number of pixels (x, y) such that (x+dx, y+dy) lies inside the
 *               W x H image, q(img(x, y)) = i and q(img(x+dx, y+dy)) = j,
 *
 * where q() reduces the raw pixel value to one of N gray levels (the
 * pre-processing step of Section I.A).  Conventions fixed by this library
 * (the paper leaves them open):
 *
 *   - Coordinates: x indexes columns, y indexes rows, y grows down the rows.
 *     Pixel (x, y) is img[y * stride + x].  The four directions of Eq. (2) at
 *     distance d are 0 deg = (d, 0), 45 deg = (-d, d), 90 deg = (0, d),
 *     135 deg = (d, d); see glcm_offset_polar().
 *   - Borders: a pair whose second pixel falls outside the image is skipped
 *     (no wrap-around to the next row, no padding), so sum P = (W-|dx|)(H-|dy|)
 *     when both factors are positive, else 0.
 *   - Orientation: P is stored row-major as out[k][i][j] with i the level of
 *     the FIRST pixel (x, y) and j the level of the SECOND pixel, following the
 *     variable order of Eq. (1).  P for (-dx, -dy) is the transpose of P for
 *     (dx, dy).
 *   - One increment per ordered pair (not symmetric), unnormalised uint32 counts.
 *   - Quantization: q(v) = 0 if v < lo; N-1 if v > hi; otherwise
 *     floor((v - lo) * N / (hi - lo + 1)), computed exactly.
 *
 * All functions return a glcm_status (0 = success, negative = error).  No
 * function aborts or prints.  Argument checks happen before any work is queued:
 * a call that returns GLCM_EINVAL has queued nothing and written nothing.
 * `stream` arguments are hipStream_t handles passed as void* (NULL = the
 * default stream of the current device).  Device pointers must belong to the
 * current HIP device.
 */
#ifndef GLCM_H
#define GLCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GLCM_ABI_VERSION 1

#ifndef GLCM_API
#define GLCM_API __attribute__((visibility("default")))
#endif

/* Pixel types. */
enum glcm_dtype { GLCM_U8 = 0, GLCM_U16 = 1 };

/* Displacement of the second pixel of a pair relative to the first. */
typedef struct glcm_offset {
    int32_t dx; /* columns, positive to the right */
    int32_t dy; /* rows, positive downwards */
} glcm_offset_t;

enum glcm_status {
    GLCM_OK = 0,
    GLCM_EINVAL = -1,       /* invalid argument; nothing was queued */
    GLCM_ENOMEM = -2,       /* device or pinned-host allocation failed */
    GLCM_EUNSUPPORTED = -3, /* valid request this build cannot serve */
    GLCM_EHIP = -4,         /* a HIP call failed; see glcm_last_hip_error() */
    GLCM_EBUSY = -5         /* the object is still in use (e.g. a request not done yet) */
};

/* Limits checked by every entry point. */
#define GLCM_MAX_LEVELS 4096    /* N */
#define GLCM_MAX_OFFSETS 64     /* K */
#define GLCM_MAX_DISPLACEMENT 32767

/* Plan flags (bitwise OR).  The FORCE_* flags select a kernel variant for
 * tests and ablations; without them the library picks the variant. */
#define GLCM_FLAG_FORCE_GENERIC     (1u << 0) /* per-pixel kernel, any layout */
#define GLCM_FLAG_FORCE_PARTITIONED (1u << 1) /* split bins into LDS-sized partitions */
#define GLCM_FLAG_FORCE_GLOBAL      (1u << 2) /* one global atomic per pair, no LDS */
#define GLCM_FLAG_SERIAL_UPLOAD     (1u << 3) /* host images: copy, then count (no overlap) */
#define GLCM_FLAG_TIMING            (1u << 4) /* time each counting-kernel launch with HIP events
                                                 its dispatch stamps; read with
                                                 glcm_plan_kernel_time() */
#define GLCM_FLAG_FORCE_SLABS       (1u << 5) /* row-slab kernel even where the strip kernel
                                                 applies */
#define GLCM_FLAG_FORCE_L2          (1u << 6) /* large-N path: pairs added straight into
                                                 per-XCD accumulators in L2, no LDS copies
                                                 (when those fit in 256 MiB) */
#define GLCM_FLAG_FORCE_BLOCKS      (1u << 7) /* block-code kernel where it applies (every
                                                 offset one of the four d = 1 directions
                                                 of Eq. (2) or its opposite, N <= 50,
                                                 max_W <= 65536): two codes per 2x2 pixel
                                                 block carry its four pairs */

typedef struct glcm_plan_s *glcm_plan_t;

/* Launch parameters of a plan, readable and (for tuning) overridable. */
typedef struct glcm_tuning {
    int replicas;       /* R: LDS copies of each GLCM per workgroup (power of two) */
    int wg_size;        /* threads per workgroup: 256, 512 or 1024 (the strip kernel runs
                           at most 512 on uint16 images with offsets reaching 2 pixels and
                           on any image with offsets reaching 3 or 4) */
    int rows_per_wave;  /* slab kernel: first-pixel rows per wavefront slab (4); 0 elsewhere */
    int tile_rows;      /* host-image upload tile height (rows) */
    int counter_bits;   /* LDS counters: 16 or 32; 0 keeps the current value.  Slab kernel:
                           two copies per dword; strip kernel: two GLCMs per dword (dwords
                           per bin 4, 8, 16 or 32); partitioned kernel: two bins per dword
                           with one copy (replicas 1), bands then kept below 2^16 pixels.
                           16-bit layouts are used only where no count can overflow */
    int merge;          /* 0: workgroups add their counts into per-XCD accumulators in L2,
                           a small kernel sums the 8 slices; 1: per-band partial counts,
                           summed by a reduce kernel */
    int path;           /* 0 generic, 1 slab kernel, 2 partitioned, 3 global, 4 strip
                           kernel, 5 L2 slices (large N), 6 block codes (d = 1).  Read-only,
                           except that a plan on the slab or strip kernel may be set to the
                           other where its offsets allow it (GLCM_EINVAL otherwise): the
                           strip kernel takes |dx|, |dy| <= 2, and 3 or 4 along the four
                           directions of Eq.(2) (dx = 0, dy = 0 or |dx| = |dy|); the slab
                           kernel any offset with |dx|, |dy| <= 4 */
    int partitions;     /* read-only: bin partitions per pass */
} glcm_tuning_t;

/* Largest K * N * N that glcm_compute_static accepts (its accumulation
 * slices: 16 of these, 16 MiB per GPU). */
#define GLCM_STATIC_MAX_WORDS (1u << 18)

/* Version of this ABI (GLCM_ABI_VERSION). */
GLCM_API int glcm_abi_version(void);

/* Static English description of a status code.  Never NULL. */
GLCM_API const char *glcm_strerror(int status);

/* hipError_t value of the last HIP failure reported as GLCM_EHIP on the
 * calling thread (0 if none). */
GLCM_API int glcm_last_hip_error(void);

/*
 * Offset of the Eq. (2) direction table.  d >= 1; theta_deg is a multiple of
 * 45 in [0, 360).  0/45/90/135 give (d,0), (-d,d), (0,d), (d,d): the second
 * pixel sits d, d*(W-1), d*W, d*(W+1) elements after the first in row-major
 * order, as in Eq. (2).  180..315 give the opposite displacements.
 * Returns GLCM_EINVAL for other angles, d < 1, d > GLCM_MAX_DISPLACEMENT or a
 * NULL out.
 */
GLCM_API int glcm_offset_polar(int d, int theta_deg, glcm_offset_t *out);

/*
 * Creates a reusable plan for images of one pixel type, one N and one offset
 * list, of size up to max_W x max_H.  The plan owns its device workspace, its
 * pinned staging buffers and its upload stream; all are released by
 * glcm_plan_destroy().  `offsets` (host, K entries) is copied.
 * Errors: GLCM_EINVAL for a NULL plan pointer, bad dtype, N outside
 * [1, GLCM_MAX_LEVELS], K outside [1, GLCM_MAX_OFFSETS], NULL offsets, a
 * displacement component beyond GLCM_MAX_DISPLACEMENT, max_W or max_H < 1 or
 * max_W * max_H > 2^32 - 1, or unknown flags.  GLCM_ENOMEM / GLCM_EHIP on
 * allocation failure.  Needs a HIP device.
 */
GLCM_API int glcm_plan_create(glcm_plan_t *plan, int dtype, int N, int K, const glcm_offset_t *offsets,
                     int max_W, int max_H, uint32_t flags);

/* Reads (and, if `set` is non-zero, first overrides) the plan's launch
 * parameters.  Overrides are validated and clamped to what the device allows;
 * GLCM_EINVAL for values outside the documented sets. */
GLCM_API int glcm_plan_tuning(glcm_plan_t plan, glcm_tuning_t *tuning, int set);

/*
 * Picks the plan's launch parameters by timing the candidate layouts (LDS
 * copies, counter width, workgroup size; for row-kernel plans both the strip
 * kernel, where every offset has |dx|, |dy| <= 2, and the slab kernel, and,
 * for a plan whose offsets are all d = 1 directions of Eq. (2) or their
 * opposites, the block-code kernel) on a representative DEVICE image: each
 * candidate counts the image `repeats` times after two warm-up runs, on
 * `stream`, starting with the plan's current parameters; the fastest is kept
 * (a later candidate must be 3% faster to replace an earlier one) and written
 * to *chosen (may be NULL).  A plan created with GLCM_FLAG_FORCE_BLOCKS keeps
 * the block-code kernel; one created with GLCM_FLAG_FORCE_SLABS keeps the
 * slab kernel.  The
 * call blocks until the timing is done and leaves the plan's results
 * unchanged in meaning (every candidate computes the same counts).
 * Errors: GLCM_EINVAL for a NULL plan or image, a host image, sizes beyond the
 * plan's maxima, lo > hi, repeats outside [1, 1000]; GLCM_EHIP / GLCM_ENOMEM.
 */
GLCM_API int glcm_plan_autotune(glcm_plan_t plan, const void *img, int W, int H, int64_t stride, uint32_t lo,
                                uint32_t hi, int repeats, void *stream, glcm_tuning_t *chosen);

/*
 * glcm_compute for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * computes exactly what glcm_compute computes (Eq. (1) for each offset) for a
 * DEVICE image on the current device, with the same kernels, but takes no plan
 * and calls no hipMalloc, hipFree or other allocating routine: the per-XCD
 * accumulation slices of its merge live in a file-scope device array of
 * 16 MiB that each GPU the library runs on holds until the process ends
 * (found once per device with hipGetSymbolAddress on its first call there).
 * A misaligned image (base or row pitch not a multiple of 16 bytes) is read
 * in place, never copied (from 2^16 pixels on, the strip and slab kernels
 * assemble its rows from the dwords that hold them; smaller images and a
 * block-code layout take the per-pixel kernels).  Calls are queued on
 * `stream` like glcm_compute; every call on one GPU shares that array, so
 * calls that overlap on one GPU (several streams, or host threads) race and
 * must be ordered by the caller.  The array is cleared at the start of each
 * call (by a kernel, so the call can be captured in a graph).
 * Errors: those of glcm_compute; GLCM_EINVAL when K * N * N exceeds
 * GLCM_STATIC_MAX_WORDS or img / out is not device memory of the current
 * device.
 */
GLCM_API int glcm_compute_static(const void *img, int W, int H, int64_t stride, int dtype, int N, uint32_t lo,
                                 uint32_t hi, const glcm_offset_t *offsets, int K, uint32_t *out, void *stream);

/*
 * For plans created with GLCM_FLAG_TIMING: waits for the recorded launches and
 * returns the summed duration (ms) of the counting kernel (the vote kernel,
 * without the merge step) over the launches since the previous call, as
 * measured by HIP events that the kernel's dispatch packet stamps with the
 * kernel's start and end (hipExtLaunchKernel), so launch latency is not
 * included; then forgets them.
 * Errors: GLCM_EINVAL for NULL arguments; GLCM_EHIP.
 */
GLCM_API int glcm_plan_kernel_time(glcm_plan_t plan, double *ms_total, int *launches);

/*
 * Re-targets a plan at another offset list (same dtype and N) of at most the K
 * it was created with, keeping its device workspace: the per-XCD accumulators
 * are zero between calls whatever K is, so only the host-side launch layout
 * is recomputed (a tuning set with glcm_plan_tuning is discarded).  For
 * callers whose offsets change from call to call, such as the request server
 * below.  Work already queued keeps the offsets it was launched with.
 * Errors: GLCM_EINVAL for a NULL plan, NULL offsets, K < 1 or above the
 * plan's creation K, or a displacement beyond GLCM_MAX_DISPLACEMENT.
 */
GLCM_API int glcm_plan_rebind(glcm_plan_t plan, const glcm_offset_t *offsets, int K);

/* Device bytes the plan holds right now (accumulators, band partials, tile
 * and descriptor buffers; some are allocated on first use).  GLCM_EINVAL for
 * NULL arguments. */
GLCM_API int glcm_plan_workspace(glcm_plan_t plan, size_t *device_bytes);

/* Releases a plan after waiting for its queued work.  NULL is accepted. */
GLCM_API int glcm_plan_destroy(glcm_plan_t plan);

/*
 * The internal plans behind calls with plan = NULL (glcm_compute,
 * glcm_histogram): one per device and call signature, reused by later calls.
 * The cache holds at most 32 plans and 512 MiB of their device workspace;
 * when a call ends over either bound, idle plans are destroyed least recently
 * used first (after their queued work completes).  Plans in use by a running
 * call are never destroyed.
 * glcm_plan_cache_stats: plans held and their device bytes (either pointer
 * may be NULL).  glcm_plan_cache_clear: destroys every idle cached plan.
 */
GLCM_API int glcm_plan_cache_stats(int *plans, uint64_t *device_bytes);
GLCM_API int glcm_plan_cache_clear(void);

/*
 * Computes out[k][i][j] (Eq. (1)) for the K offsets.
 *
 *   plan     NULL, or a plan created with the same dtype, N, K, offsets and
 *            with W <= max_W, H <= max_H (else GLCM_EINVAL).  NULL uses an
 *            internal plan cached per device and call signature.
 *   img      W x H pixels, row y at img + y*stride elements.  Device memory,
 *            pinned host memory or pageable host memory.  Host images are
 *            uploaded in row tiles (with the halo rows the offsets need) on the
 *            plan's upload stream while earlier tiles are counted on `stream`.
 *            Must be aligned to the pixel size; a device image of at least
 *            2^16 pixels whose base or pitch is not 16-byte aligned is read
 *            in place by the strip and slab kernels (the block-code kernel
 *            copies it to an aligned plan buffer first); smaller ones take
 *            the per-pixel kernels.
 *   stride   row pitch in ELEMENTS, >= W.
 *   dtype    GLCM_U8 or GLCM_U16.
 *   N, lo, hi  quantization (see above); lo <= hi <= max of dtype.
 *   offsets  host array of K displacements; components within
 *            +-GLCM_MAX_DISPLACEMENT.  Offsets reaching outside the image are
 *            legal and give all-zero matrices.
 *   out      device memory, K*N*N uint32, overwritten (not accumulated); must
 *            not overlap img.
 *   stream   hipStream_t (as void*); all device work is ordered on it.
 *
 * Device images: returns once the work is queued.  Host images: returns once
 * the last upload is queued; the caller must not modify the host image until
 * `stream` has completed.  Errors: GLCM_EINVAL (nothing queued) for NULL
 * pointers, W or H < 1, stride < W, W*H > 2^32-1, bad dtype, N or K out of
 * range, lo > hi, hi above the dtype maximum, a displacement out of range, a
 * misaligned img, an out buffer that is not device memory or overlaps img, or
 * a plan mismatch.  GLCM_EHIP / GLCM_ENOMEM on HIP failures while queueing.
 */
GLCM_API int glcm_compute(glcm_plan_t plan, const void *img, int W, int H, int64_t stride, int dtype,
                 int N, uint32_t lo, uint32_t hi, const glcm_offset_t *offsets, int K,
                 uint32_t *out, void *stream);

/*
 * Haralick statistics of K co-occurrence matrices (Introduction, Haralick's
 * texture features), out[k][0..4] = contrast, energy (angular second moment),
 * entropy (natural log), homogeneity (inverse difference moment,
 * 1/(1+(i-j)^2)), correlation.  p = P/T with T = sum of P[k].  T = 0 gives
 * five zeros; a row or column marginal with a single occupied level gives
 * correlation 1.  Energy, entropy and homogeneity are summed in fp32; the
 * contrast and the correlation come from exact integer moments (the contrast
 * as one fp64 quotient, the correlation's variances and covariance combined
 * in fp64).
 *
 *   glcm     device memory, K*N*N uint32 (the layout glcm_compute writes).
 *   out      device memory, K*5 float, overwritten.
 * Errors: GLCM_EINVAL for NULL or host pointers, K outside [1, 2^20], N
 * outside [1, GLCM_MAX_LEVELS], or a matrix whose total exceeds 2^32 - 1 (the
 * latter only detected on the device: that matrix's outputs are NaN).
 */
GLCM_API int glcm_features(const uint32_t *glcm, int K, int N, float *out, void *stream);

/*
 * 1-D gray-level histogram of a device image (the paper notes among its
 * contributions that its analysis of colliding increments carries over to
 * statistical histograms): out[i] = number of pixels (x, y) of the W x H
 * image with q(img(x, y)) = i, for i < N, counted with the same replicated
 * LDS votes as the co-occurrence matrices.
 *
 *   plan     NULL (an internal plan cached per device, dtype and N) or a plan
 *            with the same dtype and N (its offsets and maximum image size do
 *            not matter).  Its workspace holds the per-workgroup histograms and
 *            the call is ordered after the plan's previous work.
 *   img, W, H, stride, dtype, N, lo, hi   as for glcm_compute, except that img
 *            must be device memory (GLCM_EUNSUPPORTED for host memory).
 *   out      device memory, N uint32, overwritten; must not overlap img.
 * Errors as for glcm_compute.
 */
GLCM_API int glcm_histogram(glcm_plan_t plan, const void *img, int W, int H, int64_t stride, int dtype,
                            int N, uint32_t lo, uint32_t hi, uint32_t *out, void *stream);

/*
 * Variants of K co-occurrence matrices P[k]: device memory, K*N*N uint32 in
 * the layout glcm_compute writes, K in [1, 2^20], N in [1, GLCM_MAX_LEVELS].
 * Each call is one asynchronous kernel on `stream`, with a fixed order of
 * operations (the same input always gives the same bits).
 *
 * glcm_symmetrize   out[k] = P[k] + P[k]^T modulo 2^32: the symmetric GLCM,
 *                   a reading of Section I.B, where a pair increments both
 *                   coordinates.  out: K*N*N uint32; may be the input itself
 *                   (in place) but must not overlap it otherwise.
 * glcm_normalize    out[k][i][j] = P[k][i][j] / T_k, T_k = sum of P[k]: the
 *                   quotient correctly rounded in fp64, then rounded to fp32;
 *                   T_k = 0 gives zeros.  out: K*N*N float, not overlapping P.
 * glcm_average      the mean of the normalised matrices over consecutive
 *                   groups of m (for example the four directions of one
 *                   distance): out[g] = (sum over k in [g m, g m + m), in
 *                   order, of P[k] / T_k) / m in fp64, rounded to fp32.  An
 *                   empty matrix adds nothing but counts in m.  m in [1, 64],
 *                   K a multiple of m.  out: (K/m)*N*N float, not overlapping P.
 * glcm_haralick     Haralick's statistics f1..f13 (cited in the introduction;
 *                   the fourteenth, which needs an eigenvalue solver, is
 *                   glcm_haralick_mcc below).  out[k][0..12] =
 *                   angular second moment, contrast, correlation, sum of
 *                   squares (variance of the row marginal), inverse difference
 *                   moment, sum average, sum variance (about the sum average),
 *                   sum entropy, entropy, difference variance, difference
 *                   entropy, information measures of correlation 1 and 2.
 *                   Levels numbered from 0, natural logs, p = P/T.  T = 0
 *                   gives zeros; a marginal on a single level gives
 *                   correlation 1; both marginal entropies 0 give f12 = 0.
 *                   Computed in fp64, stored as fp32.  N <= 1024
 *                   (GLCM_EUNSUPPORTED above).  out: K*13 float.
 * Errors: GLCM_EINVAL for NULL, host or other-device pointers, sizes out of
 * range or overlapping buffers (nothing queued); GLCM_EHIP if the launch fails.
 */
GLCM_API int glcm_symmetrize(const uint32_t *glcm, int K, int N, uint32_t *out, void *stream);
GLCM_API int glcm_normalize(const uint32_t *glcm, int K, int N, float *out, void *stream);
GLCM_API int glcm_average(const uint32_t *glcm, int K, int N, int m, float *out, void *stream);
GLCM_API int glcm_haralick(const uint32_t *glcm, int K, int N, float *out, void *stream);

/*
 * Haralick's fourteenth statistic, the maximal correlation coefficient (cited
 * in the introduction with the others): out[k] = the square root of the
 * second largest eigenvalue of Q(i, j) = sum_c p(i, c) p(j, c) / (px(i) py(c)),
 * p = P[k] / T, px and py the row and column marginals; terms with a zero
 * marginal are 0.  Computed in fp64 from the symmetric matrix S = B B^T,
 * B(i, c) = p(i, c) / sqrt(px(i) py(c)), which has Q's eigenvalues, with cyclic
 * Jacobi rotations (at most 30 sweeps); stored as fp32.  T = 0 or N = 1 gives
 * 0.  glcm as above; N <= 64 (GLCM_EUNSUPPORTED above); out: K float, device
 * memory.  Errors as for glcm_haralick.
 */
GLCM_API int glcm_haralick_mcc(const uint32_t *glcm, int K, int N, float *out, void *stream);

/* One device-resident image of a batch. */
typedef struct glcm_tile {
    const void *img;  /* device memory, row y at img + y*stride elements, aligned to the pixel size */
    int64_t stride;   /* row pitch in elements, >= W */
    int32_t W, H;     /* 1 <= W <= plan max_W, 1 <= H <= plan max_H */
} glcm_tile_t;

/*
 * Computes the co-occurrence matrices of Eq. (1), and optionally their Haralick
 * statistics, for T independent images in one launch: one workgroup per image
 * fuses quantization, the pair visit, the LDS votes, the merge and the
 * statistics (the per-image steps of Section II.A, applied to many small
 * images at once).  Images are processed largest first; results land in the
 * caller's order.
 *
 *   plan      a plan (its dtype, N, K and offsets apply to every image).  The
 *             batch path needs K <= 4, offsets with |dx| <= 2 and |dy| <= 2, and
 *             4 copies of the K (N+1) x (N+1) matrices in one workgroup's LDS
 *             ((N+1)^2 * K * 16 bytes + 4 K N^2 + 3 KiB <= 159 KiB, e.g. N <= 43
 *             for K = 4), else GLCM_EUNSUPPORTED; images need not be 16-byte
 *             aligned (the rows of those that are not are read as aligned
 *             dwords and shifted into place; nothing is copied).
 *   tiles     host array of T image descriptors (read before returning).
 *   T         number of images, 1 .. 2^20.
 *   lo, hi    quantization range, as in glcm_compute.
 *   out       device memory, T*K*N*N uint32: out[t][k][i][j], overwritten.
 *   features  device memory, T*K*5 float (as glcm_features), or NULL.
 *   stream    hipStream_t (as void*).
 *
 * Returns once the work is queued.  The plan's descriptor staging is reused
 * by the next batch call after this one's upload has completed.  Errors:
 * GLCM_EINVAL (nothing queued) for NULL pointers, T out of range, a tile with
 * W or H < 1, W > max_W, H > max_H, stride < W, W*H > 2^32-1 or a misaligned
 * img, a tile that is not inside one device allocation of the current device
 * (host memory included), out or features not device memory of the current
 * device, out or features overlapping a tile or each other, lo > hi or hi
 * above the dtype maximum; GLCM_EUNSUPPORTED as above; GLCM_EHIP /
 * GLCM_ENOMEM on HIP failures while queueing.
 */
GLCM_API int glcm_batch_compute(glcm_plan_t plan, const glcm_tile_t *tiles, int T, uint32_t lo, uint32_t hi,
                                uint32_t *out, float *features, void *stream);

/*
 * A batch prepared once and launched many times, e.g. from a HIP graph.
 * glcm_batch_prepare uploads the T descriptors (sorted as in
 * glcm_batch_compute) into device memory owned by the returned handle; it
 * takes the plan's dtype, N, offsets and limits at that moment and blocks
 * until the upload is done.
 * The images must stay at their addresses while the handle is used (their
 * pixels may change between launches).  Errors as glcm_batch_compute (the
 * tiles are checked here, the outputs at each glcm_batch_run);
 * GLCM_ENOMEM / GLCM_EHIP.
 */
typedef struct glcm_batch_s *glcm_batch_t;
GLCM_API int glcm_batch_prepare(glcm_plan_t plan, const glcm_tile_t *tiles, int T, glcm_batch_t *batch);

/*
 * Queues the prepared batch on `stream`: the fused kernel, nothing else (no
 * copy from host memory, no allocation, no synchronisation, no memset), so the
 * call can be captured into a HIP graph and replayed.  out / features as in
 * glcm_batch_compute.  The handle's descriptors are only read, so it may run
 * on several streams at once (into distinct outputs).  GLCM_EINVAL for a NULL
 * handle or out, out or features not device memory of the current device or
 * overlapping a tile or each other, lo > hi or hi above the dtype maximum;
 * GLCM_EHIP.
 */
GLCM_API int glcm_batch_run(glcm_batch_t batch, uint32_t lo, uint32_t hi, uint32_t *out, float *features,
                            void *stream);

/*
 * Waits for the last launch glcm_batch_run queued outside a graph capture,
 * then releases the handle.  Launches still running on other streams, and
 * graphs that replay a captured launch, must have completed before this call
 * (the caller synchronises them).  NULL is accepted.
 */
GLCM_API int glcm_batch_destroy(glcm_batch_t batch);

/*
 * Layout of the batch kernel, chosen per plan.  The paper tunes the number of
 * GLCM copies per block and the block size by measurement (Section II.A,
 * Table III, Eq. (4)-(6)); the batch engine does the same for its own layout.
 *
 *   replicas  LDS copies (dwords) of every bin: 4, 8 or 16; 0 = the default
 *             rule (the most that leave room for two workgroups per CU).
 *             More copies mean fewer colliding votes but a heavier merge.
 *   min_rows  shortest run of rows a wavefront segment walks, 1 .. 256; 0 = 4.
 *             Shorter runs spread a small image over more wavefronts; longer
 *             runs cut the per-run set-up.
 *   wg_size   threads per workgroup: 256 or 512; 0 = 256.  The workgroups
 *             are persistent (as many as the CUs hold at once) and take the
 *             batch's images, largest first, from a counter; an image above
 *             2^20 pixels is split into bands of rows counted by several
 *             workgroups and summed afterwards.
 */
typedef struct glcm_batch_tuning {
    int replicas;
    int min_rows;
    int wg_size;
} glcm_batch_tuning_t;

/* Reads (set = 0) or sets (set != 0) the plan's batch layout; on return
 * *tuning holds the effective values.  GLCM_EINVAL for a NULL argument or a
 * value out of range, GLCM_EUNSUPPORTED when the copies do not fit the LDS. */
GLCM_API int glcm_batch_tuning(glcm_plan_t plan, glcm_batch_tuning_t *tuning, int set);

/*
 * Times every batch layout that fits (wg_size 256, 512 x replicas 4, 8, 16 x
 * min_rows 4, 8, 16, 32) on the given images, `repeats` runs each after one warm-up run, with the
 * statistics computed, and keeps the fastest in the plan for later batch calls
 * (glcm_batch_compute, glcm_batch_prepare).  tiles, T, lo, hi as for
 * glcm_batch_compute; repeats 1 .. 1000.  Allocates its own outputs and stream
 * and synchronises before returning.  *chosen (may be NULL) receives the
 * layout kept.  Errors as for glcm_batch_compute; on a HIP failure the plan
 * keeps its previous layout.
 */
GLCM_API int glcm_batch_autotune(glcm_plan_t plan, const glcm_tile_t *tiles, int T, uint32_t lo, uint32_t hi,
                                 int repeats, glcm_batch_tuning_t *chosen);

/* ------------------------------------------------------------------------
 * Request server: continuous admission of GLCM jobs of mixed image size, N
 * and offset lists.  A scheduler thread admits queued requests in arrival
 * order as soon as a lane (a HIP stream with its own plans, one per dtype and
 * N, re-targeted per request) is free and the request's device memory fits
 * the HBM budget; requests on different lanes run concurrently on the GPU,
 * and a lane is handed to the next request the moment its work completes
 * (a host function queued behind it).  Images stay the caller's; counts and
 * statistics go to caller buffers or to the server's device result pool,
 * where they stay until fetched or released.
 * Continuous batching: a small request (at most 2^20 pixels, at most four
 * offsets with |dx|, |dy| <= 2, N <= 255) takes along the queued requests of
 * the same job (dtype, N, lo, hi, offsets in the same order, statistics or
 * not) that are small too, up to 1024, in arrival order while their results
 * fit: the group is one launch of the fused batch kernel (glcm_batch_compute)
 * on its lane, each image's results written to its own request's buffers,
 * and its requests complete together.  The results equal those of each
 * request computed alone.
 * ------------------------------------------------------------------------ */
typedef struct glcm_server_s *glcm_server_t;

typedef struct glcm_request {
    const void *img;                /* device image, or host memory (pinned or pageable: streamed to
                                       the GPU in row tiles by the lane, never fused; the caller keeps
                                       it unchanged until the request is done); row y at
                                       img + y*stride elements */
    int32_t W, H;                   /* 1 .. 65535 each, W*H <= 2^32 - 1 */
    int64_t stride;                 /* elements, >= W */
    int32_t dtype;                  /* GLCM_U8 or GLCM_U16 */
    int32_t N;                      /* 1 .. GLCM_MAX_LEVELS */
    uint32_t lo, hi;                /* quantization range, as in glcm_compute */
    const glcm_offset_t *offsets;   /* host, K entries, copied at submit */
    int32_t K;                      /* 1 .. GLCM_MAX_OFFSETS */
    int32_t features;               /* non-zero: also the five statistics */
    uint32_t *out;                  /* device K*N*N uint32, or NULL: a server-owned buffer */
    float *feat;                    /* device K*5 float (features != 0), or NULL: server-owned */
} glcm_request_t;

typedef struct glcm_request_info {
    int32_t done;                   /* 1 once the request's work has completed (or failed) */
    int32_t status;                 /* GLCM_OK, or the error the request ended with */
    int32_t lane;                   /* lane it ran on, -1 while queued */
    int32_t fused;                  /* requests in the launch that carried it (1: alone) */
    double submit_us, admit_us, done_us;  /* host steady clock, us since server creation */
    const uint32_t *out;            /* device counts [K][N][N] (valid once done) */
    const float *feat;              /* device statistics [K][5], or NULL */
} glcm_request_info_t;

typedef struct glcm_server_stats {
    uint64_t submitted, completed, failed;
    int32_t lanes, max_inflight;    /* lanes, most requests admitted at once */
    uint64_t budget_bytes;          /* the HBM budget */
    uint64_t bytes_in_use;          /* budgeted bytes held now (plans + results) */
    uint64_t max_bytes_in_use;      /* most budgeted bytes held at once */
    uint64_t fused_launches;        /* launches that carried two or more requests */
    uint64_t fused_requests;        /* requests those launches carried */
} glcm_server_stats_t;

/*
 * Creates a server on the current device.
 *   lanes              concurrent requests, 1 .. 16 (one HIP stream each).
 *   hbm_budget         bytes the server may hold at once for plan workspaces
 *                      and server-owned results; a request is admitted only
 *                      when its results and any plan workspace it needs fit
 *                      beside what is held (idle plans are evicted first).
 *   result_pool_bytes  device pool for server-owned results (<= hbm_budget);
 *                      0: every request must bring out (and feat).
 * Errors: GLCM_EINVAL for a NULL pointer, lanes outside 1 .. 16, a zero
 * budget, a pool larger than the budget, or flags other than 0;
 * GLCM_ENOMEM / GLCM_EHIP.
 */
GLCM_API int glcm_server_create(glcm_server_t *srv, int lanes, uint64_t hbm_budget, uint64_t result_pool_bytes,
                                uint32_t flags);

/* Queues one request (validated here; nothing is queued on error) and returns
 * its ticket.  Errors: GLCM_EINVAL for a bad descriptor (as glcm_compute, plus
 * a device image on another device, or a NULL out / feat without a result pool);
 * GLCM_EUNSUPPORTED when the request alone needs more than the budget. */
GLCM_API int glcm_server_submit(glcm_server_t srv, const glcm_request_t *req, uint64_t *ticket);

/* State of a request (non-blocking).  GLCM_EINVAL for an unknown ticket. */
GLCM_API int glcm_server_query(glcm_server_t srv, uint64_t ticket, glcm_request_info_t *info);

/* Blocks until the request is done; info may be NULL.  Returns the request's
 * status (GLCM_EINVAL for an unknown ticket). */
GLCM_API int glcm_server_wait(glcm_server_t srv, uint64_t ticket, glcm_request_info_t *info);

/* Copies a done request's counts (and statistics, if it has them and feat is
 * not NULL) to caller device buffers on `stream`.  GLCM_EINVAL for an unknown
 * or unfinished ticket or a NULL out; GLCM_EHIP. */
GLCM_API int glcm_server_fetch(glcm_server_t srv, uint64_t ticket, uint32_t *out, float *feat, void *stream);

/* Forgets a done request and returns its server-owned result memory to the
 * pool.  GLCM_EINVAL for an unknown ticket, GLCM_EBUSY if it is not done. */
GLCM_API int glcm_server_release(glcm_server_t srv, uint64_t ticket);

/* Waits until every submitted request is done. */
GLCM_API int glcm_server_drain(glcm_server_t srv);

/* Counters since creation.  GLCM_EINVAL for NULL arguments. */
GLCM_API int glcm_server_stats(glcm_server_t srv, glcm_server_stats_t *stats);

/* Drains, stops the scheduler and releases streams, plans and the pool.
 * NULL is accepted. */
GLCM_API int glcm_server_destroy(glcm_server_t srv);

#ifdef __cplusplus
}
#endif

#endif /* GLCM_H */
