/*
 * CPU oracle for the gray-level co-occurrence matrix (GLCM) and five Haralick
 * statistics.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the
 * CPU-baseline leg of the benchmark call it; the library never does.  It shares
 * no source, header, table or helper with the HIP path.
 *
 * Plain definitions, written for a reader to check by eye against the paper
 * (Hong, Zheng, Pan, "Computation of gray-level co-occurrence matrix based on
 * CUDA and its optimization"):
 *
 *   quantize      Section I.A says gray levels are reduced to a few levels
 *                 (8, 16, 32) as pre-processing but gives no formula.  Reading:
 *                 q(v) = 0 below lo, N-1 above hi, else floor((v-lo)*N/(hi-lo+1)),
 *                 exact in 64-bit integers.
 *   glcm          Eq. (1): P(i,j) counts ordered pixel pairs whose first pixel
 *                 has level i and whose second pixel, displaced by (dx,dy), has
 *                 level j.  Reading of Eq. (2): (dx,dy) in image coordinates with
 *                 y growing down the rows; pairs whose second pixel falls outside
 *                 the W x H image are not counted (no wrap to the next row).
 *                 Output P[k][i][j], row-major, i = first pixel (Eq. (1) order),
 *                 unnormalised counts, one increment per ordered pair.
 *   features      Haralick's statistics, cited in the introduction without
 *                 formulas.  p = P/T with T = sum P; contrast = sum (i-j)^2 p;
 *                 energy = angular second moment = sum p^2; entropy = -sum p ln p
 *                 over p > 0; homogeneity = sum p / (1 + (i-j)^2); correlation =
 *                 sum (i-mu_i)(j-mu_j) p / (sigma_i sigma_j).  T = 0 gives all
 *                 zeros; a marginal with a single occupied level (sigma = 0)
 *                 gives correlation 1.
 *
 * Parity pins (tests/test_oracle*.py): brute-force enumeration of all pixel
 * pairs of tiny images, a vectorised numpy bincount formulation, total counts,
 * the transpose identity for opposite offsets, constant and checkerboard closed
 * forms, marginals against histograms, exhaustive quantizer checks against
 * big-integer arithmetic, and closed-form feature values.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* q(v): gray-level reduction (Section I.A), see header. */
uint32_t oracle_quantize(uint32_t v, uint32_t N, uint32_t lo, uint32_t hi)
{
    if (v < lo) return 0;
    if (v > hi) return N - 1;
    uint64_t num = (uint64_t)(v - lo) * (uint64_t)N;
    uint64_t den = (uint64_t)(hi - lo) + 1u;
    return (uint32_t)(num / den);
}

static uint32_t pixel_at(const void *img, int bytes_per_px, int64_t stride, int x, int y)
{
    int64_t idx = (int64_t)y * stride + x;
    if (bytes_per_px == 1) return ((const uint8_t *)img)[idx];
    return ((const uint16_t *)img)[idx];
}

/*
 * Eq. (1) for K offsets.  Counts pairs whose FIRST pixel lies in rows
 * [y_begin, y_end) (pass 0, H for the whole image); the second pixel may lie
 * anywhere in the image.  Returns 0, or -1 if a count would exceed 2^32-1 or
 * the arguments are out of range.  out has K*N*N entries and is overwritten.
 */
int oracle_glcm_rows(const void *img, int W, int H, int64_t stride, int bytes_per_px,
                     int N, uint32_t lo, uint32_t hi, const int32_t *offsets, int K,
                     int y_begin, int y_end, uint32_t *out)
{
    if (W < 1 || H < 1 || N < 1 || K < 1 || stride < W || lo > hi) return -1;
    if (bytes_per_px != 1 && bytes_per_px != 2) return -1;
    if (y_begin < 0 || y_end > H || y_begin > y_end) return -1;
    size_t nbins = (size_t)N * (size_t)N;
    uint64_t *acc = (uint64_t *)calloc((size_t)K * nbins, sizeof(uint64_t));
    if (!acc) return -1;
    for (int k = 0; k < K; ++k) {
        int dx = offsets[2 * k], dy = offsets[2 * k + 1];
        uint64_t *P = acc + (size_t)k * nbins;
        for (int y = y_begin; y < y_end; ++y) {
            for (int x = 0; x < W; ++x) {
                int x2 = x + dx, y2 = y + dy;
                if (x2 < 0 || x2 >= W || y2 < 0 || y2 >= H) continue;
                uint32_t i = oracle_quantize(pixel_at(img, bytes_per_px, stride, x, y), N, lo, hi);
                uint32_t j = oracle_quantize(pixel_at(img, bytes_per_px, stride, x2, y2), N, lo, hi);
                P[(size_t)i * N + j] += 1;
            }
        }
    }
    int rc = 0;
    for (size_t t = 0; t < (size_t)K * nbins; ++t) {
        if (acc[t] > 0xFFFFFFFFull) rc = -1;
        out[t] = (uint32_t)acc[t];
    }
    free(acc);
    return rc;
}

int oracle_glcm(const void *img, int W, int H, int64_t stride, int bytes_per_px, int N,
                uint32_t lo, uint32_t hi, const int32_t *offsets, int K, uint32_t *out)
{
    return oracle_glcm_rows(img, W, H, stride, bytes_per_px, N, lo, hi, offsets, K, 0, H, out);
}

/*
 * Haralick statistics in double precision, one GLCM at a time (see header).
 * out[k*5 + 0..4] = contrast, energy, entropy, homogeneity, correlation.
 */
void oracle_features(const uint32_t *glcm, int K, int N, double *out)
{
    size_t nbins = (size_t)N * (size_t)N;
    for (int k = 0; k < K; ++k) {
        const uint32_t *P = glcm + (size_t)k * nbins;
        double *f = out + 5 * (size_t)k;
        uint64_t T = 0;
        for (size_t t = 0; t < nbins; ++t) T += P[t];
        if (T == 0) {
            for (int c = 0; c < 5; ++c) f[c] = 0.0;
            continue;
        }
        double contrast = 0, energy = 0, entropy = 0, homog = 0;
        double mu_i = 0, mu_j = 0;
        for (int i = 0; i < N; ++i) {
            for (int j = 0; j < N; ++j) {
                double p = (double)P[(size_t)i * N + j] / (double)T;
                double d = (double)(i - j);
                contrast += d * d * p;
                energy += p * p;
                if (p > 0) entropy -= p * log(p);
                homog += p / (1.0 + d * d);
                mu_i += i * p;
                mu_j += j * p;
            }
        }
        /* Row and column marginals: is either concentrated on one level? */
        int rows_used = 0, cols_used = 0;
        for (int i = 0; i < N; ++i) {
            uint64_t r = 0, c = 0;
            for (int j = 0; j < N; ++j) {
                r += P[(size_t)i * N + j];
                c += P[(size_t)j * N + i];
            }
            rows_used += (r != 0);
            cols_used += (c != 0);
        }
        double var_i = 0, var_j = 0, cov = 0;
        for (int i = 0; i < N; ++i) {
            for (int j = 0; j < N; ++j) {
                double p = (double)P[(size_t)i * N + j] / (double)T;
                var_i += (i - mu_i) * (i - mu_i) * p;
                var_j += (j - mu_j) * (j - mu_j) * p;
                cov += (i - mu_i) * (j - mu_j) * p;
            }
        }
        double corr = (rows_used == 1 || cols_used == 1) ? 1.0 : cov / sqrt(var_i * var_j);
        f[0] = contrast;
        f[1] = energy;
        f[2] = entropy;
        f[3] = homog;
        f[4] = corr;
    }
}
