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
 *   histogram     The paper remarks (Contributions) that its analysis of
 *                 colliding increments carries over to statistical histograms.
 *                 h[i] = number of pixels with q(v) = i.
 *   symmetric     A reading of Section I.B (both coordinates of the pair are
 *                 incremented): S = P + P^T, wrapping modulo 2^32.
 *   normalize     p = P / T per matrix in double; T = 0 gives zeros.
 *   average       Mean over consecutive groups of m matrices of their
 *                 normalised matrices (each direction weighted equally; an
 *                 empty matrix contributes zeros): the direction-averaged GLCM.
 *   haralick      Haralick's statistics f1..f13 (the fourteen cited in the
 *                 introduction, without the maximal correlation coefficient),
 *                 levels numbered from 0: f1 angular second moment, f2 contrast,
 *                 f3 correlation, f4 sum of squares (variance of the row
 *                 marginal), f5 inverse difference moment, f6 sum average,
 *                 f7 sum variance (about f6), f8 sum entropy, f9 entropy,
 *                 f10 difference variance, f11 difference entropy, f12 and f13
 *                 the two information measures of correlation.  Natural logs.
 *                 T = 0 gives zeros; f3 = 1 for a marginal on a single level;
 *                 f12 = 0 when both marginal entropies are 0.
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

/*
 * 1-D histogram of the quantized levels (see header).  Returns 0, or -1 for
 * bad arguments.  out has N entries and is overwritten.
 */
int oracle_histogram(const void *img, int W, int H, int64_t stride, int bytes_per_px, int N,
                     uint32_t lo, uint32_t hi, uint32_t *out)
{
    if (W < 1 || H < 1 || N < 1 || stride < W || lo > hi) return -1;
    if (bytes_per_px != 1 && bytes_per_px != 2) return -1;
    memset(out, 0, (size_t)N * sizeof(uint32_t));
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            out[oracle_quantize(pixel_at(img, bytes_per_px, stride, x, y), N, lo, hi)] += 1;
    return 0;
}

/* S[k][i][j] = P[k][i][j] + P[k][j][i], modulo 2^32 (see header). */
void oracle_symmetric(const uint32_t *glcm, int K, int N, uint32_t *out)
{
    size_t nbins = (size_t)N * (size_t)N;
    for (int k = 0; k < K; ++k) {
        const uint32_t *P = glcm + (size_t)k * nbins;
        uint32_t *S = out + (size_t)k * nbins;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j)
                S[(size_t)i * N + j] = P[(size_t)i * N + j] + P[(size_t)j * N + i];
    }
}

static uint64_t total_of(const uint32_t *P, size_t nbins)
{
    uint64_t T = 0;
    for (size_t t = 0; t < nbins; ++t) T += P[t];
    return T;
}

/* p[k][i][j] = P[k][i][j] / T_k in double; T_k = 0 gives zeros. */
void oracle_normalize(const uint32_t *glcm, int K, int N, double *out)
{
    size_t nbins = (size_t)N * (size_t)N;
    for (int k = 0; k < K; ++k) {
        const uint32_t *P = glcm + (size_t)k * nbins;
        uint64_t T = total_of(P, nbins);
        for (size_t t = 0; t < nbins; ++t)
            out[(size_t)k * nbins + t] = T ? (double)P[t] / (double)T : 0.0;
    }
}

/*
 * out[g][i][j] = (1/m) * sum over k in [g m, g m + m) of P_k[i][j] / T_k, in
 * double, k ascending (see header).  K must be a multiple of m.
 */
void oracle_average(const uint32_t *glcm, int K, int N, int m, double *out)
{
    size_t nbins = (size_t)N * (size_t)N;
    for (int g = 0; g < K / m; ++g) {
        double *A = out + (size_t)g * nbins;
        for (size_t t = 0; t < nbins; ++t) A[t] = 0.0;
        for (int k = g * m; k < g * m + m; ++k) {
            const uint32_t *P = glcm + (size_t)k * nbins;
            uint64_t T = total_of(P, nbins);
            if (!T) continue;
            for (size_t t = 0; t < nbins; ++t) A[t] += (double)P[t] / (double)T;
        }
        for (size_t t = 0; t < nbins; ++t) A[t] /= (double)m;
    }
}

/* -sum v ln v over the n entries v > 0. */
static double entropy_of(const double *v, int n)
{
    double h = 0.0;
    for (int t = 0; t < n; ++t)
        if (v[t] > 0) h -= v[t] * log(v[t]);
    return h;
}

/*
 * Haralick's f1..f13 per matrix, out[k*13 + 0..12] (see header), in double.
 * Marginals and the sum / difference distributions are exact integer sums
 * divided by T.
 */
int oracle_haralick(const uint32_t *glcm, int K, int N, double *out)
{
    size_t nbins = (size_t)N * (size_t)N;
    double *px = (double *)malloc((size_t)N * sizeof(double));
    double *py = (double *)malloc((size_t)N * sizeof(double));
    double *ps = (double *)malloc((size_t)(2 * N - 1) * sizeof(double));
    double *pd = (double *)malloc((size_t)N * sizeof(double));
    uint64_t *cs = (uint64_t *)malloc((size_t)(2 * N - 1) * sizeof(uint64_t));
    uint64_t *cd = (uint64_t *)malloc((size_t)N * sizeof(uint64_t));
    if (!px || !py || !ps || !pd || !cs || !cd) {
        free(px); free(py); free(ps); free(pd); free(cs); free(cd);
        return -1;
    }
    for (int k = 0; k < K; ++k) {
        const uint32_t *P = glcm + (size_t)k * nbins;
        double *f = out + 13 * (size_t)k;
        uint64_t T = total_of(P, nbins);
        for (int c = 0; c < 13; ++c) f[c] = 0.0;
        if (T == 0) continue;
        /* marginals, sum (i + j) and difference |i - j| distributions */
        int rows_used = 0, cols_used = 0;
        for (int t = 0; t < 2 * N - 1; ++t) cs[t] = 0;
        for (int t = 0; t < N; ++t) cd[t] = 0;
        for (int i = 0; i < N; ++i) {
            uint64_t r = 0, c = 0;
            for (int j = 0; j < N; ++j) {
                r += P[(size_t)i * N + j];
                c += P[(size_t)j * N + i];
                cs[i + j] += P[(size_t)i * N + j];
                cd[i > j ? i - j : j - i] += P[(size_t)i * N + j];
            }
            px[i] = (double)r / (double)T;
            py[i] = (double)c / (double)T;
            rows_used += (r != 0);
            cols_used += (c != 0);
        }
        for (int t = 0; t < 2 * N - 1; ++t) ps[t] = (double)cs[t] / (double)T;
        for (int t = 0; t < N; ++t) pd[t] = (double)cd[t] / (double)T;
        double mux = 0, muy = 0, varx = 0, vary = 0;
        for (int i = 0; i < N; ++i) { mux += i * px[i]; muy += i * py[i]; }
        for (int i = 0; i < N; ++i) {
            varx += (i - mux) * (i - mux) * px[i];
            vary += (i - muy) * (i - muy) * py[i];
        }
        double asm_ = 0, contrast = 0, idm = 0, ent = 0, cov = 0, hxy1 = 0, hxy2 = 0;
        for (int i = 0; i < N; ++i) {
            for (int j = 0; j < N; ++j) {
                double p = (double)P[(size_t)i * N + j] / (double)T;
                double d = (double)(i - j);
                asm_ += p * p;
                contrast += d * d * p;
                idm += p / (1.0 + d * d);
                cov += (i - mux) * (j - muy) * p;
                if (p > 0) {
                    ent -= p * log(p);
                    hxy1 -= p * log(px[i] * py[j]);
                }
                double q = px[i] * py[j];
                if (q > 0) hxy2 -= q * log(q);
            }
        }
        double sa = 0, sv = 0, da = 0, dv = 0;
        for (int t = 0; t < 2 * N - 1; ++t) sa += t * ps[t];
        for (int t = 0; t < 2 * N - 1; ++t) sv += (t - sa) * (t - sa) * ps[t];
        for (int t = 0; t < N; ++t) da += t * pd[t];
        for (int t = 0; t < N; ++t) dv += (t - da) * (t - da) * pd[t];
        double hx = entropy_of(px, N), hy = entropy_of(py, N);
        double hmax = hx > hy ? hx : hy;
        double x = 1.0 - exp(-2.0 * (hxy2 - ent));
        f[0] = asm_;
        f[1] = contrast;
        f[2] = (rows_used == 1 || cols_used == 1) ? 1.0 : cov / sqrt(varx * vary);
        f[3] = varx;
        f[4] = idm;
        f[5] = sa;
        f[6] = sv;
        f[7] = entropy_of(ps, 2 * N - 1);
        f[8] = ent;
        f[9] = dv;
        f[10] = entropy_of(pd, N);
        f[11] = hmax > 0 ? (ent - hxy1) / hmax : 0.0;
        f[12] = sqrt(x > 0 ? x : 0.0);
    }
    free(px); free(py); free(ps); free(pd); free(cs); free(cd);
    return 0;
}
