// Haralick's maximal correlation coefficient (the fourteenth statistic) of K
// co-occurrence matrices, fp64 on the device.

#include <hip/hip_runtime.h>

#include "glcm_device.h"
#include "glcm_stats.h"

namespace glcm {
namespace {

// Wavefront sums by butterfly: every lane ends with the same bits (each step
// adds the same two values on both lanes of a pair), so decisions taken on
// them are uniform.
__device__ __forceinline__ double wave_sum_f64(double v) {
  for (int o = 32; o; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  for (int o = 32; o; o >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, o);
  return v;
}

unsigned grid_for(int units) { return (unsigned)(units < 8192 ? (units > 0 ? units : 1) : 8192); }

// Haralick's fourteenth statistic, the maximal correlation coefficient: the
// square root of the second largest eigenvalue of
// Q(i, j) = sum_c p(i, c) p(j, c) / (px(i) py(c)).  Q is similar to the
// symmetric S = B B^T with B(i, c) = p(i, c) / sqrt(px(i) py(c)) (0 where a
// marginal is 0), so the kernel forms S in LDS and diagonalises it with cyclic
// Jacobi rotations in fp64 (at most kMccSweeps sweeps, stopping once the
// off-diagonal norm is below 1e-13 of the diagonal's).  One 64-lane
// workgroup per matrix, N <= kMccMaxLevels.
constexpr int kMccSweeps = 30;

__global__ __launch_bounds__(64) void k_haralick_mcc(StatsArgs a) {
  extern __shared__ double mcc_sh[];  // B[N][N], S[N][N], rx[N], ry[N]
  const int N = a.N, lane = threadIdx.x;
  const uint32_t NN = (uint32_t)N * (uint32_t)N;
  double* Bm = mcc_sh;
  double* Sm = Bm + NN;
  double* rx = Sm + NN;
  double* ry = rx + N;
  __shared__ int rp[kMccMaxLevels / 2], rq[kMccMaxLevels / 2];  // the pairs of a round
  __shared__ double rc[kMccMaxLevels / 2], rs[kMccMaxLevels / 2];  // and their rotations
  for (int k = blockIdx.x; k < a.K; k += gridDim.x) {
    const uint32_t* P = a.in + (size_t)k * NN;
    uint64_t t = 0;
    for (uint32_t r = lane; r < NN; r += 64) t += P[r];
    const uint64_t T = wave_sum_u64(t);
    if (T == 0 || N == 1) {
      if (lane == 0) a.out_f[k] = 0.0f;
      continue;
    }
    const double inv = 1.0 / (double)T;
    if (lane < N) {
      uint64_t sx = 0, sy = 0;
      for (int c = 0; c < N; ++c) sx += P[lane * N + c];
      for (int i = 0; i < N; ++i) sy += P[i * N + lane];
      rx[lane] = sx ? 1.0 / sqrt((double)sx * inv) : 0.0;
      ry[lane] = sy ? 1.0 / sqrt((double)sy * inv) : 0.0;
    }
    __syncthreads();
    for (uint32_t r = lane; r < NN; r += 64) {
      const uint32_t i = divide(r, a.nmagic, a.nshift), c = r - i * (uint32_t)N;
      Bm[r] = (double)P[r] * inv * rx[i] * ry[c];
    }
    __syncthreads();
    for (uint32_t r = lane; r < NN; r += 64) {
      const uint32_t i = divide(r, a.nmagic, a.nshift), j = r - i * (uint32_t)N;
      double acc = 0.0;
      for (int c = 0; c < N; ++c) acc += Bm[i * N + c] * Bm[j * N + c];
      Sm[r] = acc;
    }
    __syncthreads();
    // Jacobi sweeps in tournament order: round r pairs the elements at
    // positions i and n2 - 1 - i of the circle (element 0 fixed, the others
    // rotated by r), so the N/2 rotations of a round touch disjoint rows and
    // columns and are applied together (an odd N gets a dummy partner)
    const int n2 = (N + 1) & ~1;
    for (int sweep = 0; sweep < kMccSweeps; ++sweep) {
      double off = 0.0, dia = 0.0;
      for (uint32_t r = lane; r < NN; r += 64) {
        const uint32_t i = divide(r, a.nmagic, a.nshift), j = r - i * (uint32_t)N;
        const double v = Sm[r];
        if (i == j) dia += v * v; else off += v * v;
      }
      off = wave_sum_f64(off);
      dia = wave_sum_f64(dia);
      // off-diagonal norm below 1e-13 of the diagonal's: the eigenvalues then
      // carry an error of order 1e-26 of the largest (second order in the
      // off-diagonal part); the same decision on every lane
      if (!(off > 1e-26 * dia)) break;
      for (int round = 0; round < n2 - 1; ++round) {
        if (lane < n2 / 2) {
          const int pa = lane, pb = n2 - 1 - lane;
          const int p = pa == 0 ? 0 : (pa - 1 + round) % (n2 - 1) + 1;
          const int q = (pb - 1 + round) % (n2 - 1) + 1;
          double cs = 1.0, sn = 0.0;
          if (p < N && q < N) {
            const double apq = Sm[p * N + q];
            if (apq != 0.0) {
              const double tau = (Sm[q * N + q] - Sm[p * N + p]) / (2.0 * apq);
              const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
              cs = 1.0 / sqrt(1.0 + tt * tt);
              sn = tt * cs;
            }
          }
          rp[lane] = p;
          rq[lane] = q;
          rc[lane] = cs;
          rs[lane] = sn;
        }
        __syncthreads();
        if (lane < N) {  // columns p and q of every pair, row `lane`
          for (int i = 0; i < n2 / 2; ++i) {
            const int p = rp[i], q = rq[i];
            if (p >= N || q >= N) continue;
            const double cs = rc[i], sn = rs[i];
            const double x = Sm[lane * N + p], y = Sm[lane * N + q];
            Sm[lane * N + p] = cs * x - sn * y;
            Sm[lane * N + q] = sn * x + cs * y;
          }
        }
        __syncthreads();
        if (lane < N) {  // rows p and q of every pair, column `lane`
          for (int i = 0; i < n2 / 2; ++i) {
            const int p = rp[i], q = rq[i];
            if (p >= N || q >= N) continue;
            const double cs = rc[i], sn = rs[i];
            const double x = Sm[p * N + lane], y = Sm[q * N + lane];
            Sm[p * N + lane] = cs * x - sn * y;
            Sm[q * N + lane] = sn * x + cs * y;
          }
        }
        __syncthreads();
      }
    }
    // the two largest diagonal entries: the first is 1 (eigenvector sqrt(px))
    const double d = lane < N ? Sm[lane * N + lane] : -1.0;
    double m1 = d;
    for (int o = 32; o; o >>= 1) m1 = fmax(m1, __shfl_xor(m1, o));
    const unsigned long long at = __ballot(d == m1);
    const int first = __ffsll((long long)at) - 1;  // one lane holding the largest
    double m2 = lane == first ? -1.0 : d;
    for (int o = 32; o; o >>= 1) m2 = fmax(m2, __shfl_xor(m2, o));
    if (lane == 0) a.out_f[k] = (float)sqrt(m2 > 0.0 ? m2 : 0.0);
    __syncthreads();  // Bm, Sm, rx, ry are rewritten for the next matrix
  }
}

}  // namespace

hipError_t launch_haralick_mcc(const StatsArgs& a, hipStream_t stream) {
  const size_t lds = (2 * (size_t)a.N * a.N + 2 * (size_t)a.N) * sizeof(double);
  hipLaunchKernelGGL(k_haralick_mcc, dim3(grid_for(a.K)), dim3(64), (uint32_t)lds, stream, a);
  return hipGetLastError();
}

}  // namespace glcm
