// Post-processing of K co-occurrence matrices (N x N uint32 counts, the layout
// glcm_compute writes): the symmetric matrix P + P^T (a reading of the pair
// increment of Section I.B), the normalised matrix P / sum P, the mean of the
// normalised matrices over groups of directions, and Haralick's statistics
// f1..f13 (cited in the introduction).  Everything is computed in fp64 and
// stored as fp32, in a fixed order of operations: the same input always gives
// the same bits.

#include <hip/hip_runtime.h>

#include "glcm_device.h"
#include "glcm_stats.h"

namespace glcm {
namespace {

constexpr int kStatsThreads = 256;
constexpr int kStatsWaves = kStatsThreads / 64;

// Sum over the workgroup, the same value returned to every thread.  The
// butterfly and the wave order are fixed, so the result is deterministic.
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* part) {
  for (int o = 32; o; o >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, o);
  __syncthreads();  // the previous call's readers are done with part
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t s = 0;
  for (int w = 0; w < kStatsWaves; ++w) s += part[w];
  return s;
}

template <int M>
__device__ __forceinline__ void block_sum_f64(double (&v)[M], double* part) {
#pragma unroll
  for (int m = 0; m < M; ++m)
    for (int o = 32; o; o >>= 1) v[m] += __shfl_xor(v[m], o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int m = 0; m < M; ++m) part[(threadIdx.x >> 6) * M + m] = v[m];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) {
    double s = 0.0;
    for (int w = 0; w < kStatsWaves; ++w) s += part[w * M + m];
    v[m] = s;
  }
}

__device__ __forceinline__ uint64_t matrix_total(const uint32_t* P, uint32_t NN, uint64_t* part) {
  uint64_t t = 0;
  for (uint32_t r = threadIdx.x; r < NN; r += blockDim.x) t += P[r];
  return block_sum_u64(t, part);
}

// S = P + P^T modulo 2^32.  The thread of bin (i, j) with i <= j reads both
// bins before writing both, so in == out is safe.
__global__ __launch_bounds__(kStatsThreads) void k_symmetrize(StatsArgs a) {
  const uint32_t N = (uint32_t)a.N, NN = N * N;
  for (int k = blockIdx.x; k < a.K; k += gridDim.x) {
    const uint32_t* P = a.in + (size_t)k * NN;
    uint32_t* S = a.out_u + (size_t)k * NN;
    for (uint32_t r = threadIdx.x; r < NN; r += blockDim.x) {
      const uint32_t i = divide(r, a.nmagic, a.nshift), j = r - i * N;
      if (i > j) continue;
      const uint32_t s = P[r] + P[j * N + i];
      S[r] = s;
      S[j * N + i] = s;
    }
  }
}

// p = P / T, the quotient correctly rounded in fp64 and then to fp32.
__global__ __launch_bounds__(kStatsThreads) void k_normalize(StatsArgs a) {
  __shared__ uint64_t part[kStatsWaves];
  const uint32_t NN = (uint32_t)a.N * (uint32_t)a.N;
  for (int k = blockIdx.x; k < a.K; k += gridDim.x) {
    const uint32_t* P = a.in + (size_t)k * NN;
    const uint64_t T = matrix_total(P, NN, part);
    const double dT = (double)T;
    float* o = a.out_f + (size_t)k * NN;
    for (uint32_t r = threadIdx.x; r < NN; r += blockDim.x) o[r] = T ? (float)((double)P[r] / dT) : 0.0f;
  }
}

// out[g] = (sum over the m matrices of group g, in order, of P_k / T_k) / m;
// an empty matrix adds nothing.
__global__ __launch_bounds__(kStatsThreads) void k_average(StatsArgs a) {
  __shared__ uint64_t part[kStatsWaves];
  __shared__ uint64_t totals[kAverageMaxGroup];
  const uint32_t NN = (uint32_t)a.N * (uint32_t)a.N;
  const int G = a.K / a.m;
  for (int g = blockIdx.x; g < G; g += gridDim.x) {
    const uint32_t* P0 = a.in + (size_t)g * a.m * NN;
    for (int q = 0; q < a.m; ++q) {
      const uint64_t T = matrix_total(P0 + (size_t)q * NN, NN, part);
      if (threadIdx.x == 0) totals[q] = T;
    }
    __syncthreads();
    float* o = a.out_f + (size_t)g * NN;
    for (uint32_t r = threadIdx.x; r < NN; r += blockDim.x) {
      double acc = 0.0;
      for (int q = 0; q < a.m; ++q) {
        const uint64_t T = totals[q];
        if (T) acc += (double)P0[(size_t)q * NN + r] / (double)T;
      }
      o[r] = (float)(acc / (double)a.m);
    }
    __syncthreads();  // totals is rewritten for the next group
  }
}

__device__ __forceinline__ double neg_plogp(double p) { return p > 0.0 ? -p * log(p) : 0.0; }

// Haralick's f1..f13 of one matrix per workgroup (levels numbered from 0):
// f1 angular second moment, f2 contrast, f3 correlation, f4 variance of the
// row marginal, f5 inverse difference moment, f6 sum average, f7 sum
// variance, f8 sum entropy, f9 entropy, f10 difference variance, f11
// difference entropy, f12 and f13 the information measures of correlation.
// The marginals and the distributions of i + j and |i - j| are exact integer
// sums over rows, columns and (anti-)diagonals divided by T.
__global__ __launch_bounds__(kStatsThreads) void k_haralick(StatsArgs a) {
  extern __shared__ double sh[];  // px[N] py[N] ps[2N - 1] pd[N] lpx[N] lpy[N]
  __shared__ uint64_t part[kStatsWaves];
  __shared__ double dpart[kStatsWaves * 10];
  const int N = a.N;
  const uint32_t NN = (uint32_t)N * (uint32_t)N;
  double* px = sh;
  double* py = px + N;
  double* ps = py + N;
  double* pd = ps + (2 * N - 1);
  double* lpx = pd + N;  // ln px (0 where px = 0)
  double* lpy = lpx + N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = blockIdx.x; k < a.K; k += gridDim.x) {
    const uint32_t* P = a.in + (size_t)k * NN;
    float* f = a.out_f + (size_t)k * kHaralickStats;
    const uint64_t T = matrix_total(P, NN, part);
    if (T == 0) {
      if (threadIdx.x < kHaralickStats) f[threadIdx.x] = 0.0f;
      continue;
    }
    const double inv = 1.0 / (double)T;  // p = P * (1/T), within an ulp of P / T
    // row marginal: a wavefront per row
    for (int i = wave; i < N; i += kStatsWaves) {
      uint64_t s = 0;
      for (int j = lane; j < N; j += 64) s += P[(size_t)i * N + j];
      for (int o = 32; o; o >>= 1) s += (uint64_t)__shfl_xor((unsigned long long)s, o);
      if (lane == 0) px[i] = (double)s * inv;
    }
    // column marginal, sum and difference distributions: a thread per entry
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
      uint64_t s = 0;
      for (int i = 0; i < N; ++i) s += P[(size_t)i * N + j];
      py[j] = (double)s * inv;
    }
    for (int t = threadIdx.x; t < 2 * N - 1; t += blockDim.x) {
      uint64_t s = 0;
      for (int i = max(0, t - N + 1); i <= min(t, N - 1); ++i) s += P[(size_t)i * N + (t - i)];
      ps[t] = (double)s * inv;
    }
    for (int d = threadIdx.x; d < N; d += blockDim.x) {
      uint64_t s = 0;
      for (int i = 0; i + d < N; ++i) s += P[(size_t)i * N + i + d];
      if (d)
        for (int i = 0; i + d < N; ++i) s += P[(size_t)(i + d) * N + i];
      pd[d] = (double)s * inv;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      lpx[i] = px[i] > 0.0 ? log(px[i]) : 0.0;
      lpy[i] = py[i] > 0.0 ? log(py[i]) : 0.0;
    }
    // first moments, entropies of the marginals and distributions, occupied rows/columns
    double m1[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      m1[0] += i * px[i];
      m1[1] += i * py[i];
      m1[3] += i * pd[i];
      m1[4] += neg_plogp(px[i]);
      m1[5] += neg_plogp(py[i]);
      m1[7] += neg_plogp(pd[i]);
      m1[8] += px[i] > 0.0 ? 1.0 : 0.0;
      m1[9] += py[i] > 0.0 ? 1.0 : 0.0;
    }
    for (int t = threadIdx.x; t < 2 * N - 1; t += blockDim.x) {
      m1[2] += t * ps[t];
      m1[6] += neg_plogp(ps[t]);
    }
    block_sum_f64<10>(m1, dpart);  // (its barriers also publish lpx, lpy)
    const double mux = m1[0], muy = m1[1], sa = m1[2], da = m1[3];
    // second moments about those means
    double m2[4] = {0, 0, 0, 0};
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      m2[0] += (i - mux) * (i - mux) * px[i];
      m2[1] += (i - muy) * (i - muy) * py[i];
      m2[3] += (i - da) * (i - da) * pd[i];
    }
    for (int t = threadIdx.x; t < 2 * N - 1; t += blockDim.x) m2[2] += (t - sa) * (t - sa) * ps[t];
    block_sum_f64<4>(m2, dpart);
    // sums over the bins
    double b[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
    for (uint32_t r = threadIdx.x; r < NN; r += blockDim.x) {
      const uint32_t i = divide(r, a.nmagic, a.nshift), j = r - i * (uint32_t)N;
      const double p = (double)P[r] * inv, d = (double)i - (double)j;
      const double q = px[i] * py[j], lq = lpx[i] + lpy[j];  // ln q = ln px + ln py
      b[0] += p * p;
      b[1] += d * d * p;
      b[2] += p / (1.0 + d * d);
      b[4] += ((double)i - mux) * ((double)j - muy) * p;
      if (p > 0.0) {
        b[3] -= p * log(p);
        b[5] -= p * lq;
      }
      if (q > 0.0) b[6] -= q * lq;
    }
    block_sum_f64<7>(b, dpart);
    if (threadIdx.x == 0) {
      const double varx = m2[0], vary = m2[1], ent = b[3], hx = m1[4], hy = m1[5];
      const double hmax = hx > hy ? hx : hy;
      const double x = 1.0 - exp(-2.0 * (b[6] - ent));
      f[0] = (float)b[0];
      f[1] = (float)b[1];
      f[2] = (float)((m1[8] == 1.0 || m1[9] == 1.0) ? 1.0 : b[4] / sqrt(varx * vary));
      f[3] = (float)varx;
      f[4] = (float)b[2];
      f[5] = (float)sa;
      f[6] = (float)m2[2];
      f[7] = (float)m1[6];
      f[8] = (float)ent;
      f[9] = (float)m2[3];
      f[10] = (float)m1[7];
      f[11] = (float)(hmax > 0.0 ? (ent - b[5]) / hmax : 0.0);
      f[12] = (float)sqrt(x > 0.0 ? x : 0.0);
    }
    __syncthreads();  // the marginals are rewritten for the next matrix
  }
}

__device__ __forceinline__ double wave_sum_f64(double v) {
  for (int o = 32; o; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  for (int o = 32; o; o >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, o);
  return v;
}

// Orders a wavefront's LDS writes before its lanes read each other's words.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kWaveMaxN = 32;

// The same statistics for N <= 32, one matrix per wavefront: the matrix is
// copied once into the wavefront's LDS (coalesced loads); lane l then forms
// px[l], py[l], pd[l] (l < N) and ps[l] (l < 2N - 1) from it, other lanes'
// entries come by shuffles, and every sum is a wavefront butterfly, so no
// workgroup barrier is needed.  p = P * (1/T) here (within an ulp of P / T);
// lane l also holds 1 / (1 + l^2) for the inverse difference moment.  The
// statistics of the marginals wait in LDS while the bins are summed, which
// keeps the register count low enough for several wavefronts per SIMD.
__global__ __launch_bounds__(kStatsThreads, 4) void k_haralick_wave(StatsArgs a) {
  __shared__ uint32_t tiles[kStatsWaves][kWaveMaxN * kWaveMaxN];
  __shared__ double parked[kStatsWaves][12];
  const int N = a.N;
  const uint32_t NN = (uint32_t)N * (uint32_t)N;
  const int lane = threadIdx.x & 63;
  uint32_t* M = tiles[threadIdx.x >> 6];
  double* st = parked[threadIdx.x >> 6];
  const double l = (double)lane, idm_w = 1.0 / (1.0 + l * l);
  const int nwaves = gridDim.x * kStatsWaves;
  for (int k = blockIdx.x * kStatsWaves + (threadIdx.x >> 6); k < a.K; k += nwaves) {
    const uint32_t* P = a.in + (size_t)k * NN;
    float* f = a.out_f + (size_t)k * kHaralickStats;
    wave_lds_sync();  // the previous matrix's reads of M and st are done
    uint64_t t = 0;
    for (uint32_t r = lane; r < NN; r += 64) {
      const uint32_t v = P[r];
      M[r] = v;
      t += v;
    }
    const uint64_t T = wave_sum_u64(t);
    if (T == 0) {
      if (lane < kHaralickStats) f[lane] = 0.0f;
      continue;
    }
    wave_lds_sync();
    const double inv = 1.0 / (double)T;
    double px, py, lpx, lpy, mux, muy;
    {
      uint64_t sx = 0, sy = 0, ss = 0, sd = 0;
      if (lane < N) {
        for (int j = 0; j < N; ++j) sx += M[lane * N + j];
        for (int i = 0; i < N; ++i) sy += M[i * N + lane];
        for (int i = 0; i + lane < N; ++i) sd += M[i * N + i + lane];
        if (lane)
          for (int i = 0; i + lane < N; ++i) sd += M[(i + lane) * N + i];
      }
      if (lane < 2 * N - 1)
        for (int i = max(0, lane - N + 1); i <= min(lane, N - 1); ++i) ss += M[i * N + (lane - i)];
      px = (double)sx * inv;
      py = (double)sy * inv;
      const double ps = (double)ss * inv, pd = (double)sd * inv;
      lpx = px > 0.0 ? log(px) : 0.0;
      lpy = py > 0.0 ? log(py) : 0.0;
      mux = wave_sum_f64(l * px);
      muy = wave_sum_f64(l * py);
      const double sa = wave_sum_f64(l * ps), da = wave_sum_f64(l * pd);
      const double v0 = wave_sum_f64(-px * lpx), v1 = wave_sum_f64(-py * lpy);
      const double v2 = wave_sum_f64(neg_plogp(ps)), v3 = wave_sum_f64(neg_plogp(pd));
      const double v4 = wave_sum_f64(px > 0.0 ? 1.0 : 0.0), v5 = wave_sum_f64(py > 0.0 ? 1.0 : 0.0);
      const double v6 = wave_sum_f64((l - mux) * (l - mux) * px), v7 = wave_sum_f64((l - muy) * (l - muy) * py);
      const double v8 = wave_sum_f64((l - sa) * (l - sa) * ps), v9 = wave_sum_f64((l - da) * (l - da) * pd);
      if (lane == 0) {
        st[0] = v0; st[1] = v1; st[2] = v2; st[3] = v3; st[4] = v4; st[5] = v5;
        st[6] = v6; st[7] = v7; st[8] = v8; st[9] = v9; st[10] = sa;
      }
    }
    double b[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
    for (uint32_t r = lane; r < NN; r += 64) {
      const uint32_t i = divide(r, a.nmagic, a.nshift), j = r - i * (uint32_t)N;
      const double p = (double)M[r] * inv, d = (double)i - (double)j;
      const double q = __shfl(px, (int)i) * __shfl(py, (int)j);
      const double lq = __shfl(lpx, (int)i) + __shfl(lpy, (int)j);
      b[0] += p * p;
      b[1] += d * d * p;
      b[2] += p * __shfl(idm_w, (int)(i > j ? i - j : j - i));
      b[4] += ((double)i - mux) * ((double)j - muy) * p;
      if (p > 0.0) {
        b[3] -= p * log(p);
        b[5] -= p * lq;
      }
      if (q > 0.0) b[6] -= q * lq;
    }
#pragma unroll
    for (int c = 0; c < 7; ++c) b[c] = wave_sum_f64(b[c]);
    wave_lds_sync();
    if (lane == 0) {
      const double hx = st[0], hy = st[1], varx = st[6], vary = st[7];
      const double ent = b[3], hmax = hx > hy ? hx : hy;
      const double x = 1.0 - exp(-2.0 * (b[6] - ent));
      f[0] = (float)b[0];
      f[1] = (float)b[1];
      f[2] = (float)((st[4] == 1.0 || st[5] == 1.0) ? 1.0 : b[4] / sqrt(varx * vary));
      f[3] = (float)varx;
      f[4] = (float)b[2];
      f[5] = (float)st[10];
      f[6] = (float)st[8];
      f[7] = (float)st[2];
      f[8] = (float)ent;
      f[9] = (float)st[9];
      f[10] = (float)st[3];
      f[11] = (float)(hmax > 0.0 ? (ent - b[5]) / hmax : 0.0);
      f[12] = (float)sqrt(x > 0.0 ? x : 0.0);
    }
  }
}

unsigned grid_for(int units) { return (unsigned)(units < 8192 ? (units > 0 ? units : 1) : 8192); }

}  // namespace

hipError_t launch_symmetrize(const StatsArgs& a, hipStream_t stream) {
  hipLaunchKernelGGL(k_symmetrize, dim3(grid_for(a.K)), dim3(kStatsThreads), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_normalize(const StatsArgs& a, hipStream_t stream) {
  hipLaunchKernelGGL(k_normalize, dim3(grid_for(a.K)), dim3(kStatsThreads), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_average(const StatsArgs& a, hipStream_t stream) {
  hipLaunchKernelGGL(k_average, dim3(grid_for(a.K / a.m)), dim3(kStatsThreads), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_haralick(const StatsArgs& a, hipStream_t stream) {
  if (a.N <= kWaveMaxN) {
    hipLaunchKernelGGL(k_haralick_wave, dim3(grid_for((a.K + kStatsWaves - 1) / kStatsWaves)), dim3(kStatsThreads), 0,
                       stream, a);
    return hipGetLastError();
  }
  const size_t lds = (size_t)(7 * a.N - 1) * sizeof(double);
  hipLaunchKernelGGL(k_haralick, dim3(grid_for(a.K)), dim3(kStatsThreads), (uint32_t)lds, stream, a);
  return hipGetLastError();
}

}  // namespace glcm
