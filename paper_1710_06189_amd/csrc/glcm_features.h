// Haralick statistics of one GLCM computed by a whole workgroup: shared by the
// features kernel and the batch kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace glcm {
namespace {

// ---------------------------------------------------------------------------
// Haralick statistics of one GLCM computed by a whole workgroup (blockDim a
// multiple of 64, at most 1024).  Exact integer sums for the contrast
// numerator and the correlation moments; fp32 for energy, entropy and
// homogeneity; fp64 (from exact 128-bit integers) for the correlation.
// Sums are reduced within each wavefront by lane exchanges, then across the
// wavefronts through LDS: three barriers in all.  redu: 7 blockDim / 64
// words, redf: 3 blockDim / 64 words of workgroup scratch.  Every thread of
// the workgroup must call it.
// ---------------------------------------------------------------------------
// Wavefront sum by DPP lane moves (no LDS round trips): prefix sums within
// each row of 16 lanes (row_shr 1, 2, 4, 8), then lane 15 of rows 0 and 2 is
// added into rows 1 and 3 (row_bcast:15) and lane 31 into rows 2 and 3
// (row_bcast:31), leaving the total in lane 63, which is returned to all.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_move(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, true);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_move(unsigned long long v) {
  return (unsigned long long)dpp_move<CTRL, ROWS>((uint32_t)v) |
         ((unsigned long long)dpp_move<CTRL, ROWS>((uint32_t)(v >> 32)) << 32);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_move(float v) {
  return __uint_as_float(dpp_move<CTRL, ROWS>(__float_as_uint(v)));
}
__device__ __forceinline__ uint32_t lane63(uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, 63); }
__device__ __forceinline__ unsigned long long lane63(unsigned long long v) {
  return (unsigned long long)lane63((uint32_t)v) | ((unsigned long long)lane63((uint32_t)(v >> 32)) << 32);
}
__device__ __forceinline__ float lane63(float v) { return __uint_as_float(lane63(__float_as_uint(v))); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp_move<0x111, 0xf>(v);  // row_shr:1
  v += dpp_move<0x112, 0xf>(v);  // row_shr:2
  v += dpp_move<0x114, 0xf>(v);  // row_shr:4
  v += dpp_move<0x118, 0xf>(v);  // row_shr:8
  v += dpp_move<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
  v += dpp_move<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
  return lane63(v);
}

// The five statistics from the exact integer sums and the fp32 sums.
__device__ __forceinline__ void features_store(unsigned long long T, unsigned long long sc, unsigned long long si,
                                               unsigned long long sj, unsigned long long sii, unsigned long long sjj,
                                               unsigned long long sij, float energy, float ent, float homog,
                                               float* o) {
  using i128 = __int128;
  const i128 tT = (i128)T;
  const i128 vi = (i128)sii * tT - (i128)si * (i128)si;  // T^2 var_i
  const i128 vj = (i128)sjj * tT - (i128)sj * (i128)sj;  // T^2 var_j
  const i128 cv = (i128)sij * tT - (i128)si * (i128)sj;  // T^2 cov
  double corr = 1.0;
  if (vi != 0 && vj != 0) corr = (double)cv / sqrt((double)vi * (double)vj);
  o[0] = (float)((double)sc / (double)T);
  o[1] = energy;
  o[2] = ent;
  o[3] = homog;
  o[4] = (float)corr;
}

__device__ __forceinline__ void glcm_features_wg(const uint32_t* P, uint32_t N, float* o, unsigned long long* redu, float* redf) {
  const uint32_t NN = N * N, nw = blockDim.x >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // pass 1: total (needed for p)
  unsigned long long T = 0;
  for (uint32_t t = threadIdx.x; t < NN; t += blockDim.x) T += P[t];
  T = wave_sum(T);
  if (lane == 0) redu[w] = T;
  __syncthreads();
  T = 0;
  for (uint32_t x = 0; x < nw; ++x) T += redu[x];
  if (T == 0 || T > 0xffffffffull) {
    if (threadIdx.x < 5) o[threadIdx.x] = T == 0 ? 0.0f : __builtin_nanf("");
    __syncthreads();
    return;
  }
  const float invT = 1.0f / (float)T;
  unsigned long long sc = 0, si = 0, sj = 0, sii = 0, sjj = 0, sij = 0;
  float energy = 0.f, ent = 0.f, homog = 0.f;
  // bin t = i N + j; (i, j) step by blockDim's digits in base N
  const uint32_t di = blockDim.x / N, dj = blockDim.x % N;
  uint32_t i = threadIdx.x / N, j = threadIdx.x % N;
  for (uint32_t t = threadIdx.x; t < NN; t += blockDim.x) {
    const uint32_t c = P[t];
    if (c != 0) {
      const unsigned long long d = i > j ? i - j : j - i;
      sc += d * d * c;
      si += (unsigned long long)i * c; sj += (unsigned long long)j * c;
      sii += (unsigned long long)i * i * c; sjj += (unsigned long long)j * j * c;
      sij += (unsigned long long)i * j * c;
      const float p = (float)c * invT;
      energy += p * p;
      // -p ln p; for p > 1/2 use log1p of the exact complement to keep accuracy
      const float lp = (2ull * c > T) ? log1pf(-(float)(T - c) * invT) : logf(p);
      ent -= p * lp;
      homog += p / (1.0f + (float)(d * d));
    }
    j += dj;
    i += di;
    if (j >= N) {
      j -= N;
      ++i;
    }
  }
  sc = wave_sum(sc); si = wave_sum(si); sj = wave_sum(sj);
  sii = wave_sum(sii); sjj = wave_sum(sjj); sij = wave_sum(sij);
  energy = wave_sum(energy); ent = wave_sum(ent); homog = wave_sum(homog);
  unsigned long long* ru = redu + nw;  // the totals above stay readable
  if (lane == 0) {
    ru[6 * w + 0] = sc; ru[6 * w + 1] = si; ru[6 * w + 2] = sj;
    ru[6 * w + 3] = sii; ru[6 * w + 4] = sjj; ru[6 * w + 5] = sij;
    redf[3 * w + 0] = energy; redf[3 * w + 1] = ent; redf[3 * w + 2] = homog;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sc = si = sj = sii = sjj = sij = 0;
    energy = ent = homog = 0.f;
    for (uint32_t x = 0; x < nw; ++x) {
      sc += ru[6 * x + 0]; si += ru[6 * x + 1]; sj += ru[6 * x + 2];
      sii += ru[6 * x + 3]; sjj += ru[6 * x + 4]; sij += ru[6 * x + 5];
      energy += redf[3 * x + 0]; ent += redf[3 * x + 1]; homog += redf[3 * x + 2];
    }
    features_store(T, sc, si, sj, sii, sjj, sij, energy, ent, homog, o);
  }
  __syncthreads();  // the scratch may be reused once every thread is past it
}

// The same statistics computed by one wavefront, with no LDS and no barrier:
// bit for bit what glcm_features_wg gives in a workgroup of one wavefront
// (there the sums of the single wavefront are added to zero, which changes
// nothing).  Every lane must call it; lane 0 writes o.
__device__ __forceinline__ void glcm_features_wave(const uint32_t* P, uint32_t N, float* o) {
  const uint32_t NN = N * N, lane = threadIdx.x & 63;
  unsigned long long T = 0;
  for (uint32_t t = lane; t < NN; t += 64u) T += P[t];
  T = wave_sum(T);
  if (T == 0 || T > 0xffffffffull) {
    if (lane < 5) o[lane] = T == 0 ? 0.0f : __builtin_nanf("");
    return;
  }
  const float invT = 1.0f / (float)T;
  unsigned long long sc = 0, si = 0, sj = 0, sii = 0, sjj = 0, sij = 0;
  float energy = 0.f, ent = 0.f, homog = 0.f;
  const uint32_t di = 64u / N, dj = 64u % N;
  uint32_t i = lane / N, j = lane % N;
  for (uint32_t t = lane; t < NN; t += 64u) {
    const uint32_t c = P[t];
    if (c != 0) {
      const unsigned long long d = i > j ? i - j : j - i;
      sc += d * d * c;
      si += (unsigned long long)i * c; sj += (unsigned long long)j * c;
      sii += (unsigned long long)i * i * c; sjj += (unsigned long long)j * j * c;
      sij += (unsigned long long)i * j * c;
      const float p = (float)c * invT;
      energy += p * p;
      const float lp = (2ull * c > T) ? log1pf(-(float)(T - c) * invT) : logf(p);
      ent -= p * lp;
      homog += p / (1.0f + (float)(d * d));
    }
    j += dj;
    i += di;
    if (j >= N) {
      j -= N;
      ++i;
    }
  }
  sc = wave_sum(sc); si = wave_sum(si); sj = wave_sum(sj);
  sii = wave_sum(sii); sjj = wave_sum(sjj); sij = wave_sum(sij);
  energy = wave_sum(energy); ent = wave_sum(ent); homog = wave_sum(homog);
  if (lane == 0) features_store(T, sc, si, sj, sii, sjj, sij, 0.f + energy, 0.f + ent, 0.f + homog, o);
}

}  // namespace
}  // namespace glcm
