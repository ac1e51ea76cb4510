// Block- and wave-level helpers for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>

#include "prgd_internal.hpp"

namespace prgd {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum over the block in a fixed order (deterministic).  `sbuf` needs
// blockDim/64 doubles of shared memory.  Result valid in every thread.
__device__ inline double block_sum(double v, double *sbuf) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) sbuf[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < nw; ++i) r += sbuf[i];
  __syncthreads();
  return r;
}

__device__ inline double block_max(double v, double *sbuf) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) sbuf[w] = v;
  __syncthreads();
  double r = sbuf[0];
  for (int i = 1; i < nw; ++i) r = fmax(r, sbuf[i]);
  __syncthreads();
  return r;
}

// Sum of s and maximum of m over the block in one pass (one exchange through
// LDS), the same values in every thread.  sbuf: 32 doubles.
__device__ inline void block_sum_max(double &s, double &m, double *sbuf) {
  s = wave_sum(s);
  m = wave_max(m);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
    sbuf[w] = s;
    sbuf[16 + w] = m;
  }
  __syncthreads();
  s = 0.0;
  m = sbuf[16];
  for (int i = 0; i < nw; ++i) {
    s += sbuf[i];
    m = fmax(m, sbuf[16 + i]);
  }
  __syncthreads();
}

// Sum nb partial vectors part[b * ne + e] (b < nb, e < ne) into out[e] (LDS),
// deterministically.  Threads split the partials into groups with several
// independent accumulators each, so many loads are in flight at once (the
// partials were written by blocks on other XCDs and arrive with long latency).
// scratch: LDS of at least blockDim.x doubles.  Ends with a barrier.
__device__ inline void reduce_partials(const double *part_, int nb, int ne, double *out, double *scratch) {
  const int nt = blockDim.x, t = threadIdx.x;
  const auto part = glb(part_);
  if (ne <= nt) {
    const int G = nt / ne;                 // groups per entry
    const int g = t / ne, e = t % ne;
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (g < G) {
      int b = g;
      for (; b + 7 * G < nb; b += 8 * G) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += part[(long long)(b + u * G) * ne + e];
      }
      for (; b < nb; b += G) a[0] += part[(long long)b * ne + e];
      scratch[g * ne + e] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
    __syncthreads();
    for (int i = t; i < ne; i += nt) {
      double v = 0.0;
      for (int gg = 0; gg < G; ++gg) v += scratch[gg * ne + i];
      out[i] = v;
    }
  } else {
    for (int e = t; e < ne; e += nt) {
      double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      int b = 0;
      for (; b + 8 <= nb; b += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += part[(long long)(b + u) * ne + e];
      }
      for (; b < nb; ++b) a[0] += part[(long long)b * ne + e];
      out[e] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
  }
  __syncthreads();
}

// Two independent sets of partials reduced in one pass (their loads in
// flight together): nbA vectors of neA doubles at partA into outA and nbB of
// neB at partB into outB (both LDS).  Deterministic; the same order within
// each set as reduce_partials when neA + neB <= blockDim.x.  scratch: LDS of
// at least blockDim.x doubles.  Ends with a barrier.
__device__ inline void reduce_partials2(const double *partA, int nbA, int neA, double *outA, const double *partB,
                                        int nbB, int neB, double *outB, double *scratch) {
  const int ne = neA + neB;
  if (ne > (int)blockDim.x) {   // too wide for one pass
    reduce_partials(partA, nbA, neA, outA, scratch);
    reduce_partials(partB, nbB, neB, outB, scratch);
    return;
  }
  const int nt = blockDim.x, t = threadIdx.x;
  const int G = nt / ne, g = t / ne, e = t % ne;
  const bool inA = e < neA;
  const auto part = glb(inA ? partA : partB);
  const int nb = inA ? nbA : nbB, w = inA ? neA : neB, ee = inA ? e : e - neA;
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (g < G) {
    int b = g;
    for (; b + 7 * G < nb; b += 8 * G) {
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += part[(long long)(b + u * G) * w + ee];
    }
    for (; b < nb; b += G) a[0] += part[(long long)b * w + ee];
    scratch[g * ne + e] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  }
  __syncthreads();
  for (int i = t; i < ne; i += nt) {
    double v = 0.0;
    for (int gg = 0; gg < G; ++gg) v += scratch[gg * ne + i];
    if (i < neA) outA[i] = v;
    else outB[i - neA] = v;
  }
  __syncthreads();
}

}  // namespace prgd
