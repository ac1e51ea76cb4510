// Block- and wave-level helpers for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>

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

// "Last block" pattern: every block publishes its partial results, then
// increments a counter; the block that brings the counter to gridDim.x sees
// all partials (release/acquire fences at device scope) and finishes the
// reduction.  The last block resets the counter for the next launch.
__device__ inline bool arrive_last(unsigned *counter) {
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = atomicAdd(counter, 1u);
    last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (last) {
    __threadfence();
    if (threadIdx.x == 0) atomicExch(counter, 0u);
  }
  return last != 0;
}

}  // namespace prgd
