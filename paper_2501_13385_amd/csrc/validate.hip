// Checks and summaries of an observation set that is already in device
// memory, so that a solve created from device buffers reads none of Omega
// back to the host: every index within its mode size, every value finite, no
// multi-index twice, the sum of squares of the values, and the sample counts
// per slice (or per index prefix) that the host needs for its chunk tables.
#include <cstring>
#include <string>
#include <vector>

#include <rocprim/rocprim.hpp>

#include "prgd_internal.hpp"
#include "solver.hpp"

namespace prgd {

namespace {

struct ObsShape {
  int m;
  long long N;
  int n[MAXM];
};

constexpr int VT = 256;   // threads per block of the check kernels
constexpr int VG = 1024;  // blocks of the check kernel (fixed: its partial sums add in block order)

// the first offending sample: index check as sample * 64 + mode (the
// smallest wins), non-finite value as the sample; per-block partial sums of
// y^2, each block's in a fixed order
template <typename V>
__global__ void __launch_bounds__(VT) k_check_obs(ObsShape sh, const int *__restrict__ idx, const V *__restrict__ val,
                                                  unsigned long long *__restrict__ bad, double *__restrict__ ysq_part) {
  __shared__ double red[VT];
  double acc = 0.0;
  for (long long j = (long long)blockIdx.x * VT + threadIdx.x; j < sh.N; j += (long long)gridDim.x * VT) {
    for (int k = 0; k < sh.m; ++k) {
      const int x = idx[(long long)k * sh.N + j];
      if (x < 0 || x >= sh.n[k]) atomicMin(&bad[0], (unsigned long long)j * 64 + (unsigned long long)k);
    }
    const double v = (double)val[j];
    if (!isfinite(v)) atomicMin(&bad[1], (unsigned long long)j);
    acc = fma(v, v, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = VT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) ysq_part[blockIdx.x] = red[0];
}

// linear index of every sample (modulo 2^64) and its number, for the sort
__global__ void __launch_bounds__(VT) k_linear_key(ObsShape sh, const int *__restrict__ idx,
                                                   unsigned long long *__restrict__ key, int *__restrict__ id) {
  for (long long j = (long long)blockIdx.x * VT + threadIdx.x; j < sh.N; j += (long long)gridDim.x * VT) {
    unsigned long long v = 0;
    for (int k = 0; k < sh.m; ++k) v = v * (unsigned long long)sh.n[k] + (unsigned long long)idx[(long long)k * sh.N + j];
    key[j] = v;
    id[j] = (int)j;
  }
}

// equal neighbours in key order: with an exact key that is a repeated
// multi-index; otherwise the run of equal keys before j is compared index by
// index (equal keys of distinct multi-indices are possible when the linear
// index wraps).  Records the smallest sample number of a repeated pair.
__global__ void __launch_bounds__(VT) k_adjacent(ObsShape sh, const int *__restrict__ idx,
                                                 const unsigned long long *__restrict__ key, const int *__restrict__ id,
                                                 int exact, unsigned long long *__restrict__ bad) {
  for (long long j = (long long)blockIdx.x * VT + threadIdx.x + 1; j < sh.N; j += (long long)gridDim.x * VT) {
    if (key[j] != key[j - 1]) continue;
    const int b = id[j];
    for (long long i = j - 1; i >= 0 && key[i] == key[j]; --i) {
      const int a = id[i];
      bool same = true;
      if (!exact)
        for (int k = 0; k < sh.m && same; ++k) same = idx[(long long)k * sh.N + a] == idx[(long long)k * sh.N + b];
      if (same) {
        atomicMin(&bad[2], (unsigned long long)(a < b ? a : b));
        break;
      }
    }
  }
}

// samples per value of one mode's index, or of the mixed-radix key of the
// first u mode indices (integer adds: the counts do not depend on order)
__global__ void __launch_bounds__(VT) k_count(ObsShape sh, const int *__restrict__ idx, int mode, int u,
                                              unsigned *__restrict__ cnt) {
  for (long long j = (long long)blockIdx.x * VT + threadIdx.x; j < sh.N; j += (long long)gridDim.x * VT) {
    unsigned v;
    if (mode >= 0) {
      v = (unsigned)idx[(long long)mode * sh.N + j];
    } else {
      v = 0;
      for (int k = 0; k < u; ++k) v = v * (unsigned)sh.n[k] + (unsigned)idx[(long long)k * sh.N + j];
    }
    atomicAdd(&cnt[v], 1u);
  }
}

ObsShape shape_of(int m, long long N, const int *n) {
  ObsShape sh{};
  sh.m = m;
  sh.N = N;
  for (int k = 0; k < m; ++k) sh.n[k] = n[k];
  return sh;
}

int grid(long long n) { return (int)std::max<long long>(1, std::min<long long>(8192, (n + VT - 1) / VT)); }

// device buffers released on every exit, after the queued work has finished
struct Scratch {
  hipStream_t s;
  std::vector<void *> p;
  ~Scratch() {
    (void)hipStreamSynchronize(s);
    for (void *q : p)
      if (q) (void)hipFree(q);
  }
  template <typename T>
  hipError_t get(T **out, size_t count) {
    void *q = nullptr;
    const hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) p.push_back(q);
    *out = (T *)q;
    return e;
  }
};

}  // namespace

prgd_status check_obs_device(int m, long long N, const int *n, const int *idx, const void *val, int values_fp64,
                             double &ysq, hipStream_t s) {
  const ObsShape sh = shape_of(m, N, n);
  Scratch sc{s, {}};
  unsigned long long *bad = nullptr;
  double *part = nullptr;
  if (sc.get(&bad, 3) != hipSuccess || sc.get(&part, VG) != hipSuccess)
    return set_error(PRGD_ENOMEM, "device allocation failed");
  const unsigned long long none[3] = {~0ull, ~0ull, ~0ull};
  if (hipMemcpyAsync(bad, none, sizeof(none), hipMemcpyHostToDevice, s) != hipSuccess)
    return set_error(PRGD_EDEVICE, "upload failed");
  if (values_fp64)
    hipLaunchKernelGGL((k_check_obs<double>), dim3(VG), dim3(VT), 0, s, sh, idx, (const double *)val, bad, part);
  else
    hipLaunchKernelGGL((k_check_obs<float>), dim3(VG), dim3(VT), 0, s, sh, idx, (const float *)val, bad, part);
  // repeated multi-indices: sort the linear keys, compare neighbours
  double dstar = 1;
  for (int k = 0; k < m; ++k) dstar *= n[k];
  const bool exact = dstar < 9.0e18;
  unsigned end_bit = 64;
  if (exact) {
    end_bit = 1;
    while (end_bit < 64 && (double)(1ull << end_bit) < dstar) ++end_bit;
  }
  unsigned long long *kin = nullptr, *kout = nullptr;
  int *iin = nullptr, *iout = nullptr;
  void *temp = nullptr;
  size_t temp_bytes = 0;
  if (sc.get(&kin, N) != hipSuccess || sc.get(&kout, N) != hipSuccess || sc.get(&iin, N) != hipSuccess ||
      sc.get(&iout, N) != hipSuccess)
    return set_error(PRGD_ENOMEM, "device allocation failed");
  hipLaunchKernelGGL(k_linear_key, dim3(grid(N)), dim3(VT), 0, s, sh, idx, kin, iin);
  if (rocprim::radix_sort_pairs(nullptr, temp_bytes, kin, kout, iin, iout, (size_t)N, 0, end_bit, s) != hipSuccess ||
      sc.get((unsigned char **)&temp, temp_bytes) != hipSuccess ||
      rocprim::radix_sort_pairs(temp, temp_bytes, kin, kout, iin, iout, (size_t)N, 0, end_bit, s) != hipSuccess)
    return set_error(PRGD_EDEVICE, "sort of the multi-index keys failed");
  hipLaunchKernelGGL(k_adjacent, dim3(grid(N)), dim3(VT), 0, s, sh, idx, kout, iout, exact ? 1 : 0, bad);
  if (hipGetLastError() != hipSuccess) return set_error(PRGD_EDEVICE, "launch of the observation checks failed");
  unsigned long long hb[3];
  std::vector<double> hp(VG);
  if (hipMemcpyAsync(hb, bad, sizeof(hb), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(hp.data(), part, VG * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(PRGD_EDEVICE, "read-back of the observation checks failed");
  if (hb[0] != ~0ull)
    return set_error(PRGD_EINVAL, ("index out of range in mode " + std::to_string(hb[0] % 64) + " at sample " +
                                   std::to_string(hb[0] / 64)).c_str());
  if (hb[1] != ~0ull)
    return set_error(PRGD_EINVAL, ("non-finite observed value at sample " + std::to_string(hb[1])).c_str());
  if (hb[2] != ~0ull) return set_error(PRGD_EDUPLICATE, "Omega contains a repeated multi-index");
  ysq = 0.0;
  for (int b = 0; b < VG; ++b) ysq += hp[b];
  return PRGD_OK;
}

hipError_t count_obs_device(int m, long long N, const int *n, const int *idx, int mode, int u, long long bins,
                            std::vector<long long> &seg, hipStream_t s) {
  const ObsShape sh = shape_of(m, N, n);
  Scratch sc{s, {}};
  unsigned *cnt = nullptr;
  hipError_t e;
  if ((e = sc.get(&cnt, (size_t)bins)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(cnt, 0, (size_t)bins * sizeof(unsigned), s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_count, dim3(grid(N)), dim3(VT), 0, s, sh, idx, mode, u, cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  std::vector<unsigned> h((size_t)bins);
  if ((e = hipMemcpyAsync(h.data(), cnt, (size_t)bins * sizeof(unsigned), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return e;
  seg.assign((size_t)bins + 1, 0);
  for (long long v = 0; v < bins; ++v) seg[v + 1] = seg[v] + h[v];
  return hipSuccess;
}

}  // namespace prgd
