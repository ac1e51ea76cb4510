// One-time preparation of the observation set on the device: group Omega by
// one mode with a stable radix sort (rocPRIM), gather the index rows and the
// values into that order, and small fill/convert kernels.
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "prgd_internal.hpp"

namespace prgd {

__global__ void k_iota(int *p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = (int)i;
}

__global__ void k_gather_idx(int m, long long N, const int *__restrict__ src, const int *__restrict__ perm,
                             int *__restrict__ dst) {
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += (long long)gridDim.x * blockDim.x) {
    const long long p = perm[j];
    for (int k = 0; k < m; ++k) dst[(long long)k * N + j] = src[(long long)k * N + p];
  }
}

template <typename Tin, typename Tout>
__global__ void k_gather_val(long long N, const Tin *__restrict__ src, const int *__restrict__ perm,
                             Tout *__restrict__ dst) {
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += (long long)gridDim.x * blockDim.x)
    dst[j] = (Tout)src[perm[j]];
}

__global__ void k_fill_f64(double *p, long long n, double v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_f32(float *p, long long n, float v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_convert_f64_f32(const double *src, float *dst, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

static int grid_for(long long n) {
  long long g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t fill_f64(double *p, long long n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t fill_f32(float *p, long long n, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t convert_f64_f32(const double *src, float *dst, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_convert_f64_f32, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

// Group Omega by mode `mode`: stable sort of the samples by their mode index.
// idx_in: [m][N] device, values_in: [N] device (float or double).
// Outputs idx_out [m][N], y64/y32 (whichever is non-null) in sorted order.
hipError_t group_by_mode(int m, long long N, int mode, int n_mode, const int *idx_in, const void *values_in,
                         int values_fp64, int *idx_out, double *y64, float *y32, hipStream_t s, int *perm) {
  hipError_t e;
  int *keys_out = nullptr, *perm_in = nullptr, *perm_out = nullptr;
  void *temp = nullptr;
  size_t temp_bytes = 0;
  // scratch freed on every exit, after the work queued on s has finished
  struct Scratch {
    hipStream_t s;
    void **p[4];
    ~Scratch() {
      (void)hipStreamSynchronize(s);
      for (void **q : p)
        if (*q) (void)hipFree(*q);
    }
  } scratch{s, {(void **)&keys_out, (void **)&perm_in, (void **)&perm_out, &temp}};
  unsigned end_bit = 1;
  while (end_bit < 31 && (1u << end_bit) < (unsigned)n_mode) ++end_bit;
  if ((e = hipMalloc((void **)&keys_out, N * sizeof(int))) != hipSuccess) return e;
  if ((e = hipMalloc((void **)&perm_in, N * sizeof(int))) != hipSuccess) return e;
  if ((e = hipMalloc((void **)&perm_out, N * sizeof(int))) != hipSuccess) return e;
  hipLaunchKernelGGL(k_iota, dim3(grid_for(N)), dim3(256), 0, s, perm_in, N);
  const int *keys_in = idx_in + (long long)mode * N;
  e = rocprim::radix_sort_pairs(nullptr, temp_bytes, keys_in, keys_out, perm_in, perm_out, (size_t)N, 0, end_bit, s);
  if (e != hipSuccess) return e;
  if ((e = hipMalloc(&temp, temp_bytes ? temp_bytes : 16)) != hipSuccess) return e;
  e = rocprim::radix_sort_pairs(temp, temp_bytes, keys_in, keys_out, perm_in, perm_out, (size_t)N, 0, end_bit, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gather_idx, dim3(grid_for(N)), dim3(256), 0, s, m, N, idx_in, perm_out, idx_out);
  if (values_fp64) {
    if (y64) hipLaunchKernelGGL((k_gather_val<double, double>), dim3(grid_for(N)), dim3(256), 0, s, N,
                                (const double *)values_in, perm_out, y64);
    if (y32) hipLaunchKernelGGL((k_gather_val<double, float>), dim3(grid_for(N)), dim3(256), 0, s, N,
                                (const double *)values_in, perm_out, y32);
  } else {
    if (y64) hipLaunchKernelGGL((k_gather_val<float, double>), dim3(grid_for(N)), dim3(256), 0, s, N,
                                (const float *)values_in, perm_out, y64);
    if (y32) hipLaunchKernelGGL((k_gather_val<float, float>), dim3(grid_for(N)), dim3(256), 0, s, N,
                                (const float *)values_in, perm_out, y32);
  }
  if (perm && (e = hipMemcpyAsync(perm, perm_out, N * sizeof(int), hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

// mixed-radix key of the first u mode indices (mode 1 most significant)
__global__ void k_prefix_key(int u, long long N, const int *__restrict__ idx, const int *__restrict__ n,
                             unsigned *__restrict__ key) {
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += (long long)gridDim.x * blockDim.x) {
    unsigned v = 0;
    for (int k = 0; k < u; ++k) v = v * (unsigned)n[k] + (unsigned)idx[(long long)k * N + j];
    key[j] = v;
  }
}

hipError_t group_by_prefix(int m, long long N, int u, const int *n, const int *idx_in, const void *values_in,
                           int values_fp64, int *idx_out, double *y64, float *y32, hipStream_t s) {
  hipError_t e;
  unsigned *keys_in = nullptr, *keys_out = nullptr;
  int *perm_in = nullptr, *perm_out = nullptr, *nd = nullptr;
  void *temp = nullptr;
  size_t temp_bytes = 0;
  struct Scratch {
    hipStream_t s;
    void **p[6];
    ~Scratch() {
      (void)hipStreamSynchronize(s);
      for (void **q : p)
        if (*q) (void)hipFree(*q);
    }
  } scratch{s, {(void **)&keys_in, (void **)&keys_out, (void **)&perm_in, (void **)&perm_out, (void **)&nd, &temp}};
  unsigned long long span = 1;
  for (int k = 0; k < u; ++k) span *= (unsigned long long)n[k];
  unsigned end_bit = 0;
  while (end_bit < 32 && (1ull << end_bit) < span) ++end_bit;
  if ((e = hipMalloc((void **)&perm_out, N * sizeof(int))) != hipSuccess) return e;
  if (end_bit == 0) {
    hipLaunchKernelGGL(k_iota, dim3(grid_for(N)), dim3(256), 0, s, perm_out, N);
  } else {
    if ((e = hipMalloc((void **)&keys_in, N * sizeof(unsigned))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&keys_out, N * sizeof(unsigned))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&perm_in, N * sizeof(int))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&nd, (size_t)(u > 0 ? u : 1) * sizeof(int))) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(nd, n, (size_t)u * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_prefix_key, dim3(grid_for(N)), dim3(256), 0, s, u, N, idx_in, (const int *)nd, keys_in);
    hipLaunchKernelGGL(k_iota, dim3(grid_for(N)), dim3(256), 0, s, perm_in, N);
    e = rocprim::radix_sort_pairs(nullptr, temp_bytes, keys_in, keys_out, perm_in, perm_out, (size_t)N, 0, end_bit, s);
    if (e != hipSuccess) return e;
    if ((e = hipMalloc(&temp, temp_bytes ? temp_bytes : 16)) != hipSuccess) return e;
    e = rocprim::radix_sort_pairs(temp, temp_bytes, keys_in, keys_out, perm_in, perm_out, (size_t)N, 0, end_bit, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_gather_idx, dim3(grid_for(N)), dim3(256), 0, s, m, N, idx_in, perm_out, idx_out);
  if (values_fp64) {
    if (y64) hipLaunchKernelGGL((k_gather_val<double, double>), dim3(grid_for(N)), dim3(256), 0, s, N,
                                (const double *)values_in, perm_out, y64);
    if (y32) hipLaunchKernelGGL((k_gather_val<double, float>), dim3(grid_for(N)), dim3(256), 0, s, N,
                                (const double *)values_in, perm_out, y32);
  } else {
    if (y64) hipLaunchKernelGGL((k_gather_val<float, double>), dim3(grid_for(N)), dim3(256), 0, s, N,
                                (const float *)values_in, perm_out, y64);
    if (y32) hipLaunchKernelGGL((k_gather_val<float, float>), dim3(grid_for(N)), dim3(256), 0, s, N,
                                (const float *)values_in, perm_out, y32);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

__global__ void k_invert_perm(long long N, const int *__restrict__ perm, int *__restrict__ pos) {
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (long long)gridDim.x * blockDim.x)
    pos[perm[p]] = (int)p;
}

__global__ void k_compose_pos(long long N, const int *__restrict__ perm0, const int *__restrict__ pos,
                              int *__restrict__ out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x)
    out[i] = pos[perm0[i]];
}

hipError_t compose_positions(long long N, const int *perm_a, const int *perm_b, int *scratch, int *out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_invert_perm, dim3(grid_for(N)), dim3(256), 0, s, N, perm_b, scratch);
  hipLaunchKernelGGL(k_compose_pos, dim3(grid_for(N)), dim3(256), 0, s, N, perm_a, scratch, out);
  return hipGetLastError();
}

// copy each batch member's State to out[i] (thread i)
__global__ void k_gather_state(const Dev *__restrict__ dt, int ns, State *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ns) out[i] = *dt[i].st;
}

hipError_t launch_gather_state(const Batch &bt, State *out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_state, dim3((bt.ns + 63) / 64), dim3(64), 0, s, bt.dt, bt.ns, out);
  return hipGetLastError();
}

}  // namespace prgd
