// prgd_eval_noalloc: TT evaluation at device-resident multi-indices that
// allocates no memory, for callers that cannot allocate (code under HIP graph
// capture, tight serving loops).  prgd_eval stages the padded cores in a
// device buffer it allocates; here that staging lives in a fixed file-scope
// device array, one per GPU, whose address is looked up once per device.
#include <mutex>

#include "../../include/prgd.h"
#include "prgd_internal.hpp"
#include "solver.hpp"

namespace prgd {

// Workspace: the core offsets (MAXM + 1 int64) in the first 64 doubles, then
// the padded cores.  4 MiB in total, held by every GPU the library runs on.
constexpr long long NOALLOC_HEADER = 64;
constexpr long long NOALLOC_DOUBLES = 1LL << 19;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

struct EvalShape {
  int m, R;
  int n[MAXM];
  int r[MAXM + 1];
  long long off[MAXM + 1];     // packed offsets of the caller's cores
  long long coff[MAXM + 1];    // padded offsets in the workspace
};

// packed (a, x, b) row-major cores -> padded slice-major [n_k][R][R] (zero
// outside the ranks), and the offsets, into the workspace
__global__ void k_pad_cores(EvalShape sh, const double *__restrict__ src, double *__restrict__ ws) {
  const long long total = sh.coff[sh.m];
  const int RR = sh.R * sh.R;
  double *dst = ws + NOALLOC_HEADER;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    int k = 0;
    while (k + 1 < sh.m && sh.coff[k + 1] <= i) ++k;
    const long long rel = i - sh.coff[k];
    const int x = (int)(rel / RR), e = (int)(rel % RR), a = e / sh.R, b = e % sh.R;
    double v = 0.0;
    if (a < sh.r[k] && b < sh.r[k + 1]) v = src[sh.off[k] + ((long long)a * sh.n[k] + x) * sh.r[k + 1] + b];
    dst[i] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x <= (unsigned)sh.m) {
    long long *hdr = reinterpret_cast<long long *>(ws);
    hdr[threadIdx.x] = sh.coff[threadIdx.x];
  }
}

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_ws_mu;
double *g_ws[NOALLOC_MAX_DEVICES] = {};
prgd_status na_fail(prgd_status st, const char *msg) { return set_error(st, msg); }

// the workspace of the current device (its address looked up on first use)
prgd_status workspace(double **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return na_fail(PRGD_EDEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return na_fail(PRGD_ENOTSUP, "device index beyond the workspace table");
  std::lock_guard<std::mutex> lock(g_ws_mu);
  if (!g_ws[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
      return na_fail(PRGD_EDEVICE, "hipGetSymbolAddress of the workspace failed");
    g_ws[dev] = (double *)p;
  }
  *out = g_ws[dev];
  return PRGD_OK;
}
}  // namespace

}  // namespace prgd

extern "C" prgd_status prgd_eval_noalloc(int32_t m, const int32_t *n, const int32_t *r, const double *cores_dev,
                                         int64_t n_obs, const int32_t *indices_dev, double *out_dev,
                                         void *stream) {
  using namespace prgd;
  if (m < 2 || m > MAXM || !n || !r) return na_fail(PRGD_EINVAL, "order must be in [2, 32] with shape and ranks");
  if (!cores_dev || !indices_dev || !out_dev || n_obs < 0) return na_fail(PRGD_EINVAL, "null argument or n_obs < 0");
  if (r[0] != 1 || r[m] != 1) return na_fail(PRGD_EINVAL, "r_0 and r_m must be 1");
  EvalShape sh{};
  sh.m = m;
  int rmax = 1;
  for (int k = 0; k <= m; ++k) {
    if (r[k] < 1) return na_fail(PRGD_EINVAL, "ranks must be >= 1");
    rmax = rmax > r[k] ? rmax : r[k];
    sh.r[k] = r[k];
  }
  static const int buckets[] = {2, 4, 6, 8, 10, 12, 16};
  sh.R = -1;
  for (int b : buckets)
    if (rmax <= b && sh.R < 0) sh.R = b;
  if (sh.R < 0) return na_fail(PRGD_ENOTSUP, "TT ranks above 16 are not supported by this build");
  long long off = 0, coff = 0;
  for (int k = 0; k < m; ++k) {
    if (n[k] < 1) return na_fail(PRGD_EINVAL, "mode sizes must be >= 1");
    sh.n[k] = n[k];
    sh.off[k] = off;
    sh.coff[k] = coff;
    off += (long long)r[k] * n[k] * r[k + 1];
    coff += (long long)n[k] * sh.R * sh.R;
    if (coff > NOALLOC_DOUBLES - NOALLOC_HEADER)
      return na_fail(PRGD_ENOMEM, "padded cores exceed the fixed workspace (524224 doubles)");
  }
  sh.off[m] = off;
  sh.coff[m] = coff;
  if (n_obs == 0) return PRGD_OK;
  double *ws = nullptr;
  prgd_status st = workspace(&ws);
  if (st != PRGD_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const long long g = (coff + 255) / 256;
  hipLaunchKernelGGL(k_pad_cores, dim3((unsigned)(g < 1024 ? g : 1024)), dim3(256), 0, s, sh, cores_dev, ws);
  if (hipGetLastError() != hipSuccess) return na_fail(PRGD_EDEVICE, "launch of the core staging kernel failed");
  const hipError_t e = launch_eval(m, sh.R, n_obs, indices_dev, ws + NOALLOC_HEADER, (const long long *)ws, out_dev, s);
  if (e != hipSuccess) return na_fail(PRGD_EDEVICE, "launch of the evaluation kernel failed");
  return PRGD_OK;
}
