// Sketched spectral initialisation T_0 ~ SVD^tt_r(P_Omega(y) / p).
//
// The initialisation the convergence analysis starts from (Theorem 1 assumes
// T_0 close to T*; the spectral choice is Algorithm 1 applied to the
// rescaled sampled tensor Z = P_Omega(y) / p, p = |Omega| / d*).  Algorithm 1
// takes, at split i, the top r_i left singular vectors of the projected
// unfolding A_i = (T^{<=i-1} kron I_{n_i})^T Z^{<i>}; its columns run over
// every later index tuple, far too many to form.  Each A_i is therefore
// replaced by the sketch Y_i = A_i Psi_i, Psi_i having for the later indices
// (x_{i+1}, ..., x_m) the row Gamma_{i,i+1}[x_{i+1}, :] * ... * Gamma_{i,m}[x_m, :]
// (elementwise; independent standard-normal Gamma, so E[Psi Psi^T] is a
// multiple of the identity and Y_i Y_i^T estimates A_i A_i^T).  Only the
// observed entries contribute:
//   Y_i[(a, x), c] = sum_{j: x_i = x} z_j ell_{i-1}(x^(j))[a] psi_i(x^(j))[c],
// with ell the left interface of the cores already built.  The core is the
// top r_i left singular vectors of Y_i, taken from the eigen-decomposition of
// its Gram matrix (U = Y V_r D_r^{-1/2}); the last core is A_m itself.
//
// Work per split: Omega is grouped by x_i (stable radix sort); the samples of
// each value x are cut into a fixed number of chunks whose workgroups
// accumulate partial rows of Y_i in a fixed order, a second kernel adds the
// chunks in order (deterministic) and forms each value's share of the Gram
// matrix, and one workgroup sums the shares, runs the Jacobi eigen-solver and
// writes the core.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "solver.hpp"
#include "small_la.hpp"

namespace prgd {
namespace {

constexpr int SK_MAXR = 16;   // TT ranks
constexpr int SK_MAXS = 32;   // sketch width
constexpr int SK_NT = 512;    // threads of the accumulation kernel (>= SK_MAXR * SK_MAXS)
constexpr int SK_B = 64;      // samples per batch

struct SketchArgs {
  int m, split, s;             // split i (0-based); split == m - 1: the last core (s = 1, psi = 1)
  long long N;
  const int *idx;              // SoA m x N, grouped by mode `split`
  const double *val;           // values in the same order
  double inv_p;                // 1 / p
  double *cores;               // packed cores; 0..split-1 built (left-orthonormal)
  long long coff[MAXM + 1];
  int n[MAXM], r[MAXM + 1];
  long long goff[MAXM];        // offset of Gamma_{split,k} in gam (k > split)
  const double *gam;
  int chunks;                  // workgroups per value of x_split
  double *Ypart;               // [chunks][r_split * n_split][s] partial sketches
  double *Y;                   // rows (a * n_split + x), s columns
  double *gpart;               // n_split blocks of s x s Gram shares (null: last core)
};

// first position in the sorted key column with key >= v
__device__ long long lower_bound_key(const int *key, long long N, int v) {
  long long lo = 0, hi = N;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if (key[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Workgroup (x, ch): chunk ch of the samples with x_split = x, partial rows
// (a, x) of Y_i into Ypart[ch].
__global__ void __launch_bounds__(SK_NT) k_sketch(const SketchArgs A) {
  __shared__ double zl[SK_B][SK_MAXR + 1], ps[SK_B][SK_MAXS + 1];
  __shared__ long long seg[2];
  const int x = blockIdx.x, ch = blockIdx.y, t = threadIdx.x, i = A.split, s = A.s;
  const int rp = A.r[i];
  const long long N = A.N;
  const int *key = A.idx + (long long)i * N;
  if (t == 0) {
    const long long b0 = lower_bound_key(key, N, x), b1 = lower_bound_key(key, N, x + 1);
    seg[0] = b0 + (b1 - b0) * ch / A.chunks;
    seg[1] = b0 + (b1 - b0) * (ch + 1) / A.chunks;
  }
  __syncthreads();
  const long long lo = seg[0], hi = seg[1];
  const int a = t / s, c = t - (t / s) * s;
  const bool act = a < rp;
  double acc = 0.0;
  for (long long base = lo; base < hi; base += SK_B) {
    if (t < SK_B) {
      const long long j = base + t;
      double ell[SK_MAXR], psi[SK_MAXS];
      for (int q = 0; q < SK_MAXR; ++q) ell[q] = q == 0 ? 1.0 : 0.0;
      for (int q = 0; q < SK_MAXS; ++q) psi[q] = 1.0;
      double zj = 0.0;
      if (j < hi) {
        zj = A.val[j] * A.inv_p;
        // ell <- ell^T T_k(x_k) over the cores already built
        for (int k = 0; k < i; ++k) {
          const int xk = A.idx[(long long)k * N + j], ra = A.r[k], rb = A.r[k + 1];
          const double *ck = A.cores + A.coff[k] + (long long)xk * rb;
          double nxt[SK_MAXR];
          for (int b = 0; b < SK_MAXR; ++b) nxt[b] = 0.0;
          for (int q = 0; q < ra; ++q) {
            const double lq = ell[q];
            const double *row = ck + (long long)q * A.n[k] * rb;
            for (int b = 0; b < rb; ++b) nxt[b] = fma(lq, row[b], nxt[b]);
          }
          for (int b = 0; b < SK_MAXR; ++b) ell[b] = nxt[b];
        }
        for (int k = i + 1; k < A.m; ++k) {
          const double *g = A.gam + A.goff[k] + (long long)A.idx[(long long)k * N + j] * s;
          for (int q = 0; q < s; ++q) psi[q] *= g[q];
        }
      }
      for (int q = 0; q < rp; ++q) zl[t][q] = zj * ell[q];
      for (int q = 0; q < s; ++q) ps[t][q] = j < hi ? psi[q] : 0.0;
    }
    __syncthreads();
    if (act)
      for (int b = 0; b < SK_B; ++b) acc = fma(zl[b][a], ps[b][c], acc);
    __syncthreads();
  }
  if (act) A.Ypart[((long long)ch * rp * A.n[i] + (long long)a * A.n[i] + x) * s + c] = acc;
}

// Workgroup x: the rows (a, x) of Y_i as the sum of the chunks in order, and
// (unless this is the last core) this value's share of Y_i^T Y_i.
__global__ void __launch_bounds__(SK_NT) k_sketch_sum(const SketchArgs A) {
  __shared__ double yb[SK_MAXR][SK_MAXS + 1];
  const int x = blockIdx.x, t = threadIdx.x, i = A.split, s = A.s;
  const int rp = A.r[i];
  const int a = t / s, c = t - (t / s) * s;
  if (a < rp) {
    double acc = 0.0;
    for (int ch = 0; ch < A.chunks; ++ch)
      acc += A.Ypart[((long long)ch * rp * A.n[i] + (long long)a * A.n[i] + x) * s + c];
    A.Y[((long long)a * A.n[i] + x) * s + c] = acc;
    yb[a][c] = acc;
  }
  if (A.gpart == nullptr) return;
  __syncthreads();
  for (int e = t; e < s * s; e += SK_NT) {
    const int c1 = e / s, c2 = e - (e / s) * s;
    double g = 0.0;
    for (int q = 0; q < rp; ++q) g = fma(yb[q][c1], yb[q][c2], g);
    A.gpart[(long long)x * s * s + e] = g;
  }
}

// Gram of Y_i (shares summed in order of x), its eigen-decomposition and the
// core U = Y V_r D_r^{-1/2}, written into the packed cores.  *bad is set when
// the sketch has numerical rank below r_{i+1} (singular value ratio 1e-7).
__global__ void __launch_bounds__(1024) k_sketch_core(const SketchArgs A, int *bad) {
  __shared__ double G[1024], V[1024], W1[1024], W2[1024], w[SK_MAXS];
  const int i = A.split, s = A.s, n = A.n[i], rn = A.r[i + 1];
  const long long rows = (long long)A.r[i] * n;
  for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
    double g = 0.0;
    for (int x = 0; x < n; ++x) g += A.gpart[(long long)x * s * s + e];
    G[e] = g;
  }
  __syncthreads();
  block_jacobi_eig(G, s, V, w, W1, W2);
  __shared__ int ok;
  if (threadIdx.x == 0) {
    // numerical rank: the Gram's eigenvalues carry rounding noise near 1e-16
    // of the largest, so rank r needs w[r-1] above 1e-14 of it (singular
    // values above 1e-7 of the largest)
    ok = (w[rn - 1] > 1e-14 * w[0]) && isfinite(w[0]);
    if (!ok) *bad = 1;
  }
  __syncthreads();
  if (!ok) return;
  double *core = A.cores + A.coff[i];
  for (long long e = threadIdx.x; e < rows * rn; e += blockDim.x) {
    const long long row = e / rn;
    const int col = (int)(e - row * rn);
    double u = 0.0;
    for (int c = 0; c < s; ++c) u = fma(A.Y[row * s + c], V[c * s + col], u);
    core[e] = u / sqrt(w[col]);
  }
}

// workgroups per mode value: about 2048 workgroups per split in all, at most 64
int sketch_chunks(int n_mode) { return std::max(1, std::min(64, (2048 + n_mode - 1) / n_mode)); }

// device buffers of one call, freed on every exit after the work queued on
// the call's stream has finished
struct DevBuf {
  hipStream_t st = nullptr;
  std::vector<void *> p;
  ~DevBuf() {
    (void)hipStreamSynchronize(st);
    for (void *q : p) (void)hipFree(q);
  }
  template <typename T>
  hipError_t get(T **out, size_t count) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) {
      p.push_back(q);
      *out = (T *)q;
    }
    return e;
  }
};

}  // namespace
}  // namespace prgd

using namespace prgd;

#define SKCHECK(x)                                                                            \
  do {                                                                                        \
    hipError_t e_ = (x);                                                                      \
    if (e_ != hipSuccess) return set_error(PRGD_EDEVICE, (std::string("HIP: ") + hipGetErrorString(e_) + " in " #x).c_str()); \
  } while (0)

extern "C" prgd_status prgd_spectral_init(int32_t m, const int32_t *n, const int32_t *r, int64_t n_obs,
                                          const int32_t *indices, const double *values, int32_t sketch,
                                          const double *gauss, double *cores_out, void *stream) {
  if (m < 2 || m > MAXM || !n || !r) return set_error(PRGD_EINVAL, "order must be 2..32 with shape and ranks given");
  if (!indices || !values || !gauss || !cores_out || n_obs < 1) return set_error(PRGD_EINVAL, "null argument or empty Omega");
  if (r[0] != 1 || r[m] != 1) return set_error(PRGD_EINVAL, "boundary TT ranks must be 1");
  int rmax = 1;
  double numel_d = 1.0;
  for (int k = 0; k < m; ++k) {
    if (n[k] < 1) return set_error(PRGD_EINVAL, "mode sizes must be positive");
    numel_d *= (double)n[k];
  }
  for (int k = 1; k < m; ++k) {
    if (r[k] < 1 || r[k] > SK_MAXR) return set_error(PRGD_ENOTSUP, "TT ranks must be 1..16");
    rmax = std::max(rmax, (int)r[k]);
  }
  if (sketch < rmax || sketch > SK_MAXS) return set_error(PRGD_EINVAL, "sketch width must be max(r) .. 32");
  for (int k = 0; k < m; ++k)
    for (int64_t j = 0; j < n_obs; ++j)
      if (indices[(int64_t)k * n_obs + j] < 0 || indices[(int64_t)k * n_obs + j] >= n[k])
        return set_error(PRGD_EINVAL, "index out of range");
  for (int64_t j = 0; j < n_obs; ++j)
    if (!std::isfinite(values[j])) return set_error(PRGD_EINVAL, "non-finite value");
  hipStream_t st = (hipStream_t)stream;

  SketchArgs A{};
  A.m = m;
  A.N = n_obs;
  A.inv_p = numel_d / (double)n_obs;
  long long numel = 0, rows_max = 0, nmax = 0, part_max = 0;
  for (int k = 0; k < m; ++k) {
    A.n[k] = n[k];
    A.coff[k] = numel;
    numel += (long long)r[k] * n[k] * r[k + 1];
    rows_max = std::max(rows_max, (long long)r[k] * n[k]);
    nmax = std::max(nmax, (long long)n[k]);
    part_max = std::max(part_max, (long long)sketch_chunks(n[k]) * r[k] * n[k]);
  }
  A.coff[m] = numel;
  for (int k = 0; k <= m; ++k) A.r[k] = r[k];
  long long ngauss = 0;
  for (int i = 0; i < m - 1; ++i)
    for (int k = i + 1; k < m; ++k) ngauss += (long long)n[k] * sketch;

  DevBuf buf;
  buf.st = st;
  int *d_idx = nullptr, *d_sidx = nullptr, *d_bad = nullptr;
  double *d_val = nullptr, *d_sval = nullptr, *d_cores = nullptr, *d_gam = nullptr, *d_Y = nullptr, *d_gp = nullptr;
  SKCHECK(buf.get(&d_idx, (size_t)m * n_obs));
  SKCHECK(buf.get(&d_sidx, (size_t)m * n_obs));
  SKCHECK(buf.get(&d_val, (size_t)n_obs));
  SKCHECK(buf.get(&d_sval, (size_t)n_obs));
  SKCHECK(buf.get(&d_cores, (size_t)numel));
  SKCHECK(buf.get(&d_gam, (size_t)ngauss));
  double *d_Yp = nullptr;
  SKCHECK(buf.get(&d_Y, (size_t)(rows_max * sketch)));
  SKCHECK(buf.get(&d_Yp, (size_t)(part_max * sketch)));
  SKCHECK(buf.get(&d_gp, (size_t)(nmax * sketch * sketch)));
  SKCHECK(buf.get(&d_bad, 1));
  SKCHECK(hipMemcpyAsync(d_idx, indices, (size_t)m * n_obs * sizeof(int), hipMemcpyHostToDevice, st));
  SKCHECK(hipMemcpyAsync(d_val, values, (size_t)n_obs * sizeof(double), hipMemcpyHostToDevice, st));
  SKCHECK(hipMemcpyAsync(d_gam, gauss, (size_t)ngauss * sizeof(double), hipMemcpyHostToDevice, st));
  SKCHECK(hipMemsetAsync(d_bad, 0, sizeof(int), st));
  A.cores = d_cores;
  A.gam = d_gam;
  A.Y = d_Y;
  A.idx = d_sidx;
  A.val = d_sval;
  long long g = 0;
  for (int i = 0; i < m; ++i) {
    SKCHECK(group_by_mode(m, n_obs, i, n[i], d_idx, d_val, 1, d_sidx, d_sval, nullptr, st));
    A.split = i;
    const bool last = i == m - 1;
    A.s = last ? 1 : sketch;
    for (int k = 0; k < MAXM; ++k) A.goff[k] = 0;
    if (!last)
      for (int k = i + 1; k < m; ++k) {
        A.goff[k] = g;
        g += (long long)n[k] * sketch;
      }
    A.Y = last ? d_cores + A.coff[m - 1] : d_Y;
    A.gpart = last ? nullptr : d_gp;
    A.chunks = sketch_chunks(n[i]);
    A.Ypart = d_Yp;
    hipLaunchKernelGGL(k_sketch, dim3(n[i], A.chunks), dim3(SK_NT), 0, st, A);
    SKCHECK(hipGetLastError());
    hipLaunchKernelGGL(k_sketch_sum, dim3(n[i]), dim3(SK_NT), 0, st, A);
    SKCHECK(hipGetLastError());
    if (!last) {
      hipLaunchKernelGGL(k_sketch_core, dim3(1), dim3(1024), 0, st, A, d_bad);
      SKCHECK(hipGetLastError());
    }
  }
  int bad = 0;
  SKCHECK(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, st));
  SKCHECK(hipMemcpyAsync(cores_out, d_cores, (size_t)numel * sizeof(double), hipMemcpyDeviceToHost, st));
  SKCHECK(hipStreamSynchronize(st));
  if (bad) return set_error(PRGD_EBREAKDOWN, "sketch rank below the target TT rank (too few samples for the ranks)");
  return PRGD_OK;
}
