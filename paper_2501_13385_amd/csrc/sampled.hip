// Sampled-entry pass: for every observed multi-index x^(j) evaluate the
// current TT iterate as a chain of core-slice products (section 2.1, TT
// format), form the residual R_j = T_l(x^(j)) - y_j (G_l = P_Omega(T_l - T*),
// Algorithm 2), accumulate the squared mode-slice norms
// s_k(x) = sum_{j: x_k = x} R_j^2 (diagonal of M_k(G_l) M_k(G_l)^T, section
// 3.2.1) and scatter the residual into the Euclidean core gradient
// Y_k(:, x_k, :) += R_j * l_{k-1}(x)^T rho_{k+1}(x)^T, where l and rho are the
// left and right interface vectors T^{<=k-1}(x_{<k}) and T^{>=k+1}(x_{>k}).
//
// The weights and the gauge of the preconditioned projection act per mode
// slice, so this one pass with the unscaled cores carries all the sampled
// information the projection of Lemma 3 needs (see dense.hip).
#include "prgd_internal.hpp"
#include "block_ops.hpp"
#include "sampled_common.hpp"

namespace prgd {

template <typename F>
__device__ inline void atomic_add(F *p, F v) {
  atomicAdd(p, v);
}

// Per-mode gradient width in the private area: row 0 of the first core, column
// 0 of the last core, the whole R x R slice of a middle core.
__host__ __device__ inline int priv_width(int k, int m, int R) { return (k == 0 || k == m - 1) ? R : R * R; }

// Gradient entry i (compact index within the mode's width) of slice x of
// core k: into the workgroup's LDS area when the mode is privatised, else a
// global atomic into the padded gradient.
template <typename F>
__device__ inline void scatter(const Dev &d, F *lp, F *Yg, int k, int x, int i, long long gofs, F v) {
  const int po = d.priv_off[k];
  if (po >= 0) atomicAdd(&lp[po + x * priv_width(k, d.m, d.R) + i], v);
  else atomic_add(&Yg[gofs], v);
}
template <typename F>
__device__ inline void scatter_s(const Dev &d, F *lp, F *sacc, int k, int x, F v) {
  const int po = d.priv_off[k];
  if (po >= 0) atomicAdd(&lp[po + d.n[k] * priv_width(k, d.m, d.R) + x], v);
  else atomic_add(&sacc[d.soff[k] + x], v);
}

// One thread per sample, each workgroup a contiguous chunk of Omega (grouped
// by the sort mode).  The right interface vectors rho_k (k = m..2) are
// computed first and kept in LDS (thread-interleaved, conflict-free); the
// left vector is then carried left to right while scattering.
template <typename F, int R>
__global__ void __launch_bounds__(256) k_sampled(const Dev *__restrict__ dt, int diag) {
  const Dev &d = dt[blockIdx.y];
  const int nbs = d.nb_sampled;
  if ((int)blockIdx.x >= nbs || (!diag && d.st->done)) return;
  extern __shared__ unsigned char lds_raw[];
  F *stack = reinterpret_cast<F *>(lds_raw);
  const F *cores = (d.prec == PREC_MIXED) ? (const F *)d.cores32 : (const F *)d.cores;
  const F *y = (d.prec == PREC_MIXED) ? (const F *)d.y32 : (const F *)d.y64;
  F *Yg = (F *)d.Y;
  F *sacc = (F *)d.s;
  const int m = d.m;
  const long long N = d.N;
  const int B = blockDim.x, t = threadIdx.x;
  constexpr int RR = R * R;
  F *lp = stack + (long long)(m - 1) * R * B;     // private accumulators
  for (int i = t; i < d.priv_len; i += B) lp[i] = (F)0;
  __syncthreads();
  const long long chunk = (N + nbs - 1) / nbs;
  const long long jlo = (long long)blockIdx.x * chunk, jhi = min(N, jlo + chunk);
  double rsq = 0.0;
  for (long long j = jlo + t; j < jhi; j += B) {
    F rho[R];
    {
      const int x = d.idx[(long long)(m - 1) * N + j];
      const F *sl = cores + d.coff[m - 1] + (long long)x * RR;
#pragma unroll
      for (int a = 0; a < R; ++a) rho[a] = sl[a * R];
    }
#pragma unroll
    for (int a = 0; a < R; ++a) stack[((m - 2) * R + a) * B + t] = rho[a];
    for (int k = m - 2; k >= 1; --k) {
      const int x = d.idx[(long long)k * N + j];
      const F *sl = cores + d.coff[k] + (long long)x * RR;
      F nr[R];
#pragma unroll
      for (int a = 0; a < R; ++a) {
        F acc = (F)0;
#pragma unroll
        for (int b = 0; b < R; ++b) acc = fma(sl[a * R + b], rho[b], acc);
        nr[a] = acc;
      }
#pragma unroll
      for (int a = 0; a < R; ++a) {
        rho[a] = nr[a];
        stack[((k - 1) * R + a) * B + t] = nr[a];
      }
    }
    // rho now holds T^{>=2}(x_{>=2}); the entry is T_1(0, x_1, :) rho
    const int x0 = d.idx[j];
    const F *sl0 = cores + d.coff[0] + (long long)x0 * RR;
    F l[R];
    F tv = (F)0;
#pragma unroll
    for (int b = 0; b < R; ++b) {
      l[b] = sl0[b];
      tv = fma(l[b], rho[b], tv);
    }
    const F res = tv - y[j];
    const F r2 = res * res;
    rsq += (double)r2;
    {
      const long long g0 = d.coff[0] + (long long)x0 * RR;
#pragma unroll
      for (int b = 0; b < R; ++b) scatter(d, lp, Yg, 0, x0, b, g0 + b, res * rho[b]);
      scatter_s(d, lp, sacc, 0, x0, r2);
    }
    for (int k = 1; k <= m - 2; ++k) {
      const int x = d.idx[(long long)k * N + j];
      const F *sl = cores + d.coff[k] + (long long)x * RR;
      const long long gk = d.coff[k] + (long long)x * RR;
      F rr[R];
#pragma unroll
      for (int b = 0; b < R; ++b) rr[b] = stack[(k * R + b) * B + t];
#pragma unroll
      for (int a = 0; a < R; ++a) {
        const F ra = res * l[a];
#pragma unroll
        for (int b = 0; b < R; ++b) scatter(d, lp, Yg, k, x, a * R + b, gk + a * R + b, ra * rr[b]);
      }
      F nl[R];
#pragma unroll
      for (int b = 0; b < R; ++b) {
        F acc = (F)0;
#pragma unroll
        for (int a = 0; a < R; ++a) acc = fma(l[a], sl[a * R + b], acc);
        nl[b] = acc;
      }
#pragma unroll
      for (int b = 0; b < R; ++b) l[b] = nl[b];
      scatter_s(d, lp, sacc, k, x, r2);
    }
    {
      const int x = d.idx[(long long)(m - 1) * N + j];
      const long long gl = d.coff[m - 1] + (long long)x * RR;
#pragma unroll
      for (int a = 0; a < R; ++a) scatter(d, lp, Yg, m - 1, x, a, gl + a * R, res * l[a]);
      scatter_s(d, lp, sacc, m - 1, x, r2);
    }
  }
  __shared__ double sbuf[16];
  const double bs = block_sum(rsq, sbuf);     // ends with a barrier: lp is complete
  if (threadIdx.x == 0) d.part[blockIdx.x] = bs;
  F *pp = (F *)d.part_priv + (long long)blockIdx.x * d.priv_len;
  for (int i = t; i < d.priv_len; i += B) pp[i] = lp[i];
}

// Sum the workgroups' private accumulators in a fixed order into the padded
// gradient and the slice sums (one output per thread).
template <typename F, int R>
__global__ void __launch_bounds__(256) k_sampled_priv_reduce(const Dev *__restrict__ dt, int diag) {
  const Dev &d = dt[blockIdx.y];
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= d.priv_len || (!diag && d.st->done)) return;
  const int m = d.m, nbs = d.nb_sampled;
  constexpr int RR = R * R;
  const F *pp = (const F *)d.part_priv;
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int b = 0;
  for (; b + 8 <= nbs; b += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += (double)pp[(long long)(b + u) * d.priv_len + o];
  }
  for (; b < nbs; ++b) a[0] += (double)pp[(long long)b * d.priv_len + o];
  const double v = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  int k = -1;      // the privatised mode whose area holds o (largest offset <= o)
  for (int kk = 0; kk < m; ++kk) {
    const int po = d.priv_off[kk];
    if (po >= 0 && po <= o && (k < 0 || po > d.priv_off[k])) k = kk;
  }
  const int W = priv_width(k, m, R), rel = o - d.priv_off[k];
  if (rel < d.n[k] * W) {
    const int x = rel / W, i = rel % W;
    long long g = d.coff[k] + (long long)x * RR;
    g += (k == m - 1 && k != 0) ? (long long)i * R : (long long)i;
    ((F *)d.Y)[g] = (F)v;
  } else {
    ((F *)d.s)[d.soff[k] + rel - d.n[k] * W] = (F)v;
  }
}

// finish of the sampled pass (one block): total ||R||^2 from the per-block
// partials, then the weights and the residual stopping test
template <typename F>
__global__ void __launch_bounds__(1024) k_sampled_fin(const Dev *__restrict__ dt, int diag) {
  const Dev &d = dt[blockIdx.y];
  if (!diag && d.st->done) return;
  const double *rsq_part = d.use3 ? d.q3.part_rsq : (d.use_chain ? d.ch_rsq : (d.use_modes ? d.mp_rsq : d.part));
  const int nb = d.use3 ? d.q3.nwg : (d.use_chain ? d.ch_nchunks : (d.use_modes ? d.mt[0].nwg : d.nb_sampled));
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) v += rsq_part[i];
  sampled_finish_total<F>(d, (F *)d.s, v, diag);   // v: this thread's share of ||R||^2
}

hipError_t launch_sampled_fin(const Batch &bt, int diag, hipStream_t s) {
  if (bt.host[0].prec == PREC_MIXED)
    hipLaunchKernelGGL(k_sampled_fin<float>, dim3(1, bt.ns), dim3(1024), 0, s, bt.dt, diag);
  else
    hipLaunchKernelGGL(k_sampled_fin<double>, dim3(1, bt.ns), dim3(1024), 0, s, bt.dt, diag);
  return hipGetLastError();
}

// Plain evaluation T(x^(j)) for prgd_eval (float64, padded cores).
template <int R>
__global__ void __launch_bounds__(256) k_eval(int m, long long N, const int *__restrict__ idx,
                                              const double *__restrict__ cores, const long long *coff_dev,
                                              double *__restrict__ out) {
  constexpr int RR = R * R;
  __shared__ long long coff[MAXM + 1];
  for (int i = threadIdx.x; i <= m; i += blockDim.x) coff[i] = coff_dev[i];
  __syncthreads();
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < N;
       j += (long long)gridDim.x * blockDim.x) {
    double l[R];
    const double *sl0 = cores + coff[0] + (long long)idx[j] * RR;
#pragma unroll
    for (int b = 0; b < R; ++b) l[b] = sl0[b];
    for (int k = 1; k < m; ++k) {
      const double *sl = cores + coff[k] + (long long)idx[(long long)k * N + j] * RR;
      double nl[R];
#pragma unroll
      for (int b = 0; b < R; ++b) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < R; ++a) acc = fma(l[a], sl[a * R + b], acc);
        nl[b] = acc;
      }
#pragma unroll
      for (int b = 0; b < R; ++b) l[b] = nl[b];
    }
    out[j] = l[0];
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

hipError_t launch_sampled_fin(const Batch &bt, int diag, hipStream_t s);

static int lds_block(int m, int R, int elem) {
  // choose the largest block (multiple of 64, <= 256) whose interface stack fits 63 KiB
  const long long per = (long long)(m - 1) * R * elem;
  for (int b = 256; b >= 64; b -= 64)
    if (per * b <= 64512) return b;
  return 0;
}

template <typename F, int R>
static hipError_t launch_sampled_t(const Batch &bt, int diag, hipStream_t s, hipEvent_t after_main) {
  const int m = bt.host[0].m;
  const int B = lds_block(m, R, (int)sizeof(F));
  if (B == 0) return hipErrorInvalidValue;
  int g = 1, pl = 0;
  for (int i = 0; i < bt.ns; ++i) {
    g = g > bt.host[i].nb_sampled ? g : bt.host[i].nb_sampled;
    pl = pl > bt.host[i].priv_len ? pl : bt.host[i].priv_len;
  }
  const size_t lds = ((size_t)(m - 1) * R * B + (size_t)pl) * sizeof(F);
  hipLaunchKernelGGL((k_sampled<F, R>), dim3(g, bt.ns), dim3(B), lds, s, bt.dt, diag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (after_main && (e = hipEventRecord(after_main, s)) != hipSuccess) return e;
  if (pl > 0) {
    hipLaunchKernelGGL((k_sampled_priv_reduce<F, R>), dim3((pl + 255) / 256, bt.ns), dim3(256), 0, s, bt.dt, diag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return launch_sampled_fin(bt, diag, s);
}

template <typename F>
static hipError_t launch_sampled_f(const Batch &bt, int diag, hipStream_t s, hipEvent_t ev) {
  switch (bt.host[0].R) {
    case 2: return launch_sampled_t<F, 2>(bt, diag, s, ev);
    case 4: return launch_sampled_t<F, 4>(bt, diag, s, ev);
    case 6: return launch_sampled_t<F, 6>(bt, diag, s, ev);
    case 8: return launch_sampled_t<F, 8>(bt, diag, s, ev);
    case 10: return launch_sampled_t<F, 10>(bt, diag, s, ev);
    case 12: return launch_sampled_t<F, 12>(bt, diag, s, ev);
    case 16: return launch_sampled_t<F, 16>(bt, diag, s, ev);
    default: return hipErrorInvalidValue;
  }
}

int sampled_block_size(int m, int R, int prec) {
  return lds_block(m, R, prec == PREC_MIXED ? 4 : 8);
}

hipError_t launch_sampled(const Batch &bt, int diag, hipStream_t s, hipEvent_t after_main) {
  if (bt.host[0].prec == PREC_MIXED) return launch_sampled_f<float>(bt, diag, s, after_main);
  return launch_sampled_f<double>(bt, diag, s, after_main);
}

hipError_t launch_eval(int m, int R, long long N, const int *idx, const double *cores, const long long *coff_dev,
                       double *out, hipStream_t s) {
  const int nb = (int)((N + 255) / 256 < 4096 ? (N + 255) / 256 : 4096);
  switch (R) {
#define PRGD_EVAL_CASE(RV) \
  case RV: hipLaunchKernelGGL((k_eval<RV>), dim3(nb), dim3(256), 0, s, m, N, idx, cores, coff_dev, out); break;
    PRGD_EVAL_CASE(2)
    PRGD_EVAL_CASE(4)
    PRGD_EVAL_CASE(6)
    PRGD_EVAL_CASE(8)
    PRGD_EVAL_CASE(10)
    PRGD_EVAL_CASE(12)
    PRGD_EVAL_CASE(16)
#undef PRGD_EVAL_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace prgd
