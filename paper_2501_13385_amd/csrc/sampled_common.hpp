// Finish of the sampled pass, shared by its variants (runs in one block).
#pragma once

#include "prgd_internal.hpp"
#include "block_ops.hpp"

namespace prgd {

// Finish the pass in one block: total ||R||^2, residual stopping test,
// eps_l = max_{k,x} s_k(x) (= ||G_l||_vee^2), metric factors
// omega_k(x) = (1 + s_k(x)/eps)^{1/(2m)} (all 1 for the Euclidean metric) and
// the normalised step (the adaptive step is set after the direction is known).
// In units normalised by eps the direction is eps^{1/2} times the paper's, so
// alpha = c eps^{1/2} / p becomes c / p and a constant alpha becomes
// alpha / eps^{1/2}; with the Euclidean metric eps plays no part (eps_n = 1).
template <typename F>
__device__ void sampled_finish_total(const Dev &d, F *sacc, double rs, int diag) {
  __shared__ double sbuf[32];
  State *st = d.st;
  // the state this block updates is read first, so that its latency overlaps
  // the loads of the slice sums
  const double y_sq = st->y_sq;
  const int it = st->iter;
  const int m = d.m;
  const int stot = diag ? 0 : d.soff[m];
  // the first KC slice sums of each thread stay in registers for the weights
  constexpr int KC = 4;
  double sv[KC];
  double emax = 0.0;
#pragma unroll
  for (int u = 0; u < KC; ++u) {
    const int i = threadIdx.x + u * blockDim.x;
    sv[u] = i < stot ? (double)sacc[i] : 0.0;
    emax = fmax(emax, sv[u]);
  }
  for (int i = threadIdx.x + KC * blockDim.x; i < stot; i += blockDim.x) emax = fmax(emax, (double)sacc[i]);
  block_sum_max(rs, emax, sbuf);   // rs enters as this thread's share of ||R||^2
  if (diag) {
    if (threadIdx.x == 0) st->res_sq = rs;
    return;
  }
  __shared__ int go;
  __shared__ double eps_sh;
  if (threadIdx.x == 0) {
    go = 0;
    st->res_sq = rs;
    const double rel = y_sq > 0.0 ? sqrt(rs / y_sq) : sqrt(rs);
    st->rel_res = rel;
    IterRecord rec;
    rec.iter = it;
    rec.flags = 0;
    rec.rel_residual = rel;
    rec.rel_change = 0.0;
    rec.rel_error = 0.0;
    rec.eps = 0.0;
    rec.alpha = 0.0;
    if (!isfinite(rs)) {
      st->status = -5;
      st->done = 1;
    } else if (d.stop_rule == STOP_RESIDUAL && rel <= d.tol) {
      st->status = 0;
      st->done = 1;
    } else if (it >= d.max_iter) {
      st->status = (d.stop_rule == STOP_NONE) ? 0 : 1;
      st->done = 1;
    } else if (emax == 0.0) {
      st->status = 0;      // G_l = 0: T_l fits every observation
      st->done = 1;
    } else {
      const double epsn = (d.metric == METRIC_EUCLIDEAN) ? 1.0 : (d.eps_fixed > 0.0 ? d.eps_fixed : emax);
      st->eps_n = epsn;
      eps_sh = epsn;
      st->alpha_n = (d.step_policy == STEP_THEORY) ? d.step / d.p
                    : (d.step_policy == STEP_CONST) ? d.step / sqrt(epsn) : 0.0;
      rec.eps = epsn;
      rec.alpha = st->alpha_n * sqrt(epsn);
      st->upd = 0;
      go = 1;
    }
    if (it < d.hist_cap) d.hist[it] = rec;
  }
  __syncthreads();
  if (go) {
    const double inv = 1.0 / eps_sh;
    const double ex = 1.0 / (2.0 * m);
    const bool euclid = d.metric == METRIC_EUCLIDEAN;
#pragma unroll
    for (int u = 0; u < KC; ++u) {
      const int i = threadIdx.x + u * blockDim.x;
      if (i < stot) {
        d.omega[i] = euclid ? 1.0 : pow(1.0 + sv[u] * inv, ex);
        sacc[i] = (F)0;
      }
    }
    for (int i = threadIdx.x + KC * blockDim.x; i < stot; i += blockDim.x) {
      d.omega[i] = euclid ? 1.0 : pow(1.0 + (double)sacc[i] * inv, ex);
      sacc[i] = (F)0;
    }
  }
}

}  // namespace prgd
