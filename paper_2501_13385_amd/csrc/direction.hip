// Adaptive step size (section 3.2.2, equation of the PRGD step size; for the
// Euclidean metric the RGD step of section 3.1).
//
// The steepest step along the direction xi in the tangent space is
//   alpha_l = ||xi||_W^2 / ||P_Omega xi||_F^2 = <G_l, xi> / ||P_Omega xi||^2,
// because xi = P~_T W^{-1} G_l with P~_T W-self-adjoint gives
// <xi, xi>_W = <W^{-1} G_l, xi>_W = <G_l, xi>, and G_l lives on Omega.  In the
// normalised units of the device (direction X = eps^{1/2} xi) the same ratio
// with X in place of xi is the normalised step alpha' = alpha eps^{-1/2}.
//
// X on Omega is the value of the tangent TT with block cores
//   [X_1, T_1],  [[T_k, 0], [X_k, T_k]],  [[T_m], [X_m]]
// (the sum of the m terms with one core replaced), evaluated per sample as a
// pair of row vectors (la carries "X used", lb "T only"); lb also yields
// T_l(x), hence the residual R = T_l(x) - y needed for <G_l, X>.
#include "prgd_internal.hpp"
#include "block_ops.hpp"

namespace prgd {

__device__ inline int xi_blocks(long long N) {
  const long long nb = (N + 2047) / 2048;
  return (int)(nb < 1 ? 1 : (nb > 1024 ? 1024 : nb));
}

template <int R>
__global__ void __launch_bounds__(256) k_xi(const Dev *__restrict__ dt) {
  const Dev &d = dt[blockIdx.y];
  const long long N = d.N;
  const int nb = xi_blocks(N);
  if ((int)blockIdx.x >= nb || d.step_policy != STEP_ADAPTIVE || d.st->done) return;
  constexpr int RR = R * R;
  const int m = d.m;
  const auto T = glb(d.cores), X = glb(d.X);
  const auto idx = glb(d.idx);
  const long long chunk = (N + nb - 1) / nb;
  const long long jlo = (long long)blockIdx.x * chunk, jhi = min(N, jlo + chunk);
  double num = 0.0, den = 0.0;
  for (long long j = jlo + threadIdx.x; j < jhi; j += blockDim.x) {
    double la[R], lb[R];
    {
      const long long s = d.coff[0] + (long long)idx[j] * RR;
#pragma unroll
      for (int b = 0; b < R; ++b) {
        la[b] = X[s + b];
        lb[b] = T[s + b];
      }
    }
    for (int c = 1; c < m - 1; ++c) {
      const long long s = d.coff[c] + (long long)idx[(long long)c * N + j] * RR;
      double na[R], nv[R];
#pragma unroll
      for (int b = 0; b < R; ++b) {
        double va = 0.0, vb = 0.0;
#pragma unroll
        for (int a = 0; a < R; ++a) {
          const double tab = T[s + a * R + b], xab = X[s + a * R + b];
          va = fma(la[a], tab, fma(lb[a], xab, va));
          vb = fma(lb[a], tab, vb);
        }
        na[b] = va;
        nv[b] = vb;
      }
#pragma unroll
      for (int b = 0; b < R; ++b) {
        la[b] = na[b];
        lb[b] = nv[b];
      }
    }
    const long long s = d.coff[m - 1] + (long long)idx[(long long)(m - 1) * N + j] * RR;
    double xv = 0.0, tv = 0.0;
#pragma unroll
    for (int a = 0; a < R; ++a) {
      const double ta = T[s + a * R], xa = X[s + a * R];
      xv = fma(la[a], ta, fma(lb[a], xa, xv));
      tv = fma(lb[a], ta, tv);
    }
    const double yv = d.prec == PREC_MIXED ? (double)glb(d.y32)[j] : glb(d.y64)[j];
    const double res = tv - yv;
    num = fma(res, xv, num);
    den = fma(xv, xv, den);
  }
  __shared__ double sbuf[16];
  num = block_sum(num, sbuf);
  den = block_sum(den, sbuf);
  if (threadIdx.x == 0) {
    d.part[2 * blockIdx.x] = num;
    d.part[2 * blockIdx.x + 1] = den;
  }
}

// alpha' = <G_l, X> / ||P_Omega X||^2 (one block per solve)
__global__ void __launch_bounds__(256) k_xi_fin(const Dev *__restrict__ dt) {
  const Dev &d = dt[blockIdx.y];
  if (d.step_policy != STEP_ADAPTIVE || d.st->done) return;
  const int nb = xi_blocks(d.N);
  double a0 = 0.0, a1 = 0.0;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    a0 += d.part[2 * k];
    a1 += d.part[2 * k + 1];
  }
  __shared__ double sbuf[16];
  a0 = block_sum(a0, sbuf);
  a1 = block_sum(a1, sbuf);
  if (threadIdx.x == 0) {
    State *st = d.st;
    const double an = a1 > 0.0 ? a0 / a1 : 0.0;
    st->alpha_n = an;
    const int it = st->iter;
    if (it < d.hist_cap) d.hist[it].alpha = an * sqrt(st->eps_n);
  }
}

hipError_t launch_adaptive_step(const Batch &bt, hipStream_t s) {
  bool any = false;
  int g = 1;
  for (int i = 0; i < bt.ns; ++i) {
    const Dev &d = bt.host[i];
    if (d.step_policy != STEP_ADAPTIVE) continue;
    any = true;
    long long nb = (d.N + 2047) / 2048;
    nb = nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
    g = g > (int)nb ? g : (int)nb;
  }
  if (!any) return hipSuccess;
  switch (bt.host[0].R) {
#define PRGD_XI_CASE(RV) \
  case RV: hipLaunchKernelGGL((k_xi<RV>), dim3(g, bt.ns), dim3(256), 0, s, bt.dt); break;
    PRGD_XI_CASE(2)
    PRGD_XI_CASE(4)
    PRGD_XI_CASE(6)
    PRGD_XI_CASE(8)
    PRGD_XI_CASE(10)
    PRGD_XI_CASE(12)
    PRGD_XI_CASE(16)
#undef PRGD_XI_CASE
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_xi_fin, dim3(1, bt.ns), dim3(256), 0, s, bt.dt);
  return hipGetLastError();
}

}  // namespace prgd
