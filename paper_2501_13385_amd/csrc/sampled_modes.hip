// Sampled pass for any order without atomics: one pass per mode.
//
// For mode k the observations are kept stably sorted by x_k, so a workgroup
// owning a contiguous chunk sees few distinct x_k ("segments") and the core
// slice T_k(x_k) is uniform across a wave.  Each sample evaluates its left
// interface l = T_1(x_1) ... T_{k-1}(x_{k-1}) (row vector; e_1 for k = 1) and
// right interface r = T_{k+1}(x_{k+1}) ... T_m(x_m) (column vector; e_1 for
// k = m), then the entry T(x) = l T_k(x_k) r (section 2.1, TT format), the
// residual R = T(x) - y, and contributes
//   dT_k(x_k) += R l^T r^T     (chain rule on the TT format)
//   s_k(x_k)  += R^2           (squared mode-slice norm, section 3.2.1).
// Within a segment the rank-64 updates of a wave are summed on the matrix
// cores (16x16x4 MFMAs whose operands are staged per wave in LDS), flushed to
// a small per-workgroup segment table when the segment changes, and the
// tables are summed in a fixed order by a second kernel.  All modes run in one
// launch (blockIdx.x selects mode and workgroup).  The pass of mode 1 also
// records ||R||^2.  Compared with one pass that scatters into every mode, this
// re-evaluates the interfaces m times but needs no global atomics.
#include <algorithm>

#include "prgd_internal.hpp"
#include "block_ops.hpp"

namespace prgd {

typedef double m_d4v __attribute__((ext_vector_type(4)));
typedef float m_f4v __attribute__((ext_vector_type(4)));

template <typename F>
struct MmaM;
template <>
struct MmaM<double> {
  typedef m_d4v acc_t;
  __device__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <>
struct MmaM<float> {
  typedef m_f4v acc_t;
  __device__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int v) { return 4 * (l >> 4) + v; }
};

__device__ inline void mp_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// LDS bytes of k_modes: per wave 64 x R operands P (R l) and Q (r), plus the
// segment table
__host__ __device__ inline size_t modes_lds_bytes(int R, int prec, int nt) {
  const size_t f = prec == PREC_MIXED ? 4 : 8;
  return ((size_t)(nt / 64) * 2 * 64 * (R + 1) + (size_t)KSEG * (R * R + 1)) * f;
}

// Cores of every mode staged in LDS when they fit in this many bytes: the
// interfaces gather a whole slice per sample and mode, which then comes from
// LDS (broadcast when lanes share a slice) instead of the caches.
constexpr size_t MODES_STAGE_MAX = 64 * 1024;

// the staged copy or the global cores (keeping the global address space)
template <bool STAGE, typename L, typename G>
__device__ __forceinline__ auto pick_cores(L staged, G global) {
  if constexpr (STAGE) return staged;
  else return global;
}

// Stored interfaces: one pass over the grouping-mode copy of Omega forms each
// sample's prefix products l_k = T_1(x_1) ... T_k(x_k) (a left sweep, which also
// gives T(x) and the residual) and suffix products r_k = T_k(x_k) ... T_m(x_m)
// (a right sweep), and writes for every mode k l_{k-1} and (r_{k+1}, R_j) at
// the sample's own position (coalesced).  Mode k's pass gathers them through
// the position map instead of re-evaluating both chains (2m slice products
// per sample instead of m (m - 1)).
template <typename F, int R, bool STAGE>
__global__ void __launch_bounds__(256) k_iface(const Dev *__restrict__ dt, int diag) {
  const Dev &d = dt[blockIdx.y];
  const ModeTab &q0 = d.mt[0];
  if ((int)blockIdx.x >= q0.nwg || (!diag && d.st->done)) return;
  constexpr int RR = R * R;
  const int m = d.m;
  const long long N = d.N;
  extern __shared__ unsigned char lds_raw[];
  F *lcores = reinterpret_cast<F *>(lds_raw);
  const auto gcores = glb((const F *)(d.prec == PREC_MIXED ? (const void *)d.cores32 : (const void *)d.cores));
  if (STAGE)
    for (long long i = threadIdx.x; i < d.coff[m]; i += blockDim.x) lcores[i] = gcores[i];
  __syncthreads();
  const auto cores = pick_cores<STAGE>((const F *)lcores, gcores);
  const auto idx = glb(d.idx);
  const auto y = glb((const F *)(d.prec == PREC_MIXED ? (const void *)d.y32 : (const void *)d.y64));
  const auto ifl = glb((F *)d.ifl), ifr = glb((F *)d.ifr);
  const long long j0 = (long long)blockIdx.x * q0.chunk, j1 = min(N, j0 + q0.chunk);
  double rsq = 0.0;
  for (long long j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    F v[R];
#pragma unroll
    for (int a = 0; a < R; ++a) v[a] = a == 0 ? (F)1 : (F)0;
    for (int k = 0; k < m; ++k) {            // left sweep: record l_{k-1}, then v <- v T_k(x_k)
      const long long rec = ((long long)k * N + j) * R;
#pragma unroll
      for (int a = 0; a < R; ++a) ifl[rec + a] = v[a];
      const auto sl = cores + d.coff[k] + (long long)idx[(long long)k * N + j] * RR;
      F nv[R];
#pragma unroll
      for (int b = 0; b < R; ++b) {
        F t = (F)0;
#pragma unroll
        for (int a = 0; a < R; ++a) t = fma(v[a], sl[a * R + b], t);
        nv[b] = t;
      }
#pragma unroll
      for (int a = 0; a < R; ++a) v[a] = nv[a];
    }
    const F res = v[0] - y[j];
    rsq += (double)res * (double)res;
#pragma unroll
    for (int a = 0; a < R; ++a) v[a] = a == 0 ? (F)1 : (F)0;
    for (int k = m - 1; k >= 0; --k) {       // right sweep: record r_{k+1} and R_j, then v <- T_k(x_k) v
      const long long rec = ((long long)k * N + j) * (R + 1);
#pragma unroll
      for (int a = 0; a < R; ++a) ifr[rec + a] = v[a];
      ifr[rec + R] = res;
      const auto sl = cores + d.coff[k] + (long long)idx[(long long)k * N + j] * RR;
      F nv[R];
#pragma unroll
      for (int a = 0; a < R; ++a) {
        F t = (F)0;
#pragma unroll
        for (int b = 0; b < R; ++b) t = fma(sl[a * R + b], v[b], t);
        nv[a] = t;
      }
#pragma unroll
      for (int a = 0; a < R; ++a) v[a] = nv[a];
    }
  }
  __shared__ double sbuf[16];
  const double bs = block_sum(rsq, sbuf);
  if (threadIdx.x == 0) glb(d.mp_rsq)[blockIdx.x] = bs;
}

template <typename F, int R, int NT, bool STAGE, bool IFACE>
__global__ void __launch_bounds__(NT) k_modes(const Dev *__restrict__ dt, int diag) {
  const Dev &d = dt[blockIdx.y];
  if ((int)blockIdx.x >= d.mt_wg || (!diag && d.st->done)) return;
  const int m = d.m;
  int k = 0;
  while (k + 1 < m && d.mt[k + 1].wg0 <= (int)blockIdx.x) ++k;
  const ModeTab &q = d.mt[k];
  const int wg = (int)blockIdx.x - q.wg0;
  typedef MmaM<F> M;
  constexpr int RR = R * R;
  constexpr int SEGW = RR + 1;
  constexpr int NW = NT / 64;
  extern __shared__ unsigned char lds_raw[];
  F *lseg = reinterpret_cast<F *>(lds_raw);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // [64][R + 1]: R_j l_j and r_j, rows padded to an odd length so that the
  // lanes' row-wise stores spread over the banks
  constexpr int RP = R + 1;
  F *P = lseg + KSEG * SEGW + (long long)w * 2 * 64 * RP;
  F *Q = P + 64 * RP;
  for (int i = threadIdx.x; i < KSEG * SEGW; i += NT) lseg[i] = (F)0;
  const auto gcores = glb((const F *)(d.prec == PREC_MIXED ? (const void *)d.cores32 : (const void *)d.cores));
  F *lcores = lseg + KSEG * SEGW + (long long)NW * 2 * 64 * RP;
  if (STAGE)
    for (long long i = threadIdx.x; i < d.coff[m]; i += NT) lcores[i] = gcores[i];
  __syncthreads();
  const auto cores = pick_cores<STAGE>((const F *)lcores, gcores);
  const auto y = glb((const F *)q.y);
  const long long N = d.N;
  const auto idx = glb(q.idx);
  const long long j0 = (long long)wg * q.chunk, j1 = min(N, j0 + q.chunk);
  const int vfirst = glb(q.vfirst)[wg];
  const long long per = ((j1 - j0) + NW - 1) / NW;
  const long long ws = j0 + w * per, we = min(j1, ws + per);
  const long long cok = d.coff[k];
  F *ovf = (F *)q.ovf;

  typename M::acc_t acc = M::zero();
  int wv = -1;
  F ws2 = (F)0;
  double rsq = 0.0;
  const int c = lane & 15;

  auto flush = [&]() {
    if (wv >= 0) {
      const int slot = wv - vfirst;
      const F s2 = (F)wave_sum((double)ws2);
      F *dst = (slot >= 0 && slot < KSEG) ? lseg + slot * SEGW : nullptr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = M::row(lane, v);
        if (i < R && c < R) {
          if (dst) atomicAdd(&dst[i * R + c], acc[v]);
          else atomicAdd(&ovf[(long long)wv * SEGW + i * R + c], acc[v]);
        }
      }
      if (lane == 0) {
        if (dst) atomicAdd(&dst[RR], s2);
        else atomicAdd(&ovf[(long long)wv * SEGW + RR], s2);
      }
    }
    acc = M::zero();
    ws2 = (F)0;
  };

  for (long long jb = ws; jb < we; jb += 64) {
    const long long j = jb + lane;
    const bool act = j < we;
    const int xk = act ? idx[(long long)k * N + j] : -1;
    // interfaces of this sample
    F lv[R], rv[R];
    F rpre = (F)0;   // stored residual
    if (IFACE) {
      const long long i = act ? glb(d.rpos)[(long long)k * N + j] : 0;
      const auto lrec = glb((const F *)d.ifl) + ((long long)k * N + i) * R;
      const auto rrec = glb((const F *)d.ifr) + ((long long)k * N + i) * (R + 1);
#pragma unroll
      for (int a = 0; a < R; ++a) {
        lv[a] = act ? lrec[a] : (F)0;
        rv[a] = act ? rrec[a] : (F)0;
      }
      rpre = act ? rrec[R] : (F)0;
    } else if (k == 0) {
#pragma unroll
      for (int a = 0; a < R; ++a) lv[a] = (a == 0) ? (F)1 : (F)0;
    } else {
      const int x0 = act ? idx[j] : 0;
      const auto sl = cores + d.coff[0] + (long long)x0 * RR;
#pragma unroll
      for (int b = 0; b < R; ++b) lv[b] = sl[b];
      for (int cc = 1; cc < k; ++cc) {
        const int x = act ? idx[(long long)cc * N + j] : 0;
        const auto s2 = cores + d.coff[cc] + (long long)x * RR;
        F nl[R];
#pragma unroll
        for (int b = 0; b < R; ++b) {
          F t = (F)0;
#pragma unroll
          for (int a = 0; a < R; ++a) t = fma(lv[a], s2[a * R + b], t);
          nl[b] = t;
        }
#pragma unroll
        for (int b = 0; b < R; ++b) lv[b] = nl[b];
      }
    }
    if (IFACE) {
    } else if (k == m - 1) {
#pragma unroll
      for (int a = 0; a < R; ++a) rv[a] = (a == 0) ? (F)1 : (F)0;
    } else {
      const int xl = act ? idx[(long long)(m - 1) * N + j] : 0;
      const auto sl = cores + d.coff[m - 1] + (long long)xl * RR;
#pragma unroll
      for (int a = 0; a < R; ++a) rv[a] = sl[a * R];
      for (int cc = m - 2; cc > k; --cc) {
        const int x = act ? idx[(long long)cc * N + j] : 0;
        const auto s2 = cores + d.coff[cc] + (long long)x * RR;
        F nr[R];
#pragma unroll
        for (int a = 0; a < R; ++a) {
          F t = (F)0;
#pragma unroll
          for (int b = 0; b < R; ++b) t = fma(s2[a * R + b], rv[b], t);
          nr[a] = t;
        }
#pragma unroll
        for (int a = 0; a < R; ++a) rv[a] = nr[a];
      }
    }
    const F yv = (!IFACE && act) ? y[j] : (F)0;
    unsigned long long pending = __ballot(act);
    while (pending) {
      const int first = __ffsll((long long)pending) - 1;
      const int v = __builtin_amdgcn_readlane(xk, first);
      const bool me = act && (xk == v);
      pending &= ~__ballot(me);
      if (v != wv) {
        flush();
        wv = v;
      }
      const auto S = cores + cok + (long long)v * RR;
      F res = (F)0;
      if (me) {
        if (IFACE) {
          res = rpre;
        } else {
          F t = (F)0;
#pragma unroll
          for (int a = 0; a < R; ++a) {
            F u = (F)0;
#pragma unroll
            for (int b = 0; b < R; ++b) u = fma(S[a * R + b], rv[b], u);
            t = fma(lv[a], u, t);
          }
          res = t - yv;
        }
        const F r2 = res * res;
        rsq += (double)r2;
        ws2 += r2;
      }
      // stage R_j l_j and r_j of this wave's lanes (zero for other segments)
#pragma unroll
      for (int a = 0; a < R; ++a) {
        P[lane * RP + a] = res * lv[a];
        Q[lane * RP + a] = me ? rv[a] : (F)0;
      }
      mp_wave_sync();
#pragma unroll
      for (int st = 0; st < 16; ++st) {
        const int kk = 4 * st + (lane >> 4);
        F av = (F)0, bv = (F)0;
        if (c < R) {
          av = P[kk * RP + c];
          bv = Q[kk * RP + c];
        }
        acc = M::step(av, bv, acc);
      }
      mp_wave_sync();
    }
  }
  flush();
  __shared__ double sbuf[16];
  const double bs = block_sum(rsq, sbuf);   // ends with a barrier: the table is complete
  auto ps = glb((F *)q.part_seg) + (long long)wg * KSEG * SEGW;
  for (int i = threadIdx.x; i < KSEG * SEGW; i += NT) ps[i] = lseg[i];
  if (!IFACE && k == 0 && threadIdx.x == 0) glb(d.mp_rsq)[wg] = bs;   // else written by k_iface
}

// Sum the segment tables of every mode in a fixed order into the padded
// gradient and the slice sums (one output per thread, all modes in one launch).
template <typename F, int R>
__global__ void __launch_bounds__(256) k_modes_reduce(const Dev *__restrict__ dt, int diag) {
  const Dev &d = dt[blockIdx.y];
  constexpr int RR = R * R;
  constexpr int SEGW = RR + 1;
  const long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= d.mt_out || (!diag && d.st->done)) return;
  int k = 0;
  while (k + 1 < d.m && d.mt[k + 1].out0 <= o) ++k;
  const ModeTab &q = d.mt[k];
  const long long oo = o - q.out0;
  const int v = (int)(oo / SEGW), e = (int)(oo % SEGW);
  const auto ovf = glb((F *)q.ovf);
  const auto ps = glb((const F *)q.part_seg);
  double acc = (double)ovf[oo];
  ovf[oo] = (F)0;
  for (int b = glb(q.blo)[v]; b <= glb(q.bhi)[v]; ++b) {
    const int slot = v - glb(q.vfirst)[b];
    if (slot >= 0 && slot < KSEG) acc += (double)ps[((long long)b * KSEG + slot) * SEGW + e];
  }
  if (e < RR) glb((F *)d.Y)[d.coff[k] + (long long)v * RR + e] = (F)acc;
  else glb((F *)d.s)[d.soff[k] + v] = (F)acc;
}

hipError_t launch_sampled_fin(const Batch &bt, int diag, hipStream_t s);

template <typename F, int R>
static hipError_t launch_modes_t(const Batch &bt, int diag, hipStream_t st, hipEvent_t after_main) {
  constexpr int NT = 256;
  int g = 1;
  long long go = 1;
  for (int i = 0; i < bt.ns; ++i) {
    g = std::max(g, bt.host[i].mt_wg);
    go = std::max<long long>(go, bt.host[i].mt_out);
  }
  size_t lds = modes_lds_bytes(R, bt.host[0].prec, NT), core_bytes = 0;
  int g0 = 1;
  for (int i = 0; i < bt.ns; ++i) {
    core_bytes = std::max(core_bytes, (size_t)bt.host[i].coff[bt.host[i].m] * sizeof(F));
    g0 = std::max(g0, bt.host[i].mt0_nwg);
  }
  const bool stage = core_bytes <= MODES_STAGE_MAX;
  if (bt.host[0].use_iface) {   // the whole batch shares the variant
    if (stage) {
      hipLaunchKernelGGL((k_iface<F, R, true>), dim3(g0, bt.ns), dim3(256), core_bytes, st, bt.dt, diag);
      if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
      hipLaunchKernelGGL((k_modes<F, R, NT, true, true>), dim3(g, bt.ns), dim3(NT), lds + core_bytes, st, bt.dt, diag);
    } else {
      hipLaunchKernelGGL((k_iface<F, R, false>), dim3(g0, bt.ns), dim3(256), 0, st, bt.dt, diag);
      if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
      hipLaunchKernelGGL((k_modes<F, R, NT, false, true>), dim3(g, bt.ns), dim3(NT), lds, st, bt.dt, diag);
    }
  } else if (stage) {
    hipLaunchKernelGGL((k_modes<F, R, NT, true, false>), dim3(g, bt.ns), dim3(NT), lds + core_bytes, st, bt.dt, diag);
  } else {
    hipLaunchKernelGGL((k_modes<F, R, NT, false, false>), dim3(g, bt.ns), dim3(NT), lds, st, bt.dt, diag);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (after_main && (e = hipEventRecord(after_main, st)) != hipSuccess) return e;
  hipLaunchKernelGGL((k_modes_reduce<F, R>), dim3((int)((go + 255) / 256), bt.ns), dim3(256), 0, st, bt.dt, diag);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return launch_sampled_fin(bt, diag, st);
}

template <typename F>
static hipError_t launch_modes_f(const Batch &bt, int diag, hipStream_t st, hipEvent_t ev) {
  switch (bt.host[0].R) {
    case 2: return launch_modes_t<F, 2>(bt, diag, st, ev);
    case 4: return launch_modes_t<F, 4>(bt, diag, st, ev);
    case 6: return launch_modes_t<F, 6>(bt, diag, st, ev);
    case 8: return launch_modes_t<F, 8>(bt, diag, st, ev);
    case 10: return launch_modes_t<F, 10>(bt, diag, st, ev);
    case 12: return launch_modes_t<F, 12>(bt, diag, st, ev);
    case 16: return launch_modes_t<F, 16>(bt, diag, st, ev);
    default: return hipErrorInvalidValue;
  }
}

size_t sampled_modes_lds_bytes(int R, int prec) { return modes_lds_bytes(R, prec, 256); }

hipError_t launch_sampled_modes(const Batch &bt, int diag, hipStream_t st, hipEvent_t after_main) {
  if (bt.host[0].prec == PREC_MIXED) return launch_modes_f<float>(bt, diag, st, after_main);
  return launch_modes_f<double>(bt, diag, st, after_main);
}

}  // namespace prgd
