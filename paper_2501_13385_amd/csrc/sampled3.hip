// Sampled pass for order-3 tensors, samples grouped by the middle mode.
//
// For x = (x1, x2, x3) the entry is T(x) = l(x1)^T S(x2) r(x3) with
// l = T_1(0, x1, :), S = T_2(:, x2, :) (r1 x r2) and r = T_3(:, x3, 0)
// (section 2.1, TT format).  With u = S r and l2 = S^T l, the residual is
// R = l.u - y and the Euclidean core gradients (chain rule) are
//   dT_1(x1) += R u,   dT_3(x3) += R l2,   dT_2(x2) += R l r^T,
// and the squared mode-slice norms s_k(x_k) += R^2 (section 3.2.1).
//
// Layout of the work: Omega is stably sorted by x2, so a workgroup that owns a
// contiguous chunk of samples sees few distinct x2 ("segments") and the
// middle-core slice S(x2) is uniform across a wave.  Per workgroup:
//   * the boundary vectors l(.) and r(.) are staged in LDS when they fit;
//   * dT_1, dT_3, s_1, s_3 are accumulated in LDS (LDS atomics) and written
//     once as a per-workgroup partial;
//   * dT_2(x2) = sum over the segment of R l r^T is a rank-K update that the
//     matrix cores accumulate: 16x16x4 MFMAs whose A/B operands (R_k l_k[c],
//     r_k[c]) are fetched directly in the MFMA lane layout, so no transpose
//     is needed, and whose samples come from the lane's own row of 16 (a DPP
//     broadcast instead of a cross-row shuffle through LDS); each wave's
//     accumulator is added into a small per-workgroup segment table in LDS
//     when the segment changes.
// A second kernel sums the partials in a fixed order and finishes the metric
// weights.  The LDS atomics inside a workgroup add in an order that varies from
// run to run, so results repeat to rounding, not bit for bit.
#include <algorithm>
#include <type_traits>
#include <utility>

#include "prgd_internal.hpp"
#include "block_ops.hpp"

namespace prgd {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename F>
struct Mma;
template <>
struct Mma<double> {
  typedef d4v acc_t;
  __device__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of the 16x16 result held in element v of lane l (column l % 16)
  __device__ static int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <>
struct Mma<float> {
  typedef f4v acc_t;
  __device__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int v) { return 4 * (l >> 4) + v; }
};

// value of lane 16 (l / 16) + N in lane l: DPP row_newbcast, which copies lane
// N of each row of 16 lanes to the whole row without going through LDS
template <int N>
__device__ __forceinline__ int row_bcast(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x150 + N, 0xF, 0xF, false);
}
template <int N>
__device__ __forceinline__ float row_bcast(float v) {
  return __int_as_float(row_bcast<N>(__float_as_int(v)));
}
template <int N>
__device__ __forceinline__ double row_bcast(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = row_bcast<N>((int)b), hi = row_bcast<N>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// dT_2(v) += sum_k res_k l1_k r3_k^T over the 64 lanes of a wave as 16 MFMA
// steps: in step S row r of the wave (the MFMA's k index) holds the sample of
// lane 16 r + S, so the operands come from the lane's own row
template <typename M, typename F, int R, int... S>
__device__ __forceinline__ void segment_mfma(typename M::acc_t &acc, F res, int x1, int x3, const F *T1,
                                             const F *T3, int c, std::integer_sequence<int, S...>) {
  (
      [&] {
        const F rk = row_bcast<S>(res);
        const int x1k = row_bcast<S>(x1), x3k = row_bcast<S>(x3);
        F av = (F)0, bv = (F)0;
        if (c < R) {
          av = rk * T1[x1k * R + c];
          bv = T3[x3k * R + c];
        }
        acc = M::step(av, bv, acc);
      }(),
      ...);
}

template <typename F, int R, int NT, bool STAGE>
__global__ void __launch_bounds__(NT) k_sampled3(const Dev *__restrict__ dt, int diag) {
  const Dev &d = dt[blockIdx.y];
  const S3 &q = d.q3;
  if ((int)blockIdx.x >= q.nwg || (!diag && d.st->done)) return;
  const auto cores = glb((const F *)(d.prec == PREC_MIXED ? (const void *)d.cores32 : (const void *)d.cores));
  const auto bnd = glb((const F *)d.bnd);
  const auto y = glb((const F *)(d.prec == PREC_MIXED ? (const void *)d.y32 : (const void *)d.y64));
  typedef Mma<F> M;
  constexpr int RR = R * R;
  constexpr int SEGW = RR + 1;
  extern __shared__ unsigned char lds_raw[];
  const int n1 = d.n[0], n3 = d.n[2];
  const long long N = d.N;
  // boundary accumulators in float64 for both precisions (LDS float64 atomics
  // measured several times faster than float32 ones for this scatter); rows
  // padded to an odd number of doubles so random rows spread over more banks
  constexpr int RS = R + 1;
  double *lY1 = reinterpret_cast<double *>(lds_raw);
  double *lY3 = lY1 + n1 * RS;
  double *ls1 = lY3 + n3 * RS;
  double *ls3 = ls1 + n1;
  const int L = n1 * R + n3 * R + n1 + n3;            // compact partial layout
  const int LA = n1 * RS + n3 * RS + n1 + n3;         // padded accumulator layout
  F *lseg = reinterpret_cast<F *>(lY1 + LA);
  F *lT1 = lseg + KSEG * SEGW;
  F *lT3 = lT1 + n1 * R;
  for (int i = threadIdx.x; i < LA; i += NT) lY1[i] = 0.0;
  for (int i = threadIdx.x; i < KSEG * SEGW; i += NT) lseg[i] = (F)0;
  const F *gT1 = (const F *)bnd;
  const F *gT3 = (const F *)bnd + (long long)n1 * R;
  if (STAGE)
    for (int i = threadIdx.x; i < (n1 + n3) * R; i += NT) lT1[i] = bnd[i];
  const F *T1 = STAGE ? lT1 : gT1;
  const F *T3 = STAGE ? lT3 : gT3;
  __syncthreads();

  const long long j0 = (long long)blockIdx.x * q.chunk;
  const long long j1 = min(N, j0 + q.chunk);
  const int vfirst = glb(q.vfirst)[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int NW = NT / 64;
  const long long per = ((j1 - j0) + NW - 1) / NW;
  const long long ws = j0 + w * per, we = min(j1, ws + per);
  const auto ix1 = glb(d.idx), ix2 = glb(d.idx) + N, ix3 = glb(d.idx) + 2 * N;
  const long long co2 = d.coff[1];
  F *ovf = (F *)q.ovf;

  typename M::acc_t acc = M::zero();
  int wv = -1;          // segment accumulated in acc
  F ws2 = (F)0;         // per-lane sum of R^2 for that segment
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

  // software pipeline: the next batch's indices and value are in flight while
  // the current batch is processed
  int nx1 = 0, nx2 = -1, nx3 = 0;
  F ny = (F)0;
  if (ws + lane < we) {
    nx1 = ix1[ws + lane];
    nx2 = ix2[ws + lane];
    nx3 = ix3[ws + lane];
    ny = y[ws + lane];
  }
  for (long long jb = ws; jb < we; jb += 64) {
    const long long j = jb + lane;
    const bool act = j < we;
    const int x1 = nx1, x2 = act ? nx2 : -1, x3 = nx3;
    const F yv = ny;
    {
      const long long jn = j + 64;
      nx2 = -1;
      if (jn < we) {
        nx1 = ix1[jn];
        nx2 = ix2[jn];
        nx3 = ix3[jn];
        ny = y[jn];
      }
    }
    unsigned long long pending = __ballot(act);
    while (pending) {
      const int first = __ffsll((long long)pending) - 1;
      const int v = __builtin_amdgcn_readlane(x2, first);
      const bool me = act && (x2 == v);
      pending &= ~__ballot(me);
      if (v != wv) {
        flush();
        wv = v;
      }
      // the middle slice is uniform across the wave: read it through the
      // constant address space so that it lands in scalar registers
      typedef __attribute__((address_space(4))) const F *cptr;
      const cptr S = (cptr)((const F *)(cores + co2 + (long long)v * RR));
      F res = (F)0;
      if (me) {
        F l1[R], r3[R], u[R], l2[R];
#pragma unroll
        for (int a = 0; a < R; ++a) {
          l1[a] = T1[x1 * R + a];
          r3[a] = T3[x3 * R + a];
          u[a] = (F)0;
          l2[a] = (F)0;
        }
#pragma unroll
        for (int a = 0; a < R; ++a) {
#pragma unroll
          for (int b = 0; b < R; ++b) {
            const F sab = S[a * R + b];
            u[a] = fma(sab, r3[b], u[a]);
            l2[b] = fma(l1[a], sab, l2[b]);
          }
        }
        F t = (F)0;
#pragma unroll
        for (int a = 0; a < R; ++a) t = fma(l1[a], u[a], t);
        res = t - yv;
        const F r2 = res * res;
        rsq += (double)r2;
        ws2 += r2;
#pragma unroll
        for (int a = 0; a < R; ++a) {
          atomicAdd(&lY1[x1 * RS + a], (double)(res * u[a]));
          atomicAdd(&lY3[x3 * RS + a], (double)(res * l2[a]));
        }
        atomicAdd(&ls1[x1], (double)r2);
        atomicAdd(&ls3[x3], (double)r2);
      }
      // dT_2(v) += sum_k res_k l1_k r3_k^T over this wave's 64 lanes (zero for others)
      segment_mfma<M, F, R>(acc, res, x1, x3, T1, T3, c, std::make_integer_sequence<int, 16>{});
    }
  }
  flush();
  __shared__ double sbuf[16];
  const double bs = block_sum(rsq, sbuf);
  __syncthreads();
  auto pb = glb((F *)q.part_bnd) + (long long)blockIdx.x * L;
  for (int i = threadIdx.x; i < L; i += NT) {
    int p;
    if (i < n1 * R) p = (i / R) * RS + i % R;
    else if (i < (n1 + n3) * R) p = n1 * RS + ((i - n1 * R) / R) * RS + (i - n1 * R) % R;
    else p = (n1 + n3) * RS + (i - (n1 + n3) * R);
    pb[i] = (F)lY1[p];
  }
  auto ps = glb((F *)q.part_seg) + (long long)blockIdx.x * KSEG * SEGW;
  for (int i = threadIdx.x; i < KSEG * SEGW; i += NT) ps[i] = lseg[i];
  if (threadIdx.x == 0) glb(q.part_rsq)[blockIdx.x] = bs;
}

// Deterministic reduction of the per-workgroup partials into the gradient
// (padded core layout) and the slice sums, then the weight finish.
// Blocks [0, nbB): 64 boundary outputs each, the 4 waves splitting the
// workgroup partials; blocks [nbB, grid): middle-core segments, one output
// per thread (2-3 pieces each).
// WAVE: the partials of the low-rank variant (one wave per chunk; each
// chunk's first and last segments in two slots, its inner segments already
// written by the main kernel).
template <typename F, int R, bool WAVE>
__global__ void __launch_bounds__(256) k_sampled3_reduce(const Dev *__restrict__ dt, int diag) {
  const Dev &d = dt[blockIdx.y];
  const S3 &q = d.q3;
  constexpr int RR = R * R;
  constexpr int SEGW = RR + 1;
  const int n1 = d.n[0], n2 = d.n[1], n3 = d.n[2];
  const int L = n1 * R + n3 * R + n1 + n3;
  const int nbB = (L + 63) / 64;
  const int nbS = (int)(((long long)n2 * SEGW + 255) / 256);
  if ((int)blockIdx.x >= nbB + nbS || (!diag && d.st->done)) return;
  const auto Y = glb((F *)d.Y);
  const auto s = glb((F *)d.s);
  const auto pb = glb((const F *)q.part_bnd);
  const auto ps = glb((const F *)q.part_seg);
  const auto ovf = glb((F *)q.ovf);
  __shared__ double red[4][64];
  if ((int)blockIdx.x < nbB) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int o = blockIdx.x * 64 + lane;
    // sixteen independent loads in flight per lane: the partials come from
    // every XCD, so the time is set by the number of dependent round trips
    double a[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) a[u] = 0.0;
    if (o < L) {
      int b = w;
      for (; b + 60 < q.nwg; b += 64) {
#pragma unroll
        for (int u = 0; u < 16; ++u) a[u] += (double)pb[(long long)(b + 4 * u) * L + o];
      }
      for (; b < q.nwg; b += 4) a[0] += (double)pb[(long long)b * L + o];
    }
#pragma unroll
    for (int h = 8; h > 0; h >>= 1)
#pragma unroll
      for (int u = 0; u < h; ++u) a[u] += a[u + h];
    red[w][lane] = a[0];
    __syncthreads();
    if (w == 0 && o < L) {
      const double acc = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
      const int i = o;
      if (i < n1 * R) {
        const int x = i / R, a = i % R;
        Y[d.coff[0] + (long long)x * RR + a] = (F)acc;          // row 0 of slice x of the first core
      } else if (i < n1 * R + n3 * R) {
        const int ii = i - n1 * R, x = ii / R, a = ii % R;
        Y[d.coff[2] + (long long)x * RR + a * R] = (F)acc;      // column 0 of slice x of the last core
      } else if (i < n1 * R + n3 * R + n1) {
        s[d.soff[0] + (i - n1 * R - n3 * R)] = (F)acc;
      } else {
        s[d.soff[2] + (i - n1 * R - n3 * R - n1)] = (F)acc;
      }
    }
  } else if (WAVE) {
    const long long tot = (long long)n2 * SEGW;
    const long long oo = (long long)(blockIdx.x - nbB) * blockDim.x + threadIdx.x;
    if (oo < tot) {
      const int v = (int)(oo / SEGW), e = (int)(oo % SEGW);
      const int lo = glb(q.blo)[v], hi = glb(q.bhi)[v];
      const bool inner = lo == hi && v != glb(q.vfirst)[lo] && v != glb(q.vlast)[lo];
      if (!inner) {   // inner segments were written by the chunk that holds them
        double acc = 0.0;   // stays zero for a segment without samples (lo > hi)
        for (int b = lo; b <= hi; ++b)
          acc += (double)ps[((long long)b * 2 + (v == glb(q.vfirst)[b] ? 0 : 1)) * SEGW + e];
        if (e < RR) Y[d.coff[1] + (long long)v * RR + e] = (F)acc;
        else s[d.soff[1] + v] = (F)acc;
      }
    }
  } else {
    const long long tot = (long long)n2 * SEGW;
    const long long oo = (long long)(blockIdx.x - nbB) * blockDim.x + threadIdx.x;
    if (oo < tot) {
      const int v = (int)(oo / SEGW), e = (int)(oo % SEGW);
      double acc = (double)ovf[oo];
      ovf[oo] = (F)0;
      for (int b = glb(q.blo)[v]; b <= glb(q.bhi)[v]; ++b) {
        const int slot = v - glb(q.vfirst)[b];
        if (slot >= 0 && slot < KSEG) acc += (double)ps[((long long)b * KSEG + slot) * SEGW + e];
      }
      if (e < RR) Y[d.coff[1] + (long long)v * RR + e] = (F)acc;
      else s[d.soff[1] + v] = (F)acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Low-rank variant (padded rank R <= 4): one wave per workgroup, owning its
// LDS table of boundary-core gradients and slice sums.
//
// For small R the pass reads 16-20 bytes per sample and does a few dozen
// flops with them, so it is bound by memory bandwidth.  Here every wave is
// its own workgroup with a private table ((n_1 + n_3)(R + 1) float64
// values), so no two waves add into the same LDS word: the
// accumulation order is the wave's program order and a pass repeats bit for
// bit.  The stream is read with G batches of 64 samples in flight per
// group and the next group's loads issued before the current group is
// processed, the boundary vectors are gathered from L2 (a few KB to tens of
// KB, shared by all waves), and the middle-core gradient R x R block is an
// outer product accumulated per lane and reduced across the wave only when
// the segment changes.  Segments inside one wave's chunk are written to the
// gradient directly (no other wave touches them); a chunk's first and last
// segments go to two slots per wave that the reduction adds in wave order.
// ---------------------------------------------------------------------------

// Sum of v over the 64 lanes, the same bits in every lane: DPP rows of 16
// (every step adds two partial sums formed in the same order, so the lanes
// of a row agree), then the four row totals in a fixed order.
__device__ __forceinline__ double wave_total(double v) {
  auto dpp = [](double x, auto ctrl) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, decltype(ctrl)::value, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), decltype(ctrl)::value, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
  };
  v += dpp(v, std::integral_constant<int, 0xB1>{});   // lane ^ 1
  v += dpp(v, std::integral_constant<int, 0x4E>{});   // lane ^ 2
  v += dpp(v, std::integral_constant<int, 0x141>{});  // row half mirror
  v += dpp(v, std::integral_constant<int, 0x140>{});  // row mirror
  auto rd = [](double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
  };
  return (rd(v, 0) + rd(v, 16)) + (rd(v, 32) + rd(v, 48));
}

template <typename F, int R, int G>
__global__ void __launch_bounds__(64) k_sampled3w(const Dev *__restrict__ dt, int diag) {
  const Dev &d = dt[blockIdx.y];
  const S3 &q = d.q3;
  if ((int)blockIdx.x >= q.nwg || (!diag && d.st->done)) return;
  constexpr int RR = R * R, RS = R + 1, SEGW = RR + 1;
  const int lane = threadIdx.x;
  const auto cores = glb((const F *)(d.prec == PREC_MIXED ? (const void *)d.cores32 : (const void *)d.cores));
  const auto bnd = glb((const F *)d.bnd);
  const auto y = glb((const F *)(d.prec == PREC_MIXED ? (const void *)d.y32 : (const void *)d.y64));
  const int n1 = d.n[0], n3 = d.n[2];
  const long long N = d.N;
  // the table in float64 for both precisions (LDS float64 atomic adds
  // measured several times faster than float32 ones for this scatter)
  extern __shared__ unsigned char lds_raw[];
  double *tab1 = reinterpret_cast<double *>(lds_raw);   // [n1][R + 1]: dT_1 row, then s_1
  double *tab3 = tab1 + n1 * RS;                          // [n3][R + 1]: dT_3 row, then s_3
  for (int i = lane; i < (n1 + n3) * RS; i += 64) tab1[i] = 0.0;
  __syncthreads();
  const auto T1 = bnd, T3 = bnd + (long long)n1 * R;
  const int w = blockIdx.x;
  const long long j0 = (long long)w * q.chunk, j1 = min(N, j0 + q.chunk);
  const int vf = glb(q.vfirst)[w], vl = glb(q.vlast)[w];
  const auto ix1 = glb(d.idx), ix2 = glb(d.idx) + N, ix3 = glb(d.idx) + 2 * N;
  const long long co2 = d.coff[1];
  const auto Yg = glb((F *)d.Y);
  const auto sg = glb((F *)d.s);
  const auto slots = glb((F *)q.part_seg) + (long long)w * 2 * SEGW;

  F g2[RR];            // this lane's share of the current segment's R x R block
  F s2 = (F)0;         // and of its slice sum
#pragma unroll
  for (int e = 0; e < RR; ++e) g2[e] = (F)0;
  int wv = -1;         // segment held in g2 (wave-uniform)
  double rsq = 0.0;

  auto flush = [&]() {
    if (wv >= 0) {
      const bool inner = wv != vf && wv != vl;   // no other wave has samples in it
      F *dst = inner ? (F *)(Yg + d.coff[1] + (long long)wv * RR) : (F *)(slots + (wv == vf ? 0 : SEGW));
#pragma unroll
      for (int e = 0; e < RR; ++e) {
        const double t = wave_total((double)g2[e]);
        if (lane == 0) dst[e] = (F)t;
      }
      const double t = wave_total((double)s2);
      if (lane == 0) {
        if (inner) sg[d.soff[1] + wv] = (F)t;
        else dst[RR] = (F)t;
      }
    }
#pragma unroll
    for (int e = 0; e < RR; ++e) g2[e] = (F)0;
    s2 = (F)0;
  };

  // one group of G batches of 64 samples: indices and values
  struct Grp3 {
    int x1[G], x2[G], x3[G];
    F yv[G];
  };
  // every lane loads (past the end it re-reads the chunk's last sample, and
  // its x2 is marked -1 when used), so the loads are straight-line code and
  // a whole group is in flight at once
  auto load = [&](Grp3 &b, long long jb) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const long long j = min(jb + 64 * g + lane, j1 - 1);
      b.x1[g] = ix1[j];
      b.x2[g] = ix2[j];
      b.x3[g] = ix3[j];
      b.yv[g] = y[j];
    }
  };
  // one sample per lane, of segment v's slice S (in scalar registers): the
  // residual, the boundary-table adds and this lane's share of the block
  auto sample = [&](const F (&S)[RR], const F (&l1)[R], const F (&r3)[R], int x1, int x3, F yv) {
    F u[R], l2[R];
#pragma unroll
    for (int a = 0; a < R; ++a) {
      u[a] = (F)0;
      l2[a] = (F)0;
    }
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = 0; b < R; ++b) {
        u[a] = fma(S[a * R + b], r3[b], u[a]);
        l2[b] = fma(l1[a], S[a * R + b], l2[b]);
      }
    F t = (F)0;
#pragma unroll
    for (int a = 0; a < R; ++a) t = fma(l1[a], u[a], t);
    const F res = t - yv;
    const F r2 = res * res;
    rsq += (double)r2;
    s2 += r2;
#pragma unroll
    for (int a = 0; a < R; ++a) {
      const F rl = res * l1[a];
#pragma unroll
      for (int b = 0; b < R; ++b) g2[a * R + b] = fma(rl, r3[b], g2[a * R + b]);
    }
    double *t1 = tab1 + x1 * RS;
    double *t3 = tab3 + x3 * RS;
#pragma unroll
    for (int a = 0; a < R; ++a) {
      atomicAdd(&t1[a], (double)(res * u[a]));
      atomicAdd(&t3[a], (double)(res * l2[a]));
    }
    atomicAdd(&t1[R], (double)r2);
    atomicAdd(&t3[R], (double)r2);
  };
  // the middle slice v, uniform across the wave: scalar loads (a wave-uniform
  // address in the constant address space)
  typedef __attribute__((address_space(4))) const F *cptr;
  auto slice = [&](F (&S)[RR], int v) {
    const long long sb = __builtin_amdgcn_readfirstlane((int)(co2 + (long long)v * RR));
    const cptr Sp = (cptr)((const F *)cores + sb);
#pragma unroll
    for (int e = 0; e < RR; ++e) S[e] = Sp[e];
  };
  F Sw[RR];            // slice of the segment wv
#pragma unroll
  for (int e = 0; e < RR; ++e) Sw[e] = (F)0;

  Grp3 cur, nxt;
  load(cur, j0);
  for (long long jb = j0; jb < j1; jb += 64 * G) {
    // boundary vectors of the whole group, gathered before the next group's
    // loads are issued: vector loads complete in order, so the wait for
    // these gathers then leaves the next group's loads in flight
    F l1[G][R], r3[G][R];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int a = 0; a < R; ++a) {
        l1[g][a] = T1[(long long)cur.x1[g] * R + a];
        r3[g][a] = T3[(long long)cur.x3[g] * R + a];
      }
    if (jb + 64 * G < j1) load(nxt, jb + 64 * G);
    // fast path (segments are long): every sample of the group in segment wv
    bool other = false;
#pragma unroll
    for (int g = 0; g < G; ++g) other = other || (jb + 64 * g + lane < j1 && cur.x2[g] != wv);
    if (__ballot(other) == 0) {
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (jb + 64 * g + lane < j1) sample(Sw, l1[g], r3[g], cur.x1[g], cur.x3[g], cur.yv[g]);
    } else {
      // a segment starts inside the group: batch by batch, segment by
      // segment, reading the indices again (cached) so that nothing is
      // indexed by a run-time batch number in registers
#pragma unroll 1
      for (int g = 0; g < G; ++g) {
        if (jb + 64 * g >= j1) break;   // lane 0 is past the chunk: the rest is empty
        const long long j = jb + 64 * g + lane;
        const bool act = j < j1;
        const long long jc = act ? j : j1 - 1;
        const int x1 = ix1[jc], x3 = ix3[jc];
        const int x2 = act ? ix2[jc] : -1;
        const F yv = y[jc];
        F lg[R], rg[R];
#pragma unroll
        for (int a = 0; a < R; ++a) {
          lg[a] = T1[(long long)x1 * R + a];
          rg[a] = T3[(long long)x3 * R + a];
        }
        unsigned long long pending = __ballot(act);
        while (pending) {
          const int first = __ffsll((long long)pending) - 1;
          const int v = __builtin_amdgcn_readlane(x2, first);
          const bool me = act && x2 == v;
          pending &= ~__ballot(me);
          if (v != wv) {
            flush();
            wv = v;
            slice(Sw, v);
          }
          if (me) sample(Sw, lg, rg, x1, x3, yv);
        }
      }
    }
    cur = nxt;
  }
  flush();
  __syncthreads();
  // the table, in the compact partial layout: dT_1 rows, dT_3 rows, s_1, s_3
  const int L = n1 * R + n3 * R + n1 + n3;
  auto pb = glb((F *)q.part_bnd) + (long long)w * L;
  for (int i = lane; i < L; i += 64) {
    int p;
    if (i < n1 * R) p = (i / R) * RS + i % R;
    else if (i < (n1 + n3) * R) p = n1 * RS + ((i - n1 * R) / R) * RS + (i - n1 * R) % R;
    else if (i < (n1 + n3) * R + n1) p = (i - (n1 + n3) * R) * RS + R;
    else p = n1 * RS + (i - (n1 + n3) * R - n1) * RS + R;
    pb[i] = (F)tab1[p];
  }
  const double tr = wave_total(rsq);
  if (lane == 0) glb(q.part_rsq)[w] = tr;
}

hipError_t launch_sampled_fin(const Batch &bt, int diag, hipStream_t s);

template <typename F, int R>
static hipError_t launch3w_t(const Batch &bt, int diag, hipStream_t st, hipEvent_t after_main) {
  size_t lds = 0;
  int nwg = 1, nred = 1;
  for (int i = 0; i < bt.ns; ++i) {
    const Dev &d = bt.host[i];
    const int n1 = d.n[0], n3 = d.n[2];
    lds = std::max(lds, (size_t)(n1 + n3) * (R + 1) * sizeof(double));
    nwg = std::max(nwg, d.q3.nwg);
    const int L = n1 * R + n3 * R + n1 + n3;
    const long long nbS = ((long long)d.n[1] * (R * R + 1) + 255) / 256;
    nred = std::max(nred, (int)((L + 63) / 64 + nbS));
  }
  hipLaunchKernelGGL((k_sampled3w<F, R, sampled3w_group<R>()>), dim3(nwg, bt.ns), dim3(64), lds, st, bt.dt, diag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (after_main && (e = hipEventRecord(after_main, st)) != hipSuccess) return e;
  hipLaunchKernelGGL((k_sampled3_reduce<F, R, true>), dim3(nred, bt.ns), dim3(256), 0, st, bt.dt, diag);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sampled_fin(bt, diag, st);
}

template <typename F, int R>
static hipError_t launch3_t(const Batch &bt, int diag, hipStream_t st, hipEvent_t after_main) {
  if constexpr (R <= SAMPLED3W_MAX_R) {
    if (bt.host[0].q3.wave) return launch3w_t<F, R>(bt, diag, st, after_main);   // the batch shares the variant
  }
  size_t lds = 0;
  int nwg = 1, nred = 1;
  const int stage = bt.host[0].q3.stage;
  for (int i = 0; i < bt.ns; ++i) {
    const Dev &d = bt.host[i];
    const int n1 = d.n[0], n3 = d.n[2];
    const size_t base = (size_t)(n1 * (R + 1) + n3 * (R + 1) + n1 + n3) * 8 + (size_t)KSEG * (R * R + 1) * sizeof(F);
    lds = std::max(lds, base + (stage ? (size_t)(n1 + n3) * R * sizeof(F) : 0));
    nwg = std::max(nwg, d.q3.nwg);
    const int L = n1 * R + n3 * R + n1 + n3;
    const long long nbS = ((long long)d.n[1] * (R * R + 1) + 255) / 256;
    nred = std::max(nred, (int)((L + 63) / 64 + nbS));
  }
  constexpr int NT = (sizeof(F) == 8 && R >= 10) ? 512 : 1024;
  if (stage)
    hipLaunchKernelGGL((k_sampled3<F, R, NT, true>), dim3(nwg, bt.ns), dim3(NT), lds, st, bt.dt, diag);
  else
    hipLaunchKernelGGL((k_sampled3<F, R, NT, false>), dim3(nwg, bt.ns), dim3(NT), lds, st, bt.dt, diag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (after_main && (e = hipEventRecord(after_main, st)) != hipSuccess) return e;
  hipLaunchKernelGGL((k_sampled3_reduce<F, R, false>), dim3(nred, bt.ns), dim3(256), 0, st, bt.dt, diag);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sampled_fin(bt, diag, st);
}

template <typename F>
static hipError_t launch3_f(const Batch &bt, int diag, hipStream_t st, hipEvent_t ev) {
  switch (bt.host[0].R) {
    case 2: return launch3_t<F, 2>(bt, diag, st, ev);
    case 4: return launch3_t<F, 4>(bt, diag, st, ev);
    case 6: return launch3_t<F, 6>(bt, diag, st, ev);
    case 8: return launch3_t<F, 8>(bt, diag, st, ev);
    case 10: return launch3_t<F, 10>(bt, diag, st, ev);
    case 12: return launch3_t<F, 12>(bt, diag, st, ev);
    case 16: return launch3_t<F, 16>(bt, diag, st, ev);
    default: return hipErrorInvalidValue;
  }
}

// LDS bytes the order-3 pass needs (without / with staged boundary vectors)
size_t sampled3_lds_bytes(int n1, int n3, int R, int prec, int stage) {
  const size_t f = prec == PREC_MIXED ? 4 : 8;
  size_t b = (size_t)(n1 * (R + 1) + n3 * (R + 1) + n1 + n3) * 8 + (size_t)KSEG * (R * R + 1) * f;
  if (stage) b += (size_t)(n1 + n3) * R * f;
  return b;
}

int sampled3_kseg() { return KSEG; }

size_t sampled3w_lds_bytes(int n1, int n3, int R, int prec) {
  (void)prec;   // float64 tables for both precisions
  return (size_t)(n1 + n3) * (R + 1) * 8;
}

hipError_t launch_sampled3(const Batch &bt, int diag, hipStream_t st, hipEvent_t after_main) {
  if (bt.host[0].prec == PREC_MIXED) return launch3_f<float>(bt, diag, st, after_main);
  return launch3_f<double>(bt, diag, st, after_main);
}

}  // namespace prgd
