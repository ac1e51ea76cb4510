// One pass over Omega for orders >= 4 with small mode sizes (n_k R^2 <= 256,
// R the padded rank in {2, 4, 8}): the order-14, n = 4 workload and its kind.
//
// What is computed (section 2.1, TT format; section 3.2.1, metric weights):
// for every sample x^(j) the entry T(x) = l_k T_k(x_k) r_{k+1} with the left
// interface l_k = T_1(x_1) ... T_{k-1}(x_{k-1}) (row vector, l_1 = e_1) and
// the right interface r_{k+1} = T_{k+1}(x_{k+1}) ... T_m(x_m) (column vector,
// r_{m+1} = e_1), the residual R_j = T(x) - y_j, and for every core k
//   dT_k(x_k) += R_j l_k^T r_{k+1}^T     (chain rule on the TT format)
//   s_k(x_k)  += R_j^2                   (squared mode-slice norm)
// plus ||R||^2.
//
// How (one HIP workgroup per chunk of Omega):
//   * Omega is sorted by its first u mode indices (mixed radix, mode 1 most
//     significant) and split into chunks that never straddle a change of that
//     prefix.  Within a chunk x_1..x_u are the same for every sample, so
//     l_{u+1} is one vector per chunk, and the contributions to cores 1..u
//     reduce to V_{u+1} = sum_j R_j r_{u+1}(x^(j)): dT_k(x_k) += l_k^T V_{k+1}^T
//     with V_k = T_k(x_k) V_{k+1}, formed once per chunk.
//   * Lane = sample.  A right sweep forms r_m, ..., r_{u+1} (slices of the
//     cores u+1..m staged in LDS, rows of a slice read as 16-byte vectors) and
//     parks r_{k+1} in LDS for the gradient; the residual follows from l_{u+1}
//     and r_{u+1}; a left sweep then carries l_k.  When a wave's LDS slots do
//     not hold every parked interface (float64 at R = 8, eight waves per
//     workgroup), the sweep parks the first cores' ones and the left sweep
//     parks the rest in segments, each by a second right sweep from core m.
//   * Gradient of core k >= u+1: a 16x16 MFMA tile whose rows are (x_hi, a)
//     and columns (x_lo, b), x_k = x_hi * (16/R) + x_lo, holds the whole
//     n_k x R x R gradient (n_k <= (16/R)^2).  A K-step takes the four samples
//     16 q + S (q = MFMA k index = lane / 16): A = l_k[a] of that sample when its
//     x_hi matches the row, B = R_j r_{k+1}[b] when its x_lo matches the column.
//     Each wave keeps one accumulator tile per core in registers for its whole
//     share of the chunk.
//   * Slice sums of cores >= u+1: a butterfly over the wave leaves every lane
//     the sum for one slice value, accumulated per lane across batches.
//   * Per chunk: the waves' tiles, slice sums and V_{u+1} are summed in LDS in
//     wave order and written as one partial; two reduction kernels sum the
//     partials over groups of chunks and then over groups, in a fixed order.
// No atomics: float64 results repeat bit for bit.
#include <algorithm>
#include <utility>

#include "prgd_internal.hpp"
#include "block_ops.hpp"

namespace prgd {

typedef double c_d4v __attribute__((ext_vector_type(4)));
typedef float c_f4v __attribute__((ext_vector_type(4)));

template <typename F>
struct MmaC;
template <>
struct MmaC<double> {
  typedef c_d4v acc_t;
  __device__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of the 16x16 result held in element v of lane l (column l % 16)
  __device__ static int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <>
struct MmaC<float> {
  typedef c_f4v acc_t;
  __device__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int v) { return 4 * (l >> 4) + v; }
};

// value of lane 16 (l / 16) + N in lane l (DPP row_newbcast)
template <int N>
__device__ __forceinline__ int cbcast(int v) {
  // every lane reads a valid source, so the destination's old value is never
  // kept: the form without one spares a move per broadcast
  return __builtin_amdgcn_mov_dpp(v, 0x150 + N, 0xF, 0xF, false);
}
template <int N>
__device__ __forceinline__ float cbcast(float v) {
  return __int_as_float(cbcast<N>(__float_as_int(v)));
}
template <int N>
__device__ __forceinline__ double cbcast(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = cbcast<N>((int)b), hi = cbcast<N>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Order of LDS accesses among the lanes of one wave.  A wave's LDS operations
// are performed in issue order, so a store by one lane is seen by a later load
// of another lane of the same wave; only the compiler must not move memory
// operations across this point (no wait on the LDS counter is needed).
__device__ __forceinline__ void chain_wave_order() {
  __builtin_amdgcn_wave_barrier();
  __asm__ __volatile__("" ::: "memory");
}

// value of lane l ^ 32 (v_permlane32_swap; whole wave active)
__device__ __forceinline__ int xor32(int v, int lane) {
  const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  // [0] holds the lower half's values in both halves, [1] the upper half's
  return (lane & 32) ? (int)p[0] : (int)p[1];
}
// value of lane l ^ 16 (v_permlane16_swap; whole wave active)
__device__ __forceinline__ int xor16(int v, int lane) {
  const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  // [0] holds rows (0, 0, 2, 2) of the input, [1] rows (1, 1, 3, 3)
  return (lane & 16) ? (int)p[0] : (int)p[1];
}
template <int OFF>
__device__ __forceinline__ int xor_lane(int v, int lane) {
  if constexpr (OFF == 32) return xor32(v, lane);
  else if constexpr (OFF == 16) return xor16(v, lane);
  else return __shfl_xor(v, OFF, 64);
}
template <int OFF>
__device__ __forceinline__ float xor_lane(float v, int lane) {
  return __int_as_float(xor_lane<OFF>(__float_as_int(v), lane));
}
template <int OFF>
__device__ __forceinline__ double xor_lane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = xor_lane<OFF>((int)b, lane), hi = xor_lane<OFF>((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// value of a partner lane that differs from lane in bit OFF and agrees with it
// in the bits above OFF (the butterfly steps below need only that): OFF 32 and
// 16 by permlane swaps, 8 and 4 by the row and half-row mirrors, 2 and 1 by
// quad permutations (DPP, no LDS round trip)
template <int OFF>
__device__ __forceinline__ int pair_lane(int v, int lane) {
  if constexpr (OFF == 32) return xor32(v, lane);
  else if constexpr (OFF == 16) return xor16(v, lane);
  else if constexpr (OFF == 8) return __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false);
  else if constexpr (OFF == 4) return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);
  else if constexpr (OFF == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
  else return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
}
template <int OFF>
__device__ __forceinline__ float pair_lane(float v, int lane) {
  return __int_as_float(pair_lane<OFF>(__float_as_int(v), lane));
}
template <int OFF>
__device__ __forceinline__ double pair_lane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = pair_lane<OFF>((int)b, lane), hi = pair_lane<OFF>((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sizes shared by the host plan and the kernel.
template <int R>
struct ChainShape {
  static constexpr int RR = R * R;
  static constexpr int XH = 16 / R;                          // slice values per tile side
  static constexpr int NX = XH * XH < 16 ? XH * XH : 16;     // slice values per core
  static constexpr int TILE = 256;
  // staging slot: R rows of 64 samples, value a of sample s at
  // a * 68 + s + s / 16: a wave's row store is consecutive, and the four
  // samples of a K-step (one per group of 16) with their R values spread over
  // the banks
  static constexpr int SP = 68;
  static constexpr int SLOTW = R * SP;
};

// Sum of v over the lanes whose index agrees in the top log2(NX) bits after
// a reduce-scatter of the one-hot vector (v at slot x) across the wave:
// returns, in lane l, the sum of v over the lanes {l ^ t} (t over the top
// bits) whose x equals l >> (6 - log2 NX).
template <typename F, int NX, int H, int OFF>
__device__ __forceinline__ void scatter_halve(F (&kept)[NX / 2], int lane) {
  if constexpr (H > 1) {
    const bool hb = (lane & OFF) != 0;
#pragma unroll
    for (int i = 0; i < H / 2; ++i) {
      const F send = hb ? kept[i] : kept[H / 2 + i];
      const F recv = pair_lane<OFF>(send, lane);
      kept[i] = (hb ? kept[H / 2 + i] : kept[i]) + recv;
    }
    scatter_halve<F, NX, H / 2, OFF / 2>(kept, lane);
  }
}

template <typename F, int NX>
__device__ __forceinline__ F slice_scatter(F v, int x, int lane) {
  constexpr int H0 = NX / 2;
  const F vp = xor_lane<32>(v, lane);
  const int xp = xor_lane<32>(x, lane);
  const int base = (lane & 32) ? H0 : 0;
  F kept[H0];
#pragma unroll
  for (int i = 0; i < H0; ++i) kept[i] = (x == base + i ? v : (F)0) + (xp == base + i ? vp : (F)0);
  scatter_halve<F, NX, H0, 16>(kept, lane);
  return kept[0];
}

// F with every bit cleared where m = 0 (m is 0 or all ones)
__device__ __forceinline__ double keep_if(double v, int m) {
  const long long b = __double_as_longlong(v);
  const int lo = (int)b & m, hi = (int)(b >> 32) & m;
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ float keep_if(float v, int m) { return __int_as_float(__float_as_int(v) & m); }

// A sample's tile position as one word: bit x_hi = x / (16/R) and bit
// 8 + x_lo, x_lo = x % (16/R); a lane of tile row (or column) block h tests
// its bit with one signed bit-field extract (0 or all ones)
template <int R>
__device__ __forceinline__ int chain_code(int x) {
  constexpr int XH = 16 / R;
  return (1 << ((unsigned)x / XH)) | (256 << ((unsigned)x % XH));
}

// One K-step S of a core's gradient tile: the four samples 16 q + S, with
// the operands av (the row's entry of R_j l_k, or of l_{u+1}) and bv (the
// column's entry of r_{k+1}) already loaded; each is kept where the sample's
// slice falls in the lane's row or column block.  AM = 0: A is the uniform
// l_{u+1} and the residual scales B.
template <typename F, int R, int S, int AM>
__device__ __forceinline__ void chain_kstep(typename MmaC<F>::acc_t &acc, int wc, F res, F av, F bv, int lane) {
  const int h = (lane & 15) / R;
  const int ws = cbcast<S>(wc);   // the sample's chain_code
  av = keep_if(av, __builtin_amdgcn_sbfe(ws, h, 1));
  if constexpr (AM == 0) bv = cbcast<S>(res) * bv;
  bv = keep_if(bv, __builtin_amdgcn_sbfe(ws, 8 + h, 1));
  acc = MmaC<F>::step(av, bv, acc);
}

// The 16 K-steps of a core's tile.  AM: A from the uniform l_{u+1} (0) or the
// staged R_j l_k (1); BM: B from the parked r_{k+1} (0), from column 0 of the
// last core's slice (1) or e_1 (2).  All operand loads are issued before the
// first MFMA, so that they are in flight together.
template <typename F, int R, int AM, int BM, int... S>
__device__ __forceinline__ void chain_mfma(typename MmaC<F>::acc_t &acc, int xc, int xl, F res, F lamA,
                                           const F *stg, const F *bsl, const F *tlast, int SL, F bE, int lane,
                                           std::integer_sequence<int, S...>) {
  const int q = lane >> 4, a = (lane & 15) % R;
  const int wc = chain_code<R>(xc);
  F av[sizeof...(S)], bv[sizeof...(S)];
  if constexpr (AM == 0) ((av[S] = lamA), ...);
  else ((av[S] = stg[a * 68 + 16 * q + S + q]), ...);
  if constexpr (BM == 0) ((bv[S] = bsl[a * 68 + 16 * q + S + q]), ...);
  else if constexpr (BM == 1) ((bv[S] = tlast[cbcast<S>(xl) * SL + a * R]), ...);
  else ((bv[S] = bE), ...);
  (chain_kstep<F, R, S, AM>(acc, wc, res, av[S], bv[S], lane), ...);
}

// 16-byte LDS vector of the working precision
template <typename F>
struct V16;
template <>
struct V16<double> {
  typedef double t __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
};
template <>
struct V16<float> {
  typedef float t __attribute__((ext_vector_type(4)));
  static constexpr int n = 4;
};

// G rows of the slice at sl (row-major R x R, 16-byte aligned) into registers,
// all loads issued before any is used
template <typename F, int R, int G>
__device__ __forceinline__ void load_rows(F (&rows)[G][R], const F *sl, int a0) {
  typedef typename V16<F>::t VT;
  constexpr int VN = V16<F>::n;
  if constexpr (R % VN == 0) {
    const VT *v = reinterpret_cast<const VT *>(sl + a0 * R);
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int b = 0; b < R / VN; ++b) {
        const VT t = v[g * (R / VN) + b];
#pragma unroll
        for (int e = 0; e < VN; ++e) rows[g][b * VN + e] = t[e];
      }
  } else {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int b = 0; b < R; ++b) rows[g][b] = sl[(a0 + g) * R + b];
  }
}

// rows per load group: enough loads in flight, bounded registers
template <typename F, int R>
struct RowGroup {
  static constexpr int G = (R * (int)sizeof(F) * 4 <= 128 ? R : (R * (int)sizeof(F) <= 64 ? 4 : 2));
};

// l <- l T(x) for one sample per lane, T the slice at sl (row-major R x R)
template <typename F, int R>
__device__ __forceinline__ void chain_left_step(F (&lam)[R], const F *sl) {
  constexpr int G = RowGroup<F, R>::G;
  F nl[R];
#pragma unroll
  for (int b = 0; b < R; ++b) nl[b] = (F)0;
#pragma unroll
  for (int a0 = 0; a0 < R; a0 += G) {
    F rows[G][R];
    load_rows<F, R, G>(rows, sl, a0);
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int b = 0; b < R; ++b) nl[b] = fma(lam[a0 + g], rows[g][b], nl[b]);
  }
#pragma unroll
  for (int b = 0; b < R; ++b) lam[b] = nl[b];
}

// r <- T(x) r
template <typename F, int R>
__device__ __forceinline__ void chain_right_step(F (&rho)[R], const F *sl) {
  constexpr int G = RowGroup<F, R>::G;
  F nr[R];
#pragma unroll
  for (int a0 = 0; a0 < R; a0 += G) {
    F rows[G][R];
    load_rows<F, R, G>(rows, sl, a0);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      F t = (F)0;
#pragma unroll
      for (int b = 0; b < R; ++b) t = fma(rows[g][b], rho[b], t);
      nr[a0 + g] = t;
    }
  }
#pragma unroll
  for (int a = 0; a < R; ++a) rho[a] = nr[a];
}

// Sum of v over the lanes that share lane's top log2(NX) bits (after
// slice_scatter every such lane holds a part of the same slice's sum).
template <typename F, int NX>
__device__ __forceinline__ F slice_finish(F v, int lane) {
  constexpr int G = 64 / NX;   // lanes per slice: 16 or 4
  static_assert(G <= 16, "a slice's lanes must lie in one row of 16");
  if constexpr (G >= 16) v += pair_lane<8>(v, lane);
  if constexpr (G >= 8) v += pair_lane<4>(v, lane);
  if constexpr (G >= 4) v += pair_lane<2>(v, lane);
  if constexpr (G >= 2) v += pair_lane<1>(v, lane);
  return v;
}

template <typename F, int R, int MAXC, int NW>
__global__ void __launch_bounds__(NW * 64) k_chain(const Dev *__restrict__ dt, int diag, int nsl) {
  const Dev &d = dt[blockIdx.y];
  if ((int)blockIdx.x >= d.ch_nchunks || (!diag && d.st->done)) return;
  typedef MmaC<F> M;
  constexpr int RR = R * R;
  constexpr int NT = NW * 64;
  // eight waves: the launch may grant fewer parking slots than generic cores
  // (segments); four waves: always all of them
  constexpr bool SEG = NW > 4;
  constexpr int NX = ChainShape<R>::NX;
  constexpr int SLOTW = ChainShape<R>::SLOTW;
  constexpr int SL = RR + 16 / (int)sizeof(F);
  const int m = d.m, u = d.ch_u, nc = m - u;
  const long long N = d.N;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const bool mixed = d.prec == PREC_MIXED;
  const auto gcores = glb((const F *)(mixed ? (const void *)d.cores32 : (const void *)d.cores));
  const auto idx = glb(d.idx);
  const auto y = glb((const F *)(mixed ? (const void *)d.y32 : (const void *)d.y64));
  extern __shared__ unsigned char lds_raw[];
  F *lc = reinterpret_cast<F *>(lds_raw);
  // LDS offsets of the staged cores u+1..m (core u + c at loff[c], slice x at x SL)
  int loff[MAXC];
  int lo = 0;
#pragma unroll
  for (int c = 0; c < MAXC; ++c) {
    loff[c] = lo;
    if (c < nc) lo += d.n[u + c] * SL;
  }
  const int lo_last = lo - d.n[m - 1] * SL;
  // parking slots per wave: one per generic core when the launch grants them
  // all, else nsl (>= 2) and the right interfaces are parked in segments
  const int nfull = chain_nslots(nc);
  const int nslots = SEG ? min(nfull, max(nsl, 2)) : nfull;
  const int WT = nc * 256, WS = nc * NX;
  const int WR = WT + WS;                                   // end-of-chunk sums per wave
  const int region = chain_region(nslots, nfull, WR, SLOTW);
  F *wsl = lc + lo + (long long)w * region;
  F *wss = lc + lo + (long long)NW * region + (long long)w * WS;   // this wave's slice sums
  F *lamu_s = lc + lo + (long long)NW * region + (long long)NW * WS;   // l_{u+1}, shared
  F *pre_l = lamu_s + R;         // [u][R]: l_k = e_1^T T_0(x_0) .. T_{k-1}(x_{k-1})
  F *pre_sl = lc + lo;           // [u][R^2]: the chunk's prefix slices T_k(x_k), k < u (in
                                 // the wave slots, free until the batch loop)
  for (int i = lane; i < WS; i += 64) wss[i] = (F)0;
  const int cs = glb(d.ch_start)[blockIdx.x], cl = glb(d.ch_len)[blockIdx.x];
  // one flat pass over the staged cores and the prefix slices, so that each
  // thread's loads are independent and in flight together
  {
    int cend[MAXC];   // element ends of the staged cores
    int acc_e = 0;
#pragma unroll
    for (int c = 0; c < MAXC; ++c) {
      if (c < nc) acc_e += d.n[u + c] * RR;
      cend[c] = acc_e;
    }
    const int ntot = acc_e + u * RR;
#pragma unroll 4
    for (int i = threadIdx.x; i < ntot; i += NT) {
      if (i < acc_e) {
        int c = 0;
#pragma unroll
        for (int cc = 0; cc < MAXC - 1; ++cc) c += (i >= cend[cc]) ? 1 : 0;
        const int rem = i - (c > 0 ? cend[c - 1] : 0);
        lc[loff[c] + (rem / RR) * SL + rem % RR] = gcores[d.coff[u + c] + rem];
      } else {
        const int t = i - acc_e, k = t / RR, e = t % RR;
        const int x = idx[(long long)k * N + cs];
        pre_sl[t] = gcores[d.coff[k] + (long long)x * RR + e];
      }
    }
  }
  __syncthreads();
  // l_0 .. l_u along the prefix: the same for every sample of the chunk
  // (lanes b < R of the first wave, one vector-matrix step at a time)
  if (threadIdx.x < R) {
    const int b = threadIdx.x;
    F lb = b == 0 ? (F)1 : (F)0;
    for (int k = 0; k < u; ++k) {
      pre_l[k * R + b] = lb;
      chain_wave_order();
      F t = (F)0;
#pragma unroll
      for (int a = 0; a < R; ++a) t = fma(pre_l[k * R + a], pre_sl[k * RR + a * R + b], t);
      lb = t;
    }
    lamu_s[b] = lb;
  }
  // e_1 in the MFMA lane layout: the A operand of core u+1 (whose tile then
  // holds G_x = sum R_j r_{u+2}; l_{u+1} is applied once per chunk) and the B
  // operand of the last core (r_{m+1} = e_1)
  const int aA = (lane & 15) % R;
  const F bE = aA == 0 ? (F)1 : (F)0;
  const F lamA = bE;
  __syncthreads();

  // generic cores c = 0 .. nc-3 (core u + c): B from the parked r_{k+1};
  // core nc-2: B from column 0 of the last core's slice; core nc-1: B = e_1
  constexpr int MG = MAXC - 2;
  typename M::acc_t acc[MG > 0 ? MG : 1];
#pragma unroll
  for (int c = 0; c < MG; ++c) acc[c] = M::zero();
  typename M::acc_t accP = M::zero(), accL = M::zero();
  double rsq = 0.0;
  const F *tlast = lc + lo_last;
  const int lo_pen = nc >= 2 ? lo_last - d.n[m - 2] * SL : 0;
  const int ng = nc - 2;                  // generic cores (may be <= 0)
  const int nbt = (cl + 63) >> 6;
  for (int bt = w; bt < nbt; bt += NW) {
    const int jj = bt * 64 + lane;
    const bool act = jj < cl;
    const long long j = (long long)cs + (act ? jj : 0);
    int xk[MG > 0 ? MG : 1];
#pragma unroll
    for (int c = 0; c < MG; ++c) xk[c] = (c < ng && act) ? idx[(long long)(u + c) * N + j] : 0;
    const int xl = act ? idx[(long long)(m - 1) * N + j] : 0;
    const int xp = (nc >= 2 && act) ? idx[(long long)(m - 2) * N + j] : 0;
    const F yv = act ? y[j] : (F)0;
    chain_wave_order();   // the previous batch's reads of the slots come first
    // right sweep: r_m = T_m(:, x_m, 0), r_{m-1} = T_{m-1}(x_{m-1}) r_m, then
    // r_k = T_k(x_k) r_{k+1} parking r_{k+1} in slot c (k = u + c <= m-3)
    F rho[R];
#pragma unroll
    for (int a = 0; a < R; ++a) rho[a] = tlast[xl * SL + a * R];
    if (nc >= 2) chain_right_step<F, R>(rho, lc + lo_pen + xp * SL);
#pragma unroll
    for (int c = MG - 1; c >= 0; --c) {
      if (c < ng) {
        if (!SEG || c < nslots) {   // the first segment's interfaces
          F *dst = wsl + c * SLOTW + lane + (lane >> 4);
#pragma unroll
          for (int a = 0; a < R; ++a) dst[a * 68] = rho[a];
        }
        chain_right_step<F, R>(rho, lc + loff[c] + xk[c] * SL);
      }
    }
    F lam[R];
#pragma unroll
    for (int a = 0; a < R; ++a) lam[a] = lamu_s[a];
    F t = (F)0;
#pragma unroll
    for (int a = 0; a < R; ++a) t = fma(lam[a], rho[a], t);
    const F res = act ? t - yv : (F)0;
    const F r2 = res * res;
    rsq += (double)r2;
    // slice sums: each wave adds one batch's per-slice totals to its table
    // (lanes with low bits 0 hold them after the butterfly)
    {
      const bool lead = (lane & (64 / NX - 1)) == 0;
      const int xs = lane / (64 / NX);
#pragma unroll
      for (int c = 0; c < MG; ++c)
        if (c < ng) {
          const F v = slice_finish<F, NX>(slice_scatter<F, NX>(r2, xk[c], lane), lane);
          if (lead) wss[c * NX + xs] += v;
        }
      if (nc >= 2) {
        const F v = slice_finish<F, NX>(slice_scatter<F, NX>(r2, xp, lane), lane);
        if (lead) wss[(nc - 2) * NX + xs] += v;
      }
      const F v = slice_finish<F, NX>(slice_scatter<F, NX>(r2, xl, lane), lane);
      if (lead) wss[(nc - 1) * NX + xs] += v;
    }
    // left sweep with the gradient tiles, generic cores in segments: the
    // cores [s0, s0 + sl) find r_{k+1} at slots 0 .. sl-1.  The first segment
    // was parked by the sweep above; a later one is parked by a second right
    // sweep from the last core down (its first core's staged R_j l_k goes to
    // slot sl, so a later segment holds at most nslots - 1 cores).
    chain_wave_order();   // the parked r_{k+1} before the tiles read them
    int s0 = 0, sl = SEG ? (ng < nslots ? ng : nslots) : ng;
    int slast = 0;        // slot of the last generic core's r_{k+1}
    while (s0 < ng) {
      if (SEG && s0 > 0) {
        F rr[R];
#pragma unroll
        for (int a = 0; a < R; ++a) rr[a] = tlast[xl * SL + a * R];
        if (nc >= 2) chain_right_step<F, R>(rr, lc + lo_pen + xp * SL);
#pragma unroll
        for (int c = MG - 1; c >= 1; --c) {
          if (c < ng && c >= s0) {
            if (c < s0 + sl) {
              F *dst = wsl + (c - s0) * SLOTW + lane + (lane >> 4);
#pragma unroll
              for (int a = 0; a < R; ++a) dst[a * 68] = rr[a];
            }
            if (c > s0) chain_right_step<F, R>(rr, lc + loff[c] + xk[c] * SL);
          }
        }
        chain_wave_order();
      }
#pragma unroll
      for (int c = 0; c < MG; ++c) {
        if (c >= s0 && c < s0 + sl) {
          const int sb = c - s0;
          // l_{k+1} is formed alongside core k's MFMA steps (independent work
          // for the scheduler to interleave); core k's A operand is the staged l_k
          if (c == 0) {
            chain_left_step<F, R>(lam, lc + loff[c] + xk[c] * SL);
            chain_mfma<F, R, 0, 0>(acc[c], xk[c], xl, res, lamA, wsl, wsl, tlast, SL, bE, lane,
                                   std::make_integer_sequence<int, 16>{});
          } else {
            // a slot whose r_{k+1} the previous core has read, or the one past the segment's
            F *stg = wsl + (sb == 0 ? sl : sb - 1) * SLOTW;
            F *dst = stg + lane + (lane >> 4);
#pragma unroll
            for (int a = 0; a < R; ++a) dst[a * 68] = res * lam[a];
            chain_wave_order();
            chain_left_step<F, R>(lam, lc + loff[c] + xk[c] * SL);
            chain_mfma<F, R, 1, 0>(acc[c], xk[c], xl, res, lamA, stg, wsl + sb * SLOTW, tlast, SL, bE, lane,
                                   std::make_integer_sequence<int, 16>{});
          }
          chain_wave_order();
        }
      }
      slast = ng - 1 - s0;
      if constexpr (!SEG) break;
      s0 += sl;
      sl = ng - s0 < nslots - 1 ? ng - s0 : nslots - 1;
    }
    const int stgP = slast, stgL = slast;   // staging of cores m-2 and m-1
    if (nc >= 2) {   // core m-2
      F *stg = wsl + stgP * SLOTW;
      if (ng >= 1) {
        F *dst = stg + lane + (lane >> 4);
#pragma unroll
        for (int a = 0; a < R; ++a) dst[a * 68] = res * lam[a];
        chain_wave_order();
        chain_left_step<F, R>(lam, lc + lo_pen + xp * SL);
        chain_mfma<F, R, 1, 1>(accP, xp, xl, res, lamA, stg, wsl, tlast, SL, bE, lane,
                               std::make_integer_sequence<int, 16>{});
      } else {
        chain_left_step<F, R>(lam, lc + lo_pen + xp * SL);
        chain_mfma<F, R, 0, 1>(accP, xp, xl, res, lamA, stg, wsl, tlast, SL, bE, lane,
                               std::make_integer_sequence<int, 16>{});
      }
      chain_wave_order();
    }
    {   // core m-1
      F *stg = wsl + stgL * SLOTW;
      if (nc >= 2) {
        F *dst = stg + lane + (lane >> 4);
#pragma unroll
        for (int a = 0; a < R; ++a) dst[a * 68] = res * lam[a];
        chain_wave_order();
        chain_mfma<F, R, 1, 2>(accL, xl, xl, res, lamA, stg, wsl, tlast, SL, bE, lane,
                               std::make_integer_sequence<int, 16>{});
      } else {
        chain_mfma<F, R, 0, 2>(accL, xl, xl, res, lamA, stg, wsl, tlast, SL, bE, lane,
                               std::make_integer_sequence<int, 16>{});
      }
      chain_wave_order();
    }
  }

  // ---- per-chunk partial: waves summed in LDS in wave order ----
  __shared__ double sbuf[16];
  const double rs_tot = block_sum(rsq, sbuf);    // ends with a barrier: every wave is past its slots
  // the prefix slices again for the shared cores' gradients, in the staged
  // cores past core u+1 (no longer read) when they fit there, else read from
  // global memory one step at a time
  const bool pre_in_lds = u * RR <= lo - loff[1 < MAXC ? 1 : 0];
  F *pre_sl2 = lc + loff[1 < MAXC ? 1 : 0];
  if (u > 0 && pre_in_lds)
    for (int t = threadIdx.x; t < u * RR; t += NT) {
      const int k = t / RR, e = t % RR;
      const int x = idx[(long long)k * N + cs];
      pre_sl2[t] = gcores[d.coff[k] + (long long)x * RR + e];
    }
  // the waves' tiles and slice sums, summed in wave order: nr regions of WR
  // in the slot area; waves w < nr write region w, the rest add into region
  // w mod nr in rounds, then the regions are summed in order
  F *red = lc + lo;
  const int nr = SEG ? min(NW, (NW * region) / WR) : NW;
  for (int t = 0; t < NW; t += nr) {
    if (w >= t && w < t + nr) {
      F *dst = red + (long long)(w - t) * WR;
      auto put_core = [&](int c, const typename M::acc_t &tile) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          F &o = dst[c * 256 + M::row(lane, v) * 16 + (lane & 15)];
          o = (SEG && t > 0) ? o + tile[v] : tile[v];
        }
      };
#pragma unroll
      for (int c = 0; c < MG; ++c)
        if (c < ng) put_core(c, acc[c]);
      if (nc >= 2) put_core(nc - 2, accP);
      put_core(nc - 1, accL);
      for (int i = lane; i < WS; i += 64) dst[WT + i] = (SEG && t > 0) ? dst[WT + i] + wss[i] : wss[i];
    }
    __syncthreads();
  }
  const int W = chain_part_width(m, u, R);
  const auto part = glb((F *)d.ch_part) + (long long)blockIdx.x * W;
  // core u+1's tile holds G_x (A = e_1) and is written as l_{u+1}[a] G_x[b]
  // below, the rest as it is
  for (int e = threadIdx.x; e < WR; e += NT) {
    F v = red[e];
    for (int rg = 1; rg < nr; ++rg) v += red[(long long)rg * WR + e];
    red[e] = v;
    if (e >= 256) part[e] = v;
  }
  __syncthreads();
  {
    constexpr int XH = 16 / R;
    const int nu = d.n[u];
    for (int e = threadIdx.x; e < 256; e += NT) {
      const int i = e >> 4, jc = e & 15, a = i % R;
      const int x = (i / R) * XH + jc / R;
      const F g = x < nu ? red[((i / R) * R) * 16 + jc] : (F)0;    // G_x[b] sits in row (x_hi, 0)
      part[e] = lamu_s[a] * g;
    }
  }
  if (threadIdx.x == 0) glb(d.ch_rsq)[blockIdx.x] = rs_tot;
  // cores 1..u: l_k^T V_{k+1}^T at the chunk's x_k, with V_{u+1} the sum of
  // the waves' R_j r_{u+1} and V_k = T_k(x_k) V_{k+1} (one wave)
  if (u > 0 && w == 0) {
    // V_{u+1} = sum_x T_{u+1}(x) G_x (core u+1 staged at loff[0])
    constexpr int XH = 16 / R;
    F V[R];
#pragma unroll
    for (int a = 0; a < R; ++a) {
      F v = (F)0;
      for (int x = 0; x < d.n[u]; ++x) {
        const F *sl = lc + x * SL;
        const int rowb = ((x / XH) * R) * 16 + (x % XH) * R;
#pragma unroll
        for (int b = 0; b < R; ++b) v = fma(sl[a * R + b], red[rowb + b], v);
      }
      V[a] = v;
    }
    for (int k = u - 1; k >= 0; --k) {
      // l_k and T_k(x_k) of the chunk's prefix, staged by the prologue
      F l[R];
#pragma unroll
      for (int a = 0; a < R; ++a) l[a] = pre_l[k * R + a];
      if (lane < RR) {
        F g = (F)0;
#pragma unroll
        for (int a = 0; a < R; ++a)
#pragma unroll
          for (int b = 0; b < R; ++b)
            if (a * R + b == lane) g = l[a] * V[b];
        part[WT + WS + k * RR + lane] = g;
      }
      const F *sl = pre_in_lds
                        ? (const F *)(pre_sl2 + k * RR)
                        : (const F *)(gcores + d.coff[k] +
                                      (long long)__builtin_amdgcn_readfirstlane(idx[(long long)k * N + cs]) * RR);
      F nv[R];
#pragma unroll
      for (int a = 0; a < R; ++a) {
        F t = (F)0;
#pragma unroll
        for (int b = 0; b < R; ++b) t = fma(sl[a * R + b], V[b], t);
        nv[a] = t;
      }
#pragma unroll
      for (int a = 0; a < R; ++a) V[a] = nv[a];
    }
  }
}

// Output o of the chain pass: core k, slice x, entry e (e < R^2: gradient
// (a, b) = (e / R, e % R); e = R^2: slice sum).  Outputs are core-major with
// n_k (R^2 + 1) per core, so core k starts at soff[k] (R^2 + 1).
template <typename F, int R>
__device__ __forceinline__ void chain_output(const Dev &d, long long o, int &k, int &x, int &e, int &off) {
  constexpr int RR = R * R;
  constexpr int XH = 16 / R;
  const int m = d.m, u = d.ch_u, nc = m - u;
  k = 0;
  while (k + 1 < m && (long long)d.soff[k + 1] * (RR + 1) <= o) ++k;
  const long long r = o - (long long)d.soff[k] * (RR + 1);
  x = (int)(r / (RR + 1));
  e = (int)(r % (RR + 1));
  const int NXv = chain_nx(R);
  if (k >= u) {
    const int c = k - u;
    if (e < RR) {
      const int a = e / R, b = e % R;
      off = c * 256 + ((x / XH) * R + a) * 16 + (x % XH) * R + b;
    } else {
      off = nc * 256 + c * NXv + x;
    }
  } else {
    off = nc * 256 + nc * NXv + k * RR + (e < RR ? e : 0);
  }
}

constexpr int CHAIN_GROUP = 32;   // chunks summed per thread in the first reduction

// First reduction: output o, chunk group g (CHAIN_GROUP consecutive chunks).
template <typename F, int R>
__global__ void __launch_bounds__(256) k_chain_reduce1(const Dev *__restrict__ dt, int diag) {
  const Dev &d = dt[blockIdx.y];
  constexpr int RR = R * R;
  const long long nout = (long long)d.soff[d.m] * (RR + 1);
  const long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int g = blockIdx.z;
  const int c0 = g * CHAIN_GROUP;
  if (o >= nout || c0 >= d.ch_nchunks || (!diag && d.st->done)) return;
  const int c1 = min(d.ch_nchunks, c0 + CHAIN_GROUP);
  int k, x, e, off;
  chain_output<F, R>(d, o, k, x, e, off);
  const int W = chain_part_width(d.m, d.ch_u, R);
  const auto part = glb((const F *)d.ch_part);
  // eight loads in flight per step; a shared core's output takes a chunk's
  // value only where the chunk's prefix index x_k equals the output's slice
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const bool shared = k < d.ch_u;
  const auto cxs = glb(d.ch_x);
  const auto rsqc = glb(d.ch_rsq);
  int c = c0;
  for (; c + 8 <= c1; c += 8) {
    double v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t)
      v[t] = (shared && e == RR) ? rsqc[c + t] : (double)part[(long long)(c + t) * W + off];
    if (shared) {
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (cxs[(long long)(c + t) * d.ch_u + k] != x) v[t] = 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) a[t] += v[t];
  }
  for (; c < c1; ++c) {
    double v = (shared && e == RR) ? rsqc[c] : (double)part[(long long)c * W + off];
    if (shared && cxs[(long long)c * d.ch_u + k] != x) v = 0.0;
    a[c & 7] += v;
  }
  glb(d.ch_red)[(long long)g * nout + o] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// Second reduction: the group sums of output o into the gradient or the slice sums.
template <typename F, int R>
__global__ void __launch_bounds__(256) k_chain_reduce2(const Dev *__restrict__ dt, int diag) {
  const Dev &d = dt[blockIdx.y];
  constexpr int RR = R * R;
  const long long nout = (long long)d.soff[d.m] * (RR + 1);
  const long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nout || (!diag && d.st->done)) return;
  const int ng = (d.ch_nchunks + CHAIN_GROUP - 1) / CHAIN_GROUP;
  const auto red = glb(d.ch_red);
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  int g = 0;
  for (; g + 4 <= ng; g += 4) {
#pragma unroll
    for (int t = 0; t < 4; ++t) a[t] += red[(long long)(g + t) * nout + o];
  }
  for (; g < ng; ++g) a[0] += red[(long long)g * nout + o];
  const double v = (a[0] + a[1]) + (a[2] + a[3]);
  int k, x, e, off;
  chain_output<F, R>(d, o, k, x, e, off);
  if (e < RR) glb((F *)d.Y)[d.coff[k] + (long long)x * RR + e] = (F)v;
  else glb((F *)d.s)[d.soff[k] + x] = (F)v;
}

hipError_t launch_sampled_fin(const Batch &bt, int diag, hipStream_t s);

// Waves per workgroup: eight for float64 at R = 8 (two per SIMD; the
// parking slots per wave are then cut to what fits, see chain_wave_slots),
// four otherwise (their full slots already leave two workgroups per CU).
int chain_waves(int R, int prec) { return (prec != PREC_MIXED && R == 8) ? 8 : 4; }

// dynamic LDS of one solve with at most nsl parking slots per wave
static size_t chain_bytes_at(int m, int u, const int *n, int R, int prec, int nsl) {
  const size_t f = prec == PREC_MIXED ? 4 : 8;
  const int nc = m - u, nw = chain_waves(R, prec);
  size_t cores = 0;
  for (int k = u; k < m; ++k) cores += (size_t)n[k] * chain_slice_stride(R, (int)f);
  const int nfull = chain_nslots(nc);
  // as in the kernel: four-wave launches always park every interface
  const int ns = nw > 4 ? std::min(nfull, std::max(nsl, 2)) : nfull;
  const int wr = nc * (256 + chain_nx(R));
  const size_t region = (size_t)chain_region(ns, nfull, wr, chain_slot_width(R));
  const size_t wss = (size_t)nc * chain_nx(R);
  const size_t prefix = (size_t)u * R;   // the chunk's prefix interfaces
  return (cores + nw * region + nw * wss + R + prefix) * f;
}

constexpr size_t CHAIN_LDS_BUDGET = (size_t)159 * 1024;

// Parking slots per wave: all (one per generic core) when they fit in LDS;
// with eight waves otherwise the most that fit, at least 2 (the later cores'
// interfaces are then recomputed by a second right sweep).
int chain_wave_slots(int m, int u, const int *n, int R, int prec) {
  const int nfull = chain_nslots(m - u);
  if (chain_waves(R, prec) == 4) return nfull;
  for (int s = nfull; s > 2; --s)
    if (chain_bytes_at(m, u, n, R, prec, s) <= CHAIN_LDS_BUDGET) return s;
  return std::min(nfull, 2);
}

size_t chain_lds_bytes(int m, int u, const int *n, int R, int prec) {
  return chain_bytes_at(m, u, n, R, prec, chain_wave_slots(m, u, n, R, prec));
}

int chain_maxc(int nc) { return nc <= 4 ? 4 : (nc <= 8 ? 8 : (nc <= 10 ? 10 : (nc <= 12 ? 12 : 16))); }

template <typename F, int R, int MAXC>
static hipError_t launch_chain_c(const Batch &bt, int diag, hipStream_t st, hipEvent_t after_main) {
  constexpr int NW = (sizeof(F) == 8 && R == 8) ? 8 : 4;
  if (chain_waves(R, bt.host[0].prec) != NW) return hipErrorInvalidValue;
  int g = 1;
  size_t lds = 0;
  long long nout = 1;
  int ng = 1;
  int nsl = 1 << 20;   // parking slots per wave, common to the solves of the launch
  for (int i = 0; i < bt.ns; ++i) {
    const Dev &h = bt.host[i];
    nsl = std::min(nsl, chain_wave_slots(h.m, h.ch_u, h.n, R, h.prec));
  }
  for (int i = 0; i < bt.ns; ++i) {
    const Dev &h = bt.host[i];
    g = std::max(g, h.ch_nchunks);
    lds = std::max(lds, chain_bytes_at(h.m, h.ch_u, h.n, R, h.prec, nsl));
    nout = std::max<long long>(nout, (long long)h.soff[h.m] * (R * R + 1));
    ng = std::max(ng, (h.ch_nchunks + CHAIN_GROUP - 1) / CHAIN_GROUP);
  }
  if (lds > CHAIN_LDS_BUDGET) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_chain<F, R, MAXC, NW>), dim3(g, bt.ns), dim3(NW * 64), lds, st, bt.dt, diag, nsl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (after_main && (e = hipEventRecord(after_main, st)) != hipSuccess) return e;
  const int nb = (int)((nout + 255) / 256);
  hipLaunchKernelGGL((k_chain_reduce1<F, R>), dim3(nb, bt.ns, ng), dim3(256), 0, st, bt.dt, diag);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((k_chain_reduce2<F, R>), dim3(nb, bt.ns), dim3(256), 0, st, bt.dt, diag);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return launch_sampled_fin(bt, diag, st);
}

template <typename F, int R>
static hipError_t launch_chain_r(const Batch &bt, int diag, hipStream_t st, hipEvent_t ev) {
  int nc = 1;
  for (int i = 0; i < bt.ns; ++i) nc = std::max(nc, bt.host[i].m - bt.host[i].ch_u);
  switch (chain_maxc(nc)) {
    case 4: return launch_chain_c<F, R, 4>(bt, diag, st, ev);
    case 8: return launch_chain_c<F, R, 8>(bt, diag, st, ev);
    case 10: return launch_chain_c<F, R, 10>(bt, diag, st, ev);
    case 12: return launch_chain_c<F, R, 12>(bt, diag, st, ev);
    default: return launch_chain_c<F, R, 16>(bt, diag, st, ev);
  }
}

template <typename F>
static hipError_t launch_chain_f(const Batch &bt, int diag, hipStream_t st, hipEvent_t ev) {
  switch (bt.host[0].R) {
    case 2: return launch_chain_r<F, 2>(bt, diag, st, ev);
    case 4: return launch_chain_r<F, 4>(bt, diag, st, ev);
    case 8: return launch_chain_r<F, 8>(bt, diag, st, ev);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sampled_chain(const Batch &bt, int diag, hipStream_t st, hipEvent_t after_main) {
  if (bt.host[0].prec == PREC_MIXED) return launch_chain_f<float>(bt, diag, st, after_main);
  return launch_chain_f<double>(bt, diag, st, after_main);
}

}  // namespace prgd
