// Small dense linear algebra (n <= 32) on LDS, run by a whole workgroup.
//
// These are chains of many tiny dependent steps, so each routine is arranged
// so that every thread handles at most one item per phase (no thread
// serialises several dependent LDS accesses) and the number of barriers per
// step is minimal.  Matrices are dense row-major in LDS.  Every routine must
// be called by all threads of the block and ends with a barrier.
#pragma once

#include <hip/hip_runtime.h>

#include "block_ops.hpp"

namespace prgd {

// 1/x and 1/sqrt(x) for finite x > 0 (normal range): the hardware estimates,
// good to about 23 bits, refined by `steps` Newton steps (each doubles the
// number of correct bits, so two reach double precision).
template <int steps>
__device__ __forceinline__ double rcp_newton(double x) {
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int k = 0; k < steps; ++k) y = fma(y, fma(-x, y, 1.0), y);
  return y;
}
template <int steps>
__device__ __forceinline__ double rsq_newton(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
#pragma unroll
  for (int k = 0; k < steps; ++k) y = fma(y, fma(-h * y, y, 0.5), y);
  return y;
}

// Ordering of LDS accesses among the lanes of one wave.  A wave's LDS
// operations are performed in issue order, so it suffices to keep the compiler
// from moving memory operations across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// one DPP exchange of a 64-bit value (both halves moved with the same pattern)
template <int ctrl>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long k) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)k, ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(k >> 32), ctrl, 0xF, 0xF, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

// value of lane l ^ 16 in lane l (the rows of 16 swapped pairwise), by
// v_permlane16_swap instead of a trip through LDS; whole wave active
__device__ __forceinline__ unsigned long long xor16_u64(unsigned long long k) {
  const int lo = (int)(unsigned)k, hi = (int)(unsigned)(k >> 32);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  // a[0] holds rows (0, 0, 2, 2) and a[1] rows (1, 1, 3, 3) of the input
  const bool odd = (threadIdx.x >> 4) & 1;
  const unsigned l = (unsigned)(odd ? a[0] : a[1]), h = (unsigned)(odd ? b[0] : b[1]);
  return ((unsigned long long)h << 32) | l;
}

// value of lane (l & 31) + 32 upper in lane l, by v_permlane32_swap; whole
// wave active
__device__ __forceinline__ double half_value(double v, bool upper) {
  const long long b = __double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane32_swap((int)b, (int)b, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((int)(b >> 32), (int)(b >> 32), false, false);
  // [0] holds the lower half's values in both halves, [1] the upper half's
  const unsigned l = (unsigned)(upper ? lo[1] : lo[0]), h = (unsigned)(upper ? hi[1] : hi[0]);
  return __longlong_as_double((long long)(((unsigned long long)h << 32) | l));
}

// value of v in lane c (c wave-uniform)
__device__ __forceinline__ double lane_value(double v, int c) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, c), hi = __builtin_amdgcn_readlane((int)(b >> 32), c);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// max of a 64-bit key over each group of 32 lanes (the two halves of the wave
// reduce separately): DPP exchanges inside rows of 16 lanes, then one swap of
// the rows.  Keys are compared as unsigned integers.  Whole wave active.
__device__ __forceinline__ unsigned long long key_max32(unsigned long long k) {
  unsigned long long o;
  o = dpp_u64<0xB1>(k);   // quad_perm [1,0,3,2]: lane ^ 1
  k = o > k ? o : k;
  o = dpp_u64<0x4E>(k);   // quad_perm [2,3,0,1]: lane ^ 2
  k = o > k ? o : k;
  o = dpp_u64<0x141>(k);  // row_half_mirror: lane i <-> 7 - i within 8
  k = o > k ? o : k;
  o = dpp_u64<0x140>(k);  // row_mirror: lane i <-> 15 - i within 16
  k = o > k ? o : k;
  o = xor16_u64(k);
  return o > k ? o : k;
}

// max of a 32-bit key over each group of 32 lanes: DPP exchanges inside rows
// of 16 lanes (each folded by the compiler into a v_max_u32 with a DPP source)
// and one swap of the rows.  Whole wave active.
__device__ __forceinline__ unsigned key_max32_u32(unsigned k) {
  k = max(k, (unsigned)__builtin_amdgcn_mov_dpp((int)k, 0xB1, 0xF, 0xF, false));   // lane ^ 1
  k = max(k, (unsigned)__builtin_amdgcn_mov_dpp((int)k, 0x4E, 0xF, 0xF, false));   // lane ^ 2
  k = max(k, (unsigned)__builtin_amdgcn_mov_dpp((int)k, 0x141, 0xF, 0xF, false));  // i <-> 7 - i in 8
  k = max(k, (unsigned)__builtin_amdgcn_mov_dpp((int)k, 0x140, 0xF, 0xF, false));  // i <-> 15 - i in 16
  const auto sw = __builtin_amdgcn_permlane16_swap(k, k, false, false);
  // [0] holds rows (0, 0, 2, 2) and [1] rows (1, 1, 3, 3) of the input
  const bool odd = (threadIdx.x >> 4) & 1;
  const unsigned o = odd ? (unsigned)sw[0] : (unsigned)sw[1];
  return max(k, o);
}

// Pivoted Cholesky of a symmetric positive semidefinite n x n matrix A (ld n,
// n <= 32, read only): F (ld n) gets columns 0..rank-1 with F F^T = A up to
// pivots below n * 2.3e-16 * max diag.  Returns the rank (in every thread).
//
// Run by the first wave alone, with no workgroup barrier per step: lane l
// holds half of row l & 31 of the working matrix in registers (columns
// 16 (l >> 5) .. + 15) and that row's diagonal entry.  The pivot (largest
// remaining diagonal entry) is found with a key holding the entry's bits
// (the high word of a non-negative double is monotone in its value) with its
// low 5 bits replaced by 31 - row, so among entries equal to 15 mantissa bits
// the smallest row wins (any such pivot is as good for the factorisation);
// its exact value is then read from the owning lane.
__device__ inline int block_pivoted_cholesky(const double *A, int n, double *F) {
  __shared__ double fcol[32];
  __shared__ int rank_s;
  const int t = threadIdx.x;
  if (t < 64) {
    const int i = t & 31, h = t >> 5;
    for (int e = t; e < n * n; e += 64) F[e] = 0.0;
    double a[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int j = 16 * h + c;
      a[c] = (i < n && j < n) ? A[i * n + j] : 0.0;
    }
    double dg = i < n ? A[i * n + i] : 0.0;
    double dm = dg;
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) dm = fmax(dm, __shfl_xor(dm, o, 64));
    const double tol = (double)n * 2.3e-16 * dm;
    bool avail = i < n;  // row not yet a pivot
    int rank = 0;
    for (int k = 0; k < n; ++k) {
      const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(fmax(dg, 0.0)) >> 32);
      const unsigned key = avail ? ((hi & ~31u) | (unsigned)(31 - i)) : 0u;
      const unsigned kmax = __builtin_amdgcn_readfirstlane(key_max32_u32(key));
      const int p = 31 - (int)(kmax & 31u);
      const double best = lane_value(dg, p);
      if (kmax == 0u || !(best > tol)) break;
      rank = k + 1;
      const double rs = rsq_newton<2>(best);  // 1 / sqrt(pivot)
      // this row's entry in column p, from the lane holding that column (the
      // register index is wave-uniform)
      const double x = half_value(a[p & 15], p >= 16);
      const double f = (i == p || avail) && i < n ? x * rs : 0.0;
      if (i == p) avail = false;
      dg = fma(-f, f, dg);
      wave_lds_sync();  // every lane has read fcol of the last step
      if (h == 0) {
        fcol[i] = f;
        if (i < n) F[i * n + k] = f;
      }
      wave_lds_sync();
#pragma unroll
      for (int c = 0; c < 16; ++c) a[c] = fma(-f, fcol[16 * h + c], a[c]);
    }
    if (t == 0) rank_s = rank;
  }
  __syncthreads();
  return rank_s;
}

// Slot of the round-robin ordering that the element in slot s moves to after
// a round (np pairs, pair P = slots (2P, 2P+1)).  Slots 2k form the top row
// and 2k+1 the bottom row of the usual tournament table; slot 0 stays, the
// other elements move one place around the table (top row to the right,
// bottom row to the left).  Every two of the 2 np elements share a pair in
// exactly one of 2 np - 1 consecutive rounds, after which all are back in
// their starting slots.
__device__ __forceinline__ int tournament_next(int s, int np) {
  if (np == 1 || s == 0) return s;
  const int k = s >> 1;
  if ((s & 1) == 0) return k == np - 1 ? s + 1 : s + 2;
  return k == 0 ? 2 : s - 2;
}

// Rotation (c, s) that zeroes the (p, q) entry of a symmetric matrix under
// J^T A J, J = [[c, s], [-s, c]] on rows/columns (p, q): t = tan(theta) is the
// root of smaller magnitude of t^2 + 2 tau t - 1 = 0, tau = (a_qq - a_pp) /
// (2 a_pq), written as t = sign(d) 2 a_pq / (|d| + sqrt(d^2 + 4 a_pq^2)) with
// d = a_qq - a_pp.  The angle only has to be accurate enough for fast
// convergence (an angle off by a relative delta leaves about delta a_pq for a
// later sweep), so t comes from the hardware estimates of 1/x and 1/sqrt(x) as
// they are; c = 1/sqrt(1+t^2) is refined to full precision so that
// c^2 + s^2 = 1 to rounding and the accumulated eigenvectors stay orthonormal.
// Entries |a_pq| <= 1e-150 are treated as zero, and so are pairs whose
// diagonal difference reaches 1e150 (the squares stay in range).
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq, double &c, double &s) {
  const double d = aqq - app, ad = fabs(d), e2 = apq + apq;
  const bool rot = fabs(apq) > 1e-150 && ad < 1e150;
  const double r2 = fma(d, d, e2 * e2);
  const double t0 = e2 * __builtin_amdgcn_rcp(fma(r2, __builtin_amdgcn_rsq(r2), ad));
  const double t = d < 0.0 ? -t0 : t0;
  const double cr = rsq_newton<2>(fma(t, t, 1.0));
  c = rot ? cr : 1.0;
  s = rot ? t * cr : 0.0;
}

// one DPP exchange of a double (both halves moved with the same pattern)
template <int ctrl>
__device__ __forceinline__ double dpp_f64(double v) {
  return __builtin_bit_cast(double, (long long)dpp_u64<ctrl>((unsigned long long)__builtin_bit_cast(long long, v)));
}

// Sums of a and b over the block, the same value in every thread (fixed
// order).  Every thread of the block must call it.  sb: 32 doubles.
__device__ inline void block_sum2(double &a, double &b, double *sb) {
  // rows of 16 lanes by DPP (the same total in every lane of a row)
  a += dpp_f64<0xB1>(a);
  b += dpp_f64<0xB1>(b);
  a += dpp_f64<0x4E>(a);
  b += dpp_f64<0x4E>(b);
  a += dpp_f64<0x141>(a);
  b += dpp_f64<0x141>(b);
  a += dpp_f64<0x140>(a);
  b += dpp_f64<0x140>(b);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  double sa = 0.0, sbv = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    sa += __shfl(a, 16 * r, 64);
    sbv += __shfl(b, 16 * r, 64);
  }
  if (lane == 0) {
    sb[w] = sa;
    sb[16 + w] = sbv;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
  for (int k = 0; k < nw; ++k) {
    a += sb[k];
    b += sb[16 + k];
  }
}

// Sum of v over the wave, the same value in every lane: DPP rows of 16 (each
// lane of a row ends with the same row total: every step adds a pair of
// equal-order partial sums), then the four row totals read in a fixed order.
__device__ __forceinline__ double wave_sum_uniform(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// The sweeps of the cyclic Jacobi method on the padded ne x ne matrix in W1
// (eigenvector accumulator in A, identity on entry); returns true when the
// result sits in (W2, V) rather than (W1, A).  WAVE: run by the first wave
// alone (ne <= 16, so the np^2 <= 64 working threads are one wave): the
// rounds are then ordered by the wave's in-order LDS accesses instead of
// workgroup barriers, and the stopping sums are wave reductions.  off and dia
// hold the initial off-diagonal and diagonal masses on entry.
template <bool WAVE>
__device__ __forceinline__ bool jacobi_sweeps(double *W1, double *W2, double *A, double *V, int ne, double off,
                                              double dia, double *sb) {
  const int t = threadIdx.x;
  const int np = ne / 2, m1 = ne - 1;
  const bool act = t < np * np;
  const int P = act ? t / np : 0, Q = act ? t - P * np : 0;
  // this thread's fixed addresses: the reads at rows/columns 2P, 2P+1 and
  // 2Q, 2Q+1, the writes at the slots those rows and columns move to
  const int r1 = 2 * P * ne, r2 = r1 + ne, c1 = 2 * Q, c2 = c1 + 1;
  const int p1 = 2 * P * (ne + 1), q1 = 2 * Q * (ne + 1);
  const int nr1 = tournament_next(2 * P, np) * ne, nr2 = tournament_next(2 * P + 1, np) * ne;
  const int nc1 = tournament_next(c1, np), nc2 = tournament_next(c2, np);
  // one round from buffers (src, vsrc) into (dst, vdst); instantiated once per
  // direction so that every address is a fixed offset from a fixed buffer
  auto one_round = [&](const double *src, double *dst, const double *vsrc, double *vdst, bool last) {
    if (act) {
      const double p11 = src[p1], p12 = src[p1 + 1], p22 = src[p1 + ne + 1];
      const double q11 = src[q1], q12 = src[q1 + 1], q22 = src[q1 + ne + 1];
      const double a11 = src[r1 + c1], a12 = src[r1 + c2];
      const double a21 = src[r2 + c1], a22 = src[r2 + c2];
      const double v11 = vsrc[r1 + c1], v12 = vsrc[r1 + c2];
      const double v21 = vsrc[r2 + c1], v22 = vsrc[r2 + c2];
      double cP, sP, cQ, sQ;
      jacobi_rotation(p11, p22, p12, cP, sP);
      jacobi_rotation(q11, q22, q12, cQ, sQ);
      // M = A J_Q, then J_P^T M
      const double m11 = cQ * a11 - sQ * a12, m12 = sQ * a11 + cQ * a12;
      const double m21 = cQ * a21 - sQ * a22, m22 = sQ * a21 + cQ * a22;
      const double b11 = cP * m11 - sP * m21, b12 = cP * m12 - sP * m22;
      const double b21 = sP * m11 + cP * m21, b22 = sP * m12 + cP * m22;
      dst[nr1 + nc1] = b11;
      dst[nr1 + nc2] = b12;
      dst[nr2 + nc1] = b21;
      dst[nr2 + nc2] = b22;
      // V J_Q on rows 2P, 2P+1 (V's rows stay; its columns move with A's)
      vdst[r1 + nc1] = cQ * v11 - sQ * v12;
      vdst[r1 + nc2] = sQ * v11 + cQ * v12;
      vdst[r2 + nc1] = cQ * v21 - sQ * v22;
      vdst[r2 + nc2] = sQ * v21 + cQ * v22;
      if (last) {
        if (P == Q) {  // b11, b22 on the diagonal
          dia += b11 * b11 + b22 * b22;
          off += b12 * b12 + b21 * b21;
        } else {
          off += b11 * b11 + b12 * b12 + b21 * b21 + b22 * b22;
        }
      }
    }
    if constexpr (WAVE) wave_lds_sync();
    else __syncthreads();
  };
  double prev = 0.0;  // off-diagonal mass before the last sweep
  bool flip = false;  // data in (W2, V) rather than (W1, A)
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (!(off > 1e-30 * (dia + off)) || (sweep > 0 && off >= prev)) break;
    prev = off;
    off = 0.0;
    dia = 0.0;
    for (int rd = 0; rd < m1; ++rd) {
      const bool last = rd == m1 - 1;
      if (flip) one_round(W2, W1, V, A, last);
      else one_round(W1, W2, A, V, last);
      flip = !flip;
    }
    if constexpr (WAVE) {
      off = wave_sum_uniform(off);
      dia = wave_sum_uniform(dia);
    } else {
      block_sum2(off, dia, sb);
    }
  }
  return flip;
}

// Cyclic Jacobi for a symmetric n x n matrix A (ld n, n <= 32), run by a whole
// block of at least 256 threads.  The matrix and the eigenvector matrix are
// held padded to ne = n + (n & 1) (a zero row and column, on which every
// rotation is exactly the identity) with ld ne.  Pairs sit in fixed slots
// (2P, 2P+1), and the round-robin ordering moves the data instead: each round
// writes the rotated matrix into the other buffer with rows and columns
// already moved to their next slots (and V's columns likewise), so every
// thread reads and writes the same addresses in every round and no index is
// computed inside the loop; after a sweep of ne - 1 rounds all slots are back
// in place.  Thread (P, Q), P, Q < ne/2, owns the 2 x 2 block (P, Q) of A and
// the 2 x 2 block of V with rows 2P, 2P+1 and columns in pair Q; it computes
// the two rotations it needs itself from the previous state.  For ne <= 16
// those threads are the first wave, which runs the sweeps alone with no
// workgroup barrier; larger matrices take one barrier per round.  The
// off-diagonal mass for the stopping rule is summed from the entries written
// in a sweep's last round.  Sweeps stop once the off-diagonal Frobenius norm
// is at most 1e-15 of the whole (a converged sweep leaves rounding residue
// near 3e-16 of it, so a tighter bound would never be met), or once a sweep
// fails to shrink it (exact rotations always do, so only rounding is left).
// On exit w[0..n) holds the eigenvalues in descending order and V (ld n) the
// eigenvectors as columns.  A is read first and its area (1024 doubles) then
// reused, as is V's; W1, W2: scratch of ne * ne doubles each.
__device__ inline void block_jacobi_eig(double *A, int n, double *V, double *w, double *W1, double *W2) {
  __shared__ double sb[32];
  __shared__ int flip_s;
  const int t = threadIdx.x, nt = blockDim.x;
  const int ne = n + (n & 1);
  double off = 0.0, dia = 0.0;
  for (int e = t; e < ne * ne; e += nt) {
    const int i = e / ne, j = e - i * ne;
    const double v = (i < n && j < n) ? A[i * n + j] : 0.0;
    W1[e] = v;
    if (i == j) dia += v * v;
    else off += v * v;
  }
  block_sum2(off, dia, sb);  // ends with a barrier: A has been read
  for (int e = t; e < ne * ne; e += nt) A[e] = (e / ne == e % ne) ? 1.0 : 0.0;
  __syncthreads();
  bool flip;
  if (ne <= 16) {
    if (t < 64) {
      const bool f = jacobi_sweeps<true>(W1, W2, A, V, ne, off, dia, sb);
      if (t == 0) flip_s = f ? 1 : 0;
    }
    __syncthreads();
    flip = flip_s != 0;
  } else {
    flip = jacobi_sweeps<false>(W1, W2, A, V, ne, off, dia, sb);
  }
  const double *cur = flip ? W2 : W1;
  double *nxt = flip ? W1 : W2;
  const double *vc = flip ? V : A;
  // the eigenvectors now sit in vc, in slot order (= original order); if that
  // is V's own area, move them out of the way first
  if (vc == V) {
    for (int e = t; e < ne * ne; e += nt) nxt[e] = vc[e];
    __syncthreads();
    vc = nxt;
  }
  // sort descending (stable by index): ranks first, then every entry of V
  __shared__ int rank_of[32];
  for (int i = t; i < n; i += nt) {
    const double wi = cur[i * ne + i];
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double wj = cur[j * ne + j];
      if (wj > wi || (wj == wi && j < i)) ++rk;
    }
    w[rk] = wi;
    rank_of[i] = rk;
  }
  __syncthreads();
  for (int e = t; e < n * n; e += nt) {
    const int rr = e / n, i = e - rr * n;
    V[rr * n + rank_of[i]] = vc[rr * ne + i];
  }
  __syncthreads();
}

// Eigen-decomposition of a symmetric positive semidefinite n x n matrix S
// (ld n, n <= 32, read only) through its pivoted Cholesky factor: S = Fc Fc^T
// (Fc: n x rank), S1 = Fc^T Fc has the same nonzero eigenvalues, and with
// S1 = W diag(w) W^T the eigenvectors of S are Fc W diag(w)^{-1/2}.  The
// pivoted factor grades S1 (large entries first, small couplings), so the
// Jacobi sweeps on S1 converge in about half as many sweeps as on S itself;
// see Demmel and Veselic (1992) on Jacobi for graded positive definite
// matrices.  On exit w[0..n) holds the eigenvalues in descending order (zeros
// past the rank) and V (ld n) the eigenvectors of the nonzero ones as columns
// (zero columns past the rank).  Returns the rank.  Fc, S1, W, W1, W2: LDS
// scratch, 1024 doubles each.  V may share S1's area and W1 may share S's
// (each is dead by the time the other is written); no other two may alias.
__device__ inline int block_psd_eig(const double *S, int n, double *V, double *w, double *Fc, double *S1, double *W,
                                    double *W1, double *W2) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int rank = block_pivoted_cholesky(S, n, Fc);   // ends with a barrier
  // S1 = Fc^T Fc, each entry of the upper triangle formed once and mirrored
  for (int e = t; e < rank * rank; e += nt) {
    const int a = e / rank, b = e - a * rank;
    if (a > b) continue;
    double v = 0.0;
    for (int i = 0; i < n; ++i) v = fma(Fc[i * n + a], Fc[i * n + b], v);
    S1[a * rank + b] = v;
    S1[b * rank + a] = v;
  }
  __syncthreads();
  if (rank > 0) block_jacobi_eig(S1, rank, W, w, W1, W2);
  for (int e = t; e < n * n; e += nt) {
    const int i = e / n, col = e - i * n;
    double v = 0.0;
    if (col < rank && w[col] > 0.0) {
      for (int j = 0; j < rank; ++j) v = fma(Fc[i * n + j], W[j * rank + col], v);
      v *= rsq_newton<2>(w[col]);
    }
    V[e] = v;
  }
  __syncthreads();
  for (int i = rank + t; i < n; i += nt) w[i] = 0.0;
  __syncthreads();
  return rank;
}

// Inverses of two SPD matrices by Gauss-Jordan elimination on [A | I] (no
// pivoting needed for SPD), the two eliminations advancing in lockstep.  The
// working matrices are double-buffered: every step reads the previous state
// from one LDS buffer and writes the next to the other, so a step costs one
// barrier: A1 (n1 x n1, ld lda1) -> O1, A2 (n2 x n2, ld lda2) -> O2, each
// written with ld ldo and zeros in the rest of its R x R block.
// scratch: 2 * 2 * (n1 * 2 n1 + n2 * 2 n2) doubles.  Returns false if a pivot
// of either matrix is not positive.
__device__ inline bool block_spd_inverse_pair(const double *A1, int lda1, int n1, double *O1, const double *A2,
                                              int lda2, int n2, double *O2, int ldo, int R, double *scratch) {
  __shared__ int bad;
  const int t = threadIdx.x, nt = blockDim.x;
  const int w1 = 2 * n1, w2 = 2 * n2, s1 = n1 * w1, s2 = n2 * w2, tot = s1 + s2;
  // the two buffers are picked with a select of LDS addresses (an array of
  // pointers indexed at run time would hide the address space and turn every
  // access into a flat one)
  double *const buf0 = scratch, *const buf1 = scratch + tot;
  // this thread's first entry (row i, column j of its matrix)
  const bool first0 = t < s1;
  const int w0 = first0 ? w1 : w2, nn0 = first0 ? n1 : n2, base0 = first0 ? 0 : s1;
  const int i0 = (t - base0) / w0, j0 = (t - base0) - i0 * w0;
  for (int e = t; e < tot; e += nt) {
    double v;
    if (e < s1) {
      const int i = e / w1, j = e % w1;
      v = (j < n1) ? A1[i * lda1 + j] : (j - n1 == i ? 1.0 : 0.0);
    } else {
      const int f = e - s1, i = f / w2, j = f % w2;
      v = (j < n2) ? A2[i * lda2 + j] : (j - n2 == i ? 1.0 : 0.0);
    }
    buf0[e] = v;
  }
  if (t == 0) bad = 0;
  __syncthreads();
  const int nmax = n1 > n2 ? n1 : n2;
  int cur = 0;
  for (int k = 0; k < nmax; ++k) {
    const double *M = cur ? buf1 : buf0;
    double *Mn = cur ? buf0 : buf1;
    for (int e = t; e < tot; e += nt) {
      bool first = first0;
      int w = w0, n = nn0, base = base0, i = i0, j = j0;
      if (e != t) {
        first = e < s1;
        w = first ? w1 : w2;
        n = first ? n1 : n2;
        base = first ? 0 : s1;
        i = (e - base) / w;
        j = (e - base) - i * w;
      }
      const int kk = k < n ? k : 0;  // keeps the loads in range when k >= n
      const double pk = M[base + kk * w + kk], pj = M[base + kk * w + j], fi = M[base + i * w + kk], me = M[e];
      const double q = pj * rcp_newton<2>(pk);
      Mn[e] = k >= n ? me : (i == k ? q : fma(-fi, q, me));
      if (k < n && j == k && i == k && (!(pk > 0.0) || !isfinite(pk))) bad = 1;
    }
    __syncthreads();
    cur ^= 1;
  }
  const double *M = cur ? buf1 : buf0;
  for (int e = t; e < 2 * R * R; e += nt) {
    const bool first = e < R * R;
    const int f = first ? e : e - R * R, i = f / R, j = f % R;
    const int n = first ? n1 : n2, w = first ? w1 : w2, base = first ? 0 : s1;
    double *O = first ? O1 : O2;
    O[i * ldo + j] = (i < n && j < n) ? 0.5 * (M[base + i * w + n + j] + M[base + j * w + n + i]) : 0.0;
  }
  __syncthreads();
  return bad == 0;
}

}  // namespace prgd
