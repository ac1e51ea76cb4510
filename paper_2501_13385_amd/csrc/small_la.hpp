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

// Pivoted Cholesky of a symmetric positive semidefinite n x n matrix A (ld n,
// destroyed): F (ld n) gets columns 0..rank-1 with F F^T = A up to pivots
// below n * 2.3e-16 * max diag.  Returns the rank.
__device__ inline int block_pivoted_cholesky(double *A, int n, double *F) {
  __shared__ int piv, rank, stop;
  __shared__ double pvs, tol;
  __shared__ unsigned used;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int e = t; e < n * n; e += nt) F[e] = 0.0;
  if (t < 64) {
    double dm = 0.0;
    for (int i = t; i < n; i += 64) dm = fmax(dm, A[i * n + i]);
    dm = wave_max(dm);
    if (t == 0) {
      tol = (double)n * 2.3e-16 * dm;
      rank = 0;
      used = 0u;
    }
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (t < 64) {
      const unsigned u = used;
      double best = -1.0;
      int bi = 64;
      if (t < n && !((u >> t) & 1u)) {
        best = A[t * n + t];
        bi = t;
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (t == 0) {
        stop = (bi >= n || !(best > tol)) ? 1 : 0;
        if (!stop) {
          piv = bi;
          pvs = sqrt(best);
          used = u | (1u << bi);
          rank = k + 1;
        }
      }
    }
    __syncthreads();
    if (stop) break;
    const int p = piv;
    const double pv = pvs;
    const unsigned u = used;
    for (int i = t; i < n; i += nt) F[i * n + k] = (((u >> i) & 1u) && i != p) ? 0.0 : A[i * n + p] / pv;
    __syncthreads();
    for (int e = t; e < n * n; e += nt) {
      const int i = e / n, j = e % n;
      A[e] -= F[i * n + k] * F[j * n + k];
    }
    __syncthreads();
  }
  __syncthreads();
  return rank;
}

// Cyclic Jacobi for a symmetric n x n matrix A (ld n, destroyed), n <= 32.
// Round-robin ordering: each round applies n/2 disjoint rotations; the
// two-sided update J^T A J is done per 2 x 2 block (one thread per block), so a
// round is one parameter phase and one update phase.  On exit w[0..n) holds
// the eigenvalues in descending order and V (ld n) the eigenvectors as columns.
// cs: 4 * 16 doubles; Vs: n n scratch.
__device__ inline void block_jacobi_eig(double *A, int n, double *V, double *w, double *Vs, double *cs) {
  __shared__ double sbuf[16];
  __shared__ int goon;
  const int t = threadIdx.x, nt = blockDim.x;
  const int ne = n + (n & 1);
  const int np = ne / 2;
  for (int e = t; e < n * n; e += nt) V[e] = (e / n == e % n) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = t; e < n * n; e += nt) {
      const double v = A[e];
      if (e / n == e % n) dia += v * v;
      else off += v * v;
    }
    off = block_sum(off, sbuf);
    dia = block_sum(dia, sbuf);
    if (t == 0) goon = (off > 1e-32 * (dia + off)) ? 1 : 0;
    __syncthreads();
    if (!goon) break;
    for (int rd = 0; rd < ne - 1; ++rd) {
      if (t < np) {
        int p, q;
        if (t == 0) {
          p = ne - 1;
          q = rd;
        } else {
          p = (rd + t) % (ne - 1);
          q = (rd - t + ne - 1) % (ne - 1);
        }
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * n + q];
          if (apq != 0.0) {
            const double tau = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        cs[4 * t + 0] = c;
        cs[4 * t + 1] = s;
        cs[4 * t + 2] = (double)p;
        cs[4 * t + 3] = (double)q;
      }
      __syncthreads();
      // 2 x 2 block (P, Q) of A: rows {p_P, q_P}, columns {p_Q, q_Q}; then the
      // rows of V (columns p, q of each pair)
      for (int it = t; it < np * np + n * np; it += nt) {
        if (it < np * np) {
          const int P = it / np, Q = it % np;
          const int i1 = (int)cs[4 * P + 2], i2 = (int)cs[4 * P + 3];
          const int j1 = (int)cs[4 * Q + 2], j2 = (int)cs[4 * Q + 3];
          const double cP = cs[4 * P], sP = cs[4 * P + 1], cQ = cs[4 * Q], sQ = cs[4 * Q + 1];
          const bool r2 = i2 < n, c2 = j2 < n;
          const double a11 = A[i1 * n + j1];
          const double a12 = c2 ? A[i1 * n + j2] : 0.0;
          const double a21 = r2 ? A[i2 * n + j1] : 0.0;
          const double a22 = (r2 && c2) ? A[i2 * n + j2] : 0.0;
          // M = A J_Q
          const double m11 = cQ * a11 - sQ * a12, m12 = sQ * a11 + cQ * a12;
          const double m21 = cQ * a21 - sQ * a22, m22 = sQ * a21 + cQ * a22;
          // J_P^T M
          A[i1 * n + j1] = cP * m11 - sP * m21;
          if (c2) A[i1 * n + j2] = cP * m12 - sP * m22;
          if (r2) A[i2 * n + j1] = sP * m11 + cP * m21;
          if (r2 && c2) A[i2 * n + j2] = sP * m12 + cP * m22;
        } else {
          const int e = it - np * np;
          const int i = e / np, Q = e % np;
          const int p = (int)cs[4 * Q + 2], q = (int)cs[4 * Q + 3];
          if (q < n) {
            const double c = cs[4 * Q], s = cs[4 * Q + 1];
            const double vp = V[i * n + p], vq = V[i * n + q];
            V[i * n + p] = c * vp - s * vq;
            V[i * n + q] = s * vp + c * vq;
          }
        }
      }
      __syncthreads();
    }
  }
  // sort descending (stable by index)
  for (int i = t; i < n; i += nt) {
    const double wi = A[i * n + i];
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double wj = A[j * n + j];
      if (wj > wi || (wj == wi && j < i)) ++rk;
    }
    w[rk] = wi;
    for (int r = 0; r < n; ++r) Vs[r * n + rk] = V[r * n + i];
  }
  __syncthreads();
  for (int e = t; e < n * n; e += nt) V[e] = Vs[e];
  __syncthreads();
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
  double *buf[2] = {scratch, scratch + tot};
  for (int e = t; e < tot; e += nt) {
    double v;
    if (e < s1) {
      const int i = e / w1, j = e % w1;
      v = (j < n1) ? A1[i * lda1 + j] : (j - n1 == i ? 1.0 : 0.0);
    } else {
      const int f = e - s1, i = f / w2, j = f % w2;
      v = (j < n2) ? A2[i * lda2 + j] : (j - n2 == i ? 1.0 : 0.0);
    }
    buf[0][e] = v;
  }
  if (t == 0) bad = 0;
  __syncthreads();
  const int nmax = n1 > n2 ? n1 : n2;
  int cur = 0;
  for (int k = 0; k < nmax; ++k) {
    const double *M = buf[cur];
    double *Mn = buf[cur ^ 1];
    for (int e = t; e < tot; e += nt) {
      const bool first = e < s1;
      const int w = first ? w1 : w2, n = first ? n1 : n2, base = first ? 0 : s1;
      const int f = e - base, i = f / w, j = f % w;
      if (k >= n) {
        Mn[e] = M[e];
        continue;
      }
      const double pk = M[base + k * w + k];
      const double pj = M[base + k * w + j];
      if (i == k) {
        Mn[e] = pj / pk;
      } else {
        const double fi = M[base + i * w + k];
        Mn[e] = M[e] - fi * (pj / pk);
      }
      if (j == k && i == k && (!(pk > 0.0) || !isfinite(pk))) bad = 1;
    }
    __syncthreads();
    cur ^= 1;
  }
  const double *M = buf[cur];
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
