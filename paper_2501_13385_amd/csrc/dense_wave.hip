// The dense stage in one workgroup per solve, for padded ranks R <= 8 and at
// most 16 slices per core: the weighted Gram sweep with the tangent components
// (k_gram_wave) and the retraction with the new cores and the stopping test
// (k_retract_wave).
//
// The retraction of Algorithm 1 on the rank-2r block TT W_l (see the notes at
// the top of dense.hip for C_c, GR_b, F_b, S, Tr_i and P_i) is a chain of
// 2(m-1) dependent steps on 2R x 2R matrices.  For R <= 8 every such matrix
// fits one 16 x 16 tile, so one wave runs each chain: the cores T and the
// tangent components X (or the gradient Y) are copied into LDS once, every
// product is four float64 16x16x4 MFMAs, and the state passed from step to
// step (GR_{b+1}, F_b, P_{i-1}) stays in registers or LDS, with no trip
// through global memory inside the chain.  The factorisations that the chain
// itself does not need (the Cholesky factors of the right Grams, the Gram
// inverses) run on the other waves of the workgroup in parallel; those on
// the chain (each cut's graded eigen-solve) are one-wave routines.
//
// Tiles use the row layout of tiles.hpp: A B needs A^T and B as tiles, and
// for symmetric A (the Grams) A^T is A, which is why the chains of products
// below need no transposes:
//   GR_b   = C (GR_{b+1} C^T)      operands GR_{b+1}, C^T, then C^T, (GR C^T)
//   G_B    = B^T B, B = P C        operands P^T, C, then B, B
//   S      = F^T (G_B F)           operands G_B, F, then F, (G_B F)
//   Tr     = F Z                   operands F^T, Z
//   P_i^T  = G_B Tr                operands G_B, Tr
// Symmetric results are mirrored from their upper triangle on the way through
// LDS, as the multi-block form does, so the factorisations see exactly
// symmetric matrices.
#include <algorithm>

#include "prgd_internal.hpp"
#include "small_la.hpp"
#include "solver.hpp"
#include "tiles.hpp"

namespace prgd {

namespace {

// row-layout tile from a row-major 16 x 16 LDS matrix, or its transpose
__device__ __forceinline__ d4 load_tile(const double *M, int lane) {
  const int r = lane >> 4, c = lane & 15;
  return d4{M[r * 16 + c], M[(r + 4) * 16 + c], M[(r + 8) * 16 + c], M[(r + 12) * 16 + c]};
}
__device__ __forceinline__ d4 load_tile_t(const double *M, int lane) {
  const int r = lane >> 4, c = lane & 15;
  return d4{M[c * 16 + r], M[c * 16 + r + 4], M[c * 16 + r + 8], M[c * 16 + r + 12]};
}

// upper triangle of a row-layout tile mirrored into the row-major n x n LDS
// matrix M (ld n); entries at or beyond n are dropped
__device__ __forceinline__ void store_sym(double *M, int n, d4 a, int lane) {
  const int c = lane & 15;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = (lane >> 4) + 4 * v;
    if (r <= c && c < n) {
      M[r * n + c] = a[v];
      M[c * n + r] = a[v];
    }
  }
}

// Where each entry of a lane's row-layout tile of C_c(x) (or of C_c(x)^T)
// comes from: the offset of T_c(x)(i mod R, j mod R) in the slice and the
// entry's quadrant (i >= R, j >= R); entries outside 2R x 2R are zero.
struct CMap {
  int off[4];
  unsigned qi, qj, valid;   // bit v: quadrant flags / inside 2R x 2R
};

template <bool TR>
__device__ __forceinline__ CMap c_map(int R, int lane) {
  CMap q;
  q.qi = q.qj = q.valid = 0u;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = (lane >> 4) + 4 * v, col = lane & 15;
    const int i = TR ? col : r, j = TR ? r : col;
    const bool ok = i < 2 * R && j < 2 * R;
    const int ii = i < R ? i : i - R, jj = j < R ? j : j - R;
    q.off[v] = ok ? ii * R + jj : 0;
    q.qi |= (i >= R ? 1u : 0u) << v;
    q.qj |= (j >= R ? 1u : 0u) << v;
    q.valid |= (ok ? 1u : 0u) << v;
  }
  return q;
}

// the tile of the block core C_c(x) of W_l = T_l - alpha xi (layout of q),
// from the slices T_c(x), X_c(x) (R x R each) in LDS: both slices are read at
// every entry's offset and the quadrant selects the value, so the loads carry
// no branch.  Middle cores [[T, 0], [X', T]], the first [X', T], the last
// [[T], [T + X']], X' = -alpha X.
__device__ __forceinline__ d4 c_tile(const double *T, const double *X, const CMap &q, int kind, double alpha) {
  d4 o;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double t = T[q.off[v]], xv = X[q.off[v]];
    const bool qi = (q.qi >> v) & 1u, qj = (q.qj >> v) & 1u;
    double e;
    if (kind == 0) e = qi ? 0.0 : (qj ? t : -alpha * xv);              // first core
    else if (kind == 2) e = qj ? 0.0 : (qi ? t - alpha * xv : t);       // last core
    else e = qi ? (qj ? t : -alpha * xv) : (qj ? 0.0 : t);              // middle cores
    o[v] = ((q.valid >> v) & 1u) ? e : 0.0;
  }
  return o;
}

__device__ __forceinline__ int core_kind(int c, int m) { return c == 0 ? 0 : (c == m - 1 ? 2 : 1); }

// global -> LDS copy of n doubles by the whole block, 16 loads in flight per
// thread
__device__ __forceinline__ void stage(double *dst, const double *src, int n) {
  const auto g = glb(src);
  const int t = threadIdx.x, nt = blockDim.x;
  int base = 0;
  for (; base + 16 * nt <= n; base += 16 * nt) {
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = g[base + k * nt + t];
#pragma unroll
    for (int k = 0; k < 16; ++k) dst[base + k * nt + t] = v[k];
  }
  for (int e = base + t; e < n; e += nt) dst[e] = g[e];
}

// the same for float data, widened to double
__device__ __forceinline__ void stage_f32(double *dst, const float *src, int n) {
  const auto g = glb(src);
  const int t = threadIdx.x, nt = blockDim.x;
  int base = 0;
  for (; base + 16 * nt <= n; base += 16 * nt) {
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = g[base + k * nt + t];
#pragma unroll
    for (int k = 0; k < 16; ++k) dst[base + k * nt + t] = (double)v[k];
  }
  for (int e = base + t; e < n; e += nt) dst[e] = (double)g[e];
}

// value of v in lane `src` of the wave (src may differ per lane)
__device__ __forceinline__ double lane_gather(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)b), hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// element k (wave-uniform) of a tile
__device__ __forceinline__ double tile_elem(d4 a, int k) {
  return k == 0 ? a[0] : (k == 1 ? a[1] : (k == 2 ? a[2] : a[3]));
}

// Pivoted Cholesky of a symmetric positive semidefinite n x n matrix (n <=
// 16) held as a row-layout tile a (zero outside n x n): returns the rank and
// puts in f (row layout) columns 0..rank-1 of F, F F^T = A up to pivots below
// n * 2.3e-16 * max diag, the same factor and pivot rule as
// block_pivoted_cholesky.  Every lane keeps the diagonal entry of its column
// (each row of 16 lanes a full copy), so the pivot is a maximum within a row
// of 16 lanes by DPP; the pivot's column and row reach the lanes by two
// cross-lane gathers (the matrix stays exactly symmetric, so row p serves as
// column p), with no LDS round trip per step.
__device__ __forceinline__ int wave_pcholesky16(d4 a, int n, int lane, d4 &f) {
  const int row0 = lane >> 4, c = lane & 15;
  // the diagonal entry A(c, c): element c >> 2 of lane 16 (c & 3) + c
  double dg = lane_gather(tile_elem(a, 0), 16 * (c & 3) + c);
  {
    const double d1 = lane_gather(a[1], 16 * (c & 3) + c), d2 = lane_gather(a[2], 16 * (c & 3) + c),
                 d3 = lane_gather(a[3], 16 * (c & 3) + c);
    const int e = c >> 2;
    dg = e == 0 ? dg : (e == 1 ? d1 : (e == 2 ? d2 : d3));
    dg = c < n ? dg : 0.0;
  }
  double dm = dg;
  dm = fmax(dm, dpp_f64<0xB1>(dm));
  dm = fmax(dm, dpp_f64<0x4E>(dm));
  dm = fmax(dm, dpp_f64<0x141>(dm));
  dm = fmax(dm, dpp_f64<0x140>(dm));
  const double tol = (double)n * 2.3e-16 * lane_value(dm, 0);
  f = zero4();
  // 1 while a row (of this lane's four) or this lane's column has not been a
  // pivot, 0 after and outside n: the factor of a pivoted row is exactly zero
  double ar[4], ac = c < n ? 1.0 : 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) ar[v] = row0 + 4 * v < n ? 1.0 : 0.0;
  int rank = 0;
  bool go = true;   // wave-uniform: no pivot has fallen below the tolerance
  // the loop leaves at its end, after a step whose pivot failed (that step
  // updates nothing: its factors are zero), so it has a single exit
  for (int k = 0; k < n; ++k) {
    const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(fmax(dg, 0.0)) >> 32);
    unsigned key = ac != 0.0 ? ((hi & ~31u) | (unsigned)(31 - c)) : 0u;
    key = max(key, (unsigned)__builtin_amdgcn_mov_dpp((int)key, 0xB1, 0xF, 0xF, false));
    key = max(key, (unsigned)__builtin_amdgcn_mov_dpp((int)key, 0x4E, 0xF, 0xF, false));
    key = max(key, (unsigned)__builtin_amdgcn_mov_dpp((int)key, 0x141, 0xF, 0xF, false));
    key = max(key, (unsigned)__builtin_amdgcn_mov_dpp((int)key, 0x140, 0xF, 0xF, false));
    const unsigned kmax = __builtin_amdgcn_readfirstlane(key);
    const int p = 31 - (int)(kmax & 31u);
    // column p of this lane's rows (lane 16 row0 + p, same elements) and row
    // p of this lane's column (lane 16 (p & 3) + c, element p >> 2)
    double col_p[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) col_p[v] = lane_gather(a[v], 16 * row0 + (p & 15));
    const double row_p = lane_gather(tile_elem(a, (p >> 2) & 3), 16 * (p & 3) + c);
    const double best = lane_value(dg, p & 15);
    go = go && kmax != 0u && best > tol;
    rank += go ? 1 : 0;
    const double rs = go ? rsq_newton<2>(best) : 0.0;
    const double fc = row_p * (rs * ac);
    const double sel = c == k ? 1.0 : 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double fr = col_p[v] * (rs * ar[v]);
      f[v] = fma(fr, sel, f[v]);
      a[v] = fma(-fr, fc, a[v]);
      ar[v] = row0 + 4 * v == p ? 0.0 : ar[v];
    }
    dg = fma(-fc, fc, dg);
    ac = c == p ? 0.0 : ac;
    if (!go) break;
  }
  return rank;
}

// The sweeps of jacobi_sweeps<true> (same slots, tournament moves, rotation
// formula, stop rule and results, bit for bit) with each rotation computed
// once: lane (P, Q) forms the rotation of pair Q from the diagonal block
// (Q, Q) and takes that of pair P from lane (P, P) by a cross-lane gather,
// instead of computing both.  The gather needs every lane, so all lanes
// compute (the idle ones on block (0, 0)) and only the working ones store.
__device__ __forceinline__ bool wave_jacobi_sweeps(double *W1, double *W2, double *A, double *V, int ne, double off,
                                                   double dia, int lane) {
  const int np = ne / 2, m1 = ne - 1;
  const bool act = lane < np * np;
  const int P = act ? lane / np : 0, Q = act ? lane - P * np : 0;
  const int r1 = 2 * P * ne, r2 = r1 + ne, c1 = 2 * Q, c2 = c1 + 1;
  const int q1 = 2 * Q * (ne + 1);
  const int lp = P * np + P;   // the lane that owns diagonal block (P, P)
  const int nr1 = tournament_next(2 * P, np) * ne, nr2 = tournament_next(2 * P + 1, np) * ne;
  const int nc1 = tournament_next(c1, np), nc2 = tournament_next(c2, np);
  auto one_round = [&](const double *src, double *dst, const double *vsrc, double *vdst, bool last) {
    const double q11 = src[q1], q12 = src[q1 + 1], q22 = src[q1 + ne + 1];
    const double a11 = src[r1 + c1], a12 = src[r1 + c2];
    const double a21 = src[r2 + c1], a22 = src[r2 + c2];
    const double v11 = vsrc[r1 + c1], v12 = vsrc[r1 + c2];
    const double v21 = vsrc[r2 + c1], v22 = vsrc[r2 + c2];
    double cQ, sQ;
    jacobi_rotation(q11, q22, q12, cQ, sQ);
    const double cP = lane_gather(cQ, lp), sP = lane_gather(sQ, lp);
    // M = A J_Q, then J_P^T M
    const double m11 = cQ * a11 - sQ * a12, m12 = sQ * a11 + cQ * a12;
    const double m21 = cQ * a21 - sQ * a22, m22 = sQ * a21 + cQ * a22;
    const double b11 = cP * m11 - sP * m21, b12 = cP * m12 - sP * m22;
    const double b21 = sP * m11 + cP * m21, b22 = sP * m12 + cP * m22;
    if (act) {
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
        if (P == Q) {   // b11, b22 on the diagonal
          dia += b11 * b11 + b22 * b22;
          off += b12 * b12 + b21 * b21;
        } else {
          off += b11 * b11 + b12 * b12 + b21 * b21 + b22 * b22;
        }
      }
    }
    wave_lds_sync();
  };
  double prev = 0.0;   // off-diagonal mass before the last sweep
  bool flip = false;   // data in (W2, V) rather than (W1, A)
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
    off = wave_sum_uniform(off);
    dia = wave_sum_uniform(dia);
  }
  return flip;
}

// block_jacobi_eig for n <= 16 run by one wave (lane = threadIdx.x & 63 of
// the first wave of the block) with no block barrier: the same sweeps
// (jacobi_sweeps, one-wave form), set-up and sorting done by the wave.
// On exit w[0..n) holds the eigenvalues in descending order and V (ld n)
// the eigenvectors as columns.  A (read, then reused), V, W1, W2: 256
// doubles each.
__device__ __forceinline__ void wave_jacobi_eig(double *A, int n, double *V, double *w, double *W1, double *W2,
                                                int lane) {
  __shared__ int rank_of[16];
  const int ne = n + (n & 1);
  double off = 0.0, dia = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = lane + 64 * q, i = e >> 4, j = e & 15;
    if (i < ne && j < ne) {
      const double v = (i < n && j < n) ? A[i * n + j] : 0.0;
      W1[i * ne + j] = v;
      if (i == j) dia += v * v;
      else off += v * v;
    }
  }
  off = wave_sum_uniform(off);
  dia = wave_sum_uniform(dia);
  wave_lds_sync();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = lane + 64 * q, i = e >> 4, j = e & 15;
    if (i < ne && j < ne) A[i * ne + j] = i == j ? 1.0 : 0.0;
  }
  wave_lds_sync();
  const bool flip = wave_jacobi_sweeps(W1, W2, A, V, ne, off, dia, lane);
  wave_lds_sync();
  const double *cur = flip ? W2 : W1;
  double *nxt = flip ? W1 : W2;
  const double *vc = flip ? V : A;
  if (vc == V) {   // the eigenvectors sit in V's own area: move them first
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = lane + 64 * q;
      if (e < ne * ne) nxt[e] = vc[e];
    }
    wave_lds_sync();
    vc = nxt;
  }
  // descending order, stable by index
  if (lane < n) {
    const double wi = cur[lane * ne + lane];
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double wj = cur[j * ne + j];
      rk += (wj > wi || (wj == wi && j < lane)) ? 1 : 0;
    }
    w[rk] = wi;
    rank_of[lane] = rk;
  }
  wave_lds_sync();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = lane + 64 * q, rr = e >> 4, i = e & 15;
    if (rr < n && i < n) V[rr * n + rank_of[i]] = vc[rr * ne + i];
  }
  wave_lds_sync();
}

__device__ __forceinline__ void breakdown(const Dev &d, int lane) {
  if (lane == 0) {
    d.st->status = -5;
    d.st->done = 1;
  }
}

}  // namespace

// bytes of dynamic LDS the one-workgroup retraction needs for solve d
static size_t retract_wave_lds(const Dev &d) {
  return sizeof(double) * (size_t)(2 * d.coff[d.m] + (long long)T16 * (d.m + 7) + 32);
}

constexpr int NWAVE = 8;   // waves of the sweep kernels (the factorisations run in parallel)
constexpr int QOFF = 8;    // second block of rows/columns in a tile (R <= 8)

__global__ void __launch_bounds__(64 * NWAVE) k_retract_wave(const Dev *__restrict__ dt, int init) {
  extern __shared__ double lds[];
  const Dev &d = dt[blockIdx.y];
  if (d.st->done) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m = d.m, R = d.R, RR = R * R;
  const int tot = (int)d.coff[m];
  const double alpha = d.st->alpha_n;
  double *sT = lds, *sX = lds + tot;
  double *Fst = sX + tot;          // GR_b, then F_b, b = 0..m-1, row-major 16 x 16, zero padded
  double *G = Fst + m * T16;       // symmetric staging
  double *A = G + T16;             // S
  double *Fc = A + T16, *S1 = Fc + T16, *W = S1 + T16, *W1 = W + T16, *W2 = W1 + T16;
  double *w = W2 + T16;            // 32 eigenvalues
  __shared__ int rank_s[MAXM + 1];
  stage(sT, d.cores, tot);
  stage(sX, d.X, tot);
  __syncthreads();
  const int row0 = lane >> 4, col = lane & 15;

  // right Grams GR_b = C_b (GR_{b+1} C_b^T), b = m-1..1, GR_m = 1 (one
  // wave: a chain of dependent products)
  if (wv == 0) {
    const CMap qt = c_map<true>(R, lane);
    d4 gn;
#pragma unroll
    for (int v = 0; v < 4; ++v) gn[v] = (row0 + 4 * v == col) ? 1.0 : 0.0;
    for (int b = m - 1; b >= 1; --b) {
      d4 acc = zero4();
      const int cb = (int)d.coff[b];
      const int kb = core_kind(b, m);
      for (int x = 0; x < d.n[b]; ++x) {
        const d4 ct = c_tile(sT + cb + x * RR, sX + cb + x * RR, qt, kb, alpha);
        const d4 mt = mm16(gn, ct, zero4());
        acc = mm16(ct, mt, acc);
      }
      double *Gb = Fst + b * T16;
      store_sym(Gb, 16, acc, lane);
      wave_lds_sync();
      gn = load_tile(Gb, lane);
    }
  }
  __syncthreads();
  // pivoted Cholesky factors F_b of the active parts of the GR_b, one wave
  // per b (no step of the chain above needs them)
  for (int b = 1 + wv; b <= m - 1; b += NWAVE) {
    double *Fb = Fst + b * T16;
    // the active indices [0, r_b) U [R, R + r_b)
    const int rb = d.r[b], na = 2 * rb;
    d4 ga, fb;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + 4 * v;
      const int gi = r < rb ? r : R + r - rb, gj = col < rb ? col : R + col - rb;
      ga[v] = (r < na && col < na) ? Fb[gi * 16 + gj] : 0.0;
    }
    const int rank = wave_pcholesky16(ga, na, lane, fb);
    // F_b over GR_b: row i of the factor goes to row gi(i) of the tile
    wave_lds_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) Fb[(row0 + 4 * v) * 16 + col] = 0.0;
    wave_lds_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + 4 * v;
      const int gi = r < rb ? r : R + r - rb;
      if (r < na) Fb[gi * 16 + col] = fb[v];
    }
    if (lane == 0) {
      rank_s[b] = rank;
      d.st->rank_f[b] = rank;
    }
    wave_lds_sync();
  }
  __syncthreads();
  __shared__ int bad_s;
  __shared__ double red_s[2 * NWAVE];
  if (threadIdx.x == 0) bad_s = 0;
  __syncthreads();
  const CMap qt = c_map<true>(R, lane), qn = c_map<false>(R, lane);
  if (wv == 0) {   // the left sweep: one wave, no block barrier
    // truncated left sweep, cut i = 1..m-1 on core c = i-1, P_0 = e_0^T
    d4 pt;
  #pragma unroll
    for (int v = 0; v < 4; ++v) pt[v] = (row0 + 4 * v == 0 && col == 0) ? 1.0 : 0.0;
    for (int i = 1; i <= m - 1; ++i) {
      const int c = i - 1, cc = (int)d.coff[c];
      d4 acc = zero4();
      const int kc = core_kind(c, m);
      for (int x = 0; x < d.n[c]; ++x) {
        const d4 cd = c_tile(sT + cc + x * RR, sX + cc + x * RR, qn, kc, alpha);
        const d4 bm = mm16(pt, cd, zero4());   // B = P_{i-1} C_c(x)
        acc = mm16(bm, bm, acc);               // G_B += B^T B
      }
      store_sym(G, 16, acc, lane);
      wave_lds_sync();
      const d4 gb = load_tile(G, lane);
      const int rk = rank_s[i], ri = d.r[i];
      if (rk < ri) {
        breakdown(d, lane);
        if (lane == 0) bad_s = 1;
        break;
      }
      const double *Fi = Fst + i * T16;
      const d4 fd = load_tile(Fi, lane);
      const d4 t1 = mm16(gb, fd, zero4());     // G_B F
      const d4 sm = mm16(fd, t1, zero4());     // S = F^T G_B F
      store_sym(A, rk, sm, lane);
      wave_lds_sync();
      // eigen-decomposition of S through its pivoted Cholesky factor, which
      // grades the matrix the Jacobi sweeps see (as block_psd_eig does): S =
      // Fc Fc^T, S1 = Fc^T Fc = W diag(w) W^T, eigenvectors Fc W diag(w)^{-1/2}
      d4 sa, fct;
  #pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + 4 * v;
        sa[v] = (r < rk && col < rk) ? A[r * rk + col] : 0.0;
      }
      const int rs = wave_pcholesky16(sa, rk, lane, fct);   // Fc, columns >= rs zero
  #pragma unroll
      for (int v = 0; v < 4; ++v) Fc[(row0 + 4 * v) * 16 + col] = fct[v];
      store_sym(S1, rs, mm16(fct, fct, zero4()), lane);   // S1 = Fc^T Fc (ld rs)
      wave_lds_sync();
      const d4 fctt = load_tile_t(Fc, lane);
      if (rs > 0) wave_jacobi_eig(S1, rs, W, w, W1, W2, lane);
      for (int e = rs + lane; e < rk; e += 64) w[e] = 0.0;
      wave_lds_sync();
      const double s0 = w[0], sr = w[ri - 1];
      if (!(sr > TRUNC_MIN_EIG_RATIO * s0) || !isfinite(s0)) {
        breakdown(d, lane);
        if (lane == 0) bad_s = 1;
        break;
      }
      // Z_r: the first r_i unit eigenvectors of S, Fc W diag(w)^{-1/2}
      d4 wt;
  #pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + 4 * v;
        wt[v] = (r < rs && col < rs) ? W[r * rs + col] : 0.0;
      }
      d4 vz = mm16(fctt, wt, zero4());
      {
        const double wc = col < rs ? w[col] : 0.0;
        const double sc = (col < ri && wc > 0.0) ? rsq_newton<2>(wc) : 0.0;
  #pragma unroll
        for (int v = 0; v < 4; ++v) vz[v] *= sc;
      }
      // Tr = F Z_r Sigma_r^{-1}
      d4 tr = mm16(load_tile_t(Fi, lane), vz, zero4());
      const double sw = col < ri ? sqrt(w[col]) : 1.0;
      const auto Tr = glb(sm_slot(d, i, S_TR));
  #pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + 4 * v;
        tr[v] = col < ri ? tr[v] / sw : 0.0;
        if (r < 2 * R && col < R) Tr[r * R + col] = tr[v];
      }
      pt = mm16(gb, tr, zero4());              // P_i^T = G_B Tr
      const auto Pn = glb(sm_slot(d, i, S_P));
  #pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + 4 * v;            // column r of P_i, row col
        if (r < 2 * R && col < R) Pn[col * 2 * R + r] = pt[v];
      }
      // Tr_i and P_i^T (2R x R each, ld 8) replace F_i, read for the last
      // time above, for the output phase
      wave_lds_sync();
      double *Ki = Fst + i * T16;
  #pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + 4 * v;
        if (col < QOFF) {
          Ki[r * QOFF + col] = tr[v];
          Ki[T16 / 2 + r * QOFF + col] = pt[v];
        }
      }
      wave_lds_sync();
    }
  }
  __syncthreads();
  if (bad_s) return;

  // new cores T'_c(x) = P_c C_c(x) Tr_{c+1} (c < m-1), P_{m-1} C_{m-1}(x),
  // slices dealt to the waves in turn; the stopping-test sums ||T'||^2 =
  // ||T'_{m-1}||^2 and <T', T> come from the last core (the others are
  // left-orthogonal), <T', T> through Z = the second block of P_{m-1}
  double nn = 0.0, cr = 0.0;
  const int nsl = d.soff[m];
  for (int sidx = wv; sidx < nsl; sidx += NWAVE) {
    int c = 0;
    while (c + 1 < m && d.soff[c + 1] <= sidx) ++c;
    const int x = sidx - d.soff[c];
    const int off = (int)d.coff[c] + x * RR;
    const double *Ks = Fst + c * T16;   // Tr_c and P_c^T
    d4 ptc;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + 4 * v;
      ptc[v] = c == 0 ? ((r == 0 && col == 0) ? 1.0 : 0.0) : (col < QOFF ? Ks[T16 / 2 + r * QOFF + col] : 0.0);
    }
    d4 out;
    if (c < m - 1) {
      const double *Kn = Fst + (c + 1) * T16;
      d4 trn;
#pragma unroll
      for (int v = 0; v < 4; ++v) trn[v] = col < QOFF ? Kn[(row0 + 4 * v) * QOFF + col] : 0.0;
      const d4 ct = c_tile(sT + off, sX + off, qt, core_kind(c, m), alpha);
      out = mm16(ptc, mm16(ct, trn, zero4()), zero4());
    } else {
      out = mm16(ptc, c_tile(sT + off, sX + off, qn, 2, alpha), zero4());
    }
    const auto gc = glb(d.cores);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + 4 * v;
      if (r < R && col < R) {
        gc[off + r * R + col] = out[v];
        if (d.prec == PREC_MIXED) glb(d.cores32)[off + r * R + col] = (float)out[v];
        long long bo = -1;
        if (c == 0 && r == 0) bo = (long long)x * R + col;
        if (c == m - 1 && col == 0) bo = (long long)d.n[0] * R + (long long)x * R + r;
        if (bo >= 0) {
          if (d.prec == PREC_MIXED) glb((float *)d.bnd)[bo] = (float)out[v];
          else glb((double *)d.bnd)[bo] = out[v];
        }
        if (c == m - 1 && col == 0) {
          double z = 0.0;
          for (int k = 0; k < R; ++k) z += Ks[T16 / 2 + (R + k) * QOFF + r] * sT[off + k * R];
          nn += out[v] * out[v];
          cr += out[v] * z;
        }
      }
    }
  }
  nn = wave_sum_uniform(nn);
  cr = wave_sum_uniform(cr);
  if (lane == 0) {
    red_s[2 * wv] = nn;
    red_s[2 * wv + 1] = cr;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a0 = 0.0, a1 = 0.0;
    for (int k = 0; k < NWAVE; ++k) {
      a0 += red_s[2 * k];
      a1 += red_s[2 * k + 1];
    }
    finish_output(d, init, a0, a1);
  }
}

// ---------------------------------------------------------------------------
// One-workgroup Gram sweep of the preconditioned projection (Lemma 3): step
// j = 1..m-1 forms
//   GL_j       = sum_x omega_{j-1}(x) T_{j-1}(x)^T GL_{j-1} T_{j-1}(x)
//   H_{m-j}    = sum_x omega_{m-j}(x) T_{m-j}(x) H_{m-j+1} T_{m-j}(x)^T
//   Theta_{j-1} = sum_x T_{j-1}(x)^T Y_{j-1}(x)
// and the inverses of GL_j and H_{m-j} on their active blocks.  The two
// chains are R x R (R <= 8), so one 16 x 16 tile carries both: the left
// chain in rows and columns 0..7, the right one in 8..15.  With the slice
// tile P(x) = diag(T_{j-1}(x), T_{m-j}(x)^T) and G = diag(GL_{j-1},
// H_{m-j+1}),
//   G P              = diag(GL T_{j-1}, H T_{m-j}^T)       (scaled per block by omega)
//   P^T (G P)        = diag(T_{j-1}^T GL T_{j-1}, T_{m-j} H T_{m-j}^T)
//   P^T diag(Y, 0)   = diag(T_{j-1}^T Y_{j-1}, 0)
// in row layout, with G and P^T needing no transpose (G symmetric; P^T in
// the A position takes P in row layout).  A core with fewer slices than the
// other contributes zero tiles past its last slice.
// ---------------------------------------------------------------------------

// Inverses of the two SPD blocks of the symmetric tile G (ld 16): the left
// Gram on rows and columns 0..7 (active size n1) and the right one on 8..15
// (active size n2), by Gauss-Jordan elimination on [A | I] without pivoting
// (SPD), both systems in one 16 x 16 tile: rows 0..7 hold [A1 | I], rows
// 8..15 [A2 | I], inactive rows and columns identity (decoupled, so every
// step leaves them unchanged).  Each lane keeps its four entries in
// registers; a step reads the pivot rows, the pivot column and the pivots
// from the LDS copy M of the tile.  The inverses, symmetrised as
// (X + X^T) / 2, go to O1 and O2 (global) and L1 and L2 (LDS), ld R, zero
// outside the active blocks.
// Returns false if a pivot of either active block is not positive.
__device__ __forceinline__ bool wave_spd_inverse_pair(const double *G, int n1, int n2, double *O1, double *O2, int R,
                                                      double *M, int lane, double *L1, double *L2) {
  const int row0 = lane >> 4, c = lane & 15;
  d4 t;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = row0 + 4 * v, b = r < QOFF ? 0 : QOFF, i = r - b, n = b ? n2 : n1;
    if (c < QOFF) t[v] = (i < n && c < n) ? G[r * 16 + b + c] : (i == c ? 1.0 : 0.0);
    else t[v] = (c - QOFF == i) ? 1.0 : 0.0;
    M[r * 16 + c] = t[v];
  }
  wave_lds_sync();
  bool bad = false;
  for (int k = 0; k < QOFF; ++k) {
    const double p1 = M[k * 16 + k], p2 = M[(QOFF + k) * 16 + k];
    const double q1 = M[k * 16 + c] * rcp_newton<2>(p1), q2 = M[(QOFF + k) * 16 + c] * rcp_newton<2>(p2);
    double f[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) f[v] = M[(row0 + 4 * v) * 16 + k];
    bad = bad || (k < n1 && !(p1 > 0.0 && isfinite(p1))) || (k < n2 && !(p2 > 0.0 && isfinite(p2)));
    wave_lds_sync();   // every read of this step precedes the writes below
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + 4 * v;
      const bool lo = r < QOFF;
      const double q = lo ? q1 : q2;
      t[v] = (r == (lo ? k : QOFF + k)) ? q : fma(-f[v], q, t[v]);
      M[r * 16 + c] = t[v];
    }
    wave_lds_sync();
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = row0 + 4 * v, b = r < QOFF ? 0 : QOFF, i = r - b, jj = c - QOFF, n = b ? n2 : n1;
    if (c >= QOFF && i < R && jj < R) {
      const double x = 0.5 * (t[v] + M[(b + jj) * 16 + QOFF + i]);
      const double o = (i < n && jj < n) ? x : 0.0;
      glb(b ? O2 : O1)[i * R + jj] = o;
      (b ? L2 : L1)[i * R + jj] = o;
    }
  }
  return !bad;
}

static size_t gram_wave_lds(const Dev &d) {
  const long long RR = (long long)d.R * d.R;
  return sizeof(double) * (size_t)(2 * d.coff[d.m] + d.soff[d.m] + (long long)T16 * (d.m + NWAVE) + RR * (4 * d.m + 2));
}

__global__ void __launch_bounds__(64 * NWAVE) k_gram_wave(const Dev *__restrict__ dt, int tangent) {
  extern __shared__ double lds[];
  const Dev &d = dt[blockIdx.y];
  if (d.st->done) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m = d.m, R = d.R, RR = R * R;
  const int tot = (int)d.coff[m], ns = d.soff[m];
  double *sT = lds, *sY = lds + tot, *sw = sY + tot;
  double *Gs = sw + ns;              // diag(GL_j, H_{m-j}) of every step j, symmetric
  double *inv = Gs + m * T16;        // working tile of the inverse pairs, one per wave
  double *GIs = inv + NWAVE * T16;   // GL_c^{-1}, c = 0..m (R x R each)
  double *HIs = GIs + (m + 1) * RR;  // H_c^{-1}, c = 0..m
  double *THs = HIs + (m + 1) * RR;  // Theta_c, then Psi_c, c = 0..m-1
  stage(sT, d.cores, tot);
  if (d.prec == PREC_MIXED) stage_f32(sY, (const float *)d.Y, tot);
  else stage(sY, (const double *)d.Y, tot);
  for (int e = threadIdx.x; e < ns; e += blockDim.x) sw[e] = glb(d.omega)[e];
  __shared__ int bad_s;
  if (threadIdx.x == 0) bad_s = 0;
  __syncthreads();
  const int row0 = lane >> 4, col = lane & 15;
  if (wv == 0) {   // the two Gram chains: one wave, dependent products
    // where each entry of the lane's tile of P(x) comes from
    int poff[4];
    unsigned pl = 0u, ph = 0u;   // bit v: entry of T_{j-1} / of T_{m-j}^T
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + 4 * v;
      const bool lo = r < QOFF && col < QOFF && r < R && col < R;
      const bool hi = r >= QOFF && col >= QOFF && r - QOFF < R && col - QOFF < R;
      poff[v] = lo ? r * R + col : (hi ? (col - QOFF) * R + (r - QOFF) : 0);
      pl |= (lo ? 1u : 0u) << v;
      ph |= (hi ? 1u : 0u) << v;
    }
    d4 g;
#pragma unroll
    for (int v = 0; v < 4; ++v) g[v] = (row0 + 4 * v == col) ? 1.0 : 0.0;   // GL_0 = H_m = 1
    for (int j = 1; j <= m - 1; ++j) {
      const int cl = j - 1, ch = m - j;
      const int nl = d.n[cl], nh = d.n[ch], nx = nl > nh ? nl : nh;
      d4 acc = zero4(), th = zero4();
      for (int x = 0; x < nx; ++x) {
        const bool xl = x < nl, xh = x < nh;
        const double *tl = sT + d.coff[cl] + (long long)(xl ? x : 0) * RR;
        const double *yl = sY + d.coff[cl] + (long long)(xl ? x : 0) * RR;
        const double *thh = sT + d.coff[ch] + (long long)(xh ? x : 0) * RR;
        const double wl = xl ? sw[d.soff[cl] + x] : 0.0, wh = xh ? sw[d.soff[ch] + x] : 0.0;
        d4 pt, yt;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double a = tl[poff[v]], b = thh[poff[v]], y = yl[poff[v]];
          const bool lo = ((pl >> v) & 1u) && xl, hi = ((ph >> v) & 1u) && xh;
          pt[v] = lo ? a : (hi ? b : 0.0);
          yt[v] = lo ? y : 0.0;
        }
        d4 n = mm16(g, pt, zero4());
        n[0] *= wl;   // rows 0..7: the left chain
        n[1] *= wl;
        n[2] *= wh;   // rows 8..15: the right chain
        n[3] *= wh;
        acc = mm16(pt, n, acc);
        th = mm16(pt, yt, th);
      }
      double *Gj = Gs + j * T16;
      store_sym(Gj, 16, acc, lane);
      const auto GLj = glb(sm_slot(d, j, S_GL)), Hb = glb(sm_slot(d, ch, S_H)), THc = glb(sm_slot(d, cl, S_TH));
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + 4 * v;
        if (r < R && col < R) {
          THc[r * R + col] = th[v];
          THs[cl * RR + r * R + col] = th[v];
        }
      }
      wave_lds_sync();
      g = load_tile(Gj, lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + 4 * v;
        if (r < R && col < R) GLj[r * R + col] = g[v];
        if (r >= QOFF && col >= QOFF && r - QOFF < R && col - QOFF < R) Hb[(r - QOFF) * R + col - QOFF] = g[v];
      }
    }
  }
  __syncthreads();
  // the inverses of GL_j and H_{m-j}, one wave per step (the chains above
  // need only the Grams themselves)
  for (int j = 1 + wv; j <= m - 1; j += NWAVE) {
    const int ch = m - j;
    const bool ok = wave_spd_inverse_pair(Gs + j * T16, d.r[j], d.r[ch], sm_slot(d, j, S_GLI), sm_slot(d, ch, S_HI), R,
                                          inv + wv * T16, lane, GIs + j * RR, HIs + ch * RR);
    if (!ok) {
      breakdown(d, lane);
      if (lane == 0) bad_s = 1;
    }
  }
  if (!tangent) return;
  // tangent components (Lemma 3):
  //   X_c(x) = omega_c(x)^{-1} GL_c^{-1} Y_c(x) H_{c+1}^{-1} - T_c(x) Psi_c,
  //   Psi_c = GL_{c+1}^{-1} Theta_c H_{c+1}^{-1} (c < m-1), Psi_{m-1} = 0,
  // and the gradient cleared for the next sampled pass; one entry per lane
  for (int e = threadIdx.x; e < RR; e += blockDim.x) {   // GL_0^{-1} = H_m^{-1} = 1
    GIs[e] = (e / R == e % R) ? 1.0 : 0.0;
    HIs[m * RR + e] = (e / R == e % R) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (bad_s) return;
  // R x R matrices as 16 x 16 tiles, zero outside R x R (row layout; _t: transposed)
  auto tile = [&](const double *M, bool tr) {
    d4 o;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + 4 * v;
      o[v] = (r < R && col < R) ? M[tr ? col * R + r : r * R + col] : 0.0;
    }
    return o;
  };
  for (int c = wv; c < m - 1; c += NWAVE) {   // Psi_c = GL_{c+1}^{-1} (Theta_c H_{c+1}^{-1}), over Theta_c
    const d4 ps = mm16(tile(GIs + (c + 1) * RR, false),
                       mm16(tile(THs + c * RR, true), tile(HIs + (c + 1) * RR, false), zero4()), zero4());
    wave_lds_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + 4 * v;
      if (r < R && col < R) THs[c * RR + r * R + col] = ps[v];
    }
  }
  __syncthreads();
  const int nsl = d.soff[m];
  for (int sidx = wv; sidx < nsl; sidx += NWAVE) {
    int c = 0;
    while (c + 1 < m && d.soff[c + 1] <= sidx) ++c;
    const int x = sidx - d.soff[c];
    const int off = (int)d.coff[c] + x * RR;
    const double iw = 1.0 / sw[d.soff[c] + x];
    // GL_c^{-1} (Y H_{c+1}^{-1}) omega^{-1} - T Psi_c
    const d4 yh = mm16(tile(sY + off, true), tile(HIs + (c + 1) * RR, false), zero4());
    d4 xt = mm16(tile(GIs + c * RR, false), yh, zero4());
    const d4 tp = c < m - 1 ? mm16(tile(sT + off, true), tile(THs + c * RR, false), zero4()) : zero4();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + 4 * v;
      if (r < R && col < R) {
        glb(d.X)[off + r * R + col] = xt[v] * iw - tp[v];
        if (d.prec == PREC_MIXED) glb((float *)d.Y)[off + r * R + col] = 0.0f;
        else glb((double *)d.Y)[off + r * R + col] = 0.0;
      }
    }
  }
}

// The one-workgroup sweeps apply when every member of the batch has R <= 8, at
// most 16 slices per core (one wave walks each core's slices in turn, so for
// long cores the slice-parallel launches win) and
// cores that fit the LDS of one workgroup next to the work tiles.
constexpr int WAVE_MAX_N = 16;
constexpr size_t WAVE_MAX_LDS = 150 * 1024;

hipError_t launch_retract_wave(const Batch &bt, hipStream_t s, int init, bool &used) {
  used = false;
  size_t lds = 0;
  for (int i = 0; i < bt.ns; ++i) {
    const Dev &d = bt.host[i];
    if (d.R > 8) return hipSuccess;
    for (int c = 0; c < d.m; ++c)
      if (d.n[c] > WAVE_MAX_N) return hipSuccess;
    lds = std::max(lds, retract_wave_lds(d));
  }
  if (lds > WAVE_MAX_LDS) return hipSuccess;
  used = true;
  hipLaunchKernelGGL(k_retract_wave, dim3(1, bt.ns), dim3(64 * NWAVE), lds, s, bt.dt, init);
  return hipGetLastError();
}

hipError_t launch_gram_wave(const Batch &bt, hipStream_t s, int tangent, bool &used) {
  used = false;
  size_t lds = 0;
  for (int i = 0; i < bt.ns; ++i) {
    const Dev &d = bt.host[i];
    if (d.R > QOFF) return hipSuccess;
    for (int c = 0; c < d.m; ++c)
      if (d.n[c] > WAVE_MAX_N) return hipSuccess;
    lds = std::max(lds, gram_wave_lds(d));
  }
  if (lds > WAVE_MAX_LDS) return hipSuccess;
  used = true;
  hipLaunchKernelGGL(k_gram_wave, dim3(1, bt.ns), dim3(64 * NWAVE), lds, s, bt.dt, tangent);
  return hipGetLastError();
}

}  // namespace prgd
