// One-wave retraction sweep for padded ranks R <= 8 and few slices per core.
//
// The retraction of Algorithm 1 on the rank-2r block TT W_l (see the notes at
// the top of dense.hip for C_c, GR_b, F_b, S, Tr_i and P_i) is a chain of
// 2(m-1) dependent steps on 2R x 2R matrices.  For R <= 8 every such matrix
// fits one 16 x 16 tile, so one wave runs the whole chain: the cores T and the
// tangent components X are copied into LDS once, every product is four
// float64 16x16x4 MFMAs, and the state passed from step to step (GR_{b+1},
// F_b, P_{i-1}) stays in registers or LDS, with no workgroup barrier and no
// trip through global memory inside the chain.  The small factorisations
// (pivoted Cholesky, Jacobi) are the one-wave routines of small_la.hpp.
//
// Register layout of a 16 x 16 matrix M ("row layout"): element v of lane l
// holds M((l >> 4) + 4 v, l & 15).  The float64 16x16x4 MFMA takes in step s
// the operand A(l & 15, 4 s + (l >> 4)) and the operand B(4 s + (l >> 4),
// l & 15): the first is element s of A^T in row layout, the second element s
// of B, and the product comes back in row layout.  So A B needs A^T and B in
// row layout; for symmetric A (the Grams) A^T is A, which is why the chain
// of products below needs no transposes:
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

namespace prgd {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int T16 = 256;   // doubles of one 16 x 16 tile

// A B from A^T and B in row layout, added to acc
__device__ __forceinline__ d4 mm16(d4 at, d4 b, d4 acc) {
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(at[0], b[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(at[1], b[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(at[2], b[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(at[3], b[3], acc, 0, 0, 0);
  return acc;
}

__device__ __forceinline__ d4 zero4() { return d4{0.0, 0.0, 0.0, 0.0}; }

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

// global -> LDS copy of n doubles by one wave, 16 loads in flight per lane
__device__ __forceinline__ void stage(double *dst, const double *src, int n, int lane) {
  const auto g = glb(src);
  int base = 0;
  for (; base + 16 * 64 <= n; base += 16 * 64) {
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = g[base + k * 64 + lane];
#pragma unroll
    for (int k = 0; k < 16; ++k) dst[base + k * 64 + lane] = v[k];
  }
  for (int e = base + lane; e < n; e += 64) dst[e] = g[e];
}

// the same for float data, widened to double
__device__ __forceinline__ void stage_f32(double *dst, const float *src, int n, int lane) {
  const auto g = glb(src);
  int base = 0;
  for (; base + 16 * 64 <= n; base += 16 * 64) {
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = g[base + k * 64 + lane];
#pragma unroll
    for (int k = 0; k < 16; ++k) dst[base + k * 64 + lane] = (double)v[k];
  }
  for (int e = base + lane; e < n; e += 64) dst[e] = (double)g[e];
}

__device__ __forceinline__ void breakdown(const Dev &d, int lane) {
  if (lane == 0) {
    d.st->status = -5;
    d.st->done = 1;
  }
}

}  // namespace

// bytes of dynamic LDS the one-wave retraction needs for solve d
static size_t retract_wave_lds(const Dev &d) {
  return sizeof(double) * (size_t)(2 * d.coff[d.m] + (long long)T16 * (d.m + 7) + 32);
}

__global__ void __launch_bounds__(64) k_retract_wave(const Dev *__restrict__ dt) {
  extern __shared__ double lds[];
  const Dev &d = dt[blockIdx.y];
  if (d.st->done) return;
  const int lane = threadIdx.x;
  const int m = d.m, R = d.R, RR = R * R;
  const int tot = (int)d.coff[m];
  const double alpha = d.st->alpha_n;
  double *sT = lds, *sX = lds + tot;
  double *Fst = sX + tot;          // F_b, b = 0..m-1, row-major 16 x 16, zero padded
  double *G = Fst + m * T16;       // symmetric staging
  double *A = G + T16;             // compressed right Gram, then S
  double *Fc = A + T16, *S1 = Fc + T16, *W = S1 + T16, *W1 = W + T16, *W2 = W1 + T16;
  double *w = W2 + T16;            // 32 eigenvalues
  __shared__ int rank_s[MAXM + 1];
  stage(sT, d.cores, tot, lane);
  stage(sX, d.X, tot, lane);
  wave_lds_sync();
  const int row0 = lane >> 4, col = lane & 15;
  const CMap qt = c_map<true>(R, lane), qn = c_map<false>(R, lane);

  // right Grams GR_b = C_b (GR_{b+1} C_b^T), b = m-1..1, GR_m = 1, and the
  // pivoted Cholesky factors F_b of their active parts
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
    store_sym(G, 16, acc, lane);
    wave_lds_sync();
    gn = load_tile(G, lane);
    // the active indices [0, r_b) U [R, R + r_b)
    const int rb = d.r[b], na = 2 * rb;
    for (int e = lane; e < T16; e += 64) {
      const int i = e >> 4, j = e & 15;
      const int gi = i < rb ? i : R + i - rb, gj = j < rb ? j : R + j - rb;
      if (i < na && j < na) A[i * na + j] = G[gi * 16 + gj];
    }
    wave_lds_sync();
    const int rank = block_pivoted_cholesky(A, na, Fc);
    double *Fb = Fst + b * T16;
    for (int e = lane; e < T16; e += 64) {
      const int gi = e >> 4, c2 = e & 15;
      int i = -1;
      if (gi < rb) i = gi;
      else if (gi >= R && gi < R + rb) i = gi - R + rb;
      Fb[e] = (i >= 0 && c2 < rank) ? Fc[i * na + c2] : 0.0;
    }
    if (lane == 0) {
      rank_s[b] = rank;
      d.st->rank_f[b] = rank;
    }
    wave_lds_sync();
  }

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
      return;
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
    const int rs = block_pivoted_cholesky(A, rk, Fc);   // ld rk, columns >= rs zero
    d4 fct, fctt;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + 4 * v;
      const bool in = r < rk && col < rk;
      fct[v] = in ? Fc[r * rk + col] : 0.0;
      fctt[v] = in ? Fc[col * rk + r] : 0.0;
    }
    store_sym(S1, rs, mm16(fct, fct, zero4()), lane);   // S1 = Fc^T Fc (ld rs)
    wave_lds_sync();
    if (rs > 0) block_jacobi_eig(S1, rs, W, w, W1, W2);
    for (int e = rs + lane; e < rk; e += 64) w[e] = 0.0;
    wave_lds_sync();
    const double s0 = w[0], sr = w[ri - 1];
    if (!(sr > TRUNC_MIN_EIG_RATIO * s0) || !isfinite(s0)) {
      breakdown(d, lane);
      return;
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
    wave_lds_sync();
  }
}

// ---------------------------------------------------------------------------
// One-wave Gram sweep of the preconditioned projection (Lemma 3): step
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
constexpr int QOFF = 8;   // first row and column of the right chain in the tile

// Inverses of the two SPD blocks of the symmetric tile G (ld 16): the left
// Gram on rows and columns 0..7 (active size n1) and the right one on 8..15
// (active size n2), by Gauss-Jordan elimination on [A | I] without pivoting
// (SPD), both systems in one 16 x 16 tile: rows 0..7 hold [A1 | I], rows
// 8..15 [A2 | I], inactive rows and columns identity (decoupled, so every
// step leaves them unchanged).  Each lane keeps its four entries in
// registers; a step reads the pivot rows, the pivot column and the pivots
// from the LDS copy M of the tile.  The inverses, symmetrised as
// (X + X^T) / 2, go to O1 and O2 (ld R, zero outside the active blocks).
// Returns false if a pivot of either active block is not positive.
__device__ __forceinline__ bool wave_spd_inverse_pair(const double *G, int n1, int n2, double *O1, double *O2, int R,
                                                      double *M, int lane) {
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
      glb(b ? O2 : O1)[i * R + jj] = (i < n && jj < n) ? x : 0.0;
    }
  }
  return !bad;
}

static size_t gram_wave_lds(const Dev &d) {
  return sizeof(double) * (size_t)(2 * d.coff[d.m] + d.soff[d.m] + 2 * T16);
}

__global__ void __launch_bounds__(64) k_gram_wave(const Dev *__restrict__ dt) {
  extern __shared__ double lds[];
  const Dev &d = dt[blockIdx.y];
  if (d.st->done) return;
  const int lane = threadIdx.x;
  const int m = d.m, R = d.R, RR = R * R;
  const int tot = (int)d.coff[m], ns = d.soff[m];
  double *sT = lds, *sY = lds + tot, *sw = sY + tot;
  double *G = sw + ns;             // symmetric staging of the two Grams
  double *inv = G + T16;           // working tile of the inverse pair
  stage(sT, d.cores, tot, lane);
  if (d.prec == PREC_MIXED) {
    stage_f32(sY, (const float *)d.Y, tot, lane);
  } else {
    stage(sY, (const double *)d.Y, tot, lane);
  }
  for (int e = lane; e < ns; e += 64) sw[e] = glb(d.omega)[e];
  wave_lds_sync();
  const int row0 = lane >> 4, col = lane & 15;
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
    store_sym(G, 16, acc, lane);
    const auto GLj = glb(sm_slot(d, j, S_GL)), Hb = glb(sm_slot(d, ch, S_H)), THc = glb(sm_slot(d, cl, S_TH));
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + 4 * v;
      if (r < R && col < R) THc[r * R + col] = th[v];
    }
    wave_lds_sync();
    g = load_tile(G, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + 4 * v;
      if (r < R && col < R) GLj[r * R + col] = g[v];
      if (r >= QOFF && col >= QOFF && r - QOFF < R && col - QOFF < R) Hb[(r - QOFF) * R + col - QOFF] = g[v];
    }
    const bool ok = wave_spd_inverse_pair(G, d.r[j], d.r[ch], sm_slot(d, j, S_GLI), sm_slot(d, ch, S_HI), R, inv, lane);
    if (!ok) {
      breakdown(d, lane);
      return;
    }
    wave_lds_sync();
  }
}

// The one-wave sweep applies when every member of the batch has R <= 8, at
// most 8 slices per core (beyond that the slice-parallel launches win) and
// cores that fit the LDS of one workgroup next to the work tiles.
constexpr int WAVE_MAX_N = 8;
constexpr size_t WAVE_MAX_LDS = 150 * 1024;

hipError_t launch_retract_wave(const Batch &bt, hipStream_t s, bool &used) {
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
  hipLaunchKernelGGL(k_retract_wave, dim3(1, bt.ns), dim3(64), lds, s, bt.dt);
  return hipGetLastError();
}

hipError_t launch_gram_wave(const Batch &bt, hipStream_t s, bool &used) {
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
  hipLaunchKernelGGL(k_gram_wave, dim3(1, bt.ns), dim3(64), lds, s, bt.dt);
  return hipGetLastError();
}

}  // namespace prgd
