// Dense stage of one PRGD iteration on the device, float64.
//
// Notation: cores T_c, c = 0..m-1 (0-based), bond b = 0..m between cores b-1
// and b, r_b the TT rank of bond b, omega_c(x) = (1 + s_c(x)/eps)^{1/(2m)} the
// metric factor of slice x of core c (the diagonal of G_{l,c}^{1/(2m)} divided
// by eps^{1/2m}; section 3.2.1 and Proposition 1), Y_c the Euclidean core
// gradient from the sampled pass.
//
// Preconditioned projection (Lemma 3).  With the weighted left and right Grams
//   GL_b = sum_x omega_{b-1}(x) T_{b-1}(x)^T GL_{b-1} T_{b-1}(x),   GL_0 = 1
//   H_b  = sum_x omega_b(x)     T_b(x) H_{b+1} T_b(x)^T,            H_m  = 1
// (Gram matrices of the left/right parts of W^{1/2} T), and
//   Theta_c = sum_x T_c(x)^T Y_c(x),
// the projected components of eq. "tsp in nm", moved back by W^{-1/2} and
// expressed in the gauge of the stored cores T_c, are
//   X_c(x) = omega_c(x)^{-1} GL_c^{-1} Y_c(x) H_{c+1}^{-1}
//            - T_c(x) GL_{c+1}^{-1} Theta_c H_{c+1}^{-1}          (c < m-1)
//   X_{m-1}(x) = omega_{m-1}(x)^{-1} GL_{m-1}^{-1} Y_{m-1}(x).
// This is the closed form of Lemma 3 after substituting the left-orthogonal
// decomposition of W^{1/2}T through its QR factors; every weight and gauge
// factor acts per mode slice, which is why the single sampled pass suffices.
// In units normalised by eps (weights 1 + s/eps), the direction scales by
// eps^{1/2}, so the step alpha = c eps^{1/2}/p becomes c/p.
//
// Update (Algorithm 2): W_l = T_l - alpha xi is the rank-2r block TT with
//   C_0 = [X'_0, T_0],  C_c = [[T_c, 0], [X'_c, T_c]],  C_{m-1} = [[T], [T + X']]
// where X' = -alpha X.
//
// Retraction (Algorithm 1 on W_l, in TT form).  The truncated SVD at cut i
// needs the left singular vectors of B_i W^{>=i}, B_i = P_{i-1} C_{i-1}.  With
// the right Gram GR_i = W^{>=i} W^{>=i,T} = F_i F_i^T (pivoted Cholesky) these
// are the left singular vectors of K = B_i F_i; from S = F^T (B^T B) F = Z
// Sigma^2 Z^T the new core is T'_{i-1} = B_i Tr_i with Tr_i = F Z_r Sigma_r^{-1},
// and P_i = T'^{<=i,T} W^{<=i} = Tr_i^T (B^T B).  The last core is
// P_{m-1} C_{m-1}.
#include <algorithm>

#include "prgd_internal.hpp"
#include "block_ops.hpp"
#include "small_la.hpp"
#include "solver.hpp"
#include "tiles.hpp"

namespace prgd {

constexpr int SMEM = 6656;   // doubles of static LDS used by the dense kernels
constexpr int SMEM_CUT = SMEM + 1024;   // kernels that run a truncation (left_cut)

// thread groups: G groups of TPG threads, each group working on its own slice
struct Grp {
  int G, TPG, g, tl;
};
__device__ inline Grp make_grp(int ne) {
  Grp q;
  q.G = (int)blockDim.x / ne;
  if (q.G < 1) q.G = 1;
  if (q.G > 64) q.G = 64;
  q.TPG = (int)blockDim.x / q.G;
  q.g = (int)threadIdx.x / q.TPG;
  q.tl = (int)threadIdx.x % q.TPG;
  return q;
}

__device__ inline double load_grad(const Dev &d, long long i) {
  return d.prec == PREC_MIXED ? (double)glb((const float *)d.Y)[i] : glb((const double *)d.Y)[i];
}
__device__ inline void zero_grad(const Dev &d, long long i) {
  if (d.prec == PREC_MIXED)
    glb((float *)d.Y)[i] = 0.0f;
  else
    glb((double *)d.Y)[i] = 0.0;
}

// core index and slice range of this block for slice-parallel kernels over all cores
__device__ inline void block_core(const Dev &d, int bx, int &c, int &x0, int &x1) {
  const int b = bx;
  c = 0;
  while (c + 1 < d.m && d.blk_off[c + 1] <= b) ++c;
  const int lb = b - d.blk_off[c];
  x0 = lb * d.spb[c];
  x1 = x0 + d.spb[c];
  if (x1 > d.n[c]) x1 = d.n[c];
}

// ---------------------------------------------------------------------------
// small dense linear algebra on LDS (block-cooperative; callers sync around)
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// weighted Gram sweeps (one launch per step j = 1..m-1)
// ---------------------------------------------------------------------------
// blocks [0, nbL): core j-1 -> GL_j and Theta_{j-1}
// blocks [nbL, nbL+nbH): core m-j -> H_{m-j}
__device__ __forceinline__ void gram_body(const Dev &d, int bx_, int j, double *smem_) {
  (void)bx_;
  (void)smem_;
  const int R = d.R, RR = R * R, m = d.m;
  const int nbL = nblocks_for(d.n[j - 1], 8), nbH = nblocks_for(d.n[m - j], 8);
  if (bx_ >= nbL + nbH || d.st->done) return;
  double *smem = smem_;
  const bool left = bx_ < nbL;
  const int c = left ? j - 1 : m - j;
  const int lb = left ? bx_ : bx_ - nbL;
  const int nbk = left ? nbL : nbH;
  const int per = (d.n[c] + nbk - 1) / nbk;
  const int x0 = lb * per;
  const int x1 = min(d.n[c], x0 + per);
  const bool want_th = left && c < m - 1;

  double *Gin = smem;                    // GL_{j-1} or H_{m-j+1}
  const double *gsrc = left ? sm_slot(d, j - 1, S_GL) : sm_slot(d, m - j + 1, S_H);
  for (int e = threadIdx.x; e < RR; e += blockDim.x) Gin[e] = gsrc[e];
  const Grp q = make_grp(RR);
  double *sT = smem + RR + q.g * 3 * RR;
  double *sY = sT + RR;
  double *tmp = sY + RR;
  double acc = 0.0, acct = 0.0;
  const int e = q.tl;                    // one output entry per thread (RR <= TPG)
  const int ea = e / R, eb = e % R;
  // the first round's slices are fetched before the barrier, with their loads
  // in flight together with those of the staged matrices above
  {
    const int x = x0 + q.g;
    const bool act = (q.g < q.G) && (x < x1);
    if (act) {
      const long long off = d.coff[c] + (long long)x * RR;
      for (int t = q.tl; t < RR; t += q.TPG) {
        sT[t] = glb(d.cores)[off + t];
        if (want_th) sY[t] = load_grad(d, off + t);
      }
    }
  }
  __syncthreads();
  for (int base = x0; base < x1; base += q.G) {
    const int x = base + q.g;
    const bool act = (q.g < q.G) && (x < x1);
    if (base != x0) {
      if (act) {
        const long long off = d.coff[c] + (long long)x * RR;
        for (int t = q.tl; t < RR; t += q.TPG) {
          sT[t] = glb(d.cores)[off + t];
          if (want_th) sY[t] = load_grad(d, off + t);
        }
      }
      __syncthreads();
    }
    if (act && e < RR) {
      if (left) {
        double v = 0.0;   // tmp = GLprev * T
        for (int k = 0; k < R; ++k) v += Gin[ea * R + k] * sT[k * R + eb];
        tmp[e] = v;
      } else {
        double v = 0.0;   // tmp = T * Hnext
        for (int k = 0; k < R; ++k) v += sT[ea * R + k] * Gin[k * R + eb];
        tmp[e] = v;
      }
    }
    __syncthreads();
    if (act && e < RR) {
      const double w = glb(d.omega)[d.soff[c] + x];
      double v = 0.0;
      if (left) {
        for (int k = 0; k < R; ++k) v += sT[k * R + ea] * tmp[k * R + eb];
        if (want_th) {
          double t2 = 0.0;
          for (int k = 0; k < R; ++k) t2 += sT[k * R + ea] * sY[k * R + eb];
          acct += t2;
        }
      } else {
        for (int k = 0; k < R; ++k) v += tmp[ea * R + k] * sT[eb * R + k];
      }
      acc += w * v;
    }
    __syncthreads();
  }
  // reduce the groups' accumulators in LDS, then publish the block partial
  double *red = smem + RR;   // reuse: G * 2 * RR <= 3 * 256 * ... fits
  __syncthreads();
  if (q.g < q.G && e < RR) {
    red[(q.g * 2 + 0) * RR + e] = acc;
    red[(q.g * 2 + 1) * RR + e] = acct;
  }
  __syncthreads();
  // left blocks: GL and Theta (2 RR each); right blocks: H only (RR each,
  // after the left blocks' partials)
  auto mypart = glb(d.part) + (left ? (long long)lb * 2 * RR : (long long)nbL * 2 * RR + (long long)lb * RR);
  for (int t = threadIdx.x; t < RR; t += blockDim.x) {
    double a0 = 0.0, a1 = 0.0;
    for (int g = 0; g < q.G; ++g) {
      a0 += red[(g * 2 + 0) * RR + t];
      a1 += red[(g * 2 + 1) * RR + t];
    }
    mypart[t] = a0;
    if (left) mypart[RR + t] = a1;
  }
}

// Slice blocks of a weighted Gram step on the matrix cores, for R <= 16 (one
// 16 x 16 tile, row layout of tiles.hpp), four waves each taking every fourth
// slice of the block:
//   left blocks (core j-1):  GL += omega T^T (GL_{j-1} T),  Theta += T^T Y
//   right blocks (core m-j): H  += omega T (H_{m-j+1} T^T)
// The Gram of the previous step enters transposed (as the A operand's
// transpose), T as itself or transposed as each product needs.  The waves'
// sums are added in wave order and written in gram_body's partial layout.
__global__ void __launch_bounds__(256) k_gram_tiles(const Dev *__restrict__ dt, int j) {
  constexpr int NW = 4;
  __shared__ double sTY[NW * 2 * 256];
  __shared__ double sw[NW];
  __shared__ double red[NW * 2 * 256];
  const Dev &d = dt[blockIdx.y];
  const int bx_ = blockIdx.x;
  const int R = d.R, RR = R * R, m = d.m;
  const int nbL = nblocks_for(d.n[j - 1], 8), nbH = nblocks_for(d.n[m - j], 8);
  if (bx_ >= nbL + nbH || d.st->done) return;
  const bool left = bx_ < nbL;
  const int c = left ? j - 1 : m - j;
  const int lb = left ? bx_ : bx_ - nbL;
  const int nbk = left ? nbL : nbH;
  const int per = (d.n[c] + nbk - 1) / nbk;
  const int x0 = lb * per, x1 = min(d.n[c], x0 + per);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, row0 = lane >> 4, col = lane & 15;
  // the previous Gram, transposed: tile entry (r, c) = G(c, r)
  d4 gt;
  {
    const auto gsrc = glb((const double *)(left ? sm_slot(d, j - 1, S_GL) : sm_slot(d, m - j + 1, S_H)));
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + 4 * v;
      gt[v] = (r < R && col < R) ? gsrc[col * R + r] : 0.0;
    }
  }
  auto tile = [&](const double *M, bool tr) {
    d4 o;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = row0 + 4 * v;
      o[v] = (r < R && col < R) ? M[tr ? col * R + r : r * R + col] : 0.0;
    }
    return o;
  };
  d4 acc = zero4(), th = zero4();
  for (int base = x0; base < x1; base += NW) {
    __syncthreads();   // the previous group's slices have been read
    const int cnt = min(NW, x1 - base);
    for (int e = threadIdx.x; e < cnt * RR; e += blockDim.x) {
      const int q = e / RR, t = e - q * RR;
      const long long off = d.coff[c] + (long long)(base + q) * RR + t;
      sTY[q * 512 + t] = glb(d.cores)[off];
      if (left) sTY[q * 512 + 256 + t] = load_grad(d, off);
    }
    if ((int)threadIdx.x < cnt) sw[threadIdx.x] = glb(d.omega)[d.soff[c] + base + threadIdx.x];
    __syncthreads();
    if (w < cnt) {
      const double *T = sTY + w * 512, *Y = T + 256;
      const double om = sw[w];
      if (left) {
        const d4 tt = tile(T, false);
        d4 n = mm16(gt, tt, zero4());   // GL_{j-1} T
#pragma unroll
        for (int v = 0; v < 4; ++v) n[v] *= om;
        acc = mm16(tt, n, acc);         // T^T (omega GL T)
        th = mm16(tt, tile(Y, false), th);
      } else {
        const d4 ttr = tile(T, true);
        d4 n = mm16(gt, ttr, zero4());  // H_{m-j+1} T^T
#pragma unroll
        for (int v = 0; v < 4; ++v) n[v] *= om;
        acc = mm16(ttr, n, acc);        // T (omega H T^T)
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = row0 + 4 * v;
    red[w * 512 + r * 16 + col] = acc[v];
    red[w * 512 + 256 + r * 16 + col] = th[v];
  }
  __syncthreads();
  auto mypart = glb(d.part) + (left ? (long long)lb * 2 * RR : (long long)nbL * 2 * RR + (long long)lb * RR);
  for (int t = threadIdx.x; t < RR; t += blockDim.x) {
    const int a = t / R, bcol = t - a * R;
    double a0 = 0.0, a1 = 0.0;
    for (int q = 0; q < NW; ++q) {
      a0 += red[q * 512 + a * 16 + bcol];
      a1 += red[q * 512 + 256 + a * 16 + bcol];
    }
    mypart[t] = a0;
    if (left) mypart[RR + t] = a1;
  }
}

__global__ void __launch_bounds__(1024) k_gram(const Dev *__restrict__ dt, int j) {
  __shared__ double smem[SMEM];
  gram_body(dt[blockIdx.y], (int)blockIdx.x, j, smem);
}

// finish of a Gram sweep step (one block): totals and inverses
__device__ __forceinline__ void gram_fin_body(const Dev &d, int bx_, int j, double *smem_) {
  (void)bx_;
  (void)smem_;
  if (d.st->done) return;
  double *smem = smem_;
  const int R = d.R, RR = R * R, m = d.m;
  const int nbL = nblocks_for(d.n[j - 1], 8), nbT = nbL + nblocks_for(d.n[m - j], 8);

  // last block: totals, inverses
  double *GLj = sm_slot(d, j, S_GL), *THc = sm_slot(d, j - 1, S_TH), *Hb = sm_slot(d, m - j, S_H);
  {
    double *tot = smem + 2048, *toth = tot + 2 * RR;   // [2 RR] GL and Theta, [RR] H
    reduce_partials2(d.part, nbL, 2 * RR, tot, d.part + (long long)nbL * 2 * RR, nbT - nbL, RR, toth, smem);
    for (int t = threadIdx.x; t < RR; t += blockDim.x) {
      GLj[t] = tot[t];
      THc[t] = tot[RR + t];
      Hb[t] = toth[t];
    }
  }
  __threadfence_block();
  __syncthreads();
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const bool ok = block_spd_inverse_pair(GLj, R, d.r[j], sm_slot(d, j, S_GLI), Hb, R, d.r[m - j],
                                         sm_slot(d, m - j, S_HI), R, R, smem);
  if (threadIdx.x == 0 && !ok) bad = 1;
  __syncthreads();
  if (bad) {
    if (threadIdx.x == 0) {
      d.st->status = -5;
      d.st->done = 1;
    }
    return;
  }
}

__global__ void __launch_bounds__(1024) k_gram_fin(const Dev *__restrict__ dt, int j) {
  __shared__ double smem[SMEM];
  gram_fin_body(dt[blockIdx.y], (int)blockIdx.x, j, smem);
}

// ---------------------------------------------------------------------------
// tangent components X_c(x) (all cores, slice-parallel); clears Y
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tangent_body(const Dev &d, int bx_, double *smem_) {
  (void)bx_;
  (void)smem_;
  if (bx_ >= d.blk_off[d.m] || d.st->done) return;
  double *smem = smem_;
  int c, x0, x1;
  block_core(d, bx_, c, x0, x1);
  const int R = d.R, RR = R * R, m = d.m;
  double *GI = smem, *HI = smem + RR, *PS = smem + 2 * RR;
  // Psi_c = GL_{c+1}^{-1} Theta_c H_{c+1}^{-1} (zero for the last core), formed
  // by every block from the finished Grams; its operands sit where the slice
  // buffers go afterwards
  double *G1 = smem + 3 * RR, *TH = G1 + RR, *T1 = TH + RR;
  const bool psi = c < m - 1;
  const double *gi = sm_slot(d, c, S_GLI), *hi = sm_slot(d, c + 1, S_HI);
  const double *g1 = sm_slot(d, psi ? c + 1 : c, S_GLI), *th = sm_slot(d, c, S_TH);
  for (int t = threadIdx.x; t < RR; t += blockDim.x) {
    GI[t] = gi[t];
    HI[t] = hi[t];
    G1[t] = g1[t];
    TH[t] = th[t];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < RR; t += blockDim.x) {
    const int a = t / R, b = t - a * R;
    double v = 0.0;
    for (int k = 0; k < R; ++k) v = fma(G1[a * R + k], TH[k * R + b], v);
    T1[t] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < RR; t += blockDim.x) {
    const int a = t / R, b = t - a * R;
    double v = 0.0;
    for (int k = 0; k < R; ++k) v = fma(T1[a * R + k], HI[k * R + b], v);
    PS[t] = psi ? v : 0.0;
  }
  const Grp q = make_grp(RR);
  double *sT = smem + 3 * RR + q.g * 3 * RR;
  double *sY = sT + RR, *tmp = sY + RR;
  const int e = q.tl, ea = e / R, eb = e % R;
  __syncthreads();
  for (int base = x0; base < x1; base += q.G) {
    const int x = base + q.g;
    const bool act = (q.g < q.G) && (x < x1);
    const long long off = d.coff[c] + (long long)x * RR;
    if (act)
      for (int t = q.tl; t < RR; t += q.TPG) {
        sT[t] = glb(d.cores)[off + t];
        sY[t] = load_grad(d, off + t);
        zero_grad(d, off + t);
      }
    __syncthreads();
    if (act && e < RR) {
      double v = 0.0;
      for (int k = 0; k < R; ++k) v += GI[ea * R + k] * sY[k * R + eb];
      tmp[e] = v;
    }
    __syncthreads();
    if (act && e < RR) {
      const double iw = 1.0 / glb(d.omega)[d.soff[c] + x];
      double v = 0.0;
      for (int k = 0; k < R; ++k) v += tmp[ea * R + k] * HI[k * R + eb];
      v *= iw;
      double u = 0.0;
      for (int k = 0; k < R; ++k) u += sT[ea * R + k] * PS[k * R + eb];
      glb(d.X)[off + e] = v - u;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(1024) k_tangent(const Dev *__restrict__ dt) {
  __shared__ double smem[SMEM];
  tangent_body(dt[blockIdx.y], (int)blockIdx.x, smem);
}

// ---------------------------------------------------------------------------
// tangent components with the three R x R contractions per slice on the
// matrix cores in bfloat16 (float32 accumulation), one wave per slice
// ---------------------------------------------------------------------------
typedef short bf_s4 __attribute__((ext_vector_type(4)));
typedef float bf_f4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ short to_bf16(float f) {
  const unsigned u = __float_as_uint(f);
  return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// power of two p with max|v| * p in [0.5, 1) (1 for an all-zero matrix): exact
// scaling that puts the bfloat16 operands of each core near unit size
__device__ __forceinline__ double unit_scale(double amax) {
  if (!(amax > 0.0)) return 1.0;
  int e;
  (void)frexp(amax, &e);
  return ldexp(1.0, -e);
}

// Same result as k_tangent (X_c(x) = omega^{-1} GL_c^{-1} Y_c(x) H_{c+1}^{-1}
// - T_c(x) Psi_c) with the slice products on 16x16x16 bfloat16 MFMAs.  The
// R x R operands are zero-padded to 16 x 16.  Lane l of a wave holds row or
// column l % 16 and the four k indices 4 (l / 16) .. +3.  The first product is
// formed transposed, (GL^{-1} Y)^T = Y^T GL^{-T}, so that its result lands in
// the A-operand layout of the second.  Scales: one power of two per core for
// GL^{-1}, H^{-1} and Psi, one per slice for Y(x), T(x) and GL^{-1} Y(x).
__device__ __forceinline__ void tangent_bf16_body(const Dev &d, int bx_, double *smem_) {
  (void)bx_;
  (void)smem_;
  if (bx_ >= d.blk_off[d.m] || d.st->done) return;
  double *smem = smem_;
  __shared__ double samax[32];
  int c, x0, x1;
  block_core(d, bx_, c, x0, x1);
  const int R = d.R, RR = R * R, m = d.m;
  double *GI = smem, *HI = smem + RR, *PS = smem + 2 * RR;
  double *G1 = smem + 3 * RR, *TH = G1 + RR, *T1 = TH + RR;
  const bool psi = c < m - 1;
  const double *gi = sm_slot(d, c, S_GLI), *hi = sm_slot(d, c + 1, S_HI);
  const double *g1 = sm_slot(d, psi ? c + 1 : c, S_GLI), *th = sm_slot(d, c, S_TH);
  for (int t = threadIdx.x; t < RR; t += blockDim.x) {
    GI[t] = gi[t];
    HI[t] = hi[t];
    G1[t] = g1[t];
    TH[t] = th[t];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < RR; t += blockDim.x) {
    const int a = t / R, b = t - a * R;
    double v = 0.0;
    for (int k = 0; k < R; ++k) v = fma(G1[a * R + k], TH[k * R + b], v);
    T1[t] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < RR; t += blockDim.x) {
    const int a = t / R, b = t - a * R;
    double v = 0.0;
    for (int k = 0; k < R; ++k) v = fma(T1[a * R + k], HI[k * R + b], v);
    PS[t] = psi ? v : 0.0;
  }
  __syncthreads();
  // per-core scales of GL^{-1}, H^{-1}, Psi
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (w < 3) {
    const double *Mx = w == 0 ? GI : (w == 1 ? HI : PS);
    double a = 0.0;
    for (int t = lane; t < RR; t += 64) a = fmax(a, fabs(Mx[t]));
    a = wave_max(a);
    if (lane == 0) samax[w] = a;
  }
  __syncthreads();
  const double sG = unit_scale(samax[0]), sH = unit_scale(samax[1]), sP = unit_scale(samax[2]);
  const int i = lane & 15, q = lane >> 4;
  // B operands fixed for the core: (GL^{-1})^T[k][i] = GL^{-1}[i][k], H^{-1}[k][i], Psi[k][i]
  bf_s4 bG, bH, bP;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int k = 4 * q + v;
    const bool in = i < R && k < R;
    bG[v] = to_bf16(in ? (float)(GI[i * R + k] * sG) : 0.0f);
    bH[v] = to_bf16(in ? (float)(HI[k * R + i] * sH) : 0.0f);
    bP[v] = to_bf16(in ? (float)(PS[k * R + i] * sP) : 0.0f);
  }
  const bf_f4 zero = {0.f, 0.f, 0.f, 0.f};
  for (int x = x0 + w; x < x1; x += nw) {
    const long long off = d.coff[c] + (long long)x * RR;
    // A of the first product: Y^T[i][k] = Y[k][i]; A of the third: T[i][k]
    double yv[4], tv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = 4 * q + v;
      const bool in = i < R && k < R;
      yv[v] = in ? load_grad(d, off + (long long)k * R + i) : 0.0;
      tv[v] = in ? glb(d.cores)[off + (long long)i * R + k] : 0.0;
    }
    double ya = fmax(fmax(fabs(yv[0]), fabs(yv[1])), fmax(fabs(yv[2]), fabs(yv[3])));
    double ta = fmax(fmax(fabs(tv[0]), fabs(tv[1])), fmax(fabs(tv[2]), fabs(tv[3])));
    ya = wave_max(ya);
    ta = wave_max(ta);
    const double sY = unit_scale(ya), sT = unit_scale(ta);
    bf_s4 aY, aT;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      aY[v] = to_bf16((float)(yv[v] * sY));
      aT[v] = to_bf16((float)(tv[v] * sT));
    }
    // (GL^{-1} Y)^T, scaled by sY sG: element v of lane l is (GL^{-1} Y)[i][4q + v]
    const bf_f4 gy = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aY, bG, zero, 0, 0, 0);
    double ga = fmax(fmax(fabs((double)gy[0]), fabs((double)gy[1])), fmax(fabs((double)gy[2]), fabs((double)gy[3])));
    ga = wave_max(ga);
    const double sM = unit_scale(ga);
    bf_s4 aM;
#pragma unroll
    for (int v = 0; v < 4; ++v) aM[v] = to_bf16((float)(gy[v] * sM));
    const bf_f4 vv = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aM, bH, zero, 0, 0, 0);
    const bf_f4 uu = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aT, bP, zero, 0, 0, 0);
    const double iw = 1.0 / glb(d.omega)[d.soff[c] + x];
    const double kv = iw / (sY * sG * sM * sH), ku = 1.0 / (sT * sP);
    // element v: row 4q + v, column i
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 4 * q + v;
      if (r < R && i < R) glb(d.X)[off + (long long)r * R + i] = (double)vv[v] * kv - (double)uu[v] * ku;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = 4 * q + v;
      if (i < R && k < R) zero_grad(d, off + (long long)k * R + i);
    }
  }
}

__global__ void __launch_bounds__(1024) k_tangent_bf16(const Dev *__restrict__ dt) {
  __shared__ double smem[SMEM];
  tangent_bf16_body(dt[blockIdx.y], (int)blockIdx.x, smem);
}

// block core C_c(x) of W_l = T_l - alpha xi as a 2R x 2R matrix in LDS
__device__ inline void build_block(const Dev &d, int c, const double *sT, const double *sX, double alpha,
                                   double *C, int tl, int tpg) {
  const int R = d.R, R2 = 2 * R, m = d.m;
  for (int t = tl; t < R2 * R2; t += tpg) {
    const int i = t / R2, jj = t % R2;
    double v = 0.0;
    if (c == 0) {
      if (i < R) v = (jj < R) ? -alpha * sX[i * R + jj] : sT[i * R + jj - R];
    } else if (c == m - 1) {
      if (jj < R) v = (i < R) ? sT[i * R + jj] : sT[(i - R) * R + jj] - alpha * sX[(i - R) * R + jj];
    } else {
      if (i < R) v = (jj < R) ? sT[i * R + jj] : 0.0;
      else v = (jj < R) ? -alpha * sX[(i - R) * R + jj] : sT[(i - R) * R + jj - R];
    }
    C[t] = v;
  }
}

// ---------------------------------------------------------------------------
// right Grams of the block TT: GR_b = sum_x C_b(x) GR_{b+1} C_b(x)^T, b = m-1..1
// last block: pivoted Cholesky factor F_b of GR_b on its active indices
// ---------------------------------------------------------------------------
// Gram of the first left cut, G_B = sum_x B(x)^T B(x) with B(x) = row 0 of
// C_0(x) (P_0 = 1): it does not depend on the right sweep, so the first
// right-Gram launch computes its partials in extra blocks (at GB1_OFF of the
// partial buffer) and the finish of the last right-Gram step uses them.
constexpr long long GB1_OFF = 1LL << 19;

// The 2R x 2R Gram partials are symmetric: producers write the upper triangle
// only (row-major, n (n + 1) / 2 entries), which halves what the one-block
// finishers read back.
__device__ __forceinline__ int sym_index(int a, int b, int n) { return (a * (2 * n - a + 1)) / 2 + (b - a); }

// total of nb packed symmetric partials, unpacked into full[n * n] (LDS);
// packed: LDS of n (n + 1) / 2 doubles, scratch: blockDim.x doubles
__device__ __forceinline__ void reduce_sym_partials(const double *part, int nb, int n, double *full, double *packed,
                                                    double *scratch) {
  reduce_partials(part, nb, n * (n + 1) / 2, packed, scratch);
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int a = t / n, b = t - a * n;
    full[t] = packed[a <= b ? sym_index(a, b, n) : sym_index(b, a, n)];
  }
  __syncthreads();
}


__device__ __forceinline__ void left_cut(const Dev &d, int i, double *smem);

__device__ void gram_first_cut(const Dev &d, int lb) {
  const int R = d.R, R2 = 2 * R, NE = R2 * R2, RR = R * R;
  const int nbl = nblocks_for(d.n[0], 4);
  const int per = (d.n[0] + nbl - 1) / nbl;
  const int x0 = lb * per, x1 = min(d.n[0], x0 + per);
  const double alpha = d.st->alpha_n;
  const auto T = glb(d.cores), X = glb(d.X);
  const int NP = R2 * (R2 + 1) / 2;
  for (int f = threadIdx.x; f < NE; f += blockDim.x) {
    const int a = f / R2, bb = f % R2;
    if (a > bb) continue;
    double acc = 0.0;
    for (int x = x0; x < x1; ++x) {
      const long long off = d.coff[0] + (long long)x * RR;
      const double va = (a < R) ? -alpha * X[off + a] : T[off + a - R];
      const double vb = (bb < R) ? -alpha * X[off + bb] : T[off + bb - R];
      acc += va * vb;
    }
    glb(d.part)[GB1_OFF + (long long)lb * NP + sym_index(a, bb, R2)] = acc;
  }
}

__device__ __forceinline__ void rgram_body(const Dev &d, int bx_, int b, double *smem_) {
  (void)bx_;
  (void)smem_;
  const int nb = nblocks_for(d.n[b], 4);
  const int m = d.m;
  if (d.st->done) return;
  if (bx_ >= nb) {
    const int lb = bx_ - nb;
    if (b == m - 1 && lb < nblocks_for(d.n[0], 4)) gram_first_cut(d, lb);
    return;
  }
  double *smem = smem_;
  const int R = d.R, R2 = 2 * R, NE = R2 * R2;
  const int per = (d.n[b] + nb - 1) / nb;
  const int x0 = bx_ * per, x1 = min(d.n[b], x0 + per);
  const double alpha = d.st->alpha_n;
  double *GN = smem;   // GR_{b+1}
  const double *gn = sm_slot(d, b + 1, S_GR);
  for (int t = threadIdx.x; t < NE; t += blockDim.x) GN[t] = (b == m - 1) ? ((t / R2 == t % R2) ? 1.0 : 0.0) : gn[t];
  const Grp q = make_grp(NE);
  double *C = smem + NE + q.g * (2 * NE + 2 * R * R);
  double *tmp = C + NE;
  double *sT = tmp + NE, *sX = sT + R * R;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // the first round's slices are fetched before the barrier, with their loads
  // in flight together with those of the staged matrices above
  {
    const int x = x0 + q.g;
    const bool act = (q.g < q.G) && (x < x1);
    const long long off = d.coff[b] + (long long)x * R * R;
    if (act)
      for (int t = q.tl; t < R * R; t += q.TPG) {
        sT[t] = glb(d.cores)[off + t];
        sX[t] = glb(d.X)[off + t];
      }
  }
  __syncthreads();
  for (int base = x0; base < x1; base += q.G) {
    const int x = base + q.g;
    const bool act = (q.g < q.G) && (x < x1);
    const long long off = d.coff[b] + (long long)x * R * R;
    if (base != x0) {
      if (act)
        for (int t = q.tl; t < R * R; t += q.TPG) {
          sT[t] = glb(d.cores)[off + t];
          sX[t] = glb(d.X)[off + t];
        }
      __syncthreads();
    }
    if (act) build_block(d, b, sT, sX, alpha, C, q.tl, q.TPG);
    __syncthreads();
    if (act)
      for (int t = q.tl; t < NE; t += q.TPG) {
        const int i = t / R2, jj = t % R2;
        double v = 0.0;
        for (int k = 0; k < R2; ++k) v += C[i * R2 + k] * GN[k * R2 + jj];
        tmp[t] = v;
      }
    __syncthreads();
    if (act) {
      int u = 0;
      for (int t = q.tl; t < NE; t += q.TPG, ++u) {
        const int i = t / R2, jj = t % R2;
        double v = 0.0;
        for (int k = 0; k < R2; ++k) v += tmp[i * R2 + k] * C[jj * R2 + k];
        acc[u] += v;
      }
    }
    __syncthreads();
  }
  double *red = smem + NE;
  __syncthreads();
  if (q.g < q.G) {
    int u = 0;
    for (int t = q.tl; t < NE; t += q.TPG, ++u) red[q.g * NE + t] = acc[u];
  }
  __syncthreads();
  auto mypart = glb(d.part) + (long long)bx_ * (R2 * (R2 + 1) / 2);
  for (int t = threadIdx.x; t < NE; t += blockDim.x) {
    const int a = t / R2, bb = t - a * R2;
    if (a > bb) continue;
    double v = 0.0;
    for (int g = 0; g < q.G; ++g) v += red[g * NE + t];
    mypart[sym_index(a, bb, R2)] = v;
  }
}

// Slice blocks of a right-Gram step on the matrix cores, for 2R <= 16 NT:
// the 2R x 2R matrices as NT x NT tiles of 16 x 16 (row layout of tiles.hpp),
// four waves each taking every fourth slice of the block:
//   M^T = GR_{b+1} C^T,   GR += C M^T
// tile by tile, (C^T)'s tiles serving both as the B operand of the first
// product and, transposed in place of C, as the A operand of the second
// (GR_{b+1} is symmetric).  Only the upper triangle's tiles of the sum are
// formed.  The waves' sums are added in wave order and the block's partial
// is written as rgram_body writes it (packed upper triangle), so the finish
// is shared.  The block's slices of T and X are staged in LDS four at a time.
template <int NT>
__global__ void __launch_bounds__(256) k_rgram_tiles(const Dev *__restrict__ dt, int b) {
  constexpr int NW = 4, W = 16 * NT;
  __shared__ double sTX[NW * 2 * 256];
  __shared__ double red[NW * W * W];
  const Dev &d = dt[blockIdx.y];
  const int bx_ = blockIdx.x, m = d.m;
  const int nb = nblocks_for(d.n[b], 4);
  if (d.st->done) return;
  if (bx_ >= nb) {
    const int lb = bx_ - nb;
    if (b == m - 1 && lb < nblocks_for(d.n[0], 4)) gram_first_cut(d, lb);
    return;
  }
  const int R = d.R, R2 = 2 * R, RR = R * R;
  const int per = (d.n[b] + nb - 1) / nb;
  const int x0 = bx_ * per, x1 = min(d.n[b], x0 + per);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, row0 = lane >> 4, col = lane & 15;
  const double alpha = d.st->alpha_n;
  // tiles of GR_{b+1} (the identity for the last core)
  d4 g[NT][NT];
  {
    const auto gn = glb((const double *)sm_slot(d, b + 1, S_GR));
#pragma unroll
    for (int P = 0; P < NT; ++P)
#pragma unroll
      for (int Q = 0; Q < NT; ++Q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * P + row0 + 4 * v, j = 16 * Q + col;
          g[P][Q][v] = (i < R2 && j < R2) ? (b == m - 1 ? (i == j ? 1.0 : 0.0) : gn[i * R2 + j]) : 0.0;
        }
  }
  d4 acc[NT][NT];
#pragma unroll
  for (int I = 0; I < NT; ++I)
#pragma unroll
    for (int J = 0; J < NT; ++J) acc[I][J] = zero4();
  for (int base = x0; base < x1; base += NW) {
    __syncthreads();   // the previous group's slices have been read
    const int cnt = min(NW, x1 - base);
    for (int e = threadIdx.x; e < cnt * RR; e += blockDim.x) {
      const int q = e / RR, t = e - q * RR;
      const long long off = d.coff[b] + (long long)(base + q) * RR + t;
      sTX[q * 2 * 256 + t] = glb(d.cores)[off];
      sTX[q * 2 * 256 + 256 + t] = glb(d.X)[off];
    }
    __syncthreads();
    if (w < cnt) {
      const double *T = sTX + w * 2 * 256, *X = T + 256;
      d4 ct[NT][NT];   // tile (K, J) of C^T: entry (r, c) = C(16 J + c, 16 K + r)
#pragma unroll
      for (int K = 0; K < NT; ++K)
#pragma unroll
        for (int J = 0; J < NT; ++J)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            ct[K][J][v] = block_core_entry(T, X, R, b, m, alpha, 16 * J + col, 16 * K + row0 + 4 * v);
      d4 mt[NT][NT];   // M^T = GR_{b+1} C^T
#pragma unroll
      for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int J = 0; J < NT; ++J) {
          d4 t = zero4();
#pragma unroll
          for (int K = 0; K < NT; ++K) t = mm16(g[K][I], ct[K][J], t);
          mt[I][J] = t;
        }
#pragma unroll
      for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int J = I; J < NT; ++J)
#pragma unroll
          for (int K = 0; K < NT; ++K) acc[I][J] = mm16(ct[K][I], mt[K][J], acc[I][J]);
    }
  }
  // the waves' sums, added in wave order, as the packed upper triangle
#pragma unroll
  for (int I = 0; I < NT; ++I)
#pragma unroll
    for (int J = I; J < NT; ++J)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[w * W * W + (16 * I + row0 + 4 * v) * W + 16 * J + col] = acc[I][J][v];
  __syncthreads();
  auto mypart = glb(d.part) + (long long)bx_ * (R2 * (R2 + 1) / 2);
  for (int t = threadIdx.x; t < R2 * R2; t += blockDim.x) {
    const int a = t / R2, bb = t - a * R2;
    if (a > bb) continue;
    double v = 0.0;
    for (int q = 0; q < NW; ++q) v += red[q * W * W + a * W + bb];
    mypart[sym_index(a, bb, R2)] = v;
  }
}

__global__ void __launch_bounds__(1024) k_rgram(const Dev *__restrict__ dt, int b) {
  __shared__ double smem[SMEM];
  rgram_body(dt[blockIdx.y], (int)blockIdx.x, b, smem);
}

// finish of a right-Gram step (one block): total GR_b and its pivoted Cholesky factor
__device__ __forceinline__ void rgram_fin_body(const Dev &d, int bx_, int b, double *smem_) {
  (void)bx_;
  (void)smem_;
  const int nb = nblocks_for(d.n[b], 4);
  if (d.st->done) return;
  double *smem = smem_;
  const int R = d.R, R2 = 2 * R, NE = R2 * R2;

  double *GR = sm_slot(d, b, S_GR);
  reduce_sym_partials(d.part, nb, R2, smem + 3072, smem + 5120, smem);
  for (int t = threadIdx.x; t < NE; t += blockDim.x) GR[t] = smem[3072 + t];
  // compress to the active indices [0, r_b) U [R, R + r_b)
  const int rb = d.r[b], na = 2 * rb;
  double *A = smem, *Fc = smem + 1024;
  for (int t = threadIdx.x; t < na * na; t += blockDim.x) {
    const int i = t / na, jj = t % na;
    const int gi = i < rb ? i : R + i - rb, gj = jj < rb ? jj : R + jj - rb;
    A[t] = smem[3072 + gi * R2 + gj];
  }
  __syncthreads();
  const int rank = block_pivoted_cholesky(A, na, Fc);
  double *F = sm_slot(d, b, S_F);
  for (int t = threadIdx.x; t < NE; t += blockDim.x) {
    const int gi = t / R2, col = t % R2;
    int i = -1;
    if (gi < rb) i = gi;
    else if (gi >= R && gi < R + rb) i = gi - R + rb;
    F[t] = (i >= 0 && col < rank) ? Fc[i * na + col] : 0.0;
  }
  if (threadIdx.x == 0) d.st->rank_f[b] = rank;
  if (b == 1) {
    // the first left cut: its Gram came from the first right-Gram launch
    __threadfence_block();
    __syncthreads();
    reduce_sym_partials(d.part + GB1_OFF, nblocks_for(d.n[0], 4), R2, smem, smem + 5120, smem + 1024);
    left_cut(d, 1, smem);
  }
}

__global__ void __launch_bounds__(1024) k_rgram_fin(const Dev *__restrict__ dt, int b) {
  __shared__ double smem[SMEM_CUT];
  rgram_fin_body(dt[blockIdx.y], (int)blockIdx.x, b, smem);
}

// ---------------------------------------------------------------------------
// left sweep of the retraction, cut i = 1..m-1 (core c = i-1)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void left_body(const Dev &d, int bx_, int i, double *smem_) {
  (void)bx_;
  (void)smem_;
  const int nb = nblocks_for(d.n[i - 1], 4);
  if (bx_ >= nb || d.st->done) return;
  double *smem = smem_;
  const int R = d.R, R2 = 2 * R, NE = R2 * R2, m = d.m, c = i - 1;
  const int per = (d.n[c] + nb - 1) / nb;
  const int x0 = bx_ * per, x1 = min(d.n[c], x0 + per);
  const double alpha = d.st->alpha_n;
  double *P = smem;    // R x 2R
  const double *ps = sm_slot(d, c, S_P);
  for (int t = threadIdx.x; t < R * R2; t += blockDim.x) P[t] = (c == 0) ? (t == 0 ? 1.0 : 0.0) : ps[t];
  const Grp q = make_grp(NE);
  double *C = smem + R * R2 + q.g * (NE + R * R2 + 2 * R * R);
  double *B = C + NE;
  double *sT = B + R * R2, *sX = sT + R * R;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // the first round's slices are fetched before the barrier, with their loads
  // in flight together with those of the staged matrices above
  {
    const int x = x0 + q.g;
    const bool act = (q.g < q.G) && (x < x1);
    const long long off = d.coff[c] + (long long)x * R * R;
    if (act)
      for (int t = q.tl; t < R * R; t += q.TPG) {
        sT[t] = glb(d.cores)[off + t];
        sX[t] = glb(d.X)[off + t];
      }
  }
  __syncthreads();
  for (int base = x0; base < x1; base += q.G) {
    const int x = base + q.g;
    const bool act = (q.g < q.G) && (x < x1);
    const long long off = d.coff[c] + (long long)x * R * R;
    if (base != x0) {
      if (act)
        for (int t = q.tl; t < R * R; t += q.TPG) {
          sT[t] = glb(d.cores)[off + t];
          sX[t] = glb(d.X)[off + t];
        }
      __syncthreads();
    }
    if (act) build_block(d, c, sT, sX, alpha, C, q.tl, q.TPG);
    __syncthreads();
    if (act)
      for (int t = q.tl; t < R * R2; t += q.TPG) {
        const int a = t / R2, jj = t % R2;
        double v = 0.0;
        for (int k = 0; k < R2; ++k) v += P[a * R2 + k] * C[k * R2 + jj];
        B[t] = v;
      }
    __syncthreads();
    if (act) {
      int u = 0;
      for (int t = q.tl; t < NE; t += q.TPG, ++u) {
        const int a = t / R2, bb = t % R2;
        double v = 0.0;
        for (int k = 0; k < R; ++k) v += B[k * R2 + a] * B[k * R2 + bb];
        acc[u] += v;
      }
    }
    __syncthreads();
  }
  double *red = smem + R * R2;
  __syncthreads();
  if (q.g < q.G) {
    int u = 0;
    for (int t = q.tl; t < NE; t += q.TPG, ++u) red[q.g * NE + t] = acc[u];
  }
  __syncthreads();
  auto mypart = glb(d.part) + (long long)bx_ * (R2 * (R2 + 1) / 2);
  for (int t = threadIdx.x; t < NE; t += blockDim.x) {
    const int a = t / R2, bb = t - a * R2;
    if (a > bb) continue;
    double v = 0.0;
    for (int g = 0; g < q.G; ++g) v += red[g * NE + t];
    mypart[sym_index(a, bb, R2)] = v;
  }
}

// Slice blocks of a left-sweep cut on the matrix cores, for 2R <= 16 NT: B =
// P_{i-1} C_c(x) has only R <= 16 nonzero rows, so it is one row of NT tiles,
// and G_B = sum_x B^T B is formed on the upper triangle's tiles, four waves
// each taking every fourth slice of the block.  P enters transposed (the A
// operand's transpose), C and B as themselves.  Partials as left_body's.
template <int NT>
__global__ void __launch_bounds__(256) k_left_tiles(const Dev *__restrict__ dt, int i) {
  constexpr int NW = 4, W = 16 * NT;
  __shared__ double sTX[NW * 2 * 256];
  __shared__ double red[NW * W * W];
  const Dev &d = dt[blockIdx.y];
  const int bx_ = blockIdx.x, m = d.m, c = i - 1;
  const int nb = nblocks_for(d.n[c], 4);
  if (bx_ >= nb || d.st->done) return;
  const int R = d.R, R2 = 2 * R, RR = R * R;
  const int per = (d.n[c] + nb - 1) / nb;
  const int x0 = bx_ * per, x1 = min(d.n[c], x0 + per);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, row0 = lane >> 4, col = lane & 15;
  const double alpha = d.st->alpha_n;
  // tiles (K, 0) of P^T: entry (r, q) = P(q, 16 K + r), P = e_0^T for the first core
  d4 ptr[NT];
  {
    const auto ps = glb((const double *)sm_slot(d, c, S_P));
#pragma unroll
    for (int K = 0; K < NT; ++K)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * K + row0 + 4 * v;
        ptr[K][v] = (col < R && r < R2) ? (c == 0 ? (col == 0 && r == 0 ? 1.0 : 0.0) : ps[col * R2 + r]) : 0.0;
      }
  }
  d4 acc[NT][NT];
#pragma unroll
  for (int I = 0; I < NT; ++I)
#pragma unroll
    for (int J = 0; J < NT; ++J) acc[I][J] = zero4();
  for (int base = x0; base < x1; base += NW) {
    __syncthreads();   // the previous group's slices have been read
    const int cnt = min(NW, x1 - base);
    for (int e = threadIdx.x; e < cnt * RR; e += blockDim.x) {
      const int q = e / RR, t = e - q * RR;
      const long long off = d.coff[c] + (long long)(base + q) * RR + t;
      sTX[q * 2 * 256 + t] = glb(d.cores)[off];
      sTX[q * 2 * 256 + 256 + t] = glb(d.X)[off];
    }
    __syncthreads();
    if (w < cnt) {
      const double *T = sTX + w * 2 * 256, *X = T + 256;
      d4 bt[NT];   // tiles (0, J) of B = P C
#pragma unroll
      for (int J = 0; J < NT; ++J) {
        d4 t = zero4();
#pragma unroll
        for (int K = 0; K < NT; ++K) {
          d4 ck;   // tile (K, J) of C
#pragma unroll
          for (int v = 0; v < 4; ++v)
            ck[v] = block_core_entry(T, X, R, c, m, alpha, 16 * K + row0 + 4 * v, 16 * J + col);
          t = mm16(ptr[K], ck, t);
        }
        bt[J] = t;
      }
#pragma unroll
      for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int J = I; J < NT; ++J) acc[I][J] = mm16(bt[I], bt[J], acc[I][J]);
    }
  }
#pragma unroll
  for (int I = 0; I < NT; ++I)
#pragma unroll
    for (int J = I; J < NT; ++J)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[w * W * W + (16 * I + row0 + 4 * v) * W + 16 * J + col] = acc[I][J][v];
  __syncthreads();
  auto mypart = glb(d.part) + (long long)bx_ * (R2 * (R2 + 1) / 2);
  for (int t = threadIdx.x; t < R2 * R2; t += blockDim.x) {
    const int a = t / R2, bb = t - a * R2;
    if (a > bb) continue;
    double v = 0.0;
    for (int q = 0; q < NW; ++q) v += red[q * W * W + a * W + bb];
    mypart[sym_index(a, bb, R2)] = v;
  }
}

__global__ void __launch_bounds__(1024) k_left(const Dev *__restrict__ dt, int i) {
  __shared__ double smem[SMEM];
  left_body(dt[blockIdx.y], (int)blockIdx.x, i, smem);
}

// finish of a left-sweep cut (one block): S = F^T (B^T B) F, eigen-decomposition,
// truncation to r_i: Tr_i and P_i
// Truncation at cut i from G_B (in smem[0, NE)) and F_i (sm slot): S = F^T G_B F,
// eigen-decomposition, Tr_i and P_i (one block).
__device__ __forceinline__ void left_cut(const Dev &d, int i, double *smem) {
  const int R = d.R, R2 = 2 * R, NE = R2 * R2;

  // last block: S = F^T GB F, eigen-decomposition, truncation to r_i
  double *GB = smem;                 // NE
  double *F = smem + 1024;           // 2R x rank (ld R2)
  double *T1 = smem + 2048;          // GB F (2R x rank); then the Cholesky factor of S
  double *S = smem + 3072;           // rank x rank; then eigen-solver scratch
  double *W = smem + 4096;           // eigenvectors of the graded matrix
  double *V = smem + 5120;           // eigenvectors of S (after the graded matrix, same area)
  double *w = smem + 6144;           // 32
  double *W2 = smem + SMEM;          // eigen-solver scratch (1024)
  const double *fs = sm_slot(d, i, S_F);
  for (int t = threadIdx.x; t < NE; t += blockDim.x) F[t] = fs[t];
  __syncthreads();
  const int rk = d.st->rank_f[i];
  const int ri = d.r[i];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = (rk < ri) ? 1 : 0;
  __syncthreads();
  if (bad) {
    if (threadIdx.x == 0) {
      d.st->status = -5;
      d.st->done = 1;
    }
    return;
  }
  for (int t = threadIdx.x; t < R2 * rk; t += blockDim.x) {
    const int a = t / rk, bcol = t % rk;
    double v = 0.0;
    for (int k = 0; k < R2; ++k) v += GB[a * R2 + k] * F[k * R2 + bcol];
    T1[a * rk + bcol] = v;
  }
  __syncthreads();
  // S is symmetric: each entry of the upper triangle is formed once and
  // mirrored, so the matrix handed to Jacobi is exactly symmetric
  for (int t = threadIdx.x; t < rk * rk; t += blockDim.x) {
    const int a = t / rk, bcol = t % rk;
    if (a > bcol) continue;
    double v = 0.0;
    for (int k = 0; k < R2; ++k) v += F[k * R2 + a] * T1[k * rk + bcol];
    S[a * rk + bcol] = v;
    S[bcol * rk + a] = v;
  }
  __syncthreads();
  block_psd_eig(S, rk, V, w, T1, V, W, S, W2);  // T1 is free once S is formed
  if (threadIdx.x == 0) {
    const double s0 = w[0];
    if (!(w[ri - 1] > TRUNC_MIN_EIG_RATIO * s0) || !isfinite(s0)) bad = 1;
  }
  __syncthreads();
  if (bad) {
    if (threadIdx.x == 0) {
      d.st->status = -5;
      d.st->done = 1;
    }
    return;
  }
  // Tr = F Z_r Sigma_r^{-1}  (2R x R; columns >= r_i zero)
  double *Tr = sm_slot(d, i, S_TR);
  double *TrL = smem + 3072;  // reuse S area: 2R x R
  for (int t = threadIdx.x; t < R2 * R; t += blockDim.x) {
    const int a = t / R, col = t % R;
    double v = 0.0;
    if (col < ri) {
      for (int k = 0; k < rk; ++k) v += F[a * R2 + k] * V[k * rk + col];
      v /= sqrt(w[col]);
    }
    TrL[t] = v;
    Tr[t] = v;
  }
  __syncthreads();
  // P_i = Tr^T GB  (R x 2R)
  double *Pn = sm_slot(d, i, S_P);
  for (int t = threadIdx.x; t < R * R2; t += blockDim.x) {
    const int a = t / R2, bcol = t % R2;
    double v = 0.0;
    for (int k = 0; k < R2; ++k) v += TrL[k * R + a] * GB[k * R2 + bcol];
    Pn[t] = v;
  }
}

__device__ __forceinline__ void left_fin_body(const Dev &d, int bx_, int i, double *smem_) {
  (void)bx_;
  (void)smem_;
  const int nb = nblocks_for(d.n[i - 1], 4);
  if (d.st->done) return;
  double *smem = smem_;
  reduce_sym_partials(d.part, nb, 2 * d.R, smem, smem + 5120, smem + 1024);
  left_cut(d, i, smem);
}

__global__ void __launch_bounds__(1024) k_left_fin(const Dev *__restrict__ dt, int i) {
  __shared__ double smem[SMEM_CUT];
  left_fin_body(dt[blockIdx.y], (int)blockIdx.x, i, smem);
}

// ---------------------------------------------------------------------------
// output: new cores T'_c(x) = P_c C_c(x) Tr_{c+1} (c < m-1), P_{m-1} C_{m-1}(x);
// stop-test reductions ||T'||^2 = ||T'_{m-1}||^2 and <T', T>
// ---------------------------------------------------------------------------
__device__ __forceinline__ void output_body(const Dev &d, int bx_, int init, double *smem_) {
  (void)bx_;
  (void)smem_;
  if (bx_ >= d.blk_off[d.m] || d.st->done) return;
  double *smem = smem_;
  int c, x0, x1;
  block_core(d, bx_, c, x0, x1);
  const int R = d.R, R2 = 2 * R, m = d.m, RR = R * R;
  const double alpha = d.st->alpha_n;
  double *P = smem;                  // R x 2R
  double *Tr = smem + R * R2;        // 2R x R
  double *Zc = Tr + R2 * R;          // R x R (second block of P_{m-1})
  const double *ps = sm_slot(d, c, S_P);
  const double *trs = sm_slot(d, c + 1, S_TR);
  for (int t = threadIdx.x; t < R * R2; t += blockDim.x) {
    P[t] = (c == 0) ? (t == 0 ? 1.0 : 0.0) : ps[t];
    if (c < m - 1) Tr[t] = trs[t];
  }
  for (int t = threadIdx.x; t < RR; t += blockDim.x)
    Zc[t] = (c == m - 1) ? sm_slot(d, m - 1, S_P)[(t / R) * R2 + R + t % R] : 0.0;
  const Grp q = make_grp(R * R2);
  double *C = Zc + RR + q.g * (R2 * R2 + R * R2 + 3 * RR);
  double *PC = C + R2 * R2;
  double *sT = PC + R * R2, *sX = sT + RR, *out = sX + RR;
  double nn = 0.0, cr = 0.0;
  // the first round's slices are fetched before the barrier, with their loads
  // in flight together with those of the staged matrices above
  {
    const int x = x0 + q.g;
    const bool act = (q.g < q.G) && (x < x1);
    const long long off = d.coff[c] + (long long)x * RR;
    if (act)
      for (int t = q.tl; t < RR; t += q.TPG) {
        sT[t] = glb(d.cores)[off + t];
        sX[t] = glb(d.X)[off + t];
      }
  }
  __syncthreads();
  for (int base = x0; base < x1; base += q.G) {
    const int x = base + q.g;
    const bool act = (q.g < q.G) && (x < x1);
    const long long off = d.coff[c] + (long long)x * RR;
    if (base != x0) {
      if (act)
        for (int t = q.tl; t < RR; t += q.TPG) {
          sT[t] = glb(d.cores)[off + t];
          sX[t] = glb(d.X)[off + t];
        }
      __syncthreads();
    }
    if (act) build_block(d, c, sT, sX, alpha, C, q.tl, q.TPG);
    __syncthreads();
    if (act)
      for (int t = q.tl; t < R * R2; t += q.TPG) {
        const int a = t / R2, jj = t % R2;
        double v = 0.0;
        for (int k = 0; k < R2; ++k) v += P[a * R2 + k] * C[k * R2 + jj];
        PC[t] = v;
      }
    __syncthreads();
    if (act)
      for (int t = q.tl; t < RR; t += q.TPG) {
        const int a = t / R, bcol = t % R;
        double v = 0.0;
        if (c < m - 1) {
          for (int k = 0; k < R2; ++k) v += PC[a * R2 + k] * Tr[k * R + bcol];
        } else {
          v = PC[a * R2 + bcol];
        }
        out[t] = v;
      }
    __syncthreads();
    if (act) {
      for (int t = q.tl; t < RR; t += q.TPG) {
        glb(d.cores)[off + t] = out[t];
        if (d.prec == PREC_MIXED) glb(d.cores32)[off + t] = (float)out[t];
      }
      if (c == 0 || c == m - 1) {
        const long long bo = (c == 0) ? (long long)x * R : (long long)d.n[0] * R + (long long)x * R;
        for (int a = q.tl; a < R; a += q.TPG) {
          const double v = (c == 0) ? out[a] : out[a * R];
          if (d.prec == PREC_MIXED) glb((float *)d.bnd)[bo + a] = (float)v;
          else glb((double *)d.bnd)[bo + a] = v;
        }
      }
      if (c == m - 1)
        for (int a = q.tl; a < R; a += q.TPG) {
          const double v = out[a * R];
          nn += v * v;
          double z = 0.0;
          for (int k = 0; k < R; ++k) z += Zc[a * R + k] * sT[k * R];
          cr += v * z;
        }
    }
    __syncthreads();
  }
  __shared__ double sbuf[16];
  nn = block_sum(nn, sbuf);
  cr = block_sum(cr, sbuf);
  if (threadIdx.x == 0) {
    glb(d.part)[2 * bx_] = nn;
    glb(d.part)[2 * bx_ + 1] = cr;
  }
}

// New cores on the matrix cores, for 2R <= 16 NT: T'_c(x) = P_c (C_c(x)
// Tr_{c+1}) (c < m-1) or P_{m-1} C_{m-1}(x), with C Tr formed first so that
// every operand is a tile as stored (C^T's tiles as the A operand of C Tr;
// P^T and Tr loaded as their tiles), four waves each taking every fourth
// slice of the block.  Writes and stopping-test partials as output_body's.
template <int NT>
__global__ void __launch_bounds__(256) k_output_tiles(const Dev *__restrict__ dt, int init) {
  constexpr int NW = 4;
  __shared__ double sTX[NW * 2 * 256];
  __shared__ double sbuf[16];
  (void)init;
  const Dev &d = dt[blockIdx.y];
  const int bx_ = blockIdx.x;
  if (bx_ >= d.blk_off[d.m] || d.st->done) return;
  int c, x0, x1;
  block_core(d, bx_, c, x0, x1);
  const int R = d.R, R2 = 2 * R, m = d.m, RR = R * R;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, row0 = lane >> 4, col = lane & 15;
  const double alpha = d.st->alpha_n;
  const auto ps = glb((const double *)sm_slot(d, c, S_P));
  const auto trs = glb((const double *)sm_slot(d, c + 1, S_TR));
  // tiles (K, 0) of P^T (entry (r, q) = P(q, 16 K + r)) and (L, 0) of Tr
  d4 ptr[NT], trt[NT];
#pragma unroll
  for (int K = 0; K < NT; ++K)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * K + row0 + 4 * v;
      ptr[K][v] = (col < R && r < R2) ? (c == 0 ? (col == 0 && r == 0 ? 1.0 : 0.0) : ps[col * R2 + r]) : 0.0;
      trt[K][v] = (c < m - 1 && col < R && r < R2) ? trs[r * R + col] : 0.0;
    }
  double nn = 0.0, cr = 0.0;
  for (int base = x0; base < x1; base += NW) {
    __syncthreads();   // the previous group's slices have been read
    const int cnt = min(NW, x1 - base);
    for (int e = threadIdx.x; e < cnt * RR; e += blockDim.x) {
      const int q = e / RR, t = e - q * RR;
      const long long off = d.coff[c] + (long long)(base + q) * RR + t;
      sTX[q * 2 * 256 + t] = glb(d.cores)[off];
      sTX[q * 2 * 256 + 256 + t] = glb(d.X)[off];
    }
    __syncthreads();
    if (w < cnt) {
      const int x = base + w;
      const double *T = sTX + w * 2 * 256, *X = T + 256;
      d4 out = zero4();
      if (c < m - 1) {
#pragma unroll
        for (int K = 0; K < NT; ++K) {
          d4 ctr = zero4();   // tile (K, 0) of C Tr
#pragma unroll
          for (int L = 0; L < NT; ++L) {
            d4 ctl;   // tile (L, K) of C^T: entry (r, q) = C(16 K + q, 16 L + r)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              ctl[v] = block_core_entry(T, X, R, c, m, alpha, 16 * K + col, 16 * L + row0 + 4 * v);
            ctr = mm16(ctl, trt[L], ctr);
          }
          out = mm16(ptr[K], ctr, out);
        }
      } else {
#pragma unroll
        for (int K = 0; K < NT; ++K) {
          d4 ck;   // tile (K, 0) of C
#pragma unroll
          for (int v = 0; v < 4; ++v)
            ck[v] = block_core_entry(T, X, R, c, m, alpha, 16 * K + row0 + 4 * v, col);
          out = mm16(ptr[K], ck, out);
        }
      }
      const long long off = d.coff[c] + (long long)x * RR;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = row0 + 4 * v;
        if (a < R && col < R) {
          glb(d.cores)[off + a * R + col] = out[v];
          if (d.prec == PREC_MIXED) glb(d.cores32)[off + a * R + col] = (float)out[v];
          long long bo = -1;
          if (c == 0 && a == 0) bo = (long long)x * R + col;
          if (c == m - 1 && col == 0) bo = (long long)d.n[0] * R + (long long)x * R + a;
          if (bo >= 0) {
            if (d.prec == PREC_MIXED) glb((float *)d.bnd)[bo] = (float)out[v];
            else glb((double *)d.bnd)[bo] = out[v];
          }
          if (c == m - 1 && col == 0) {
            double z = 0.0;   // (Z T_{m-1}(x))_a, Z the second block of P_{m-1}
            for (int k = 0; k < R; ++k) z += ps[a * R2 + R + k] * T[k * R];
            nn += out[v] * out[v];
            cr += out[v] * z;
          }
        }
      }
    }
  }
  nn = block_sum(nn, sbuf);
  cr = block_sum(cr, sbuf);
  if (threadIdx.x == 0) {
    glb(d.part)[2 * bx_] = nn;
    glb(d.part)[2 * bx_ + 1] = cr;
  }
}

__global__ void __launch_bounds__(1024) k_output(const Dev *__restrict__ dt, int init) {
  __shared__ double smem[SMEM];
  output_body(dt[blockIdx.y], (int)blockIdx.x, init, smem);
}

// finish of the output step (one block): relative change, iteration count, stop test
__device__ __forceinline__ void output_fin_body(const Dev &d, int bx_, int init, double *smem_) {
  (void)bx_;
  (void)smem_;
  const int nb = d.blk_off[d.m];
  if (d.st->done) return;
  __shared__ double sbuf[32];
  double a0 = 0.0, a1 = 0.0;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    a0 += glb(d.part)[2 * k];
    a1 += glb(d.part)[2 * k + 1];
  }
  block_sum2(a0, a1, sbuf);
  if (threadIdx.x == 0) finish_output(d, init, a0, a1);
}

__global__ void __launch_bounds__(1024) k_output_fin(const Dev *__restrict__ dt, int init) {
  output_fin_body(dt[blockIdx.y], (int)blockIdx.x, init, nullptr);
}

// ---------------------------------------------------------------------------
// cross Gram sweep with the truth: Z_{c+1} = sum_x A_c(x)^T Z_c B_c(x)
// mode 0: A = iterate, B = truth (relative error); mode 1: A = B = truth (||T*||^2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cross_body(const Dev &d, int bx_, int c, int mode, double *smem_) {
  (void)bx_;
  (void)smem_;
  const int nb = nblocks_for(d.n[c], 4);
  if (bx_ >= nb || !d.has_truth || (mode == 0 && !d.st->upd)) return;
  double *smem = smem_;
  const int R = d.R, RR = R * R, m = d.m;
  const int per = (d.n[c] + nb - 1) / nb;
  const int x0 = bx_ * per, x1 = min(d.n[c], x0 + per);
  const double *Acore = (mode == 0) ? d.cores : d.truth;
  double *Z = smem;
  const double *zs = sm_slot(d, c, S_ZT);
  for (int t = threadIdx.x; t < RR; t += blockDim.x) Z[t] = (c == 0) ? ((t / R == t % R) ? 1.0 : 0.0) : zs[t];
  const Grp q = make_grp(RR);
  double *sA = smem + RR + q.g * 3 * RR, *sB = sA + RR, *tmp = sB + RR;
  const int e = q.tl, ea = e / R, eb = e % R;
  double acc = 0.0;
  __syncthreads();
  for (int base = x0; base < x1; base += q.G) {
    const int x = base + q.g;
    const bool act = (q.g < q.G) && (x < x1);
    const long long off = d.coff[c] + (long long)x * RR;
    if (act)
      for (int t = q.tl; t < RR; t += q.TPG) {
        sA[t] = glb(Acore)[off + t];
        sB[t] = glb(d.truth)[off + t];
      }
    __syncthreads();
    if (act && e < RR) {
      double v = 0.0;
      for (int k = 0; k < R; ++k) v += Z[ea * R + k] * sB[k * R + eb];
      tmp[e] = v;
    }
    __syncthreads();
    if (act && e < RR) {
      double v = 0.0;
      for (int k = 0; k < R; ++k) v += sA[k * R + ea] * tmp[k * R + eb];
      acc += v;
    }
    __syncthreads();
  }
  double *red = smem + RR;
  __syncthreads();
  if (q.g < q.G && e < RR) red[q.g * RR + e] = acc;
  __syncthreads();
  auto mypart = glb(d.part) + (long long)bx_ * RR;
  for (int t = threadIdx.x; t < RR; t += blockDim.x) {
    double v = 0.0;
    for (int g = 0; g < q.G; ++g) v += red[g * RR + t];
    mypart[t] = v;
  }
}

__global__ void __launch_bounds__(1024) k_cross(const Dev *__restrict__ dt, int c, int mode) {
  __shared__ double smem[SMEM];
  cross_body(dt[blockIdx.y], (int)blockIdx.x, c, mode, smem);
}

// finish of a cross-Gram step (one block)
__device__ __forceinline__ void cross_fin_body(const Dev &d, int bx_, int c, int mode, double *smem_) {
  (void)bx_;
  (void)smem_;
  const int nb = nblocks_for(d.n[c], 4);
  if (!d.has_truth || (mode == 0 && !d.st->upd)) return;
  double *smem = smem_;
  const int R = d.R, RR = R * R, m = d.m;
  double *Zn = sm_slot(d, c + 1, S_ZT);
  reduce_partials(d.part, nb, RR, smem + 1024, smem);
  for (int t = threadIdx.x; t < RR; t += blockDim.x) Zn[t] = smem[1024 + t];
  __threadfence_block();
  __syncthreads();
  if (c == m - 1 && threadIdx.x == 0) {
    State *st = d.st;
    const double ip = Zn[0];
    if (mode == 1) {
      st->truth_sq = ip;
    } else {
      const double diff = fmax(0.0, st->tnorm_sq - 2.0 * ip + st->truth_sq);
      const double re = sqrt(diff) / sqrt(st->truth_sq);
      st->rel_error = re;
      const int it = st->iter - 1;
      if (it >= 0 && it < d.hist_cap) {
        d.hist[it].rel_error = re;
        d.hist[it].flags |= 2;
      }
      if (d.stop_rule == STOP_ERROR && re <= d.tol && !st->done) {
        st->status = 0;
        st->done = 1;
      }
    }
  }
}

__global__ void __launch_bounds__(1024) k_cross_fin(const Dev *__restrict__ dt, int c, int mode) {
  __shared__ double smem[SMEM];
  cross_fin_body(dt[blockIdx.y], (int)blockIdx.x, c, mode, smem);
}

// ---------------------------------------------------------------------------
// Steps with few slice blocks (small mode sizes): the blocks and the finish
// in one launch.  One workgroup runs the g slice blocks in turn and then the
// finish, which reads their partials after a workgroup barrier; arithmetic
// and summation order are those of the two-launch form, so results are the
// same bits.  This saves a launch and a kernel start per step on the long
// chains of dependent one-block steps that orders >= 4 with small n produce.
// ---------------------------------------------------------------------------
constexpr int FUSE_MAX = 2;   // slice blocks run in turn by one workgroup

__global__ void __launch_bounds__(1024) k_gram_fused(const Dev *__restrict__ dt, int j, int g) {
  __shared__ double smem[SMEM];
  const Dev &d = dt[blockIdx.y];
  for (int bx = 0; bx < g; ++bx) {
    gram_body(d, bx, j, smem);
    __syncthreads();
  }
  gram_fin_body(d, 0, j, smem);
}

__global__ void __launch_bounds__(1024) k_rgram_fused(const Dev *__restrict__ dt, int b, int g) {
  __shared__ double smem[SMEM_CUT];
  const Dev &d = dt[blockIdx.y];
  for (int bx = 0; bx < g; ++bx) {
    rgram_body(d, bx, b, smem);
    __syncthreads();
  }
  rgram_fin_body(d, 0, b, smem);
}

__global__ void __launch_bounds__(1024) k_left_fused(const Dev *__restrict__ dt, int i, int g) {
  __shared__ double smem[SMEM_CUT];
  const Dev &d = dt[blockIdx.y];
  for (int bx = 0; bx < g; ++bx) {
    left_body(d, bx, i, smem);
    __syncthreads();
  }
  left_fin_body(d, 0, i, smem);
}

__global__ void __launch_bounds__(1024) k_cross_fused(const Dev *__restrict__ dt, int c, int mode, int g) {
  __shared__ double smem[SMEM];
  const Dev &d = dt[blockIdx.y];
  for (int bx = 0; bx < g; ++bx) {
    cross_body(d, bx, c, mode, smem);
    __syncthreads();
  }
  cross_fin_body(d, 0, c, mode, smem);
}

// Whole sweeps in one launch when every step of the sweep is small (at most
// FUSE_MAX slice blocks): one workgroup per solve runs the steps in order
// with a workgroup barrier between dependent steps, in place of one launch
// per step.  Steps, arithmetic and order are those of the per-step launches.
__global__ void __launch_bounds__(1024) k_gram_sweep(const Dev *__restrict__ dt) {
  __shared__ double smem[SMEM];
  const Dev &d = dt[blockIdx.y];
  const int m = d.m;
  for (int j = 1; j <= m - 1; ++j) {
    const int g = nblocks_for(d.n[j - 1], 8) + nblocks_for(d.n[m - j], 8);
    for (int bx = 0; bx < g; ++bx) {
      gram_body(d, bx, j, smem);
      __syncthreads();
    }
    gram_fin_body(d, 0, j, smem);
    __syncthreads();
  }
}

__global__ void __launch_bounds__(1024) k_retract_sweep(const Dev *__restrict__ dt) {
  __shared__ double smem[SMEM_CUT];
  const Dev &d = dt[blockIdx.y];
  const int m = d.m;
  for (int b = m - 1; b >= 1; --b) {   // right Grams; b = 1 also truncates cut 1
    const int g = nblocks_for(d.n[b], 4) + (b == m - 1 ? nblocks_for(d.n[0], 4) : 0);
    for (int bx = 0; bx < g; ++bx) {
      rgram_body(d, bx, b, smem);
      __syncthreads();
    }
    rgram_fin_body(d, 0, b, smem);
    __syncthreads();
  }
  for (int i = 2; i <= m - 1; ++i) {   // the truncated left sweep
    const int g = nblocks_for(d.n[i - 1], 4);
    for (int bx = 0; bx < g; ++bx) {
      left_body(d, bx, i, smem);
      __syncthreads();
    }
    left_fin_body(d, 0, i, smem);
    __syncthreads();
  }
}

__global__ void __launch_bounds__(1024) k_cross_sweep(const Dev *__restrict__ dt, int mode) {
  __shared__ double smem[SMEM];
  const Dev &d = dt[blockIdx.y];
  for (int c = 0; c < d.m; ++c) {
    const int g = nblocks_for(d.n[c], 4);
    for (int bx = 0; bx < g; ++bx) {
      cross_body(d, bx, c, mode, smem);
      __syncthreads();
    }
    cross_fin_body(d, 0, c, mode, smem);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// launchers (grids sized for the largest member of the batch)
// ---------------------------------------------------------------------------
hipError_t launch_adaptive_step(const Batch &bt, hipStream_t s);

template <typename Fn>
static int max_over(const Batch &b, Fn f) {
  int v = 1;
  for (int i = 0; i < b.ns; ++i) v = std::max(v, f(b.host[i]));
  return v;
}

// phase 1: metric-weighted Gram sweeps and the tangent components
hipError_t launch_project(const Batch &bt, hipStream_t s) {
  const int m = bt.host[0].m, ns = bt.ns;
  int gmax = 1;
  for (int j = 1; j <= m - 1; ++j)
    gmax = std::max(gmax, max_over(bt, [&](const Dev &d) { return nblocks_for(d.n[j - 1], 8) + nblocks_for(d.n[m - j], 8); }));
  bool wave = false;
  const bool bf16 = bt.host[0].tangent_bf16 != 0;   // the whole batch shares the variant
  hipError_t ew = launch_gram_wave(bt, s, bf16 ? 0 : 1, wave);
  if (ew != hipSuccess) return ew;
  if (!wave && gmax <= FUSE_MAX) hipLaunchKernelGGL(k_gram_sweep, dim3(1, ns), dim3(1024), 0, s, bt.dt);
  for (int j = 1; j <= m - 1 && !wave && gmax > FUSE_MAX; ++j) {
    const int g = max_over(bt, [&](const Dev &d) { return nblocks_for(d.n[j - 1], 8) + nblocks_for(d.n[m - j], 8); });
    if (g <= FUSE_MAX) {
      hipLaunchKernelGGL(k_gram_fused, dim3(1, ns), dim3(1024), 0, s, bt.dt, j, g);
    } else {
      if (max_over(bt, [&](const Dev &d) { return d.R; }) <= 16)
        hipLaunchKernelGGL(k_gram_tiles, dim3(g, ns), dim3(256), 0, s, bt.dt, j);
      else
        hipLaunchKernelGGL(k_gram, dim3(g, ns), dim3(1024), 0, s, bt.dt, j);
      hipLaunchKernelGGL(k_gram_fin, dim3(1, ns), dim3(1024), 0, s, bt.dt, j);
    }
  }
  const int g = max_over(bt, [&](const Dev &d) { return d.blk_off[m]; });
  if (bf16)
    hipLaunchKernelGGL(k_tangent_bf16, dim3(g, ns), dim3(1024), 0, s, bt.dt);
  else if (!wave)   // the one-workgroup sweep formed the tangent itself
    hipLaunchKernelGGL(k_tangent, dim3(g, ns), dim3(1024), 0, s, bt.dt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_adaptive_step(bt, s);    // members with the adaptive step only
}

// phase 2: retraction sweeps (right Grams of W_l, then the truncated left sweep)
hipError_t launch_retract(const Batch &bt, hipStream_t s, int init, bool &output_done) {
  const int m = bt.host[0].m, ns = bt.ns;
  output_done = false;
  const hipError_t ew = launch_retract_wave(bt, s, init, output_done);
  if (output_done || ew != hipSuccess) return ew;
  int gmax = 1;
  for (int b = m - 1; b >= 1; --b)
    gmax = std::max(gmax, max_over(bt, [&](const Dev &d) {
      return nblocks_for(d.n[b], 4) + (b == m - 1 ? nblocks_for(d.n[0], 4) : 0);
    }));
  for (int i = 2; i <= m - 1; ++i)
    gmax = std::max(gmax, max_over(bt, [&](const Dev &d) { return nblocks_for(d.n[i - 1], 4); }));
  if (gmax <= FUSE_MAX) {
    hipLaunchKernelGGL(k_retract_sweep, dim3(1, ns), dim3(1024), 0, s, bt.dt);
    return hipGetLastError();
  }
  for (int b = m - 1; b >= 1; --b) {
    const int g = max_over(bt, [&](const Dev &d) {
      return nblocks_for(d.n[b], 4) + (b == m - 1 ? nblocks_for(d.n[0], 4) : 0);
    });
    if (g <= FUSE_MAX) {   // b = 1 also truncates cut 1
      hipLaunchKernelGGL(k_rgram_fused, dim3(1, ns), dim3(1024), 0, s, bt.dt, b, g);
    } else {
      const int rmax = max_over(bt, [&](const Dev &d) { return d.R; });
      if (rmax <= 8) hipLaunchKernelGGL(k_rgram_tiles<1>, dim3(g, ns), dim3(256), 0, s, bt.dt, b);
      else if (rmax <= 16) hipLaunchKernelGGL(k_rgram_tiles<2>, dim3(g, ns), dim3(256), 0, s, bt.dt, b);
      else hipLaunchKernelGGL(k_rgram, dim3(g, ns), dim3(1024), 0, s, bt.dt, b);
      hipLaunchKernelGGL(k_rgram_fin, dim3(1, ns), dim3(1024), 0, s, bt.dt, b);
    }
  }
  for (int i = 2; i <= m - 1; ++i) {
    const int g = max_over(bt, [&](const Dev &d) { return nblocks_for(d.n[i - 1], 4); });
    if (g <= FUSE_MAX) {
      hipLaunchKernelGGL(k_left_fused, dim3(1, ns), dim3(1024), 0, s, bt.dt, i, g);
    } else {
      const int rmax = max_over(bt, [&](const Dev &d) { return d.R; });
      if (rmax <= 8) hipLaunchKernelGGL(k_left_tiles<1>, dim3(g, ns), dim3(256), 0, s, bt.dt, i);
      else if (rmax <= 16) hipLaunchKernelGGL(k_left_tiles<2>, dim3(g, ns), dim3(256), 0, s, bt.dt, i);
      else hipLaunchKernelGGL(k_left, dim3(g, ns), dim3(1024), 0, s, bt.dt, i);
      hipLaunchKernelGGL(k_left_fin, dim3(1, ns), dim3(1024), 0, s, bt.dt, i);
    }
  }
  return hipGetLastError();
}

// phase 3: new cores and the stopping-test reductions
hipError_t launch_output(const Batch &bt, hipStream_t s, int init) {
  const int m = bt.host[0].m, ns = bt.ns;
  const int g = max_over(bt, [&](const Dev &d) { return d.blk_off[m]; });
  const int rmax = max_over(bt, [&](const Dev &d) { return d.R; });
  if (rmax <= 8) hipLaunchKernelGGL(k_output_tiles<1>, dim3(g, ns), dim3(256), 0, s, bt.dt, init);
  else if (rmax <= 16) hipLaunchKernelGGL(k_output_tiles<2>, dim3(g, ns), dim3(256), 0, s, bt.dt, init);
  else hipLaunchKernelGGL(k_output, dim3(g, ns), dim3(1024), 0, s, bt.dt, init);
  hipLaunchKernelGGL(k_output_fin, dim3(1, ns), dim3(1024), 0, s, bt.dt, init);
  return hipGetLastError();
}

hipError_t launch_dense_iteration(const Batch &bt, hipStream_t s, int init) {
  hipError_t e;
  if (!init && (e = launch_project(bt, s)) != hipSuccess) return e;
  bool done = false;
  if ((e = launch_retract(bt, s, init, done)) != hipSuccess) return e;
  return done ? hipSuccess : launch_output(bt, s, init);
}

// relative error against the truth (members without truth cores skip it)
hipError_t launch_truth_sweep(const Batch &bt, hipStream_t s, int mode) {
  const int m = bt.host[0].m, ns = bt.ns;
  bool any = false;
  for (int i = 0; i < ns; ++i) any = any || bt.host[i].has_truth;
  if (!any) return hipSuccess;
  int gmax = 1;
  for (int c = 0; c < m; ++c) gmax = std::max(gmax, max_over(bt, [&](const Dev &d) { return nblocks_for(d.n[c], 4); }));
  if (gmax <= FUSE_MAX) {
    hipLaunchKernelGGL(k_cross_sweep, dim3(1, ns), dim3(1024), 0, s, bt.dt, mode);
    return hipGetLastError();
  }
  for (int c = 0; c < m; ++c) {
    const int g = max_over(bt, [&](const Dev &d) { return nblocks_for(d.n[c], 4); });
    if (g <= FUSE_MAX) {
      hipLaunchKernelGGL(k_cross_fused, dim3(1, ns), dim3(1024), 0, s, bt.dt, c, mode, g);
    } else {
      hipLaunchKernelGGL(k_cross, dim3(g, ns), dim3(1024), 0, s, bt.dt, c, mode);
      hipLaunchKernelGGL(k_cross_fin, dim3(1, ns), dim3(1024), 0, s, bt.dt, c, mode);
    }
  }
  return hipGetLastError();
}

}  // namespace prgd
