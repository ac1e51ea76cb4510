// Internal definitions shared by the host runtime and the HIP kernels.
//
// Device layout of one solve (all sizes in elements):
//   cores   : core k stored slice-major, padded: [n_k][R][R] at coff[k], where
//             R >= max r_k is the padded slice dimension.  Entries outside the
//             true ranks are exactly zero.  Core 0 uses row 0 only, core m-1
//             column 0 only.
//   idx     : int32 [m][N], Omega grouped (stably sorted) by mode `sort_mode`,
//             or by its first ch_u mode indices for the one-pass chain kernel.
//   y       : observed values [N] in the working precision, same order.
//   Y       : gradient accumulator, layout of the cores (float or double).
//   X       : tangent components, layout of the cores (double).
//   s/omega : [sum n_k] mode-slice sums and metric factors at soff[k].
//   sm      : small-matrix workspace, SM_SLOTS slots of SLOT doubles per bond
//             b = 0..m (bond b sits between cores b-1 and b).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace prgd {

constexpr int MAXM = 32;
constexpr int RMAX = 16;
constexpr int SLOT = 4 * RMAX * RMAX;   // one 2R x 2R double matrix

// small-matrix slots per bond
enum Slot {
  S_GL = 0,   // weighted left Gram  GL_b = sum_x w T^T GL_{b-1} T        (R x R)
  S_GLI,      // inverse of GL_b on its active r_b x r_b block            (R x R)
  S_H,        // weighted right Gram H_b = sum_x w T H_{b+1} T^T          (R x R)
  S_HI,       // inverse of H_b                                           (R x R)
  S_TH,       // Theta_b = sum_x T_b^T Y_b  (core b)                       (R x R)
  S_GR,       // right Gram of the block TT W^{>=b}                       (2R x 2R)
  S_F,        // factor F_b with F F^T = GR_b (columns 0..rankF-1)       (2R x 2R)
  S_P,        // P_b = T'^{<=b,T} W^{<=b}                                (R x 2R)
  S_TR,       // truncation map Tr_b = F Z_r Sigma_r^{-1}                 (2R x R)
  S_ZT,       // cross Gram with the truth  T'^{<=b,T} T*^{<=b}           (R x R)
  SM_SLOTS
};

enum Precision { PREC_FP64 = 0, PREC_MIXED = 1 };
enum StepPolicy { STEP_THEORY = 0, STEP_CONST = 1, STEP_ADAPTIVE = 2 };
enum Metric { METRIC_DATA = 0, METRIC_EUCLIDEAN = 1 };
enum StopRule { STOP_RESIDUAL = 0, STOP_CHANGE = 1, STOP_ERROR = 2, STOP_NONE = 3 };

// counters used by the "last block finishes the reduction" pattern
enum Counter { C_SAMPLED = 0, C_GRAM, C_GR, C_LEFT, C_OUT, C_TRUTH, C_COUNT };

struct IterRecord {      // mirrors prgd_iter_info
  int iter;
  int flags;
  double rel_residual;
  double rel_change;
  double rel_error;
  double eps;
  double alpha;
};

struct State {
  double y_sq;          // ||y||^2
  double res_sq;        // ||R||^2 of the last evaluated iterate
  double eps_n;         // eps used to normalise the metric (eps_l or eps_fixed)
  double alpha_n;       // step in normalised units (see dense kernels)
  double tnorm_sq;      // ||T_l||^2
  double truth_sq;      // ||T*||^2
  double newnorm_sq;    // ||T_{l+1}||^2 (scratch of the output kernel)
  double cross;         // <T_{l+1}, T_l>
  double rel_res;
  double rel_change;
  double rel_error;
  int iter;             // completed iterations
  int done;             // 1: no further work
  int status;           // 0 ok/running, 1 not converged, <0 error
  int upd;              // 1: the current iteration produced T_{l+1}
  int rank_f[MAXM + 1]; // numerical rank of F_b
  unsigned counter[C_COUNT];
};

// order-3 sampled pass: per-workgroup partials (see sampled3.hip)
constexpr int KSEG = 8;   // segment slots per workgroup table
constexpr int SAMPLED3W_MAX_R = 4;   // padded ranks served by the one-wave-per-chunk variant
template <int R>
constexpr int sampled3w_group() { return R <= 2 ? 16 : 8; }   // batches of 64 samples per pipeline group in that variant
constexpr size_t SAMPLED3W_MAX_LDS = 57344;   // table bytes for that variant (>= 2 waves per CU)

struct S3 {
  long long chunk;       // samples per workgroup
  int nwg;
  int stage;             // 1: boundary vectors staged in LDS
  int wave;              // 1: one wave per chunk with a private table (low ranks)
  const int *vfirst;     // [nwg] first segment (middle-mode index) of each workgroup's chunk
  const int *vlast;      // [nwg] last segment of each chunk (wave variant)
  const int *blo;        // [n_1] first workgroup covering segment v (blo > bhi: empty segment)
  const int *bhi;        // [n_1]
  void *part_bnd;        // [nwg][L]: dT_0 [n_0 R] | dT_2 [n_2 R] | s_0 [n_0] | s_2 [n_2]
  void *part_seg;        // [nwg][KSEG][R*R + 1]: middle-core gradient pieces and s_1
                         // (wave variant: [nwg][2][R*R + 1], the chunk's first and last segments)
  void *ovf;             // [n_1][R*R + 1] overflow accumulator (zero between passes)
  double *part_rsq;      // [nwg]
};

// one mode of the mode-by-mode sampled pass (see sampled_modes.hip)
struct ModeTab {
  const int *idx;        // [m][N] Omega stably sorted by this mode
  const void *y;         // [N] observed values in that order (working precision)
  long long chunk;       // samples per workgroup
  int nwg;               // workgroups of this mode
  int wg0;               // first workgroup of this mode in the merged grid
  long long out0;        // first output of this mode in the merged reduction
  const int *vfirst;     // [nwg] first segment of each workgroup's chunk
  const int *blo;        // [n_k] first workgroup covering segment v (blo > bhi: empty)
  const int *bhi;        // [n_k]
  void *part_seg;        // [nwg][KSEG][R*R + 1] segment tables
  void *ovf;             // [n_k][R*R + 1] overflow accumulator (zero between passes)
};

struct Dev {
  int m;
  int R;                       // padded slice dimension
  int prec;
  int tangent_bf16;            // 1: tangent contractions on bfloat16 MFMAs (prec is then PREC_MIXED)
  int step_policy;
  int metric;                  // Metric
  int stop_rule;
  int max_iter;
  int sort_mode;
  int has_truth;
  long long N;
  double step;
  double eps_fixed;
  double tol;
  double p;                    // sampling ratio N / d*
  int n[MAXM];
  int r[MAXM + 1];
  long long coff[MAXM + 1];    // core offsets (padded)
  int soff[MAXM + 1];          // slice-vector offsets
  int blk_off[MAXM + 1];       // per-core block offsets for slice-parallel kernels
  int spb[MAXM];               // slices per block for core k
  const int *idx;
  const double *y64;
  const float *y32;
  double *cores;               // current iterate T_l (float64 master)
  float *cores32;              // float32 copy (mixed precision)
  const double *truth;         // truth cores (padded) or null
  void *Y;                     // gradient accumulator (float or double per prec)
  void *s;                     // slice sums (float or double per prec)
  double *omega;               // metric factors omega_k(x)
  void *bnd;                   // compact boundary vectors in the working precision:
                               // [n_0][R] row 0 of core 0, then [n_{m-1}][R] column 0 of core m-1
  double *X;                   // tangent components
  double *sm;                  // small matrices
  double *part;                // per-block partial results
  State *st;
  IterRecord *hist;
  int hist_cap;
  int use3;                    // 1: order-3 grouped sampled pass with the tables in q3
  int nb_sampled;              // grid of the any-order sampled pass
  // any-order sampled pass: modes whose gradient and slice sums fit in LDS are
  // accumulated per workgroup there (priv_off[k] = offset in the private
  // area, -1: global atomics) and reduced in a fixed order afterwards
  int priv_off[MAXM];
  int priv_len;                // elements of the private area per workgroup
  void *part_priv;             // [nb_sampled][priv_len] in the working precision
  // mode-by-mode sampled pass (no atomics; see sampled_modes.hip)
  int use_modes;
  int mt_wg;                   // workgroups of all modes together
  long long mt_out;            // outputs of all modes together (n_k (R*R + 1) each)
  const ModeTab *mt;           // device array [m]
  double *mp_rsq;              // [mt[0].nwg] partial ||R||^2
  // stored interfaces for the mode passes: one pass over the grouping-mode
  // copy writes, for every sample i of that copy and mode k, l_{k-1} into
  // ifl[k][i] and (r_{k+1}, residual) into ifr[k][i]; mode k's pass finds the
  // sample at its position p at i = rpos[k][p]
  int use_iface;
  int mt0_nwg;                 // workgroups of mode 0's pass (host copy of mt[0].nwg)
  const int *rpos;             // [m][N]
  void *ifl;                   // [m][N][R] in the working precision
  void *ifr;                   // [m][N][R + 1] in the working precision
  S3 q3;
  // one-pass sampled pass for small mode sizes (see sampled_chain.hip): Omega
  // sorted by its first ch_u mode indices and cut into chunks that keep that
  // prefix; every chunk writes one partial of ch_W elements
  int use_chain;
  int ch_u;                    // leading modes uniform within a chunk
  int ch_nchunks;
  const int *ch_start;         // [ch_nchunks] first sample of each chunk
  const int *ch_len;           // [ch_nchunks] samples of each chunk
  const int *ch_x;             // [ch_nchunks][ch_u] the chunk's shared leading indices
  void *ch_part;               // [ch_nchunks][width] in the working precision
  double *ch_rsq;              // [ch_nchunks] ||R||^2 of each chunk
  double *ch_red;              // [groups][outputs] first-stage sums
};

// Sizes of the one-pass chain kernel (sampled_chain.hip), shared with the host plan.
__host__ __device__ inline int chain_nx(int R) {
  const int xh = 16 / R;
  return xh * xh < 16 ? xh * xh : 16;
}
// LDS stride of one staged slice: R^2 plus 16 bytes, so that the slices of a
// core start on different banks
__host__ __device__ inline int chain_slice_stride(int R, int fbytes) { return R * R + 16 / fbytes; }
__host__ __device__ inline int chain_slot_width(int R) { return R * 68; }
// width of one chunk's partial (elements): tiles, slice sums, uniform gradients
__host__ __device__ inline int chain_part_width(int m, int u, int R) {
  const int nc = m - u;
  return nc * 256 + nc * chain_nx(R) + u * R * R;
}
__host__ __device__ inline int chain_nslots(int nc) { return nc - 2 > 1 ? nc - 2 : 1; }
// LDS elements of one wave's region: the parking slots, and with all of them
// granted also room for the wave's end-of-chunk sums (wr elements); with fewer
// slots the sums share the regions of all waves
__host__ __device__ inline int chain_region(int nslots, int nfull, int wr, int slotw) {
  const int sl = nslots * slotw;
  return nslots < nfull ? sl : (sl > wr ? sl : wr);
}

// Blocks of a slice-parallel reduction kernel over n slices: at least
// `target` slices per block and at most 128 blocks, so that the finishing
// block reads few partials.
__host__ __device__ inline int nblocks_for(int n, int target) {
  int per = (n + 127) / 128;
  if (per < target) per = target;
  int nb = (n + per - 1) / per;
  return nb < 1 ? 1 : nb;
}

// A set of solves advanced by the same launches.  Every kernel takes the
// device array `dt` of their descriptors and serves solve blockIdx.y; grids
// are sized for the largest member and surplus blocks return at once.  All
// members share m, R, the precision and the sampled-pass variant.
// Breakdown rule of the truncation at a cut.  The kept singular vectors come
// from the eigen-decomposition of S = M^T M, M the unfolding being truncated,
// so the eigenvalues carry rounding of about eps * w[0] and the new core
// M Z_r Sigma_r^{-1} departs from orthonormality by about
// eps * (sigma_1 / sigma_r)^2.  A kept singular value below 1e-6 of the
// largest (eigenvalue ratio 1e-12, orthonormality defect up to ~2e-4) stops
// the solve with PRGD_EBREAKDOWN rather than continuing on inaccurate cores.
// An SVD of M itself (Algorithm 1 as written) resolves ratios down to ~1e-15;
// this limit belongs to the Gram form only.
constexpr double TRUNC_MIN_EIG_RATIO = 1e-12;

// End of an iteration's output step (one thread), from a0 = ||T_{l+1}||^2 and
// a1 = <T_{l+1}, T_l>: the relative change ||T_{l+1} - T_l|| / max(1,
// ||T_l||) with ||T_l||^2 kept from the previous iteration, the iteration
// count, the history record and the change stopping rule (section 5.1).  At
// the initial rounding (init) only ||T_0||^2 is stored.
__device__ inline void finish_output(const Dev &d, int init, double a0, double a1) {
  State *st = d.st;
  if (init) {
    st->tnorm_sq = a0;
    return;
  }
  const double old = st->tnorm_sq;
  const int it = st->iter;
  const double diff = fmax(0.0, a0 - 2.0 * a1 + old);
  const double rc = sqrt(diff) / fmax(1.0, sqrt(old));
  st->rel_change = rc;
  st->tnorm_sq = a0;
  if (it < d.hist_cap) {
    d.hist[it].rel_change = rc;
    d.hist[it].flags |= 1;
  }
  st->iter = it + 1;
  st->upd = 1;
  if (d.stop_rule == STOP_CHANGE && rc <= d.tol) {
    st->status = 0;
    st->done = 1;
  }
}

struct Batch {
  const Dev *dt;     // device array [ns]
  const Dev *host;   // host copies [ns] (grid sizing)
  int ns;
};

// The kernels read their pointers from the descriptor table in device memory,
// so the compiler cannot tell that they point to global memory and would use
// flat (generic) instructions, which also occupy the LDS wait counter.  Hot
// accesses go through glb(), which states the address space.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *glb(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}

__host__ __device__ inline double *sm_slot(const Dev &d, int bond, int slot) {
  return d.sm + ((long long)bond * SM_SLOTS + slot) * SLOT;
}

}  // namespace prgd
