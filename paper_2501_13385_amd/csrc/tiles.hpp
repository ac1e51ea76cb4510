// 16 x 16 float64 tiles on the matrix cores, one wave per tile.
//
// Row layout of a 16 x 16 matrix M: element v of lane l holds
// M((l >> 4) + 4 v, l & 15).  The float64 16x16x4 MFMA takes in step s the
// operand A(l & 15, 4 s + (l >> 4)) and the operand B(4 s + (l >> 4), l & 15):
// the first is element s of A^T in row layout, the second element s of B, and
// the product comes back in row layout.  So A B needs A^T and B as row-layout
// tiles; for a symmetric A, A^T is A.
#pragma once

#include <hip/hip_runtime.h>

namespace prgd {

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

// entry (i, j) of the block core C_c(x) of W_l = T_l - alpha xi from the
// slices T_c(x), X_c(x) (R x R each, row-major): middle cores
// [[T, 0], [X', T]], the first [X', T], the last [[T], [T + X']],
// X' = -alpha X; zero outside 2R x 2R
__device__ __forceinline__ double block_core_entry(const double *T, const double *X, int R, int c, int m, double alpha,
                                                   int i, int j) {
  if (i >= 2 * R || j >= 2 * R) return 0.0;
  const int ii = i < R ? i : i - R, jj = j < R ? j : j - R;
  const double t = T[ii * R + jj], xv = X[ii * R + jj];
  const bool qi = i >= R, qj = j >= R;
  if (c == 0) return qi ? 0.0 : (qj ? t : -alpha * xv);
  if (c == m - 1) return qj ? 0.0 : (qi ? t - alpha * xv : t);
  return qi ? (qj ? t : -alpha * xv) : (qj ? 0.0 : t);
}

}  // namespace prgd
