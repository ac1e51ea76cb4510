// Host-side state of one solve and the internal entry points shared by the
// single-solve API and the request server.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/prgd.h"
#include "prgd_internal.hpp"

namespace prgd {
// the sampled pass; `after_main` (may be null) is recorded after its main kernel
hipError_t launch_sampled(const Batch &bt, int diag, hipStream_t s, hipEvent_t after_main = nullptr);
int sampled_block_size(int m, int R, int prec);
hipError_t launch_eval(int m, int R, long long N, const int *idx, const double *cores, const long long *coff_dev,
                       double *out, hipStream_t s);
hipError_t launch_dense_iteration(const Batch &bt, hipStream_t s, int init);
hipError_t launch_project(const Batch &bt, hipStream_t s);
// retraction; output_done = true when the launch also formed the new cores
// and ran the stopping test (launch_output is then skipped)
hipError_t launch_retract(const Batch &bt, hipStream_t s, int init, bool &output_done);
// one-workgroup retraction for small ranks and slices, with the output step
// and its stopping test; used = false when it does not apply to the batch
// (nothing launched)
hipError_t launch_retract_wave(const Batch &bt, hipStream_t s, int init, bool &used);
// one-workgroup Gram sweep of the projection under the same conditions, with
// the tangent components when `tangent` is set
hipError_t launch_gram_wave(const Batch &bt, hipStream_t s, int tangent, bool &used);
hipError_t launch_output(const Batch &bt, hipStream_t s, int init);
hipError_t launch_truth_sweep(const Batch &bt, hipStream_t s, int mode);
// Stable grouping of Omega by one mode; perm (if not null) receives, for each
// grouped position, the position of that sample in the input.
hipError_t group_by_mode(int m, long long N, int mode, int n_mode, const int *idx_in, const void *values_in,
                         int values_fp64, int *idx_out, double *y64, float *y32, hipStream_t s,
                         int *perm = nullptr);
// pos[perm_b[p]] = p for p < N (inverse permutation of perm_b), then
// out[i] = pos[perm_a[i]]: for the sample at position i under perm_a, its
// position under perm_b
hipError_t compose_positions(long long N, const int *perm_a, const int *perm_b, int *scratch, int *out,
                             hipStream_t s);
hipError_t fill_f64(double *p, long long n, double v, hipStream_t s);
hipError_t fill_f32(float *p, long long n, float v, hipStream_t s);
hipError_t convert_f64_f32(const double *src, float *dst, long long n, hipStream_t s);
size_t sampled3_lds_bytes(int n1, int n3, int R, int prec, int stage);
size_t sampled3w_lds_bytes(int n1, int n3, int R, int prec);
hipError_t launch_sampled3(const Batch &bt, int diag, hipStream_t st, hipEvent_t after_main = nullptr);
hipError_t launch_sampled_modes(const Batch &bt, int diag, hipStream_t st, hipEvent_t after_main = nullptr);
size_t sampled_modes_lds_bytes(int R, int prec);
hipError_t launch_sampled_chain(const Batch &bt, int diag, hipStream_t st, hipEvent_t after_main = nullptr);
size_t chain_lds_bytes(int m, int u, const int *n, int R, int prec);
// Stable grouping of Omega by the mixed-radix key of its first u mode indices
// (mode 1 most significant); u = 0 copies it unchanged.
hipError_t group_by_prefix(int m, long long N, int u, const int *n, const int *idx_in, const void *values_in,
                           int values_fp64, int *idx_out, double *y64, float *y32, hipStream_t s);
// one PRGD iteration for every member of the batch (sampled pass, dense stage,
// truth sweep where a member has truth cores)
hipError_t enqueue_batch_iterations(const Batch &bt, int iters, hipStream_t s);
// copy each member's State into out[ns] (device)
hipError_t launch_gather_state(const Batch &bt, State *out, hipStream_t s);
}  // namespace prgd

struct prgd_solver_s {
  prgd::Dev d{};
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int m = 0, R = 0;
  std::vector<int> n, r;
  std::vector<long long> coff;
  long long N = 0;
  int64_t numel = 0;
  prgd::Dev *d_dev = nullptr;  // device copy of d (constant after create)
  bool has_truth = false;
  std::vector<void *> allocs;
  std::vector<size_t> sizes;  // bytes of each allocation
  size_t bytes = 0;           // device bytes held now
  size_t peak_bytes = 0;      // largest bytes held at once
  double last_seconds = 0.0;

  ~prgd_solver_s() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (void *p : allocs) (void)hipFree(p);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
  prgd::Batch batch() const { return prgd::Batch{d_dev, &d, 1}; }
  void release(void *p) {
    for (size_t i = 0; i < allocs.size(); ++i)
      if (allocs[i] == p) {
        (void)hipFree(p);
        bytes -= sizes[i];
        allocs.erase(allocs.begin() + i);
        sizes.erase(sizes.begin() + i);
        return;
      }
  }
  template <typename T>
  hipError_t alloc(T **p, long long count) {
    void *q = nullptr;
    const size_t nb = (size_t)std::max<long long>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&q, nb);
    if (e == hipSuccess) {
      allocs.push_back(q);
      sizes.push_back(nb);
      bytes += nb;
      peak_bytes = std::max(peak_bytes, bytes);
      *p = (T *)q;
    }
    return e;
  }
};

namespace prgd {
// prgd_create's body; `validated` skips the host validation (already done).
prgd_status solver_create(const prgd_desc *ds, prgd_solver *out, bool validated);
// prgd_create's host validation of shapes, ranks, options, index ranges,
// distinct multi-indices and finite values (host arrays).
prgd_status validate_desc(const prgd_desc *ds, const int32_t *idx_host, const void *vals_host);
// Upper bound of the device bytes a solve described by ds holds at any time
// during creation and iteration (-1 if the descriptor is invalid).
int64_t solver_footprint(const prgd_desc *ds);
// Record a failure message for prgd_last_error() and return st.
prgd_status set_error(prgd_status st, const char *msg);
// observation set in device memory: range, finiteness and repeated
// multi-index checks with sum of y^2 (validate.hip); sample counts per index
// value of one mode (mode >= 0) or per mixed-radix key of the first u modes
prgd_status check_obs_device(int m, long long N, const int *n, const int *idx, const void *val, int values_fp64,
                             double &ysq, hipStream_t s);
hipError_t count_obs_device(int m, long long N, const int *n, const int *idx, int mode, int u, long long bins,
                            std::vector<long long> &seg, hipStream_t s);
}  // namespace prgd
