// Host runtime of the PRGD library: validation, device memory, launch
// sequencing and the C ABI declared in include/prgd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/prgd.h"
#include "prgd_internal.hpp"
#include "solver.hpp"


using namespace prgd;

namespace {

thread_local std::string g_err;

prgd_status fail(prgd_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

#define HIPCHECK(call)                                                                                   \
  do {                                                                                                   \
    hipError_t _e = (call);                                                                              \
    if (_e != hipSuccess) return fail(PRGD_EDEVICE, std::string(#call) + ": " + hipGetErrorString(_e)); \
  } while (0)

int padded_dim(int rmax) {
  static const int buckets[] = {2, 4, 6, 8, 10, 12, 16};
  for (int b : buckets)
    if (rmax <= b) return b;
  return -1;
}

bool checked_numel(int m, const int32_t *n, const int32_t *r, int64_t &out) {
  if (m < 2 || m > MAXM || !n || !r) return false;
  if (r[0] != 1 || r[m] != 1) return false;
  int64_t tot = 0;
  for (int k = 0; k < m; ++k) {
    if (n[k] < 1 || r[k] < 1 || r[k + 1] < 1) return false;
    tot += (int64_t)r[k] * n[k] * r[k + 1];
  }
  out = tot;
  return true;
}

// packed (a, x, b) row-major per core  ->  padded slice-major (x, a, b), R x R slices
void pack_cores(int m, const int *n, const int *r, int R, const double *src, std::vector<double> &dst,
                const std::vector<long long> &coff) {
  dst.assign(coff[m], 0.0);
  long long p = 0;
  for (int k = 0; k < m; ++k)
    for (int a = 0; a < r[k]; ++a)
      for (int x = 0; x < n[k]; ++x)
        for (int b = 0; b < r[k + 1]; ++b) dst[coff[k] + ((long long)x * R + a) * R + b] = src[p++];
}

void unpack_cores(int m, const int *n, const int *r, int R, const double *src, double *dst,
                  const std::vector<long long> &coff) {
  long long p = 0;
  for (int k = 0; k < m; ++k)
    for (int a = 0; a < r[k]; ++a)
      for (int x = 0; x < n[k]; ++x)
        for (int b = 0; b < r[k + 1]; ++b) dst[p++] = src[coff[k] + ((long long)x * R + a) * R + b];
}

}  // namespace

namespace {

// Any-order sampled pass: the modes whose gradient and slice sums are
// accumulated per workgroup in LDS (smallest first, while they fit next to
// the interface stack), their offsets in the private area, and the grid.
void sampled_plan(int m, const int *n, int R, int prec, long long N, int *off, long long &tot, int &nbs) {
  const int B = sampled_block_size(m, R, prec);
  const size_t f = prec == PREC_MIXED ? sizeof(float) : sizeof(double);
  const size_t stack = (size_t)(m - 1) * R * B * f;
  const size_t budget = (size_t)160 * 1024 - stack - 1024;
  std::vector<std::pair<long long, int>> sz;
  for (int k = 0; k < m; ++k) {
    const long long w = (k == 0 || k == m - 1) ? R : (long long)R * R;
    sz.push_back({(long long)n[k] * (w + 1), k});
  }
  std::sort(sz.begin(), sz.end());
  tot = 0;
  for (int k = 0; k < m; ++k) off[k] = -1;
  for (auto &p : sz)
    if ((size_t)(tot + p.first) * f <= budget) {
      off[p.second] = (int)tot;
      tot += p.first;
    }
  long long nb = (N + B - 1) / B;
  if (tot > 0) {
    // fewer, longer workgroups when each one writes a private area
    nb = (N + 4LL * B - 1) / (4LL * B);
    nb = std::min<long long>(nb, 1024);
    while (nb > 1 && (size_t)nb * tot * f > ((size_t)64 << 20)) nb /= 2;
  } else {
    nb = std::min<long long>(nb, 2048);
  }
  nbs = (int)std::max<long long>(nb, 1);
}

// The mode-by-mode sampled pass replaces the single pass when a middle mode
// would need global atomics (its accumulators do not fit in LDS) or has so
// few slices that LDS atomics from a whole workgroup would collide.
bool use_mode_passes(int m, const int *n, int R, int prec, long long N) {
  if (m < 3) return false;
  int off[MAXM];
  long long tot = 0;
  int nbs = 1;
  sampled_plan(m, n, R, prec, N, off, tot, nbs);
  for (int k = 1; k < m - 1; ++k)
    if (off[k] < 0 || n[k] < 32) return true;
  return false;
}

// One-pass chain kernel (orders >= 4, small mode sizes): the number u of
// leading modes that are uniform within a chunk, or -1 when it does not apply.
// Cores u..m-1 must fit one MFMA tile (n_k at most the kernel's slice range),
// the prefixes must leave at least CHAIN_SEG_MIN samples each on average, and
// the staged cores and per-wave slots must fit in LDS; the largest such u wins
// (more of the chain shared per chunk).
constexpr double CHAIN_SEG_MIN = 1024.0;
int chain_plan(int m, const int *n, int R, int prec, long long N) {
  if (m < 4 || (R != 2 && R != 4 && R != 8)) return -1;
  const int nx = chain_nx(R);
  int best = -1;
  double span = 1.0;
  for (int u = 0; u <= m - 2; ++u) {
    if (u > 0) {
      span *= (double)n[u - 1];
      if (span > (double)(1 << 22) || (double)N / span < CHAIN_SEG_MIN) break;
    }
    bool fit = m - u <= 16;
    for (int k = u; k < m && fit; ++k) fit = n[k] <= nx;
    if (fit && chain_lds_bytes(m, u, n, R, prec) <= (size_t)159 * 1024) best = u;
  }
  return best;
}

// largest chunk of the chain kernel: 8 batches of 64 per wave of 4, fewer for
// small Omega so that there are several hundred chunks
long long chain_chunk_max(long long N) {
  long long c = ((N / 512 + 63) / 64) * 64;
  return std::max<long long>(64, std::min<long long>(2048, c));
}

// workgroups of one mode's pass
long long mode_pass_wgs(long long N) { return std::min<long long>(1024, std::max<long long>(1, (N + 2047) / 2048)); }

// whether the mode passes read stored interfaces (option: 1 yes, -1 no, 0 when
// the order is at least 6 and the padded rank at most 8, so that 2m slice
// products instead of m (m - 1) outweigh writing and gathering the records,
// Omega is large enough to amortise one more launch, N >= 65536, and the
// records and position maps take at most 8 GiB)
bool use_stored_interfaces(int option, int m, int R, int prec, long long N) {
  if (option != 0) return option > 0;
  const long long f = prec == PREC_MIXED ? 4 : 8;
  return m >= 6 && R <= 8 && N >= 65536 && (long long)m * N * ((2LL * R + 1) * f + 4) <= (8LL << 30);
}

// true if two samples of Omega (SoA idx, m x N) share their multi-index
bool has_repeated_multi_index(int m, const int32_t *n, long long N, const int32_t *idx, bool exact) {
  constexpr int NB = 256;
  const int nth = (int)std::max<long long>(1, std::min<long long>(8, N / 65536));
  std::vector<uint64_t> key(N);
  auto bucket = [](uint64_t v) { return (int)((v * 0x9E3779B97F4A7C15ull) >> 56); };
  std::vector<std::vector<long long>> cnt(nth, std::vector<long long>(NB, 0));
  auto chunk = [&](int t, long long &lo, long long &hi) {
    lo = N * t / nth;
    hi = N * (t + 1) / nth;
  };
  auto run = [&](auto fn) {
    std::vector<std::thread> th;
    for (int t = 1; t < nth; ++t) th.emplace_back(fn, t);
    fn(0);
    for (auto &x : th) x.join();
  };
  run([&](int t) {
    long long lo, hi;
    chunk(t, lo, hi);
    for (long long j = lo; j < hi; ++j) {
      uint64_t v = 0;
      for (int k = 0; k < m; ++k) v = v * (uint64_t)n[k] + (uint64_t)idx[(long long)k * N + j];
      key[j] = v;
      ++cnt[t][bucket(v)];
    }
  });
  std::vector<long long> start(NB + 1, 0);
  std::vector<std::vector<long long>> off(nth, std::vector<long long>(NB, 0));
  for (int b = 0; b < NB; ++b) {
    long long p = start[b];
    for (int t = 0; t < nth; ++t) {
      off[t][b] = p;
      p += cnt[t][b];
    }
    start[b + 1] = p;
  }
  std::vector<std::pair<uint64_t, int>> item(N);
  run([&](int t) {
    long long lo, hi;
    chunk(t, lo, hi);
    for (long long j = lo; j < hi; ++j) item[off[t][bucket(key[j])]++] = {key[j], (int)j};
  });
  auto same = [&](int a, int b) {
    for (int k = 0; k < m; ++k)
      if (idx[(long long)k * N + a] != idx[(long long)k * N + b]) return false;
    return true;
  };
  std::vector<char> found(nth, 0);
  run([&](int t) {
    for (int b = t; b < NB && !found[t]; b += nth) {
      auto first = item.begin() + start[b], last = item.begin() + start[b + 1];
      std::sort(first, last);
      for (auto it = first + (first != last ? 1 : 0); it < last && !found[t]; ++it) {
        if (it->first != (it - 1)->first) continue;
        if (exact) {
          found[t] = 1;
          break;
        }
        // equal keys of distinct multi-indices are possible: compare the run
        auto e = it;
        while (e + 1 < last && (e + 1)->first == it->first) ++e;
        for (auto a = it - 1; a <= e && !found[t]; ++a)
          for (auto c = a + 1; c <= e && !found[t]; ++c) found[t] = same(a->second, c->second);
        it = e;
      }
    }
  });
  for (int t = 0; t < nth; ++t)
    if (found[t]) return true;
  return false;
}

// Checks of the descriptor; with idx and vals (host copies of Omega) also the
// observations (indices in range, values finite, no repeated multi-index).
prgd_status validate_host(const prgd_desc *ds, const int32_t *idx, const void *vals, int64_t &numel) {
  const int m = ds->order;
  if (m < 2 || m > MAXM) return fail(m < 2 ? PRGD_EINVAL : PRGD_ENOTSUP, "order must be in [2, 32]");
  if (!checked_numel(m, ds->mode_sizes, ds->tt_ranks, numel))
    return fail(PRGD_EINVAL, "invalid mode sizes or ranks (need n_k >= 1, r_0 = r_m = 1, r_k >= 1)");
  const int32_t *n = ds->mode_sizes, *r = ds->tt_ranks;
  for (int k = 1; k < m; ++k) {
    if (r[k] > RMAX) return fail(PRGD_ENOTSUP, "TT ranks above 16 are not supported by this build");
    double left = 1, right = 1;
    for (int i = 0; i < k; ++i) left *= n[i];
    for (int i = k; i < m; ++i) right *= n[i];
    if ((double)r[k] > left || (double)r[k] > right)
      return fail(PRGD_EINVAL, "rank r_" + std::to_string(k) + " exceeds the size of the separation");
  }
  const long long N = ds->n_obs;
  if (N < 1 || N >= (1LL << 31)) return fail(PRGD_EINVAL, "n_obs must be in [1, 2^31)");
  if (!(ds->tol >= 0.0) || ds->max_iter < 0) return fail(PRGD_EINVAL, "tol must be >= 0 and max_iter >= 0");
  if (!(ds->step > 0.0) || !std::isfinite(ds->step)) return fail(PRGD_EINVAL, "step must be positive");
  if (ds->precision != PRGD_PREC_FP64 && ds->precision != PRGD_PREC_MIXED && ds->precision != PRGD_PREC_MIXED_BF16)
    return fail(PRGD_EINVAL, "precision");
  if (ds->step_policy != PRGD_STEP_THEORY && ds->step_policy != PRGD_STEP_CONST &&
      ds->step_policy != PRGD_STEP_ADAPTIVE)
    return fail(PRGD_EINVAL, "step_policy");
  if (ds->metric != PRGD_METRIC_DATA && ds->metric != PRGD_METRIC_EUCLIDEAN) return fail(PRGD_EINVAL, "metric");
  if (ds->mode_interfaces < -1 || ds->mode_interfaces > 1) return fail(PRGD_EINVAL, "mode_interfaces must be -1, 0 or 1");
  if (ds->pass_kind < PRGD_PASS_AUTO || ds->pass_kind > PRGD_PASS_MODES) return fail(PRGD_EINVAL, "pass_kind");
  if (ds->step_policy == PRGD_STEP_CONST && ds->metric == PRGD_METRIC_DATA && !(ds->eps_fixed > 0.0))
    return fail(PRGD_EINVAL, "the constant step policy needs eps_fixed > 0");
  if (ds->stop_rule < PRGD_STOP_RESIDUAL || ds->stop_rule > PRGD_STOP_NONE) return fail(PRGD_EINVAL, "stop_rule");
  if (ds->stop_rule == PRGD_STOP_ERROR && !ds->truth_cores) return fail(PRGD_EINVAL, "STOP_ERROR needs truth_cores");
  if (!ds->init_cores) return fail(PRGD_EINVAL, "init_cores is required");
  if (ds->sort_mode < -1 || ds->sort_mode >= m) return fail(PRGD_EINVAL, "sort_mode");
  for (int64_t i = 0; i < numel; ++i)
    if (!std::isfinite(ds->init_cores[i])) return fail(PRGD_EINVAL, "init_cores has a non-finite entry");
  if (ds->truth_cores)
    for (int64_t i = 0; i < numel; ++i)
      if (!std::isfinite(ds->truth_cores[i])) return fail(PRGD_EINVAL, "truth_cores has a non-finite entry");
  if (!idx || !vals) return PRGD_OK;   // device-resident Omega: checked on the device
  // indices in range, values finite
  for (int k = 0; k < m; ++k) {
    const int32_t *row = idx + (long long)k * N;
    for (long long j = 0; j < N; ++j)
      if (row[j] < 0 || row[j] >= n[k])
        return fail(PRGD_EINVAL, "index out of range in mode " + std::to_string(k) + " at sample " + std::to_string(j));
  }
  for (long long j = 0; j < N; ++j) {
    const double v = ds->values_fp64 ? ((const double *)vals)[j] : (double)((const float *)vals)[j];
    if (!std::isfinite(v)) return fail(PRGD_EINVAL, "non-finite observed value at sample " + std::to_string(j));
  }
  // distinct multi-indices: a 64-bit key per sample (the linear index when it
  // fits, else that index modulo 2^64, verified on equal keys), spread over
  // 256 buckets by a multiplicative hash, each bucket sorted and scanned;
  // keys, bucketing and the per-bucket work run on up to 8 threads
  double dstar = 1;
  for (int k = 0; k < m; ++k) dstar *= n[k];
  const bool exact = dstar < 9.0e18;
  const bool dup = has_repeated_multi_index(m, n, N, idx, exact);
  if (dup) return fail(PRGD_EDUPLICATE, "Omega contains a repeated multi-index");
  return PRGD_OK;
}

hipError_t sampled_pass(prgd_solver s, int diag, hipEvent_t after_main = nullptr) {
  if (s->d.use3) return launch_sampled3(s->batch(), diag, s->stream, after_main);
  if (s->d.use_chain) return launch_sampled_chain(s->batch(), diag, s->stream, after_main);
  if (s->d.use_modes) return launch_sampled_modes(s->batch(), diag, s->stream, after_main);
  return launch_sampled(s->batch(), diag, s->stream, after_main);
}

prgd_status enqueue_iterations(prgd_solver s, int iters) {
  HIPCHECK(enqueue_batch_iterations(s->batch(), iters, s->stream));
  return PRGD_OK;
}

prgd_status read_state(prgd_solver s, State &st) {
  HIPCHECK(hipStreamSynchronize(s->stream));
  HIPCHECK(hipMemcpy(&st, s->d.st, sizeof(State), hipMemcpyDeviceToHost));
  return PRGD_OK;
}

void fill_report(prgd_solver s, const State &st, prgd_report *rep) {
  if (!rep) return;
  rep->iterations = st.iter;
  rep->rel_residual = st.rel_res;
  rep->rel_change = st.iter > 0 ? st.rel_change : NAN;
  rep->rel_error = s->has_truth ? st.rel_error : NAN;
  rep->seconds = s->last_seconds;
  if (st.status < 0) rep->status = st.status;
  else if (st.done) rep->status = st.status;
  else rep->status = PRGD_NOT_CONVERGED;
}

}  // namespace

namespace prgd {

prgd_status set_error(prgd_status st, const char *msg) { return fail(st, msg); }

hipError_t enqueue_batch_iterations(const Batch &bt, int iters, hipStream_t s) {
  const bool use3 = bt.host[0].use3 != 0, modes = bt.host[0].use_modes != 0, chain = bt.host[0].use_chain != 0;
  bool truth = false;
  for (int i = 0; i < bt.ns; ++i) truth = truth || bt.host[i].has_truth;
  for (int it = 0; it < iters; ++it) {
    hipError_t e = use3    ? launch_sampled3(bt, 0, s)
                   : chain ? launch_sampled_chain(bt, 0, s)
                   : modes ? launch_sampled_modes(bt, 0, s)
                           : launch_sampled(bt, 0, s);
    if (e != hipSuccess) return e;
    if ((e = launch_dense_iteration(bt, s, 0)) != hipSuccess) return e;
    if (truth && (e = launch_truth_sweep(bt, s, 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

int64_t solver_footprint(const prgd_desc *ds) {
  if (!ds) return -1;
  const int m = ds->order;
  int64_t numel = 0;
  if (!checked_numel(m, ds->mode_sizes, ds->tt_ranks, numel)) return -1;
  int rmax = 1;
  for (int k = 0; k <= m; ++k) rmax = std::max(rmax, (int)ds->tt_ranks[k]);
  const int R = padded_dim(rmax);
  if (R < 0) return -1;
  const int64_t N = ds->n_obs;
  int64_t pn = 0, soff = 0;
  for (int k = 0; k < m; ++k) {
    pn += (int64_t)ds->mode_sizes[k] * R * R;
    soff += ds->mode_sizes[k];
  }
  const bool mixed = ds->precision != PRGD_PREC_FP64;
  const int wprec = mixed ? PREC_MIXED : PREC_FP64;   // working precision of the sampled pass
  const int64_t f = mixed ? 4 : 8, vb = ds->values_fp64 ? 8 : 4;
  int64_t b = 0;
  b += 4 * m * N;                                     // grouped indices
  b += 8 * pn * 2 + (mixed ? 4 * pn * 2 : 8 * pn);    // cores, X, (cores32,) Y
  b += 8 * soff + f * soff;                           // omega, s
  b += 8LL * (m + 1) * SM_SLOTS * SLOT;               // small matrices
  b += 8LL << 20;                                     // partials
  b += (int64_t)sizeof(State) + (int64_t)sizeof(Dev) + (int64_t)sizeof(IterRecord) * (ds->max_iter + 1);
  b += f * N;                                         // values in the working precision
  b += f * (int64_t)(ds->mode_sizes[0] + ds->mode_sizes[m - 1]) * R;   // boundary vectors
  if (ds->truth_cores) b += 8 * pn;
  {                                                   // any-order pass (upper bound)
    int off[MAXM];
    long long tot = 0;
    int nbs = 1;
    std::vector<int> nv(ds->mode_sizes, ds->mode_sizes + m);
    const int cu = (ds->pass_kind == PRGD_PASS_MODES || m == 3) ? -1 : chain_plan(m, nv.data(), R, wprec, N);
    if (cu >= 0) {
      long long span = 1;
      for (int k = 0; k < cu; ++k) span *= nv[k];
      const int64_t nch = span + N / 64 + 1;                        // chunks (upper bound)
      b += nch * (chain_part_width(m, cu, R) * f + 16);             // partials, rsq, chunk table
      b += ((nch + 31) / 32) * soff * (R * R + 1) * 8;              // first-stage sums
      b += 8 * span + 12 * N;                                       // host-side segment scan, sort keys
    } else if (sampled_block_size(m, R, wprec) > 0) {
      if (use_mode_passes(m, nv.data(), R, wprec, N)) {
        const int64_t segw = (int64_t)R * R + 1, nwg = mode_pass_wgs(N);
        b += (int64_t)(m - 1) * (4 * m * N + f * N);      // sorted copies per mode
        for (int k = 0; k < m; ++k) b += nwg * (KSEG * segw * f + 4) + (int64_t)nv[k] * (segw * f + 8);
        b += 8 * nwg + (int64_t)m * (int64_t)sizeof(ModeTab) + 64 * 256 * 6 * m;
        if (use_stored_interfaces(ds->mode_interfaces, m, R, wprec, N))
          b += (int64_t)m * N * ((2 * R + 1) * f + 4) + 12 * N;   // records, position maps, permutations
      } else {
        sampled_plan(m, nv.data(), R, wprec, N, off, tot, nbs);
        b += (int64_t)nbs * tot * f;
      }
    }
  }
  if (m == 3) {                                       // order-3 tables (upper bound)
    const int64_t L = (int64_t)(ds->mode_sizes[0] + ds->mode_sizes[2]) * (R + 1);
    const int64_t segw = (int64_t)R * R + 1;
    b += 256 * (L + KSEG * segw) * f + (int64_t)ds->mode_sizes[1] * (segw * f + 8) + 256 * 12;
    if (R <= SAMPLED3W_MAX_R && L * 8 <= (int64_t)SAMPLED3W_MAX_LDS)   // one-wave chunks: up to 16 per CU
      b += 4096 * ((L + 2 * segw) * f + 12);
  }
  // transient during creation: unsorted copies, sort keys/permutations and
  // the radix-sort scratch
  if (!ds->mem_device) b += 4 * m * N + vb * N;
  b += 12 * N + 16 * N + (1LL << 20);
  b += 64 * 256;                                      // allocation granularity slack per buffer
  return b;
}

}  // namespace prgd

extern "C" {

int64_t prgd_cores_numel(int32_t m, const int32_t *n, const int32_t *r) {
  int64_t t = 0;
  return checked_numel(m, n, r, t) ? t : -1;
}

const char *prgd_last_error(void) { return g_err.c_str(); }

const char *prgd_status_str(prgd_status st) {
  switch (st) {
    case PRGD_OK: return "ok";
    case PRGD_NOT_CONVERGED: return "not converged (max_iter reached)";
    case PRGD_PENDING: return "pending";
    case PRGD_EINVAL: return "invalid argument";
    case PRGD_EDUPLICATE: return "duplicate multi-index in Omega";
    case PRGD_ENOMEM: return "out of memory";
    case PRGD_EDEVICE: return "HIP device error";
    case PRGD_EBREAKDOWN: return "numerical breakdown";
    case PRGD_ESTATE: return "invalid solver state";
    case PRGD_ENOTSUP: return "not supported by this build";
    default: return "unknown status";
  }
}

prgd_status prgd_create(const prgd_desc *ds, prgd_solver *out) { return solver_create(ds, out, false); }

}  // extern "C"

namespace prgd {

prgd_status validate_desc(const prgd_desc *ds, const int32_t *idx_host, const void *vals_host) {
  int64_t numel = 0;
  return validate_host(ds, idx_host, vals_host, numel);
}

prgd_status solver_create(const prgd_desc *ds, prgd_solver *out, bool validated) {
  if (!ds || !out) return fail(PRGD_EINVAL, "null descriptor or output handle");
  *out = nullptr;
  if (!ds->indices || !ds->values) return fail(PRGD_EINVAL, "indices and values are required");
  if (ds->order < 2 || ds->order > MAXM) return fail(ds->order < 2 ? PRGD_EINVAL : PRGD_ENOTSUP, "order must be in [2, 32]");
  if (ds->n_obs < 1 || ds->n_obs >= (1LL << 31)) return fail(PRGD_EINVAL, "n_obs must be in [1, 2^31)");
  const int m = ds->order;
  const long long N = ds->n_obs;
  const size_t vbytes = ds->values_fp64 ? sizeof(double) : sizeof(float);

  // Omega on the host, or (device buffers) checked and summarised on the
  // device below without a copy back: idx_h / val_h are then null
  const int32_t *idx_h = ds->mem_device ? nullptr : ds->indices;
  const void *val_h = ds->mem_device ? nullptr : ds->values;
  (void)vbytes;
  int64_t numel = 0;
  if (validated) {
    if (!checked_numel(m, ds->mode_sizes, ds->tt_ranks, numel)) return fail(PRGD_EINVAL, "invalid mode sizes or ranks");
  } else {
    prgd_status vs = validate_host(ds, idx_h, val_h, numel);
    if (vs != PRGD_OK) return vs;
  }

  prgd_solver s = new (std::nothrow) prgd_solver_s();
  if (!s) return fail(PRGD_ENOMEM, "host allocation failed");
  auto cleanup = [&](prgd_status st) {
    delete s;
    return st;
  };
  HIPCHECK(hipGetDevice(&s->device));
  if (ds->stream) {
    s->stream = (hipStream_t)ds->stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(fail(PRGD_EDEVICE, "hipStreamCreate failed"));
    s->own_stream = true;
  }
  // a device-resident Omega is checked (and y^2 summed) on the device
  double ysq_dev = 0.0;
  if (ds->mem_device) {
    const prgd_status vs =
        check_obs_device(m, N, ds->mode_sizes, ds->indices, ds->values, ds->values_fp64, ysq_dev, s->stream);
    if (vs != PRGD_OK) return cleanup(vs);
  }
  s->m = m;
  s->N = N;
  s->numel = numel;
  s->n.assign(ds->mode_sizes, ds->mode_sizes + m);
  s->r.assign(ds->tt_ranks, ds->tt_ranks + m + 1);
  int rmax = 1;
  for (int k = 0; k <= m; ++k) rmax = std::max(rmax, s->r[k]);
  s->R = padded_dim(rmax);
  const int R = s->R;
  s->coff.assign(m + 1, 0);
  for (int k = 0; k < m; ++k) s->coff[k + 1] = s->coff[k] + (long long)s->n[k] * R * R;
  const long long pn = s->coff[m];

  Dev &d = s->d;
  d.m = m;
  d.R = R;
  d.prec = ds->precision == PRGD_PREC_FP64 ? PREC_FP64 : PREC_MIXED;
  d.tangent_bf16 = ds->precision == PRGD_PREC_MIXED_BF16 ? 1 : 0;
  d.step_policy = ds->step_policy;
  d.metric = ds->metric;
  d.stop_rule = ds->stop_rule;
  d.max_iter = ds->max_iter;
  d.N = N;
  d.step = ds->step;
  d.eps_fixed = ds->eps_fixed;
  d.tol = ds->tol;
  double dstar = 1.0;
  for (int k = 0; k < m; ++k) dstar *= (double)s->n[k];
  d.p = (double)N / dstar;
  int sm = ds->sort_mode;
  if (sm < 0) {
    sm = 0;
    for (int k = 1; k < m; ++k)
      if ((long long)s->r[k] * s->r[k + 1] > (long long)s->r[sm] * s->r[sm + 1]) sm = k;
  }
  d.sort_mode = sm;
  int soff = 0;
  int blk = 0;
  for (int k = 0; k < m; ++k) {
    d.n[k] = s->n[k];
    d.coff[k] = s->coff[k];
    d.soff[k] = soff;
    soff += s->n[k];
    int spb = (s->n[k] + 255) / 256;
    if (spb < 4) spb = std::min(4, s->n[k]);
    d.spb[k] = spb;
    d.blk_off[k] = blk;
    blk += (s->n[k] + spb - 1) / spb;
  }
  d.coff[m] = s->coff[m];
  d.soff[m] = soff;
  d.blk_off[m] = blk;
  for (int k = 0; k <= m; ++k) d.r[k] = s->r[k];
  if (sampled_block_size(m, R, d.prec) == 0)
    return cleanup(fail(PRGD_ENOTSUP, "order x rank too large for the sampled-pass interface stack"));

  const bool mixed = d.prec == PREC_MIXED;
  // sampled-pass variant (decided here because the stored-interface form needs
  // the permutation of the first grouping)
  const bool use3_cand = m == 3 && sm == 1 && sampled3_lds_bytes(s->n[0], s->n[2], R, d.prec, 0) <= 163840;
  const int chain_u = ds->pass_kind == PRGD_PASS_MODES ? -1 : chain_plan(m, s->n.data(), R, d.prec, N);
  if (ds->pass_kind == PRGD_PASS_CHAIN && chain_u < 0)
    return cleanup(fail(PRGD_ENOTSUP, "the one-pass chain kernel does not apply to this shape"));
  const bool chain_cand = !use3_cand && chain_u >= 0;
  const bool modes_cand = !use3_cand && !chain_cand && use_mode_passes(m, s->n.data(), R, d.prec, N);
  const bool want_iface = modes_cand && use_stored_interfaces(ds->mode_interfaces, m, R, d.prec, N);
  int *perm0 = nullptr, *perm_k = nullptr, *inv_k = nullptr;
  // allocations
  int *idx_raw = nullptr, *idx_sorted = nullptr;
  void *val_raw = nullptr;
  double *y64 = nullptr;
  float *y32 = nullptr;
  auto A = [&](hipError_t e) { return e == hipSuccess; };
  bool ok = A(s->alloc(&idx_sorted, (long long)m * N)) && A(s->alloc(&d.cores, pn)) && A(s->alloc(&d.X, pn)) &&
            A(s->alloc(&d.omega, soff)) && A(s->alloc(&d.sm, (long long)(m + 1) * SM_SLOTS * SLOT)) &&
            A(s->alloc(&d.part, 1 << 20)) && A(s->alloc(&d.st, 1));
  d.hist_cap = ds->max_iter + 1;
  ok = ok && A(s->alloc(&d.hist, d.hist_cap));
  const long long nbnd = (long long)(s->n[0] + s->n[m - 1]) * R;
  if (mixed) {
    ok = ok && A(s->alloc(&y32, N)) && A(s->alloc(&d.cores32, pn)) && A(s->alloc((float **)&d.Y, pn)) &&
         A(s->alloc((float **)&d.s, soff)) && A(s->alloc((float **)&d.bnd, nbnd));
  } else {
    ok = ok && A(s->alloc(&y64, N)) && A(s->alloc((double **)&d.Y, pn)) && A(s->alloc((double **)&d.s, soff)) &&
         A(s->alloc((double **)&d.bnd, nbnd));
  }
  if (!ok) return cleanup(fail(PRGD_ENOMEM, "device allocation failed"));
  d.y64 = y64;
  d.y32 = y32;
  d.idx = idx_sorted;

  // observation set: to device, then grouped by the sort mode
  const int32_t *idx_dev = ds->indices;
  const void *val_dev = ds->values;
  if (!ds->mem_device) {
    if (!A(s->alloc(&idx_raw, (long long)m * N)) || !A(s->alloc((unsigned char **)&val_raw, (long long)N * vbytes)))
      return cleanup(fail(PRGD_ENOMEM, "device allocation failed"));
    hipError_t e1 = hipMemcpyAsync(idx_raw, ds->indices, (size_t)m * N * sizeof(int32_t), hipMemcpyHostToDevice, s->stream);
    hipError_t e2 = hipMemcpyAsync(val_raw, ds->values, (size_t)N * vbytes, hipMemcpyHostToDevice, s->stream);
    if (e1 != hipSuccess || e2 != hipSuccess) return cleanup(fail(PRGD_EDEVICE, "copy of Omega failed"));
    idx_dev = idx_raw;
    val_dev = val_raw;
  }
  if (want_iface && (!A(s->alloc(&perm0, N)) || !A(s->alloc(&perm_k, N)) || !A(s->alloc(&inv_k, N))))
    return cleanup(fail(PRGD_ENOMEM, "device allocation failed"));
  {
    hipError_t e = chain_cand ? group_by_prefix(m, N, chain_u, s->n.data(), idx_dev, val_dev, ds->values_fp64,
                                                idx_sorted, y64, y32, s->stream)
                              : group_by_mode(m, N, sm, s->n[sm], idx_dev, val_dev, ds->values_fp64, idx_sorted, y64,
                                              y32, s->stream, perm0);
    if (e != hipSuccess) return cleanup(fail(PRGD_EDEVICE, std::string("grouping Omega: ") + hipGetErrorString(e)));
  }

  // cores
  std::vector<double> packed;
  pack_cores(m, s->n.data(), s->r.data(), R, ds->init_cores, packed, s->coff);
  if (hipMemcpyAsync(d.cores, packed.data(), pn * sizeof(double), hipMemcpyHostToDevice, s->stream) != hipSuccess)
    return cleanup(fail(PRGD_EDEVICE, "copy of cores failed"));
  std::vector<double> tpacked;
  if (ds->truth_cores) {
    double *tr = nullptr;
    if (!A(s->alloc(&tr, pn))) return cleanup(fail(PRGD_ENOMEM, "device allocation failed"));
    pack_cores(m, s->n.data(), s->r.data(), R, ds->truth_cores, tpacked, s->coff);
    if (hipMemcpyAsync(tr, tpacked.data(), pn * sizeof(double), hipMemcpyHostToDevice, s->stream) != hipSuccess)
      return cleanup(fail(PRGD_EDEVICE, "copy of truth failed"));
    d.truth = tr;
    d.has_truth = 1;
    s->has_truth = true;
  }
  // state and constant small matrices
  State st0{};
  double ysq = ysq_dev;
  if (val_h)
    for (long long j = 0; j < N; ++j) {
      const double v = ds->values_fp64 ? ((const double *)val_h)[j] : (double)((const float *)val_h)[j];
      ysq += v * v;
    }
  st0.y_sq = ysq;
  st0.alpha_n = 0.0;
  st0.rel_change = NAN;
  st0.rel_error = NAN;
  st0.rel_res = NAN;
  std::vector<double> smh((size_t)(m + 1) * SM_SLOTS * SLOT, 0.0);
  auto slot = [&](int b, int sl) { return smh.data() + ((size_t)b * SM_SLOTS + sl) * SLOT; };
  for (int i = 0; i < R; ++i) {
    slot(0, S_GL)[i * R + i] = 1.0;
    slot(0, S_GLI)[i * R + i] = 1.0;
    slot(m, S_H)[i * R + i] = 1.0;
    slot(m, S_HI)[i * R + i] = 1.0;
  }
  if (hipMemcpyAsync(d.st, &st0, sizeof(State), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
      hipMemcpyAsync(d.sm, smh.data(), smh.size() * sizeof(double), hipMemcpyHostToDevice, s->stream) != hipSuccess)
    return cleanup(fail(PRGD_EDEVICE, "state upload failed"));
  if (fill_f64(d.X, pn, 0.0, s->stream) != hipSuccess || fill_f64(d.omega, soff, 1.0, s->stream) != hipSuccess)
    return cleanup(fail(PRGD_EDEVICE, "fill failed"));
  if (mixed) {
    if (fill_f32((float *)d.Y, pn, 0.0f, s->stream) != hipSuccess || fill_f32((float *)d.s, soff, 0.0f, s->stream) != hipSuccess)
      return cleanup(fail(PRGD_EDEVICE, "fill failed"));
  } else {
    if (fill_f64((double *)d.Y, pn, 0.0, s->stream) != hipSuccess || fill_f64((double *)d.s, soff, 0.0, s->stream) != hipSuccess)
      return cleanup(fail(PRGD_EDEVICE, "fill failed"));
  }
  // samples per index value of `mode` (or per mixed-radix key of the first u
  // modes when mode < 0) as offsets seg[0..bins]: from the host copy of Omega,
  // or counted on the device from the grouped copy
  auto counts = [&](int mode, int u, long long bins, std::vector<long long> &seg) -> bool {
    if (!idx_h) return count_obs_device(m, N, ds->mode_sizes, d.idx, mode, u, bins, seg, s->stream) == hipSuccess;
    seg.assign((size_t)bins + 1, 0);
    for (long long j = 0; j < N; ++j) {
      long long v = 0;
      if (mode >= 0) v = idx_h[(long long)mode * N + j];
      else
        for (int k = 0; k < u; ++k) v = v * s->n[k] + idx_h[(long long)k * N + j];
      seg[v + 1]++;
    }
    for (long long v = 0; v < bins; ++v) seg[v + 1] += seg[v];
    return true;
  };
  // order-3 grouped sampled pass: per-workgroup chunks of the samples sorted by the middle mode
  if (m == 3 && sm == 1 && sampled3_lds_bytes(s->n[0], s->n[2], R, d.prec, 0) <= 163840) {
    S3 &q = d.q3;
    q.stage = sampled3_lds_bytes(s->n[0], s->n[2], R, d.prec, 1) <= 163840 ? 1 : 0;
    // low ranks: one wave per chunk with its own table, as many chunks as can
    // be resident at once, each chunk long enough that its table partial is at
    // most half of the index/value bytes it reads
    const size_t wlds = sampled3w_lds_bytes(s->n[0], s->n[2], R, d.prec);
    q.wave = (R <= SAMPLED3W_MAX_R && wlds <= SAMPLED3W_MAX_LDS) ? 1 : 0;
    long long nwg;
    if (q.wave) {
      // resident waves per CU: the tables' LDS and the registers of the
      // deep load pipeline (about 390 VGPRs at R = 2, 180 at R = 4)
      const long long per_cu = std::min<long long>(R <= 2 ? 4 : 8, 163840 / (long long)wlds);
      const long long fb = mixed ? 4 : 8;
      const long long min_chunk = std::max<long long>(256, 2 * (long long)wlds * fb / 8 / (12 + fb));
      nwg = std::min<long long>(256 * per_cu, std::max<long long>(1, N / min_chunk));
    } else {
      nwg = std::min<long long>(256, std::max<long long>(1, (N + 63) / 64));
    }
    q.chunk = (N + nwg - 1) / nwg;
    nwg = (N + q.chunk - 1) / q.chunk;
    q.nwg = (int)nwg;
    const int n1 = s->n[1];
    std::vector<long long> seg;
    if (!counts(1, 0, n1, seg)) return cleanup(fail(PRGD_EDEVICE, "counting the middle-mode slices failed"));
    std::vector<int> vfirst(nwg), vlast(nwg), blo(n1), bhi(n1);
    for (long long b = 0; b < nwg; ++b) {
      const long long j0 = b * q.chunk, jl = std::min(N, j0 + q.chunk) - 1;
      vfirst[b] = (int)(std::upper_bound(seg.begin(), seg.end(), j0) - seg.begin()) - 1;
      vlast[b] = (int)(std::upper_bound(seg.begin(), seg.end(), jl) - seg.begin()) - 1;
    }
    for (int v = 0; v < n1; ++v) {
      if (seg[v + 1] > seg[v]) {
        blo[v] = (int)(seg[v] / q.chunk);
        bhi[v] = (int)((seg[v + 1] - 1) / q.chunk);
      } else {
        blo[v] = 1;
        bhi[v] = 0;
      }
    }
    const size_t f = mixed ? 4 : 8;
    const long long L = (long long)(s->n[0] + s->n[2]) * (R + 1);
    const long long segw = (long long)R * R + 1;
    int *dvf = nullptr, *dvl = nullptr, *dlo = nullptr, *dhi = nullptr;
    unsigned char *pbnd = nullptr, *pseg = nullptr, *povf = nullptr;
    const long long nslot = q.wave ? 2 : KSEG;
    if (!A(s->alloc(&dvf, nwg)) || !A(s->alloc(&dvl, nwg)) || !A(s->alloc(&dlo, n1)) || !A(s->alloc(&dhi, n1)) ||
        !A(s->alloc(&pbnd, nwg * L * (long long)f)) || !A(s->alloc(&pseg, nwg * nslot * segw * (long long)f)) ||
        !A(s->alloc(&povf, n1 * segw * (long long)f)) || !A(s->alloc(&q.part_rsq, nwg)))
      return cleanup(fail(PRGD_ENOMEM, "device allocation failed"));
    if (hipMemcpyAsync(dvf, vfirst.data(), nwg * sizeof(int), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(dvl, vlast.data(), nwg * sizeof(int), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(dlo, blo.data(), n1 * sizeof(int), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(dhi, bhi.data(), n1 * sizeof(int), hipMemcpyHostToDevice, s->stream) != hipSuccess)
      return cleanup(fail(PRGD_EDEVICE, "upload of the segment map failed"));
    const long long novf = n1 * segw;
    hipError_t fe = mixed ? fill_f32((float *)povf, novf, 0.0f, s->stream) : fill_f64((double *)povf, novf, 0.0, s->stream);
    if (fe != hipSuccess) return cleanup(fail(PRGD_EDEVICE, "fill failed"));
    q.vfirst = dvf;
    q.vlast = dvl;
    q.blo = dlo;
    q.bhi = dhi;
    q.part_bnd = pbnd;
    q.part_seg = pseg;
    q.ovf = povf;
    d.use3 = 1;
  }
  // any-order sampled pass: grid, and the modes accumulated per workgroup in LDS
  for (int k = 0; k < MAXM; ++k) d.priv_off[k] = -1;
  d.priv_len = 0;
  d.part_priv = nullptr;
  d.nb_sampled = 1;
  d.use_modes = 0;
  d.mt = nullptr;
  d.mp_rsq = nullptr;
  d.mt_wg = 0;
  d.mt_out = 0;
  d.use_iface = 0;
  d.rpos = nullptr;
  d.ifl = nullptr;
  d.ifr = nullptr;
  d.use_chain = 0;
  d.ch_u = 0;
  d.ch_nchunks = 0;
  d.ch_start = d.ch_len = d.ch_x = nullptr;
  d.ch_part = nullptr;
  d.ch_rsq = d.ch_red = nullptr;
  if (!d.use3 && chain_cand) {
    // segments of equal leading indices (the sort above is stable and by
    // that key, so segment v occupies [seg[v], seg[v+1])), cut into chunks
    const int u = chain_u;
    long long span = 1;
    for (int k = 0; k < u; ++k) span *= s->n[k];
    std::vector<long long> seg;
    if (!counts(-1, u, span, seg)) return cleanup(fail(PRGD_EDEVICE, "counting the index prefixes failed"));
    // the largest chunk: from the base size up to four times it, the one
    // whose chunk count fills the last round of resident workgroups best (the
    // chunks of a launch run in rounds of one workgroup per CU and LDS slot;
    // 1,043 chunks on 256 CUs would take five rounds for four rounds of work)
    const long long resident =
        256LL * std::max<long long>(1, (long long)(163840 / std::max<size_t>(1, chain_lds_bytes(m, u, s->n.data(), R, d.prec))));
    auto chunks_for = [&](long long cm) {
      long long c = 0;
      for (long long v = 0; v < span; ++v)
        if (seg[v + 1] > seg[v]) c += (seg[v + 1] - seg[v] + cm - 1) / cm;
      return c;
    };
    const long long c0 = chain_chunk_max(N);
    long long cmax = c0;
    double best_fill = -1.0;
    for (long long cm = c0; cm <= 4 * c0; cm += c0 / 4 > 64 ? c0 / 4 : 64) {
      const long long c = chunks_for(cm);
      const double fill = (double)c / (double)(((c + resident - 1) / resident) * resident);
      if (fill > best_fill + 0.02) {
        best_fill = fill;
        cmax = cm;
      }
    }
    std::vector<int> cstart, clen, cx;
    for (long long v = 0; v < span; ++v) {
      const long long a = seg[v], b = seg[v + 1];
      if (b <= a) continue;
      const long long pieces = (b - a + cmax - 1) / cmax;
      for (long long p = 0; p < pieces; ++p) {
        const long long lo = a + (b - a) * p / pieces, hi = a + (b - a) * (p + 1) / pieces;
        cstart.push_back((int)lo);
        clen.push_back((int)(hi - lo));
        // the prefix x_0 .. x_{u-1} of segment v (mixed radix, mode 1 most significant)
        long long r = v;
        const size_t at = cx.size();
        cx.resize(at + (size_t)u);
        for (int k = u - 1; k >= 0; --k) {
          cx[at + k] = (int)(r % s->n[k]);
          r /= s->n[k];
        }
      }
    }
    const int nch = (int)cstart.size();
    const long long W = chain_part_width(m, u, R);
    const long long nout = (long long)soff * (R * R + 1);
    const long long ng = (nch + 31) / 32;
    int *dst = nullptr, *dln = nullptr, *dcx = nullptr;
    unsigned char *pp = nullptr;
    if (!A(s->alloc(&dst, nch)) || !A(s->alloc(&dln, nch)) || !A(s->alloc(&dcx, std::max<long long>(1, (long long)nch * u))) ||
        !A(s->alloc(&pp, (long long)nch * W * (mixed ? 4 : 8))) ||
        !A(s->alloc(&d.ch_rsq, nch)) || !A(s->alloc(&d.ch_red, ng * nout)))
      return cleanup(fail(PRGD_ENOMEM, "device allocation failed"));
    if (hipMemcpyAsync(dst, cstart.data(), nch * sizeof(int), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(dln, clen.data(), nch * sizeof(int), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        (u > 0 && hipMemcpyAsync(dcx, cx.data(), cx.size() * sizeof(int), hipMemcpyHostToDevice, s->stream) != hipSuccess) ||
        hipStreamSynchronize(s->stream) != hipSuccess)
      return cleanup(fail(PRGD_EDEVICE, "upload of the chunk table failed"));
    d.ch_start = dst;
    d.ch_len = dln;
    d.ch_x = dcx;
    d.ch_part = pp;
    d.ch_u = u;
    d.ch_nchunks = nch;
    d.use_chain = 1;
  } else if (!d.use3 && modes_cand) {
    const long long f = mixed ? 4 : 8;
    const long long segw = (long long)R * R + 1;
    std::vector<ModeTab> mt(m);
    int *rpos = nullptr;
    unsigned char *ifl = nullptr, *ifr = nullptr;
    if (want_iface && (!A(s->alloc(&rpos, (long long)m * N)) || !A(s->alloc(&ifl, (long long)m * N * R * f)) ||
                       !A(s->alloc(&ifr, (long long)m * N * (R + 1) * f))))
      return cleanup(fail(PRGD_ENOMEM, "device allocation failed"));
    int wg0 = 0;
    long long out0 = 0;
    for (int k = 0; k < m; ++k) {
      ModeTab &t = mt[k];
      const int nk = s->n[k];
      if (k == sm) {
        t.idx = idx_sorted;
        t.y = mixed ? (const void *)y32 : (const void *)y64;
      } else {
        int *ip = nullptr;
        double *y6 = nullptr;
        float *y3 = nullptr;
        if (!A(s->alloc(&ip, (long long)m * N)) || !(mixed ? A(s->alloc(&y3, N)) : A(s->alloc(&y6, N))))
          return cleanup(fail(PRGD_ENOMEM, "device allocation failed"));
        hipError_t e = group_by_mode(m, N, k, nk, idx_dev, val_dev, ds->values_fp64, ip, y6, y3, s->stream,
                                     want_iface ? perm_k : nullptr);
        if (e != hipSuccess) return cleanup(fail(PRGD_EDEVICE, std::string("grouping Omega: ") + hipGetErrorString(e)));
        t.idx = ip;
        t.y = mixed ? (const void *)y3 : (const void *)y6;
      }
      if (want_iface) {   // which sample of the grouping-mode copy sits at each position of this mode's copy
        hipError_t e = compose_positions(N, k == sm ? perm0 : perm_k, perm0, inv_k, rpos + (long long)k * N, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);   // perm_k is reused by the next mode
        if (e != hipSuccess) return cleanup(fail(PRGD_EDEVICE, std::string("position maps: ") + hipGetErrorString(e)));
      }
      long long nwg = mode_pass_wgs(N);
      t.chunk = (N + nwg - 1) / nwg;
      nwg = (N + t.chunk - 1) / t.chunk;
      t.nwg = (int)nwg;
      t.wg0 = wg0;
      wg0 += (int)nwg;
      t.out0 = out0;
      out0 += (long long)nk * segw;
      std::vector<long long> seg;
      if (!counts(k, 0, nk, seg)) return cleanup(fail(PRGD_EDEVICE, "counting the mode slices failed"));
      std::vector<int> vfirst(nwg), blo(nk), bhi(nk);
      for (long long b = 0; b < nwg; ++b)
        vfirst[b] = (int)(std::upper_bound(seg.begin(), seg.end(), b * t.chunk) - seg.begin()) - 1;
      for (int v = 0; v < nk; ++v) {
        if (seg[v + 1] > seg[v]) {
          blo[v] = (int)(seg[v] / t.chunk);
          bhi[v] = (int)((seg[v + 1] - 1) / t.chunk);
        } else {
          blo[v] = 1;
          bhi[v] = 0;
        }
      }
      int *dvf = nullptr, *dlo = nullptr, *dhi = nullptr;
      unsigned char *pseg = nullptr, *povf = nullptr;
      if (!A(s->alloc(&dvf, nwg)) || !A(s->alloc(&dlo, nk)) || !A(s->alloc(&dhi, nk)) ||
          !A(s->alloc(&pseg, nwg * KSEG * segw * f)) || !A(s->alloc(&povf, (long long)nk * segw * f)))
        return cleanup(fail(PRGD_ENOMEM, "device allocation failed"));
      if (hipMemcpy(dvf, vfirst.data(), nwg * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(dlo, blo.data(), nk * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(dhi, bhi.data(), nk * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(PRGD_EDEVICE, "upload of the segment maps failed"));
      hipError_t fe = mixed ? fill_f32((float *)povf, (long long)nk * segw, 0.0f, s->stream)
                            : fill_f64((double *)povf, (long long)nk * segw, 0.0, s->stream);
      if (fe != hipSuccess) return cleanup(fail(PRGD_EDEVICE, "fill failed"));
      t.vfirst = dvf;
      t.blo = dlo;
      t.bhi = dhi;
      t.part_seg = pseg;
      t.ovf = povf;
    }
    ModeTab *dmt = nullptr;
    if (!A(s->alloc(&dmt, m)) || !A(s->alloc(&d.mp_rsq, mt[0].nwg)))
      return cleanup(fail(PRGD_ENOMEM, "device allocation failed"));
    if (hipMemcpy(dmt, mt.data(), m * sizeof(ModeTab), hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(fail(PRGD_EDEVICE, "upload of the mode tables failed"));
    d.mt = dmt;
    d.mt_wg = wg0;
    d.mt_out = out0;
    d.mt0_nwg = mt[0].nwg;
    d.use_modes = 1;
    if (want_iface) {
      d.use_iface = 1;
      d.rpos = rpos;
      d.ifl = ifl;
      d.ifr = ifr;
    }
  } else if (!d.use3) {
    long long tot = 0;
    int nbs = 1;
    sampled_plan(m, s->n.data(), R, d.prec, N, d.priv_off, tot, nbs);
    d.priv_len = (int)tot;
    d.nb_sampled = nbs;
    if (tot > 0) {
      unsigned char *pp = nullptr;
      const long long f = mixed ? 4 : 8;
      if (!A(s->alloc(&pp, (long long)nbs * tot * f))) return cleanup(fail(PRGD_ENOMEM, "device allocation failed"));
      d.part_priv = pp;
    }
  }
  if (!A(s->alloc(&s->d_dev, 1))) return cleanup(fail(PRGD_ENOMEM, "device allocation failed"));
  if (hipMemcpyAsync(s->d_dev, &d, sizeof(Dev), hipMemcpyHostToDevice, s->stream) != hipSuccess)
    return cleanup(fail(PRGD_EDEVICE, "descriptor upload failed"));
  // left-orthogonalise T_0 (TT-SVD to its own ranks with a zero direction) and
  // measure ||T_0||, ||T*||
  if (launch_dense_iteration(s->batch(), s->stream, 1) != hipSuccess) return cleanup(fail(PRGD_EDEVICE, "init launch failed"));
  if (s->has_truth && launch_truth_sweep(s->batch(), s->stream, 1) != hipSuccess)
    return cleanup(fail(PRGD_EDEVICE, "truth norm launch failed"));
  if (mixed && convert_f64_f32(d.cores, d.cores32, pn, s->stream) != hipSuccess)
    return cleanup(fail(PRGD_EDEVICE, "convert failed"));
  State st;
  if (read_state(s, st) != PRGD_OK) return cleanup(PRGD_EDEVICE);
  if (st.status < 0) return cleanup(fail(PRGD_EBREAKDOWN, "left-orthogonalisation of init_cores broke down"));
  if (idx_raw) {   // the unsorted copies are no longer needed (read_state synchronised)
    s->release(idx_raw);
    s->release(val_raw);
  }
  if (perm0) {     // nor the permutations behind the position maps
    s->release(perm0);
    s->release(perm_k);
    s->release(inv_k);
  }
  *out = s;
  return PRGD_OK;
}

}  // namespace prgd

extern "C" {

prgd_status prgd_iterate(prgd_solver s, int32_t iters) {
  if (!s) return fail(PRGD_ESTATE, "null solver");
  if (iters < 0) return fail(PRGD_EINVAL, "iters < 0");
  return enqueue_iterations(s, iters);
}

prgd_status prgd_iterate_timed(prgd_solver s, int32_t iters, int32_t stride, double *main_ms, double *total_ms) {
  if (!s) return fail(PRGD_ESTATE, "null solver");
  if (iters < 0 || stride < 1 || !main_ms || !total_ms) return fail(PRGD_EINVAL, "iters < 0, stride < 1 or null output");
  *main_ms = 0.0;
  *total_ms = 0.0;
  if (iters == 0) return PRGD_OK;
  // for the k-th bracketed iteration: ev[2 k] before it, ev[2 k + 1] after its
  // main sampled kernel; ev.back() after the last iteration
  const int nbr = (iters + stride - 1) / stride;
  std::vector<hipEvent_t> ev((size_t)2 * nbr + 1);
  for (auto &e : ev) HIPCHECK(hipEventCreate(&e));
  const Batch bt = s->batch();
  hipError_t err = hipSuccess;
  auto chk = [&](hipError_t x) { if (x != hipSuccess && err == hipSuccess) err = x; };
  for (int it = 0; it < iters && err == hipSuccess; ++it) {
    const bool br = it % stride == 0;
    const int k = it / stride;
    if (br) chk(hipEventRecord(ev[2 * k], s->stream));
    chk(sampled_pass(s, 0, br ? ev[2 * k + 1] : nullptr));
    chk(launch_dense_iteration(bt, s->stream, 0));
    if (s->has_truth) chk(launch_truth_sweep(bt, s->stream, 0));
  }
  chk(hipEventRecord(ev.back(), s->stream));
  prgd_status rc = PRGD_OK;
  if (err != hipSuccess) rc = fail(PRGD_EDEVICE, std::string("launch: ") + hipGetErrorString(err));
  if (rc == PRGD_OK && hipStreamSynchronize(s->stream) != hipSuccess) rc = fail(PRGD_EDEVICE, "sync failed");
  if (rc == PRGD_OK) {
    for (int k = 0; k < nbr; ++k) {
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]);
      *main_ms += ms;
    }
    *main_ms /= nbr;
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, ev[0], ev.back());
    *total_ms = ms;
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  return rc;
}

prgd_status prgd_iterate_profiled(prgd_solver s, int32_t iters, double *phase_ms) {
  if (!s) return fail(PRGD_ESTATE, "null solver");
  if (iters < 0 || !phase_ms) return fail(PRGD_EINVAL, "iters < 0 or null phase_ms");
  constexpr int NP = PRGD_NPHASES;
  for (int p = 0; p < NP; ++p) phase_ms[p] = 0.0;
  if (iters == 0) return PRGD_OK;
  std::vector<hipEvent_t> ev((size_t)iters * (NP + 1));
  for (auto &e : ev) HIPCHECK(hipEventCreate(&e));
  prgd_status rc = PRGD_OK;
  for (int it = 0; it < iters && rc == PRGD_OK; ++it) {
    hipEvent_t *e = ev.data() + (size_t)it * (NP + 1);
    hipError_t err = hipSuccess;
    auto chk = [&](hipError_t x) { if (x != hipSuccess && err == hipSuccess) err = x; };
    chk(hipEventRecord(e[0], s->stream));
    chk(sampled_pass(s, 0, e[1]));
    chk(hipEventRecord(e[2], s->stream));
    chk(launch_project(s->batch(), s->stream));
    chk(hipEventRecord(e[3], s->stream));
    bool out_done = false;
    chk(launch_retract(s->batch(), s->stream, 0, out_done));
    chk(hipEventRecord(e[4], s->stream));
    if (!out_done) chk(launch_output(s->batch(), s->stream, 0));
    chk(hipEventRecord(e[5], s->stream));
    if (s->has_truth) chk(launch_truth_sweep(s->batch(), s->stream, 0));
    chk(hipEventRecord(e[6], s->stream));
    if (err != hipSuccess) rc = fail(PRGD_EDEVICE, std::string("launch: ") + hipGetErrorString(err));
  }
  if (rc == PRGD_OK && hipStreamSynchronize(s->stream) != hipSuccess) rc = fail(PRGD_EDEVICE, "sync failed");
  if (rc == PRGD_OK)
    for (int it = 0; it < iters; ++it)
      for (int p = 0; p < NP; ++p) {
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, ev[(size_t)it * (NP + 1) + p], ev[(size_t)it * (NP + 1) + p + 1]);
        phase_ms[p] += ms;
      }
  for (auto &e : ev) hipEventDestroy(e);
  return rc;
}

prgd_status prgd_sync(prgd_solver s) {
  if (!s) return fail(PRGD_ESTATE, "null solver");
  HIPCHECK(hipStreamSynchronize(s->stream));
  return PRGD_OK;
}

prgd_status prgd_run(prgd_solver s, prgd_report *rep) {
  if (!s) return fail(PRGD_ESTATE, "null solver");
  State st;
  prgd_status e = read_state(s, st);
  if (e != PRGD_OK) return e;
  const auto t0 = std::chrono::steady_clock::now();
  int chunk = 1;
  while (!st.done) {
    e = enqueue_iterations(s, chunk);
    if (e != PRGD_OK) return e;
    e = read_state(s, st);
    if (e != PRGD_OK) return e;
    chunk = std::min(chunk * 2, 32);
  }
  s->last_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  fill_report(s, st, rep);
  if (st.status < 0) return fail((prgd_status)st.status, "iteration broke down (non-SPD Gram, non-finite residual or rank-deficient truncation)");
  return st.status == 0 ? PRGD_OK : PRGD_NOT_CONVERGED;
}

prgd_status prgd_get_report(prgd_solver s, prgd_report *rep) {
  if (!s) return fail(PRGD_ESTATE, "null solver");
  State st;
  prgd_status e = read_state(s, st);
  if (e != PRGD_OK) return e;
  fill_report(s, st, rep);
  return PRGD_OK;
}

prgd_status prgd_get_cores(prgd_solver s, double *out, int64_t cap) {
  if (!s) return fail(PRGD_ESTATE, "null solver");
  if (!out || cap < s->numel) return fail(PRGD_EINVAL, "output buffer too small");
  std::vector<double> padded(s->coff[s->m]);
  HIPCHECK(hipStreamSynchronize(s->stream));
  HIPCHECK(hipMemcpy(padded.data(), s->d.cores, padded.size() * sizeof(double), hipMemcpyDeviceToHost));
  unpack_cores(s->m, s->n.data(), s->r.data(), s->R, padded.data(), out, s->coff);
  return PRGD_OK;
}

prgd_status prgd_get_history(prgd_solver s, prgd_iter_info *out, int32_t cap, int32_t *count) {
  if (!s) return fail(PRGD_ESTATE, "null solver");
  State st;
  prgd_status e = read_state(s, st);
  if (e != PRGD_OK) return e;
  int nrec = st.iter + ((st.done && st.iter < s->d.hist_cap && st.status >= 0) ? 1 : 0);
  nrec = std::min(nrec, s->d.hist_cap);
  std::vector<IterRecord> h(std::max(nrec, 1));
  if (nrec > 0) HIPCHECK(hipMemcpy(h.data(), s->d.hist, nrec * sizeof(IterRecord), hipMemcpyDeviceToHost));
  const int w = std::min(nrec, cap);
  for (int i = 0; i < w; ++i) {
    out[i].iter = h[i].iter;
    out[i].flags = h[i].flags;
    out[i].rel_residual = h[i].rel_residual;
    out[i].rel_change = h[i].rel_change;
    out[i].rel_error = h[i].rel_error;
    out[i].eps = h[i].eps;
    out[i].alpha = h[i].alpha;
  }
  if (count) *count = w;
  return PRGD_OK;
}

prgd_status prgd_sampled_pass(prgd_solver s, double *grad, double *slice_sq, double *res_sq) {
  if (!s) return fail(PRGD_ESTATE, "null solver");
  Dev &d = s->d;
  const long long pn = s->coff[s->m];
  const int soff = d.soff[s->m];
  const bool mixed = d.prec == PREC_MIXED;
  if (mixed) {
    HIPCHECK(fill_f32((float *)d.Y, pn, 0.0f, s->stream));
    HIPCHECK(fill_f32((float *)d.s, soff, 0.0f, s->stream));
  } else {
    HIPCHECK(fill_f64((double *)d.Y, pn, 0.0, s->stream));
    HIPCHECK(fill_f64((double *)d.s, soff, 0.0, s->stream));
  }
  HIPCHECK(sampled_pass(s, 1));
  HIPCHECK(hipStreamSynchronize(s->stream));
  std::vector<double> gp(pn), sv(soff);
  if (mixed) {
    std::vector<float> gf(pn), sf(soff);
    HIPCHECK(hipMemcpy(gf.data(), d.Y, pn * sizeof(float), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(sf.data(), d.s, soff * sizeof(float), hipMemcpyDeviceToHost));
    for (long long i = 0; i < pn; ++i) gp[i] = gf[i];
    for (int i = 0; i < soff; ++i) sv[i] = sf[i];
  } else {
    HIPCHECK(hipMemcpy(gp.data(), d.Y, pn * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(sv.data(), d.s, soff * sizeof(double), hipMemcpyDeviceToHost));
  }
  State st;
  HIPCHECK(hipMemcpy(&st, d.st, sizeof(State), hipMemcpyDeviceToHost));
  if (grad) unpack_cores(s->m, s->n.data(), s->r.data(), s->R, gp.data(), grad, s->coff);
  if (slice_sq) std::copy(sv.begin(), sv.end(), slice_sq);
  if (res_sq) *res_sq = st.res_sq;
  // leave the accumulators clear for the iteration
  if (mixed) {
    HIPCHECK(fill_f32((float *)d.Y, pn, 0.0f, s->stream));
    HIPCHECK(fill_f32((float *)d.s, soff, 0.0f, s->stream));
  } else {
    HIPCHECK(fill_f64((double *)d.Y, pn, 0.0, s->stream));
    HIPCHECK(fill_f64((double *)d.s, soff, 0.0, s->stream));
  }
  HIPCHECK(hipStreamSynchronize(s->stream));
  return PRGD_OK;
}

prgd_status prgd_eval(int32_t m, const int32_t *n, const int32_t *r, const double *cores, int64_t n_obs,
                      const int32_t *indices, double *out, int32_t mem_device, void *stream) {
  int64_t numel = 0;
  if (!checked_numel(m, n, r, numel)) return fail(PRGD_EINVAL, "invalid shape or ranks");
  if (!cores || !indices || !out || n_obs < 0) return fail(PRGD_EINVAL, "null argument");
  int rmax = 1;
  for (int k = 0; k <= m; ++k) rmax = std::max(rmax, (int)r[k]);
  const int R = padded_dim(rmax);
  if (R < 0) return fail(PRGD_ENOTSUP, "TT ranks above 16 are not supported by this build");
  if (n_obs == 0) return PRGD_OK;
  if (!mem_device)
    for (int k = 0; k < m; ++k)
      for (int64_t j = 0; j < n_obs; ++j)
        if (indices[k * n_obs + j] < 0 || indices[k * n_obs + j] >= n[k]) return fail(PRGD_EINVAL, "index out of range");
  hipStream_t st = (hipStream_t)stream;
  std::vector<long long> coff(m + 1, 0);
  for (int k = 0; k < m; ++k) coff[k + 1] = coff[k] + (long long)n[k] * R * R;
  std::vector<double> packed;
  pack_cores(m, n, r, R, cores, packed, coff);
  double *dc = nullptr, *dout = nullptr;
  long long *dcoff = nullptr;
  int *didx = nullptr;
  // device buffers freed on every exit, after the work queued on st has finished
  struct Bufs {
    hipStream_t st;
    void **p[4];
    ~Bufs() {
      (void)hipStreamSynchronize(st);
      for (void **q : p)
        if (*q) (void)hipFree(*q);
    }
  } bufs{st, {(void **)&dc, (void **)&dout, (void **)&dcoff, (void **)&didx}};
  HIPCHECK(hipMalloc(&dc, packed.size() * sizeof(double)));
  HIPCHECK(hipMalloc(&dcoff, coff.size() * sizeof(long long)));
  HIPCHECK(hipMemcpy(dc, packed.data(), packed.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(dcoff, coff.data(), coff.size() * sizeof(long long), hipMemcpyHostToDevice));
  const int *ip = indices;
  double *op = out;
  if (!mem_device) {
    HIPCHECK(hipMalloc(&didx, (size_t)m * n_obs * sizeof(int)));
    HIPCHECK(hipMalloc(&dout, (size_t)n_obs * sizeof(double)));
    HIPCHECK(hipMemcpy(didx, indices, (size_t)m * n_obs * sizeof(int), hipMemcpyHostToDevice));
    ip = didx;
    op = dout;
  }
  HIPCHECK(launch_eval(m, R, n_obs, ip, dc, dcoff, op, st));
  HIPCHECK(hipStreamSynchronize(st));
  if (!mem_device) HIPCHECK(hipMemcpy(out, dout, (size_t)n_obs * sizeof(double), hipMemcpyDeviceToHost));

  return PRGD_OK;
}

prgd_status prgd_destroy(prgd_solver s) {
  if (!s) return fail(PRGD_ESTATE, "null solver");
  delete s;
  return PRGD_OK;
}

}  // extern "C"
