// Request server: continuous batching of independent PRGD solves on one
// device (the prgd_server_* calls of include/prgd.h).
//
// One scheduler thread owns the device work.  Each round it
//   1. admits queued requests in arrival order while a slot is free and the
//      admission estimate of the request's device footprint fits the budget
//      (creation = the same code as prgd_create: copy, grouping of Omega,
//      orthogonalisation of T_0);
//   2. for every group of live solves that share (order, padded rank,
//      precision, sampled-pass variant) launches `iters_per_tick` iterations
//      with one launch per kernel for the whole group (blockIdx.y selects the
//      solve), then gathers each member's State into pinned host memory;
//   3. reads the gathered states of completed rounds, takes finished solves
//      out of their group, and once no launched round references them any
//      more copies their cores out and frees their device memory.
// A solve stops on the device by its own stopping rule (its State.done flag
// turns later launches into no-ops for it), so the iteration count and the
// result never depend on the round length or on the other members.
// At most two rounds per group are in flight, so the device always has
// queued work while the host processes the previous round.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "solver.hpp"

using namespace prgd;

namespace {

using Clock = std::chrono::steady_clock;

struct Group;

struct Request {
  uint64_t ticket = 0;
  // owned copies of the caller's inputs (released after admission)
  std::vector<int32_t> n, r, idx;
  std::vector<unsigned char> vals;
  std::vector<double> init, truth;
  prgd_desc desc{};
  int64_t est = 0;
  int64_t numel = 0;
  double t_submit = 0.0, t_admit = NAN, t_finish = NAN;
  prgd_solver solver = nullptr;
  Group *group = nullptr;
  uint64_t last_tick = 0;   // sequence number of the last round that launched work for it
  bool leaving = false;     // finished on the device; freed once its rounds have drained
  State final_state{};
  // result (valid once finished)
  bool finished = false;
  prgd_status status = PRGD_PENDING;
  prgd_report rep{};
  std::vector<double> cores;
};

struct GroupKey {
  int m, R, prec, use3, stage;
  bool operator<(const GroupKey &o) const {
    if (m != o.m) return m < o.m;
    if (R != o.R) return R < o.R;
    if (prec != o.prec) return prec < o.prec;
    if (use3 != o.use3) return use3 < o.use3;
    return stage < o.stage;
  }
};

struct Tick {
  uint64_t seq;
  hipEvent_t ev;
  int buf;
  std::vector<Request *> members;   // order of the descriptor table of this round
};

struct Group {
  GroupKey key{};
  hipStream_t stream = nullptr;
  std::vector<Request *> members;   // live solves stepped by the next round
  bool dirty = true;                // membership changed since the table was uploaded
  int cap = 0;
  Dev *dt_dev = nullptr;            // device descriptor table (stream-ordered uploads)
  State *st_dev = nullptr;          // gathered states
  Dev *dt_pin[2] = {nullptr, nullptr};
  State *st_pin[2] = {nullptr, nullptr};
  std::vector<Dev> host;            // host copies (grid sizing during an enqueue)
  std::deque<Tick> inflight;
  uint64_t done_seq = 0;
  int next_buf = 0;
};

}  // namespace

struct prgd_server_s {
  int device = 0;
  int64_t budget = 0;
  int max_slots = 1;
  int iters = 4;
  Clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_sched;   // wakes the scheduler (new request, stop)
  std::condition_variable cv_done;    // wakes waiters (a request finished)
  bool stop = false;
  uint64_t next_ticket = 1;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::deque<Request *> pending;
  int live = 0;
  int64_t in_use = 0;
  int n_finished = 0;
  std::string thread_error;

  // scheduler-thread state
  std::map<GroupKey, std::unique_ptr<Group>> groups;
  std::vector<Request *> leaving;
  uint64_t next_seq = 1;
  std::thread th;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
  void loop();
  void admit();
  bool enqueue_tick(Group &g);
  void finish_tick(Group &g);
  void retire_drained();
  void finish_request(Request *q, prgd_status st);
  bool grow(Group &g, int need);
  void shutdown();
};

namespace {

void free_group(Group &g) {
  if (g.stream) hipStreamSynchronize(g.stream);
  for (auto &t : g.inflight) hipEventDestroy(t.ev);
  g.inflight.clear();
  if (g.dt_dev) hipFree(g.dt_dev);
  if (g.st_dev) hipFree(g.st_dev);
  for (int b = 0; b < 2; ++b) {
    if (g.dt_pin[b]) hipHostFree(g.dt_pin[b]);
    if (g.st_pin[b]) hipHostFree(g.st_pin[b]);
  }
  if (g.stream) hipStreamDestroy(g.stream);
  g = Group{};
}

}  // namespace

bool prgd_server_s::grow(Group &g, int need) {
  if (need <= g.cap) return true;
  int cap = std::max(16, g.cap);
  while (cap < need) cap *= 2;
  // tables are only replaced between rounds of this group's stream
  hipStreamSynchronize(g.stream);
  if (g.dt_dev) hipFree(g.dt_dev);
  if (g.st_dev) hipFree(g.st_dev);
  for (int b = 0; b < 2; ++b) {
    if (g.dt_pin[b]) hipHostFree(g.dt_pin[b]);
    if (g.st_pin[b]) hipHostFree(g.st_pin[b]);
    g.dt_pin[b] = nullptr;
    g.st_pin[b] = nullptr;
  }
  g.dt_dev = nullptr;
  g.st_dev = nullptr;
  g.cap = 0;
  if (hipMalloc(&g.dt_dev, (size_t)cap * sizeof(Dev)) != hipSuccess) return false;
  if (hipMalloc(&g.st_dev, (size_t)cap * sizeof(State)) != hipSuccess) return false;
  for (int b = 0; b < 2; ++b) {
    if (hipHostMalloc((void **)&g.dt_pin[b], (size_t)cap * sizeof(Dev), hipHostMallocDefault) != hipSuccess) return false;
    if (hipHostMalloc((void **)&g.st_pin[b], (size_t)cap * sizeof(State), hipHostMallocDefault) != hipSuccess) return false;
  }
  g.cap = cap;
  g.dirty = true;
  return true;
}

void prgd_server_s::finish_request(Request *q, prgd_status st) {
  std::lock_guard<std::mutex> lk(mu);
  q->status = st;
  q->t_finish = now();
  q->finished = true;
  q->idx.clear();
  q->idx.shrink_to_fit();
  q->vals.clear();
  q->vals.shrink_to_fit();
  q->init.clear();
  q->init.shrink_to_fit();
  q->truth.clear();
  q->truth.shrink_to_fit();
  live -= 1;
  in_use -= q->est;
  n_finished += 1;
  cv_done.notify_all();
}

void prgd_server_s::admit() {
  for (;;) {
    Request *q = nullptr;
    {
      std::lock_guard<std::mutex> lk(mu);
      if (stop || pending.empty()) return;
      Request *h = pending.front();
      if (live >= max_slots || in_use + h->est > budget) return;
      pending.pop_front();
      live += 1;
      in_use += h->est;
      q = h;
    }
    prgd_solver s = nullptr;
    const prgd_status st = solver_create(&q->desc, &s, true);
    q->t_admit = now();
    if (st != PRGD_OK) {
      finish_request(q, st);
      continue;
    }
    q->solver = s;
    {
      // inputs now live on the device
      std::lock_guard<std::mutex> lk(mu);
      q->idx.clear();
      q->idx.shrink_to_fit();
      q->vals.clear();
      q->vals.shrink_to_fit();
    }
    const Dev &d = s->d;
    const int variant = d.use3 ? 1 : (d.use_chain ? 4 : (d.use_modes ? (d.use_iface ? 3 : 2) : 0));   // sampled-pass kernel family
    const GroupKey key{d.m, d.R, d.prec + 2 * d.tangent_bf16, variant, d.use3 ? (d.q3.wave ? 2 : d.q3.stage) : 0};
    auto it = groups.find(key);
    if (it == groups.end()) {
      auto g = std::make_unique<Group>();
      g->key = key;
      if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) {
        prgd_destroy(s);
        q->solver = nullptr;
        finish_request(q, PRGD_EDEVICE);
        continue;
      }
      it = groups.emplace(key, std::move(g)).first;
    }
    Group &g = *it->second;
    q->group = &g;
    g.members.push_back(q);
    g.dirty = true;
  }
}

bool prgd_server_s::enqueue_tick(Group &g) {
  const int ns = (int)g.members.size();
  if (!grow(g, ns)) return false;
  const int b = g.next_buf;
  g.next_buf ^= 1;
  g.host.resize(ns);
  for (int i = 0; i < ns; ++i) g.host[i] = g.members[i]->solver->d;
  if (g.dirty) {
    // the pinned buffer b was last read by the round before the previous one,
    // which has completed (at most two rounds in flight)
    std::memcpy(g.dt_pin[b], g.host.data(), (size_t)ns * sizeof(Dev));
    if (hipMemcpyAsync(g.dt_dev, g.dt_pin[b], (size_t)ns * sizeof(Dev), hipMemcpyHostToDevice, g.stream) != hipSuccess)
      return false;
    g.dirty = false;
  }
  const Batch bt{g.dt_dev, g.host.data(), ns};
  if (enqueue_batch_iterations(bt, iters, g.stream) != hipSuccess) return false;
  if (launch_gather_state(bt, g.st_dev, g.stream) != hipSuccess) return false;
  if (hipMemcpyAsync(g.st_pin[b], g.st_dev, (size_t)ns * sizeof(State), hipMemcpyDeviceToHost, g.stream) != hipSuccess)
    return false;
  Tick t;
  t.seq = next_seq++;
  t.buf = b;
  t.members = g.members;
  if (hipEventCreateWithFlags(&t.ev, hipEventDisableTiming) != hipSuccess) return false;
  if (hipEventRecord(t.ev, g.stream) != hipSuccess) {
    hipEventDestroy(t.ev);
    return false;
  }
  for (Request *q : g.members) q->last_tick = t.seq;
  g.inflight.push_back(std::move(t));
  return true;
}

void prgd_server_s::finish_tick(Group &g) {
  Tick t = std::move(g.inflight.front());
  g.inflight.pop_front();
  g.done_seq = t.seq;
  hipEventDestroy(t.ev);
  const State *sts = g.st_pin[t.buf];
  for (size_t i = 0; i < t.members.size(); ++i) {
    Request *q = t.members[i];
    if (q->leaving || !sts[i].done) continue;
    q->leaving = true;
    q->final_state = sts[i];
    g.members.erase(std::find(g.members.begin(), g.members.end(), q));
    g.dirty = true;
    leaving.push_back(q);
  }
}

void prgd_server_s::retire_drained() {
  for (size_t i = 0; i < leaving.size();) {
    Request *q = leaving[i];
    if (q->last_tick > q->group->done_seq) {
      ++i;
      continue;
    }
    leaving.erase(leaving.begin() + i);
    const State &st = q->final_state;
    std::vector<double> out((size_t)q->numel);
    prgd_status rc = prgd_get_cores(q->solver, out.data(), q->numel);
    prgd_report rep{};
    rep.iterations = st.iter;
    rep.rel_residual = st.rel_res;
    rep.rel_change = st.iter > 0 ? st.rel_change : NAN;
    rep.rel_error = q->solver->has_truth ? st.rel_error : NAN;
    rep.seconds = now() - q->t_admit;
    rep.status = st.status;
    prgd_destroy(q->solver);
    q->solver = nullptr;
    {
      std::lock_guard<std::mutex> lk(mu);
      q->rep = rep;
      q->cores = std::move(out);
    }
    finish_request(q, rc != PRGD_OK ? rc : (prgd_status)st.status);
  }
}

void prgd_server_s::loop() {
  hipSetDevice(device);
  for (;;) {
    admit();
    bool ok = true;
    for (auto &kv : groups) {
      Group &g = *kv.second;
      if (!g.members.empty() && g.inflight.size() < 2) ok = ok && enqueue_tick(g);
    }
    bool progressed = false;
    Group *oldest = nullptr;
    for (auto &kv : groups) {
      Group &g = *kv.second;
      while (!g.inflight.empty() && hipEventQuery(g.inflight.front().ev) == hipSuccess) {
        finish_tick(g);
        progressed = true;
      }
      if (!g.inflight.empty() && (!oldest || g.inflight.front().seq < oldest->inflight.front().seq)) oldest = &g;
    }
    retire_drained();
    if (!ok) {
      std::lock_guard<std::mutex> lk(mu);
      thread_error = "device error in the scheduler";
      stop = true;
    }
    {
      std::unique_lock<std::mutex> lk(mu);
      if (stop) break;
      if (!progressed) {
        if (oldest) {
          lk.unlock();
          hipEventSynchronize(oldest->inflight.front().ev);
        } else if (leaving.empty()) {
          cv_sched.wait_for(lk, std::chrono::milliseconds(2),
                            [&] { return stop || (!pending.empty() && live < max_slots); });
        }
      }
    }
  }
  shutdown();
}

void prgd_server_s::shutdown() {
  for (auto &kv : groups) hipStreamSynchronize(kv.second->stream);
  for (auto &kv : groups)
    for (Request *q : kv.second->members)
      if (q->solver) {
        prgd_destroy(q->solver);
        q->solver = nullptr;
      }
  for (Request *q : leaving)
    if (q->solver) {
      prgd_destroy(q->solver);
      q->solver = nullptr;
    }
  leaving.clear();
  for (auto &kv : groups) free_group(*kv.second);
  groups.clear();
}

namespace {

prgd_status copy_in(const prgd_desc *ds, Request &q) {
  const int m = ds->order;
  const long long N = ds->n_obs;
  const size_t vb = ds->values_fp64 ? sizeof(double) : sizeof(float);
  q.n.assign(ds->mode_sizes, ds->mode_sizes + m);
  q.r.assign(ds->tt_ranks, ds->tt_ranks + m + 1);
  q.idx.resize((size_t)m * N);
  q.vals.resize((size_t)N * vb);
  if (ds->mem_device) {
    if (hipMemcpy(q.idx.data(), ds->indices, q.idx.size() * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(q.vals.data(), ds->values, q.vals.size(), hipMemcpyDeviceToHost) != hipSuccess)
      return set_error(PRGD_EDEVICE, "copy of device inputs failed");
  } else {
    std::memcpy(q.idx.data(), ds->indices, q.idx.size() * sizeof(int32_t));
    std::memcpy(q.vals.data(), ds->values, q.vals.size());
  }
  q.init.assign(ds->init_cores, ds->init_cores + q.numel);
  if (ds->truth_cores) q.truth.assign(ds->truth_cores, ds->truth_cores + q.numel);
  q.desc = *ds;
  q.desc.mode_sizes = q.n.data();
  q.desc.tt_ranks = q.r.data();
  q.desc.indices = q.idx.data();
  q.desc.values = q.vals.data();
  q.desc.mem_device = 0;
  q.desc.init_cores = q.init.data();
  q.desc.truth_cores = ds->truth_cores ? q.truth.data() : nullptr;
  q.desc.stream = nullptr;
  return PRGD_OK;
}

}  // namespace

extern "C" {

prgd_status prgd_server_create(const prgd_server_desc *desc, prgd_server *out) {
  if (!desc || !out) return set_error(PRGD_EINVAL, "null descriptor or output handle");
  *out = nullptr;
  if (desc->max_slots < 1 || desc->max_slots > 4096) return set_error(PRGD_EINVAL, "max_slots must be in [1, 4096]");
  auto sv = std::make_unique<prgd_server_s>();
  if (hipGetDevice(&sv->device) != hipSuccess) return set_error(PRGD_EDEVICE, "no HIP device");
  int64_t budget = desc->hbm_budget_bytes;
  if (budget <= 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return set_error(PRGD_EDEVICE, "hipMemGetInfo failed");
    budget = (int64_t)(fr / 4 * 3);
  }
  sv->budget = budget;
  sv->max_slots = desc->max_slots;
  sv->iters = desc->iters_per_tick > 0 ? desc->iters_per_tick : 4;
  sv->t0 = Clock::now();
  prgd_server_s *p = sv.get();
  try {
    sv->th = std::thread([p] { p->loop(); });
  } catch (...) {
    return set_error(PRGD_ENOMEM, "could not start the scheduler thread");
  }
  *out = sv.release();
  return PRGD_OK;
}

prgd_status prgd_server_submit(prgd_server sv, const prgd_desc *ds, uint64_t *ticket) {
  if (!sv) return set_error(PRGD_ESTATE, "null server");
  if (!ds || !ticket) return set_error(PRGD_EINVAL, "null descriptor or ticket");
  if (!ds->indices || !ds->values || !ds->init_cores) return set_error(PRGD_EINVAL, "indices, values and init_cores are required");
  if (ds->order < 2 || ds->order > MAXM) return set_error(ds->order < 2 ? PRGD_EINVAL : PRGD_ENOTSUP, "order must be in [2, 32]");
  if (ds->n_obs < 1 || ds->n_obs >= (1LL << 31)) return set_error(PRGD_EINVAL, "n_obs must be in [1, 2^31)");
  const int64_t numel = prgd_cores_numel(ds->order, ds->mode_sizes, ds->tt_ranks);
  if (numel < 0) return set_error(PRGD_EINVAL, "invalid mode sizes or ranks");
  auto q = std::make_unique<Request>();
  q->numel = numel;
  prgd_status st = copy_in(ds, *q);
  if (st != PRGD_OK) return st;
  // everything prgd_create checks, in the caller's thread
  st = validate_desc(&q->desc, q->idx.data(), q->vals.data());
  if (st != PRGD_OK) return st;
  q->est = solver_footprint(&q->desc);
  if (q->est < 0) return set_error(PRGD_EINVAL, "invalid descriptor");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return set_error(PRGD_ESTATE, sv->thread_error.empty() ? "server stopped" : sv->thread_error.c_str());
    if (q->est > sv->budget) return set_error(PRGD_ENOMEM, "request footprint exceeds the server's memory budget");
    q->ticket = sv->next_ticket++;
    q->t_submit = sv->now();
    *ticket = q->ticket;
    sv->pending.push_back(q.get());
    sv->reqs.emplace(q->ticket, std::move(q));
  }
  sv->cv_sched.notify_one();
  return PRGD_OK;
}

prgd_status prgd_server_poll(prgd_server sv, uint64_t ticket, prgd_ticket_info *info, double *cores, int64_t cap) {
  if (!sv) return set_error(PRGD_ESTATE, "null server");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return set_error(PRGD_ESTATE, "unknown or released ticket");
  Request &q = *it->second;
  if (!q.finished) return PRGD_PENDING;
  const bool have = q.status >= 0 && (int64_t)q.cores.size() >= q.numel;
  if (cores && have && cap < q.numel) return set_error(PRGD_EINVAL, "output buffer too small");
  if (info) {
    info->report = q.rep;
    if (q.status < 0) info->report.status = q.status;
    info->submit_s = q.t_submit;
    info->admit_s = q.t_admit;
    info->finish_s = q.t_finish;
    info->footprint_bytes = q.est;
  }
  if (cores && have) std::memcpy(cores, q.cores.data(), (size_t)q.numel * sizeof(double));
  const prgd_status st = q.status;
  sv->reqs.erase(it);
  sv->n_finished -= 1;
  if (st < 0) set_error(st, "the request failed (see its status)");
  return st;
}

prgd_status prgd_server_wait(prgd_server sv, uint64_t ticket, double timeout_s) {
  if (!sv) return set_error(PRGD_ESTATE, "null server");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto done = [&] {
    auto it = sv->reqs.find(ticket);
    return it == sv->reqs.end() || it->second->finished || sv->stop;
  };
  if (sv->reqs.find(ticket) == sv->reqs.end()) return set_error(PRGD_ESTATE, "unknown or released ticket");
  if (timeout_s < 0) {
    sv->cv_done.wait(lk, done);
  } else if (!sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
    return PRGD_PENDING;
  }
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return set_error(PRGD_ESTATE, "ticket released while waiting");
  if (!it->second->finished) return set_error(PRGD_ESTATE, sv->thread_error.empty() ? "server stopped" : sv->thread_error.c_str());
  return PRGD_OK;
}

prgd_status prgd_server_stats(prgd_server sv, int32_t *queued, int32_t *live, int32_t *finished, int64_t *bytes) {
  if (!sv) return set_error(PRGD_ESTATE, "null server");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (queued) *queued = (int32_t)sv->pending.size();
  if (live) *live = sv->live;
  if (finished) *finished = sv->n_finished;
  if (bytes) *bytes = sv->in_use;
  return PRGD_OK;
}

prgd_status prgd_server_destroy(prgd_server sv) {
  if (!sv) return set_error(PRGD_ESTATE, "null server");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_sched.notify_all();
  sv->cv_done.notify_all();
  if (sv->th.joinable()) sv->th.join();
  delete sv;
  return PRGD_OK;
}

}  // extern "C"
